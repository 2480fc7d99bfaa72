// Autotuner of the transform kernels.  Every level keeps, per size bucket, the
// variant it launches for the Legendre synthesis, the ring stage and the
// Legendre analysis (pfsh_internal.h lists the variants).  pfsh_level_autotune
// times each variant on the level's own workspace at the given batch and keeps
// the fastest; pfsh_level_set_variant pins one by hand.
#include "pfsh_internal.h"

namespace pfsh {
int leg_variant_count(int op, int stage);
int ring_variant_count();

int variant_count(const pfsh_level* lv, int stage) {
  if (stage == TS_RING) return ring_variant_count();
  // recurrence mode: generate-once or per-column-tile kernels, no fused node
  if (lv->rec_mode) return stage == TS_FUSE ? 1 : 3;
  if (stage == TS_FUSE) return 2;
  return leg_variant_count(lv->op, stage);
}
}  // namespace pfsh

using namespace pfsh;

namespace {

// the bucket that an RHS evaluation of `batch` states uses in each stage
int stage_bucket(int stage, int batch) {
  if (stage == TS_FUSE) return tune_bucket(batch);
  if (stage == TS_SYNTH) return tune_bucket((2 * 4 * batch + 15) / 16);
  if (stage == TS_ANAL) return tune_bucket((2 * 5 * batch + 15) / 16);
  return tune_bucket(batch);
}

hipError_t launch_stage(const pfsh_level* lv, int stage, int batch, hipStream_t s) {
  if (stage == TS_SYNTH) return launch_leg_synth(lv, 2 * 4 * batch, 4, s);
  if (stage == TS_RING) return launch_ring_rhs(lv, batch, s);
  return launch_leg_anal(lv, 2 * 5 * batch, 5, s);
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

extern "C" int pfsh_variant_count(const pfsh_level* lv, int stage) {
  if (!lv || stage < 0 || stage >= TS_COUNT) return PFSH_EINVAL;
  return variant_count(lv, stage);
}

extern "C" pfsh_status pfsh_level_set_variant(pfsh_level* lv, int stage, int batch, int variant) {
  if (!lv || stage < 0 || stage >= TS_COUNT) return PFSH_EINVAL;
  if (batch < 1 || batch > lv->d.max_batch) return PFSH_ESHAPE;
  if (variant < 0 || variant >= variant_count(lv, stage)) return PFSH_EINVAL;
  lv->variant[stage][stage_bucket(stage, batch)] = (unsigned char)variant;
  return PFSH_OK;
}

extern "C" pfsh_status pfsh_level_get_variant(const pfsh_level* lv, int stage, int batch,
                                              int* variant) {
  if (!lv || !variant || stage < 0 || stage >= TS_COUNT) return PFSH_EINVAL;
  if (batch < 1 || batch > lv->d.max_batch) return PFSH_ESHAPE;
  *variant = lv->variant[stage][stage_bucket(stage, batch)];
  return PFSH_OK;
}

extern "C" pfsh_status pfsh_level_autotune_ex(pfsh_level* lv, int batch, int reps, int flags,
                                              void* stream, float* us_out) {
  if (!lv || reps < 1 || reps > 1000 || (flags & ~PFSH_TUNE_COLD)) return PFSH_EINVAL;
  if (batch < 1 || batch > lv->d.max_batch) return PFSH_ESHAPE;
  DeviceGuard g(lv->device);
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) return PFSH_EHIP;
  if (cap != hipStreamCaptureStatusNone) return PFSH_EUNSUPPORTED;
  // cold: a buffer larger than the L2 and Infinity caches together, rewritten
  // before every timed launch, so that the kernel reads its tables and
  // operands from HBM as it does between the other kernels of a sweep
  const bool cold = (flags & PFSH_TUNE_COLD) != 0;
  constexpr size_t kScrubBytes = (size_t)512 << 20;
  void* scrub = nullptr;
  if (cold && hipMalloc(&scrub, kScrubBytes) != hipSuccess) return PFSH_ENOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) {
    if (scrub) (void)hipFree(scrub);
    return PFSH_EHIP;
  }
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    if (scrub) (void)hipFree(scrub);
    return PFSH_EHIP;
  }
  // Three rounds over the variants (interleaved, so that clock and cache
  // drift hit all of them alike); each variant's time is its best round.  A
  // variant replaces the default only if it is at least 3% faster.
  constexpr int kRounds = 3;
  hipError_t err = hipSuccess;
  for (int stage = 0; stage < TS_TUNED && err == hipSuccess; ++stage) {
    unsigned char& slot = lv->variant[stage][stage_bucket(stage, batch)];
    const unsigned char keep = slot;
    const int nv = variant_count(lv, stage);
    float best_us[PFSH_MAX_VARIANTS];
    for (int v = 0; v < nv; ++v) best_us[v] = 3.0e38f;
    for (int r = 0; r < kRounds && err == hipSuccess; ++r) {
      for (int v = 0; v < nv && err == hipSuccess; ++v) {
        slot = (unsigned char)v;
        err = launch_stage(lv, stage, batch, s);                  // warm-up
        float ms = 0.0f;
        if (!cold) {   // reps launches back to back
          if (err == hipSuccess) err = hipEventRecord(e0, s);
          for (int q = 0; q < reps && err == hipSuccess; ++q) err = launch_stage(lv, stage, batch, s);
          if (err == hipSuccess) err = hipEventRecord(e1, s);
          if (err == hipSuccess) err = hipEventSynchronize(e1);
          if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        } else {       // each launch timed alone after the caches are rewritten
          for (int q = 0; q < reps && err == hipSuccess; ++q) {
            err = hipMemsetAsync(scrub, q & 0xff, kScrubBytes, s);
            if (err == hipSuccess) err = hipEventRecord(e0, s);
            if (err == hipSuccess) err = launch_stage(lv, stage, batch, s);
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float one = 0.0f;
            if (err == hipSuccess) err = hipEventElapsedTime(&one, e0, e1);
            ms += one;
          }
        }
        const float us = 1e3f * ms / (float)reps;
        if (us < best_us[v]) best_us[v] = us;
      }
    }
    int best = 0;
    for (int v = 1; v < nv; ++v)
      if (best_us[v] < best_us[best]) best = v;
    if (best_us[best] > 0.97f * best_us[0]) best = 0;
    if (us_out)
      for (int v = 0; v < nv; ++v) us_out[stage * PFSH_MAX_VARIANTS + v] = best_us[v];
    slot = (unsigned char)(err == hipSuccess ? best : keep);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (scrub && hipStreamSynchronize(s) == hipSuccess) (void)hipFree(scrub);
  return err == hipSuccess ? PFSH_OK : PFSH_EHIP;
}

extern "C" pfsh_status pfsh_level_autotune(pfsh_level* lv, int batch, int reps, void* stream,
                                           float* us_out) {
  return pfsh_level_autotune_ex(lv, batch, reps, 0, stream, us_out);
}
