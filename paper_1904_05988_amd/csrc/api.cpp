// Public compute entry points of libpfsh: argument validation on the host,
// then the kernel sequence of each call enqueued on the caller's stream.
#include <cmath>
#include <cstdlib>
#include <vector>

#include "pfsh_internal.h"

using namespace pfsh;

namespace {

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

inline pfsh_status st_of(hipError_t e) { return e == hipSuccess ? PFSH_OK : PFSH_EHIP; }

#define PFSH_TRY(expr)                    \
  do {                                    \
    hipError_t e_ = (expr);               \
    if (e_ != hipSuccess) return e_;      \
  } while (0)

}  // namespace

namespace pfsh {

// Legendre synthesis, ring stage and Legendre analysis of the operand that the
// preceding kernel wrote (batch states); the products end in the analysis
// workspace Y.
static hipError_t transforms(const pfsh_level* lv, int batch, hipStream_t s) {
  {
    ProfScope p(lv, PFSH_K_LEG_SYNTH, s, batch);
    PFSH_TRY(launch_leg_synth(lv, 2 * 4 * batch, 4, s));
  }
  {
    ProfScope p(lv, PFSH_K_RING, s, batch);
    PFSH_TRY(launch_ring_rhs(lv, batch, s));
  }
  ProfScope p(lv, PFSH_K_LEG_ANAL, s, batch);
  return launch_leg_anal(lv, 2 * 5 * batch, 5, s);
}

// F_E (and optionally F_I) at `batch` states spaced `sstride` complex values
// apart; outputs spaced fes / fis apart.
hipError_t rhs_strided(const pfsh_level* lv, const double* state, long long sstride, double* fe,
                       long long fes, double* fi, long long fis, int batch, hipStream_t s) {
  {
    ProfScope p(lv, PFSH_K_PREP, s, batch);
    PFSH_TRY(launch_prep_rhs(lv, state, sstride, fi, fis, batch, s));
  }
  if (!fe) return hipSuccess;
  PFSH_TRY(transforms(lv, batch, s));
  ProfScope p(lv, PFSH_K_ASSEMBLE, s, batch);
  return launch_assemble(lv, fe, fes, batch, s);
}

// One sweep on [batch][nn][3][K] arrays (validated by the caller): per node the
// fused node kernel (update, implicit solve, F_I, synthesis input; on node 1
// also the old-iterate terms) and the transforms of the new state; the F_E
// assembly of each node runs in the next node's kernel, the last one on its
// own.  src: node 0 (state, F_E, F_I) is taken from there by node 1's kernel.
hipError_t sweep_impl(const pfsh_level* lv, double dt, double* th, double* fe, double* fi,
                      const double* tau, int batch, hipStream_t s, const StepSrc& src,
                      bool defer_last) {
  const long long n3k = 3LL * lv->K;
  const long long stride = lv->nn * n3k;
  const bool fused = node_fused_ok(lv, batch);
  if (!fused && (defer_last || src.fe_pending)) return hipErrorInvalidValue;
  if (src.fe_pending && (src.fe_pending != src.fe || !src.th)) return hipErrorInvalidValue;
  if (fused) {
    // per node: fused kernel (analysis of the previous node's products +
    // assembly + node update + synthesis), then the ring stage; a last fused
    // kernel analyses and assembles F_E of node M
    for (int i = 1; i <= lv->M; ++i) {
      {
        ProfScope p(lv, PFSH_K_SWEEP_NODE, s, batch);
        PFSH_TRY(launch_node_fused(lv, i, i > 1 ? i - 1 : -1, dt, th, fe, fi, tau, batch,
                                   i == 1 ? src : StepSrc(), s));
      }
      ProfScope p(lv, PFSH_K_RING, s, batch);
      PFSH_TRY(launch_ring_rhs(lv, batch, s));
    }
    if (defer_last) return hipSuccess;
    ProfScope p(lv, PFSH_K_SWEEP_NODE, s, batch);
    return launch_node_fused(lv, 0, lv->M, dt, th, fe, fi, tau, batch, StepSrc(), s);
  }
  for (int i = 1; i <= lv->M; ++i) {
    const int asm_node = i > 1 ? i - 1 : -1;
    {
      ProfScope p(lv, PFSH_K_SWEEP_NODE, s, batch);
      PFSH_TRY(launch_sweep_step(lv, i, asm_node, dt, th, fe, fi, tau, batch,
                                 i == 1 ? src : StepSrc(), s));
    }
    PFSH_TRY(transforms(lv, batch, s));
  }
  ProfScope p(lv, PFSH_K_ASSEMBLE, s, batch);
  return launch_assemble(lv, fe + 2 * lv->M * n3k, stride, batch, s);
}

}  // namespace pfsh

static bool bad_batch(const pfsh_level* lv, int batch) {
  return batch < 1 || batch > lv->d.max_batch;
}

extern "C" pfsh_status pfsh_sh_synthesis(pfsh_level* lv, const void* spec, void* grid, int nfields,
                                         void* stream) {
  if (!lv || !spec || !grid) return PFSH_EINVAL;
  if (nfields < 1 || nfields > 4 * lv->d.max_batch) return PFSH_ESHAPE;
  DeviceGuard g(lv->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_prep_scalar(lv, (const double*)spec, nfields, s);
  if (e == hipSuccess) e = launch_leg_synth(lv, 2 * nfields, nfields, s);
  if (e == hipSuccess) e = launch_ring_synth(lv, nfields, (double*)grid, s);
  return st_of(e);
}

extern "C" pfsh_status pfsh_sh_analysis(pfsh_level* lv, const void* grid, void* spec, int nfields,
                                        void* stream) {
  if (!lv || !spec || !grid) return PFSH_EINVAL;
  if (nfields < 1 || nfields > 5 * lv->d.max_batch) return PFSH_ESHAPE;
  DeviceGuard g(lv->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_ring_anal(lv, nfields, (const double*)grid, s);
  if (e == hipSuccess) e = launch_leg_anal(lv, 2 * nfields, nfields, s);
  if (e == hipSuccess) e = launch_unpack_scalar(lv, (double*)spec, nfields, s);
  return st_of(e);
}

extern "C" pfsh_status pfsh_rhs(pfsh_level* lv, const void* state, void* f_expl, void* f_impl,
                                int batch, void* stream) {
  if (!lv || !state || (!f_expl && !f_impl)) return PFSH_EINVAL;
  if (bad_batch(lv, batch)) return PFSH_ESHAPE;
  DeviceGuard g(lv->device);
  const long long n3k = 3LL * lv->K;
  return st_of(rhs_strided(lv, (const double*)state, n3k, (double*)f_expl, n3k, (double*)f_impl,
                           n3k, batch, (hipStream_t)stream));
}

extern "C" pfsh_status pfsh_implicit_solve(pfsh_level* lv, double beta, const void* b, void* x,
                                           int batch, void* stream) {
  if (!lv || !b || !x) return PFSH_EINVAL;
  if (!(beta >= 0) || !std::isfinite(beta)) return PFSH_EINVAL;
  if (bad_batch(lv, batch)) return PFSH_ESHAPE;
  DeviceGuard g(lv->device);
  return st_of(launch_implicit_solve(lv, beta, (const double*)b, (double*)x, batch,
                                     (hipStream_t)stream));
}

extern "C" pfsh_status pfsh_sdc_sweep(pfsh_level* lv, double dt, void* theta, void* f_expl,
                                      void* f_impl, const void* tau, int batch, void* stream) {
  if (!lv || !theta || !f_expl || !f_impl) return PFSH_EINVAL;
  if (!(dt > 0) || !std::isfinite(dt)) return PFSH_EINVAL;
  if (bad_batch(lv, batch)) return PFSH_ESHAPE;
  DeviceGuard g(lv->device);
  return st_of(sweep_impl(lv, dt, (double*)theta, (double*)f_expl, (double*)f_impl,
                          (const double*)tau, batch, (hipStream_t)stream));
}

extern "C" pfsh_status pfsh_level_set_implicit(pfsh_level* lv, int mode) {
  if (!lv || (mode != PFSH_IMPLICIT_COMBINED && mode != PFSH_IMPLICIT_SPLIT)) return PFSH_EINVAL;
  lv->implicit_split = mode == PFSH_IMPLICIT_SPLIT ? 1 : 0;
  return PFSH_OK;
}

extern "C" pfsh_status pfsh_residual(pfsh_level* lv, double dt, const void* theta,
                                     const void* f_expl, const void* f_impl, const void* tau,
                                     double* out, int batch, void* stream) {
  if (!lv || !theta || !f_expl || !f_impl || !out) return PFSH_EINVAL;
  if (!(dt > 0) || !std::isfinite(dt)) return PFSH_EINVAL;
  if (bad_batch(lv, batch)) return PFSH_ESHAPE;
  DeviceGuard g(lv->device);
  return st_of(launch_residual(lv, dt, (const double*)theta, (const double*)f_expl,
                               (const double*)f_impl, (const double*)tau, out, batch,
                               (hipStream_t)stream));
}

extern "C" pfsh_status pfsh_residual_noalloc(pfsh_level* lv, double dt, const void* theta,
                                             const void* f_expl, const void* f_impl,
                                             const void* tau, double* out, int batch,
                                             void* stream) {
  if (!lv || !theta || !f_expl || !f_impl || !out) return PFSH_EINVAL;
  if (!(dt > 0) || !std::isfinite(dt)) return PFSH_EINVAL;
  if (batch < 1 || batch > 65535) return PFSH_ESHAPE;
  if (residual_part_len(lv, batch) > kResidualScratchDoubles) return PFSH_ESHAPE;
  double* part = residual_scratch(lv->device);   // looked up when the level was created
  if (!part) return PFSH_EHIP;
  DeviceGuard g(lv->device);
  return st_of(launch_residual_into(lv, dt, (const double*)theta, (const double*)f_expl,
                                    (const double*)f_impl, (const double*)tau, out, part, batch,
                                    (hipStream_t)stream));
}

extern "C" pfsh_status pfsh_check_finite(const double* values, int count, void* stream) {
  if (!values || count < 0) return PFSH_EINVAL;
  if (count == 0) return PFSH_OK;
  std::vector<double> h((size_t)count);
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(h.data(), values, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return PFSH_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return PFSH_EHIP;
  for (double v : h)
    if (!std::isfinite(v)) return PFSH_ENONFINITE;
  return PFSH_OK;
}

extern "C" pfsh_status pfsh_spread(pfsh_level* lv, void* theta, void* f_expl, void* f_impl,
                                   int batch, void* stream) {
  if (!lv || (!theta && !f_expl && !f_impl)) return PFSH_EINVAL;
  if (bad_batch(lv, batch)) return PFSH_ESHAPE;
  DeviceGuard g(lv->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (theta) e = launch_spread(lv, (double*)theta, batch, s);
  if (e == hipSuccess && f_expl) e = launch_spread(lv, (double*)f_expl, batch, s);
  if (e == hipSuccess && f_impl) e = launch_spread(lv, (double*)f_impl, batch, s);
  return st_of(e);
}

static pfsh_status check_pair(const pfsh_level* f, const pfsh_level* c, int batch) {
  if (!f || !c) return PFSH_EINVAL;
  if (c->T > f->T) return PFSH_ESHAPE;
  if (f->device != c->device) return PFSH_EINVAL;
  if (batch < 1 || batch > f->d.max_batch || batch > c->d.max_batch) return PFSH_ESHAPE;
  return PFSH_OK;
}

extern "C" pfsh_status pfsh_restrict(const pfsh_level* f, const pfsh_level* c, const void* in_f,
                                     void* out_c, int batch, void* stream) {
  pfsh_status st = check_pair(f, c, batch);
  if (st != PFSH_OK) return st;
  if (!in_f || !out_c) return PFSH_EINVAL;
  DeviceGuard g(f->device);
  return st_of(launch_restrict(f, c, (const double*)in_f, (double*)out_c, batch, (hipStream_t)stream));
}

extern "C" pfsh_status pfsh_interpolate_add(const pfsh_level* c, const pfsh_level* f,
                                            const void* new_c, const void* old_c, void* inout_f,
                                            int batch, void* stream) {
  pfsh_status st = check_pair(f, c, batch);
  if (st != PFSH_OK) return st;
  if (!new_c || !inout_f) return PFSH_EINVAL;
  DeviceGuard g(f->device);
  return st_of(launch_interp_add(c, f, (const double*)new_c, (const double*)old_c,
                                 (double*)inout_f, batch, (hipStream_t)stream));
}

extern "C" pfsh_status pfsh_fas_tau(const pfsh_level* f, const pfsh_level* c, double dt,
                                    const void* fe_f, const void* fi_f, const void* fe_c,
                                    const void* fi_c, void* tau_c, int batch, void* stream) {
  pfsh_status st = check_pair(f, c, batch);
  if (st != PFSH_OK) return st;
  if (!fe_f || !fi_f || !fe_c || !fi_c || !tau_c) return PFSH_EINVAL;
  if (!(dt > 0) || !std::isfinite(dt)) return PFSH_EINVAL;
  DeviceGuard g(f->device);
  return st_of(launch_fas_tau(f, c, dt, (const double*)fe_f, (const double*)fi_f,
                              (const double*)fe_c, (const double*)fi_c, (double*)tau_c, batch,
                              (hipStream_t)stream));
}

static void prof_clear(pfsh_level* lv) {
  for (auto& v : lv->prof) {
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    v.clear();
  }
  for (auto& v : lv->prof_batch) v.clear();
}

extern "C" pfsh_status pfsh_profile_enable(pfsh_level* lv, int on) {
  if (!lv) return PFSH_EINVAL;
  DeviceGuard g(lv->device);
  if (on) {
    (void)hipDeviceSynchronize();
    prof_clear(lv);
  }
  lv->prof_on = on != 0;
  return PFSH_OK;
}

extern "C" pfsh_status pfsh_profile_read_batch(pfsh_level* lv, int kernel, int batch,
                                               int* launches, double* total_ms) {
  if (!lv || kernel < 0 || kernel >= PFSH_K_COUNT) return PFSH_EINVAL;
  DeviceGuard g(lv->device);
  double sum = 0.0;
  int n = 0;
  const auto& ev = lv->prof[kernel];
  const auto& bt = lv->prof_batch[kernel];
  for (size_t i = 0; i < ev.size(); ++i) {
    if (batch > 0 && bt[i] != batch) continue;
    if (hipEventSynchronize(ev[i].second) != hipSuccess) return PFSH_EHIP;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ev[i].first, ev[i].second) != hipSuccess) return PFSH_EHIP;
    sum += ms;
    ++n;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = sum;
  return PFSH_OK;
}

extern "C" pfsh_status pfsh_profile_read(pfsh_level* lv, int kernel, int* launches, double* total_ms) {
  return pfsh_profile_read_batch(lv, kernel, 0, launches, total_ms);
}
