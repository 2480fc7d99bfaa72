// Internal definitions of libpfsh: level object, packed-operand layouts and
// kernel launchers shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "pfsh.h"

namespace pfsh {

// ---------------------------------------------------------------- layouts
// Spectral m-major slot of (m, n), n = m..T.
__host__ __device__ inline int spec_off(int T, int m) { return m * (T + 1) - m * (m - 1) / 2; }
// Extended m-major slot of (m, n), n = m..T+1 (the transform stages work to
// degree T+1 so that (1-mu^2) dP/dmu folds into P contractions).
__host__ __device__ inline int ext_off(int T, int m) { return m * (T + 2) - m * (m - 1) / 2; }
// Number of degrees n = m+p, m+p+2, ... <= T+1 of parity p for order m.
__host__ __device__ inline int npar(int T, int m, int p) {
  return (m + p <= T + 1) ? ((T + 1 - m - p) / 2 + 1) : 0;
}
// Position of degree n (m <= n <= T+1) of order m in the analysis output: per
// order the degrees of parity 0 (n - m even) first, then those of parity 1, so
// that the workgroup of one parity writes whole cache lines.
__host__ __device__ inline int ext_pos(int T, int m, int n) {
  const int d = n - m;
  return ext_off(T, m) + ((d & 1) ? npar(T, m, 0) : 0) + (d >> 1);
}

// Fourier workspace (the Legendre synthesis writes it, the ring stage reads
// it): per slice b and northern ring j a region of 2 x Lp x nf complex values
// in the transform type, ordered [parity][m / MG][field][m % MG], MG = 64 bytes
// of complex values (8 FP32, 4 FP64).  A synthesis workgroup holds MG
// consecutive orders of one parity, so the runs of all its fields are
// adjacent and its stores fill whole cache lines; the ring stage reads the
// region of its (b, j) front to back.  Lp is a multiple of 8.
__host__ __device__ constexpr int f4_mg(int real_bytes) { return 32 / real_bytes; }
__host__ __device__ inline size_t f4_index(int b, int j, int f, int p, int m, int J, int nf,
                                           int Lp, int MG) {
  return (((size_t)b * J + j) * 2 + p) * (size_t)Lp * nf + (size_t)(m / MG) * MG * nf +
         (size_t)f * MG + (m % MG);
}

// MFMA operand blocks.  FP64/FP32 use 16x16x4 MFMA: a block is 16 (row or
// column) x 4 (k) elements and lane l holds element (l % 16, l / 16).  BF16x3
// uses 16x16x32 MFMA: a block is 16 x 32 and lane l holds elements
// (l % 16, 8 (l / 16) + e), e = 0..7, stored as 8 hi then 8 lo bf16 values.
enum OpKind { OP_F64 = 0, OP_F32 = 1, OP_BF16X3 = 2 };
__host__ __device__ inline int op_kb(int op) { return op == OP_BF16X3 ? 32 : 4; }
// bytes of one 64-lane block
__host__ __device__ inline int op_block_bytes(int op) {
  return op == OP_F64 ? 64 * 8 : (op == OP_F32 ? 64 * 4 : 64 * 16 * 2);
}
// lane and element of (r, k) inside a block (k < KB)
__host__ __device__ inline int op_lane(int op, int r, int k) {
  return op == OP_BF16X3 ? ((k >> 3) << 4) + r : (k << 4) + r;
}
__host__ __device__ inline int op_elem(int op, int k) { return op == OP_BF16X3 ? (k & 7) : 0; }

// k-blocks per 16-byte group of the analysis table: 4 FP32, 2 FP64, 1 (plain
// blocks) BF16x3; element of k-block k, block t (stride S blocks per k-block),
// lane l of a region that starts at block base (a multiple of KG).
__host__ __device__ inline int kgroup_of(int op) {
  return op == OP_BF16X3 ? 1 : (op == OP_F64 ? 2 : 4);
}
__host__ __device__ inline long long kgroup_elem(long long base, long long S, long long k,
                                                 long long t, int lane, int KG) {
  return base * 64 + (((k / KG) * S + t) * 64 + lane) * KG + k % KG;
}

// Per-(m, p) bookkeeping of the packed tables and operands (index mp = 2m+p).
struct MPInfo {
  int m, p, np;       // order, parity, number of degrees
  int kbS;            // synthesis: k-blocks (ceil(np / KB))
  int rbA;            // analysis: row blocks (ceil(np / 16))
  long long tabS;     // synthesis table: first block
  long long tabA;     // analysis table: first block
  long long xS;       // synthesis data operand: first block
  long long seed;     // recurrence mode: first restart chunk of this (m, p)
};

// Recurrence mode (PFSH_LEGENDRE_RECURRENCE): the degrees i = 0..np-1 of one
// (m, p) are cut into chunks of kRecChunk; chunk c restarts from the stored pair
// (P_{n0-2}, P_{n0}), n0 = m + p + 2 kRecChunk c (P_{n0-2} = 0 below m), one
// pair per padded ring j < Jp at seeds[(q.seed + c) Jp + j].  rec[ext_off(T, m)
// + n - m] holds (a, b, c, 0) of P_{n+2} = a ((mu^2 - b) P_n - c P_{n-2}).
constexpr int kRecChunk = 32;
__host__ __device__ inline int rec_chunks(int np) { return (np + kRecChunk - 1) / kRecChunk; }

struct WorkItem {      // one workgroup tile of a Legendre contraction
  int mp;              // (m, p) index; synthesis: first order of the m-chunk, 2 m0 + p
  int tile;            // row tile (64 rows)
};

// Synthesis orders per workgroup: the Fourier coefficients of MC consecutive m
// of one ring are contiguous, so each lane pair writes 64 bytes at once.
__host__ __device__ inline int synth_mc(int op) { return op == OP_F64 ? 4 : 8; }

// Kernel variants chosen per level and per size bucket (pfsh_level_autotune):
// the Legendre synthesis (orders per workgroup, prefetch depth), the Legendre
// analysis (prefetch depth) and the ring stage (largest FFT radix).  Variant 0
// is the built-in default.  Bucket b holds sizes in (2^(b-1), 2^b]; the size is
// the number of 16-column blocks for the Legendre stages and the batch for
// the ring stage.
// A fourth stage, not timed by the tuner, selects the sweep path for batches of
// one or two slices: 0 = fused per-order node kernel (FP64 / FP32 levels),
// 1 = separate kernels.
enum TuneStage { TS_SYNTH = 0, TS_ANAL = 1, TS_RING = 2, TS_TUNED = 3, TS_FUSE = 3, TS_COUNT = 4 };
constexpr int kTuneBuckets = 13;
inline int tune_bucket(int n) {
  int b = 0;
  while (b < kTuneBuckets - 1 && (1 << b) < n) ++b;
  return b;
}
struct ProfScope;
}  // namespace pfsh

struct pfsh_level {
  pfsh_level_desc d;
  int device;
  int op;                  // pfsh::OpKind
  int T, L, K, Kx, J, Jp, nlat, nlon, nn, M;
  int Lp;                  // m-stride of the Fourier workspace (L rounded up to 8)
  int MC;                  // orders m per synthesis workgroup (4 FP64, 8 otherwise)
  int KB, RB, kb2;         // k-block, synthesis row blocks (Jp/16), analysis k-blocks (Jp/KB)
  int kb2g;                // k-blocks of the analysis data operand (Jp/4: 16 x 4 blocks)
  int CBs, CBa;            // column blocks of the synthesis / analysis data operands
  std::vector<pfsh::MPInfo> mp;
  std::vector<double> mu_h, w_h;          // full grid, north to south
  double nodes[9], Q[81], QE[81], QI[81];
  // device tables
  void* tabS = nullptr;    // packed synthesis table (A operand, rows = rings)
  void* tabA = nullptr;    // packed analysis table (A operand, rows = degrees)
  bool rec_mode = false;   // PFSH_LEGENDRE_RECURRENCE: no tables, seeds + rec instead
  double* seeds_d = nullptr;   // [chunks][Jp] (P_{n0-2}, P_{n0}) pairs
  double* rec_d = nullptr;     // [Kx] (a, b, c, 0) of the two-degree recurrence
  pfsh::MPInfo* mp_d = nullptr;
  pfsh::WorkItem* itemsS = nullptr;  int nitemsS = 0;
  pfsh::WorkItem* itemsA = nullptr;  int nitemsA = 0;
  double* mu_d = nullptr;  // [J] northern Gaussian latitudes
  double* w_d = nullptr;   // [J] weights
  void* tw_d = nullptr;    // [nlon] e^{2 pi i t/nlon} in the transform real type
  double* eps_d = nullptr; // [Kx] eps_n^m of the extended layout
  // workspace
  void* X = nullptr;       // synthesis data operand
  void* F4 = nullptr;      // Fourier coefficients, f4_index layout (transform type)
  void* G = nullptr;       // analysis data operand (16 x 4 blocks, transform real type)
  void* Y = nullptr;       // analysis result [batch*5][Kx] complex (transform accumulate type)
  double* S = nullptr;     // sweep pre-accumulation [batch][M][3][K] complex
  double* red = nullptr;   // residual partial maxima
  size_t red_len = 0;
  size_t bytes_tables = 0, bytes_work = 0;
  unsigned char variant[pfsh::TS_COUNT][pfsh::kTuneBuckets] = {};   // chosen kernel variants
  int implicit_split = 0;  // sweeps: implicit step in two substeps (pfsh_level_set_implicit)
  // diagnostic kernel timing (pfsh_profile_*)
  mutable bool prof_on = false;
  mutable std::vector<std::pair<hipEvent_t, hipEvent_t>> prof[PFSH_K_COUNT];
  mutable std::vector<int> prof_batch[PFSH_K_COUNT];   // batch of each bracketed launch
  mutable pfsh::ProfScope* prof_open = nullptr;         // the launch being profiled (ProfScope)
};

namespace pfsh {

// Timing of one kernel launch when profiling is on: the scope opens a pair of
// events on the level, and the next launch through PFSH_LAUNCH on that level
// takes them as the kernel's own start and end timestamps
// (hipExtLaunchKernelGGL), so the measured time is the kernel's alone, without
// the gap between launches.  A scope whose launch did not happen drops its
// events.
struct ProfScope {
  const pfsh_level* lv;
  int id;
  hipStream_t s;
  int batch;
  hipEvent_t b = nullptr, e = nullptr;
  bool used = false;
  ProfScope* prev = nullptr;
  ProfScope(const pfsh_level* l, int k, hipStream_t st, int nb = 0) : lv(l), id(k), s(st), batch(nb) {
    if (!lv->prof_on) return;
    if (hipEventCreate(&b) != hipSuccess) { b = nullptr; return; }
    if (hipEventCreate(&e) != hipSuccess) { (void)hipEventDestroy(b); b = e = nullptr; return; }
    prev = lv->prof_open;
    lv->prof_open = this;
  }
  ~ProfScope() {
    if (!b) return;
    lv->prof_open = prev;
    if (used) {
      lv->prof[id].push_back({b, e});
      lv->prof_batch[id].push_back(batch);
    } else {
      (void)hipEventDestroy(b);
      (void)hipEventDestroy(e);
    }
  }
};

// Launch of a level's kernel: plain, or, inside an open ProfScope on that
// level, with the scope's events as the kernel's start and end timestamps.
#define PFSH_LAUNCH(lv, kernel, grid, block, shm, stream, ...)                            \
  do {                                                                                    \
    pfsh::ProfScope* ps_ = (lv)->prof_open;                                               \
    if (ps_ && !ps_->used) {                                                              \
      ps_->used = true;                                                                   \
      hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, ps_->b, ps_->e, 0,          \
                            __VA_ARGS__);                                                 \
    } else {                                                                              \
      hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);                  \
    }                                                                                     \
  } while (0)

// ------------------------------------------------------------- host tables
void gauss_legendre(int nlat, std::vector<double>& mu, std::vector<double>& w);
void sdc_matrices(int nn, double* nodes, double* Q, double* QE, double* QI);
void lagrange_matrix(int nsrc, const double* src, int ndst, const double* dst, double* out);
// Build packed tables for a level (host), returns bytes.
void build_tables(pfsh_level* lv, std::vector<unsigned char>& tabS, std::vector<unsigned char>& tabA,
                  std::vector<double>& eps_ext);

// Recurrence mode: restart pairs and coefficients (layouts at kRecChunk);
// fills q.seed of every (m, p).  seeds: 2 doubles per (chunk, padded ring).
void build_recurrence(pfsh_level* lv, std::vector<double>& seeds, std::vector<double>& rec);

// Kernel variants of a stage on this level (recurrence mode: 2 per Legendre
// stage, generate-once and per-column-tile; 1 sweep path).
int variant_count(const pfsh_level* lv, int stage);

// ------------------------------------------------------------- launchers
// All return hipSuccess or the launch error.
hipError_t launch_leg_synth(const pfsh_level* lv, int ncols, int nf, hipStream_t s);
hipError_t launch_leg_anal(const pfsh_level* lv, int ncols, int nf, hipStream_t s);
hipError_t launch_ring_rhs(const pfsh_level* lv, int batch, hipStream_t s);
hipError_t launch_ring_synth(const pfsh_level* lv, int nfields, double* grid, hipStream_t s);
hipError_t launch_ring_anal(const pfsh_level* lv, int nfields, const double* grid, hipStream_t s);

// spectral kernels (FP64)
hipError_t launch_prep_rhs(const pfsh_level* lv, const double* state, long long state_stride,
                           double* f_impl, long long fi_stride, int batch, hipStream_t s);
hipError_t launch_prep_scalar(const pfsh_level* lv, const double* spec, int nfields, hipStream_t s);
hipError_t launch_unpack_scalar(const pfsh_level* lv, double* spec, int nfields, hipStream_t s);
hipError_t launch_assemble(const pfsh_level* lv, double* f_expl, long long fe_stride, int batch,
                           hipStream_t s);
hipError_t launch_implicit_solve(const pfsh_level* lv, double beta, const double* b, double* x,
                                 int batch, hipStream_t s);
// Node-0 values received from elsewhere (state, F_E, F_I; nullptr = none).
struct StepSrc {
  const double* th = nullptr;
  const double* fe = nullptr;
  const double* fi = nullptr;
  long long stride = 0;   // complex values between batch entries
  // non-null (fused small-batch path only): F_E at the source node is not yet
  // assembled; it is the analysis of this level's current ring output (the
  // source step's last node), written here (the same array as fe) first
  double* fe_pending = nullptr;
};

// Compositions of the kernels above (api.cpp): the RHS of strided states; one
// sweep (its node 0 optionally received from `src` first).
hipError_t rhs_strided(const pfsh_level* lv, const double* state, long long sstride, double* fe,
                       long long fes, double* fi, long long fis, int batch, hipStream_t s);
// defer_last (fused small-batch path only): leave F_E of the last node to the
// next sweep on this level, which takes this sweep's last node as its source
// with fe_pending set.
hipError_t sweep_impl(const pfsh_level* lv, double dt, double* th, double* fe, double* fi,
                      const double* tau, int batch, hipStream_t s,
                      const StepSrc& src = StepSrc(), bool defer_last = false);

// Sweep node `node` (1..M) fused with the F_E assembly of node `asm_node`
// (-1: none), the old-iterate accumulation (node 1, optionally taking node 0
// from `src`) and the synthesis input of the new node state; leaves the
// analysis of that state to the caller.
hipError_t launch_sweep_step(const pfsh_level* lv, int node, int asm_node, double dt, double* th,
                             double* fe, double* fi, const double* tau, int batch,
                             const StepSrc& src, hipStream_t s);
// One order per workgroup through analysis (of the preceding ring stage's
// output, when asm_node >= 0) + F_E assembly + node update + synthesis (when
// node >= 1); batches of one or two slices, FP64 / FP32 levels
// (node_fused_ok).
bool node_fused_ok(const pfsh_level* lv, int batch);
hipError_t launch_node_fused(const pfsh_level* lv, int node, int asm_node, double dt, double* th,
                             double* fe, double* fi, const double* tau, int batch,
                             const StepSrc& src, hipStream_t s);
hipError_t launch_residual(const pfsh_level* lv, double dt, const double* theta, const double* fe,
                           const double* fi, const double* tau, double* out, int batch,
                           hipStream_t s);
// The same with the partial maxima in `part` (residual_part_len(lv, batch)
// doubles) instead of the level's workspace.
long long residual_part_len(const pfsh_level* lv, int batch);
hipError_t launch_residual_into(const pfsh_level* lv, double dt, const double* theta,
                                const double* fe, const double* fi, const double* tau, double* out,
                                double* part, int batch, hipStream_t s);
// Allocation-free residual scratch: a static device array of
// kResidualScratchDoubles doubles per GPU.  residual_scratch_setup looks up the
// current device's copy (call with `device` current; once per device, later
// calls return at once); residual_scratch returns it (nullptr before setup).
constexpr long long kResidualScratchDoubles = PFSH_RESIDUAL_SCRATCH_DOUBLES;
hipError_t residual_scratch_setup(int device);
double* residual_scratch(int device);
hipError_t launch_spread(const pfsh_level* lv, double* a, int batch, hipStream_t s);
hipError_t launch_restrict(const pfsh_level* f, const pfsh_level* c, const double* in_f,
                           double* out_c, int batch, hipStream_t s);
hipError_t launch_interp_add(const pfsh_level* c, const pfsh_level* f, const double* new_c,
                             const double* old_c, double* inout_f, int batch, hipStream_t s);
// the same for `count` (1-3) array triples in one launch
hipError_t launch_interp_add3(const pfsh_level* c, const pfsh_level* f, int count,
                              const double* const* new_c, const double* const* old_c,
                              double* const* inout_f, int batch, hipStream_t s);
hipError_t launch_fas_tau(const pfsh_level* f, const pfsh_level* c, double dt, const double* fe_f,
                          const double* fi_f, const double* fe_c, const double* fi_c, double* tau,
                          int batch, hipStream_t s);
hipError_t launch_ic_correct(const pfsh_level* f, const pfsh_level* c, const double* recv_f,
                             long long recv_stride, const double* ic_c, long long ic_stride,
                             double* out_f, long long out_stride, int batch, hipStream_t s);
// state, F_E and F_I of one node per batch entry in one launch
hipError_t launch_copy_node3(const double* ts, const double* es, const double* is,
                             long long sstride, double* td, double* ed, double* id,
                             long long dstride, long long n_per, int batch, hipStream_t s);
hipError_t launch_copy_state(const double* src, long long src_stride, double* dst,
                             long long dst_stride, long long n_per, int batch, hipStream_t s);
hipError_t launch_count_nonfinite(const double* v, int n, int* flag, hipStream_t s);

}  // namespace pfsh
