// Two-level PFASST block on one device (Sec. 5.2, Algorithm 1).  The time
// steps and ensemble members are one batch (slice s = step * members + member);
// the sends and receives of the algorithm are device copies along the batch
// axis; the coarse step C stays a serial chain over time steps.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "pfsh_internal.h"

using namespace pfsh;

struct pfsh_pfasst {
  pfsh_level* f = nullptr;
  pfsh_level* c = nullptr;
  int n_ts = 0, members = 0, B = 0;
  double* thc = nullptr;   // coarse [B][Mc+1][3][Kc]
  double* fec = nullptr;
  double* fic = nullptr;
  double* tthc = nullptr;  // saved copies of step B
  double* tfec = nullptr;
  double* tfic = nullptr;
  double* tau = nullptr;
  double* base = nullptr;  // predictor: restricted spread initial condition
  double* snap = nullptr;  // fine last-node values sent in step A [B][3][Kf]
  double* fmail = nullptr; // wavefront: fine last-node values, two super-steps [2][B][3][Kf]
  double* cmail = nullptr; // wavefront: coarse last-node state, F_E, F_I [2][B][3][3][Kc]
  double* res = nullptr;   // fine residual per slice and variable [B][3] (pfsh_pfasst_run_tol)
  bool graphs = false;     // replay captured iterations
  struct Cached {
    const void *thf, *fef, *fif;
    const pfsh_level *f, *c, *alt;
    double dt;
    int last;        // iterate: last flag; wavefront run: -(n_iter)
    int k_switch;
    hipStream_t s;
    hipGraph_t g;
    hipGraphExec_t x;
  };
  std::vector<Cached> cache;
};

namespace {

#define PF_TRY(expr)                  \
  do {                                \
    hipError_t e_ = (expr);           \
    if (e_ != hipSuccess) return e_;  \
  } while (0)

void drop_graphs(pfsh_pfasst* x) {
  for (auto& c : x->cache) {
    (void)hipGraphExecDestroy(c.x);
    (void)hipGraphDestroy(c.g);
  }
  x->cache.clear();
}

void free_ctx(pfsh_pfasst* x) {
  drop_graphs(x);
  double* p[] = {x->thc, x->fec, x->fic, x->tthc, x->tfec, x->tfic, x->tau, x->base, x->snap,
                 x->fmail, x->cmail, x->res};
  for (double* q : p)
    if (q) (void)hipFree(q);
  delete x;
}

struct Sizes {
  long long n3kf, n3kc, stf, stc;  // complex values per state / per space-time slice
};
Sizes sizes(const pfsh_pfasst* x) {
  Sizes z;
  z.n3kf = 3LL * x->f->K;
  z.n3kc = 3LL * x->c->K;
  z.stf = x->f->nn * z.n3kf;
  z.stc = x->c->nn * z.n3kc;
  return z;
}

// F at every node of [batch][nn][3][K] arrays, node by node
// F at every node of `batch` space-time slices: one RHS call over all
// batch x nodes states when the level's workspace holds them (the states of a
// slice's nodes are contiguous), else one call per node.
hipError_t eval_all(const pfsh_level* lv, double* th, double* fe, double* fi, int batch,
                    hipStream_t s) {
  const long long n3k = 3LL * lv->K, st = lv->nn * n3k;
  if ((long long)batch * lv->nn <= lv->d.max_batch)
    return rhs_strided(lv, th, n3k, fe, n3k, fi, n3k, batch * lv->nn, s);
  for (int i = 0; i < lv->nn; ++i)
    PF_TRY(rhs_strided(lv, th + 2 * i * n3k, st, fe + 2 * i * n3k, st, fi + 2 * i * n3k, st, batch, s));
  return hipSuccess;
}

hipError_t predict(pfsh_pfasst* x, double dt, const double* th0, double* thf, double* fef,
                   double* fif, hipStream_t s) {
  const Sizes z = sizes(x);
  const int mem = x->members, B = x->B, Mc = x->c->M;
  // broadcast: node 0 of every step gets theta0 of its member
  for (int n = 0; n < x->n_ts; ++n)
    PF_TRY(launch_copy_state(th0, z.n3kf, thf + 2 * (size_t)n * mem * z.stf, z.stf, z.n3kf, mem, s));
  PF_TRY(launch_spread(x->f, thf, B, s));
  PF_TRY(launch_restrict(x->f, x->c, thf, x->thc, B, s));
  PF_TRY(launch_copy_state(x->thc, z.stc, x->base, z.stc, z.stc, B, s));
  PF_TRY(rhs_strided(x->c, x->thc, z.stc, x->fec, z.stc, x->fic, z.stc, B, s));
  PF_TRY(launch_spread(x->c, x->fec, B, s));
  PF_TRY(launch_spread(x->c, x->fic, B, s));
  // wavefront: stage j sweeps steps j..n_ts-1; step n >= 1 first takes the
  // stage-(j-1) last-node value of step n-1, with the F the stage-(j-1) sweep
  // evaluated there (the same state on the same level: no new evaluation)
  for (int j = 0; j < x->n_ts; ++j) {
    const int b0 = j * mem, nb = B - b0;
    double* th = x->thc + 2 * (size_t)b0 * z.stc;
    double* fe = x->fec + 2 * (size_t)b0 * z.stc;
    double* fi = x->fic + 2 * (size_t)b0 * z.stc;
    StepSrc src;
    if (j >= 1) {
      const size_t last = 2 * ((size_t)(b0 - mem) * z.stc + (size_t)Mc * z.n3kc);
      if (Mc >= 2) {   // node 1's kernel takes node 0 (it writes no node >= 2 of any slice)
        src = StepSrc{x->thc + last, x->fec + last, x->fic + last, z.stc};
      } else {
        PF_TRY(launch_copy_node3(x->thc + last, x->fec + last, x->fic + last, z.stc, th, fe, fi,
                                 z.stc, z.n3kc, nb, s));
      }
    }
    PF_TRY(sweep_impl(x->c, dt, th, fe, fi, nullptr, nb, s, src));
  }
  // fine prediction and its F at all nodes
  PF_TRY(launch_interp_add(x->c, x->f, x->thc, x->base, thf, B, s));
  return eval_all(x->f, thf, fef, fif, B, s);
}

// Steps B-D of an iteration (after its fine sweep, step A).
hipError_t iterate_bd(pfsh_pfasst* x, double dt, double* thf, double* fef, double* fif,
                      hipStream_t s) {
  const Sizes z = sizes(x);
  const int mem = x->members, B = x->B, Mf = x->f->M, Mc = x->c->M;
  PF_TRY(launch_copy_state(thf + 2 * (size_t)Mf * z.n3kf, z.stf, x->snap, z.n3kf, z.n3kf, B, s));
  // B) restrict, coarse F, saved copies, tau
  PF_TRY(launch_restrict(x->f, x->c, thf, x->thc, B, s));
  PF_TRY(eval_all(x->c, x->thc, x->fec, x->fic, B, s));
  PF_TRY(launch_copy_node3(x->thc, x->fec, x->fic, z.stc, x->tthc, x->tfec, x->tfic, z.stc, z.stc,
                           B, s));
  PF_TRY(launch_fas_tau(x->f, x->c, dt, fef, fif, x->fec, x->fic, x->tau, B, s));
  // C) serial coarse chain.  On the fused small-batch path a step leaves the
  // assembly of F_E at its last node to the next step's first node kernel
  // (the same kernels' arithmetic in one launch fewer per step).
  const bool fused_c = node_fused_ok(x->c, mem);
  bool pending = false;
  for (int n = 0; n < x->n_ts; ++n) {
    const size_t o = 2 * (size_t)n * mem * z.stc;
    double* th = x->thc + o;
    double* fe = x->fec + o;
    double* fi = x->fic + o;
    StepSrc src;   // receive: last-node state of step n-1 and the F there
    if (n >= 1) {
      const size_t last = 2 * ((size_t)(n - 1) * mem * z.stc + (size_t)Mc * z.n3kc);
      src = StepSrc{x->thc + last, x->fec + last, x->fic + last, z.stc};
      if (pending) src.fe_pending = x->fec + last;
    }
    const bool defer = fused_c && n + 1 < x->n_ts;
    PF_TRY(sweep_impl(x->c, dt, th, fe, fi, x->tau + o, mem, s, src, defer));
    pending = defer;
  }
  // D) interpolate the coarse increments; new fine initial conditions
  {
    const double* nw[3] = {x->thc, x->fec, x->fic};
    const double* od[3] = {x->tthc, x->tfec, x->tfic};
    double* io[3] = {thf, fef, fif};
    PF_TRY(launch_interp_add3(x->c, x->f, 3, nw, od, io, B, s));
  }
  // (one time step per block: no initial condition changes, and the
  // interpolated node-0 increment is exactly zero, so F there stands)
  if (x->n_ts == 1) return hipSuccess;
  PF_TRY(launch_ic_correct(x->f, x->c, x->snap, z.n3kf, x->thc + 2 * (size_t)mem * z.stc, z.stc,
                           thf + 2 * (size_t)mem * z.stf, z.stf, B - mem, s));
  return rhs_strided(x->f, thf, z.stf, fef, z.stf, fif, z.stf, B, s);
}

// Node 0 of every slice from the state there: F at node 0, then state and F
// copied to every node (spread initial iterate).
hipError_t start_step(const pfsh_level* lv, double* th, double* fe, double* fi, int batch,
                      hipStream_t s) {
  const long long st = lv->nn * 3LL * lv->K;
  PF_TRY(rhs_strided(lv, th, st, fe, st, fi, st, batch, s));
  PF_TRY(launch_spread(lv, th, batch, s));
  PF_TRY(launch_spread(lv, fe, batch, s));
  return launch_spread(lv, fi, batch, s);
}

// The last node's state of every slice to node 0 (the next step's initial
// condition).
hipError_t next_step(const pfsh_level* lv, double* th, int batch, hipStream_t s) {
  const long long n3k = 3LL * lv->K, st = lv->nn * n3k;
  return launch_copy_state(th + 2 * (size_t)lv->M * n3k, st, th, st, n3k, batch, s);
}

hipError_t iterate(pfsh_pfasst* x, double dt, double* thf, double* fef, double* fif, bool last,
                   hipStream_t s) {
  // A) fine sweep of all steps
  PF_TRY(sweep_impl(x->f, dt, thf, fef, fif, nullptr, x->B, s));
  if (last) return hipSuccess;
  return iterate_bd(x, dt, thf, fef, fif, s);
}

// n_iter iterations in wavefront order.  Super-step t advances every step n
// whose iteration k = t - n lies in [0, n_iter): the work of a super-step is the
// work of Algorithm 1 on a contiguous range of steps (batched), and each step
// only needs values its left neighbour produced in super-step t-1 (coarse
// last-node value after C, fine last-node value after A) or that it produced
// itself in t-1.  The arithmetic is that of n_iter iterate() calls.
// Iterations k >= k_switch sweep on `alt` (and the F re-evaluation of step D
// before such an iteration uses `alt` too).
hipError_t run_wavefront(pfsh_pfasst* x, double dt, double* thf, double* fef, double* fif,
                         int n_iter, const pfsh_level* alt, int k_switch, hipStream_t s) {
  const Sizes z = sizes(x);
  const int mem = x->members, Mf = x->f->M, Mc = x->c->M, nts = x->n_ts;
  if (!alt) k_switch = n_iter;
  const size_t ff = 2 * (size_t)z.stf, fc = 2 * (size_t)z.stc;   // doubles per step-member slice
  for (int t = 0; t <= nts + n_iter - 2; ++t) {
    const int n_lo = std::max(0, t - (n_iter - 1)), n_hi = std::min(t, nts - 1);
    if (n_lo > n_hi) continue;
    // A) fine sweeps, split where the iteration index crosses k_switch
    //    (k = t - n decreases with n, so steps n <= t - k_switch use alt)
    const int split = std::min(n_hi, t - k_switch);   // last step on alt
    auto sweep_range = [&](int a, int b, const pfsh_level* lv) -> hipError_t {
      if (a > b) return hipSuccess;
      const size_t o = (size_t)a * mem * ff;
      return sweep_impl(lv, dt, thf + o, fef + o, fif + o, nullptr, (b - a + 1) * mem, s);
    };
    PF_TRY(sweep_range(n_lo, split, alt));
    PF_TRY(sweep_range(std::max(n_lo, split + 1), n_hi, x->f));
    // steps in their last iteration stop after A
    const int b_lo = (t - n_lo == n_iter - 1) ? n_lo + 1 : n_lo, b_hi = n_hi;
    if (b_lo > b_hi) continue;
    const int nb = (b_hi - b_lo + 1) * mem;
    const size_t of = (size_t)b_lo * mem * ff, oc = (size_t)b_lo * mem * fc;
    double* fm_now = x->fmail + (size_t)(t & 1) * x->B * 2 * z.n3kf;
    double* fm_prev = x->fmail + (size_t)((t + 1) & 1) * x->B * 2 * z.n3kf;
    double* cm_now = x->cmail + (size_t)(t & 1) * x->B * 2 * 3 * z.n3kc;
    double* cm_prev = x->cmail + (size_t)((t + 1) & 1) * x->B * 2 * 3 * z.n3kc;
    const size_t omf = (size_t)b_lo * mem * 2 * z.n3kf, omc = (size_t)b_lo * mem * 2 * z.n3kc;
    PF_TRY(launch_copy_state(thf + of + 2 * (size_t)Mf * z.n3kf, z.stf, fm_now + omf, z.n3kf,
                             z.n3kf, nb, s));
    // B) restrict, coarse F, saved copies, tau
    PF_TRY(launch_restrict(x->f, x->c, thf + of, x->thc + oc, nb, s));
    PF_TRY(eval_all(x->c, x->thc + oc, x->fec + oc, x->fic + oc, nb, s));
    PF_TRY(launch_copy_node3(x->thc + oc, x->fec + oc, x->fic + oc, z.stc, x->tthc + oc,
                             x->tfec + oc, x->tfic + oc, z.stc, z.stc, nb, s));
    PF_TRY(launch_fas_tau(x->f, x->c, dt, fef + of, fif + of, x->fec + oc, x->fic + oc,
                          x->tau + oc, nb, s));
    // C) coarse initial conditions (and the F there) from the left neighbours
    //    (super-step t-1), coarse sweeps, send
    //    (when every step of the range receives, node 1's kernel takes node 0)
    const int r_lo = std::max(b_lo, 1);
    StepSrc rcv;
    if (r_lo <= b_hi) {
      const int nr = (b_hi - r_lo + 1) * mem;
      const size_t ocr = (size_t)r_lo * mem * fc;
      const double* src = cm_prev + (size_t)(r_lo - 1) * mem * 2 * 3 * z.n3kc;
      if (r_lo == b_lo)
        rcv = StepSrc{src, src + 2 * z.n3kc, src + 4 * z.n3kc, 3 * z.n3kc};
      else
        PF_TRY(launch_copy_node3(src, src + 2 * z.n3kc, src + 4 * z.n3kc, 3 * z.n3kc, x->thc + ocr,
                                 x->fec + ocr, x->fic + ocr, z.stc, z.n3kc, nr, s));
    }
    PF_TRY(sweep_impl(x->c, dt, x->thc + oc, x->fec + oc, x->fic + oc, x->tau + oc, nb, s, rcv));
    {
      const size_t lastc = oc + 2 * (size_t)Mc * z.n3kc;
      double* dst = cm_now + 3 * omc;
      PF_TRY(launch_copy_node3(x->thc + lastc, x->fec + lastc, x->fic + lastc, z.stc, dst,
                               dst + 2 * z.n3kc, dst + 4 * z.n3kc, 3 * z.n3kc, z.n3kc, nb, s));
    }
    // D) interpolate the coarse increments, new fine initial conditions, fine F
    //    at node 0 (on the level of the next iteration)
    {
      const double* nw[3] = {x->thc + oc, x->fec + oc, x->fic + oc};
      const double* od[3] = {x->tthc + oc, x->tfec + oc, x->tfic + oc};
      double* io[3] = {thf + of, fef + of, fif + of};
      PF_TRY(launch_interp_add3(x->c, x->f, 3, nw, od, io, nb, s));
    }
    if (r_lo <= b_hi) {
      const int nr = (b_hi - r_lo + 1) * mem;
      PF_TRY(launch_ic_correct(x->f, x->c, fm_prev + (size_t)(r_lo - 1) * mem * 2 * z.n3kf, z.n3kf,
                               x->thc + (size_t)r_lo * mem * fc, z.stc,
                               thf + (size_t)r_lo * mem * ff, z.stf, nr, s));
    }
    // next iteration k+1 = t - n + 1 >= k_switch  <=>  n <= t + 1 - k_switch
    const int split_d = std::min(b_hi, t + 1 - k_switch);
    auto f0_range = [&](int a, int b, const pfsh_level* lv) -> hipError_t {
      if (a > b) return hipSuccess;
      const size_t o = (size_t)a * mem * ff;
      return rhs_strided(lv, thf + o, z.stf, fef + o, z.stf, fif + o, z.stf, (b - a + 1) * mem, s);
    };
    PF_TRY(f0_range(b_lo, split_d, alt));
    PF_TRY(f0_range(std::max(b_lo, split_d + 1), b_hi, x->f));
  }
  return hipSuccess;
}

}  // namespace

extern "C" pfsh_status pfsh_pfasst_create(pfsh_level* f, pfsh_level* c, int n_ts, int members,
                                          pfsh_pfasst** out) {
  if (!out) return PFSH_EINVAL;
  *out = nullptr;
  if (!f || !c || n_ts < 1 || members < 1) return PFSH_EINVAL;
  if (f->device != c->device || c->T > f->T) return PFSH_ESHAPE;
  const long long B = (long long)n_ts * members;
  if (B > f->d.max_batch || B > c->d.max_batch) return PFSH_ESHAPE;
  pfsh_pfasst* x = new (std::nothrow) pfsh_pfasst();
  if (!x) return PFSH_ENOMEM;
  x->f = f;
  x->c = c;
  x->n_ts = n_ts;
  x->members = members;
  x->B = (int)B;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(f->device);
  const Sizes z = sizes(x);
  const size_t bc = (size_t)B * z.stc * 16, bf = (size_t)B * z.n3kf * 16;
  hipError_t e = hipSuccess;
  double** bufs[] = {&x->thc, &x->fec, &x->fic, &x->tthc, &x->tfec, &x->tfic, &x->tau, &x->base};
  for (double** p : bufs)
    if (e == hipSuccess) e = hipMalloc((void**)p, bc);
  if (e == hipSuccess) e = hipMalloc((void**)&x->snap, bf);
  if (e == hipSuccess) e = hipMalloc((void**)&x->fmail, 2 * bf);
  if (e == hipSuccess) e = hipMalloc((void**)&x->cmail, 2 * (size_t)B * 3 * z.n3kc * 16);
  if (e == hipSuccess) e = hipMalloc((void**)&x->res, (size_t)B * 3 * sizeof(double));
  if (e == hipSuccess)
    for (double** p : bufs)
      if (e == hipSuccess) e = hipMemset(*p, 0, bc);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    free_ctx(x);
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? PFSH_ENOMEM : PFSH_EHIP;
  }
  *out = x;
  return PFSH_OK;
}

extern "C" void pfsh_pfasst_destroy(pfsh_pfasst* x) {
  if (!x) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(x->f->device);
  (void)hipDeviceSynchronize();
  free_ctx(x);
  (void)hipSetDevice(prev);
}

extern "C" pfsh_status pfsh_pfasst_predict(pfsh_pfasst* x, double dt, const void* theta0,
                                           void* theta_f, void* fe_f, void* fi_f, void* stream) {
  if (!x || !theta0 || !theta_f || !fe_f || !fi_f) return PFSH_EINVAL;
  if (!(dt > 0)) return PFSH_EINVAL;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(x->f->device);
  hipError_t e = predict(x, dt, (const double*)theta0, (double*)theta_f, (double*)fe_f,
                         (double*)fi_f, (hipStream_t)stream);
  (void)hipSetDevice(prev);
  return e == hipSuccess ? PFSH_OK : PFSH_EHIP;
}

// One iteration, replayed from a captured graph when graphs are on and the
// stream is an ordinary (non-null, not already capturing) stream.
static hipError_t iterate_maybe_graph(pfsh_pfasst* x, double dt, double* thf, double* fef,
                                      double* fif, bool last, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const bool can = x->graphs && s != nullptr && !x->f->prof_on && !x->c->prof_on &&
                   hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
  if (!can) return iterate(x, dt, thf, fef, fif, last, s);
  for (auto& c : x->cache)
    if (c.thf == thf && c.fef == fef && c.fif == fif && c.f == x->f && c.c == x->c &&
        c.alt == nullptr && c.dt == dt && c.last == (int)last && c.k_switch == 0 && c.s == s)
      return hipGraphLaunch(c.x, s);
  PF_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t e = iterate(x, dt, thf, fef, fif, last, s);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(s, &g);
  if (e != hipSuccess || e2 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return e != hipSuccess ? e : (e2 != hipSuccess ? e2 : hipErrorUnknown);
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return e;
  }
  x->cache.push_back({thf, fef, fif, x->f, x->c, nullptr, dt, (int)last, 0, s, g, ex});
  return hipGraphLaunch(ex, s);
}

static hipError_t run_maybe_graph(pfsh_pfasst* x, double dt, double* thf, double* fef, double* fif,
                                  int n_iter, const pfsh_level* alt, int k_switch, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const bool can = x->graphs && s != nullptr && !x->f->prof_on && !x->c->prof_on &&
                   !(alt && alt->prof_on) && hipStreamIsCapturing(s, &cs) == hipSuccess &&
                   cs == hipStreamCaptureStatusNone;
  if (!can) return run_wavefront(x, dt, thf, fef, fif, n_iter, alt, k_switch, s);
  for (auto& c : x->cache)
    if (c.thf == thf && c.fef == fef && c.fif == fif && c.f == x->f && c.c == x->c &&
        c.alt == alt && c.dt == dt && c.last == -n_iter && c.k_switch == k_switch && c.s == s)
      return hipGraphLaunch(c.x, s);
  PF_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t e = run_wavefront(x, dt, thf, fef, fif, n_iter, alt, k_switch, s);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(s, &g);
  if (e != hipSuccess || e2 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return e != hipSuccess ? e : (e2 != hipSuccess ? e2 : hipErrorUnknown);
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return e;
  }
  x->cache.push_back({thf, fef, fif, x->f, x->c, alt, dt, -n_iter, k_switch, s, g, ex});
  return hipGraphLaunch(ex, s);
}

static bool same_geometry(const pfsh_level* a, const pfsh_level* b);

extern "C" pfsh_status pfsh_pfasst_run(pfsh_pfasst* x, double dt, void* theta_f, void* fe_f,
                                       void* fi_f, int n_iter, pfsh_level* fine_alt, int k_switch,
                                       void* stream) {
  if (!x || !theta_f || !fe_f || !fi_f) return PFSH_EINVAL;
  if (!(dt > 0) || n_iter < 1) return PFSH_EINVAL;
  if (fine_alt && (!same_geometry(x->f, fine_alt) || x->B > fine_alt->d.max_batch)) return PFSH_ESHAPE;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(x->f->device);
  hipError_t e = run_maybe_graph(x, dt, (double*)theta_f, (double*)fe_f, (double*)fi_f, n_iter,
                                 fine_alt, fine_alt ? std::max(0, k_switch) : n_iter,
                                 (hipStream_t)stream);
  (void)hipSetDevice(prev);
  return e == hipSuccess ? PFSH_OK : PFSH_EHIP;
}

extern "C" pfsh_status pfsh_pfasst_iterate(pfsh_pfasst* x, double dt, void* theta_f, void* fe_f,
                                           void* fi_f, int last, void* stream) {
  if (!x || !theta_f || !fe_f || !fi_f) return PFSH_EINVAL;
  if (!(dt > 0)) return PFSH_EINVAL;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(x->f->device);
  hipError_t e = iterate_maybe_graph(x, dt, (double*)theta_f, (double*)fe_f, (double*)fi_f,
                                     last != 0, (hipStream_t)stream);
  (void)hipSetDevice(prev);
  return e == hipSuccess ? PFSH_OK : PFSH_EHIP;
}

static bool same_geometry(const pfsh_level* a, const pfsh_level* b) {
  return a->T == b->T && a->nlat == b->nlat && a->nlon == b->nlon && a->nn == b->nn &&
         a->device == b->device;
}

extern "C" pfsh_status pfsh_pfasst_set_levels(pfsh_pfasst* x, pfsh_level* fine, pfsh_level* coarse) {
  if (!x || !fine || !coarse) return PFSH_EINVAL;
  if (!same_geometry(x->f, fine) || !same_geometry(x->c, coarse)) return PFSH_ESHAPE;
  if (x->B > fine->d.max_batch || x->B > coarse->d.max_batch) return PFSH_ESHAPE;
  x->f = fine;
  x->c = coarse;
  return PFSH_OK;
}

extern "C" pfsh_status pfsh_pfasst_set_graphs(pfsh_pfasst* x, int on) {
  if (!x) return PFSH_EINVAL;
  if (!on) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(x->f->device);
    (void)hipDeviceSynchronize();
    drop_graphs(x);
    (void)hipSetDevice(prev);
  }
  x->graphs = on != 0;
  return PFSH_OK;
}

extern "C" pfsh_status pfsh_pfasst_run_tol(pfsh_pfasst* x, double dt, void* theta_f, void* fe_f,
                                           void* fi_f, int max_iter, const double* tol,
                                           int* iterations, double* residuals, void* stream) {
  if (iterations) *iterations = 0;
  if (!x || !theta_f || !fe_f || !fi_f || !tol) return PFSH_EINVAL;
  if (!(dt > 0) || max_iter < 1) return PFSH_EINVAL;
  for (int v = 0; v < 3; ++v)
    if (!(tol[v] >= 0)) return PFSH_EINVAL;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(x->f->device);
  hipStream_t s = (hipStream_t)stream;
  double* thf = (double*)theta_f;
  double* fef = (double*)fe_f;
  double* fif = (double*)fi_f;
  std::vector<double> r((size_t)x->B * 3);
  pfsh_status st = PFSH_OK;
  for (int k = 0; k < max_iter; ++k) {
    // A) fine sweep, then the fine collocation residual of every slice
    hipError_t e = sweep_impl(x->f, dt, thf, fef, fif, nullptr, x->B, s);
    if (e == hipSuccess) e = launch_residual(x->f, dt, thf, fef, fif, nullptr, x->res, x->B, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(r.data(), x->res, r.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      st = PFSH_EHIP;
      break;
    }
    if (iterations) *iterations = k + 1;
    if (residuals) std::copy(r.begin(), r.end(), residuals + (size_t)k * r.size());
    bool done = true, finite = true;
    for (size_t i = 0; i < r.size(); ++i) {
      if (!std::isfinite(r[i])) finite = false;
      if (!(r[i] <= tol[i % 3])) done = false;
    }
    if (!finite) {
      st = PFSH_ENONFINITE;
      break;
    }
    if (done || k == max_iter - 1) break;
    if (iterate_bd(x, dt, thf, fef, fif, s) != hipSuccess) {
      st = PFSH_EHIP;
      break;
    }
  }
  (void)hipSetDevice(prev);
  return st;
}

extern "C" pfsh_status pfsh_sdc_run(pfsh_level* lv, double dt, void* theta, void* f_expl,
                                    void* f_impl, int nsteps, int nsweeps, int batch, void* stream) {
  if (!lv || !theta || !f_expl || !f_impl) return PFSH_EINVAL;
  if (!(dt > 0) || !std::isfinite(dt) || nsteps < 0 || nsweeps < 1) return PFSH_EINVAL;
  if (batch < 1 || batch > lv->d.max_batch) return PFSH_ESHAPE;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(lv->device);
  hipStream_t s = (hipStream_t)stream;
  double* th = (double*)theta;
  double* fe = (double*)f_expl;
  double* fi = (double*)f_impl;
  hipError_t e = hipSuccess;
  for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
    e = start_step(lv, th, fe, fi, batch, s);
    for (int k = 0; k < nsweeps && e == hipSuccess; ++k)
      e = sweep_impl(lv, dt, th, fe, fi, nullptr, batch, s);
    if (e == hipSuccess) e = next_step(lv, th, batch, s);
  }
  (void)hipSetDevice(prev);
  return e == hipSuccess ? PFSH_OK : PFSH_EHIP;
}

extern "C" pfsh_status pfsh_mlsdc_run(pfsh_pfasst* x, double dt, void* theta_f, void* fe_f,
                                      void* fi_f, int nsteps, int n_iter, void* stream) {
  if (!x || !theta_f || !fe_f || !fi_f) return PFSH_EINVAL;
  if (!(dt > 0) || !std::isfinite(dt) || nsteps < 0 || n_iter < 1) return PFSH_EINVAL;
  if (x->n_ts != 1) return PFSH_ESHAPE;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(x->f->device);
  hipStream_t s = (hipStream_t)stream;
  double* th = (double*)theta_f;
  double* fe = (double*)fe_f;
  double* fi = (double*)fi_f;
  hipError_t e = hipSuccess;
  for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
    e = start_step(x->f, th, fe, fi, x->B, s);
    for (int k = 0; k < n_iter && e == hipSuccess; ++k) {
      e = sweep_impl(x->f, dt, th, fe, fi, nullptr, x->B, s);
      if (e == hipSuccess) e = iterate_bd(x, dt, th, fe, fi, s);
    }
    if (e == hipSuccess) e = next_step(x->f, th, x->B, s);
  }
  (void)hipSetDevice(prev);
  return e == hipSuccess ? PFSH_OK : PFSH_EHIP;
}
