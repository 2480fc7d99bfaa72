// Two-level PFASST block on one device (Sec. 5.2, Algorithm 1).  The time
// steps and ensemble members are one batch (slice s = step * members + member);
// the sends and receives of the algorithm are device copies along the batch
// axis; the coarse step C stays a serial chain over time steps.
#include <new>
#include <vector>

#include "pfsh_internal.h"

namespace pfsh {
hipError_t rhs_strided(const pfsh_level* lv, const double* state, long long sstride, double* fe,
                       long long fes, double* fi, long long fis, int batch, hipStream_t s);
hipError_t sweep_impl(const pfsh_level* lv, double dt, double* th, double* fe, double* fi,
                      const double* tau, int batch, hipStream_t s);
}  // namespace pfsh

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
  bool graphs = false;     // replay captured iterations
  struct Cached {
    const void *thf, *fef, *fif;
    const pfsh_level *f, *c;
    double dt;
    bool last;
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
  double* p[] = {x->thc, x->fec, x->fic, x->tthc, x->tfec, x->tfic, x->tau, x->base, x->snap};
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
hipError_t eval_all(const pfsh_level* lv, double* th, double* fe, double* fi, int batch,
                    hipStream_t s) {
  const long long n3k = 3LL * lv->K, st = lv->nn * n3k;
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
  // stage-(j-1) last-node value of step n-1
  for (int j = 0; j < x->n_ts; ++j) {
    const int b0 = j * mem, nb = B - b0;
    double* th = x->thc + 2 * (size_t)b0 * z.stc;
    double* fe = x->fec + 2 * (size_t)b0 * z.stc;
    double* fi = x->fic + 2 * (size_t)b0 * z.stc;
    if (j >= 1) {
      const double* src = x->thc + 2 * ((size_t)(b0 - mem) * z.stc + (size_t)Mc * z.n3kc);
      PF_TRY(launch_copy_state(src, z.stc, th, z.stc, z.n3kc, nb, s));
      PF_TRY(rhs_strided(x->c, th, z.stc, fe, z.stc, fi, z.stc, nb, s));
    }
    PF_TRY(sweep_impl(x->c, dt, th, fe, fi, nullptr, nb, s));
  }
  // fine prediction and its F at all nodes
  PF_TRY(launch_interp_add(x->c, x->f, x->thc, x->base, thf, B, s));
  return eval_all(x->f, thf, fef, fif, B, s);
}

hipError_t iterate(pfsh_pfasst* x, double dt, double* thf, double* fef, double* fif, bool last,
                   hipStream_t s) {
  const Sizes z = sizes(x);
  const int mem = x->members, B = x->B, Mf = x->f->M, Mc = x->c->M;
  // A) fine sweep of all steps
  PF_TRY(sweep_impl(x->f, dt, thf, fef, fif, nullptr, B, s));
  if (last) return hipSuccess;
  PF_TRY(launch_copy_state(thf + 2 * (size_t)Mf * z.n3kf, z.stf, x->snap, z.n3kf, z.n3kf, B, s));
  // B) restrict, coarse F, saved copies, tau
  PF_TRY(launch_restrict(x->f, x->c, thf, x->thc, B, s));
  PF_TRY(eval_all(x->c, x->thc, x->fec, x->fic, B, s));
  PF_TRY(launch_copy_state(x->thc, z.stc, x->tthc, z.stc, z.stc, B, s));
  PF_TRY(launch_copy_state(x->fec, z.stc, x->tfec, z.stc, z.stc, B, s));
  PF_TRY(launch_copy_state(x->fic, z.stc, x->tfic, z.stc, z.stc, B, s));
  PF_TRY(launch_fas_tau(x->f, x->c, dt, fef, fif, x->fec, x->fic, x->tau, B, s));
  // C) serial coarse chain
  for (int n = 0; n < x->n_ts; ++n) {
    const size_t o = 2 * (size_t)n * mem * z.stc;
    double* th = x->thc + o;
    double* fe = x->fec + o;
    double* fi = x->fic + o;
    if (n >= 1) {
      const double* src = x->thc + 2 * ((size_t)(n - 1) * mem * z.stc + (size_t)Mc * z.n3kc);
      PF_TRY(launch_copy_state(src, z.stc, th, z.stc, z.n3kc, mem, s));
      PF_TRY(rhs_strided(x->c, th, z.stc, fe, z.stc, fi, z.stc, mem, s));
    }
    PF_TRY(sweep_impl(x->c, dt, th, fe, fi, x->tau + o, mem, s));
  }
  // D) interpolate the coarse increments; new fine initial conditions
  PF_TRY(launch_interp_add(x->c, x->f, x->thc, x->tthc, thf, B, s));
  PF_TRY(launch_interp_add(x->c, x->f, x->fec, x->tfec, fef, B, s));
  PF_TRY(launch_interp_add(x->c, x->f, x->fic, x->tfic, fif, B, s));
  if (x->n_ts > 1)
    PF_TRY(launch_ic_correct(x->f, x->c, x->snap, z.n3kf, x->thc + 2 * (size_t)mem * z.stc, z.stc,
                             thf + 2 * (size_t)mem * z.stf, z.stf, B - mem, s));
  return rhs_strided(x->f, thf, z.stf, fef, z.stf, fif, z.stf, B, s);
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
    if (c.thf == thf && c.fef == fef && c.fif == fif && c.f == x->f && c.c == x->c && c.dt == dt &&
        c.last == last && c.s == s)
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
  x->cache.push_back({thf, fef, fif, x->f, x->c, dt, last, s, g, ex});
  return hipGraphLaunch(ex, s);
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
