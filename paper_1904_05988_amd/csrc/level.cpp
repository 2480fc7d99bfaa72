// Level objects: descriptor validation, creation (grid, tables, workspace),
// destruction and queries.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "pfsh_internal.h"

using namespace pfsh;

extern "C" const char* pfsh_status_string(pfsh_status s) {
  switch (s) {
    case PFSH_OK: return "ok";
    case PFSH_EINVAL: return "invalid argument";
    case PFSH_ESHAPE: return "inconsistent sizes";
    case PFSH_ENOMEM: return "device out of memory";
    case PFSH_EHIP: return "HIP runtime error";
    case PFSH_EUNSUPPORTED: return "unsupported configuration";
    case PFSH_ENONFINITE: return "non-finite value";
  }
  return "unknown status";
}

static bool nlon_supported(int n) {
  if (n < 16 || n > 1536) return false;
  while (n % 2 == 0) n /= 2;
  return n == 1 || n == 3;
}

extern "C" pfsh_status pfsh_level_desc_check(const pfsh_level_desc* d) {
  if (!d) return PFSH_EINVAL;
  if (d->T < 1 || d->T > 767) return PFSH_ESHAPE;
  if (d->nlat % 2 != 0 || d->nlat < d->T + 2) return PFSH_ESHAPE;
  if (d->nlon < 2 * d->T + 2) return PFSH_ESHAPE;
  if (!nlon_supported(d->nlon)) return PFSH_EUNSUPPORTED;
  if (d->n_nodes < 2 || d->n_nodes > 9) return PFSH_ESHAPE;
  if (d->max_batch < 1 || d->max_batch > 4096) return PFSH_ESHAPE;
  if (!(d->radius > 0) || !std::isfinite(d->radius)) return PFSH_EINVAL;
  if (!std::isfinite(d->omega) || !std::isfinite(d->phibar) || !(d->phibar >= 0)) return PFSH_EINVAL;
  if (!(d->nu >= 0) || !std::isfinite(d->nu)) return PFSH_EINVAL;
  const int prec = d->precision & ~PFSH_LEGENDRE_RECURRENCE;
  if (prec < PFSH_FP64 || prec > PFSH_BF16X3) return PFSH_EINVAL;
  if ((d->precision & PFSH_LEGENDRE_RECURRENCE) && prec == PFSH_BF16X3) return PFSH_EINVAL;
  return PFSH_OK;
}

static void free_level(pfsh_level* lv) {
  for (auto& v : lv->prof)
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  void* ptrs[] = {lv->tabS, lv->tabA, lv->seeds_d, lv->rec_d, lv->mp_d, lv->itemsS, lv->itemsA, lv->mu_d, lv->w_d,
                  lv->tw_d, lv->eps_d, lv->X, lv->F4, lv->G, lv->Y, lv->S, lv->red};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete lv;
}

template <class T>
static hipError_t alloc_copy(T** dst, const void* src, size_t bytes) {
  hipError_t e = hipMalloc((void**)dst, bytes ? bytes : 16);
  if (e != hipSuccess) return e;
  if (src && bytes) return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  return hipMemset(*dst, 0, bytes ? bytes : 16);
}

extern "C" pfsh_status pfsh_level_create(const pfsh_level_desc* d, int device, pfsh_level** out) {
  if (!out) return PFSH_EINVAL;
  *out = nullptr;
  pfsh_status st = pfsh_level_desc_check(d);
  if (st != PFSH_OK) return st;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PFSH_EINVAL;
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) return PFSH_EHIP;
  // this device's copy of the static residual scratch (pfsh_residual_noalloc)
  if (residual_scratch_setup(device) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipSetDevice(prev);
    return PFSH_EHIP;
  }

  pfsh_level* lv = new (std::nothrow) pfsh_level();
  if (!lv) return PFSH_ENOMEM;
  lv->d = *d;
  lv->device = device;
  const int prec = d->precision & ~PFSH_LEGENDRE_RECURRENCE;
  lv->op = prec == PFSH_FP64 ? OP_F64 : (prec == PFSH_FP32 ? OP_F32 : OP_BF16X3);
  lv->rec_mode = (d->precision & PFSH_LEGENDRE_RECURRENCE) != 0;
  lv->T = d->T;
  lv->L = d->T + 1;
  lv->K = (d->T + 1) * (d->T + 2) / 2;
  lv->Kx = ext_off(d->T, d->T + 1);
  lv->nlat = d->nlat;
  lv->nlon = d->nlon;
  lv->J = d->nlat / 2;
  lv->Jp = (lv->J + 31) / 32 * 32;
  lv->Lp = (lv->L + 7) / 8 * 8;
  lv->nn = d->n_nodes;
  lv->M = d->n_nodes - 1;
  lv->KB = op_kb(lv->op);
  lv->MC = synth_mc(lv->op);
  lv->RB = lv->Jp / 16;
  lv->kb2 = lv->Jp / lv->KB;
  lv->kb2g = lv->Jp / 4;
  lv->CBs = (2 * 4 * d->max_batch + 15) / 16;
  lv->CBa = (2 * 5 * d->max_batch + 15) / 16;

  // per (m, p) bookkeeping
  lv->mp.resize(2 * lv->L);
  long long tS = 0, tA = 0, xS = 0;
  for (int m = 0; m <= lv->T; ++m)
    for (int p = 0; p < 2; ++p) {
      MPInfo& q = lv->mp[2 * m + p];
      q.m = m;
      q.p = p;
      q.np = npar(lv->T, m, p);
      q.kbS = (q.np + lv->KB - 1) / lv->KB;
      q.rbA = (q.np + 15) / 16;
      q.tabS = tS;
      q.tabA = tA;
      q.xS = xS;
      {   // synthesis table region: k-blocks padded to whole 16-byte groups
        const int kg = kgroup_of(lv->op);
        tS += (long long)((q.kbS + kg - 1) / kg * kg) * lv->RB;
      }
      tA += (long long)lv->kb2 * q.rbA;
      xS += (long long)q.kbS * lv->CBs;
    }
  // work lists, heaviest first so that the hardware's in-order dispatch
  // balances the triangular per-m work
  std::vector<std::pair<long long, WorkItem>> ws, wa;
  // synthesis: one entry per (m-chunk, parity); its ring tiles and column tiles
  // are spread by the kernel (all on one XCD, so the chunk's data operand and
  // table rows are re-read from that XCD's L2)
  for (int m0 = 0; m0 <= lv->T; m0 += lv->MC)
    for (int p = 0; p < 2; ++p) {
      const long long work = lv->mp[2 * m0 + p].kbS;   // the chunk's longest order
      ws.push_back({work, WorkItem{2 * m0 + p, 0}});
    }
  for (int i = 0; i < 2 * lv->L; ++i) {
    const MPInfo& q = lv->mp[i];
    if (q.np == 0) continue;
    for (int t = 0; t < (q.rbA + 3) / 4; ++t)
      wa.push_back({(long long)std::min(4, q.rbA - 4 * t), WorkItem{i, t}});
  }
  auto by_work = [](const std::pair<long long, WorkItem>& a, const std::pair<long long, WorkItem>& b) {
    return a.first > b.first;
  };
  std::stable_sort(ws.begin(), ws.end(), by_work);
  std::vector<WorkItem> its, ita;
  for (auto& x : ws) its.push_back(x.second);
  // analysis: the degree tiles of one (m, p) all read its data operand, so they
  // run back to back on one XCD (its L2 then serves the re-reads).  The kernel
  // deals item i to XCD i mod 8, so (m, p) groups are assigned whole to the 8
  // XCD sequences (heaviest group first, to the least loaded sequence) and the
  // sequences interleaved; short sequences are padded with empty items (a tile
  // past the last degree block, which the kernel skips).
  {
    std::vector<std::pair<long long, std::vector<WorkItem>>> groups;
    for (auto& x : wa) {
      if (groups.empty() || groups.back().second[0].mp != x.second.mp) groups.push_back({0, {}});
      groups.back().first += x.first;
      groups.back().second.push_back(x.second);
    }
    std::stable_sort(groups.begin(), groups.end(),
                     [](const auto& a, const auto& b) { return a.first > b.first; });
    std::vector<WorkItem> seq[8];
    long long load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (auto& g : groups) {
      int x = 0;
      for (int y = 1; y < 8; ++y)
        if (load[y] < load[x]) x = y;
      load[x] += g.first;
      for (auto& w : g.second) seq[x].push_back(w);
    }
    size_t len = 0;
    for (auto& q : seq) len = std::max(len, q.size());
    const WorkItem empty{0, 1 << 20};
    for (size_t k = 0; k < len; ++k)
      for (int x = 0; x < 8; ++x) ita.push_back(k < seq[x].size() ? seq[x][k] : empty);
  }
  lv->nitemsS = (int)its.size();
  lv->nitemsA = (int)ita.size();

  // grid and time tables
  gauss_legendre(lv->nlat, lv->mu_h, lv->w_h);
  sdc_matrices(lv->nn, lv->nodes, lv->Q, lv->QE, lv->QI);

  std::vector<unsigned char> tabS, tabA;
  std::vector<double> unused, seeds, rec;
  if (lv->rec_mode)
    build_recurrence(lv, seeds, rec);
  else
    build_tables(lv, tabS, tabA, unused);

  const size_t rsz = lv->op == OP_F64 ? 8 : 4;  // transform real type
  std::vector<unsigned char> tw(2 * rsz * lv->nlon);
  for (int t = 0; t < lv->nlon; ++t) {
    long double a = 2.0L * 3.141592653589793238462643383279502884L * t / lv->nlon;
    long double c = std::cos(a), s = std::sin(a);
    if (rsz == 8) {
      double v[2] = {(double)c, (double)s};
      std::memcpy(tw.data() + 16 * t, v, 16);
    } else {
      float v[2] = {(float)c, (float)s};
      std::memcpy(tw.data() + 8 * t, v, 8);
    }
  }

  const size_t bb = (size_t)op_block_bytes(lv->op);
  const int B = d->max_batch;
  const size_t bytesX = (size_t)xS * bb;
  const size_t bytesF4 = (size_t)B * lv->J * 5 * 2 * lv->Lp * 2 * rsz;
  // analysis data operand: 16 x 4 blocks of the transform real type for every
  // precision (BF16x3 splits into hi/lo when it loads its fragments)
  const size_t bytesG = (size_t)2 * lv->L * lv->kb2g * lv->CBa * 64 * rsz;
  const size_t bytesY = (size_t)B * 5 * lv->Kx * 2 * rsz;
  const size_t bytesS = (size_t)B * lv->M * 3 * lv->K * 16;
  const int rblk = 256;
  lv->red_len = (size_t)B * 3 * ((lv->K + rblk - 1) / rblk);

  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  if (lv->rec_mode) {
    chk(alloc_copy(&lv->seeds_d, seeds.data(), seeds.size() * sizeof(double)));
    chk(alloc_copy(&lv->rec_d, rec.data(), rec.size() * sizeof(double)));
  } else {
    chk(alloc_copy(&lv->tabS, tabS.data(), tabS.size()));
    chk(alloc_copy(&lv->tabA, tabA.data(), tabA.size()));
  }
  chk(alloc_copy(&lv->mp_d, lv->mp.data(), lv->mp.size() * sizeof(MPInfo)));
  chk(alloc_copy(&lv->itemsS, its.data(), its.size() * sizeof(WorkItem)));
  chk(alloc_copy(&lv->itemsA, ita.data(), ita.size() * sizeof(WorkItem)));
  chk(alloc_copy(&lv->mu_d, lv->mu_h.data(), lv->J * sizeof(double)));
  chk(alloc_copy(&lv->w_d, lv->w_h.data(), lv->J * sizeof(double)));
  chk(alloc_copy(&lv->tw_d, tw.data(), tw.size()));
  chk(alloc_copy(&lv->X, nullptr, bytesX));
  chk(alloc_copy(&lv->F4, nullptr, bytesF4));
  chk(alloc_copy(&lv->G, nullptr, bytesG));
  chk(alloc_copy(&lv->Y, nullptr, bytesY));
  chk(alloc_copy(&lv->S, nullptr, bytesS));
  chk(alloc_copy(&lv->red, nullptr, lv->red_len * sizeof(double)));
  chk(hipDeviceSynchronize());
  lv->bytes_tables = tabS.size() + tabA.size() + (seeds.size() + rec.size()) * sizeof(double);
  lv->bytes_work = bytesX + bytesF4 + bytesG + bytesY + bytesS;
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    free_level(lv);
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? PFSH_ENOMEM : PFSH_EHIP;
  }
  *out = lv;
  return PFSH_OK;
}

extern "C" void pfsh_level_destroy(pfsh_level* lv) {
  if (!lv) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(lv->device);
  (void)hipDeviceSynchronize();
  free_level(lv);
  (void)hipSetDevice(prev);
}

extern "C" pfsh_status pfsh_level_query(const pfsh_level* lv, int* K, int* n_nodes, double* nodes,
                                        double* q, double* qe, double* qi, double* mu, double* w) {
  if (!lv) return PFSH_EINVAL;
  const int nn = lv->nn;
  if (K) *K = lv->K;
  if (n_nodes) *n_nodes = nn;
  if (nodes) std::memcpy(nodes, lv->nodes, nn * sizeof(double));
  if (q) std::memcpy(q, lv->Q, nn * nn * sizeof(double));
  if (qe) std::memcpy(qe, lv->QE, nn * nn * sizeof(double));
  if (qi) std::memcpy(qi, lv->QI, nn * nn * sizeof(double));
  if (mu) std::memcpy(mu, lv->mu_h.data(), lv->nlat * sizeof(double));
  if (w) std::memcpy(w, lv->w_h.data(), lv->nlat * sizeof(double));
  return PFSH_OK;
}

extern "C" pfsh_status pfsh_level_bytes(const pfsh_level* lv, unsigned long long* tables,
                                        unsigned long long* workspace) {
  if (!lv) return PFSH_EINVAL;
  if (tables) *tables = lv->bytes_tables;
  if (workspace) *workspace = lv->bytes_work;
  return PFSH_OK;
}
