// Legendre stage of the spherical-harmonic transform on MFMA (Sec. 3, second
// step of the two-step transform).
//
// For each zonal wavenumber m the contraction over total wavenumber n (and the
// quadrature over latitude) is a dense product.  Using the equatorial symmetry
// P_n^m(-mu) = (-1)^{n-m} P_n^m(mu), the degrees are split by parity p = (n-m)
// mod 2 and only the northern rings j = 0..J-1 are stored:
//   synthesis  E/O_p[j][c] = sum_i P_{m+p+2i}^m(mu_j) X_p[i][c]        (rows j, k = i)
//              north ring = E + O, south ring = E - O     (combined in the ring stage)
//   analysis   Y_p[i][c]   = sum_j P_{m+p+2i}^m(mu_j) G_p[j][c]        (rows i, k = j)
//              G_0 = w (north + south), G_1 = w (north - south)  (built in the ring stage)
// Columns c = 2 (field + nf * batch) + {re, im}.  Degrees run to T+1 so that the
// (1-mu^2) dP/dmu terms of the vector transforms fold into P contractions.
//
// One workgroup = 4 waves = one (m, p) and a 64-row x 64-column tile; every
// wave owns 2x2 MFMA blocks of 16x16.  Operands are pre-packed in MFMA lane
// order (tables at level creation, data by the producing kernels), so each
// lane loads its fragment with one contiguous load.
#include "mfma_ops.h"

namespace pfsh {

template <class Op>
__global__ __launch_bounds__(256) void k_leg_synth(const void* __restrict__ tab,
                                                  const void* __restrict__ X,
                                                  typename Op::R* __restrict__ F4,
                                                  const MPInfo* __restrict__ mpi,
                                                  const WorkItem* __restrict__ items, int RB,
                                                  int CBs, int CBn, int ncols, int nf, int J,
                                                  int L) {
  const WorkItem it = items[blockIdx.x];
  const MPInfo q = mpi[it.mp];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rb0 = it.tile * 4 + (wave >> 1) * 2;
  const int cb0 = blockIdx.y * 4 + (wave & 1) * 2;
  if (rb0 >= RB || cb0 >= CBn) return;  // whole wave idle (no barriers in this kernel)
  const bool r1 = rb0 + 1 < RB, c1 = cb0 + 1 < CBn;
  typename Op::C acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
  long long ta = q.tabS + rb0;
  long long xb = q.xS + cb0;
  for (int kb = 0; kb < q.kbS; ++kb, ta += RB, xb += CBs) {
    typename Op::A a0 = Op::load(tab, ta, lane);
    typename Op::A b0 = Op::load(X, xb, lane);
    typename Op::A a1 = r1 ? Op::load(tab, ta + 1, lane) : Op::zero();
    typename Op::A b1 = c1 ? Op::load(X, xb + 1, lane) : Op::zero();
    acc00 = Op::mma(a0, b0, acc00);
    if (c1) acc01 = Op::mma(a0, b1, acc01);
    if (r1) acc10 = Op::mma(a1, b0, acc10);
    if (r1 && c1) acc11 = Op::mma(a1, b1, acc11);
  }
  auto put = [&](const typename Op::C& acc, int rb, int cb) {
    const int c = cb * 16 + (lane & 15);
    if (c >= ncols) return;
    const int ri = c & 1, bf = c >> 1, f = bf % nf, b = bf / nf;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = rb * 16 + Op::row(lane, v);
      if (j < J)
        F4[(((((size_t)b * J + j) * nf + f) * 2 + q.p) * L + q.m) * 2 + ri] =
            (typename Op::R)acc[v];
    }
  };
  put(acc00, rb0, cb0);
  if (c1) put(acc01, rb0, cb0 + 1);
  if (r1) put(acc10, rb0 + 1, cb0);
  if (r1 && c1) put(acc11, rb0 + 1, cb0 + 1);
}

template <class Op>
__global__ __launch_bounds__(256) void k_leg_anal(const void* __restrict__ tab,
                                                 const void* __restrict__ G,
                                                 typename Op::R* __restrict__ Y,
                                                 const MPInfo* __restrict__ mpi,
                                                 const WorkItem* __restrict__ items, int kb2,
                                                 int CBa, int CBn, int ncols, int Kx, int T) {
  const WorkItem it = items[blockIdx.x];
  const MPInfo q = mpi[it.mp];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rb0 = it.tile * 4 + (wave >> 1) * 2;
  const int cb0 = blockIdx.y * 4 + (wave & 1) * 2;
  if (rb0 >= q.rbA || cb0 >= CBn) return;
  const bool r1 = rb0 + 1 < q.rbA, c1 = cb0 + 1 < CBn;
  typename Op::C acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
  long long ta = q.tabA + rb0;
  long long gb = (long long)it.mp * kb2 * CBa + cb0;
  for (int kb = 0; kb < kb2; ++kb, ta += q.rbA, gb += CBa) {
    typename Op::A a0 = Op::load(tab, ta, lane);
    typename Op::A b0 = Op::load(G, gb, lane);
    typename Op::A a1 = r1 ? Op::load(tab, ta + 1, lane) : Op::zero();
    typename Op::A b1 = c1 ? Op::load(G, gb + 1, lane) : Op::zero();
    acc00 = Op::mma(a0, b0, acc00);
    if (c1) acc01 = Op::mma(a0, b1, acc01);
    if (r1) acc10 = Op::mma(a1, b0, acc10);
    if (r1 && c1) acc11 = Op::mma(a1, b1, acc11);
  }
  const int base = ext_off(T, q.m);
  auto put = [&](const typename Op::C& acc, int rb, int cb) {
    const int c = cb * 16 + (lane & 15);
    if (c >= ncols) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = rb * 16 + Op::row(lane, v);
      if (i < q.np)
        Y[((size_t)(c >> 1) * Kx + base + q.p + 2 * i) * 2 + (c & 1)] = (typename Op::R)acc[v];
    }
  };
  put(acc00, rb0, cb0);
  if (c1) put(acc01, rb0, cb0 + 1);
  if (r1) put(acc10, rb0 + 1, cb0);
  if (r1 && c1) put(acc11, rb0 + 1, cb0 + 1);
}

template <class Op>
static hipError_t synth_impl(const pfsh_level* lv, int ncols, int nf, hipStream_t s) {
  const int CBn = (ncols + 15) / 16;
  dim3 grid(lv->nitemsS, (CBn + 3) / 4);
  hipLaunchKernelGGL(k_leg_synth<Op>, grid, dim3(256), 0, s, lv->tabS, lv->X,
                     (typename Op::R*)lv->F4, lv->mp_d, lv->itemsS, lv->RB, lv->CBs, CBn, ncols,
                     nf, lv->J, lv->L);
  return hipGetLastError();
}

template <class Op>
static hipError_t anal_impl(const pfsh_level* lv, int ncols, hipStream_t s) {
  const int CBn = (ncols + 15) / 16;
  dim3 grid(lv->nitemsA, (CBn + 3) / 4);
  hipLaunchKernelGGL(k_leg_anal<Op>, grid, dim3(256), 0, s, lv->tabA, lv->G,
                     (typename Op::R*)lv->Y, lv->mp_d, lv->itemsA, lv->kb2, lv->CBa, CBn, ncols,
                     lv->Kx, lv->T);
  return hipGetLastError();
}

hipError_t launch_leg_synth(const pfsh_level* lv, int ncols, int nf, hipStream_t s) {
  switch (lv->op) {
    case OP_F64: return synth_impl<OpF64>(lv, ncols, nf, s);
    case OP_F32: return synth_impl<OpF32>(lv, ncols, nf, s);
    default: return synth_impl<OpBF3>(lv, ncols, nf, s);
  }
}

hipError_t launch_leg_anal(const pfsh_level* lv, int ncols, int /*nf*/, hipStream_t s) {
  switch (lv->op) {
    case OP_F64: return anal_impl<OpF64>(lv, ncols, s);
    case OP_F32: return anal_impl<OpF32>(lv, ncols, s);
    default: return anal_impl<OpBF3>(lv, ncols, s);
  }
}

}  // namespace pfsh
