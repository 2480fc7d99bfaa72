// FP64 spectral-space kernels: transform pre/post steps, the linear operator
// and implicit solve, the SDC sweep accumulation, the collocation residual and
// the space-time transfers.  All are bandwidth-bound element-wise passes over
// [batch][...][3][K] complex128 arrays.
#include <mutex>

#include "mfma_ops.h"

namespace pfsh {

struct C2 {
  double x, y;
};
__device__ __forceinline__ C2 ld2(const double* p) {
  const double2 v = *reinterpret_cast<const double2*>(p);
  return {v.x, v.y};
}
__device__ __forceinline__ void st2(double* p, C2 v) {
  *reinterpret_cast<double2*>(p) = make_double2(v.x, v.y);
}

__device__ __forceinline__ double eps_nm(int n, int m) {
  return n > m ? sqrt((double)(n * n - m * m) / (double)(4 * n * n - 1)) : 0.0;
}

// slot k -> (m, n) of the m-major layout
__device__ __forceinline__ void slot_mn(int T, int k, int& m, int& n) {
  const double b = 2.0 * T + 3.0;
  int mm = (int)((b - sqrt(b * b - 8.0 * k)) * 0.5);
  if (mm < 0) mm = 0;
  while (mm > 0 && spec_off(T, mm) > k) --mm;
  while (mm < T && spec_off(T, mm + 1) <= k) ++mm;
  m = mm;
  n = mm + (k - spec_off(T, mm));
}

struct Phys {
  double a, omega, phibar, nu;
};

// -------------------------------------------------------------- RHS prep
// Synthesis data operand of the four fields Phi', zeta, U, V at degree
// n' = m..T+1 of order m (Sec. 2-3):
//   Phi'_n' = Phi_n' (minus sqrt(2) Phibar at (0,0)), zeta_n'      (0 at n' = T+1)
//   U_n' = (1/a) [ i m chi_n' - psit_n' ],  V_n' = (1/a) [ i m psi_n' + chit_n' ]
//   psit_n' = -(n'-1) eps_n' psi_{n'-1} + (n'+2) eps_{n'+1} psi_{n'+1}
// (the H_n^m = (1-mu^2) dP_n^m/dmu terms rewritten on P_{n'}), with
// psi = -a^2 zeta/(n(n+1)), chi = -a^2 delta/(n(n+1)) (Helmholtz, Sec. 2).
// `get(v, nn)` returns variable v (0 Phi, 1 zeta, 2 delta) at degree nn of
// order m, for m <= nn <= T.
template <class Get>
__device__ __forceinline__ void prep_fields(Get get, int m, int n, int T, Phys ph, C2 out[4]) {
  const double ia = 1.0 / ph.a, a2 = ph.a * ph.a;
  auto inv_lap = [&](int v, int nn) -> C2 {
    if (nn < m || nn > T || nn == 0) return {0.0, 0.0};
    const C2 z = get(v, nn);
    const double sc = -a2 / ((double)nn * (nn + 1));
    return {sc * z.x, sc * z.y};
  };
  C2 phi = {0, 0}, zeta = {0, 0};
  if (n <= T) {
    phi = get(0, n);
    zeta = get(1, n);
  }
  if (n == 0) phi.x -= 1.4142135623730950488 * ph.phibar;
  const double e0 = eps_nm(n, m), e1 = eps_nm(n + 1, m);
  const C2 ps_m = inv_lap(1, n - 1), ps_p = inv_lap(1, n + 1), ps_0 = inv_lap(1, n);
  const C2 ch_m = inv_lap(2, n - 1), ch_p = inv_lap(2, n + 1), ch_0 = inv_lap(2, n);
  const double cm = -(double)(n - 1) * e0, cp = (double)(n + 2) * e1;
  const C2 pst = {cm * ps_m.x + cp * ps_p.x, cm * ps_m.y + cp * ps_p.y};
  const C2 cht = {cm * ch_m.x + cp * ch_p.x, cm * ch_m.y + cp * ch_p.y};
  // i m chi = (-m chi.y, m chi.x)
  out[0] = phi;
  out[1] = zeta;
  out[2] = {ia * (-m * ch_0.y - pst.x), ia * (m * ch_0.x - pst.y)};
  out[3] = {ia * (-m * ps_0.y + cht.x), ia * (m * ps_0.x + cht.y)};
}

// Store the 16 columns (2 slices x 4 fields x re/im) of degree n of order m
// into the synthesis data operand.
template <class Op>
__device__ __forceinline__ void store_operand(void* X, const MPInfo* __restrict__ mpi, int m, int n,
                                              int CBs, int b0, const typename Op::R* vals) {
  typedef typename Op::R R;
  const int p = (n - m) & 1, i = (n - m) >> 1;
  const MPInfo q = mpi[2 * m + p];
  const int KB = Op::KB;
  const long long blk = q.xS + (long long)(i / KB) * CBs + (b0 * 8) / 16;
  const int kk = i % KB;
  if constexpr (Op::KIND == OP_BF16X3) {
#pragma unroll
    for (int c = 0; c < 16; ++c) Op::store(X, blk, (kk >> 3) * 16 + c, kk & 7, vals[c]);
  } else {
    R* dst = reinterpret_cast<R*>(X) + blk * 64 + kk * 16;   // 16 consecutive lanes
    if constexpr (sizeof(R) == 4) {
#pragma unroll
      for (int c = 0; c < 16; c += 4)
        *reinterpret_cast<float4*>(dst + c) = make_float4(vals[c], vals[c + 1], vals[c + 2], vals[c + 3]);
    } else {
#pragma unroll
      for (int c = 0; c < 16; c += 2)
        *reinterpret_cast<double2*>(dst + c) = make_double2(vals[c], vals[c + 1]);
    }
  }
}

// F_I = L(Theta) of one mode (Sec. 2): lam = -n(n+1)/a^2.
__device__ __forceinline__ void linear_mode(double lam, Phys ph, C2 p, C2 z, C2 d, C2 out[3]) {
  out[0] = {-ph.phibar * d.x + ph.nu * lam * p.x, -ph.phibar * d.y + ph.nu * lam * p.y};
  out[1] = {ph.nu * lam * z.x, ph.nu * lam * z.y};
  out[2] = {-lam * p.x + ph.nu * lam * d.x, -lam * p.y + ph.nu * lam * d.y};
}

// One workgroup per (m, pair of slices): the synthesis operand of the states
// (and optionally F_I = L(Theta) per mode).
template <class Op>
__global__ __launch_bounds__(128) void k_prep_rhs(const double* __restrict__ th, long long sstride,
                                                 double* __restrict__ fi, long long fstride,
                                                 void* __restrict__ X, const MPInfo* __restrict__ mpi,
                                                 int T, int CBs, int batch, Phys ph) {
  typedef typename Op::R R;
  const int m = blockIdx.x, b0 = 2 * blockIdx.y;   // two slices per workgroup: 16 columns
  const int K = (T + 1) * (T + 2) / 2;
  const int off = spec_off(T, m);
  for (int n = m + threadIdx.x; n <= T + 1; n += blockDim.x) {
    R vals[16];
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const int b = b0 + bb;
      C2 v4[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
      if (b < batch) {
        const double* P = th + (size_t)b * sstride * 2;
        auto get = [&](int v, int nn) { return ld2(P + 2 * ((size_t)v * K + off + nn - m)); };
        if (fi && n <= T) {
          const double lam = -(double)n * (n + 1) / (ph.a * ph.a);
          C2 f[3];
          linear_mode(lam, ph, get(0, n), get(1, n), get(2, n), f);
          double* F = fi + (size_t)b * fstride * 2;
          for (int v = 0; v < 3; ++v) st2(F + 2 * ((size_t)v * K + off + n - m), f[v]);
        }
        prep_fields(get, m, n, T, ph, v4);
      }
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        vals[bb * 8 + 2 * f] = (R)v4[f].x;
        vals[bb * 8 + 2 * f + 1] = (R)v4[f].y;
      }
    }
    store_operand<Op>(X, mpi, m, n, CBs, b0, vals);
  }
}

// scalar synthesis input: nfields spectra [f][K] -> operand (degree T+1 = 0)
template <class Op>
__global__ __launch_bounds__(128) void k_prep_scalar(const double* __restrict__ spec,
                                                    void* __restrict__ X,
                                                    const MPInfo* __restrict__ mpi, int T,
                                                    int CBs) {
  const int m = blockIdx.x, f = blockIdx.y;
  const int K = (T + 1) * (T + 2) / 2, off = spec_off(T, m);
  for (int n = m + threadIdx.x; n <= T + 1; n += blockDim.x) {
    C2 z = {0, 0};
    if (n <= T) z = ld2(spec + 2 * ((size_t)f * K + off + n - m));
    const int p = (n - m) & 1, i = (n - m) >> 1;
    const MPInfo q = mpi[2 * m + p];
    const int KB = Op::KB;
    const long long blk0 = q.xS + (long long)(i / KB) * CBs;
    const int kk = i % KB;
    const int e = (Op::KIND == OP_BF16X3) ? (kk & 7) : 0;
    const int lk = (Op::KIND == OP_BF16X3) ? (kk >> 3) : kk;
    const int c = 2 * f;
    Op::store(X, blk0 + c / 16, lk * 16 + (c % 16), e, (typename Op::R)z.x);
    Op::store(X, blk0 + (c + 1) / 16, lk * 16 + ((c + 1) % 16), e, (typename Op::R)z.y);
  }
}

// scalar analysis output: Y [f][Kx] -> spec [f][K], Im of m = 0 set to 0
template <typename R>
__global__ void k_unpack_scalar(const R* __restrict__ Y, double* __restrict__ spec, int T,
                                int nf) {
  const int K = (T + 1) * (T + 2) / 2, Kx = ext_off(T, T + 1);
  const long long tot = (long long)nf * K;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int f = (int)(idx / K), k = (int)(idx - (long long)f * K);
    int m, n;
    slot_mn(T, k, m, n);
    const R* y = Y + 2 * ((size_t)f * Kx + ext_pos(T, m, n));
    st2(spec + 2 * idx, {(double)y[0], m == 0 ? 0.0 : (double)y[1]});
  }
}

// -------------------------------------------------------------- assembly
// F_E from the analysed products (Sec. 2, transform method):
//   D[X,Y]_n = (1/a) [ i m X_n - ( -n eps_{n+1} Y_{n+1} + (n+1) eps_n Y_{n-1} ) ]
//   N_zeta = -D[A,B], N_delta = D[B,-A] + n(n+1)/a^2 E_n, N_Phi = -D[C,D]
// where X_n, Y_n are the weighted P-contractions (degrees to T+1) of one slice;
// get(f, n) returns product f at degree n (0 outside m..T+1).
template <class GetY>
__device__ __forceinline__ void assemble_core(GetY get, int m, int n, double a, C2 out[3]) {
  const double ia = 1.0 / a;
  const double cp = -(double)n * eps_nm(n + 1, m), cm = (double)(n + 1) * eps_nm(n, m);
  // H-weighted parts: hY = cp Y_{n+1} + cm Y_{n-1}
  const C2 An = get(0, n), Bn = get(1, n), Cn = get(2, n), En = get(4, n);
  const C2 Ap = get(0, n + 1), Am = get(0, n - 1);
  const C2 Bp = get(1, n + 1), Bm = get(1, n - 1);
  const C2 Dp = get(3, n + 1), Dm = get(3, n - 1);
  const C2 hB = {cp * Bp.x + cm * Bm.x, cp * Bp.y + cm * Bm.y};
  const C2 hA = {cp * Ap.x + cm * Am.x, cp * Ap.y + cm * Am.y};
  const C2 hD = {cp * Dp.x + cm * Dm.x, cp * Dp.y + cm * Dm.y};
  // D[X,Y] = (1/a)(i m X - hY);  i m X = (-m X.y, m X.x)
  const C2 dAB = {ia * (-m * An.y - hB.x), ia * (m * An.x - hB.y)};
  const C2 dBmA = {ia * (-m * Bn.y + hA.x), ia * (m * Bn.x + hA.y)};
  const C2 dCD = {ia * (-m * Cn.y - hD.x), ia * (m * Cn.x - hD.y)};
  const double ke = (double)n * (n + 1) * ia * ia;
  out[0] = {-dCD.x, -dCD.y};
  out[1] = {-dAB.x, -dAB.y};
  out[2] = {dBmA.x + ke * En.x, dBmA.y + ke * En.y};
  if (m == 0) {
    out[0].y = 0;
    out[1].y = 0;
    out[2].y = 0;
  }
}

// Products of one slice in global memory, Yb = [5 products][Kx] complex, each
// order's degrees parity-split from eoff = ext_off(T, m) (ext_pos).
template <typename R>
__device__ __forceinline__ void assemble_mode(const R* __restrict__ Yb, int Kx, int eoff, int m,
                                              int n, int T, double a, C2 out[3]) {
  const int np0 = npar(T, m, 0);
  // degrees outside m..T+1 read 0; the load itself goes to degree m (in
  // range) and is discarded, so no load sits behind a branch
  auto get = [&](int f, int nn) -> C2 {
    const bool in = nn >= m && nn <= T + 1;
    const int q = in ? nn - m : 0;
    const R* p = Yb + 2 * ((size_t)f * Kx + eoff + (q & 1 ? np0 : 0) + (q >> 1));
    const double x = (double)p[0], y = (double)p[1];
    return C2{in ? x : 0.0, in ? y : 0.0};
  };
  assemble_core(get, m, n, a, out);
}

// One workgroup per (pair of orders, slice): order g goes with order T + 1 - g
// (as in k_sweep_step), so that every workgroup has about T + 2 modes.
template <typename R>
__global__ __launch_bounds__(256) void k_assemble(const R* __restrict__ Y, double* __restrict__ fe,
                                                 long long fstride, int T, double a) {
  const int L = T + 1, g = blockIdx.x, b = blockIdx.y;
  const int ma = g, mb = (g >= 1 && L - g > g) ? L - g : -1;
  const int na = L - ma, nb = mb >= 0 ? L - mb : 0;
  const int K = (T + 1) * (T + 2) / 2, Kx = ext_off(T, T + 1);
  const R* Yb = Y + (size_t)b * 5 * Kx * 2;
  double* F = fe + (size_t)b * fstride * 2;
  for (int t = threadIdx.x; t < na + nb; t += blockDim.x) {
    const bool first = t < na;
    const int m = first ? ma : mb, n = m + (first ? t : t - na);
    C2 o[3];
    assemble_mode(Yb, Kx, ext_off(T, m), m, n, T, a, o);
    const int off = spec_off(T, m);
    for (int v = 0; v < 3; ++v) st2(F + 2 * ((size_t)v * K + off + n - m), o[v]);
  }
}

// -------------------------------------------------------------- implicit
__device__ __forceinline__ void solve_mode(double lam, double beta, Phys ph, C2 bp, C2 bz, C2 bd,
                                           C2& xp, C2& xz, C2& xd) {
  const double d = 1.0 - beta * ph.nu * lam;
  const double det = d * d - beta * beta * ph.phibar * lam;
  const double id = 1.0 / d, idet = 1.0 / det;
  xz = {bz.x * id, bz.y * id};
  xp = {(d * bp.x - beta * ph.phibar * bd.x) * idet, (d * bp.y - beta * ph.phibar * bd.y) * idet};
  xd = {(d * bd.x - beta * lam * bp.x) * idet, (d * bd.y - beta * lam * bp.y) * idet};
}

__global__ void k_implicit_solve(const double* __restrict__ bv, double* __restrict__ x, int T,
                                 int batch, double beta, Phys ph) {
  const int K = (T + 1) * (T + 2) / 2;
  const long long tot = (long long)batch * K;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(idx / K), k = (int)(idx - (long long)b * K);
    int m, n;
    slot_mn(T, k, m, n);
    const double lam = -(double)n * (n + 1) / (ph.a * ph.a);
    const double* B = bv + (size_t)b * 3 * K * 2;
    C2 xp, xz, xd;
    solve_mode(lam, beta, ph, ld2(B + 2 * k), ld2(B + 2 * (K + k)), ld2(B + 2 * (2 * K + k)), xp,
               xz, xd);
    double* X = x + (size_t)b * 3 * K * 2;
    st2(X + 2 * k, xp);
    st2(X + 2 * (K + k), xz);
    st2(X + 2 * (2 * K + k), xd);
  }
}

// -------------------------------------------------------------- SDC sweep
struct SdcMat {
  double Q[81], QE[81], QI[81];
  int nn;
  int split;   // implicit step in two substeps (physical linear, then diffusion)
};

// Node-0 values received from elsewhere (state, F_E, F_I), as raw pointers;
// fe_pending (fused node kernel only): F_E there is assembled first, into this
// array (the same as fe), from the level's current ring output.
struct SrcPtrs {
  const double* th;
  const double* fe;
  const double* fi;
  long long stride;   // complex values between batch entries
  double* fe_pending;
};

// One node of the IMEX sweep in Q form (Sec. 5.1.1, eq.
// update_equation_sdcq_discrete_form), node = 1..M, for
// one mode k = (m, n) of slice b of [batch][nn][3][K] arrays:
//  node == 1: (optionally first taking node 0 -- state, F_E, F_I -- from src
//      and storing it) S_i = Theta^0 + dt sum_j Q_ij (F_E^j + F_I^j)
//        - dt sum_{j=1}^{i-1} qE_ij F_E^j - dt sum_{j=1}^{i} qI_ij F_I^j + tau_i
//      for i = 1..M, every term of the node-i update that uses only the
//      previous iterate (S_i of i >= 2 kept in S for the later nodes);
//  then b = S_node + dt sum_{j=1}^{node-1} (qE F_E^j + qI F_I^j) (new F), the
//  implicit solve with beta = dt qI_{node,node}, Theta^node and
//  F_I^node = L Theta^node, stored; returns Theta^node.
// ND > 0 fixes the node at compile time (node_rt is then ignored): for a node
// >= 2 every load of the mode (S and F_E, F_I of the earlier nodes, all three
// variables) is issued before any arithmetic, one memory round trip instead of
// one per term, and fe_prev (if given) holds F_E of node - 1 for the three
// variables, already in registers.  Each term is fma(qE, F_E, qI F_I), added
// in order j = 1, 2, ..., so both forms give the same bits.
template <int NN, int ND = 0>
__device__ __forceinline__ void node_update(double* __restrict__ th, double* __restrict__ fe,
                                            double* __restrict__ fi, const double* __restrict__ tau,
                                            double* __restrict__ S, const SrcPtrs& src, int K,
                                            int b, int k, int n, int node_rt, double dt,
                                            const SdcMat& sm, const Phys& ph, C2 x[3],
                                            const C2* fe_prev = nullptr) {
  constexpr int nn = NN, M = NN - 1;
  const int node = ND > 0 ? ND : node_rt;
  const double lam = -(double)n * (n + 1) / (ph.a * ph.a);
  const double beta = dt * sm.QI[node * nn + node];
  const size_t base = (size_t)b * nn * 3 * K;
  C2 rhs[3];
  if constexpr (ND >= 2) {
    C2 E[3][ND], F[3][ND];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const size_t vk = (size_t)v * K + k;
      rhs[v] = ld2(S + 2 * (((size_t)b * M + (ND - 1)) * 3 * K + vk));
#pragma unroll
      for (int j = 1; j < ND; ++j) {
        const size_t o = base + (size_t)j * 3 * K + vk;
        E[v][j] = (fe_prev && j == ND - 1) ? fe_prev[v] : ld2(fe + 2 * o);
        F[v][j] = ld2(fi + 2 * o);
      }
    }
    __builtin_amdgcn_sched_barrier(0);   // keep the loads above, all in flight
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int j = 1; j < ND; ++j) {
        const double ce = dt * sm.QE[ND * nn + j], ci = dt * sm.QI[ND * nn + j];
        rhs[v].x += fma(ce, E[v][j].x, ci * F[v][j].x);
        rhs[v].y += fma(ce, E[v][j].y, ci * F[v][j].y);
      }
  } else
  for (int v = 0; v < 3; ++v) {
    const size_t vk = (size_t)v * K + k;
    C2 r;
    if (node == 1) {
      C2 E[NN], I[NN];
#pragma unroll
      for (int j = 0; j < nn; ++j) {
        E[j] = ld2(fe + 2 * (base + (size_t)j * 3 * K + vk));
        I[j] = ld2(fi + 2 * (base + (size_t)j * 3 * K + vk));
      }
      C2 t0;
      if (src.th) {   // node 0 received from src (state and F there), stored first
        const size_t so = 2 * ((size_t)b * src.stride + vk);
        t0 = ld2(src.th + so);
        E[0] = ld2(src.fe + so);
        I[0] = ld2(src.fi + so);
        st2(th + 2 * (base + vk), t0);
        st2(fe + 2 * (base + vk), E[0]);
        st2(fi + 2 * (base + vk), I[0]);
      } else {
        t0 = ld2(th + 2 * (base + vk));
      }
#pragma unroll
      for (int i = 1; i <= M; ++i) {
        double sx = 0, sy = 0;
#pragma unroll
        for (int j = 0; j < nn; ++j) {
          const double c = sm.Q[i * nn + j];
          sx += c * (E[j].x + I[j].x);
          sy += c * (E[j].y + I[j].y);
        }
#pragma unroll
        for (int j = 1; j < i; ++j) {
          sx -= sm.QE[i * nn + j] * E[j].x;
          sy -= sm.QE[i * nn + j] * E[j].y;
        }
#pragma unroll
        for (int j = 1; j <= i; ++j) {
          sx -= sm.QI[i * nn + j] * I[j].x;
          sy -= sm.QI[i * nn + j] * I[j].y;
        }
        C2 si = {t0.x + dt * sx, t0.y + dt * sy};
        if (tau) {
          const C2 tv = ld2(tau + 2 * (base + (size_t)i * 3 * K + vk));
          si.x += tv.x;
          si.y += tv.y;
        }
        if (i == 1)
          r = si;
        else
          st2(S + 2 * (((size_t)b * M + (i - 1)) * 3 * K + vk), si);
      }
    } else {
      r = ld2(S + 2 * (((size_t)b * M + (node - 1)) * 3 * K + vk));
      auto term = [&](int j) {
        const size_t o = base + (size_t)j * 3 * K + vk;
        const C2 e = ld2(fe + 2 * o), f = ld2(fi + 2 * o);
        const double ce = dt * sm.QE[node * nn + j], ci = dt * sm.QI[node * nn + j];
        r.x += fma(ce, e.x, ci * f.x);
        r.y += fma(ce, e.y, ci * f.y);
      };
      for (int j = 1; j < node; ++j) term(j);
    }
    rhs[v] = r;
  }
  if (sm.split) {
    // Two substeps (Sec. 5.1.1, last paragraph): L = L1 + L2 with L1 the
    // physical linear terms and L2 = nu lap.  Theta* = (I - beta L1)^{-1}
    // (b + beta L2 Theta_old), then Theta = (I - beta L2)^{-1} (Theta* - beta
    // L2 Theta_old), Theta_old the previous iterate at this node.
    C2 o[3], bs[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) o[v] = ld2(th + 2 * (base + ((size_t)node * 3 + v) * K + k));
    const double dl = ph.nu * lam;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      o[v] = {dl * o[v].x, dl * o[v].y};                       // L2 Theta_old
      bs[v] = {rhs[v].x + beta * o[v].x, rhs[v].y + beta * o[v].y};
    }
    const double det = 1.0 - beta * beta * ph.phibar * lam, idet = 1.0 / det;
    const C2 s0 = {(bs[0].x - beta * ph.phibar * bs[2].x) * idet, (bs[0].y - beta * ph.phibar * bs[2].y) * idet};
    const C2 s2 = {(bs[2].x - beta * lam * bs[0].x) * idet, (bs[2].y - beta * lam * bs[0].y) * idet};
    const C2 xs[3] = {s0, bs[1], s2};
    const double id = 1.0 / (1.0 - beta * dl);
#pragma unroll
    for (int v = 0; v < 3; ++v)
      x[v] = {(xs[v].x - beta * o[v].x) * id, (xs[v].y - beta * o[v].y) * id};
  } else {
    solve_mode(lam, beta, ph, rhs[0], rhs[1], rhs[2], x[0], x[1], x[2]);
  }
  C2 f[3];
  linear_mode(lam, ph, x[0], x[1], x[2], f);
  for (int v = 0; v < 3; ++v) {
    const size_t o = base + ((size_t)node * 3 + v) * K + k;
    st2(th + 2 * o, x[v]);
    st2(fi + 2 * o, f[v]);
  }
}

// One sweep node fused with the passes that border it:
//  (a) asm_node >= 0: F_E at node asm_node from the analysed products Y;
//  (b) node_update (node 1 also accumulates the old-iterate terms);
//  (c) the synthesis operand of Theta^node (prep_fields), reading the new
//      states of this order from LDS.
// One workgroup of 512 threads per (pair of orders, pair of slices): order g
// goes with order T + 1 - g, so that every workgroup holds T + 1 degrees per
// slice (order 0 and, for even T + 1, order (T + 1) / 2 stand alone).  The
// (slice, order, degree) items of (a)-(b) are spread over all threads, (c)
// takes one (order, degree) per thread.
template <class Op, int NN, int ND>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(NN <= 5 ? 4 : 1, ND > 1 ? 4 : 8)))
void k_sweep_step(double* __restrict__ th, double* __restrict__ fe,
                                                   double* __restrict__ fi,
                                                   const double* __restrict__ tau,
                                                   double* __restrict__ S,
                                                   const typename Op::R* __restrict__ Y,
                                                   void* __restrict__ X,
                                                   const MPInfo* __restrict__ mpi, int T, int CBs,
                                                   int batch, int node, int asm_node, double dt,
                                                   SdcMat sm, Phys ph, SrcPtrs src) {
  typedef typename Op::R R;
  constexpr int nn = NN;
  extern __shared__ unsigned char smem_raw[];
  C2* sh = reinterpret_cast<C2*>(smem_raw);            // [2 slices][3 vars][T+1]: order a, then b
  const int L = T + 1, g = blockIdx.x, b0 = 2 * blockIdx.y;
  const int ma = g, mb = (g >= 1 && L - g > g) ? L - g : -1;   // mb < 0: no second order
  const int na = L - ma, nb = mb >= 0 ? L - mb : 0;    // degrees of each order
  const int K = (T + 1) * (T + 2) / 2, Kx = ext_off(T, T + 1);
  const int nsl = min(2, batch - b0);                  // slices of this workgroup
  const int per = na + nb;
  for (int it = threadIdx.x; it < nsl * per; it += blockDim.x) {
    const int bb = it / per, idx = it - bb * per;
    const bool first = idx < na;
    const int m = first ? ma : mb, n = m + (first ? idx : idx - na);
    const int b = b0 + bb;
    const int k = spec_off(T, m) + n - m;
    // a compile-time node >= 2 always assembles F_E of node - 1 first
    const int an = ND >= 2 ? ND - 1 : asm_node;
    C2 o[3];
    if (an >= 0) {
      assemble_mode(Y + (size_t)b * 5 * Kx * 2, Kx, ext_off(T, m), m, n, T, ph.a, o);
      const size_t base = (size_t)b * nn * 3 * K;
      for (int v = 0; v < 3; ++v) st2(fe + 2 * (base + ((size_t)an * 3 + v) * K + k), o[v]);
    }
    C2 x[3];
    node_update<NN, ND>(th, fe, fi, tau, S, src, K, b, k, n, node, dt, sm, ph, x,
                        ND >= 2 ? o : nullptr);
    for (int v = 0; v < 3; ++v) sh[(bb * 3 + v) * L + idx] = x[v];
  }
  __syncthreads();
  // degrees m..T+1 of each order (T+1 is the extra degree of the vector terms)
  for (int t = threadIdx.x; t < (na + 1) + (nb > 0 ? nb + 1 : 0); t += blockDim.x) {
    const bool first = t <= na;
    const int m = first ? ma : mb, n = m + (first ? t : t - (na + 1));
    const int base = first ? 0 : na;                   // this order's LDS offset
    R vals[16];
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      C2 v4[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
      if (b0 + bb < batch) {
        auto get = [&](int v, int q) { return sh[(bb * 3 + v) * L + base + (q - m)]; };
        prep_fields(get, m, n, T, ph, v4);
      }
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        vals[bb * 8 + 2 * f] = (R)v4[f].x;
        vals[bb * 8 + 2 * f + 1] = (R)v4[f].y;
      }
    }
    store_operand<Op>(X, mpi, m, n, CBs, b0, vals);
  }
}

// ------------------------------------------------ fused node for small batches
// With one or two slices the serial coarse chain is bound by kernel latency,
// so one workgroup takes one order m through every stage but the ring stage:
//  (1) asm_node >= 0: the Legendre analysis of order m (both parities, all
//      degrees and columns) into LDS, then F_E at node asm_node;
//  (2) node >= 1: node_update of every degree, the new states into LDS;
//  (3) node >= 1: the synthesis operand of order m in LDS, then the Legendre
//      synthesis of order m (both parities, all rings) into the Fourier
//      workspace.
// The contractions use the MFMA fragments and K order of k_leg_anal /
// k_leg_synth (synthesis from the highest degree down), and every spectral
// step the expressions of the separate kernels, so the results are the same
// bits.  FP64 and FP32 transform types.  16 waves per workgroup: the heaviest
// orders (m near 0) have up to ~2 x (T/32) MFMA blocks per contraction, which
// then run side by side instead of in rounds of one K chain after another.
// Workgroup -> order for the fused node.  Workgroups are dealt to the 8 XCDs in
// turn (workgroup b to XCD b mod 8); this bijection gives each XCD whole groups
// of 8 consecutive orders, so that the runs of the Fourier workspace (4 or 8
// consecutive orders of one field and ring) are written whole through one
// XCD's L2 instead of in pieces through several.  With a multiple of 128
// orders, XCD x takes groups x and 15 - x of every 16 (a heavy and a light
// group, as the orders' degree counts fall with m); else one range of
// consecutive orders.
__device__ __forceinline__ int xcd_order(int b, int n) {
  constexpr int NX = 8;
  const int x = b % NX, l = b / NX;
  if (n % 128 == 0) {
    const int s = l / 8, g = 16 * (s / 2) + ((s & 1) ? 15 - x : x);
    return 8 * g + (l & 7);
  }
  const int q = n / NX, r = n % NX;
  return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

template <class Op, int NN>
__global__ __launch_bounds__(1024) void k_node_fused(double* __restrict__ th, double* __restrict__ fe,
                                                   double* __restrict__ fi,
                                                   const double* __restrict__ tau,
                                                   double* __restrict__ S,
                                                   const void* __restrict__ tabA,
                                                   const void* __restrict__ G,
                                                   const void* __restrict__ tabS,
                                                   typename Op::R* __restrict__ F4,
                                                   const MPInfo* __restrict__ mpi, int T, int J,
                                                   int Lp, int kb2, int CBa, int RB, int kbmax,
                                                   int batch, int node, int asm_node, double dt,
                                                   SdcMat sm, Phys ph, SrcPtrs src) {
  typedef typename Op::R R;
  constexpr int nn = NN, PF = 4;
  const int m = xcd_order(blockIdx.x, gridDim.x);   // gridDim.x = T + 1
  const int K = (T + 1) * (T + 2) / 2;
  const int off = spec_off(T, m), nm = T + 1 - m, nx = T + 2 - m;
  const int nsl = batch;                               // 1 or 2 slices
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int NW = 16;   // waves
  extern __shared__ unsigned char smem_raw[];
  C2* sh = reinterpret_cast<C2*>(smem_raw);                     // [2][3][T+1]
  R* Yl = reinterpret_cast<R*>(sh + 2 * 3 * (T + 1));          // [20 columns][T+2]
  R* Xl = Yl + 20 * (T + 2);                                    // [2 parities][kbmax][64]
  for (int i = threadIdx.x; i < 2 * kbmax * 64; i += blockDim.x) Xl[i] = (R)0;

  const bool asm_src = src.fe_pending != nullptr;   // with node 1 only (asm_node < 0)
  if (asm_node >= 0 || asm_src) {
    // (1) analysis: 16 x 16 blocks (parity, degree block, column block)
    const int ncols = 10 * nsl, CBn = (ncols + 15) / 16;
    const MPInfo q0 = mpi[2 * m], q1 = mpi[2 * m + 1];
    const int ntask = (q0.rbA + q1.rbA) * CBn;
    for (int t = wave; t < ntask; t += NW) {
      const int cb = t % CBn, r = t / CBn;
      const int p = r < q0.rbA ? 0 : 1, rb = p ? r - q0.rbA : r;
      const MPInfo& q = p ? q1 : q0;
      typename Op::C acc = {}, d1 = {}, d2 = {}, d3 = {};
      constexpr int KG = KGroup<Op>::KG;   // k-grouped analysis table
      mma_loop_grp<Op, PF / 2>(tabA, G, q.tabA / KG + rb, (long long)q.rbA,
                               (long long)(2 * m + p) * kb2 * CBa + cb, (long long)CBa, kb2 / KG,
                               0, false, false, lane, acc, d1, d2, d3);
      const int c = cb * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = rb * 16 + Op::row(lane, v);
        if (i < q.np && c < ncols) Yl[c * nx + p + 2 * i] = (R)acc[v];
      }
    }
    __syncthreads();
  }
  for (int it = threadIdx.x; it < nsl * nm; it += blockDim.x) {
    const int bb = it / nm, n = m + (it - bb * nm);
    const int k = off + n - m;
    if (asm_node >= 0 || asm_src) {
      auto get = [&](int f, int q) -> C2 {
        if (q < m || q > T + 1) return {0.0, 0.0};
        const int c = (bb * 5 + f) * 2;
        return {(double)Yl[c * nx + q - m], (double)Yl[(c + 1) * nx + q - m]};
      };
      C2 o[3];
      assemble_core(get, m, n, ph.a, o);
      if (asm_src) {   // the source's F_E, read back by this thread in node_update below
        for (int v = 0; v < 3; ++v)
          st2(src.fe_pending + 2 * ((size_t)bb * src.stride + (size_t)v * K + k), o[v]);
      } else {
        const size_t base = (size_t)bb * nn * 3 * K;
        for (int v = 0; v < 3; ++v) st2(fe + 2 * (base + ((size_t)asm_node * 3 + v) * K + k), o[v]);
      }
    }
    if (node >= 1) {
      C2 x[3];
      node_update<NN>(th, fe, fi, tau, S, src, K, bb, k, n, node, dt, sm, ph, x);
      for (int v = 0; v < 3; ++v) sh[(bb * 3 + v) * (T + 1) + (n - m)] = x[v];
    }
  }
  if (node < 1) return;
  __syncthreads();
  // (3a) synthesis operand of order m: [parity][k-block][lane = k * 16 + column]
  for (int n = m + threadIdx.x; n <= T + 1; n += blockDim.x) {
    const int p = (n - m) & 1, i = (n - m) >> 1;
    R* dst = Xl + ((size_t)p * kbmax + i / Op::KB) * 64 + (i % Op::KB) * 16;
    for (int bb = 0; bb < nsl; ++bb) {
      auto get = [&](int v, int q) { return sh[(bb * 3 + v) * (T + 1) + (q - m)]; };
      C2 v4[4];
      prep_fields(get, m, n, T, ph, v4);
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        dst[bb * 8 + 2 * f] = (R)v4[f].x;
        dst[bb * 8 + 2 * f + 1] = (R)v4[f].y;
      }
    }
  }
  __syncthreads();
  // (3b) synthesis: 16 x 16 blocks (parity, ring block), highest degree first
  const int ntask = 2 * RB;
  for (int t = wave; t < ntask; t += NW) {
    const int p = t / RB, rb = t - p * RB;
    const MPInfo q = mpi[2 * m + p];
    if (q.kbS == 0) continue;
    const long long last = q.kbS - 1;
    typename Op::C acc = {}, d1 = {}, d2 = {}, d3 = {};
    constexpr int KG = KGroup<Op>::KG;   // table k-grouped from the highest k-block down
    mma_loop_grp<Op, (PF + KG - 1) / KG>(tabS, Xl, q.tabS / KG + rb, (long long)RB,
                                         (long long)p * kbmax + last, -1LL, q.kbS / KG,
                                         q.kbS % KG, false, false, lane, acc, d1, d2, d3);
    const int c = lane & 15;
    if (c < 8 * nsl) {
      const int b = c >> 3, f = (c & 7) >> 1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = rb * 16 + Op::row(lane, v);
        if (j < J) F4[2 * f4_index(b, j, f, p, m, J, 4, Lp, f4_mg(sizeof(R))) + (c & 1)] = (R)acc[v];
      }
    }
  }
}

// -------------------------------------------------------------- residual
__device__ __forceinline__ double nanmax(double r, double a) {
  return (isnan(a) || a > r) ? a : r;
}

// partial maxima per (batch, variable, block); |r| with
// r^i = Theta^0 + dt (Q F)_i + tau_i - Theta^i, i = 1..M
template <int NN>
__global__ __launch_bounds__(256) void k_residual_part(const double* __restrict__ th,
                                                      const double* __restrict__ fe,
                                                      const double* __restrict__ fi,
                                                      const double* __restrict__ tau,
                                                      double* __restrict__ part, int K,
                                                      double dt, SdcMat sm) {
  constexpr int nn = NN;
  const int b = blockIdx.z, v = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  double r = 0.0;
  if (k < K) {
    const size_t base = (size_t)b * nn * 3 * K + (size_t)v * K + k;
    C2 F[NN];
#pragma unroll
    for (int j = 0; j < nn; ++j) {
      const C2 e = ld2(fe + 2 * (base + (size_t)j * 3 * K));
      const C2 f = ld2(fi + 2 * (base + (size_t)j * 3 * K));
      F[j] = {e.x + f.x, e.y + f.y};
    }
    const C2 t0 = ld2(th + 2 * base);
#pragma unroll
    for (int i = 1; i < nn; ++i) {
      double sx = 0, sy = 0;
#pragma unroll
      for (int j = 0; j < nn; ++j) {
        sx += sm.Q[i * nn + j] * F[j].x;
        sy += sm.Q[i * nn + j] * F[j].y;
      }
      const C2 ti = ld2(th + 2 * (base + (size_t)i * 3 * K));
      double rx = t0.x + dt * sx - ti.x, ry = t0.y + dt * sy - ti.y;
      if (tau) {
        const C2 tv = ld2(tau + 2 * (base + (size_t)i * 3 * K));
        rx += tv.x;
        ry += tv.y;
      }
      r = nanmax(r, sqrt(rx * rx + ry * ry));
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = r;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = nanmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[((size_t)b * 3 + v) * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_residual_final(const double* __restrict__ part, double* __restrict__ out,
                                 int nblk, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double r = 0.0;
  for (int q = 0; q < nblk; ++q) r = nanmax(r, part[(size_t)i * nblk + q]);
  out[i] = r;
}

__global__ void k_count_nonfinite(const double* __restrict__ v, int n, int* __restrict__ flag) {
  int bad = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    if (!isfinite(v[i])) bad = 1;
  if (bad) flag[0] = 1;
}

// -------------------------------------------------------------- copies
// node 0 -> nodes 1..M of a [batch][nn][3K] complex array
__global__ void k_spread(double* __restrict__ a, int nn, long long n3k, int batch) {
  const long long tot = (long long)batch * (nn - 1) * n3k;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long b = idx / ((nn - 1) * n3k);
    const long long r = idx - b * (nn - 1) * n3k;
    const long long i = 1 + r / n3k, e = r - (i - 1) * n3k;
    const size_t base = (size_t)b * nn * n3k;
    st2(a + 2 * (base + i * n3k + e), ld2(a + 2 * (base + e)));
  }
}

// strided batch copy of n_per complex values
__global__ void k_copy_state(const double* __restrict__ src, long long sstride,
                             double* __restrict__ dst, long long dstride, long long n_per,
                             int batch) {
  const long long tot = (long long)batch * n_per;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long b = idx / n_per, e = idx - b * n_per;
    st2(dst + 2 * (b * dstride + e), ld2(src + 2 * (b * sstride + e)));
  }
}

// three arrays at once (state, F_E, F_I of one node), batch entries strided
__global__ void k_copy_node3(const double* __restrict__ ts, const double* __restrict__ es,
                             const double* __restrict__ is, long long sstride,
                             double* __restrict__ td, double* __restrict__ ed,
                             double* __restrict__ id, long long dstride, long long n_per,
                             int batch) {
  const long long tot = (long long)batch * n_per;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long b = idx / n_per, e = idx - b * n_per;
    const long long so = 2 * (b * sstride + e), d = 2 * (b * dstride + e);
    st2(td + d, ld2(ts + so));
    st2(ed + d, ld2(es + so));
    st2(id + d, ld2(is + so));
  }
}

// -------------------------------------------------------------- transfers
struct TMat {
  double P[81];  // [ndst][nsrc]
};

// restriction: out_c[b][i][v][kc] = sum_j Pi_cf[i][j] in_f[b][j][v][kf(kc)]
__global__ void k_restrict(const double* __restrict__ in, double* __restrict__ out, int Tf, int Tc,
                           int nf, int nc, int batch, TMat pm) {
  const int Kc = (Tc + 1) * (Tc + 2) / 2, Kf = (Tf + 1) * (Tf + 2) / 2;
  const long long tot = (long long)batch * nc * 3 * Kc;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    long long r = idx;
    const int kc = (int)(r % Kc); r /= Kc;
    const int v = (int)(r % 3); r /= 3;
    const int i = (int)(r % nc);
    const int b = (int)(r / nc);
    int m, n;
    slot_mn(Tc, kc, m, n);
    const int kf = spec_off(Tf, m) + n - m;
    double sx = 0, sy = 0;
    for (int j = 0; j < nf; ++j) {
      const double c = pm.P[i * nf + j];
      if (c == 0.0) continue;
      const C2 z = ld2(in + 2 * ((((size_t)b * nf + j) * 3 + v) * Kf + kf));
      sx += c * z.x;
      sy += c * z.y;
    }
    st2(out + 2 * idx, {sx, sy});
  }
}

// interpolation of an increment: inout_f[b][i][v][kf(kc)] += sum_j Pi_fc[i][j] (new - old)[b][j][v][kc]
// One thread per (b, v, kc): the nc coarse increments are loaded once and
// spread to all nf fine nodes (node loops unrolled to the 9-node maximum, so
// the per-node values stay in registers).
// Up to three (new, old, in-out) array triples, one per blockIdx.y (state, F_E,
// F_I of PFASST step D in one launch).
struct InterpArrays {
  const double* nw[3];
  const double* old[3];
  double* io[3];
};
// NCT, NFT: the node counts at compile time (0: the run-time nc, nf, up to 9),
// so that the common (3, 5) pair keeps only the registers and loads it needs.
template <int NCT, int NFT>
__global__ void k_interp_add(InterpArrays arr, int Tc, int Tf, int nc_rt, int nf_rt, int batch,
                             TMat pm) {
  constexpr int MC = NCT ? NCT : 9, MF = NFT ? NFT : 9;
  const int nc = NCT ? NCT : nc_rt, nf = NFT ? NFT : nf_rt;
  const double* __restrict__ nw = arr.nw[blockIdx.y];
  const double* __restrict__ old = arr.old[blockIdx.y];
  double* __restrict__ io = arr.io[blockIdx.y];
  const int Kc = (Tc + 1) * (Tc + 2) / 2, Kf = (Tf + 1) * (Tf + 2) / 2;
  const long long tot = (long long)batch * 3 * Kc;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    long long r = idx;
    const int kc = (int)(r % Kc); r /= Kc;
    const int v = (int)(r % 3);
    const int b = (int)(r / 3);
    int m, n;
    slot_mn(Tc, kc, m, n);
    const int kf = spec_off(Tf, m) + n - m;
    C2 dz[MC];
#pragma unroll
    for (int j = 0; j < MC; ++j) {
      if (j < nc) {
        const size_t o = (((size_t)b * nc + j) * 3 + v) * Kc + kc;
        dz[j] = ld2(nw + 2 * o);
        if (old) {
          const C2 y = ld2(old + 2 * o);
          dz[j].x -= y.x;
          dz[j].y -= y.y;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < MF; ++i) {
      if (i < nf) {
        double sx = 0, sy = 0;
#pragma unroll
        for (int j = 0; j < MC; ++j) {
          if (j < nc) {
            const double c = pm.P[i * nc + j];
            if (c != 0.0) {
              sx += c * dz[j].x;
              sy += c * dz[j].y;
            }
          }
        }
        double* p = io + 2 * ((((size_t)b * nf + i) * 3 + v) * Kf + kf);
        C2 t = ld2(p);
        st2(p, {t.x + sx, t.y + sy});
      }
    }
  }
}

// tau_c = dt [ sum_j Pi_cf[i][j] sum_l Qf[j][l] F_f^l (kf)  -  sum_l Qc[i][l] F_c^l (kc) ]
struct TauMat {
  double Pcf[81], Qf[81], Qc[81];
};
template <int NFT, int NCT>
__global__ void k_fas_tau(const double* __restrict__ fef, const double* __restrict__ fif,
                          const double* __restrict__ fec, const double* __restrict__ fic,
                          double* __restrict__ tau, int Tf, int Tc, int nf_rt, int nc_rt,
                          int batch, double dt, TauMat tm) {
  constexpr int MF = NFT ? NFT : 9, MC = NCT ? NCT : 9;   // as k_interp_add
  const int nf = NFT ? NFT : nf_rt, nc = NCT ? NCT : nc_rt;
  const int Kc = (Tc + 1) * (Tc + 2) / 2, Kf = (Tf + 1) * (Tf + 2) / 2;
  const long long tot = (long long)batch * 3 * Kc;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    long long r = idx;
    const int kc = (int)(r % Kc); r /= Kc;
    const int v = (int)(r % 3);
    const int b = (int)(r / 3);
    int m, n;
    slot_mn(Tc, kc, m, n);
    const int kf = spec_off(Tf, m) + n - m;
    // node loops unrolled to the node count (or the 9-node maximum): the
    // per-node values stay in registers (runtime-indexed arrays would live in
    // scratch memory)
    C2 Ff[MF], Fc[MC];
#pragma unroll
    for (int l = 0; l < MF; ++l) {
      if (l < nf) {
        const size_t o = (((size_t)b * nf + l) * 3 + v) * Kf + kf;
        const C2 e = ld2(fef + 2 * o), f = ld2(fif + 2 * o);
        Ff[l] = {e.x + f.x, e.y + f.y};
      }
    }
#pragma unroll
    for (int l = 0; l < MC; ++l) {
      if (l < nc) {
        const size_t o = (((size_t)b * nc + l) * 3 + v) * Kc + kc;
        const C2 e = ld2(fec + 2 * o), f = ld2(fic + 2 * o);
        Fc[l] = {e.x + f.x, e.y + f.y};
      }
    }
#pragma unroll
    for (int i = 0; i < MC; ++i) {
      if (i >= nc) continue;
      double fx = 0, fy = 0;
#pragma unroll
      for (int j = 0; j < MF; ++j) {
        if (j >= nf) continue;
        const double c = tm.Pcf[i * nf + j];
        if (c == 0.0) continue;
        double qx = 0, qy = 0;
#pragma unroll
        for (int l = 0; l < MF; ++l) {
          if (l < nf) {
            qx += tm.Qf[j * nf + l] * Ff[l].x;
            qy += tm.Qf[j * nf + l] * Ff[l].y;
          }
        }
        fx += c * qx;
        fy += c * qy;
      }
      double cx = 0, cy = 0;
#pragma unroll
      for (int l = 0; l < MC; ++l) {
        if (l < nc) {
          cx += tm.Qc[i * nc + l] * Fc[l].x;
          cy += tm.Qc[i * nc + l] * Fc[l].y;
        }
      }
      st2(tau + 2 * ((((size_t)b * nc + i) * 3 + v) * Kc + kc), {dt * fx - dt * cx, dt * fy - dt * cy});
    }
  }
}

// PFASST step D: new fine initial condition = received fine value with its
// (m, n <= Tc) modes moved by (coarse initial condition - restriction of it).
__global__ void k_ic_correct(const double* __restrict__ recv, long long rstride,
                             const double* __restrict__ icc, long long cstride,
                             double* __restrict__ out, long long ostride, int Tf, int Tc,
                             int batch) {
  const int Kf = (Tf + 1) * (Tf + 2) / 2, Kc = (Tc + 1) * (Tc + 2) / 2;
  const long long tot = (long long)batch * 3 * Kf;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(idx / (3 * Kf));
    const int r = (int)(idx - (long long)b * 3 * Kf);
    const int v = r / Kf, kf = r - v * Kf;
    int m, n;
    slot_mn(Tf, kf, m, n);
    C2 z = ld2(recv + 2 * ((size_t)b * rstride + r));
    if (m <= Tc && n <= Tc) {
      const int kc = spec_off(Tc, m) + n - m;
      const C2 c = ld2(icc + 2 * ((size_t)b * cstride + (size_t)v * Kc + kc));
      z = {z.x + (c.x - z.x), z.y + (c.y - z.y)};
    }
    st2(out + 2 * ((size_t)b * ostride + r), z);
  }
}

// ---------------------------------------------------------------- launchers
static inline unsigned nblocks(long long work, int bs) {
  long long g = (work + bs - 1) / bs;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}
static inline Phys phys_of(const pfsh_level* lv) {
  return Phys{lv->d.radius, lv->d.omega, lv->d.phibar, lv->d.nu};
}
static inline SdcMat sdc_of(const pfsh_level* lv) {
  SdcMat s;
  for (int i = 0; i < 81; ++i) { s.Q[i] = lv->Q[i]; s.QE[i] = lv->QE[i]; s.QI[i] = lv->QI[i]; }
  s.nn = lv->nn;
  s.split = lv->implicit_split;
  return s;
}

hipError_t launch_prep_rhs(const pfsh_level* lv, const double* state, long long sstride,
                           double* f_impl, long long fstride, int batch, hipStream_t s) {
  dim3 grid(lv->L, (batch + 1) / 2);
  switch (lv->op) {
    case OP_F64:
      PFSH_LAUNCH(lv, k_prep_rhs<OpF64>, grid, dim3(128), 0, s, state, sstride, f_impl,
                         fstride, lv->X, lv->mp_d, lv->T, lv->CBs, batch, phys_of(lv));
      break;
    case OP_F32:
      PFSH_LAUNCH(lv, k_prep_rhs<OpF32>, grid, dim3(128), 0, s, state, sstride, f_impl,
                         fstride, lv->X, lv->mp_d, lv->T, lv->CBs, batch, phys_of(lv));
      break;
    default:
      PFSH_LAUNCH(lv, k_prep_rhs<OpBF3>, grid, dim3(128), 0, s, state, sstride, f_impl,
                         fstride, lv->X, lv->mp_d, lv->T, lv->CBs, batch, phys_of(lv));
  }
  return hipGetLastError();
}

hipError_t launch_prep_scalar(const pfsh_level* lv, const double* spec, int nfields, hipStream_t s) {
  dim3 grid(lv->L, nfields);
  switch (lv->op) {
    case OP_F64:
      PFSH_LAUNCH(lv, k_prep_scalar<OpF64>, grid, dim3(128), 0, s, spec, lv->X, lv->mp_d,
                         lv->T, lv->CBs);
      break;
    case OP_F32:
      PFSH_LAUNCH(lv, k_prep_scalar<OpF32>, grid, dim3(128), 0, s, spec, lv->X, lv->mp_d,
                         lv->T, lv->CBs);
      break;
    default:
      PFSH_LAUNCH(lv, k_prep_scalar<OpBF3>, grid, dim3(128), 0, s, spec, lv->X, lv->mp_d,
                         lv->T, lv->CBs);
  }
  return hipGetLastError();
}

hipError_t launch_unpack_scalar(const pfsh_level* lv, double* spec, int nfields, hipStream_t s) {
  const long long work = (long long)nfields * lv->K;
  if (lv->op == OP_F64)
    PFSH_LAUNCH(lv, k_unpack_scalar<double>, dim3(nblocks(work, 256)), dim3(256), 0, s,
                       (const double*)lv->Y, spec, lv->T, nfields);
  else
    PFSH_LAUNCH(lv, k_unpack_scalar<float>, dim3(nblocks(work, 256)), dim3(256), 0, s,
                       (const float*)lv->Y, spec, lv->T, nfields);
  return hipGetLastError();
}

hipError_t launch_assemble(const pfsh_level* lv, double* f_expl, long long fstride, int batch,
                           hipStream_t s) {
  // order pairs (g, L - g): order 0, L/2 - 1 or (L-1)/2 pairs, and order L/2 for even L
  dim3 grid(lv->L / 2 + 1, batch);
  if (lv->op == OP_F64)
    PFSH_LAUNCH(lv, k_assemble<double>, grid, dim3(256), 0, s, (const double*)lv->Y, f_expl,
                       fstride, lv->T, lv->d.radius);
  else
    PFSH_LAUNCH(lv, k_assemble<float>, grid, dim3(256), 0, s, (const float*)lv->Y, f_expl,
                       fstride, lv->T, lv->d.radius);
  return hipGetLastError();
}

hipError_t launch_implicit_solve(const pfsh_level* lv, double beta, const double* b, double* x,
                                 int batch, hipStream_t s) {
  const long long work = (long long)batch * lv->K;
  PFSH_LAUNCH(lv, k_implicit_solve, dim3(nblocks(work, 256)), dim3(256), 0, s, b, x, lv->T,
                     batch, beta, phys_of(lv));
  return hipGetLastError();
}

#define PFSH_NN_SWITCH(nn, CALL) \
  switch (nn) {                  \
    case 2: CALL(2); break;      \
    case 3: CALL(3); break;      \
    case 4: CALL(4); break;      \
    case 5: CALL(5); break;      \
    case 6: CALL(6); break;      \
    case 7: CALL(7); break;      \
    case 8: CALL(8); break;      \
    default: CALL(9); break;     \
  }

template <class Op, int NN, int ND>
static hipError_t sweep_step_nd(const pfsh_level* lv, int node, int asm_node, double dt,
                                double* th, double* fe, double* fi, const double* tau, int batch,
                                const StepSrc& src, hipStream_t s) {
  const size_t shm = (size_t)2 * 3 * (lv->T + 1) * sizeof(C2);
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)k_sweep_step<Op, NN, ND>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  // order pairs (g, L - g): order 0, L/2 - 1 or (L-1)/2 pairs, and order L/2 for even L
  PFSH_LAUNCH(lv, (k_sweep_step<Op, NN, ND>), dim3(lv->L / 2 + 1, (batch + 1) / 2), dim3(512), shm,
                     s, th, fe, fi, tau, lv->S, (const typename Op::R*)lv->Y, lv->X, lv->mp_d,
                     lv->T, lv->CBs, batch, node, asm_node, dt, sdc_of(lv), phys_of(lv),
                     SrcPtrs{src.th, src.fe, src.fi, src.stride, src.fe_pending});
  return hipGetLastError();
}

// Up to 5 nodes the node is a template argument (one kernel per node; a node
// >= 2 then assembles F_E of node - 1, the sweep's order), above that a
// run-time argument.
template <class Op, int NN>
static hipError_t sweep_step_impl(const pfsh_level* lv, int node, int asm_node, double dt,
                                  double* th, double* fe, double* fi, const double* tau, int batch,
                                  const StepSrc& src, hipStream_t s) {
#define PFSH_ND(D) sweep_step_nd<Op, NN, D>(lv, node, asm_node, dt, th, fe, fi, tau, batch, src, s)
  if constexpr (NN <= 5) {
    if (node == 1) return PFSH_ND(1);
    if (asm_node != node - 1) return PFSH_ND(0);
    if (NN > 2 && node == 2) return PFSH_ND((NN > 2 ? 2 : 0));
    if (NN > 3 && node == 3) return PFSH_ND((NN > 3 ? 3 : 0));
    if (NN > 4 && node == 4) return PFSH_ND((NN > 4 ? 4 : 0));
  }
  return PFSH_ND(0);
#undef PFSH_ND
}

template <class Op, int NN>
static hipError_t node_fused_impl(const pfsh_level* lv, int node, int asm_node, double dt,
                                  double* th, double* fe, double* fi, const double* tau, int batch,
                                  const StepSrc& src, hipStream_t s) {
  typedef typename Op::R R;
  const int kbmax = (npar(lv->T, 0, 0) + Op::KB - 1) / Op::KB;
  const size_t shm = (size_t)2 * 3 * (lv->T + 1) * sizeof(C2) + (size_t)20 * (lv->T + 2) * sizeof(R) +
                     (size_t)2 * kbmax * 64 * sizeof(R);
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)k_node_fused<Op, NN>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  PFSH_LAUNCH(lv, (k_node_fused<Op, NN>), dim3(lv->L), dim3(1024), shm, s, th, fe, fi, tau, lv->S,
                     lv->tabA, lv->G, lv->tabS, (R*)lv->F4, lv->mp_d, lv->T, lv->J, lv->Lp, lv->kb2,
                     lv->CBa, lv->RB, kbmax, batch, node, asm_node, dt, sdc_of(lv), phys_of(lv),
                     SrcPtrs{src.th, src.fe, src.fi, src.stride, src.fe_pending});
  return hipGetLastError();
}

bool node_fused_ok(const pfsh_level* lv, int batch) {
  if (batch < 1 || batch > 2 || (lv->op != OP_F64 && lv->op != OP_F32)) return false;
  if (lv->rec_mode) return false;   // the fused node reads the tables
  const size_t rsz = lv->op == OP_F64 ? 8 : 4;
  const int kbmax = (npar(lv->T, 0, 0) + 3) / 4;
  const size_t shm = (size_t)2 * 3 * (lv->T + 1) * 16 + (size_t)20 * (lv->T + 2) * rsz +
                     (size_t)2 * kbmax * 64 * rsz;
  return shm <= 160 * 1024 && lv->variant[TS_FUSE][tune_bucket(batch)] == 0;
}

hipError_t launch_node_fused(const pfsh_level* lv, int node, int asm_node, double dt, double* th,
                             double* fe, double* fi, const double* tau, int batch,
                             const StepSrc& src, hipStream_t s) {
#define PFSH_FUSED(NN)                                                                          \
  return lv->op == OP_F64                                                                      \
             ? node_fused_impl<OpF64, NN>(lv, node, asm_node, dt, th, fe, fi, tau, batch, src, s) \
             : node_fused_impl<OpF32, NN>(lv, node, asm_node, dt, th, fe, fi, tau, batch, src, s)
  PFSH_NN_SWITCH(lv->nn, PFSH_FUSED)
#undef PFSH_FUSED
  return hipSuccess;
}

template <class Op>
static hipError_t sweep_step_op(const pfsh_level* lv, int node, int asm_node, double dt, double* th,
                                double* fe, double* fi, const double* tau, int batch,
                                const StepSrc& src, hipStream_t s) {
#define PFSH_STEP(NN) \
  return sweep_step_impl<Op, NN>(lv, node, asm_node, dt, th, fe, fi, tau, batch, src, s)
  PFSH_NN_SWITCH(lv->nn, PFSH_STEP)
#undef PFSH_STEP
  return hipSuccess;
}

hipError_t launch_sweep_step(const pfsh_level* lv, int node, int asm_node, double dt, double* th,
                             double* fe, double* fi, const double* tau, int batch,
                             const StepSrc& src, hipStream_t s) {
  switch (lv->op) {
    case OP_F64: return sweep_step_op<OpF64>(lv, node, asm_node, dt, th, fe, fi, tau, batch, src, s);
    case OP_F32: return sweep_step_op<OpF32>(lv, node, asm_node, dt, th, fe, fi, tau, batch, src, s);
    default: return sweep_step_op<OpBF3>(lv, node, asm_node, dt, th, fe, fi, tau, batch, src, s);
  }
}

long long residual_part_len(const pfsh_level* lv, int batch) {
  return (long long)batch * 3 * ((lv->K + 255) / 256);
}

// The residual's partial maxima go to `part` (residual_part_len doubles).
hipError_t launch_residual_into(const pfsh_level* lv, double dt, const double* theta,
                                const double* fe, const double* fi, const double* tau, double* out,
                                double* part, int batch, hipStream_t s) {
  const int nblk = (lv->K + 255) / 256;
  const SdcMat sm = sdc_of(lv);
#define PFSH_RES(NN)                                                                          \
  hipLaunchKernelGGL(k_residual_part<NN>, dim3(nblk, 3, batch), dim3(256), 0, s, theta, fe, fi, \
                     tau, part, lv->K, dt, sm)
  PFSH_NN_SWITCH(lv->nn, PFSH_RES)
#undef PFSH_RES
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_residual_final, dim3((batch * 3 + 127) / 128), dim3(128), 0, s, part,
                     out, nblk, batch * 3);
  return hipGetLastError();
}

hipError_t launch_residual(const pfsh_level* lv, double dt, const double* theta, const double* fe,
                           const double* fi, const double* tau, double* out, int batch,
                           hipStream_t s) {
  return launch_residual_into(lv, dt, theta, fe, fi, tau, out, lv->red, batch, s);
}

// ----------------------------------------- residual scratch without allocation
// The partial maxima of pfsh_residual_noalloc live in this file-scope device
// array instead of a level's workspace: every GPU the library runs on holds
// its own copy until the process ends.  In host code the name `scratch` only
// stands for the symbol; the device address of each GPU's copy comes from
// hipGetSymbolAddress (residual_scratch_setup, called once per device with
// that device current) and only that address is handed to kernels.  Every
// call on one GPU shares the array; the partial-maxima kernel writes every
// entry it later reads, so nothing has to start at zero.
__attribute__((used)) static __device__ __align__(256) double scratch[kResidualScratchDoubles];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t residual_scratch_setup(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return hipSuccess;
}

double* residual_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_spread(const pfsh_level* lv, double* a, int batch, hipStream_t s) {
  const long long n3k = 3LL * lv->K;
  const long long work = (long long)batch * (lv->nn - 1) * n3k;
  hipLaunchKernelGGL(k_spread, dim3(nblocks(work, 256)), dim3(256), 0, s, a, lv->nn, n3k, batch);
  return hipGetLastError();
}

hipError_t launch_copy_node3(const double* ts, const double* es, const double* is,
                             long long sstride, double* td, double* ed, double* id,
                             long long dstride, long long n_per, int batch, hipStream_t s) {
  const long long work = (long long)batch * n_per;
  hipLaunchKernelGGL(k_copy_node3, dim3(nblocks(work, 256)), dim3(256), 0, s, ts, es, is, sstride,
                     td, ed, id, dstride, n_per, batch);
  return hipGetLastError();
}

hipError_t launch_copy_state(const double* src, long long sstride, double* dst, long long dstride,
                             long long n_per, int batch, hipStream_t s) {
  const long long work = (long long)batch * n_per;
  hipLaunchKernelGGL(k_copy_state, dim3(nblocks(work, 256)), dim3(256), 0, s, src, sstride, dst,
                     dstride, n_per, batch);
  return hipGetLastError();
}

hipError_t launch_restrict(const pfsh_level* f, const pfsh_level* c, const double* in_f,
                           double* out_c, int batch, hipStream_t s) {
  TMat pm;
  lagrange_matrix(f->nn, f->nodes, c->nn, c->nodes, pm.P);
  const long long work = (long long)batch * c->nn * 3 * c->K;
  hipLaunchKernelGGL(k_restrict, dim3(nblocks(work, 256)), dim3(256), 0, s, in_f, out_c, f->T,
                     c->T, f->nn, c->nn, batch, pm);
  return hipGetLastError();
}

hipError_t launch_interp_add3(const pfsh_level* c, const pfsh_level* f, int count,
                              const double* const* new_c, const double* const* old_c,
                              double* const* inout_f, int batch, hipStream_t s) {
  if (count < 1 || count > 3) return hipErrorInvalidValue;
  TMat pm;
  lagrange_matrix(c->nn, c->nodes, f->nn, f->nodes, pm.P);
  InterpArrays arr{};
  for (int i = 0; i < count; ++i) {
    arr.nw[i] = new_c[i];
    arr.old[i] = old_c[i];
    arr.io[i] = inout_f[i];
  }
  const long long work = (long long)batch * 3 * c->K;
  const dim3 grid(nblocks(work, 256), count);
  if (c->nn == 3 && f->nn == 5)
    hipLaunchKernelGGL((k_interp_add<3, 5>), grid, dim3(256), 0, s, arr, c->T, f->T, c->nn, f->nn,
                       batch, pm);
  else
    hipLaunchKernelGGL((k_interp_add<0, 0>), grid, dim3(256), 0, s, arr, c->T, f->T, c->nn, f->nn,
                       batch, pm);
  return hipGetLastError();
}

hipError_t launch_interp_add(const pfsh_level* c, const pfsh_level* f, const double* new_c,
                             const double* old_c, double* inout_f, int batch, hipStream_t s) {
  return launch_interp_add3(c, f, 1, &new_c, &old_c, &inout_f, batch, s);
}

hipError_t launch_fas_tau(const pfsh_level* f, const pfsh_level* c, double dt, const double* fe_f,
                          const double* fi_f, const double* fe_c, const double* fi_c, double* tau,
                          int batch, hipStream_t s) {
  TauMat tm;
  lagrange_matrix(f->nn, f->nodes, c->nn, c->nodes, tm.Pcf);
  for (int i = 0; i < 81; ++i) { tm.Qf[i] = 0; tm.Qc[i] = 0; }
  for (int i = 0; i < f->nn * f->nn; ++i) tm.Qf[i] = f->Q[i];
  for (int i = 0; i < c->nn * c->nn; ++i) tm.Qc[i] = c->Q[i];
  const long long work = (long long)batch * 3 * c->K;
  if (f->nn == 5 && c->nn == 3)
    hipLaunchKernelGGL((k_fas_tau<5, 3>), dim3(nblocks(work, 256)), dim3(256), 0, s, fe_f, fi_f,
                       fe_c, fi_c, tau, f->T, c->T, f->nn, c->nn, batch, dt, tm);
  else
    hipLaunchKernelGGL((k_fas_tau<0, 0>), dim3(nblocks(work, 256)), dim3(256), 0, s, fe_f, fi_f,
                       fe_c, fi_c, tau, f->T, c->T, f->nn, c->nn, batch, dt, tm);
  return hipGetLastError();
}

hipError_t launch_ic_correct(const pfsh_level* f, const pfsh_level* c, const double* recv_f,
                             long long recv_stride, const double* ic_c, long long ic_stride,
                             double* out_f, long long out_stride, int batch, hipStream_t s) {
  const long long work = (long long)batch * 3 * f->K;
  hipLaunchKernelGGL(k_ic_correct, dim3(nblocks(work, 256)), dim3(256), 0, s, recv_f, recv_stride,
                     ic_c, ic_stride, out_f, out_stride, f->T, c->T, batch);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite(const double* v, int n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_count_nonfinite, dim3(nblocks(n, 256)), dim3(256), 0, s, v, n, flag);
  return hipGetLastError();
}

}  // namespace pfsh
