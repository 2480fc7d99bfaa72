// Host-side tables of a level: Gaussian grid, normalized associated Legendre
// functions packed in MFMA operand order, Gauss-Lobatto SDC matrices.
//
// Sec. 3: Gaussian latitudes mu_j (roots of P_nlat) with their quadrature
// weights; normalized P_n^m (int P^2 dmu = 1, P_m^m > 0), evaluated by the
// sectoral seed and the three-term recurrence in x87 80-bit precision so that
// the seed (1-mu^2)^{m/2} does not underflow near the poles at high order.
// Sec. 5.1.1: Lobatto nodes, integration matrix Q, forward-Euler qE and
// qI = U^T of the LU factorization (no pivoting) of Q^T on nodes 1..M.
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "pfsh_internal.h"

namespace pfsh {

typedef long double ld;

// Legendre polynomial P_n(x) and derivative (unnormalized) by recurrence.
static void legendre_pd(int n, ld x, ld& p, ld& dp) {
  ld p0 = 1, p1 = x;
  if (n == 0) { p = 1; dp = 0; return; }
  for (int k = 1; k < n; ++k) {
    ld p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = n * (p0 - x * p1) / (1 - x * x);
}

void gauss_legendre(int nlat, std::vector<double>& mu, std::vector<double>& w) {
  mu.resize(nlat);
  w.resize(nlat);
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < nlat; ++i) {
    ld x = std::cos(pi * (i + 0.75L) / (nlat + 0.5L));
    ld p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre_pd(nlat, x, p, dp);
      ld dx = p / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-19L) break;
    }
    legendre_pd(nlat, x, p, dp);
    mu[i] = (double)x;                      // cos guess is already descending
    w[i] = (double)(2 / ((1 - x * x) * dp * dp));
  }
}

// Lobatto nodes on [0,1]: 0, roots of P'_M, 1 (Newton on P'_M).
static void lobatto(int nn, ld* x01) {
  int M = nn - 1;
  const ld pi = 3.141592653589793238462643383279502884L;
  x01[0] = 0;
  x01[M] = 1;
  for (int i = 1; i < M; ++i) {
    ld x = -std::cos(pi * i / M);
    for (int it = 0; it < 100; ++it) {
      ld p, dp;
      legendre_pd(M, x, p, dp);
      ld d2 = (2 * x * dp - M * (M + 1) * p) / (1 - x * x);
      ld dx = dp / d2;
      x -= dx;
      if (std::fabs(dx) < 1e-19L) break;
    }
    x01[i] = (x + 1) / 2;
  }
}

static ld lagrange(int n, const ld* nodes, int j, ld t) {
  ld v = 1;
  for (int k = 0; k < n; ++k)
    if (k != j) v *= (t - nodes[k]) / (nodes[j] - nodes[k]);
  return v;
}

void lagrange_matrix(int nsrc, const double* src, int ndst, const double* dst, double* out) {
  std::vector<ld> s(nsrc);
  for (int i = 0; i < nsrc; ++i) s[i] = src[i];
  for (int i = 0; i < ndst; ++i)
    for (int j = 0; j < nsrc; ++j) {
      ld v = lagrange(nsrc, s.data(), j, (ld)dst[i]);
      if (std::fabs(v) < 1e-15L) v = 0;                 // exact zeros for nested nodes
      if (std::fabs(v - 1) < 1e-15L) v = 1;
      out[i * nsrc + j] = (double)v;
    }
}

void sdc_matrices(int nn, double* nodes, double* Q, double* QE, double* QI) {
  ld x[16];
  lobatto(nn, x);
  for (int i = 0; i < nn; ++i) nodes[i] = (double)x[i];
  // Q_ij = int_0^{x_i} l_j(s) ds by an 8-point Gauss rule on [0, x_i]
  // (exact: l_j has degree nn-1 <= 8).
  const int G = 8;
  std::vector<double> gm, gw;
  gauss_legendre(G, gm, gw);
  for (int i = 0; i < nn; ++i)
    for (int j = 0; j < nn; ++j) {
      ld acc = 0;
      for (int g = 0; g < G; ++g) {
        ld s = x[i] * ((ld)gm[g] + 1) / 2;
        acc += (ld)gw[g] * lagrange(nn, x, j, s);
      }
      Q[i * nn + j] = (double)(acc * x[i] / 2);
    }
  for (int i = 0; i < nn; ++i)
    for (int j = 0; j < nn; ++j) QE[i * nn + j] = (j < i) ? (double)(x[j + 1] - x[j]) : 0.0;
  // qI: U of A = Q[1:,1:]^T = L U (no pivoting); QI[1:,1:] = U^T.
  int M = nn - 1;
  std::vector<ld> U(M * M);
  for (int r = 0; r < M; ++r)
    for (int c = 0; c < M; ++c) U[r * M + c] = Q[(c + 1) * nn + (r + 1)];
  for (int k = 0; k < M; ++k)
    for (int r = k + 1; r < M; ++r) {
      ld f = U[r * M + k] / U[k * M + k];
      for (int c = k; c < M; ++c) U[r * M + c] -= f * U[k * M + c];
    }
  for (int i = 0; i < nn * nn; ++i) QI[i] = 0;
  for (int r = 0; r < M; ++r)
    for (int c = r; c < M; ++c) QI[(c + 1) * nn + (r + 1)] = (double)U[r * M + c];
}

// bf16 round-to-nearest-even of a float
static uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static float from_bf16(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

static void put(int op, unsigned char* base, long long block, int lane, int elem, double v) {
  size_t bb = (size_t)op_block_bytes(op);
  unsigned char* b = base + (size_t)block * bb;
  if (op == OP_F64) {
    reinterpret_cast<double*>(b)[lane] = v;
  } else if (op == OP_F32) {
    reinterpret_cast<float*>(b)[lane] = (float)v;
  } else {
    uint16_t* h = reinterpret_cast<uint16_t*>(b);
    uint16_t hi = to_bf16((float)v);
    uint16_t lo = to_bf16((float)(v - (double)from_bf16(hi)));
    h[lane * 16 + elem] = hi;
    h[lane * 16 + 8 + elem] = lo;
  }
}

void build_tables(pfsh_level* lv, std::vector<unsigned char>& tabS, std::vector<unsigned char>& tabA,
                  std::vector<double>& /*unused*/) {
  const int T = lv->T, J = lv->J, op = lv->op;
  const size_t bb = (size_t)op_block_bytes(op);
  long long nS = 0, nA = 0;
  for (auto& q : lv->mp) {
    const int kg = kgroup_of(op);
    nS = std::max(nS, q.tabS + (long long)((q.kbS + kg - 1) / kg * kg) * lv->RB);
    nA = std::max(nA, q.tabA + (long long)lv->kb2 * q.rbA);
  }
  tabS.assign((size_t)nS * bb, 0);
  tabA.assign((size_t)nA * bb, 0);
  // eps_n^m and 1/eps_n^m of the extended layout (n = m..T+1)
  std::vector<ld> eps((size_t)lv->Kx), ieps((size_t)lv->Kx);
  for (int m = 0; m <= T; ++m)
    for (int n = m; n <= T + 1; ++n) {
      ld e = (n > m) ? std::sqrt((ld)(n * n - m * m) / (ld)(4 * n * n - 1)) : 0;
      eps[ext_off(T, m) + n - m] = e;
      ieps[ext_off(T, m) + n - m] = (n > m) ? 1 / e : 0;
    }
  // recurrence per northern ring
  std::vector<ld> row(T + 3);
  for (int j = 0; j < J; ++j) {
    ld x = lv->mu_h[j];
    ld s = std::sqrt((1 - x) * (1 + x));
    ld pmm = 1 / std::sqrt((ld)2);
    for (int m = 0; m <= T; ++m) {
      if (m > 0) pmm = std::sqrt((ld)(2 * m + 1) / (ld)(2 * m)) * s * pmm;
      row[0] = pmm;
      row[1] = std::sqrt((ld)(2 * m + 3)) * x * pmm;
      const ld* em = eps.data() + ext_off(T, m) - m;     // em[n] = eps_n^m
      const ld* im = ieps.data() + ext_off(T, m) - m;
      for (int n = m + 2; n <= T + 1; ++n)
        row[n - m] = (x * row[n - m - 1] - em[n - 1] * row[n - m - 2]) * im[n];
      for (int p = 0; p < 2; ++p) {
        const MPInfo& q = lv->mp[2 * m + p];
        for (int i = 0; i < q.np; ++i) {
          double v = (double)row[p + 2 * i];
          if (std::fabs(v) < 1e-290) v = 0.0;
          // synthesis: rows = rings j, k = i; FP32 / FP64 in k-groups counted
          // from the highest k-block down (the order the contraction runs)
          {
            int KB = lv->KB;
            if (op == OP_BF16X3) {
              long long blk = q.tabS + (long long)(i / KB) * lv->RB + j / 16;
              put(op, tabS.data(), blk, op_lane(op, j % 16, i % KB), op_elem(op, i % KB), v);
            } else {
              const long long r = (long long)(q.kbS - 1) - i / KB;   // descending k-block
              const long long e = kgroup_elem(q.tabS, lv->RB, r, j / 16,
                                              op_lane(op, j % 16, i % KB), kgroup_of(op));
              if (op == OP_F64)
                reinterpret_cast<double*>(tabS.data())[e] = v;
              else
                reinterpret_cast<float*>(tabS.data())[e] = (float)v;
            }
          }
          // analysis: rows = degrees i, k = rings j; FP32 / FP64 in k-groups
          {
            int KB = lv->KB;
            if (op == OP_BF16X3) {
              long long blk = q.tabA + (long long)(j / KB) * q.rbA + i / 16;
              put(op, tabA.data(), blk, op_lane(op, i % 16, j % KB), op_elem(op, j % KB), v);
            } else {
              const long long e = kgroup_elem(q.tabA, q.rbA, j / KB, i / 16,
                                              op_lane(op, i % 16, j % KB), kgroup_of(op));
              if (op == OP_F64)
                reinterpret_cast<double*>(tabA.data())[e] = v;
              else
                reinterpret_cast<float*>(tabA.data())[e] = (float)v;
            }
          }
        }
      }
    }
  }
}

// Recurrence mode: instead of the packed tables, the values that restart the
// two-degree recurrence every kRecChunk degrees of one parity, and its
// coefficients.  With x P_k = e_{k+1} P_{k+1} + e_k P_{k-1} applied twice,
//   e_{n+1} e_{n+2} P_{n+2} = (x^2 - e_{n+1}^2 - e_n^2) P_n - e_n e_{n-1} P_{n-2},
// so a = 1 / (e_{n+1} e_{n+2}), b = e_{n+1}^2 + e_n^2, c = e_n e_{n-1} (e_k = 0
// for k <= m).  The restart pairs come from the same 80-bit recurrence as the
// tables, one ring at a time.
void build_recurrence(pfsh_level* lv, std::vector<double>& seeds, std::vector<double>& rec) {
  const int T = lv->T, J = lv->J, Jp = lv->Jp;
  long long nch = 0;
  for (auto& q : lv->mp) {
    q.seed = nch;
    nch += rec_chunks(q.np);
  }
  seeds.assign((size_t)nch * Jp * 2, 0.0);
  rec.assign((size_t)lv->Kx * 4, 0.0);
  // e_n^m of the extended layout (n = m..T+1)
  std::vector<ld> ev((size_t)lv->Kx);
  for (int m = 0; m <= T; ++m)
    for (int n = m; n <= T + 1; ++n)
      ev[ext_off(T, m) + n - m] = n > m ? std::sqrt((ld)(n * n - m * m) / (ld)(4 * n * n - 1)) : 0;
  auto eps = [&](int n, int m) -> ld { return ev[ext_off(T, m) + n - m]; };
  for (int m = 0; m <= T; ++m)
    for (int n = m; n + 2 <= T + 1; ++n) {
      const ld e0 = eps(n, m), e1 = eps(n + 1, m), e2 = eps(n + 2, m);
      const ld em = n - 1 >= m ? eps(n - 1, m) : 0;
      double* r = rec.data() + (size_t)(ext_off(T, m) + n - m) * 4;
      r[0] = (double)(1 / (e1 * e2));
      r[1] = (double)(e1 * e1 + e0 * e0);
      r[2] = (double)(e0 * em);
    }
  std::vector<ld> row(T + 3);
  for (int j = 0; j < J; ++j) {
    const ld x = lv->mu_h[j];
    const ld sn = std::sqrt((1 - x) * (1 + x));
    ld pmm = 1 / std::sqrt((ld)2);
    for (int m = 0; m <= T; ++m) {
      if (m > 0) pmm = std::sqrt((ld)(2 * m + 1) / (ld)(2 * m)) * sn * pmm;
      row[0] = pmm;
      row[1] = std::sqrt((ld)(2 * m + 3)) * x * pmm;
      for (int n = m + 2; n <= T + 1; ++n)
        row[n - m] = (x * row[n - m - 1] - eps(n - 1, m) * row[n - m - 2]) / eps(n, m);
      for (int p = 0; p < 2; ++p) {
        const MPInfo& q = lv->mp[2 * m + p];
        for (int c = 0; c < rec_chunks(q.np); ++c) {
          const int d0 = p + 2 * kRecChunk * c;             // n0 - m
          double* sd = seeds.data() + ((size_t)(q.seed + c) * Jp + j) * 2;
          sd[0] = d0 >= 2 ? (double)row[d0 - 2] : 0.0;
          sd[1] = (double)row[d0];
        }
      }
    }
  }
}

}  // namespace pfsh
