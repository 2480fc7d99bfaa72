// Longitude stage of the transform (Sec. 3, first step) and the grid-point
// nonlinear products of Sec. 2, one pair of equator-symmetric rings per
// workgroup, everything resident in LDS.
//
// Two real rings are carried as one complex signal (north in the real part,
// south in the imaginary part), so a length-nlon complex FFT transforms both.
// The FFT is a self-sorting (Stockham) transform with radix-16 stages first
// (then 8/4/2 and a final radix 3): at every stage each thread reads its
// butterflies' inputs into registers, the workgroup synchronizes, and the
// outputs are written back in place; LDS signals are padded against bank
// conflicts.  The last stage of the inverse transforms is fused with the grid
// products (each thread owns its butterflies' points in all four fields).
//
// k_ring_rhs: Fourier coefficients of Phi', zeta, U = u cos(phi), V = v cos(phi)
//   (parity form E/O per m) -> grid -> eta = zeta + 2 Omega mu, A = eta U,
//   B = eta V, C = Phi' U, D = Phi' V, E = (U^2 + V^2)/2 -> Fourier coefficients
//   weighted by w_j / ((1 - mu_j^2) nlon), in parity form (north +- south),
//   written as the analysis data operand; workgroups are ordered XCD-aware.
//   256 or 512 threads per workgroup (a tuner variant).
// k_ring_synth / k_ring_anal: the same longitude step for scalar fields.
#include "mfma_ops.h"

namespace pfsh {

// Aligned to its full size, so that an LDS access of one complex is a single
// 64-bit (FP32) or 128-bit (FP64) access: a pair of 32-bit (64-bit) accesses
// with stride-2 lanes would reach only half of the banks per pass.
template <typename R>
struct alignas(2 * sizeof(R)) cpx {
  R x, y;
};
template <typename R>
__device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// LDS signals are padded by one element every 16 so that the strided
// accesses of the Stockham stages spread over the banks.
__host__ __device__ constexpr int padded(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded_len(int n) { return n + (n >> 4); }
// Stride between signals: one element more than the padded length, so that the
// same index of consecutive signals (read together when lanes run over the
// fields) falls in different banks; padded lengths are often whole multiples
// of the 128-byte bank row.
__host__ __device__ constexpr int sig_stride(int n) { return padded_len(n) + 1; }

// radix of stage s for a length-N transform with radices up to CAP (16, 8 or
// 4): the largest first, then 8, 4, 2, then a 3
__host__ __device__ constexpr int radix_of(int N, int s, int CAP = 16) {
  int n = N, st = 0;
  while (CAP >= 16 && n % 16 == 0) { if (st == s) return 16; n /= 16; ++st; }
  while (CAP >= 8 && n % 8 == 0) { if (st == s) return 8; n /= 8; ++st; }
  while (n % 4 == 0) { if (st == s) return 4; n /= 4; ++st; }
  while (n % 2 == 0) { if (st == s) return 2; n /= 2; ++st; }
  while (n % 3 == 0) { if (st == s) return 3; n /= 3; ++st; }
  return 0;
}
__host__ __device__ constexpr int nstages(int N, int CAP = 16) {
  int s = 0;
  while (radix_of(N, s, CAP) != 0) ++s;
  return s;
}
// NS (product of the earlier radices) of stage s
__host__ __device__ constexpr int ns_before(int N, int s, int CAP) {
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= radix_of(N, i, CAP);
  return ns;
}
// Offset of stage s's twiddle table, laid out [r - 1][k] (r = 1..RAD-1,
// k = 0..NS-1) with the stages that have NS > 1 back to back, and the total.
__host__ __device__ constexpr int tw_off(int N, int s, int CAP) {
  int o = 0;
  for (int i = 0; i < s; ++i) {
    const int ns = ns_before(N, i, CAP);
    if (ns > 1) o += (radix_of(N, i, CAP) - 1) * ns;
  }
  return o;
}
__host__ __device__ constexpr int tw_total(int N, int CAP) { return tw_off(N, nstages(N, CAP), CAP); }

// e^{SIGN 2 pi i k / 16}
template <int SIGN, typename R>
__device__ __forceinline__ cpx<R> w16(int k) {
  constexpr double c[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                            0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                            -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                            0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
  return {(R)c[k & 15], (R)(SIGN * c[(k + 12) & 15])};
}

template <int SIGN, typename R>
__device__ __forceinline__ void bfly4(cpx<R>& a0, cpx<R>& a1, cpx<R>& a2, cpx<R>& a3) {
  cpx<R> s02 = a0 + a2, d02 = a0 - a2, s13 = a1 + a3, d13 = a1 - a3;
  cpx<R> jd = {-(R)SIGN * d13.y, (R)SIGN * d13.x};
  a0 = s02 + s13;
  a1 = d02 + jd;
  a2 = s02 - s13;
  a3 = d02 - jd;
}

// In-register DFT of length RAD: y[k] = sum_p a[p] e^{SIGN 2 pi i p k / RAD}.
// RAD = R1 R2 is split as a[q + R1 p] -> inner length-R2 DFTs over p, twiddles
// e^{SIGN 2 pi i q s / RAD}, outer length-R1 DFTs over q, y[s + R2 t].
template <int RAD, int SIGN, typename R>
__device__ __forceinline__ void butterfly(cpx<R>* a) {
  if constexpr (RAD == 2) {
    cpx<R> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
  } else if constexpr (RAD == 3) {
    const R h = (R)0.86602540378443864676;  // sqrt(3)/2
    cpx<R> t = a[1] + a[2], d = a[1] - a[2];
    cpx<R> m = {a[0].x - (R)0.5 * t.x, a[0].y - (R)0.5 * t.y};
    cpx<R> r = {-(R)SIGN * h * d.y, (R)SIGN * h * d.x};
    a[0] = a[0] + t;
    a[1] = m + r;
    a[2] = m - r;
  } else if constexpr (RAD == 4) {
    bfly4<SIGN>(a[0], a[1], a[2], a[3]);
  } else if constexpr (RAD == 8) {
    // R1 = 2, R2 = 4
    bfly4<SIGN>(a[0], a[2], a[4], a[6]);
    bfly4<SIGN>(a[1], a[3], a[5], a[7]);
    cpx<R> b1[4] = {a[1], cmul(a[3], w16<SIGN, R>(2)), cmul(a[5], w16<SIGN, R>(4)),
                    cmul(a[7], w16<SIGN, R>(6))};
    cpx<R> b0[4] = {a[0], a[2], a[4], a[6]};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      a[s] = b0[s] + b1[s];
      a[s + 4] = b0[s] - b1[s];
    }
  } else {  // 16: R1 = R2 = 4
    cpx<R> b[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cpx<R> t0 = a[q], t1 = a[q + 4], t2 = a[q + 8], t3 = a[q + 12];
      bfly4<SIGN>(t0, t1, t2, t3);
      b[q][0] = t0;
      b[q][1] = q ? cmul(t1, w16<SIGN, R>(q)) : t1;
      b[q][2] = q ? cmul(t2, w16<SIGN, R>(2 * q)) : t2;
      b[q][3] = q ? cmul(t3, w16<SIGN, R>(3 * q)) : t3;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      cpx<R> t0 = b[0][s], t1 = b[1][s], t2 = b[2][s], t3 = b[3][s];
      bfly4<SIGN>(t0, t1, t2, t3);
      a[s] = t0;
      a[s + 4] = t1;
      a[s + 8] = t2;
      a[s + 12] = t3;
    }
  }
}

// a * w (SIGN > 0) or a * conj(w) (SIGN < 0)
template <int SIGN, typename R>
__device__ __forceinline__ cpx<R> cmul_s(cpx<R> a, cpx<R> w) {
  if constexpr (SIGN > 0) return {a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x};
  else return {a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
}

// Twiddle factors of butterfly k (k = j mod NS) of a stage with NS > 1, from
// this stage's LDS table [r - 1][k] (TWLDS: consecutive k, constant offsets)
// or from the base table e^{2 pi i t / N}, t = r k N / (NS RAD).
template <typename R, int N, int RAD, int SIGN, int NS, bool TWLDS>
__device__ __forceinline__ void stage_twiddles(cpx<R>* v, const cpx<R>* tw, int k) {
  if constexpr (NS > 1) {
    constexpr int STEP = N / (NS * RAD);
    if constexpr (TWLDS) {
      const cpx<R>* tk = tw + k;
#pragma unroll
      for (int r = 1; r < RAD; ++r) v[r] = cmul_s<SIGN>(v[r], tk[(r - 1) * NS]);
    } else {
      const cpx<R>* tk = tw + k * STEP;
#pragma unroll
      for (int r = 1; r < RAD; ++r) v[r] = cmul_s<SIGN>(v[r], tk[(r - 1) * k * STEP]);
    }
  }
}

// One Stockham stage on NSIG padded signals of length N stored back to back
// in buf (stride sig_stride(N)); twiddles from this stage's LDS table
// (TWLDS) or from the base table tw[t] = e^{2 pi i t / N}.  Element i of a
// signal sits at padded(i).  When the RAD inputs j + r NB of a butterfly (and
// its outputs base + r NS) stay in step with the padding -- NB (NS) a multiple
// of 16, or an output run of RAD | 16 elements aligned to RAD -- their padded
// addresses are one base plus r times a constant, so the LDS accesses take
// immediate offsets instead of per-element index arithmetic.
template <typename R, int N, int RAD, int NSIG, int NT, int SIGN, int NS, bool TWLDS>
__device__ __forceinline__ void fft_stage(cpx<R>* buf, const cpx<R>* tw) {
  constexpr int NB = N / RAD;
  constexpr int TOT = NB * NSIG;
  constexpr int PER = (TOT + NT - 1) / NT;
  constexpr int STEP = N / (NS * RAD);
  constexpr int SP = sig_stride(N);
  constexpr bool kInConst = NB % 16 == 0;
  constexpr bool kOutConst = NS % 16 == 0 || (NS == 1 && 16 % RAD == 0);
  constexpr int IN_STRIDE = padded_len(NB);
  constexpr int OUT_STRIDE = NS % 16 == 0 ? padded_len(NS) : 1;
  cpx<R> v[PER][RAD];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = threadIdx.x + q * NT;
    if (TOT % NT == 0 || t < TOT) {
      const int sig = t / NB, j = t - sig * NB, k = j % NS;
      const cpx<R>* b = buf + sig * SP;
      if constexpr (kInConst) {
        const cpx<R>* pj = b + padded(j);
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[q][r] = pj[r * IN_STRIDE];
      } else {
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[q][r] = b[padded(j + r * NB)];
      }
      stage_twiddles<R, N, RAD, SIGN, NS, TWLDS>(v[q], tw, k);
      butterfly<RAD, SIGN>(v[q]);
    }
  }
  // The last stage (NB = NS) writes each butterfly's outputs where its inputs
  // were, in the same thread, so it needs no barrier between reads and writes.
  if constexpr (NB != NS) __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = threadIdx.x + q * NT;
    if (TOT % NT == 0 || t < TOT) {
      const int sig = t / NB, j = t - sig * NB, k = j % NS;
      cpx<R>* b = buf + sig * SP;
      const int base = (j / NS) * NS * RAD + k;
      if constexpr (kOutConst) {
        cpx<R>* pb = b + padded(base);
#pragma unroll
        for (int r = 0; r < RAD; ++r) pb[r * OUT_STRIDE] = v[q][r];
      } else {
#pragma unroll
        for (int r = 0; r < RAD; ++r) b[padded(base + r * NS)] = v[q][r];
      }
    }
  }
  __syncthreads();
}

// Twiddles: for FP32 each workgroup builds the per-stage tables (tw_off
// layout) in LDS from the base table, so that a stage's threads read
// consecutive entries; FP64 reads the base table through the cache from global
// memory (staging measured slower there).
template <typename R, int N, int CAP>
struct Twiddles {
  static constexpr bool kLds = sizeof(R) == 4;
  static constexpr int kLdsElems = kLds ? tw_total(N, CAP) : 0;
  // stage S's table: entry (r - 1) NS + k = e^{2 pi i r k STEP / N}, STEP = N / (NS RAD)
  template <int S = 0, int NS = 1>
  __device__ static __forceinline__ void fill(cpx<R>* lds, const cpx<R>* __restrict__ g) {
    if constexpr (S < nstages(N, CAP)) {
      constexpr int RAD = radix_of(N, S, CAP);
      if constexpr (NS > 1) {
        constexpr int off = tw_off(N, S, CAP), cnt = (RAD - 1) * NS, STEP = N / (NS * RAD);
        for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
          const int r = 1 + q / NS, kk = q - (r - 1) * NS;
          lds[off + q] = g[r * kk * STEP];
        }
      }
      fill<S + 1, NS * RAD>(lds, g);
    }
  }
  __device__ static __forceinline__ const cpx<R>* setup(cpx<R>* lds, const cpx<R>* __restrict__ g) {
    if constexpr (kLds) {
      fill(lds, g);
      return lds;  // the caller's next __syncthreads publishes the tables
    } else {
      return g;
    }
  }
};

// stages S .. SEND - 1 (SEND < 0: all)
template <typename R, int N, int NSIG, int NT, int SIGN, int CAP = 16, int SEND = -1, int S = 0,
          int NS = 1>
__device__ __forceinline__ void fft_run(cpx<R>* buf, const cpx<R>* tw) {
  if constexpr (S < (SEND < 0 ? nstages(N, CAP) : SEND)) {
    constexpr int RAD = radix_of(N, S, CAP);
    constexpr bool L = Twiddles<R, N, CAP>::kLds;
    fft_stage<R, N, RAD, NSIG, NT, SIGN, NS, L>(buf, L ? tw + tw_off(N, S, CAP) : tw);
    fft_run<R, N, NSIG, NT, SIGN, CAP, SEND, S + 1, NS * RAD>(buf, tw);
  }
}

// The analysis data operand is kept in 16 x 4 blocks of the transform real
// type for every precision (BF16x3 splits it into hi/lo when loading).
template <class Op>
struct GOp {
  typedef OpF32 T;
};
template <>
struct GOp<OpF64> {
  typedef OpF64 T;
};

// Write one complex value (re, im at columns c, c+1) of degree-parity p of
// order m for ring j into the analysis data operand.
template <class Op>
__device__ __forceinline__ void put_g(void* G, int kb2, int CBa, int m, int p, int j, int c,
                                      typename Op::R re, typename Op::R im) {
  const int KB = Op::KB;
  const long long blk0 = ((long long)(2 * m + p) * kb2 + j / KB) * CBa;
  const int k = j % KB;
  const int e = (Op::KIND == OP_BF16X3) ? (k & 7) : 0;
  const int lk = (Op::KIND == OP_BF16X3) ? (k >> 3) : k;
  Op::store(G, blk0 + c / 16, lk * 16 + (c % 16), e, re);
  const int c1 = c + 1;
  Op::store(G, blk0 + c1 / 16, lk * 16 + (c1 % 16), e, im);
}

// Fourier coefficients of a north/south pair from the parity form -> two-for-one
// complex spectrum (positive exponent synthesis convention).
template <typename R>
__device__ __forceinline__ void load_pair(cpx<R>* sig, int N, int m, cpx<R> E, cpx<R> O) {
  cpx<R> xn = E + O, xs = E - O;
  if (m == 0) {
    sig[0] = {xn.x, xs.x};
  } else {
    sig[padded(m)] = {xn.x - xs.y, xn.y + xs.x};
    sig[padded(N - m)] = {xn.x + xs.y, xs.x - xn.y};
  }
}

// Split the forward spectrum of north + i south into the two real spectra.
template <typename R>
__device__ __forceinline__ void split_pair(const cpx<R>* sig, int N, int m, cpx<R>& yn,
                                           cpx<R>& ys) {
  cpx<R> z = sig[padded(m)], w = sig[padded(m ? N - m : 0)];
  yn = {(R)0.5 * (z.x + w.x), (R)0.5 * (z.y - w.y)};
  ys = {(R)0.5 * (z.y + w.y), (R)0.5 * (w.x - z.x)};
}

template <class Op, int N, int CAP, int NT>
__global__ __launch_bounds__(NT) void k_ring_rhs(const typename Op::R* __restrict__ F4,
                                                 void* __restrict__ G,
                                                 const double* __restrict__ mu,
                                                 const double* __restrict__ wq,
                                                 const cpx<typename Op::R>* __restrict__ twg, int J,
                                                 int nstate, int L, int Lp, int kb2, int CBa,
                                                 double two_omega) {
  typedef typename Op::R R;
  constexpr int SP = sig_stride(N);
  extern __shared__ unsigned char smem_raw[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem_raw);
  cpx<R>* twl = buf + 5 * SP;
  // Block id -> (ring pair j, state b), XCD-aware: the hardware deals block ids
  // to the 8 XCDs in turn, so XCD x takes the contiguous range [x per, (x+1) per)
  // of (j, b) with b fastest.  The workgroups that write the same cache lines
  // of the analysis operand (ring pairs j, j^1 and neighbouring states) then run
  // on one XCD close in time, and its L2 merges their partial lines.
  const int nwg = J * nstate, per = (nwg + 7) / 8;
  const int slot = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (slot >= nwg) return;                              // whole workgroup, before any barrier
  const int j = slot / nstate, b = slot - j * nstate, tid = threadIdx.x;
  const cpx<R>* tw = Twiddles<R, N, CAP>::setup(twl, twg);
  // orders L .. N - L carry no coefficient; the loads below fill the others
  for (int t = L + tid; t <= N - L; t += NT) {
#pragma unroll
    for (int f = 0; f < 4; ++f) buf[f * SP + padded(t)] = {(R)0, (R)0};
  }
  // the (b, j) region of the Fourier workspace, parity 0 then parity 1, each
  // [m / MG][field][m % MG]: consecutive threads read consecutive values
  constexpr int MG = f4_mg(sizeof(R));
  const cpx<R>* src = reinterpret_cast<const cpx<R>*>(F4) + f4_index(b, j, 0, 0, 0, J, 4, Lp, MG);
  for (int i = tid; i < 4 * Lp; i += NT) {
    const int mi = i % MG, f = (i / MG) & 3, m = (i / (4 * MG)) * MG + mi;
    if (m < L) load_pair<R>(buf + f * SP, N, m, src[i], src[4 * Lp + i]);
  }
  __syncthreads();
  const double muj = mu[j];
  const R fn = (R)(two_omega * muj), fs = -fn;
  // grid products at one point k of the four fields (north in x, south in y)
  auto products = [&](int pk, cpx<R> ph, cpx<R> ze, cpx<R> u, cpx<R> v) {
    const R en = ze.x + fn, es = ze.y + fs;
    buf[pk] = {en * u.x, es * u.y};
    buf[SP + pk] = {en * v.x, es * v.y};
    buf[2 * SP + pk] = {ph.x * u.x, ph.y * u.y};
    buf[3 * SP + pk] = {ph.x * v.x, ph.y * v.y};
    buf[4 * SP + pk] = {(R)0.5 * (u.x * u.x + v.x * v.x), (R)0.5 * (u.y * u.y + v.y * v.y)};
  };
  constexpr int SL = nstages(N, CAP) - 1;                 // last stage: NB = NS = N / RAD
  constexpr int RL = radix_of(N, SL, CAP), NBL = N / RL;
  if constexpr (NBL % 16 == 0) {
    // The last inverse stage and the products in one pass: a thread owns
    // butterfly j of all four signals, whose outputs j + r NB are the points
    // it read, so nothing else touches them before the next barrier.
    fft_run<R, N, 4, NT, +1, CAP, SL>(buf, tw);
    constexpr bool TL = Twiddles<R, N, CAP>::kLds;
    const cpx<R>* twl_last = TL ? tw + tw_off(N, SL, CAP) : tw;
    for (int jb = tid; jb < NBL; jb += NT) {
      cpx<R> v[4][RL];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const cpx<R>* pj = buf + f * SP + padded(jb);
#pragma unroll
        for (int r = 0; r < RL; ++r) v[f][r] = pj[r * padded_len(NBL)];
        stage_twiddles<R, N, RL, +1, NBL, TL>(v[f], twl_last, jb);
        butterfly<RL, +1>(v[f]);
      }
#pragma unroll
      for (int r = 0; r < RL; ++r)
        products(padded(jb) + r * padded_len(NBL), v[0][r], v[1][r], v[2][r], v[3][r]);
    }
  } else {
    fft_run<R, N, 4, NT, +1, CAP>(buf, tw);
    for (int k = tid; k < N; k += NT) {
      const int pk = padded(k);
      products(pk, buf[pk], buf[SP + pk], buf[2 * SP + pk], buf[3 * SP + pk]);
    }
  }
  __syncthreads();
  fft_run<R, N, 5, NT, -1, CAP>(buf, tw);
  const R scale = (R)(wq[j] / ((1.0 - muj * muj) * (double)N));
  // Analysis operand: 16 x 4 blocks [m][parity][j / 4][column / 16] of the
  // transform real type, ring j % 4 and column % 16 within; field f of state b
  // is the column pair (re, im) 10 b + 2 f, both in one block and adjacent.
  // Lanes run over (m, f) with f fastest, so that a store instruction writes
  // the 40-byte runs of a dozen orders rather than 64 scattered pairs.
  const size_t pstride = (size_t)kb2 * CBa * 32;   // parity step, in pairs
  cpx<R>* gj = reinterpret_cast<cpx<R>*>(reinterpret_cast<R*>(G) + (size_t)(j >> 2) * CBa * 64 + (j & 3) * 16);
  for (int i = tid; i < 5 * L; i += NT) {
    const int m = i / 5, f = i - m * 5;
    cpx<R> yn, ys;
    split_pair<R>(buf + f * SP, N, m, yn, ys);
    const int c = b * 10 + 2 * f;
    cpx<R>* g0 = gj + (size_t)m * (2 * pstride) + (((c >> 4) * 64 + (c & 15)) >> 1);
    cpx<R> gp = {(yn.x + ys.x) * scale, (yn.y + ys.y) * scale};
    cpx<R> gm = {(yn.x - ys.x) * scale, (yn.y - ys.y) * scale};
    if (m == 0) { gp.y = 0; gm.y = 0; }
    g0[0] = gp;
    g0[pstride] = gm;
  }
}

// scalar synthesis: Fourier workspace (slice 0, nf fields) -> grid [nf][nlat][N]
template <class Op, int N>
__global__ __launch_bounds__(256) void k_ring_synth(const typename Op::R* __restrict__ F4,
                                                   double* __restrict__ grid,
                                                   const cpx<typename Op::R>* __restrict__ twg,
                                                   int J, int L, int Lp, int nf) {
  typedef typename Op::R R;
  constexpr int SP = sig_stride(N);
  extern __shared__ unsigned char smem_raw[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem_raw);
  cpx<R>* twl = buf + 4 * SP;
  constexpr int NT = 256;
  const int j = blockIdx.x, f0 = blockIdx.y * 4, tid = threadIdx.x;
  const cpx<R>* tw = Twiddles<R, N, 16>::setup(twl, twg);
  for (int i = tid; i < 4 * SP; i += NT) buf[i] = {(R)0, (R)0};
  __syncthreads();
  for (int i = tid; i < 4 * L; i += NT) {
    const int fl = i / L, m = i - fl * L, f = f0 + fl;
    if (f >= nf) continue;
    const R* e = F4 + 2 * f4_index(0, j, f, 0, m, J, nf, Lp, f4_mg(sizeof(R)));
    const R* o = F4 + 2 * f4_index(0, j, f, 1, m, J, nf, Lp, f4_mg(sizeof(R)));
    load_pair<R>(buf + fl * SP, N, m, cpx<R>{e[0], e[1]}, cpx<R>{o[0], o[1]});
  }
  __syncthreads();
  fft_run<R, N, 4, NT, +1>(buf, tw);
  const int nlat = 2 * J;
  for (int i = tid; i < 4 * N; i += NT) {
    const int fl = i / N, k = i - fl * N, f = f0 + fl;
    if (f >= nf) continue;
    const cpx<R> z = buf[fl * SP + padded(k)];
    grid[((size_t)f * nlat + j) * N + k] = (double)z.x;
    grid[((size_t)f * nlat + (nlat - 1 - j)) * N + k] = (double)z.y;
  }
}

// scalar analysis: grid [nf][nlat][N] -> analysis data operand, weight w_j / N
template <class Op, int N>
__global__ __launch_bounds__(256) void k_ring_anal(const double* __restrict__ grid,
                                                  void* __restrict__ G,
                                                  const double* __restrict__ wq,
                                                  const cpx<typename Op::R>* __restrict__ twg,
                                                  int J, int L, int nf, int kb2, int CBa) {
  typedef typename Op::R R;
  constexpr int SP = sig_stride(N);
  extern __shared__ unsigned char smem_raw[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem_raw);
  cpx<R>* twl = buf + 4 * SP;
  constexpr int NT = 256;
  const int j = blockIdx.x, f0 = blockIdx.y * 4, tid = threadIdx.x;
  const int nlat = 2 * J;
  const cpx<R>* tw = Twiddles<R, N, 16>::setup(twl, twg);
  for (int i = tid; i < 4 * N; i += NT) {
    const int fl = i / N, k = i - fl * N, f = f0 + fl;
    cpx<R> z = {(R)0, (R)0};
    if (f < nf)
      z = {(R)grid[((size_t)f * nlat + j) * N + k], (R)grid[((size_t)f * nlat + (nlat - 1 - j)) * N + k]};
    buf[fl * SP + padded(k)] = z;
  }
  __syncthreads();
  fft_run<R, N, 4, NT, -1>(buf, tw);
  const R scale = (R)(wq[j] / (double)N);
  for (int i = tid; i < 4 * L; i += NT) {
    const int m = i / 4, fl = i - m * 4, f = f0 + fl;
    if (f >= nf) continue;
    cpx<R> yn, ys;
    split_pair<R>(buf + fl * SP, N, m, yn, ys);
    cpx<R> gp = {(yn.x + ys.x) * scale, (yn.y + ys.y) * scale};
    cpx<R> gm = {(yn.x - ys.x) * scale, (yn.y - ys.y) * scale};
    if (m == 0) { gp.y = 0; gm.y = 0; }
    put_g<typename GOp<Op>::T>(G, kb2, CBa, m, 0, j, 2 * f, gp.x, gp.y);
    put_g<typename GOp<Op>::T>(G, kb2, CBa, m, 1, j, 2 * f, gm.x, gm.y);
  }
}

// ---------------------------------------------------------------- dispatch
template <class Op, int N, int CAP, int NT = 256>
static hipError_t ring_launch(int kind, const pfsh_level* lv, int count, const double* gin,
                              double* gout, hipStream_t s) {
  typedef typename Op::R R;
  const cpx<R>* tw = reinterpret_cast<const cpx<R>*>(lv->tw_d);
  size_t shm;
  const size_t twl = (size_t)Twiddles<R, N, 16>::kLdsElems * sizeof(cpx<R>);
  if (kind == 0) {
    shm = (size_t)5 * sig_stride(N) * sizeof(cpx<R>) +
          (size_t)Twiddles<R, N, CAP>::kLdsElems * sizeof(cpx<R>);
    if (shm > 65536)
      (void)hipFuncSetAttribute((const void*)k_ring_rhs<Op, N, CAP, NT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    const int per = (lv->J * count + 7) / 8;
    PFSH_LAUNCH(lv, (k_ring_rhs<Op, N, CAP, NT>), dim3(8 * per), dim3(NT), shm, s,
                       (const R*)lv->F4, lv->G, lv->mu_d, lv->w_d, tw, lv->J, count, lv->L, lv->Lp,
                       lv->kb2g, lv->CBa, 2.0 * lv->d.omega);
  } else if (kind == 1) {
    shm = (size_t)4 * sig_stride(N) * sizeof(cpx<R>) + twl;
    if (shm > 65536)
      (void)hipFuncSetAttribute((const void*)k_ring_synth<Op, N>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    PFSH_LAUNCH(lv, (k_ring_synth<Op, N>), dim3(lv->J, (count + 3) / 4), dim3(256), shm, s,
                       (const R*)lv->F4, gout, tw, lv->J, lv->L, lv->Lp, count);
  } else {
    shm = (size_t)4 * sig_stride(N) * sizeof(cpx<R>) + twl;
    if (shm > 65536)
      (void)hipFuncSetAttribute((const void*)k_ring_anal<Op, N>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    PFSH_LAUNCH(lv, (k_ring_anal<Op, N>), dim3(lv->J, (count + 3) / 4), dim3(256), shm, s,
                       gin, lv->G, lv->w_d, tw, lv->J, lv->L, count, lv->kb2g, lv->CBa);
  }
  return hipGetLastError();
}

// Ring-stage variants (index 0 = default): the largest FFT radix, 16, 8 or 4,
// with 256 threads per workgroup, and radix 16 with 512 threads (twice the
// waves per CU where the LDS of a ring pair allows few workgroups, e.g. FP64 or
// T511); RHS kernel only, the scalar transforms use radix 16 and 256 threads.
int ring_variant_count() { return 4; }

template <class Op, int N>
static hipError_t ring_cap(int kind, const pfsh_level* lv, int count, const double* gin,
                           double* gout, hipStream_t s) {
  const int v = kind == 0 ? lv->variant[TS_RING][tune_bucket(count)] : 0;
  if (v == 1) return ring_launch<Op, N, 8>(kind, lv, count, gin, gout, s);
  if (v == 2) return ring_launch<Op, N, 4>(kind, lv, count, gin, gout, s);
  if (v == 3) return ring_launch<Op, N, 16, 512>(kind, lv, count, gin, gout, s);
  return ring_launch<Op, N, 16>(kind, lv, count, gin, gout, s);
}

template <class Op>
static hipError_t ring_by_n(int kind, const pfsh_level* lv, int count, const double* gin,
                            double* gout, hipStream_t s) {
  switch (lv->nlon) {
    case 16: return ring_cap<Op, 16>(kind, lv, count, gin, gout, s);
    case 24: return ring_cap<Op, 24>(kind, lv, count, gin, gout, s);
    case 32: return ring_cap<Op, 32>(kind, lv, count, gin, gout, s);
    case 48: return ring_cap<Op, 48>(kind, lv, count, gin, gout, s);
    case 64: return ring_cap<Op, 64>(kind, lv, count, gin, gout, s);
    case 96: return ring_cap<Op, 96>(kind, lv, count, gin, gout, s);
    case 128: return ring_cap<Op, 128>(kind, lv, count, gin, gout, s);
    case 192: return ring_cap<Op, 192>(kind, lv, count, gin, gout, s);
    case 256: return ring_cap<Op, 256>(kind, lv, count, gin, gout, s);
    case 384: return ring_cap<Op, 384>(kind, lv, count, gin, gout, s);
    case 512: return ring_cap<Op, 512>(kind, lv, count, gin, gout, s);
    case 768: return ring_cap<Op, 768>(kind, lv, count, gin, gout, s);
    case 1024: return ring_cap<Op, 1024>(kind, lv, count, gin, gout, s);
    case 1536: return ring_cap<Op, 1536>(kind, lv, count, gin, gout, s);
  }
  return hipErrorInvalidValue;
}

static hipError_t ring_dispatch(int kind, const pfsh_level* lv, int count, const double* gin,
                                double* gout, hipStream_t s) {
  switch (lv->op) {
    case OP_F64: return ring_by_n<OpF64>(kind, lv, count, gin, gout, s);
    case OP_F32: return ring_by_n<OpF32>(kind, lv, count, gin, gout, s);
    default: return ring_by_n<OpBF3>(kind, lv, count, gin, gout, s);
  }
}

hipError_t launch_ring_rhs(const pfsh_level* lv, int batch, hipStream_t s) {
  return ring_dispatch(0, lv, batch, nullptr, nullptr, s);
}
hipError_t launch_ring_synth(const pfsh_level* lv, int nfields, double* grid, hipStream_t s) {
  return ring_dispatch(1, lv, nfields, nullptr, grid, s);
}
hipError_t launch_ring_anal(const pfsh_level* lv, int nfields, const double* grid, hipStream_t s) {
  return ring_dispatch(2, lv, nfields, grid, nullptr, s);
}

}  // namespace pfsh
