// MFMA operand types of the three transform precisions (gfx950).
//
//   OpF64   v_mfma_f64_16x16x4_f64            FP64 operands, FP64 accumulate
//   OpF32   v_mfma_f32_16x16x4_f32            FP32 operands, FP32 accumulate
//   OpBF3   v_mfma_f32_16x16x32_bf16 (x3)     x = hi + lo (bf16 each), products
//                                             hi*hi + hi*lo + lo*hi, FP32 accumulate
// Operand blocks: lane l holds A[l % 16][k] and B[k][l % 16] with k = l / 16
// (16x16x4) or k = 8 (l / 16) + e, e = 0..7 (16x16x32).  A 16x16 output block
// holds column l % 16 in lane l; the rows differ: FP32 and BF16 accumulate rows
// 4 (l / 16) + v, FP64 rows (l / 16) + 4 v, v = 0..3 (checked on gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "pfsh_internal.h"

namespace pfsh {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

struct Bf16Pair {
  bf8_t hi, lo;
};

__device__ __forceinline__ unsigned short bf16_bits_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_float(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}

struct OpF64 {
  typedef double R;       // transform real type
  typedef double Acc;     // accumulator scalar
  typedef double A;       // per-lane operand
  typedef d4_t C;
  static constexpr int KIND = OP_F64;
  static constexpr int KB = 4;
  __device__ static __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
  __device__ static __forceinline__ A load(const void* base, long long blk, int lane) {
    return reinterpret_cast<const double*>(base)[blk * 64 + lane];
  }
  __device__ static __forceinline__ A zero() { return 0.0; }
  __device__ static __forceinline__ C mma(A a, A b, C c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ void store(void* base, long long blk, int lane, int, R v) {
    reinterpret_cast<double*>(base)[blk * 64 + lane] = v;
  }
};

struct OpF32 {
  typedef float R;
  typedef float Acc;
  typedef float A;
  typedef f4_t C;
  static constexpr int KIND = OP_F32;
  static constexpr int KB = 4;
  __device__ static __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  __device__ static __forceinline__ A load(const void* base, long long blk, int lane) {
    return reinterpret_cast<const float*>(base)[blk * 64 + lane];
  }
  __device__ static __forceinline__ A zero() { return 0.0f; }
  __device__ static __forceinline__ C mma(A a, A b, C c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ void store(void* base, long long blk, int lane, int, R v) {
    reinterpret_cast<float*>(base)[blk * 64 + lane] = v;
  }
};

struct OpBF3 {
  typedef float R;
  typedef float Acc;
  typedef Bf16Pair A;
  typedef f4_t C;
  static constexpr int KIND = OP_BF16X3;
  static constexpr int KB = 32;
  __device__ static __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  __device__ static __forceinline__ A load(const void* base, long long blk, int lane) {
    const bf8_t* p = reinterpret_cast<const bf8_t*>(base) + (blk * 64 + lane) * 2;
    A a;
    a.hi = p[0];
    a.lo = p[1];
    return a;
  }
  __device__ static __forceinline__ A zero() {
    A a;
    for (int i = 0; i < 8; ++i) {
      a.hi[i] = (__bf16)0.0f;
      a.lo[i] = (__bf16)0.0f;
    }
    return a;
  }
  __device__ static __forceinline__ C mma(const A& a, const A& b, C c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, c, 0, 0, 0);
    return c;
  }
  // element e of lane `lane`: hi at [lane*16 + e], lo at [lane*16 + 8 + e]
  __device__ static __forceinline__ void store(void* base, long long blk, int lane, int e, R v) {
    unsigned short* h = reinterpret_cast<unsigned short*>(base) + (blk * 64 + lane) * 16;
    unsigned short hi = bf16_bits_rne(v);
    unsigned short lo = bf16_bits_rne(v - bf16_bits_to_float(hi));
    h[e] = hi;
    h[8 + e] = lo;
  }
};

// K loop of one wave's 2x2 blocks: A blocks at ta, ta+1 (+astep per k-block),
// B blocks at tb, tb+1 (+bstep); R1 / C1: the second block row / column
// exists.  Operands are loaded PF k-blocks ahead into a register ring, so the
// memory latency overlaps PF k-blocks of matrix work.  The loop body has no
// branches (prefetch addresses past the last k-block are clamped to it, and
// those copies are never used; the last nk mod PF k-blocks run in a tail), so
// every MFMA waits only for its own operands.
// A wave-uniform value moved to scalar registers (address arithmetic on the
// scalar unit; only the lane offset stays per lane).
__device__ __forceinline__ long long wave_uniform(long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v & 0xffffffffu));
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// FP32 accumulation runs in two chains, k-blocks of even and of odd index
// (added at the end): each sequential sum is half as long, which halves the
// accumulated round-off of the long Legendre sums.  Every FP32 K loop below
// uses the same rule, so all tile variants give the same bits.
template <class Op>
struct SplitAcc {
  static constexpr bool value = Op::KIND == OP_F32;
};

template <class Op, int PF, bool R1, bool C1>
__device__ __forceinline__ void mma_loop_rc(const void* __restrict__ A, const void* __restrict__ B,
                                            long long ta, long long astep, long long tb,
                                            long long bstep, int nk, int lane,
                                            typename Op::C& acc00, typename Op::C& acc01,
                                            typename Op::C& acc10, typename Op::C& acc11) {
  constexpr bool SPL = SplitAcc<Op>::value;
  static_assert(!SPL || PF % 2 == 0, "two accumulation chains need an even prefetch depth");
  ta = wave_uniform(ta);
  tb = wave_uniform(tb);
  astep = wave_uniform(astep);
  bstep = wave_uniform(bstep);
  nk = __builtin_amdgcn_readfirstlane(nk);
  if (nk <= 0) return;
  typename Op::C x00 = {}, x01 = {}, x10 = {}, x11 = {};   // odd k-blocks (SPL)
  typename Op::A a0[PF], a1[PF], b0[PF], b1[PF];
#pragma unroll
  for (int s = 0; s < PF; ++s) {
    const long long k = s < nk ? s : nk - 1;
    a0[s] = Op::load(A, ta + k * astep, lane);
    if (R1) a1[s] = Op::load(A, ta + k * astep + 1, lane);
    b0[s] = Op::load(B, tb + k * bstep, lane);
    if (C1) b1[s] = Op::load(B, tb + k * bstep + 1, lane);
  }
  // k-block k0 + s has the parity of s (k0 is a multiple of PF)
  auto step = [&](int s) {
    typename Op::C& c00 = (SPL && (s & 1)) ? x00 : acc00;
    typename Op::C& c01 = (SPL && (s & 1)) ? x01 : acc01;
    typename Op::C& c10 = (SPL && (s & 1)) ? x10 : acc10;
    typename Op::C& c11 = (SPL && (s & 1)) ? x11 : acc11;
    c00 = Op::mma(a0[s], b0[s], c00);
    if (C1) c01 = Op::mma(a0[s], b1[s], c01);
    if (R1) c10 = Op::mma(a1[s], b0[s], c10);
    if (R1 && C1) c11 = Op::mma(a1[s], b1[s], c11);
  };
  int k0 = 0;
  for (; k0 + PF <= nk; k0 += PF) {
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      step(s);
      const int kn = k0 + s + PF;
      const long long k = kn < nk ? kn : nk - 1;
      a0[s] = Op::load(A, ta + k * astep, lane);
      if (R1) a1[s] = Op::load(A, ta + k * astep + 1, lane);
      b0[s] = Op::load(B, tb + k * bstep, lane);
      if (C1) b1[s] = Op::load(B, tb + k * bstep + 1, lane);
    }
  }
#pragma unroll
  for (int s = 0; s < PF - 1; ++s)
    if (k0 + s < nk) step(s);
  if constexpr (SPL) {
    acc00 += x00;
    acc01 += x01;
    acc10 += x10;
    acc11 += x11;
  }
}

// The 2x2 K loop with the edge flags taken once per wave.  Every argument but
// the accumulators and `lane` must be uniform over the wave.
// k-grouped A operand (the analysis table of FP32 and FP64 levels): KG
// consecutive k-blocks of one lane are contiguous, 16 bytes, so one load
// instruction brings a lane KG k-blocks.  The vector memory path issues about
// as many wave loads per cycle for 16 bytes per lane as for 4, so this cuts the
// table's load instructions by KG.  Element of k-block k, block t (stride S
// blocks per k-block), lane l, in a region starting at block base:
// kgroup_elem(base, S, k, t, l, KG) (pfsh_internal.h).  The data operand keeps
// the plain block layout: its producer, the ring stage, writes one ring per
// workgroup, and k-grouped it would write 4-byte pieces of 16-byte groups
// shared by four workgroups (measured: ring stage 48 -> 77 us at T255 x 16).
template <class Op>
struct KGroup {
  static constexpr int KG = Op::KIND == OP_BF16X3 ? 1 : 16 / (int)sizeof(typename Op::R);
};

template <class Op>
struct GrpVec;
template <>
struct GrpVec<OpF32> {
  typedef f4_t V;
};
template <>
struct GrpVec<OpF64> {
  typedef d2_t V;
};

// K loop of one wave's 2x2 blocks with a k-grouped A operand: A group-block
// index ta (+astep per group of KG k-blocks), B plain blocks at tb (+bstep per
// k-block, negative for the synthesis, which runs from the highest k-block
// down and groups its table in that order), ng whole groups, then rem (0..KG-1)
// k-blocks of a last, padded group.  The MFMAs of a group run in k order, so
// every block sees the k-blocks in the order (and FP32 chains) of
// mma_loop_rc: the same bits.  Branch-free like mma_loop_rc but for the rem
// tail.
template <class Op, int PF, bool R1, bool C1>
__device__ __forceinline__ void mma_loop_grp_rc(const void* __restrict__ A,
                                                const void* __restrict__ B, long long ta,
                                                long long astep, long long tb, long long bstep,
                                                int ng, int rem, int lane, typename Op::C& acc00,
                                                typename Op::C& acc01, typename Op::C& acc10,
                                                typename Op::C& acc11) {
  typedef typename GrpVec<Op>::V V;
  constexpr int KG = KGroup<Op>::KG;
  constexpr bool SPL = SplitAcc<Op>::value;
  static_assert(!SPL || KG % 2 == 0, "two accumulation chains need an even group");
  const V* Av = reinterpret_cast<const V*>(A);
  ta = wave_uniform(ta);
  tb = wave_uniform(tb);
  astep = wave_uniform(astep);
  bstep = wave_uniform(bstep);
  ng = __builtin_amdgcn_readfirstlane(ng);
  rem = __builtin_amdgcn_readfirstlane(rem);
  typename Op::C x00 = {}, x01 = {}, x10 = {}, x11 = {};   // odd k-blocks (SPL)
  V a0[PF], a1[PF];
  typename Op::A b0[PF][KG], b1[PF][KG];
  auto load = [&](int s, long long g) {
    a0[s] = Av[(ta + g * astep) * 64 + lane];
    if (R1) a1[s] = Av[(ta + g * astep + 1) * 64 + lane];
#pragma unroll
    for (int e = 0; e < KG; ++e) {
      const long long kb = tb + (g * KG + e) * bstep;
      b0[s][e] = Op::load(B, kb, lane);
      if (C1) b1[s][e] = Op::load(B, kb + 1, lane);
    }
  };
  auto mma_e = [&](int s, int e) {
    typename Op::C& c00 = (SPL && (e & 1)) ? x00 : acc00;
    typename Op::C& c01 = (SPL && (e & 1)) ? x01 : acc01;
    typename Op::C& c10 = (SPL && (e & 1)) ? x10 : acc10;
    typename Op::C& c11 = (SPL && (e & 1)) ? x11 : acc11;
    c00 = Op::mma(a0[s][e], b0[s][e], c00);
    if (C1) c01 = Op::mma(a0[s][e], b1[s][e], c01);
    if (R1) c10 = Op::mma(a1[s][e], b0[s][e], c10);
    if (R1 && C1) c11 = Op::mma(a1[s][e], b1[s][e], c11);
  };
  auto step = [&](int s) {
#pragma unroll
    for (int e = 0; e < KG; ++e) mma_e(s, e);
  };
  if (ng > 0) {
#pragma unroll
    for (int s = 0; s < PF; ++s) load(s, s < ng ? s : ng - 1);
    int g0 = 0;
    for (; g0 + PF <= ng; g0 += PF) {
#pragma unroll
      for (int s = 0; s < PF; ++s) {
        step(s);
        const int gn = g0 + s + PF;
        load(s, gn < ng ? gn : ng - 1);
      }
    }
#pragma unroll
    for (int s = 0; s < PF - 1; ++s)
      if (g0 + s < ng) step(s);
  }
  if (rem > 0) {   // k-blocks g KG + e, e < rem, of the last group
    a0[0] = Av[(ta + ng * astep) * 64 + lane];
    if (R1) a1[0] = Av[(ta + ng * astep + 1) * 64 + lane];
#pragma unroll
    for (int e = 0; e < KG - 1; ++e) {
      if (e < rem) {
        const long long kb = tb + ((long long)ng * KG + e) * bstep;
        b0[0][e] = Op::load(B, kb, lane);
        if (C1) b1[0][e] = Op::load(B, kb + 1, lane);
      }
    }
#pragma unroll
    for (int e = 0; e < KG - 1; ++e)
      if (e < rem) mma_e(0, e);
  }
  if constexpr (SPL) {
    acc00 += x00;
    acc01 += x01;
    acc10 += x10;
    acc11 += x11;
  }
}

template <class Op, int PF>
__device__ __forceinline__ void mma_loop_grp(const void* __restrict__ A,
                                             const void* __restrict__ B, long long ta,
                                             long long astep, long long tb, long long bstep,
                                             int ng, int rem, bool r1, bool c1, int lane,
                                             typename Op::C& acc00, typename Op::C& acc01,
                                             typename Op::C& acc10, typename Op::C& acc11) {
  if (r1 && c1)
    mma_loop_grp_rc<Op, PF, true, true>(A, B, ta, astep, tb, bstep, ng, rem, lane, acc00, acc01, acc10, acc11);
  else if (r1)
    mma_loop_grp_rc<Op, PF, true, false>(A, B, ta, astep, tb, bstep, ng, rem, lane, acc00, acc01, acc10, acc11);
  else if (c1)
    mma_loop_grp_rc<Op, PF, false, true>(A, B, ta, astep, tb, bstep, ng, rem, lane, acc00, acc01, acc10, acc11);
  else
    mma_loop_grp_rc<Op, PF, false, false>(A, B, ta, astep, tb, bstep, ng, rem, lane, acc00, acc01, acc10, acc11);
}

// K loop of one wave's RT x CT blocks with a k-grouped A operand (the
// synthesis table, grouped from its highest k-block down): A group-blocks ta +
// r (+astep per group), B plain blocks tb + c (+bstep per k-block), ng whole
// groups then rem k-blocks of a padded last group.  Rows r >= nr and columns
// c >= nc repeat the last valid one (their results are not stored), so the
// loop has no branches; each valid block sees the k-blocks in the order and
// FP32 chains of mma_loop_rc: the same bits.
template <class Op, int PF, int RT, int CT>
__device__ __forceinline__ void mma_tile_grp(const void* __restrict__ A, const void* __restrict__ B,
                                             long long ta, long long astep, long long tb,
                                             long long bstep, int ng, int rem, int nr, int nc,
                                             int lane, typename Op::C (&acc)[RT][CT]) {
  typedef typename GrpVec<Op>::V V;
  constexpr int KG = KGroup<Op>::KG;
  constexpr bool SPL = SplitAcc<Op>::value;
  const V* Av = reinterpret_cast<const V*>(A);
  ta = wave_uniform(ta);
  tb = wave_uniform(tb);
  astep = wave_uniform(astep);
  bstep = wave_uniform(bstep);
  ng = __builtin_amdgcn_readfirstlane(ng);
  rem = __builtin_amdgcn_readfirstlane(rem);
  nr = __builtin_amdgcn_readfirstlane(nr);
  nc = __builtin_amdgcn_readfirstlane(nc);
  int ro[RT], co[CT];
#pragma unroll
  for (int r = 0; r < RT; ++r) ro[r] = r < nr ? r : nr - 1;
#pragma unroll
  for (int c = 0; c < CT; ++c) co[c] = c < nc ? c : nc - 1;
  typename Op::C x[RT][CT] = {};   // odd k-blocks (SPL)
  V a[PF][RT];
  typename Op::A b[PF][KG][CT];
  auto load = [&](int s, long long g) {
#pragma unroll
    for (int r = 0; r < RT; ++r) a[s][r] = Av[(ta + g * astep + ro[r]) * 64 + lane];
#pragma unroll
    for (int e = 0; e < KG; ++e)
#pragma unroll
      for (int c = 0; c < CT; ++c) b[s][e][c] = Op::load(B, tb + (g * KG + e) * bstep + co[c], lane);
  };
  auto mma_e = [&](int s, int e) {
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        typename Op::C& t = (SPL && (e & 1)) ? x[r][c] : acc[r][c];
        t = Op::mma(a[s][r][e], b[s][e][c], t);
      }
  };
  if (ng > 0) {
#pragma unroll
    for (int s = 0; s < PF; ++s) load(s, s < ng ? s : ng - 1);
    int g0 = 0;
    for (; g0 + PF <= ng; g0 += PF) {
#pragma unroll
      for (int s = 0; s < PF; ++s) {
#pragma unroll
        for (int e = 0; e < KG; ++e) mma_e(s, e);
        const int gn = g0 + s + PF;
        load(s, gn < ng ? gn : ng - 1);
      }
    }
#pragma unroll
    for (int s = 0; s < PF - 1; ++s)
      if (g0 + s < ng) {
#pragma unroll
        for (int e = 0; e < KG; ++e) mma_e(s, e);
      }
  }
  if (rem > 0) {   // k-blocks ng KG + e, e < rem, of the last group
#pragma unroll
    for (int r = 0; r < RT; ++r) a[0][r] = Av[(ta + ng * astep + ro[r]) * 64 + lane];
#pragma unroll
    for (int e = 0; e < KG - 1; ++e)
      if (e < rem) {
#pragma unroll
        for (int c = 0; c < CT; ++c)
          b[0][e][c] = Op::load(B, tb + ((long long)ng * KG + e) * bstep + co[c], lane);
      }
#pragma unroll
    for (int e = 0; e < KG - 1; ++e)
      if (e < rem) mma_e(0, e);
  }
  if constexpr (SPL) {
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[r][c] += x[r][c];
  }
}

// K loop of one wave's NR x 2 blocks (NR = 1..4 degree blocks, C1: second
// column block present) with a k-grouped A operand, as mma_loop_grp_rc: the
// data operand is loaded once per k-block and column for NR row blocks, so a
// taller tile needs fewer load instructions per MFMA (4 x 2: 12 loads per 32
// MFMAs against 10 per 16 for 2 x 2).  Same k order and chains: same bits.
template <class Op, int PF, int NR, bool C1>
__device__ __forceinline__ void mma_loop_grp_tall(const void* __restrict__ A,
                                                  const void* __restrict__ B, long long ta,
                                                  long long astep, long long tb, long long bstep,
                                                  int ng, int lane, typename Op::C (&acc)[4][2]) {
  typedef typename GrpVec<Op>::V V;
  constexpr int KG = KGroup<Op>::KG;
  constexpr bool SPL = SplitAcc<Op>::value;
  const V* Av = reinterpret_cast<const V*>(A);
  ta = wave_uniform(ta);
  tb = wave_uniform(tb);
  astep = wave_uniform(astep);
  bstep = wave_uniform(bstep);
  ng = __builtin_amdgcn_readfirstlane(ng);
  if (ng <= 0) return;
  typename Op::C x[NR][2] = {};   // odd k-blocks (SPL)
  V a[PF][NR];
  typename Op::A b[PF][KG][2];
  auto load = [&](int s, long long g) {
#pragma unroll
    for (int r = 0; r < NR; ++r) a[s][r] = Av[(ta + g * astep + r) * 64 + lane];
#pragma unroll
    for (int e = 0; e < KG; ++e) {
      const long long kb = tb + (g * KG + e) * bstep;
      b[s][e][0] = Op::load(B, kb, lane);
      if (C1) b[s][e][1] = Op::load(B, kb + 1, lane);
    }
  };
#pragma unroll
  for (int s = 0; s < PF; ++s) load(s, s < ng ? s : ng - 1);
  auto step = [&](int s) {
#pragma unroll
    for (int e = 0; e < KG; ++e)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        typename Op::C& c0 = (SPL && (e & 1)) ? x[r][0] : acc[r][0];
        c0 = Op::mma(a[s][r][e], b[s][e][0], c0);
        if (C1) {
          typename Op::C& c1 = (SPL && (e & 1)) ? x[r][1] : acc[r][1];
          c1 = Op::mma(a[s][r][e], b[s][e][1], c1);
        }
      }
  };
  int g0 = 0;
  for (; g0 + PF <= ng; g0 += PF) {
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      step(s);
      const int gn = g0 + s + PF;
      load(s, gn < ng ? gn : ng - 1);
    }
  }
#pragma unroll
  for (int s = 0; s < PF - 1; ++s)
    if (g0 + s < ng) step(s);
  if constexpr (SPL) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      acc[r][0] += x[r][0];
      if (C1) acc[r][1] += x[r][1];
    }
  }
}

template <class Op, int PF>
__device__ __forceinline__ void mma_loop(const void* __restrict__ A, const void* __restrict__ B,
                                         long long ta, long long astep, long long tb,
                                         long long bstep, int nk, bool r1, bool c1, int lane,
                                         typename Op::C& acc00, typename Op::C& acc01,
                                         typename Op::C& acc10, typename Op::C& acc11) {
  if (r1 && c1)
    mma_loop_rc<Op, PF, true, true>(A, B, ta, astep, tb, bstep, nk, lane, acc00, acc01, acc10, acc11);
  else if (r1)
    mma_loop_rc<Op, PF, true, false>(A, B, ta, astep, tb, bstep, nk, lane, acc00, acc01, acc10, acc11);
  else if (c1)
    mma_loop_rc<Op, PF, false, true>(A, B, ta, astep, tb, bstep, nk, lane, acc00, acc01, acc10, acc11);
  else
    mma_loop_rc<Op, PF, false, false>(A, B, ta, astep, tb, bstep, nk, lane, acc00, acc01, acc10, acc11);
}

}  // namespace pfsh
