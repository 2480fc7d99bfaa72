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
// Default tiles: analysis, one workgroup of 4 waves per (m, p) and 64 degrees x
// 64 columns; synthesis, one wave per order for MC consecutive orders of one
// parity, 32 rings x 32 columns each; every wave owns 2x2 MFMA blocks of 16x16.
// Tuner variants change the prefetch depth and the tile (64 x 64 per wave,
// one degree block per wave), never the order of a sum.  Operands are
// pre-packed in MFMA lane order (tables at level creation, data by the
// producing kernels), so each lane loads its fragment with one contiguous load;
// the analysis table of FP32 and FP64 levels is k-grouped (four or two
// k-blocks of a lane in 16 bytes), since the rate of wave load instructions,
// not bytes, bounds these contractions.  The K loops (mfma_ops.h) run without
// branches, FP32 in two accumulation chains.
#include <algorithm>

#include "mfma_ops.h"

namespace pfsh {

// Block id -> (work item, column tile), XCD-aware: the hardware deals
// consecutive block ids to the 8 XCDs in turn, so item i goes to XCD i % 8 and
// all column tiles of an item run on that XCD back to back, sharing its table
// and operand lines in that XCD's L2.  Items keep their heaviest-first order.
__device__ __forceinline__ bool xcd_tile(int nitems, int nct, int& item, int& ct) {
  const int L = blockIdx.x, xcd = L & 7, r = L >> 3;
  ct = r % nct;
  item = (r / nct) * 8 + xcd;
  return item < nitems;
}

// The same with `per` sub-tiles per item (ring tile x column tile): all of an
// item's sub-tiles run on one XCD, back to back.
__device__ __forceinline__ bool xcd_group(int nitems, int per, int& item, int& sub) {
  const int L = blockIdx.x, xcd = L & 7, r = L >> 3;
  sub = r % per;
  item = (r / per) * 8 + xcd;
  return item < nitems;
}

template <typename R, int MC>
__device__ __forceinline__ void store_run(R* dst, const R* v) {
  if constexpr (sizeof(R) == 4) {
#pragma unroll
    for (int h = 0; h < MC; h += 4)
      *reinterpret_cast<float4*>(dst + h) = make_float4(v[h], v[h + 1], v[h + 2], v[h + 3]);
  } else {
#pragma unroll
    for (int h = 0; h < MC; h += 2)
      *reinterpret_cast<double2*>(dst + h) = make_double2(v[h], v[h + 1]);
  }
}

// Store a staged output tile: NROWS rings from j0 (stage rows of 32 real
// columns, SM = MC + 1 per column) x 16 complex columns from real column c0,
// MC consecutive orders from m0, into the Fourier workspace (f4_index, MG =
// MC).  One 16-byte store per thread with lanes over (order quarter, column,
// ring): a wave writes the whole-field runs of four slices of one ring, 4 x 256
// contiguous bytes (FP32 or FP64, 4 fields).
template <typename R, int MC, int NROWS>
__device__ __forceinline__ void store_f4_tile(R* __restrict__ F4, const R* stage, int j0, int c0,
                                              int J, int ncols, int nf, int p, int m0, int Lp) {
  static_assert(MC == f4_mg(sizeof(R)), "one synthesis workgroup holds one order group");
  constexpr int SM = MC + 1, VPT = 16 / (2 * (int)sizeof(R)), NQ = MC / VPT;
  for (int t = threadIdx.x; t < NROWS * 16 * NQ; t += blockDim.x) {
    const int qq = t % NQ, cp = (t / NQ) & 15, r = t / (NQ * 16);
    const int j = j0 + r, c = c0 + 2 * cp;
    if (j >= J || c >= ncols) continue;
    const int bf = c >> 1, f = bf % nf, b = bf / nf;
    const R* re = stage + (r * 32 + 2 * cp) * SM + qq * VPT;
    const R* im = re + SM;
    R out[2 * VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v) {
      out[2 * v] = re[v];
      out[2 * v + 1] = im[v];
    }
    store_run<R, 2 * VPT>(F4 + 2 * f4_index(b, j, f, p, m0 + qq * VPT, J, nf, Lp, MC), out);
  }
}

// One workgroup: MC consecutive orders m0..m0+MC-1 of one parity, a tile of
// 32 rings x 32 columns; wave w computes order m0 + w (2x2 MFMA blocks).  The
// waves then exchange their tiles through LDS, and the tile is stored in
// whole-field runs of the MC orders (store_f4_tile) for the ring stage.
template <class Op, int MC, int PF, int HS = 32>
__global__ __launch_bounds__(64 * MC) void k_leg_synth(const void* __restrict__ tab,
                                                      const void* __restrict__ X,
                                                      typename Op::R* __restrict__ F4,
                                                      const MPInfo* __restrict__ mpi,
                                                      const WorkItem* __restrict__ items,
                                                      int nitems, int ntile, int nct, int RB, int CBs,
                                                      int CBn, int ncols, int nf, int J, int T,
                                                      int Lp) {
  typedef typename Op::R R;
  constexpr int SM = MC + 1;                  // padded m-stride of the LDS tile
  __shared__ R stage[HS * 32 * SM];           // [row][column][m], HS rows per round
  int item;
  int sub;
  if (!xcd_group(nitems, ntile * nct, item, sub)) return;
  const int tile = sub / nct, ct = sub - tile * nct;
  const WorkItem it = items[item];
  const int p = it.mp & 1, m0 = it.mp >> 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rb0 = tile * 2, cb0 = ct * 2;
  const bool r1 = rb0 + 1 < RB, c1 = cb0 + 1 < CBn;
  const int m = m0 + wave;
  typename Op::C acc[4] = {};
  if (m <= T) {
    // degrees from the highest down: the coefficients decay with n, so the
    // small terms are summed before the large low-degree ones
    const MPInfo q = mpi[2 * m + p];
    const long long last = q.kbS - 1;
    constexpr int KG = KGroup<Op>::KG;
    if constexpr (KG > 1) {
      // table k-grouped from the highest k-block down: (PF + KG - 1) / KG groups ahead
      mma_loop_grp<Op, (PF + KG - 1) / KG>(tab, X, q.tabS / KG + rb0, (long long)RB,
                                           q.xS + cb0 + last * CBs, -(long long)CBs, q.kbS / KG,
                                           q.kbS % KG, r1, c1, lane, acc[0], acc[1], acc[2],
                                           acc[3]);
    } else {
      mma_loop<Op, PF>(tab, X, q.tabS + rb0 + last * RB, -(long long)RB,
                       q.xS + cb0 + last * CBs, -(long long)CBs, q.kbS, r1, c1, lane, acc[0],
                       acc[1], acc[2], acc[3]);
    }
  }
  // HS = 32: one exchange of the whole tile; HS = 16: two rounds of one row
  // block each (half the LDS, so more workgroups fit on a CU)
#pragma unroll
  for (int h = 0; h < 32 / HS; ++h) {
    if (h > 0) __syncthreads();                          // the previous round has been read
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
      if (HS == 16 && (blk >> 1) != h) continue;
      const int rr = HS == 16 ? 0 : (blk >> 1) * 16, cc = (blk & 1) * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        stage[((rr + Op::row(lane, v)) * 32 + cc) * SM + wave] = (R)acc[blk][v];
    }
    __syncthreads();
    store_f4_tile<R, MC, HS>(F4, stage, rb0 * 16 + h * HS, cb0 * 16, J, ncols, nf, p, m0, Lp);
  }
}

// The same with a 64-ring x 64-column tile per wave (4x4 MFMA blocks: the
// table and the data operand are each read half as often).  The LDS exchange
// runs in four rounds of one 32 x 32 quadrant, so it needs no more LDS.
template <class Op, int MC, int PF>
__global__ __launch_bounds__(64 * MC) void k_leg_synth_t4(const void* __restrict__ tab,
                                                         const void* __restrict__ X,
                                                         typename Op::R* __restrict__ F4,
                                                         const MPInfo* __restrict__ mpi,
                                                         const WorkItem* __restrict__ items,
                                                         int nitems, int ntile, int nct, int RB,
                                                         int CBs, int CBn, int ncols, int nf, int J,
                                                         int T, int Lp) {
  typedef typename Op::R R;
  constexpr int SM = MC + 1;
  __shared__ R stage[32 * 32 * SM];
  int item;
  int sub;
  if (!xcd_group(nitems, ntile * nct, item, sub)) return;
  const int tile = sub / nct, ct = sub - tile * nct;
  const WorkItem it = items[item];
  const int p = it.mp & 1, m0 = it.mp >> 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rb0 = tile * 4, cb0 = ct * 4;
  const int nr = min(4, RB - rb0), nc = min(4, CBn - cb0);
  const int m = m0 + wave;
  typename Op::C acc[4][4] = {};
  if (m <= T) {
    const MPInfo q = mpi[2 * m + p];
    const long long last = q.kbS - 1;
    constexpr int KG = KGroup<Op>::KG;
    mma_tile_grp<Op, (PF + KG - 1) / KG, 4, 4>(tab, X, q.tabS / KG + rb0, (long long)RB,
                                               q.xS + cb0 + last * CBs, -(long long)CBs,
                                               q.kbS / KG, q.kbS % KG, nr, nc, lane, acc);
  }
#pragma unroll
  for (int qd = 0; qd < 4; ++qd) {
    const int qr = qd >> 1, qc = qd & 1;
    if (2 * qr >= nr || 2 * qc >= nc) continue;          // uniform over the workgroup
    if (qd > 0) __syncthreads();                          // the previous round has been read
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
      const int rr = (blk >> 1) * 16, cc = (blk & 1) * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        stage[((rr + Op::row(lane, v)) * 32 + cc) * SM + wave] =
            (R)acc[2 * qr + (blk >> 1)][2 * qc + (blk & 1)][v];
    }
    __syncthreads();
    store_f4_tile<R, MC, 32>(F4, stage, (rb0 + 2 * qr) * 16, (cb0 + 2 * qc) * 16, J, ncols, nf, p,
                             m0, Lp);
  }
}

// Tile shapes: SHAPE 0 = 64 degrees x 64 columns (2x2 blocks per wave),
// SHAPE 1 = 64 degrees x 32 columns with one row block per wave (1x2 blocks),
// which keeps all four waves busy when there are only one or two column
// blocks (small batches).
// BF16x3 B fragment of one 32-ring k-block from the FP32 analysis operand: lane
// l takes rings 8 (l / 16) + e, e = 0..7, of column l % 16, i.e. four rows of
// each of two consecutive 16 x 4 blocks (g points at the first block's column,
// `next` blocks apart), split x = hi + lo with both halves rounded to nearest.
__device__ __forceinline__ Bf16Pair load_g_bf3(const float* __restrict__ g, long long next) {
  Bf16Pair r;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float v = g[(e >> 2) * next + (e & 3) * 16];
    const unsigned short hi = bf16_bits_rne(v);
    const unsigned short lo = bf16_bits_rne(v - bf16_bits_to_float(hi));
    r.hi[e] = __builtin_bit_cast(__bf16, hi);
    r.lo[e] = __builtin_bit_cast(__bf16, lo);
  }
  return r;
}

// K loop of one wave's 2x2 BF16x3 blocks with the B operand converted on load;
// g0 = this lane's first float (k-block 0, column block cb0).  Branch-free like
// mma_loop_rc: edge flags as template arguments, clamped prefetch, a tail.
template <int PF, bool R1, bool C1>
__device__ __forceinline__ void mma_loop_bf3g_rc(const void* __restrict__ A,
                                                 const float* __restrict__ G, long long ta,
                                                 long long astep, long long g0, long long gstep,
                                                 long long next, long long gcol, int nk, int lane,
                                                 f4_t& acc00, f4_t& acc01, f4_t& acc10,
                                                 f4_t& acc11) {
  ta = wave_uniform(ta);
  astep = wave_uniform(astep);
  nk = __builtin_amdgcn_readfirstlane(nk);
  if (nk <= 0) return;
  Bf16Pair a0[PF], a1[PF], b0[PF], b1[PF];
#pragma unroll
  for (int s = 0; s < PF; ++s) {
    const long long k = s < nk ? s : nk - 1;
    a0[s] = OpBF3::load(A, ta + k * astep, lane);
    if (R1) a1[s] = OpBF3::load(A, ta + k * astep + 1, lane);
    b0[s] = load_g_bf3(G + g0 + k * gstep, next);
    if (C1) b1[s] = load_g_bf3(G + g0 + k * gstep + gcol, next);
  }
  int k0 = 0;
  for (; k0 + PF <= nk; k0 += PF) {
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      acc00 = OpBF3::mma(a0[s], b0[s], acc00);
      if (C1) acc01 = OpBF3::mma(a0[s], b1[s], acc01);
      if (R1) acc10 = OpBF3::mma(a1[s], b0[s], acc10);
      if (R1 && C1) acc11 = OpBF3::mma(a1[s], b1[s], acc11);
      const int kn = k0 + s + PF;
      const long long k = kn < nk ? kn : nk - 1;
      a0[s] = OpBF3::load(A, ta + k * astep, lane);
      if (R1) a1[s] = OpBF3::load(A, ta + k * astep + 1, lane);
      b0[s] = load_g_bf3(G + g0 + k * gstep, next);
      if (C1) b1[s] = load_g_bf3(G + g0 + k * gstep + gcol, next);
    }
  }
#pragma unroll
  for (int s = 0; s < PF - 1; ++s) {
    if (k0 + s < nk) {
      acc00 = OpBF3::mma(a0[s], b0[s], acc00);
      if (C1) acc01 = OpBF3::mma(a0[s], b1[s], acc01);
      if (R1) acc10 = OpBF3::mma(a1[s], b0[s], acc10);
      if (R1 && C1) acc11 = OpBF3::mma(a1[s], b1[s], acc11);
    }
  }
}

template <int PF>
__device__ __forceinline__ void mma_loop_bf3g(const void* __restrict__ A, const float* __restrict__ G,
                                              long long ta, long long astep, long long g0,
                                              long long gstep, long long next, long long gcol,
                                              int nk, bool r1, bool c1, int lane,
                                              f4_t& acc00, f4_t& acc01, f4_t& acc10, f4_t& acc11) {
  if (r1 && c1)
    mma_loop_bf3g_rc<PF, true, true>(A, G, ta, astep, g0, gstep, next, gcol, nk, lane, acc00, acc01, acc10, acc11);
  else if (r1)
    mma_loop_bf3g_rc<PF, true, false>(A, G, ta, astep, g0, gstep, next, gcol, nk, lane, acc00, acc01, acc10, acc11);
  else if (c1)
    mma_loop_bf3g_rc<PF, false, true>(A, G, ta, astep, g0, gstep, next, gcol, nk, lane, acc00, acc01, acc10, acc11);
  else
    mma_loop_bf3g_rc<PF, false, false>(A, G, ta, astep, g0, gstep, next, gcol, nk, lane, acc00, acc01, acc10, acc11);
}

template <class Op, int PF, int SHAPE>
__global__ __launch_bounds__(256) void k_leg_anal(const void* __restrict__ tab,
                                                 const void* __restrict__ G,
                                                 typename Op::R* __restrict__ Y,
                                                 const MPInfo* __restrict__ mpi,
                                                 const WorkItem* __restrict__ items, int nitems,
                                                 int nct, int kb2, int kb2g, int CBa, int CBn,
                                                 int ncols, int Kx, int T) {
  int item, ct;
  if (!xcd_tile(nitems, nct, item, ct)) return;
  const WorkItem it = items[item];
  const MPInfo q = mpi[it.mp];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rb0 = SHAPE == 0 ? it.tile * 4 + (wave >> 1) * 2 : it.tile * 4 + wave;
  const int cb0 = SHAPE == 0 ? ct * 4 + (wave & 1) * 2 : ct * 2;
  if (rb0 >= q.rbA || cb0 >= CBn) return;
  const bool r1 = SHAPE == 0 && rb0 + 1 < q.rbA, c1 = cb0 + 1 < CBn;
  typename Op::C acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
  if constexpr (Op::KIND == OP_BF16X3) {
    // data operand in 16 x 4 FP32 blocks [mp][kb2g][CBa]: 32-ring k-block kb of
    // lane l starts at 4-ring block 8 kb + 2 (l / 16)
    const long long g0 = (((long long)it.mp * kb2g + 2 * (lane >> 4)) * CBa + cb0) * 64 + (lane & 15);
    mma_loop_bf3g<PF>(tab, reinterpret_cast<const float*>(G), q.tabA + rb0, (long long)q.rbA, g0,
                      8LL * CBa * 64, (long long)CBa * 64, 64, kb2, r1, c1, lane, acc00, acc01,
                      acc10, acc11);
  } else {
    // k-grouped table: PF groups of KG k-blocks in flight
    constexpr int KG = KGroup<Op>::KG;
    mma_loop_grp<Op, PF>(tab, G, q.tabA / KG + rb0, (long long)q.rbA,
                         (long long)it.mp * kb2 * CBa + cb0, (long long)CBa, kb2 / KG, 0, r1,
                         c1, lane, acc00, acc01, acc10, acc11);
  }
  const int base = ext_off(T, q.m) + (q.p ? npar(T, q.m, 0) : 0);   // this parity's run
  auto put = [&](const typename Op::C& acc, int rb, int cb) {
    const int c = cb * 16 + (lane & 15);
    if (c >= ncols) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = rb * 16 + Op::row(lane, v);
      if (i < q.np)
        Y[((size_t)(c >> 1) * Kx + base + i) * 2 + (c & 1)] = (typename Op::R)acc[v];
    }
  };
  put(acc00, rb0, cb0);
  if (c1) put(acc01, rb0, cb0 + 1);
  if (r1) put(acc10, rb0 + 1, cb0);
  if (r1 && c1) put(acc11, rb0 + 1, cb0 + 1);
}

// Tall wave tiles (FP32 / FP64): one workgroup of 2 waves per item (4 degree
// blocks) and tile of 4 column blocks, each wave 4 x 2 blocks; the items and
// column tiles of k_leg_anal's shape 0.  With the k-grouped table, the data
// operand's loads dominate, and a taller tile shares each of them among 4
// degree blocks.
template <class Op, int PF>
__global__ __launch_bounds__(128) void k_leg_anal_tall(const void* __restrict__ tab,
                                                      const void* __restrict__ G,
                                                      typename Op::R* __restrict__ Y,
                                                      const MPInfo* __restrict__ mpi,
                                                      const WorkItem* __restrict__ items,
                                                      int nitems, int nct, int kb2, int CBa,
                                                      int CBn, int ncols, int Kx, int T) {
  int item, ct;
  if (!xcd_tile(nitems, nct, item, ct)) return;
  const WorkItem it = items[item];
  const MPInfo q = mpi[it.mp];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rb0 = it.tile * 4, cb0 = ct * 4 + wave * 2;
  if (rb0 >= q.rbA || cb0 >= CBn) return;
  const int nr = min(4, q.rbA - rb0);
  const bool c1 = cb0 + 1 < CBn;
  constexpr int KG = KGroup<Op>::KG;
  typename Op::C acc[4][2] = {};
  const long long ta = q.tabA / KG + rb0, tb = (long long)it.mp * kb2 * CBa + cb0;
#define PFSH_TALL(N, C)                                                                        \
  mma_loop_grp_tall<Op, PF, N, C>(tab, G, ta, (long long)q.rbA, tb, (long long)CBa, kb2 / KG, \
                                  lane, acc)
  switch (__builtin_amdgcn_readfirstlane(nr) * 2 + (c1 ? 1 : 0)) {
    case 2: PFSH_TALL(1, false); break;
    case 3: PFSH_TALL(1, true); break;
    case 4: PFSH_TALL(2, false); break;
    case 5: PFSH_TALL(2, true); break;
    case 6: PFSH_TALL(3, false); break;
    case 7: PFSH_TALL(3, true); break;
    case 8: PFSH_TALL(4, false); break;
    default: PFSH_TALL(4, true); break;
  }
#undef PFSH_TALL
  const int base = ext_off(T, q.m) + (q.p ? npar(T, q.m, 0) : 0);   // this parity's run
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      if (r >= nr || (cc == 1 && !c1)) continue;
      const int c = (cb0 + cc) * 16 + (lane & 15);
      if (c >= ncols) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = (rb0 + r) * 16 + Op::row(lane, v);
        if (i < q.np)
          Y[((size_t)(c >> 1) * Kx + base + i) * 2 + (c & 1)] = (typename Op::R)acc[r][cc][v];
      }
    }
}

// ------------------------------------------------------------ recurrence mode
// Levels created with PFSH_LEGENDRE_RECURRENCE hold no tables: each workgroup
// evaluates the P_n^m(mu_j) its contraction needs, in FP64, by the two-degree
// recurrence P_{n+2} = a ((mu^2 - b) P_n - c P_{n-2}) restarted every
// kRecChunk degrees of one parity from a stored pair, rounds them to the
// transform type and keeps them in LDS in MFMA operand order; the data operand
// and the outputs are those of the tabulated kernels.

// Makes a wave's LDS writes visible to its own later LDS reads (the LDS
// serves one wave's accesses in order; the fences keep the compiler from
// moving accesses across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One recurrence chunk of one ring: the pair (P_{n0-2}, P_{n0}) from `sd`,
// then kRecChunk values P_{n0}, P_{n0+2}, ... (value t uses the coefficients
// cf[3 (t0 + t)]), each handed to put(t, value); degrees at or past np are 0.
template <typename Put>
__device__ __forceinline__ void rec_chunk(const double* __restrict__ sd, bool live, double x2,
                                          const double* cf, int t0, int i0, int np, Put put) {
  double s0 = 0.0, s1 = 0.0;
  if (live) {
    s0 = sd[0];
    s1 = sd[1];
  }
  put(0, i0 < np ? s1 : 0.0);
#pragma unroll 4
  for (int t = 1; t < kRecChunk; ++t) {
    const double* c3 = cf + 3 * (t0 + t);
    const double s2 = c3[0] * ((x2 - c3[1]) * s1 - c3[2] * s0);
    s0 = s1;
    s1 = s2;
    put(t, i0 + t < np ? s1 : 0.0);
  }
}

// Synthesis, the items and tiles of k_leg_synth (MC orders of one parity, wave
// w takes order m0 + w, 32 rings x 32 columns).  Each wave walks its order's
// degrees from the highest down in slabs of 2 kRecChunk: it loads the slab's
// data-operand fragments, stages the slab's recurrence coefficients, lets lane
// (ring r, chunk h) generate 32 degrees of ring r into its private LDS slab and
// runs the slab's k-blocks, highest first (FP32: two chains by k-block
// parity).  The results go out through the LDS exchange of k_leg_synth.
template <class Op, int MC>
__global__ __launch_bounds__(64 * MC) void k_leg_synth_rec(
    const double* __restrict__ seeds, const double* __restrict__ rec, const double* __restrict__ mu,
    const void* __restrict__ X, typename Op::R* __restrict__ F4, const MPInfo* __restrict__ mpi,
    const WorkItem* __restrict__ items, int nitems, int ntile, int nct, int CBs, int CBn,
    int ncols, int nf, int J, int Jp, int T, int Lp) {
  typedef typename Op::R R;
  typedef typename Op::C C;
  constexpr int SM = MC + 1;
  constexpr int SLAB = 2 * kRecChunk, KPS = SLAB / 4;   // degrees and k-blocks per slab
  constexpr bool SPL = SplitAcc<Op>::value;
  extern __shared__ unsigned char smem_raw[];
  R* slabs = reinterpret_cast<R*>(smem_raw);                                  // [MC][KPS][2][64]
  double* coef = reinterpret_cast<double*>(smem_raw + (size_t)MC * KPS * 128 * sizeof(R));  // [MC][SLAB][3]
  R* stage = slabs;   // the output exchange reuses the slabs once every wave is done
  int item;
  int sub;
  if (!xcd_group(nitems, ntile * nct, item, sub)) return;
  const int tile = sub / nct, ct = sub - tile * nct;
  const WorkItem it = items[item];
  const int p = it.mp & 1, m0 = it.mp >> 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rb0 = tile * 2, cb0 = ct * 2;
  const bool c1 = cb0 + 1 < CBn;
  const int m = m0 + wave;
  C acc[4] = {}, odd[4] = {};
  if (m <= T) {
    const MPInfo q = mpi[2 * m + p];
    R* slab = slabs + (size_t)wave * KPS * 128;
    double* cf = coef + (size_t)wave * SLAB * 3;
    const int r = lane & 31, h = lane >> 5, j = rb0 * 16 + r;
    const double x = j < J ? mu[j] : 0.0, x2 = x * x;
    const int nch = rec_chunks(q.np);
    const int ebase = ext_off(T, m) + p;
    for (int s = (q.np + SLAB - 1) / SLAB - 1; s >= 0; --s) {
      const int kb_lo = s * KPS, kb_hi = min(q.kbS, kb_lo + KPS);
      typename Op::A b0[KPS], b1[KPS];
#pragma unroll
      for (int kl = 0; kl < KPS; ++kl) {
        const long long kb = kb_lo + kl < kb_hi ? kb_lo + kl : kb_hi - 1;
        b0[kl] = Op::load(X, q.xS + cb0 + kb * CBs, lane);
        b1[kl] = c1 ? Op::load(X, q.xS + cb0 + 1 + kb * CBs, lane) : b0[kl];
      }
      wave_lds_sync();   // this wave's reads of the previous slab are done
      {
        const int i = s * SLAB + lane;    // degree index whose coefficients lane stages
        double a = 0.0, b = 0.0, c = 0.0;
        if (i >= 1 && i < q.np) {
          const double* rc = rec + (size_t)(ebase + 2 * (i - 1)) * 4;
          a = rc[0];
          b = rc[1];
          c = rc[2];
        }
        cf[3 * lane] = a;
        cf[3 * lane + 1] = b;
        cf[3 * lane + 2] = c;
      }
      wave_lds_sync();
      const int ch = 2 * s + h;
      rec_chunk(seeds + ((size_t)(q.seed + ch) * Jp + j) * 2, ch < nch && j < J, x2, cf,
                h * kRecChunk, ch * kRecChunk, q.np, [&](int t, double v) {
                  const int dl = h * kRecChunk + t;
                  slab[((dl >> 2) * 2 + (r >> 4)) * 64 + (dl & 3) * 16 + (r & 15)] = (R)v;
                });
      wave_lds_sync();
#pragma unroll
      for (int kl = KPS - 1; kl >= 0; --kl) {
        if (kb_lo + kl >= kb_hi) continue;   // uniform
        const typename Op::A a0 = slab[(kl * 2) * 64 + lane], a1 = slab[(kl * 2 + 1) * 64 + lane];
        auto blocks = [&](C (&d)[4]) {
          d[0] = Op::mma(a0, b0[kl], d[0]);
          if (c1) d[1] = Op::mma(a0, b1[kl], d[1]);
          d[2] = Op::mma(a1, b0[kl], d[2]);
          if (c1) d[3] = Op::mma(a1, b1[kl], d[3]);
        };
        if (SPL && (kl & 1))
          blocks(odd);
        else
          blocks(acc);
      }
    }
  }
  if constexpr (SPL) {
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] += odd[b];
  }
  __syncthreads();   // every wave is done with its slab before the exchange reuses it
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) {
    const int rr = (blk >> 1) * 16, cc = (blk & 1) * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) stage[((rr + Op::row(lane, v)) * 32 + cc) * SM + wave] = (R)acc[blk][v];
  }
  __syncthreads();
  store_f4_tile<R, MC, 32>(F4, stage, rb0 * 16, cb0 * 16, J, ncols, nf, p, m0, Lp);
}

// K loop of one wave's NR x (1 + C1) blocks with the A operand in LDS: the
// lane's element of iteration it at a_lane[it * astep] (second row block 64
// elements on), the data operand from global memory PF k-blocks ahead.  The
// structure of mma_loop_rc: a branch-free main loop (prefetch addresses past
// the end clamped) and a tail; FP32 accumulates in two chains by iteration
// parity, added at the end.
template <class Op, int PF, int NR, bool C1>
__device__ __forceinline__ void mma_loop_lds(const typename Op::R* a_lane, int astep,
                                             const void* __restrict__ B, long long tb,
                                             long long bstep, int nk, int lane,
                                             typename Op::C& acc00, typename Op::C& acc01,
                                             typename Op::C& acc10, typename Op::C& acc11) {
  constexpr bool SPL = SplitAcc<Op>::value;
  static_assert(!SPL || PF % 2 == 0, "two chains need an even prefetch depth");
  tb = wave_uniform(tb);
  bstep = wave_uniform(bstep);
  nk = __builtin_amdgcn_readfirstlane(nk);
  if (nk <= 0) return;
  typename Op::C x00 = {}, x01 = {}, x10 = {}, x11 = {};
  typename Op::A b0[PF], b1[PF];
#pragma unroll
  for (int s = 0; s < PF; ++s) {
    const long long k = s < nk ? s : nk - 1;
    b0[s] = Op::load(B, tb + k * bstep, lane);
    if (C1) b1[s] = Op::load(B, tb + k * bstep + 1, lane);
  }
  auto step = [&](int s, int it) {
    typename Op::C& c00 = (SPL && (s & 1)) ? x00 : acc00;
    typename Op::C& c01 = (SPL && (s & 1)) ? x01 : acc01;
    typename Op::C& c10 = (SPL && (s & 1)) ? x10 : acc10;
    typename Op::C& c11 = (SPL && (s & 1)) ? x11 : acc11;
    const typename Op::A a0 = a_lane[it * astep];
    c00 = Op::mma(a0, b0[s], c00);
    if (C1) c01 = Op::mma(a0, b1[s], c01);
    if (NR > 1) {
      const typename Op::A a1 = a_lane[it * astep + 64];
      c10 = Op::mma(a1, b0[s], c10);
      if (C1) c11 = Op::mma(a1, b1[s], c11);
    }
  };
  int k0 = 0;
  for (; k0 + PF <= nk; k0 += PF) {
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      step(s, k0 + s);
      const int kn = k0 + s + PF;
      const long long k = kn < nk ? kn : nk - 1;
      b0[s] = Op::load(B, tb + k * bstep, lane);
      if (C1) b1[s] = Op::load(B, tb + k * bstep + 1, lane);
    }
  }
#pragma unroll
  for (int s = 0; s < PF - 1; ++s)
    if (k0 + s < nk) step(s, k0 + s);
  if constexpr (SPL) {
    acc00 += x00;
    acc01 += x01;
    acc10 += x10;
    acc11 += x11;
  }
}

// Analysis, the items and column tiles of k_leg_anal shape 0 (one (m, p) and
// 64 degrees = two recurrence chunks per workgroup, 4 waves of 2 x 2 blocks).
// The rings are taken in slabs of SR (64 degrees x SR rings fill 64 KiB): the
// workgroup generates the slab's operand (thread task = (ring, chunk)), then
// every wave runs its blocks over the slab's k-blocks with the data operand
// PF k-blocks ahead (FP32: two chains by k-block parity).  A k-block row of
// the LDS tile is padded by one element so that the generating threads, which
// run over rings, spread over the banks.
template <class Op, int PF>
__global__ __launch_bounds__(256) void k_leg_anal_rec(
    const double* __restrict__ seeds, const double* __restrict__ rec, const double* __restrict__ mu,
    const void* __restrict__ G, typename Op::R* __restrict__ Y, const MPInfo* __restrict__ mpi,
    const WorkItem* __restrict__ items, int nitems, int nct, int kb2, int CBa, int CBn,
    int ncols, int Kx, int J, int Jp, int T) {
  typedef typename Op::R R;
  typedef typename Op::C C;
  constexpr int SR = 65536 / (64 * (int)sizeof(R));   // rings per slab
  constexpr int KS = 4 * 64 + 1;                       // padded k-block row of the tile
  extern __shared__ unsigned char smem_raw[];
  R* As = reinterpret_cast<R*>(smem_raw);                                      // [SR/4][KS]
  double* cf = reinterpret_cast<double*>(smem_raw + (size_t)(SR / 4) * KS * sizeof(R));  // [64][3]
  int item, ct;
  if (!xcd_tile(nitems, nct, item, ct)) return;
  const WorkItem it = items[item];
  const MPInfo q = mpi[it.mp];
  if (it.tile * 4 >= q.rbA) return;                    // padding item (whole workgroup)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rbl = (wave >> 1) * 2, cb0 = ct * 4 + (wave & 1) * 2;
  const bool live = cb0 < CBn, c1 = cb0 + 1 < CBn;
  const int deg0 = it.tile * 64, nch = rec_chunks(q.np), ebase = ext_off(T, q.m) + q.p;
  if (threadIdx.x < 64) {
    const int i = deg0 + threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    if (i >= 1 && i < q.np) {
      const double* rc = rec + (size_t)(ebase + 2 * (i - 1)) * 4;
      a = rc[0];
      b = rc[1];
      c = rc[2];
    }
    cf[3 * threadIdx.x] = a;
    cf[3 * threadIdx.x + 1] = b;
    cf[3 * threadIdx.x + 2] = c;
  }
  C acc[4] = {};
  for (int j0 = 0; j0 < Jp; j0 += SR) {
    const int sr = min(SR, Jp - j0);
    __syncthreads();   // coefficients staged; the previous slab has been read
    for (int task = threadIdx.x; task < 2 * sr; task += 256) {
      const int jj = task % sr, hh = task / sr, j = j0 + jj, ch = 2 * it.tile + hh;
      const double x = j < J ? mu[j] : 0.0;
      R* dst = As + (jj >> 2) * KS + (jj & 3) * 16;
      rec_chunk(seeds + ((size_t)(q.seed + ch) * Jp + j) * 2, ch < nch && j < J, x * x, cf,
                hh * kRecChunk, ch * kRecChunk, q.np, [&](int t, double v) {
                  const int dl = hh * kRecChunk + t;
                  dst[(dl >> 4) * 64 + (dl & 15)] = (R)v;
                });
    }
    __syncthreads();
    if (live) {
      const long long tb = ((long long)it.mp * kb2 + j0 / 4) * CBa + cb0;
      const R* a_lane = As + rbl * 64 + lane;
      if (c1)
        mma_loop_lds<Op, PF, 2, true>(a_lane, KS, G, tb, (long long)CBa, sr / 4, lane, acc[0],
                                      acc[1], acc[2], acc[3]);
      else
        mma_loop_lds<Op, PF, 2, false>(a_lane, KS, G, tb, (long long)CBa, sr / 4, lane, acc[0],
                                       acc[1], acc[2], acc[3]);
    }
  }
  if (!live) return;
  const int base = ext_off(T, q.m) + (q.p ? npar(T, q.m, 0) : 0);   // this parity's run
  const int rb0 = it.tile * 4 + rbl;
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) {
    const int rb = rb0 + (blk >> 1), cb = cb0 + (blk & 1);
    if ((blk & 1) && !c1) continue;
    const int c = cb * 16 + (lane & 15);
    if (c >= ncols) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = rb * 16 + Op::row(lane, v);
      if (i < q.np) Y[((size_t)(c >> 1) * Kx + base + i) * 2 + (c & 1)] = (R)acc[blk][v];
    }
  }
}

// The same contractions with the whole operand block generated once per
// workgroup and kept in LDS while the workgroup runs every column tile: the
// recurrence then costs once per (order, ring block) or (order, degree tile)
// instead of once per column tile.  Used when the block fits in LDS (the
// synthesis up to T511; the analysis tile of 64 degrees x all rings up to 608
// northern rings in FP32 and 288 in FP64); the kernels above serve the rest.

// Synthesis: workgroup = MC orders of one parity x one block of 16 NRB rings,
// wave w the column of order m0 + w ([k-block][NRB row blocks][64 lanes],
// 16 NRB rings x all degrees).  Lane (ring r, chunk h) generates 64 / (16
// NRB) chunks per round; the coefficient staging and then the output exchange
// share one LDS region.  NRB = 2 halves the data-operand loads per MFMA where
// the columns fit.
template <class Op, int MC, int PF, int NRB>
__global__ __launch_bounds__(64 * MC) void k_leg_synth_rec_cols(
    const double* __restrict__ seeds, const double* __restrict__ rec, const double* __restrict__ mu,
    const void* __restrict__ X, typename Op::R* __restrict__ F4, const MPInfo* __restrict__ mpi,
    const WorkItem* __restrict__ items, int nitems, int nrb, int kbmax, int CBs, int CBn,
    int ncols, int nf, int J, int Jp, int T, int Lp) {
  typedef typename Op::R R;
  typedef typename Op::C C;
  constexpr int SM = MC + 1, RW = 16 * NRB;        // rings per workgroup
  constexpr int CPR = 64 / RW, GEN = CPR * kRecChunk;   // chunks and degrees per round
  extern __shared__ unsigned char smem_raw[];
  R* cols = reinterpret_cast<R*>(smem_raw);                          // [MC][kbmax][NRB][64]
  unsigned char* aux = smem_raw + (size_t)MC * kbmax * NRB * 64 * sizeof(R);
  double* coef = reinterpret_cast<double*>(aux);                     // [MC][GEN][3], then
  R* stage = reinterpret_cast<R*>(aux);                              // [16][32][SM]
  int item, rbk;
  if (!xcd_group(nitems, nrb, item, rbk)) return;
  const WorkItem it = items[item];
  const int p = it.mp & 1, m0 = it.mp >> 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = m0 + wave;
  R* P = cols + (size_t)wave * kbmax * NRB * 64;
  int kbS = 0;
  long long xS = 0;
  if (m <= T) {
    const MPInfo q = mpi[2 * m + p];
    kbS = q.kbS;
    xS = q.xS;
    const int r = lane % RW, h = lane / RW, j = rbk * RW + r;
    const double x = j < J ? mu[j] : 0.0, x2 = x * x;
    const int nch = rec_chunks(q.np), ebase = ext_off(T, m) + p;
    double* cf = coef + (size_t)wave * GEN * 3;
    for (int g0 = 0; g0 < q.np; g0 += GEN) {
      wave_lds_sync();   // the previous round's coefficient reads are done
      for (int l = lane; l < GEN; l += 64) {
        const int i = g0 + l;
        double a = 0.0, b = 0.0, c = 0.0;
        if (i >= 1 && i < q.np) {
          const double* rc = rec + (size_t)(ebase + 2 * (i - 1)) * 4;
          a = rc[0];
          b = rc[1];
          c = rc[2];
        }
        cf[3 * l] = a;
        cf[3 * l + 1] = b;
        cf[3 * l + 2] = c;
      }
      wave_lds_sync();
      const int ch = g0 / kRecChunk + h;
      rec_chunk(seeds + ((size_t)(q.seed + ch) * Jp + j) * 2, ch < nch && j < J, x2, cf,
                h * kRecChunk, ch * kRecChunk, q.np, [&](int t, double v) {
                  const int i = ch * kRecChunk + t;
                  if (i < 4 * kbS)
                    P[((i >> 2) * NRB + r / 16) * 64 + (i & 3) * 16 + (r & 15)] = (R)v;
                });
    }
    wave_lds_sync();
  }
  for (int cb0 = 0; cb0 < CBn; cb0 += 2) {
    const bool c1 = cb0 + 1 < CBn;
    C acc[4] = {};
    if (kbS > 0) {   // highest degrees first
      const long long tb = xS + cb0 + (long long)(kbS - 1) * CBs;
      const R* a_lane = P + (size_t)(kbS - 1) * NRB * 64 + lane;
      if (c1)
        mma_loop_lds<Op, PF, NRB, true>(a_lane, -NRB * 64, X, tb, -(long long)CBs, kbS, lane,
                                        acc[0], acc[1], acc[2], acc[3]);
      else
        mma_loop_lds<Op, PF, NRB, false>(a_lane, -NRB * 64, X, tb, -(long long)CBs, kbS, lane,
                                         acc[0], acc[1], acc[2], acc[3]);
    }
    // exchange one 16-ring block at a time
#pragma unroll
    for (int hb = 0; hb < NRB; ++hb) {
      __syncthreads();   // the exchange region is free (coefficients, previous round)
#pragma unroll
      for (int cbk = 0; cbk < 2; ++cbk) {
        const int cc = cbk * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          stage[(Op::row(lane, v) * 32 + cc) * SM + wave] = (R)acc[2 * hb + cbk][v];
      }
      __syncthreads();
      store_f4_tile<R, MC, 16>(F4, stage, rbk * RW + hb * 16, cb0 * 16, J, ncols, nf, p, m0, Lp);
    }
  }
}

// Analysis: workgroup = one (m, p) and 64 degrees with all rings in LDS, NW
// waves; after the generation each wave runs its two degree blocks against
// every (NW / 2)-th pair of column blocks.
template <class Op, int PF, int NW>
__global__ __launch_bounds__(64 * NW) void k_leg_anal_rec_cols(
    const double* __restrict__ seeds, const double* __restrict__ rec, const double* __restrict__ mu,
    const void* __restrict__ G, typename Op::R* __restrict__ Y, const MPInfo* __restrict__ mpi,
    const WorkItem* __restrict__ items, int nitems, int kb2, int CBa, int CBn, int ncols, int Kx,
    int J, int Jp, int T) {
  typedef typename Op::R R;
  typedef typename Op::C C;
  constexpr int KS = 4 * 64 + 1;
  extern __shared__ unsigned char smem_raw[];
  R* As = reinterpret_cast<R*>(smem_raw);                                           // [Jp/4][KS]
  double* cf = reinterpret_cast<double*>(smem_raw + (size_t)(Jp / 4) * KS * sizeof(R));  // [64][3]
  int item, ct;
  if (!xcd_tile(nitems, 1, item, ct)) return;
  const WorkItem it = items[item];
  const MPInfo q = mpi[it.mp];
  if (it.tile * 4 >= q.rbA) return;                    // padding item (whole workgroup)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int deg0 = it.tile * 64, nch = rec_chunks(q.np), ebase = ext_off(T, q.m) + q.p;
  if (threadIdx.x < 64) {
    const int i = deg0 + threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    if (i >= 1 && i < q.np) {
      const double* rc = rec + (size_t)(ebase + 2 * (i - 1)) * 4;
      a = rc[0];
      b = rc[1];
      c = rc[2];
    }
    cf[3 * threadIdx.x] = a;
    cf[3 * threadIdx.x + 1] = b;
    cf[3 * threadIdx.x + 2] = c;
  }
  __syncthreads();
  for (int task = threadIdx.x; task < 2 * Jp; task += 64 * NW) {
    const int j = task % Jp, hh = task / Jp, ch = 2 * it.tile + hh;
    const double x = j < J ? mu[j] : 0.0;
    R* dst = As + (j >> 2) * KS + (j & 3) * 16;
    rec_chunk(seeds + ((size_t)(q.seed + ch) * Jp + j) * 2, ch < nch && j < J, x * x, cf,
              hh * kRecChunk, ch * kRecChunk, q.np, [&](int t, double v) {
                const int dl = hh * kRecChunk + t;
                dst[(dl >> 4) * 64 + (dl & 15)] = (R)v;
              });
  }
  __syncthreads();
  // wave w: degree blocks 2 ((w / 2) % 2) + {0, 1}; the NW / 2 waves of one
  // degree pair take column pairs 2 (w % 2) + 4 (w / 4) in steps of NW blocks
  const int rbl = ((wave >> 1) & 1) * 2, rb0 = it.tile * 4 + rbl;
  const int base = ext_off(T, q.m) + (q.p ? npar(T, q.m, 0) : 0);   // this parity's run
  for (int cb0 = (wave & 1) * 2 + (wave >> 2) * 4; cb0 < CBn; cb0 += NW) {
    const bool c1 = cb0 + 1 < CBn;
    C acc[4] = {};
    const long long tb = (long long)it.mp * kb2 * CBa + cb0;
    const R* a_lane = As + rbl * 64 + lane;
    if (c1)
      mma_loop_lds<Op, PF, 2, true>(a_lane, KS, G, tb, (long long)CBa, Jp / 4, lane, acc[0],
                                    acc[1], acc[2], acc[3]);
    else
      mma_loop_lds<Op, PF, 2, false>(a_lane, KS, G, tb, (long long)CBa, Jp / 4, lane, acc[0],
                                     acc[1], acc[2], acc[3]);
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
      const int rb = rb0 + (blk >> 1), cb = cb0 + (blk & 1);
      if ((blk & 1) && !c1) continue;
      const int c = cb * 16 + (lane & 15);
      if (c >= ncols) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = rb * 16 + Op::row(lane, v);
        if (i < q.np) Y[((size_t)(c >> 1) * Kx + base + i) * 2 + (c & 1)] = (R)acc[blk][v];
      }
    }
  }
}

static inline unsigned xcd_grid(int nitems, int nct) {
  return (unsigned)(((nitems + 7) / 8) * 8 * nct);
}

template <class Op, int MC, int PF, int HS = 32>
static hipError_t synth_impl(const pfsh_level* lv, int ncols, int nf, hipStream_t s) {
  const int CBn = (ncols + 15) / 16, nct = (CBn + 1) / 2, ntile = (lv->RB + 1) / 2;
  PFSH_LAUNCH(lv, (k_leg_synth<Op, MC, PF, HS>), dim3(xcd_grid(lv->nitemsS, ntile * nct)),
                     dim3(64 * MC), 0, s, lv->tabS, lv->X, (typename Op::R*)lv->F4, lv->mp_d,
                     lv->itemsS, lv->nitemsS, ntile, nct, lv->RB, lv->CBs, CBn, ncols, nf, lv->J,
                     lv->T, lv->Lp);
  return hipGetLastError();
}

template <class Op, int MC, int PF>
static hipError_t synth_t4_impl(const pfsh_level* lv, int ncols, int nf, hipStream_t s) {
  const int CBn = (ncols + 15) / 16, nct = (CBn + 3) / 4, ntile = (lv->RB + 3) / 4;
  PFSH_LAUNCH(lv, (k_leg_synth_t4<Op, MC, PF>), dim3(xcd_grid(lv->nitemsS, ntile * nct)),
                     dim3(64 * MC), 0, s, lv->tabS, lv->X, (typename Op::R*)lv->F4, lv->mp_d,
                     lv->itemsS, lv->nitemsS, ntile, nct, lv->RB, lv->CBs, CBn, ncols, nf, lv->J,
                     lv->T, lv->Lp);
  return hipGetLastError();
}

template <class Op, int PF>
static hipError_t anal_tall_impl(const pfsh_level* lv, int ncols, hipStream_t s) {
  const int CBn = (ncols + 15) / 16, nct = (CBn + 3) / 4;
  PFSH_LAUNCH(lv, (k_leg_anal_tall<Op, PF>), dim3(xcd_grid(lv->nitemsA, nct)), dim3(128), 0, s,
                     lv->tabA, lv->G, (typename Op::R*)lv->Y, lv->mp_d, lv->itemsA, lv->nitemsA,
                     nct, lv->kb2, lv->CBa, CBn, ncols, lv->Kx, lv->T);
  return hipGetLastError();
}

template <class Op, int PF, int SHAPE>
static hipError_t anal_impl(const pfsh_level* lv, int ncols, hipStream_t s) {
  const int CBn = (ncols + 15) / 16, nct = SHAPE == 0 ? (CBn + 3) / 4 : (CBn + 1) / 2;
  PFSH_LAUNCH(lv, (k_leg_anal<Op, PF, SHAPE>), dim3(xcd_grid(lv->nitemsA, nct)), dim3(256), 0, s,
                     lv->tabA, lv->G, (typename Op::R*)lv->Y, lv->mp_d, lv->itemsA, lv->nitemsA,
                     nct, lv->kb2, lv->kb2g, lv->CBa, CBn, ncols, lv->Kx, lv->T);
  return hipGetLastError();
}

// LDS of the generate-once recurrence kernels (0: does not fit, take the
// per-column-tile kernels)
static size_t synth_rec_cols_lds(const pfsh_level* lv, int nrb) {
  const size_t rsz = lv->op == OP_F64 ? 8 : 4;
  const int MC = lv->MC, kbmax = (npar(lv->T, 0, 0) + 3) / 4;
  const size_t aux = std::max((size_t)MC * (4 / nrb) * kRecChunk * 3 * 8,
                              (size_t)16 * 32 * (MC + 1) * rsz);
  const size_t b = (size_t)MC * kbmax * nrb * 64 * rsz + aux;
  return b <= 160 * 1024 ? b : 0;
}
static size_t anal_rec_cols_lds(const pfsh_level* lv) {
  const size_t rsz = lv->op == OP_F64 ? 8 : 4;
  const size_t b = (size_t)(lv->Jp / 4) * (4 * 64 + 1) * rsz + 64 * 3 * 8;
  return b <= 160 * 1024 ? b : 0;
}

template <class Op, int NRB>
static hipError_t synth_rec_cols_impl(const pfsh_level* lv, int ncols, int nf, size_t shm,
                                      hipStream_t s) {
  typedef typename Op::R R;
  constexpr int MC = Op::KIND == OP_F64 ? 4 : 8;
  const int CBn = (ncols + 15) / 16, nrb = lv->Jp / (16 * NRB);
  const int kbmax = (npar(lv->T, 0, 0) + 3) / 4;
  (void)hipFuncSetAttribute((const void*)k_leg_synth_rec_cols<Op, MC, 4, NRB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  PFSH_LAUNCH(lv, (k_leg_synth_rec_cols<Op, MC, 4, NRB>), dim3(xcd_grid(lv->nitemsS, nrb)),
                     dim3(64 * MC), shm, s, lv->seeds_d, lv->rec_d, lv->mu_d, lv->X, (R*)lv->F4,
                     lv->mp_d, lv->itemsS, lv->nitemsS, nrb, kbmax, lv->CBs, CBn, ncols, nf,
                     lv->J, lv->Jp, lv->T, lv->Lp);
  return hipGetLastError();
}

template <class Op, int NW>
static hipError_t anal_rec_cols_impl(const pfsh_level* lv, int ncols, size_t shm, hipStream_t s) {
  typedef typename Op::R R;
  const int CBn = (ncols + 15) / 16;
  (void)hipFuncSetAttribute((const void*)k_leg_anal_rec_cols<Op, 4, NW>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  PFSH_LAUNCH(lv, (k_leg_anal_rec_cols<Op, 4, NW>), dim3(xcd_grid(lv->nitemsA, 1)), dim3(64 * NW), shm,
                     s, lv->seeds_d, lv->rec_d, lv->mu_d, lv->G, (R*)lv->Y, lv->mp_d, lv->itemsA,
                     lv->nitemsA, lv->kb2, lv->CBa, CBn, ncols, lv->Kx, lv->J, lv->Jp, lv->T);
  return hipGetLastError();
}

template <class Op>
static hipError_t synth_rec_impl(const pfsh_level* lv, int ncols, int nf, hipStream_t s) {
  typedef typename Op::R R;
  constexpr int MC = Op::KIND == OP_F64 ? 4 : 8;
  const int CBn = (ncols + 15) / 16, nct = (CBn + 1) / 2, ntile = (lv->RB + 1) / 2;
  const size_t shm = (size_t)MC * (2 * kRecChunk / 4) * 128 * sizeof(R) +
                     (size_t)MC * 2 * kRecChunk * 3 * sizeof(double);
  (void)hipFuncSetAttribute((const void*)k_leg_synth_rec<Op, MC>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  PFSH_LAUNCH(lv, (k_leg_synth_rec<Op, MC>), dim3(xcd_grid(lv->nitemsS, ntile * nct)),
                     dim3(64 * MC), shm, s, lv->seeds_d, lv->rec_d, lv->mu_d, lv->X,
                     (R*)lv->F4, lv->mp_d, lv->itemsS, lv->nitemsS, ntile, nct, lv->CBs, CBn,
                     ncols, nf, lv->J, lv->Jp, lv->T, lv->Lp);
  return hipGetLastError();
}

template <class Op>
static hipError_t anal_rec_impl(const pfsh_level* lv, int ncols, hipStream_t s) {
  typedef typename Op::R R;
  const int CBn = (ncols + 15) / 16, nct = (CBn + 3) / 4;
  constexpr int SR = 65536 / (64 * (int)sizeof(R));
  const size_t shm = (size_t)(SR / 4) * (4 * 64 + 1) * sizeof(R) + (size_t)64 * 3 * sizeof(double);
  (void)hipFuncSetAttribute((const void*)k_leg_anal_rec<Op, 4>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  PFSH_LAUNCH(lv, (k_leg_anal_rec<Op, 4>), dim3(xcd_grid(lv->nitemsA, nct)), dim3(256), shm, s,
                     lv->seeds_d, lv->rec_d, lv->mu_d, lv->G, (R*)lv->Y, lv->mp_d, lv->itemsA,
                     lv->nitemsA, nct, lv->kb2, lv->CBa, CBn, ncols, lv->Kx, lv->J, lv->Jp, lv->T);
  return hipGetLastError();
}

// Variant lists (index 0 = default):
//   synthesis, prefetch depth of the K loop (t4: 4x4-block wave tiles):
//     FP64 / FP32 4 2 8 t4-4 t4-2 4h (4h: LDS exchange in two row halves);
//     BF16x3 2 4
//   analysis, (prefetch depth, tile shape): FP64 / FP32 (2,0) (1,0) (4,0) (2,1)
//     (4,1) (1,tall) (2,tall), depth in 16-byte k-groups; BF16x3 (2,0) (4,0)
//     (2,1) (4,1), depth in k-blocks of 32
// None changes the order of any sum, so all variants give the same bits.
int leg_variant_count(int op, int stage) {
  if (stage == TS_SYNTH) return op == OP_BF16X3 ? 2 : 6;
  return op == OP_BF16X3 ? 4 : 7;
}

hipError_t launch_leg_synth(const pfsh_level* lv, int ncols, int nf, hipStream_t s) {
  if (lv->rec_mode) {
    // variant 0: generate-once kernel, 32 rings per workgroup where they fit,
    // else 16; 1: per-column-tile slabs; 2: generate-once with 16 rings
    const int v = lv->variant[TS_SYNTH][tune_bucket((ncols + 15) / 16)];
    const size_t shm2 = synth_rec_cols_lds(lv, 2), shm1 = synth_rec_cols_lds(lv, 1);
    if (v == 0 && shm2)
      return lv->op == OP_F64 ? synth_rec_cols_impl<OpF64, 2>(lv, ncols, nf, shm2, s)
                              : synth_rec_cols_impl<OpF32, 2>(lv, ncols, nf, shm2, s);
    if (v != 1 && shm1)
      return lv->op == OP_F64 ? synth_rec_cols_impl<OpF64, 1>(lv, ncols, nf, shm1, s)
                              : synth_rec_cols_impl<OpF32, 1>(lv, ncols, nf, shm1, s);
    return lv->op == OP_F64 ? synth_rec_impl<OpF64>(lv, ncols, nf, s)
                            : synth_rec_impl<OpF32>(lv, ncols, nf, s);
  }
  const int v = lv->variant[TS_SYNTH][tune_bucket((ncols + 15) / 16)];
  switch (lv->op) {
    case OP_F64:
      return v == 1 ? synth_impl<OpF64, 4, 2>(lv, ncols, nf, s)
           : v == 2 ? synth_impl<OpF64, 4, 8>(lv, ncols, nf, s)
           : v == 3 ? synth_t4_impl<OpF64, 4, 4>(lv, ncols, nf, s)
           : v == 4 ? synth_t4_impl<OpF64, 4, 2>(lv, ncols, nf, s)
           : v == 5 ? synth_impl<OpF64, 4, 4, 16>(lv, ncols, nf, s)
                    : synth_impl<OpF64, 4, 4>(lv, ncols, nf, s);
    case OP_F32:
      return v == 1 ? synth_impl<OpF32, 8, 2>(lv, ncols, nf, s)
           : v == 2 ? synth_impl<OpF32, 8, 8>(lv, ncols, nf, s)
           : v == 3 ? synth_t4_impl<OpF32, 8, 4>(lv, ncols, nf, s)
           : v == 4 ? synth_t4_impl<OpF32, 8, 2>(lv, ncols, nf, s)
           : v == 5 ? synth_impl<OpF32, 8, 4, 16>(lv, ncols, nf, s)
                    : synth_impl<OpF32, 8, 4>(lv, ncols, nf, s);
    default:
      return v == 1 ? synth_impl<OpBF3, 8, 4>(lv, ncols, nf, s)
                    : synth_impl<OpBF3, 8, 2>(lv, ncols, nf, s);
  }
}

template <class Op>
static hipError_t anal_variant(const pfsh_level* lv, int v, int ncols, hipStream_t s) {
  if constexpr (Op::KIND == OP_BF16X3) {
    switch (v) {
      case 1: return anal_impl<Op, 4, 0>(lv, ncols, s);
      case 2: return anal_impl<Op, 2, 1>(lv, ncols, s);
      case 3: return anal_impl<Op, 4, 1>(lv, ncols, s);
      default: return anal_impl<Op, 2, 0>(lv, ncols, s);
    }
  } else {
    switch (v) {
      case 1: return anal_impl<Op, 1, 0>(lv, ncols, s);
      case 2: return anal_impl<Op, 4, 0>(lv, ncols, s);
      case 3: return anal_impl<Op, 2, 1>(lv, ncols, s);
      case 4: return anal_impl<Op, 4, 1>(lv, ncols, s);
      case 5: return anal_tall_impl<Op, 1>(lv, ncols, s);
      case 6: return anal_tall_impl<Op, 2>(lv, ncols, s);
      default: return anal_impl<Op, 2, 0>(lv, ncols, s);
    }
  }
}

hipError_t launch_leg_anal(const pfsh_level* lv, int ncols, int /*nf*/, hipStream_t s) {
  if (lv->rec_mode) {
    const size_t shm = anal_rec_cols_lds(lv);
    const int v = lv->variant[TS_ANAL][tune_bucket((ncols + 15) / 16)];
    if (shm && v != 1)
      return lv->op == OP_F64 ? (v == 0 ? anal_rec_cols_impl<OpF64, 8>(lv, ncols, shm, s)
                                        : anal_rec_cols_impl<OpF64, 4>(lv, ncols, shm, s))
                              : (v == 0 ? anal_rec_cols_impl<OpF32, 8>(lv, ncols, shm, s)
                                        : anal_rec_cols_impl<OpF32, 4>(lv, ncols, shm, s));
    return lv->op == OP_F64 ? anal_rec_impl<OpF64>(lv, ncols, s) : anal_rec_impl<OpF32>(lv, ncols, s);
  }
  const int v = lv->variant[TS_ANAL][tune_bucket((ncols + 15) / 16)];
  switch (lv->op) {
    case OP_F64: return anal_variant<OpF64>(lv, v, ncols, s);
    case OP_F32: return anal_variant<OpF32>(lv, v, ncols, s);
    default: return anal_variant<OpBF3>(lv, v, ncols, s);
  }
}

}  // namespace pfsh
