// Mode-k products on the in-place unfolding X_(k)[i, p*S + s] = X[p, i, s].
//
// Two contractions cover the method's three products (and a fused kernel
// runs both products of an FP32 power step in one pass, further below):
//  * column reduction  part = X_(k) B   (sketch Y = X_(k) Omega_k and the
//    second half of the power step Y = X_(k) Z): a long reduction over the
//    m_k columns, split over workgroups, summed in a fixed order later;
//  * row contraction   out = X_(k)^T W  (Z = X_(k)^T Q of the power step and
//    the core step X x_k U^T): a short reduction over the n_k rows per
//    column tile, written in the [P, lw, S] layout of the result tensor.
//
// Operands go from HBM straight into matrix-core registers with 16-byte
// loads; there is no LDS staging and no barrier in the main loops:
//  * when the reduction index is the contiguous one (column reduction with
//    S > 1, row contraction with S == 1) a lane loads KC consecutive
//    reduction elements and feeds them to consecutive MFMA k-steps; A and B
//    use the same k order, so the sum is unchanged;
//  * when the output row index is the contiguous one (column reduction with
//    S == 1, row contraction with S > 1) the MV elements of a 16-byte vector
//    go to MV interleaved 16-row tiles.
// Instructions: v_mfma_f32_16x16x4_f32 (FP32), v_mfma_f64_16x16x4_f64 (FP64),
// v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32 accumulation).
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace tk {

template <int MK>
struct Pol;
template <>
struct Pol<MF_F32> {
  using T = float;
  using acc_t = floatx4;
  using part_t = float;
  static constexpr int KL = 1;  // reduction elements per lane per MFMA
  static constexpr int KC = 4;  // consecutive reduction elements per 16-byte load
  static constexpr int MV = 4;  // consecutive output rows per 16-byte load
};
template <>
struct Pol<MF_F64> {
  using T = double;
  using acc_t = doublex4;
  using part_t = double;
  static constexpr int KL = 1;
  static constexpr int KC = 2;
  static constexpr int MV = 2;
};
template <>
struct Pol<MF_BF16> {
  using T = float;
  using acc_t = floatx4;
  using part_t = float;
  static constexpr int KL = 8;
  static constexpr int KC = 8;
  static constexpr int MV = 4;
};

// Row of the 16x16 result held by (lane, element v): the FP32 and BF16
// instructions return 4 consecutive rows per lane group, the FP64 one
// interleaves them with a stride of 4.
template <int MK>
__device__ __forceinline__ int mfma_drow(int lane, int v) {
  if constexpr (MK == MF_F64) {
    return (lane >> 4) + 4 * v;
  } else {
    return 4 * (lane >> 4) + v;
  }
}

template <int MK>
__device__ __forceinline__ typename Pol<MK>::acc_t mma(const typename Pol<MK>::T* a, const typename Pol<MK>::T* b,
                                                      typename Pol<MK>::acc_t c) {
  if constexpr (MK == MF_F32) {
    return mfma_f32(a[0], b[0], c);
  } else if constexpr (MK == MF_F64) {
    return mfma_f64(a[0], b[0], c);
  } else {
    const bf16x8 av = {(__bf16)a[0], (__bf16)a[1], (__bf16)a[2], (__bf16)a[3],
                       (__bf16)a[4], (__bf16)a[5], (__bf16)a[6], (__bf16)a[7]};
    const bf16x8 bv = {(__bf16)b[0], (__bf16)b[1], (__bf16)b[2], (__bf16)b[3],
                       (__bf16)b[4], (__bf16)b[5], (__bf16)b[6], (__bf16)b[7]};
    return mfma_bf16(av, bv, c);
  }
}

// Wave index within the workgroup, known to the compiler as wave-uniform (a
// scalar register), so that loop bounds and tile choices derived from it
// become scalar branches rather than exec-mask loops.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// 16 raw bytes with only 4-byte alignment: global loads and stores of this
// type are single dwordx4 accesses at any element address, so rows of any
// length (odd unfolding widths, sub-tensors at odd offsets) take the wide path.
typedef float f4u_t __attribute__((ext_vector_type(4), aligned(4)));

// N consecutive elements at p; `cnt` of them exist (<= 0: none). A whole
// group is read with 16-byte loads; a short group with guarded element loads.
template <typename T, int N>
__device__ __forceinline__ void load_n(const T* __restrict__ p, int cnt, T* out) {
  static_assert((sizeof(T) * N) % 16 == 0, "vector width");
  if (cnt >= N) {
#pragma unroll
    for (int q = 0; q < (int)(sizeof(T) * N / 16); ++q) {
      const f4u_t v = *reinterpret_cast<const f4u_t*>(reinterpret_cast<const char*>(p) + 16 * q);
      *reinterpret_cast<f4u_t*>(reinterpret_cast<char*>(out) + 16 * q) = v;
    }
  } else {
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = (e < cnt) ? p[e] : T(0);
  }
}

// The 16 bytes of VE elements at p as raw float4, `cnt` of them present.
template <typename T, int VE>
__device__ __forceinline__ float4 load16(const T* __restrict__ p, int cnt) {
  T v[VE];
  load_n<T, VE>(p, cnt, v);
  return *reinterpret_cast<const float4*>(v);
}

// Workgroup -> (split, row block) so that the workgroups of one split, which
// read the same slice of the skinny operand, run on the same XCD (workgroups
// are dealt to the 8 XCDs round robin).
__device__ __forceinline__ bool xcd_decode(int bid, int nsplit, int nblocks, int* split, int* rblock) {
  const int x = bid & 7, li = bid >> 3;
  *rblock = li % nblocks;
  *split = (li / nblocks) * 8 + x;
  return *split < nsplit;
}

// Copy of a KB-element fragment.
template <typename T, int KB>
__device__ __forceinline__ void copy_frag(T* dst, const T* src) {
#pragma unroll
  for (int e = 0; e < KB; ++e) dst[e] = src[e];
}

// ---------------------------------------------------------------------------
// Column reduction, S > 1, staged through LDS: part[split][i][j] = sum over
// the split's columns c of X_(k)[i, c] Bt[j, c]. A workgroup owns 64 rows
// (16 per wave) and one split; a stage is KT consecutive columns of one p
// (256 bytes of every row). The stage's X and Bt tiles are read from HBM
// with whole-row 16-byte vector loads (a wave covers 4 rows x 256 B per
// instruction), kept two stages ahead in registers, written to a double
// buffered LDS tile (BF16: converted once here) and read back by the matrix
// cores as 16-byte fragments. LDS rows are padded by 16 bytes so the 16
// lanes of each fragment read hit distinct banks. One barrier per stage.
// ---------------------------------------------------------------------------
template <int MK>
struct LdsPol;
template <>
struct LdsPol<MF_F32> {
  using LT = float;
  static constexpr int KT = 64, RV = 4;  // stage width (elements), elements per 16-byte fragment
};
template <>
struct LdsPol<MF_F64> {
  using LT = double;
  static constexpr int KT = 32, RV = 2;
};
template <>
struct LdsPol<MF_BF16> {
  using LT = __bf16;
  static constexpr int KT = 64, RV = 8;
};

// EDGE: 0 when KT divides S (no edge stage), 1 when the 16-byte group
// divides S (an edge-stage group is whole or absent), 2 otherwise.
template <int MK, int NJ, int EDGE>
__device__ __forceinline__ void cr_lds_body(const typename Pol<MK>::T* __restrict__ X,
                                                const typename Pol<MK>::T* __restrict__ Bt, int64_t n, int64_t S,
                                                int l, int64_t m, int64_t spp, int64_t nsteps, int nsplit,
                                                typename Pol<MK>::part_t* __restrict__ part, int split, int rb,
                                                double* __restrict__ nslot = nullptr) {
  using Po = Pol<MK>;
  using T = typename Po::T;
  using LT = typename LdsPol<MK>::LT;
  constexpr int KT = LdsPol<MK>::KT, RV = LdsPol<MK>::RV, KL = Po::KL;
  constexpr int VE = 16 / (int)sizeof(T);          // elements of T per 16-byte global load
  constexpr int UPR = KT / VE;                     // 16-byte units per row per stage (16)
  constexpr int LS = KT + 16 / (int)sizeof(LT);    // padded LDS row (elements)
  constexpr int XU = 64 * UPR / 256, BU = 16 * NJ * UPR / 256;  // units per thread: X tile, Bt tile
  __shared__ __align__(16) LT xs[2][64][LS];
  __shared__ __align__(16) LT bs[2][16 * NJ][LS];

  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  const int mm = lane & 15, g = lane >> 4;
  const int64_t r0 = (int64_t)rb * 64;
  const int64_t t0 = nsteps * split / nsplit, t1 = nsteps * (split + 1) / nsplit;

  using V4 = float4;  // 16 raw bytes
  // Stage loads. A stage whose KT columns all lie inside the row (every stage
  // but the last of each p when KT does not divide S), and the edge stage when
  // a 16-byte group divides S (EDGE 1), are read with unconditional loads:
  // rows past n and Bt rows past l are clamped (they feed only outputs that
  // are never written), a stage past the split re-reads its last stage (it is
  // never computed), and EDGE 1 groups at or past S are clamped to the row's
  // last group and zeroed in X. Without a branch around a load the compiler
  // keeps the prefetched stage in flight across the compute. EDGE 2 edge
  // stages count their elements.
  // Stage cursor (p, s0 of the next stage to load): one division per split,
  // then advanced by scalar selects; it stays on the split's last stage.
  int64_t cp = t0 / spp, cs = (t0 - (t0 / spp) * spp) * KT, cleft = t1 - t0;
  const int64_t rowlen = spp * KT;
  auto gload = [&](int64_t t, V4 (&xr)[XU], V4 (&br)[BU]) {
    const int64_t p = cp, s0 = cs;
    {
      const bool adv = cleft > 1;
      const int64_t ns = cs + KT;
      const bool wrap = ns == rowlen;
      cs = adv ? (wrap ? 0 : ns) : cs;
      cp = adv && wrap ? cp + 1 : cp;
      cleft = adv ? cleft - 1 : cleft;
    }
    if (EDGE != 2 || s0 + KT <= S) {
#pragma unroll
      for (int q = 0; q < XU; ++q) {
        const int L = q * 256 + tid, row = L / UPR, u = L % UPR;
        const int64_t i = min<int64_t>(r0 + row, n - 1);
        const int64_t sg = s0 + (int64_t)u * VE;
        const bool in = EDGE == 0 || sg < S;
        f4u_t v = *reinterpret_cast<const f4u_t*>(X + (p * n + i) * S + (in ? sg : S - VE));
        if (EDGE != 0) v = in ? v : f4u_t{0.f, 0.f, 0.f, 0.f};
        xr[q] = V4{v[0], v[1], v[2], v[3]};
      }
#pragma unroll
      for (int q = 0; q < BU; ++q) {
        const int L = q * 256 + tid, j = min(L / UPR, l - 1), u = L % UPR;
        const int64_t sg = s0 + (int64_t)u * VE;
        const f4u_t v = *reinterpret_cast<const f4u_t*>(Bt + (int64_t)j * m + p * S + (EDGE == 0 || sg < S ? sg : S - VE));
        br[q] = V4{v[0], v[1], v[2], v[3]};
      }
      return;
    }
    const bool live = t < t1;
#pragma unroll
    for (int q = 0; q < XU; ++q) {
      const int L = q * 256 + tid, row = L / UPR, u = L % UPR;
      const int64_t i = r0 + row, s = s0 + (int64_t)u * VE;
      const int cnt = (live && i < n) ? (int)max<int64_t>(0, min<int64_t>(VE, S - s)) : 0;
      xr[q] = load16<T, VE>(X + (p * n + i) * S + s, cnt);
    }
#pragma unroll
    for (int q = 0; q < BU; ++q) {
      const int L = q * 256 + tid, j = L / UPR, u = L % UPR;
      const int64_t s = s0 + (int64_t)u * VE;
      const int cnt = (live && j < l) ? (int)max<int64_t>(0, min<int64_t>(VE, S - s)) : 0;
      br[q] = load16<T, VE>(Bt + (int64_t)j * m + p * S + s, cnt);
    }
  };
  auto sput = [&](LT* dst, const V4& v) {
    if constexpr (MK == MF_BF16) {
      const float* f = reinterpret_cast<const float*>(&v);
      typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
      const bf16x4 b = {(__bf16)f[0], (__bf16)f[1], (__bf16)f[2], (__bf16)f[3]};
      *reinterpret_cast<bf16x4*>(dst) = b;
    } else {
      *reinterpret_cast<V4*>(dst) = v;
    }
  };
  auto lstore = [&](int buf, const V4 (&xr)[XU], const V4 (&br)[BU]) {
#pragma unroll
    for (int q = 0; q < XU; ++q) {
      const int L = q * 256 + tid, row = L / UPR, u = L % UPR;
      sput(&xs[buf][row][u * VE], xr[q]);
    }
#pragma unroll
    for (int q = 0; q < BU; ++q) {
      const int L = q * 256 + tid, j = L / UPR, u = L % UPR;
      sput(&bs[buf][j][u * VE], br[q]);
    }
  };

  // With nslot != nullptr the workgroup also sums the squares of the X
  // elements it stages (FP64, in stage order; rows past n and stages past the
  // split excluded), for ||X||_F^2 at no extra pass over X. Every element of
  // X is staged by exactly one workgroup once.
  double nacc = 0.0;
  auto nsum = [&](const V4 (&xr)[XU], bool live) {
    if (nslot == nullptr || !live) return;
#pragma unroll
    for (int q = 0; q < XU; ++q) {
      const int L = q * 256 + tid, row = L / UPR;
      if (r0 + row < n) {
        if constexpr (sizeof(T) == 8) {
          typedef double d2_t __attribute__((ext_vector_type(2)));
          const d2_t d = __builtin_bit_cast(d2_t, xr[q]);
          nacc = fma(d[0], d[0], nacc);
          nacc = fma(d[1], d[1], nacc);
        } else {
          const float e[4] = {xr[q].x, xr[q].y, xr[q].z, xr[q].w};
#pragma unroll
          for (int c = 0; c < 4; ++c) nacc = fma((double)e[c], (double)e[c], nacc);
        }
      }
    }
  };

  typename Po::acc_t acc[NJ];
#pragma unroll
  for (int u = 0; u < NJ; ++u) acc[u] = typename Po::acc_t{0, 0, 0, 0};
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4 * RV) {
      LT a[RV];
      *reinterpret_cast<V4*>(a) = *reinterpret_cast<const V4*>(&xs[buf][16 * wave + mm][kk + RV * g]);
      LT b[NJ][RV];
#pragma unroll
      for (int u = 0; u < NJ; ++u)
        *reinterpret_cast<V4*>(b[u]) = *reinterpret_cast<const V4*>(&bs[buf][16 * u + mm][kk + RV * g]);
      if constexpr (MK == MF_BF16) {
#pragma unroll
        for (int u = 0; u < NJ; ++u)
          acc[u] = mfma_bf16(*reinterpret_cast<const bf16x8*>(a), *reinterpret_cast<const bf16x8*>(b[u]), acc[u]);
      } else {
#pragma unroll
        for (int e = 0; e < RV; e += KL)
#pragma unroll
          for (int u = 0; u < NJ; ++u) acc[u] = mma<MK>(&a[e], &b[u][e], acc[u]);
      }
    }
  };

  V4 xa[XU], ba[BU], xb[XU], bb[BU];
  if (t0 < t1) {  // a split always holds a stage; the guard keeps every address in range
    gload(t0, xa, ba);
    gload(t0 + 1, xb, bb);
    lstore(0, xa, ba);
    nsum(xa, true);
    lds_barrier();
    // pairs of stages with no exit inside the body (an exit would let the
    // compiler sink the stage t + 2 loads below it, after the t + 3 loads)
    int64_t t = t0;
    for (; t + 1 < t1; t += 2) {
      // stage t in buffer 0, stage t + 1 in registers xb/bb
      gload(t + 2, xa, ba);
      __builtin_amdgcn_sched_barrier(0);
      compute(0);
      lstore(1, xb, bb);
      nsum(xb, true);
      lds_barrier();
      gload(t + 3, xb, bb);
      __builtin_amdgcn_sched_barrier(0);
      compute(1);
      lstore(0, xa, ba);
      nsum(xa, t + 2 < t1);
      lds_barrier();
    }
    if (t < t1) compute(0);  // odd stage count: the last stage is in buffer 0
  }
  if (nslot != nullptr) {
    // fixed order: a butterfly over the lanes (every lane ends with the same
    // sum), then the four waves in index order
    __shared__ double nred[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nacc += __shfl_xor(nacc, o, 64);
    if (lane == 0) nred[wave] = nacc;
    __syncthreads();
    if (tid == 0) *nslot = (nred[0] + nred[1]) + (nred[2] + nred[3]);
  }
#pragma unroll
  for (int u = 0; u < NJ; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 16 * wave + mfma_drow<MK>(lane, v);
      const int col = 16 * u + mm;
      if (row < n && col < l) part[((int64_t)split * n + row) * l + col] = acc[u][v];
    }
}

template <int MK, int NJ, int EDGE>
__global__ __launch_bounds__(256) void k_cr_lds(const typename Pol<MK>::T* __restrict__ X,
                                                const typename Pol<MK>::T* __restrict__ Bt, int64_t n, int64_t S,
                                                int l, int64_t m, int64_t spp, int64_t nsteps, int nsplit,
                                                int nrblocks, typename Pol<MK>::part_t* __restrict__ part,
                                                double* __restrict__ npart) {
  int split, rb;
  if (!xcd_decode((int)blockIdx.x, nsplit, nrblocks, &split, &rb)) return;
  cr_lds_body<MK, NJ, EDGE>(X, Bt, n, S, l, m, spp, nsteps, nsplit, part, split, rb,
                            npart != nullptr ? npart + (int64_t)split * nrblocks + rb : nullptr);
}

// ---------------------------------------------------------------------------
// Column reduction, S > 1, FP32 storage on the BF16 matrix cores: NP = 3
// forms FP32 products through the three-piece split, NP = 1 rounds both
// operands to BF16 once. part[split][i][j] as for k_cr_lds. A workgroup owns
// 128 rows (32 per wave, two 16-row tiles) and one split; a stage is 32
// columns of one p. X goes from HBM straight into each wave's registers in
// the operand layout of v_mfma_f32_16x16x32_bf16: lane (mm, g) of tile h
// holds row 32 w + 16 h + mm at stage columns 4 g .. 4 g + 3 (k slots 8 g ..
// 8 g + 3) and 16 + 4 g .. 16 + 4 g + 3 (k slots 8 g + 4 .. 8 g + 7), so a
// row's 128 bytes are two 64-byte runs, each read by one instruction, and X
// never passes through LDS. The stage's Bt tile (FP32) is read by the whole
// workgroup, converted once into BF16 pieces in the same k order and kept in
// LDS (rows padded by 16 bytes), where every wave reads it for its two tiles.
// X and Bt are kept two stages ahead in registers; one barrier per stage.
// With NORM (npart given), the workgroup also sums the squares of the X elements it
// reads (FP64, stage order, rows past n and stages past the split excluded)
// into the slots of its two 64-row halves (slot split * nslots + 64-row
// block), the layout colreduce_norm_slots describes.
// EDGE as for k_cr_lds (0: 32 divides S; 1: 4 divides S; 2: otherwise).
// ---------------------------------------------------------------------------
// FP32 products on the BF16 matrix cores. An FP32 value splits into three
// BF16 pieces, x = x0 + x1 + x2 + e with |e| <= 2^-24 |x| (each piece the
// round-to-nearest BF16 of what the previous ones leave; each product of two
// pieces is exact in FP32). A product a b is taken as the six partial
// products whose pieces' orders sum to at most 2 (a0 b0, a0 b1, a1 b0, a0 b2,
// a1 b1, a2 b0); the three left out are below 3 2^-24 |a b| together. The
// sums run in the FP32 accumulators of v_mfma_f32_16x16x32_bf16, whose BF16
// rate on gfx950 is about 15 times its FP32 one, so six of them cost less
// than half of one FP32 16x16x4 step of the same work. With one piece (NP =
// 1) the same kernels take BF16 operands.
// Pieces of pairs of FP32 values: fptrunc and fpext of two-element vectors
// become one v_cvt_pk_bf16_f32 per pair and one shift or mask per element.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));

template <int NP>
__device__ __forceinline__ void pair_pieces(f32x2_t v, bf16x2_t (&p)[NP]) {
  const bf16x2_t a = __builtin_convertvector(v, bf16x2_t);
  p[0] = a;
  if constexpr (NP == 3) {
    const f32x2_t r1 = v - __builtin_convertvector(a, f32x2_t);
    const bf16x2_t b = __builtin_convertvector(r1, bf16x2_t);
    p[1] = b;
    p[2] = __builtin_convertvector(r1 - __builtin_convertvector(b, f32x2_t), bf16x2_t);
  }
}

template <int NP>
__device__ __forceinline__ void bf_pieces(const float (&x)[8], bf16x8 (&p)[NP]) {
  bf16x2_t q[4][NP];
#pragma unroll
  for (int e = 0; e < 4; ++e) pair_pieces<NP>(f32x2_t{x[2 * e], x[2 * e + 1]}, q[e]);
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    const bf16x4_t lo = __builtin_shufflevector(q[0][c], q[1][c], 0, 1, 2, 3);
    const bf16x4_t hi = __builtin_shufflevector(q[2][c], q[3][c], 0, 1, 2, 3);
    p[c] = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
  }
}

template <int NP>
__device__ __forceinline__ void bf_pieces4(const float (&x)[4], bf16x4_t (&p)[NP]) {
  bf16x2_t q[2][NP];
#pragma unroll
  for (int e = 0; e < 2; ++e) pair_pieces<NP>(f32x2_t{x[2 * e], x[2 * e + 1]}, q[e]);
#pragma unroll
  for (int c = 0; c < NP; ++c) p[c] = __builtin_shufflevector(q[0][c], q[1][c], 0, 1, 2, 3);
}

// The products of a pair of pieced operands, smallest first: (piece of A,
// piece of B) with orders summing to at most 2 for the split, (0, 0) for BF16.
template <int NP>
struct BfProducts;
template <>
struct BfProducts<1> {
  static constexpr int N = 1;
  static constexpr int A[1] = {0}, B[1] = {0};
};
template <>
struct BfProducts<3> {
  static constexpr int N = 6;
  static constexpr int A[6] = {2, 1, 0, 1, 0, 0}, B[6] = {0, 1, 2, 0, 1, 0};
};

// The body takes one (split, 128-row block) item; the kernel below maps its
// workgroups onto items XCD by XCD, the batched launch through its item table.
template <int NP, int NJ, int EDGE, bool NORM>
__device__ __forceinline__ void cr_split_body(const float* __restrict__ X, const float* __restrict__ Bt, int64_t n,
                                              int64_t S, int l, int64_t m, int64_t spp, int64_t nsteps, int nsplit,
                                              int nslots, float* __restrict__ part, double* __restrict__ npart,
                                              int split, int rb) {
  constexpr int KT = 32;
  constexpr int NJB = (NJ + 1) & ~1;       // Bt rows staged per stage: whole 32-row units
  constexpr int BU = NJB / 2;              // 16-byte Bt units per thread per stage
  constexpr int LS = KT + 8;               // padded LDS row (BF16 elements)
  using PR = BfProducts<NP>;
  __shared__ __align__(16) __bf16 bs[2][NP][16 * NJB][LS];
  __shared__ double nred[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  const int mm = lane & 15, g = lane >> 4;
  const int64_t r0 = (int64_t)rb * 128 + 32 * wave;
  const int64_t t0 = nsteps * split / nsplit, t1 = nsteps * (split + 1) / nsplit;
  // the lane's rows in the two tiles, clamped (rows past n feed only outputs
  // that are never written)
  const int64_t ia = min<int64_t>(r0 + mm, n - 1), ib = min<int64_t>(r0 + 16 + mm, n - 1);
  const bool rowa = r0 + mm < n, rowb = r0 + 16 + mm < n;
  typedef float fv4 __attribute__((ext_vector_type(4)));

  // stage cursors as in k_cr_lds, one for X and one for Bt (their loads run
  // at different distances): (p, s0) of the next stage to load; a cursor
  // stays on the split's last stage, so loads past the split re-read that stage
  struct Cursor {
    int64_t p, s, left;
  };
  const int64_t rowlen = spp * KT;
  Cursor xc{t0 / spp, (t0 - (t0 / spp) * spp) * KT, t1 - t0}, bc = xc;
  auto advance = [&](Cursor& c, int64_t& p, int64_t& s0) {
    p = c.p;
    s0 = c.s;
    const bool adv = c.left > 1;
    const int64_t ns = c.s + KT;
    const bool wrap = ns == rowlen;
    c.s = adv ? (wrap ? 0 : ns) : c.s;
    c.p = adv && wrap ? c.p + 1 : c.p;
    c.left = adv ? c.left - 1 : c.left;
  };
  // X of stage t: [tile a cols 4g.., tile a cols 16+4g.., tile b .., tile b ..]
  auto xload = [&](int64_t t, fv4 (&xr)[4]) {
    int64_t p, s0;
    advance(xc, p, s0);
    const float* xa = X + (p * n + ia) * S;
    const float* xb = X + (p * n + ib) * S;
    const int64_t c0 = s0 + 4 * g, c1 = s0 + 16 + 4 * g;
    if (EDGE != 2 || s0 + KT <= S) {
      const bool in0 = EDGE == 0 || c0 < S, in1 = EDGE == 0 || c1 < S;
      const int64_t a0 = in0 ? c0 : S - 4, a1 = in1 ? c1 : S - 4;
      f4u_t v[4] = {*reinterpret_cast<const f4u_t*>(xa + a0), *reinterpret_cast<const f4u_t*>(xa + a1),
                    *reinterpret_cast<const f4u_t*>(xb + a0), *reinterpret_cast<const f4u_t*>(xb + a1)};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool in = (q & 1) ? in1 : in0;
        xr[q] = (EDGE == 0 || in) ? fv4{v[q][0], v[q][1], v[q][2], v[q][3]} : fv4{0.f, 0.f, 0.f, 0.f};
      }
      return;
    }
    // EDGE 2 edge stage: element loads, counted
    const bool live = t < t1;
    const int n0 = live ? (int)max<int64_t>(0, min<int64_t>(4, S - c0)) : 0;
    const int n1 = live ? (int)max<int64_t>(0, min<int64_t>(4, S - c1)) : 0;
    float v[4][4];
    load_n<float, 4>(xa + c0, n0, v[0]);
    load_n<float, 4>(xa + c1, n1, v[1]);
    load_n<float, 4>(xb + c0, n0, v[2]);
    load_n<float, 4>(xb + c1, n1, v[3]);
#pragma unroll
    for (int q = 0; q < 4; ++q) xr[q] = fv4{v[q][0], v[q][1], v[q][2], v[q][3]};
  };
  // Bt tile of stage t: unit q * 256 + tid is row j, columns 4 u .. 4 u + 3
  auto bload = [&](int64_t t, fv4 (&br)[BU]) {
    int64_t p, s0;
    advance(bc, p, s0);
    if (EDGE != 2 || s0 + KT <= S) {
#pragma unroll
      for (int q = 0; q < BU; ++q) {
        const int L = q * 256 + tid, j = min(L / 8, l - 1), u = L % 8;
        const int64_t sg = s0 + 4 * u;
        const f4u_t b = *reinterpret_cast<const f4u_t*>(Bt + (int64_t)j * m + p * S + (EDGE == 0 || sg < S ? sg : S - 4));
        br[q] = fv4{b[0], b[1], b[2], b[3]};
      }
      return;
    }
    const bool live = t < t1;
#pragma unroll
    for (int q = 0; q < BU; ++q) {
      const int L = q * 256 + tid, j = L / 8, u = L % 8;
      const int64_t sg = s0 + 4 * u;
      const int cnt = (live && j < l) ? (int)max<int64_t>(0, min<int64_t>(4, S - sg)) : 0;
      float b[4];
      load_n<float, 4>(Bt + (int64_t)j * m + p * S + sg, cnt, b);
      br[q] = fv4{b[0], b[1], b[2], b[3]};
    }
  };
  // Bt units -> LDS pieces: unit u of row j holds stage columns 4 u .. 4 u + 3,
  // k slots 8 u .. 8 u + 3 (u < 4) or 8 (u - 4) + 4 .. + 3
  auto lstore = [&](int buf, const fv4 (&br)[BU]) {
#pragma unroll
    for (int q = 0; q < BU; ++q) {
      const int L = q * 256 + tid, j = L / 8, u = L % 8;
      const int kk = u < 4 ? 8 * u : 8 * (u - 4) + 4;
      const float f[4] = {br[q][0], br[q][1], br[q][2], br[q][3]};
      bf16x4_t pc[NP];
      bf_pieces4<NP>(f, pc);
#pragma unroll
      for (int c = 0; c < NP; ++c) *reinterpret_cast<bf16x4_t*>(&bs[buf][c][j][kk]) = pc[c];
    }
  };

  floatx4 acc[2][NJ];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int u = 0; u < NJ; ++u) acc[h][u] = floatx4{0.f, 0.f, 0.f, 0.f};
  double nacc = 0.0;
  // X of a stage into pieces (and, for a stage of the split, its squares
  // into the norm sum)
  auto prep = [&](const fv4 (&xr)[4], bf16x8 (&ap)[2][NP], bool counted) {
    if constexpr (NORM) {  // no branch: a branch would end the block the products share
      double sq = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double v = (q < 2 ? rowa : rowb) ? (double)xr[q][e] : 0.0;
          sq = fma(v, v, sq);
        }
      nacc += counted ? sq : 0.0;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float f[8] = {xr[2 * h][0],     xr[2 * h][1],     xr[2 * h][2],     xr[2 * h][3],
                          xr[2 * h + 1][0], xr[2 * h + 1][1], xr[2 * h + 1][2], xr[2 * h + 1][3]};
      bf_pieces<NP>(f, ap[h]);
    }
  };
  // the stage's products, two j tiles at a time (four independent chains)
  auto mma = [&](int buf, const bf16x8 (&ap)[2][NP]) {
#pragma unroll
    for (int u0 = 0; u0 < NJ; u0 += 2) {
      constexpr int W2 = 2;
      bf16x8 bp[W2][NP];
#pragma unroll
      for (int uu = 0; uu < W2; ++uu)
        if (u0 + uu < NJ)
#pragma unroll
          for (int c = 0; c < NP; ++c)
            bp[uu][c] = *reinterpret_cast<const bf16x8*>(&bs[buf][c][16 * (u0 + uu) + mm][8 * g]);
#pragma unroll
      for (int k = 0; k < PR::N; ++k)
#pragma unroll
        for (int uu = 0; uu < W2; ++uu)
          if (u0 + uu < NJ)
#pragma unroll
            for (int h = 0; h < 2; ++h)
              acc[h][u0 + uu] = mfma_bf16(ap[h][PR::A[k]], bp[uu][PR::B[k]], acc[h][u0 + uu]);
    }
  };

  // Software pipeline over the split's K stages, stage k = t0 + k. X loads
  // run four stages ahead through a ring of four register slots (slot
  // k % 4), Bt loads (mostly L2 hits: the row blocks of a split share them)
  // two ahead through two; while the matrix cores take stage k (pieces from
  // the previous step, Bt pieces in LDS buffer k % 2), the vector unit splits
  // stage k + 1's X and stages its Bt into the other buffer. The loop is
  // unrolled by four so that every slot index is a constant.
  const int64_t K = t1 - t0;
  fv4 xs[4][4], bsl[2][BU];
  bf16x8 apc[2][2][NP];
  auto step = [&](int64_t k, auto sc) {
    constexpr int sl = decltype(sc)::value, cur = sl & 1, nxt = cur ^ 1;
    xload(t0 + k + 4, xs[sl]);
    bload(t0 + k + 2, bsl[cur]);
    __builtin_amdgcn_sched_barrier(0);
    mma(cur, apc[cur]);
    prep(xs[(sl + 1) & 3], apc[nxt], k + 1 < K);
    lstore(nxt, bsl[nxt]);
    // issue order: the first pair of j tiles' piece reads, then the stage's
    // products, each followed by two vector instructions (the next stage's
    // split); the later piece reads go where their products need them
    constexpr int FIRST_READS = NP * (NJ < 2 ? NJ : 2), NMFMA = PR::N * 2 * NJ;
    __builtin_amdgcn_sched_group_barrier(0x100, FIRST_READS, 0);
#pragma unroll
    for (int i = 0; i < NMFMA; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
    }
    lds_barrier();
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  using S3 = std::integral_constant<int, 3>;
  if (K > 0) {
    xload(t0, xs[0]);
    bload(t0, bsl[0]);
    xload(t0 + 1, xs[1]);
    bload(t0 + 1, bsl[1]);
    xload(t0 + 2, xs[2]);
    xload(t0 + 3, xs[3]);
    prep(xs[0], apc[0], true);
    lstore(0, bsl[0]);
    lds_barrier();
    int64_t k = 0;
    for (; k + 4 <= K; k += 4) {
      step(k, S0{});
      step(k + 1, S1{});
      step(k + 2, S2{});
      step(k + 3, S3{});
    }
    if (k < K) step(k, S0{});
    if (k + 1 < K) step(k + 1, S1{});
    if (k + 2 < K) step(k + 2, S2{});
  }
  if constexpr (NORM) {
    // fixed order: a butterfly over the lanes, then the two waves of each
    // 64-row half in index order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nacc += __shfl_xor(nacc, o, 64);
    if (lane == 0) nred[wave] = nacc;
    __syncthreads();
    if (tid < 2) {
      const int64_t b64 = 2 * (int64_t)rb + tid;
      if (b64 < nslots) npart[(int64_t)split * nslots + b64] = nred[2 * tid] + nred[2 * tid + 1];
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int u = 0; u < NJ; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 16 * h + 4 * g + v;
        const int col = 16 * u + mm;
        if (row < n && col < l) part[((int64_t)split * n + row) * l + col] = acc[h][u][v];
      }
}

template <int NP, int NJ, int EDGE, bool NORM>
__global__ __launch_bounds__(256, 2) void k_cr_split(const float* __restrict__ X, const float* __restrict__ Bt, int64_t n,
                                                  int64_t S, int l, int64_t m, int64_t spp, int64_t nsteps,
                                                  int nsplit, int nrblocks, int nslots, float* __restrict__ part,
                                                  double* __restrict__ npart) {
  int split, rb;
  if (!xcd_decode((int)blockIdx.x, nsplit, nrblocks, &split, &rb)) return;
  cr_split_body<NP, NJ, EDGE, NORM>(X, Bt, n, S, l, m, spp, nsteps, nsplit, nslots, part, npart, split, rb);
}

// ---------------------------------------------------------------------------
// Column reduction, S == 1: X is [P, n] with rows p contiguous along i (the
// output row index). A batch covers 4 * KB consecutive p; k-slot g of the
// MFMA takes p = pbase + KB g + q, q < KB, for both operands.
// ---------------------------------------------------------------------------
template <int MK, int NJ>
__device__ __forceinline__ void cr_cols_body(const typename Pol<MK>::T* __restrict__ X,
                                                 const typename Pol<MK>::T* __restrict__ Bt, int64_t P, int64_t n,
                                                 int l, int64_t nsteps, int nsplit,
                                                 typename Pol<MK>::part_t* __restrict__ part, int split, int rb) {
  using Po = Pol<MK>;
  using T = typename Po::T;
  constexpr int KL = Po::KL, MV = Po::MV, NH = 4 / MV;
  constexpr int KB = (KL == 1) ? 4 : KL;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int mm = lane & 15, g = lane >> 4;
  const int64_t r0 = ((int64_t)rb * 4 + wave) * 64;
  if (r0 >= n) return;
  const int64_t t0 = nsteps * split / nsplit, t1 = nsteps * (split + 1) / nsplit;

  typename Po::acc_t acc[4][NJ];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NJ; ++b) acc[a][b] = typename Po::acc_t{0, 0, 0, 0};

  auto fetch = [&](int64_t t, T (&fa)[4][KB], T (&fb)[NJ][KB]) {
    const int64_t pq = t * 4 * KB + KB * g;
    const int pcnt = t < t1 ? (int)min<int64_t>(KB, P - pq) : 0;
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      const int64_t p = pq + q;
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int64_t base = r0 + h * 16 * MV + MV * mm;
        T v[MV];
        load_n<T, MV>(X + p * n + base, q < pcnt ? (int)min<int64_t>(MV, n - base) : 0, v);
#pragma unroll
        for (int vv = 0; vv < MV; ++vv) fa[h * MV + vv][q] = v[vv];
      }
    }
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
      const int j = 16 * u + mm;
      load_n<T, KB>(Bt + (int64_t)j * P + pq, j < l ? pcnt : 0, fb[u]);
    }
  };
  auto compute = [&](T (&fa)[4][KB], T (&fb)[NJ][KB]) {
#pragma unroll
    for (int q = 0; q < KB; q += KL)
#pragma unroll
      for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int u = 0; u < NJ; ++u) acc[tm][u] = mma<MK>(&fa[tm][q], &fb[u][q], acc[tm][u]);
  };
  T a0[4][KB], b0[NJ][KB], a1[4][KB], b1[NJ][KB];
  fetch(t0, a0, b0);
  fetch(t0 + 1, a1, b1);
  for (int64_t t = t0; t < t1; t += 2) {
    compute(a0, b0);
    fetch(t + 2, a0, b0);
    compute(a1, b1);
    fetch(t + 3, a1, b1);
  }
  // tile tm = h * MV + vv holds output rows r0 + h*16*MV + MV*dr + vv
#pragma unroll
  for (int tm = 0; tm < 4; ++tm)
#pragma unroll
    for (int u = 0; u < NJ; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int h = tm / MV, vv = tm % MV;
        const int64_t row = r0 + h * 16 * MV + MV * mfma_drow<MK>(lane, v) + vv;
        const int col = 16 * u + mm;
        if (row < n && col < l) part[((int64_t)split * n + row) * l + col] = acc[tm][u][v];
      }
}

template <int MK, int NJ>
__global__ __launch_bounds__(256) void k_cr_cols(const typename Pol<MK>::T* __restrict__ X,
                                                 const typename Pol<MK>::T* __restrict__ Bt, int64_t P, int64_t n,
                                                 int l, int64_t nsteps, int nsplit, int nrblocks,
                                                 typename Pol<MK>::part_t* __restrict__ part) {
  int split, rb;
  if (!xcd_decode((int)blockIdx.x, nsplit, nrblocks, &split, &rb)) return;
  cr_cols_body<MK, NJ>(X, Bt, P, n, l, nsteps, nsplit, part, split, rb);
}

static void cr_geom(tucker_precision prec, const View3& v, int64_t* nsteps, int64_t* spp, int* nrblocks) {
  if (v.S == 1) {
    const int kb = prec == TUCKER_BF16 ? 8 : 4;
    *spp = 0;
    *nsteps = (v.P + 4 * kb - 1) / (4 * kb);
    *nrblocks = (int)((v.n + 255) / 256);
  } else {
    const int kt = prec == TUCKER_FP64 ? 32 : 64;  // stage width of k_cr_lds
    *spp = (v.S + kt - 1) / kt;
    *nsteps = v.P * *spp;
    *nrblocks = (int)((v.n + 63) / 64);
  }
}

int colreduce_splits_prec(const View3& v, tucker_precision prec) {
  int64_t nsteps, spp;
  int nrb;
  cr_geom(prec, v, &nsteps, &spp, &nrb);
  // S == 1: about 2048 waves (2 per SIMD), each wave at least 8 steps.
  // S > 1: about 1536 workgroups (two resident per CU), each at least 8 stages.
  int64_t ns;
  if (v.S == 1) {
    const int64_t waves_per_split = std::min<int64_t>((v.n + 63) / 64, 4 * (int64_t)nrb);
    ns = (2048 + waves_per_split - 1) / waves_per_split;
  } else {
    ns = (1536 + nrb - 1) / nrb;
  }
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, nsteps / (v.S == 1 ? 2 : 8)));
  // a multiple of 8 so the XCD mapping has no holes
  if (ns > 8) ns = ns / 8 * 8;
  return (int)std::max<int64_t>(1, ns);
}

int colreduce_splits(const View3& v, int l) {
  (void)l;
  return colreduce_splits_prec(v, TUCKER_FP32);
}

// The split count a column reduction of this precision launches with. The
// split kernel (FP32 products, S > 1) runs 128-row workgroups, two resident
// per CU (512 on the 256 CUs): the rule above, made for 64-row workgroups,
// gives it about 1.5 rounds of them, and the half-full last round costs a
// quarter of the time. Here it takes the splits that fill one round (each at
// least 8 stages; never more than the rule above, which sizes the workspace).
// The BF16-operand kernel (64-row workgroups) holds four per CU at l <= 32
// (128 registers) and two above: where the rule gives it between one and two
// rounds, it takes one as well.
int colreduce_splits_for(const View3& v, int l, tucker_precision prec) {
  const int ns = colreduce_splits(v, l);
  if (v.S == 1) return ns;
  if (prec == TUCKER_BF16) {
    const int64_t resident = l <= 32 ? 1024 : 512, nrb = (v.n + 63) / 64;
    if ((int64_t)ns * nrb <= resident || (int64_t)ns * nrb >= 2 * resident) return ns;
    int64_t t = std::max<int64_t>(1, resident / nrb);
    if (t > 8) t = t / 8 * 8;
    return (int)std::min<int64_t>(t, ns);
  }
  if (prec != TUCKER_FP32 || !fp32_split_products()) return ns;
  constexpr int64_t kResident = 512;
  int64_t nsteps, spp;
  int nrb;
  cr_split_geometry(v, &nsteps, &spp, &nrb);
  int64_t t = std::max<int64_t>(1, kResident / nrb);
  t = std::min<int64_t>(t, std::max<int64_t>(1, nsteps / 8));
  if (t > 8) t = t / 8 * 8;
  return (int)std::min<int64_t>(t, ns);
}

size_t colreduce_part_bytes(const View3& v, int l, tucker_precision prec) {
  const int ns = std::max(colreduce_splits_prec(v, prec), colreduce_splits_prec(v, TUCKER_FP32));
  const size_t b = (size_t)ns * (size_t)v.n * (size_t)l * elem_bytes(prec);
  // FP32 and BF16 plans (whose last step runs on FP32 operands) may take the fused power step
  return prec == TUCKER_FP64 ? b : std::max(b, power_fused_part_bytes(v, l, TUCKER_FP32));
}

template <int MK, int NJ>
static hipError_t cr_launch(const View3& v, const void* X, const void* Bt, int l, void* part, int nsplit,
                            double* npart, hipStream_t st) {
  using Po = Pol<MK>;
  using T = typename Po::T;
  using PT = typename Po::part_t;
  const tucker_precision prec = MK == MF_F64 ? TUCKER_FP64 : (MK == MF_BF16 ? TUCKER_BF16 : TUCKER_FP32);
  int64_t nsteps, spp;
  int nrb;
  cr_geom(prec, v, &nsteps, &spp, &nrb);
  const unsigned blocks = (unsigned)(((nsplit + 7) / 8) * 8 * nrb);
  const int64_t m = v.P * v.S;
  if (v.S == 1) {
    TK_LAUNCH((k_cr_cols<MK, NJ>), dim3(blocks), dim3(256), 0, st, (const T*)X, (const T*)Bt, v.P, v.n, l, nsteps,
              nsplit, nrb, (PT*)part);
  } else {
    constexpr int VE = 16 / (int)sizeof(T);
    const int edge = v.S % LdsPol<MK>::KT == 0 ? 0 : (v.S % VE == 0 ? 1 : 2);
#define TK_CR_LDS(E)                                                                                       \
  TK_LAUNCH((k_cr_lds<MK, NJ, E>), dim3(blocks), dim3(256), 0, st, (const T*)X, (const T*)Bt, v.n, v.S, l, \
                     m, spp, nsteps, nsplit, nrb, (PT*)part, npart)
    if (edge == 0) TK_CR_LDS(0);
    else if (edge == 1) TK_CR_LDS(1);
    else TK_CR_LDS(2);
#undef TK_CR_LDS
  }
  return hipGetLastError();
}

template <int MK>
static hipError_t cr_dispatch(const View3& v, const void* X, const void* Bt, int l, void* part, int nsplit,
                              double* npart, hipStream_t st) {
  switch ((l + 15) / 16) {
    case 1: return cr_launch<MK, 1>(v, X, Bt, l, part, nsplit, npart, st);
    case 2: return cr_launch<MK, 2>(v, X, Bt, l, part, nsplit, npart, st);
    case 3: return cr_launch<MK, 3>(v, X, Bt, l, part, nsplit, npart, st);
    case 4: return cr_launch<MK, 4>(v, X, Bt, l, part, nsplit, npart, st);
    default: return hipErrorInvalidValue;
  }
}

// FP32 storage through k_cr_split (S > 1): NP = 3 pieces (FP32 products) or
// 1 (BF16 operands). Stages of 32 columns, 128-row workgroups; the split
// count (and so the partial layout) is the one colreduce_splits_prec gives.
template <int NP, int NJ>
static hipError_t crs_launch(const View3& v, const void* X, const void* Bt, int l, void* part, int nsplit,
                             double* npart, hipStream_t st) {
  constexpr int KT = 32;
  const int64_t spp = (v.S + KT - 1) / KT, nsteps = v.P * spp;
  const int nrb = (int)((v.n + 127) / 128), nslots = (int)((v.n + 63) / 64);
  const unsigned blocks = (unsigned)(((nsplit + 7) / 8) * 8 * nrb);
  const int64_t m = v.P * v.S;
  const int edge = v.S % KT == 0 ? 0 : (v.S % 4 == 0 ? 1 : 2);
#define TK_CRS(E, NM)                                                                                              \
  TK_LAUNCH((k_cr_split<NP, NJ, E, NM>), dim3(blocks), dim3(256), 0, st, (const float*)X, (const float*)Bt, v.n, \
            v.S, l, m, spp, nsteps, nsplit, nrb, nslots, (float*)part, npart)
  if (npart != nullptr) {
    if (edge == 0) TK_CRS(0, true);
    else if (edge == 1) TK_CRS(1, true);
    else TK_CRS(2, true);
  } else {
    if (edge == 0) TK_CRS(0, false);
    else if (edge == 1) TK_CRS(1, false);
    else TK_CRS(2, false);
  }
#undef TK_CRS
  return hipGetLastError();
}

template <int NP>
static hipError_t crs_dispatch(const View3& v, const void* X, const void* Bt, int l, void* part, int nsplit,
                               double* npart, hipStream_t st) {
  switch ((l + 15) / 16) {
    case 1: return crs_launch<NP, 1>(v, X, Bt, l, part, nsplit, npart, st);
    case 2: return crs_launch<NP, 2>(v, X, Bt, l, part, nsplit, npart, st);
    case 3: return crs_launch<NP, 3>(v, X, Bt, l, part, nsplit, npart, st);
    case 4: return crs_launch<NP, 4>(v, X, Bt, l, part, nsplit, npart, st);
    default: return hipErrorInvalidValue;
  }
}

int colreduce_norm_slots(const View3& v, int nsplit) {
  return v.S > 1 ? nsplit * (int)((v.n + 63) / 64) : 0;
}

hipError_t launch_colreduce(tucker_precision prec, const View3& v, const void* X, const void* Bt, int l,
                            void* part, int nsplit, hipStream_t st, double* npart) {
  const double N = (double)v.P * v.n * v.S, es = (double)elem_bytes(prec);
  if (v.S == 1) npart = nullptr;
  TimingScope ts(KC_COLREDUCE, st, N * es + N / v.n * l * es, 2.0 * N * l, true);
  switch (prec) {
    case TUCKER_FP64: return cr_dispatch<MF_F64>(v, X, Bt, l, part, nsplit, npart, st);
    case TUCKER_FP32:
      return v.S > 1 && fp32_split_products() ? crs_dispatch<3>(v, X, Bt, l, part, nsplit, npart, st)
                                              : cr_dispatch<MF_F32>(v, X, Bt, l, part, nsplit, npart, st);
    case TUCKER_BF16:  // the LDS-staged kernel: its 256-byte row runs read HBM faster here
      return cr_dispatch<MF_BF16>(v, X, Bt, l, part, nsplit, npart, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of the split partials, with the -alpha Q term.
// 8 threads per element, each summing a fixed eighth of the splits; the eight
// partial sums are added in lane order, so the result does not depend on
// scheduling.
// ---------------------------------------------------------------------------
template <typename PT, typename QT>
__device__ __forceinline__ void reduce_splits_body(const PT* __restrict__ part, int nsplit, int64_t nl,
                                                       const QT* __restrict__ qsub,
                                                       const double* __restrict__ alpha, double* __restrict__ Y, int bid) {
  const int sub = threadIdx.x & 7;
  const int64_t e = (int64_t)bid * 32 + (threadIdx.x >> 3);
  double s = 0.0;
  if (e < nl) {
    const int s0 = (int)((int64_t)nsplit * sub / 8), s1 = (int)((int64_t)nsplit * (sub + 1) / 8);
    // eight loads in flight, added in split order (the same sum as one by one)
    int sp = s0;
    for (; sp + 8 <= s1; sp += 8) {
      PT v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = part[(int64_t)(sp + q) * nl + e];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += (double)v[q];
    }
    for (; sp < s1; ++sp) s += (double)part[(int64_t)sp * nl + e];
  }
  double t[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) t[q] = __shfl(s, (int)(threadIdx.x & ~7u) + q, 64);
  if (sub != 0 || e >= nl) return;
  double y = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
  if (qsub != nullptr) y -= (*alpha) * (double)qsub[e];
  Y[e] = y;
}

template <typename PT, typename QT>
__global__ __launch_bounds__(256) void k_reduce_splits(const PT* __restrict__ part, int nsplit, int64_t nl,
                                                       const QT* __restrict__ qsub,
                                                       const double* __restrict__ alpha, double* __restrict__ Y) {
  reduce_splits_body<PT, QT>(part, nsplit, nl, qsub, alpha, Y, (int)blockIdx.x);
}

hipError_t launch_reduce_splits(tucker_precision part_prec, const void* part, int nsplit, int64_t nl,
                                const void* qsub, tucker_precision qsub_prec, const double* alpha, double* Y,
                                hipStream_t st) {
  const unsigned blocks = (unsigned)((nl + 31) / 32);
  if (blocks == 0) return hipSuccess;
  TimingScope ts(KC_REDUCE, st, (double)nsplit * nl * elem_bytes(part_prec) + 8.0 * nl, 0.0);
  const bool pd = part_prec == TUCKER_FP64, qd = qsub_prec == TUCKER_FP64;
  if (pd && qd)
    hipLaunchKernelGGL((k_reduce_splits<double, double>), dim3(blocks), dim3(256), 0, st, (const double*)part,
                       nsplit, nl, (const double*)qsub, alpha, Y);
  else if (pd)
    hipLaunchKernelGGL((k_reduce_splits<double, float>), dim3(blocks), dim3(256), 0, st, (const double*)part,
                       nsplit, nl, (const float*)qsub, alpha, Y);
  else if (qd)
    hipLaunchKernelGGL((k_reduce_splits<float, double>), dim3(blocks), dim3(256), 0, st, (const float*)part,
                       nsplit, nl, (const double*)qsub, alpha, Y);
  else
    hipLaunchKernelGGL((k_reduce_splits<float, float>), dim3(blocks), dim3(256), 0, st, (const float*)part,
                       nsplit, nl, (const float*)qsub, alpha, Y);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row contraction, S > 1: out(p, j, s) = sum_i X[p, i, s] W(i, j), with
// W(i, j) = W[i * wsi + j * wsj] and out(p, j, s) = out[p * osp + j * osj + s].
// Output rows are s (contiguous). Each wave owns a 64-column tile of one p
// (4 interleaved 16-row MFMA tiles), 4 waves per workgroup, all n rows per
// wave, in batches of 4 * KB rows: k-slot g takes i = i0 + KB g + q, q < KB.
// ---------------------------------------------------------------------------
template <int MK, int NJ, bool WVEC, bool KSPLIT>
__device__ __forceinline__ void rc_rows_body(const typename Pol<MK>::T* __restrict__ X,
                                                 const typename Pol<MK>::T* __restrict__ W, int64_t n, int64_t S,
                                                 int lw, int64_t wsi, int64_t wsj, int64_t tiles_per_p,
                                                 int64_t ntiles, typename Pol<MK>::T* __restrict__ out,
                                                 int64_t osp, int64_t osj, int bid) {
  constexpr bool ksplit = KSPLIT;
  using Po = Pol<MK>;
  using T = typename Po::T;
  constexpr int KL = Po::KL, MV = Po::MV, NH = 4 / MV;
  constexpr int KB = (KL == 1) ? 4 : KL, ROWS = 4 * KB;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int mm = lane & 15, g = lane >> 4;
  // ksplit: the 4 waves of a workgroup share one tile and split the n rows
  // (in whole batches), adding their partial tiles in wave order at the end
  // (few tiles); otherwise each wave owns a tile and all n rows.
  const int64_t tile = ksplit ? (int64_t)bid : (int64_t)bid * 4 + wave;
  if (ksplit ? tile >= ntiles : (int64_t)bid * 4 >= ntiles) return;
  const bool live = tile < ntiles;
  const int64_t p = live ? tile / tiles_per_p : 0;
  const int64_t s0 = (tile - p * tiles_per_p) * 64;
  const T* xp = X + p * n * S;
  const int64_t nbat = (n + ROWS - 1) / ROWS;
  const int64_t iw0 = ksplit ? nbat * wave / 4 * ROWS : 0;
  const int64_t iw1 = !live ? 0 : ksplit ? min<int64_t>(n, nbat * (wave + 1) / 4 * ROWS) : n;

  typename Po::acc_t acc[4][NJ];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NJ; ++b) acc[a][b] = typename Po::acc_t{0, 0, 0, 0};

  auto fetch = [&](int64_t i0, T (&fa)[4][KB], T (&fb)[NJ][KB]) {
    const int64_t iq = i0 + KB * g;
    const int icnt = (int)max<int64_t>(-1, min<int64_t>(KB, iw1 - iq));
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      const int64_t i = iq + q;
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int64_t base = s0 + h * 16 * MV + MV * mm;
        T v[MV];
        load_n<T, MV>(xp + i * S + base, q < icnt ? (int)min<int64_t>(MV, S - base) : 0, v);
#pragma unroll
        for (int vv = 0; vv < MV; ++vv) fa[h * MV + vv][q] = v[vv];
      }
    }
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
      const int j = 16 * u + mm;
      if constexpr (WVEC) {
        load_n<T, KB>(W + (int64_t)j * wsj + iq, j < lw ? icnt : 0, fb[u]);
      } else {
#pragma unroll
        for (int q = 0; q < KB; ++q) fb[u][q] = (q < icnt && j < lw) ? W[(iq + q) * wsi + (int64_t)j * wsj] : T(0);
      }
    }
  };
  auto compute = [&](T (&fa)[4][KB], T (&fb)[NJ][KB]) {
#pragma unroll
    for (int q = 0; q < KB; q += KL)
#pragma unroll
      for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int u = 0; u < NJ; ++u) acc[tm][u] = mma<MK>(&fa[tm][q], &fb[u][q], acc[tm][u]);
  };
  // Interior: pairs of whole batches of a full-width tile, read with
  // unconditional loads (W rows j >= lw are clamped to lw - 1: they feed only
  // output columns that are never written). With no branch around a load the
  // compiler keeps the next batch in flight across this batch's MFMAs; the
  // prefetch past the last pair re-reads that pair. The remaining rows (and
  // every row of an edge tile) take the guarded path.
  const bool wide = live && s0 + 64 <= S;
  const int64_t npair = (WVEC && wide) ? (iw1 - iw0) / (2 * ROWS) : 0;
  auto ffetch = [&](int64_t i0, T (&fa)[4][KB], T (&fb)[NJ][KB]) {
    const int64_t iq = i0 + KB * g;
#pragma unroll
    for (int q = 0; q < KB; ++q) {
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        T v[MV];
        *reinterpret_cast<f4u_t*>(v) =
            *reinterpret_cast<const f4u_t*>(xp + (iq + q) * S + s0 + h * 16 * MV + MV * mm);
#pragma unroll
        for (int vv = 0; vv < MV; ++vv) fa[h * MV + vv][q] = v[vv];
      }
    }
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
      const T* wr = W + (int64_t)min(16 * u + mm, lw - 1) * wsj + iq;
#pragma unroll
      for (int c = 0; c < (int)(sizeof(T) * KB / 16); ++c)
        *reinterpret_cast<f4u_t*>(reinterpret_cast<char*>(fb[u]) + 16 * c) =
            *reinterpret_cast<const f4u_t*>(reinterpret_cast<const char*>(wr) + 16 * c);
    }
  };
  T a0[4][KB], b0[NJ][KB], a1[4][KB], b1[NJ][KB];
  int64_t ig = iw0;  // first row of the guarded remainder
  if (npair > 0) {
    const int64_t last = iw0 + (2 * npair - 2) * ROWS;
    // the fence keeps the prologue's loads in the loop's order (batch 0, then
    // batch 1): the wait-count pass merges the orders of both paths into the
    // loop head, and interleaved prologue loads made every iteration wait for
    // nearly all loads in flight, the batch just issued included
    ffetch(iw0, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    ffetch(iw0 + ROWS, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    for (int64_t k = 0; k < npair; ++k) {
      const int64_t nx = min<int64_t>(iw0 + (2 * k + 2) * ROWS, last);
      // scheduling fences keep the pipeline order: a batch's loads are issued
      // right after the MFMAs that free its registers, one batch ahead
      compute(a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      ffetch(nx, a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      compute(a1, b1);
      __builtin_amdgcn_sched_barrier(0);
      ffetch(nx + ROWS, a1, b1);
      __builtin_amdgcn_sched_barrier(0);
    }
    ig = iw0 + 2 * npair * ROWS;
  }
  if (ig < iw1) {
    fetch(ig, a0, b0);
    fetch(ig + ROWS, a1, b1);
    for (int64_t i0 = ig; i0 < iw1; i0 += 2 * ROWS) {
      compute(a0, b0);
      fetch(i0 + 2 * ROWS, a0, b0);  // zero-filled past the wave's last row
      compute(a1, b1);
      fetch(i0 + 3 * ROWS, a1, b1);
    }
  }
  if constexpr (KSPLIT) {
    // (only this instantiation reserves the LDS: without it the row
    // contraction's occupancy is bounded by registers alone)
    using AE = typename Po::part_t;
    __shared__ AE red[3][16 * NJ][64];
    if (wave > 0) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NJ; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) red[wave - 1][(a * NJ + b) * 4 + v][lane] = acc[a][b][v];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NJ; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[a][b][v] += red[w][(a * NJ + b) * 4 + v][lane];
  } else if (!live) {
    return;
  }
  // tile tm = h * MV + vv, result row dr -> column s0 + h*16*MV + MV*dr + vv
  T* op = out + p * osp;
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int j = 16 * u + mm;
    if (j >= lw) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int dr = mfma_drow<MK>(lane, v);
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int64_t c = s0 + h * 16 * MV + MV * dr;
        T* dst = op + (int64_t)j * osj + c;
        if constexpr (MV == 4) {
          if (c + 3 < S) {
            const f4u_t o = {(float)acc[h * MV + 0][u][v], (float)acc[h * MV + 1][u][v],
                             (float)acc[h * MV + 2][u][v], (float)acc[h * MV + 3][u][v]};
            *reinterpret_cast<f4u_t*>(dst) = o;
            continue;
          }
        }
#pragma unroll
        for (int vv = 0; vv < MV; ++vv)
          if (c + vv < S) dst[vv] = (T)acc[h * MV + vv][u][v];
      }
    }
  }
}

template <int MK, int NJ, bool WVEC, bool KSPLIT>
__global__ __launch_bounds__(256) void k_rc_rows(const typename Pol<MK>::T* __restrict__ X,
                                                 const typename Pol<MK>::T* __restrict__ W, int64_t n, int64_t S,
                                                 int lw, int64_t wsi, int64_t wsj, int64_t tiles_per_p,
                                                 int64_t ntiles, typename Pol<MK>::T* __restrict__ out,
                                                 int64_t osp, int64_t osj) {
  rc_rows_body<MK, NJ, WVEC, KSPLIT>(X, W, n, S, lw, wsi, wsj, tiles_per_p, ntiles, out, osp, osj, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Row contraction, S > 1, FP32 storage on the BF16 matrix cores (NP as for
// k_cr_split; taken from 1024 tiles of 32 columns): out(p, j, s) = sum_i X[p, i, s] W(i, j), W(i, j) =
// W[i * wsi + j * wsj]. Each wave owns a 32-column tile of one p (2
// interleaved 16-row tiles: tile t, result row dr -> column s0 + 2 dr + t;
// a lane reads 8 bytes of each row, a row's 128 bytes per instruction), 4
// waves per workgroup, all n rows in batches of 32: k slot 8 g + q is row
// i0 + 8 g + q for X and W alike. A batch of W (32 rows x 16 NJ columns) is
// read by the whole workgroup, converted once into BF16 pieces and kept in
// LDS (double buffered), where all four waves read it; each wave converts
// its own X. The next batch's loads go out before the current batch's
// products. A partial batch (n not a multiple of 32) is taken first, with
// guarded loads; the full batches follow with unconditional ones. Waves past
// the last tile work on the last tile (their loads stay in bounds and they
// take part in the barriers) and write nothing. The small per-wave state
// (two tiles) fits three waves on each SIMD, which the launch bound asks for
// (without it the compiler took 172 registers, two waves).
// WVEC: W contiguous along i (wsi = 1), a unit's 8 rows are two 16-byte loads.
// ---------------------------------------------------------------------------
constexpr int RCS_COLS = 32;  // output columns s per wave

typedef float f2u_t __attribute__((ext_vector_type(2), aligned(4)));

template <int NP, int NJ, bool WVEC>
__device__ __forceinline__ void rc_split_body(const float* __restrict__ X, const float* __restrict__ W, int64_t n,
                                              int64_t S, int lw, int64_t wsi, int64_t wsj, int64_t tiles_per_p,
                                              int64_t ntiles, float* __restrict__ out, int64_t osp, int64_t osj,
                                              int bid) {
  constexpr int LS = 32 + 8;  // padded LDS row (BF16 elements)
  using PR = BfProducts<NP>;
  __shared__ __align__(16) __bf16 ws[2][NP][16 * NJ][LS];
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  const int mm = lane & 15, g = lane >> 4;
  const int64_t traw = (int64_t)bid * 4 + wave;
  const bool live = traw < ntiles;
  const int64_t tile = live ? traw : ntiles - 1;
  const int64_t p = tile / tiles_per_p;
  const int64_t s0 = (tile - p * tiles_per_p) * RCS_COLS;
  const float* xp = X + p * n * S;
  const int64_t sc = s0 + 2 * mm;  // the lane's 2 columns
  // this thread's W unit: column tid / 4 (clamped: columns past lw feed only
  // outputs that are never written), rows 8 (tid % 4) .. + 7 of the batch;
  // threads past 64 NJ load a clamped unit and store nothing
  const int wj = tid >> 2, wq = tid & 3;
  const bool wunit = wj < 16 * NJ;
  const float* wcol = W + (int64_t)min(wj, lw - 1) * wsj;
  const int64_t nfull = n / 32;
  const bool tail = n % 32 != 0;

  floatx4 acc[2][NJ];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < NJ; ++u) acc[t][u] = floatx4{0.f, 0.f, 0.f, 0.f};
  float xr[8][2];  // X of a batch: rows i0 + 8 g + q, columns sc, sc + 1
  float wr[8];     // the W unit of a batch

  // GUARD: rows at or past n read as zero (the partial batch)
  auto wload = [&](int64_t i0, auto guard_c) {
    constexpr bool GUARD = decltype(guard_c)::value;
    const int64_t ib = i0 + 8 * wq;
    if constexpr (WVEC && !GUARD) {
      const f4u_t v0 = *reinterpret_cast<const f4u_t*>(wcol + ib);
      const f4u_t v1 = *reinterpret_cast<const f4u_t*>(wcol + ib + 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        wr[e] = v0[e];
        wr[4 + e] = v1[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t i = ib + e;
        const float v = wcol[(GUARD ? min<int64_t>(i, n - 1) : i) * wsi];
        wr[e] = (!GUARD || i < n) ? v : 0.f;
      }
    }
  };
  auto wstore = [&](int buf) {
    if (!wunit) return;
    bf16x8 pc[NP];
    bf_pieces<NP>(wr, pc);
#pragma unroll
    for (int c = 0; c < NP; ++c) *reinterpret_cast<bf16x8*>(&ws[buf][c][wj][8 * wq]) = pc[c];
  };
  // WIDE: the tile's columns lie inside the row (else columns at or past S
  // read as zero, element by element)
  auto xload = [&](int64_t i0, auto guard_c, auto wide_c) {
    constexpr bool GUARD = decltype(guard_c)::value, WIDE = decltype(wide_c)::value;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t i = i0 + 8 * g + q;
      const int64_t ir = GUARD ? min<int64_t>(i, n - 1) : i;
      const bool rin = !GUARD || i < n;
      const float* rp = xp + ir * S;
      if constexpr (WIDE) {
        const f2u_t v = *reinterpret_cast<const f2u_t*>(rp + sc);
        xr[q][0] = rin ? v[0] : 0.f;
        xr[q][1] = rin ? v[1] : 0.f;
      } else {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int64_t c = sc + e;
          const float v = rp[min<int64_t>(c, S - 1)];
          xr[q][e] = (rin && c < S) ? v : 0.f;
        }
      }
    }
  };
  auto prep = [&](bf16x8 (&ap)[2][NP]) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      float col[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) col[q] = xr[q][t];
      bf_pieces<NP>(col, ap[t]);
    }
  };
  // the batch's products, two j tiles at a time (four independent chains)
  auto mma = [&](int buf, const bf16x8 (&ap)[2][NP]) {
#pragma unroll
    for (int u0 = 0; u0 < NJ; u0 += 2) {
      bf16x8 bp[2][NP];
#pragma unroll
      for (int uu = 0; uu < 2; ++uu)
        if (u0 + uu < NJ)
#pragma unroll
          for (int c = 0; c < NP; ++c)
            bp[uu][c] = *reinterpret_cast<const bf16x8*>(&ws[buf][c][16 * (u0 + uu) + mm][8 * g]);
#pragma unroll
      for (int k = 0; k < PR::N; ++k)
#pragma unroll
        for (int uu = 0; uu < 2; ++uu)
          if (u0 + uu < NJ)
#pragma unroll
            for (int t = 0; t < 2; ++t)
              acc[t][u0 + uu] = mfma_bf16(ap[t][PR::A[k]], bp[uu][PR::B[k]], acc[t][u0 + uu]);
    }
  };
  using tru = std::integral_constant<bool, true>;
  using fal = std::integral_constant<bool, false>;
  auto run = [&](auto wide_c) {
    bf16x8 ap[2][NP];
    if (nfull == 0) {  // n < 32: one partial batch
      wload(0, tru{});
      wstore(0);
      xload(0, tru{}, wide_c);
      lds_barrier();
      prep(ap);
      mma(0, ap);
      return;
    }
    // batch 0: the partial one when there is one, else full batch 0; batch
    // k > 0: full batch k - 1 or k
    if (tail) {
      wload(32 * nfull, tru{});
      xload(32 * nfull, tru{}, wide_c);
    } else {
      wload(0, fal{});
      xload(0, fal{}, wide_c);
    }
    wstore(0);
    lds_barrier();
    const int64_t nb = nfull + (tail ? 1 : 0);
    for (int64_t k = 0; k < nb; ++k) {
      prep(ap);
      // the next full batch (the last one again past the end: staged, never used)
      const int64_t f = min<int64_t>(k + 1 - (tail ? 1 : 0), nfull - 1);
      wload(32 * f, fal{});
      xload(32 * f, fal{}, wide_c);
      __builtin_amdgcn_sched_barrier(0);
      mma((int)(k & 1), ap);
      wstore((int)((k + 1) & 1));
      lds_barrier();
    }
  };
  if (s0 + RCS_COLS <= S) run(tru{});
  else run(fal{});
  if (!live) return;
  // tile t, result row dr = 4 g + v -> column s0 + 2 dr + t, output row j
  float* op = out + p * osp;
#pragma unroll
  for (int u = 0; u < NJ; ++u) {
    const int j = 16 * u + mm;
    if (j >= lw) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t c = s0 + 2 * (4 * g + v);
      float* dst = op + (int64_t)j * osj + c;
      if (c + 1 < S) {
        const f2u_t o = {acc[0][u][v], acc[1][u][v]};
        *reinterpret_cast<f2u_t*>(dst) = o;
      } else if (c < S) {
        dst[0] = acc[0][u][v];
      }
    }
  }
}

template <int NP, int NJ, bool WVEC>
__global__ __launch_bounds__(256, 3) void k_rc_split(const float* __restrict__ X, const float* __restrict__ W, int64_t n,
                                                  int64_t S, int lw, int64_t wsi, int64_t wsj, int64_t tiles_per_p,
                                                  int64_t ntiles, float* __restrict__ out, int64_t osp, int64_t osj) {
  rc_split_body<NP, NJ, WVEC>(X, W, n, S, lw, wsi, wsj, tiles_per_p, ntiles, out, osp, osj, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Row contraction, S == 1: X is [P, n] (rows p contiguous along i, the
// reduction index); out(p, j) = out[p * osp + j * osj]; each wave owns 64
// rows p, 4 waves per workgroup.
// ---------------------------------------------------------------------------
template <int MK, int NJ, bool WVEC>
__device__ __forceinline__ void rc_cols_body(const typename Pol<MK>::T* __restrict__ X,
                                                 const typename Pol<MK>::T* __restrict__ W, int64_t P, int64_t n,
                                                 int lw, int64_t wsi, int64_t wsj, typename Pol<MK>::T* __restrict__ out,
                                                 int64_t osp, int64_t osj, int bid) {
  using Po = Pol<MK>;
  using T = typename Po::T;
  constexpr int KC = Po::KC;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int mm = lane & 15, g = lane >> 4;
  const int64_t p0 = (int64_t)bid * 64;
  if (p0 >= P) return;
  // the 4 waves split the n reduction rows (in whole batches of 4 KC) and add
  // their partial tiles in wave order at the end
  const int64_t nbat = (n + 4 * KC - 1) / (4 * KC);
  const int64_t iw0 = nbat * wave / 4 * 4 * KC, iw1 = min<int64_t>(n, nbat * (wave + 1) / 4 * 4 * KC);

  typename Po::acc_t acc[4][NJ];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NJ; ++b) acc[a][b] = typename Po::acc_t{0, 0, 0, 0};

  auto fetch = [&](int64_t i0, T (&fa)[4][KC], T (&fb)[NJ][KC]) {
    const int64_t ib = i0 + KC * g;
    const int cnt = (int)max<int64_t>(-1, min<int64_t>(KC, iw1 - ib));
#pragma unroll
    for (int tm = 0; tm < 4; ++tm) {
      const int64_t p = p0 + 16 * tm + mm;
      load_n<T, KC>(X + p * n + ib, p < P ? cnt : 0, fa[tm]);
    }
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
      const int j = 16 * u + mm;
      if constexpr (WVEC) {
        load_n<T, KC>(W + (int64_t)j * wsj + ib, j < lw ? cnt : 0, fb[u]);
      } else {
#pragma unroll
        for (int e = 0; e < KC; ++e) fb[u][e] = (e < cnt && j < lw) ? W[(ib + e) * wsi + (int64_t)j * wsj] : T(0);
      }
    }
  };
  auto compute = [&](T (&fa)[4][KC], T (&fb)[NJ][KC]) {
#pragma unroll
    for (int e = 0; e < KC; e += Po::KL)
#pragma unroll
      for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int u = 0; u < NJ; ++u) acc[tm][u] = mma<MK>(&fa[tm][e], &fb[u][e], acc[tm][u]);
  };
  T a0[4][KC], b0[NJ][KC], a1[4][KC], b1[NJ][KC];
  fetch(iw0, a0, b0);
  fetch(iw0 + 4 * KC, a1, b1);
  for (int64_t i0 = iw0; i0 < iw1; i0 += 8 * KC) {
    compute(a0, b0);
    fetch(i0 + 8 * KC, a0, b0);  // zero-filled past the wave's last row
    compute(a1, b1);
    fetch(i0 + 12 * KC, a1, b1);
  }
  using AE = typename Po::part_t;
  __shared__ AE red[3][16 * NJ][64];
  if (wave > 0) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NJ; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wave - 1][(a * NJ + b) * 4 + v][lane] = acc[a][b][v];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NJ; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[a][b][v] += red[w][(a * NJ + b) * 4 + v][lane];
#pragma unroll
  for (int tm = 0; tm < 4; ++tm)
#pragma unroll
    for (int u = 0; u < NJ; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t p = p0 + 16 * tm + mfma_drow<MK>(lane, v);
        const int j = 16 * u + mm;
        if (p < P && j < lw) out[p * osp + (int64_t)j * osj] = (T)acc[tm][u][v];
      }
}

template <int MK, int NJ, bool WVEC>
__global__ __launch_bounds__(256) void k_rc_cols(const typename Pol<MK>::T* __restrict__ X,
                                                 const typename Pol<MK>::T* __restrict__ W, int64_t P, int64_t n,
                                                 int lw, int64_t wsi, int64_t wsj, typename Pol<MK>::T* __restrict__ out,
                                                 int64_t osp, int64_t osj) {
  rc_cols_body<MK, NJ, WVEC>(X, W, P, n, lw, wsi, wsj, out, osp, osj, (int)blockIdx.x);
}

template <int MK, int NJ>
static hipError_t rc_launch(const View3& v, const void* X, const void* W, int64_t wsi, int64_t wsj, int lw, void* out,
                            bool out_jmajor, hipStream_t st) {
  using T = typename Pol<MK>::T;
  const int64_t m = v.P * v.S;
  const bool wvec = wsi == 1;  // W contiguous along the reduction index
  if (v.S == 1) {
    const int64_t osp = out_jmajor ? 1 : lw, osj = out_jmajor ? m : 1;
    const unsigned blocks = (unsigned)((v.P + 63) / 64);
#define TK_RC_COLS(WV)                                                                                         \
  TK_LAUNCH((k_rc_cols<MK, NJ, WV>), dim3(blocks), dim3(256), 0, st, (const T*)X, (const T*)W, v.P, v.n, \
                     lw, wsi, wsj, (T*)out, osp, osj)
    if (wvec) TK_RC_COLS(true);
    else TK_RC_COLS(false);
#undef TK_RC_COLS
  } else {
    const int64_t osp = out_jmajor ? v.S : (int64_t)lw * v.S, osj = out_jmajor ? m : v.S;
    const int64_t tpp = (v.S + 63) / 64;
    const int64_t ntiles = v.P * tpp;
    // split the rows while the tiles fill fewer than two rounds of the ~2048
    // resident waves (one partial round would leave most of the chip idle)
    const int ksplit = ntiles < 4096 ? 1 : 0;
    // FP32 storage on the BF16 matrix cores: split FP32 products, or BF16
    // operands. Its 32-column tiles keep the chip busy down to about 1024 tiles
    // (50 x 1000 x 1000, mode 1: 1600 tiles, 135 -> 62 us against the FP32
    // row-split kernel), where the 64-column kernels split the rows
    if constexpr (MK == MF_F32 || MK == MF_BF16) {
      const int64_t tpp2 = (v.S + RCS_COLS - 1) / RCS_COLS, nt2 = v.P * tpp2;
      if ((!ksplit || nt2 >= 1024) && (MK == MF_BF16 || fp32_split_products())) {
        constexpr int NP = MK == MF_BF16 ? 1 : 3;
        const unsigned b = (unsigned)((nt2 + 3) / 4);
#define TK_RCS(WV)                                                                                          \
  TK_LAUNCH((k_rc_split<NP, NJ, WV>), dim3(b), dim3(256), 0, st, (const float*)X, (const float*)W, v.n, v.S, \
            lw, wsi, wsj, tpp2, nt2, (float*)out, osp, osj)
        if (wvec) TK_RCS(true);
        else TK_RCS(false);
#undef TK_RCS
        return hipGetLastError();
      }
    }
    const unsigned blocks = (unsigned)(ksplit ? ntiles : (ntiles + 3) / 4);
#define TK_RC_ROWS(WV, KS)                                                                                        \
  TK_LAUNCH((k_rc_rows<MK, NJ, WV, KS>), dim3(blocks), dim3(256), 0, st, (const T*)X, (const T*)W, v.n, v.S, \
                     lw, wsi, wsj, tpp, ntiles, (T*)out, osp, osj)
    if (wvec && ksplit) TK_RC_ROWS(true, true);
    else if (wvec) TK_RC_ROWS(true, false);
    else if (ksplit) TK_RC_ROWS(false, true);
    else TK_RC_ROWS(false, false);
#undef TK_RC_ROWS
  }
  return hipGetLastError();
}

template <int MK>
static hipError_t rc_dispatch(const View3& v, const void* X, const void* W, int64_t wsi, int64_t wsj, int lw,
                              void* out, bool out_jmajor, hipStream_t st) {
  switch ((lw + 15) / 16) {
    case 1: return rc_launch<MK, 1>(v, X, W, wsi, wsj, lw, out, out_jmajor, st);
    case 2: return rc_launch<MK, 2>(v, X, W, wsi, wsj, lw, out, out_jmajor, st);
    case 3: return rc_launch<MK, 3>(v, X, W, wsi, wsj, lw, out, out_jmajor, st);
    case 4: return rc_launch<MK, 4>(v, X, W, wsi, wsj, lw, out, out_jmajor, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rowcontract(tucker_precision mk, const View3& v, const void* X, const void* W, int64_t wsi,
                              int64_t wsj, int lw, void* out, bool out_jmajor, hipStream_t st) {
  const double N = (double)v.P * v.n * v.S, es = (double)elem_bytes(mk);
  TimingScope ts(KC_ROWCONTRACT, st, N * es + N / v.n * lw * es, 2.0 * N * lw, true);
  switch (mk) {
    case TUCKER_FP64: return rc_dispatch<MF_F64>(v, X, W, wsi, wsj, lw, out, out_jmajor, st);
    case TUCKER_FP32: return rc_dispatch<MF_F32>(v, X, W, wsi, wsj, lw, out, out_jmajor, st);
    case TUCKER_BF16: return rc_dispatch<MF_BF16>(v, X, W, wsi, wsj, lw, out, out_jmajor, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Both products of a power step in one pass over X (FP32, S > 1):
//   part[g][i][j] = sum over the column blocks b dealt to workgroup g of
//                   sum_{c in b} X_(k)[i, c] Z[c, j],
//   Z[c, j] = sum_i X_(k)[i, c] Q[i, j]   (Q given j-major, Qt[j n + i]).
// A block is 64 consecutive columns s of one p, all n rows (at most
// PF_NMAX). It crosses HBM once and is staged in LDS: rows of 16 float4
// slots, the slot index XOR-ed with the row's low 4 bits so that the lanes
// of a fragment read hit distinct banks; rows past n are zero. Eight waves,
// two per SIMD, so that one wave's LDS and L2 waits are covered by the
// other's matrix-core work:
//  * Z_b = X_b^T Q: wave w forms the 16 columns 16 (w % 4) .. + 15 over the
//    row groups of half w / 4 (A from LDS, Q's rows from L2, two groups
//    ahead); the two halves go to LDS j-major and are added in that order;
//  * Y += X_b Z_b: wave w owns the 16-row groups w, w + 8, ... and keeps
//    their Y tiles in matrix-core registers across the workgroup's blocks.
// The blocks form NC chunks, chunk c holding blocks c, c + NC, ...; a
// workgroup takes chunks from a counter (chunk = fetched value - base) and
// writes chunk c's Y as split partial c, so the result does not depend on
// which workgroup took a chunk. A workgroup that starts late (its CU held by
// a kernel of another stream) finds the chunks taken and leaves, instead of
// delaying the whole launch. Every workgroup stops at its first fetch past
// the chunks, so a launch advances the counter by exactly NC + gridDim.x:
// the caller passes the base (the launches since the counter was zeroed
// times that).
// The loads of the next block are issued after the first product (whose Q
// loads would otherwise wait behind them) and are in flight through the
// second; the barriers order LDS only. Loads take clamped addresses with
// no branch (a branch around a load made the compiler wait for every load
// in flight); values from clamped rows or columns are replaced by zeros or
// feed only outputs that are never written. The block fills most of the
// LDS: one workgroup per CU.
// Requires n % 4 == 0 (a 4-row group of Q is whole, or lies past n where
// the staged X rows are zero) and S % 4 == 0 (a 4-column group of X is
// whole or absent).
// ---------------------------------------------------------------------------
constexpr int PF_NMAX = 512;  // rows: 32 groups of 16, 4 per wave

__device__ __forceinline__ int pf_swz(int row, int slot) { return row * 16 + (slot ^ (row & 15)); }

template <int JT, int GW>
__global__ __launch_bounds__(512) void k_power_fused(const float* __restrict__ X, const float* __restrict__ Qt,
                                                     int64_t n, int64_t S, int l, int64_t nbs, int64_t nblocks,
                                                     int nchunks, int* __restrict__ ctr, int base,
                                                     float* __restrict__ part, int* __restrict__ err) {
  constexpr int XROWS = 8 * GW * 16;
  constexpr int ZH = 16 * JT * 16;  // one half's Z_b (float4 slots)
  static_assert(XROWS <= PF_NMAX, "row groups");
  __shared__ floatx4 lds[XROWS * 16 + 2 * ZH];
  __shared__ int chunk_s;
  floatx4* Xs = lds;               // [XROWS rows i][16 slots of c]
  floatx4* Zs = lds + XROWS * 16;  // [2 halves][16 JT rows j][16 slots of c]
  const float* Xsf = reinterpret_cast<const float*>(Xs);

  const int lane = threadIdx.x & 63, w = wave_id();
  const int g = lane >> 4, f = lane & 15;
  const int ng = (int)((n + 15) >> 4);
  const int ngw = (ng - w + 7) >> 3;  // this wave's row groups: w + 8 gg, gg < ngw
  const int ct = w & 3, h = w >> 2;   // first product: column tile and row half
  const int th = (ng + 1) >> 1;
  const int t0 = h * th, t1 = min(ng, t0 + th);
  const int64_t NC = nchunks;

  // lane (g, f) loads rows 16 (w + 8 gg) + 4 g + q, columns s0 + 4 f .. + 3
  floatx4 xr[GW][4];
  auto load_block = [&](int64_t b) {
    const int64_t p = b / nbs, s = (b - p * nbs) * 64 + 4 * f;
    const bool in = s < S;
    const float* base = X + p * n * S + (in ? s : S - 4);
#pragma unroll
    for (int gg = 0; gg < GW; ++gg)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t i = min<int64_t>(16 * (w + 8 * gg) + 4 * g + q, n - 1);
        const f4u_t v = *reinterpret_cast<const f4u_t*>(base + i * S);
        xr[gg][q] = in ? floatx4{v[0], v[1], v[2], v[3]} : floatx4{0.f, 0.f, 0.f, 0.f};
      }
  };
  // Q rows 16 t + 4 g .. + 3 of column j = 16 jt + f (clamped to valid rows
  // and columns: past n they meet zero X rows, past l they feed unused Z)
  int64_t qcol[JT];
#pragma unroll
  for (int jt = 0; jt < JT; ++jt) qcol[jt] = (int64_t)min(16 * jt + f, l - 1) * n;
  auto load_q = [&](int t, floatx4* qv) {
    const int64_t i0 = min<int64_t>(16 * t + 4 * g, n - 4);
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) {
      const f4u_t v = *reinterpret_cast<const f4u_t*>(Qt + qcol[jt] + i0);
      qv[jt] = floatx4{v[0], v[1], v[2], v[3]};
    }
  };

  // A chunk number is fetched only when the previous chunk is done: fetched
  // one chunk ahead, the first workgroups to start took second chunks before
  // the last ones had started, and the launch took up to twice as long.
  for (;;) {
    // the next chunk (the previous chunk ended with a barrier after every
    // wave's last read of chunk_s)
    if (threadIdx.x == 0) chunk_s = atomicAdd(ctr, 1) - base;
    lds_barrier();
    const int chunk = __builtin_amdgcn_readfirstlane(chunk_s);
    if (chunk < 0 || chunk >= nchunks) {
      // a launch fetches exactly nchunks + gridDim.x numbers from base on; a
      // value outside that range means the counter and the host's base
      // disagree (some chunks would keep stale partials): flag it
      if ((chunk < 0 || chunk >= nchunks + (int)gridDim.x) && err != nullptr && threadIdx.x == 0)
        atomicOr(err, TUCKER_INFO_INTERNAL);
      break;
    }
    floatx4 yacc[GW][JT];
#pragma unroll
    for (int gg = 0; gg < GW; ++gg)
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) yacc[gg][jt] = floatx4{0.f, 0.f, 0.f, 0.f};

    int64_t b = chunk;
    load_block(b);
    for (; b < nblocks; b += NC) {
      // Q's first row groups of this wave's half, in flight while the block is
      // staged (issued in buffer order, as in the loop below: the wait before
      // a buffer's use counts the loads issued after it on every path). The
      // empty asm keeps these loads in the loop: hoisted, their values would
      // hold 12 JT registers through the second product.
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) __asm__ volatile("" : "+v"(qcol[jt]));
      floatx4 qa[JT], qb[JT], qc[JT];
      load_q(min(t0, ng - 1), qa);
      __builtin_amdgcn_sched_barrier(0);
      load_q(min(t0 + 1, ng - 1), qb);
      __builtin_amdgcn_sched_barrier(0);
      load_q(min(t0 + 2, ng - 1), qc);
      __builtin_amdgcn_sched_barrier(0);
      // 1. stage the block (the previous block's second product is done with the LDS)
      lds_barrier();
#pragma unroll
      for (int gg = 0; gg < GW; ++gg)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * (w + 8 * gg) + 4 * g + q;
          Xs[pf_swz(r, f)] = r < n ? xr[gg][q] : floatx4{0.f, 0.f, 0.f, 0.f};
        }
      lds_barrier();
      // 2. Z_b columns 16 ct + r (tile row r = f for the A operand), all j,
      //    over row groups t0 .. t1 - 1: k-slot g at step q of group t is row
      //    16 t + 4 g + q. Three Q buffers, each refilled right after its last
      //    use and consumed three groups later (a copy between buffers would
      //    wait for its load).
      floatx4 zacc[JT];
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) zacc[jt] = floatx4{0.f, 0.f, 0.f, 0.f};
      const int aslot = 4 * ct + (f >> 2), ael = f & 3;
      auto zstep = [&](int t, const floatx4* qv) {
        float a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * t + 4 * g + q;
          a[q] = Xsf[4 * (16 * r + (aslot ^ (r & 15))) + ael];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int jt = 0; jt < JT; ++jt) zacc[jt] = mfma_f32(a[q], qv[jt][q], zacc[jt]);
      };
      for (int t = t0; t < t1; t += 3) {
        zstep(t, qa);
        load_q(min(t + 3, ng - 1), qa);
        if (t + 1 < t1) zstep(t + 1, qb);
        load_q(min(t + 4, ng - 1), qb);
        if (t + 2 < t1) zstep(t + 2, qc);
        load_q(min(t + 5, ng - 1), qc);
      }
      // lane holds rows 4 g + e of tile jt: column c = 16 ct + 4 g + e, j = 16 jt + f
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) Zs[h * ZH + pf_swz(16 * jt + f, 4 * ct + g)] = zacc[jt];
      // 3. the next block's loads, in flight through the second product
      load_block(b + NC < nblocks ? b + NC : b);
      lds_barrier();
      // 4. Y += X_b Z_b: tile (gg, jt) row r is row 16 G' + r, k-slot g at
      //    step q is column 16 cc + 4 g + q (column chunks outermost: one
      //    chunk of Z_b is held at a time)
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        floatx4 zb[JT];
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) {
          const int o = pf_swz(16 * jt + f, 4 * cc + g);
          zb[jt] = Zs[o] + Zs[ZH + o];
        }
#pragma unroll
        for (int gg = 0; gg < GW; ++gg)
          if (gg < ngw) {
            const floatx4 a = Xs[pf_swz(16 * (w + 8 * gg) + f, 4 * cc + g)];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int jt = 0; jt < JT; ++jt) yacc[gg][jt] = mfma_f32(a[q], zb[jt][q], yacc[gg][jt]);
          }
      }
    }
    // lane holds rows 4 g + e of tile (gg, jt): i = 16 G' + 4 g + e, j = 16 jt + f
    float* dst = part + (int64_t)chunk * n * l;
#pragma unroll
    for (int gg = 0; gg < GW; ++gg)
      if (gg < ngw) {
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) {
          const int j = 16 * jt + f;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t i = 16 * (w + 8 * gg) + 4 * g + e;
            if (i < n && j < l) dst[i * l + j] = yacc[gg][jt][e];
          }
        }
      }
    lds_barrier();  // chunk_s is rewritten next
  }
}

// Qt[j n + i] = Q[i l + j] (FP32).
__global__ __launch_bounds__(256) void k_transpose_f32(const float* __restrict__ Q, int64_t n, int l,
                                                       float* __restrict__ Qt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * l) return;
  const int64_t j = e / n, i = e - j * n;
  Qt[e] = Q[i * l + j];
}

hipError_t launch_transpose_f32(const float* Q, int64_t n, int l, float* Qt, hipStream_t st) {
  const int64_t cnt = n * l;
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_f32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, Q, n, l, Qt);
  return hipGetLastError();
}

// The one-pass kernels hold a whole CU per workgroup (LDS, or every register)
// for the launch's duration. Their grids stop short of the 256 CUs so that a
// small SVD launched beside them on a side stream always finds a CU (when it
// found none, it waited for the whole power step: 2.3 ms for a 0.5 ms SVD at
// 1000^3): at most 248 chunks plus four spare workgroups, 252 CUs.
constexpr int64_t kOnePassChunks = 248;

// Chunks (split partials) of the fused power step: the fewest rounds over the
// blocks with at most kOnePassChunks chunks (one workgroup per CU), then as
// few chunks as give that many rounds. A function of the shape only, so the
// plan that sizes the partials and the launch agree. 0 when the fused kernel
// does not apply.
int power_fused_splits(const View3& v, int l, tucker_precision prec) {
  if (prec != TUCKER_FP32 || v.S < 64 || v.S % 4 != 0 || v.n % 4 != 0 || v.n > PF_NMAX || l > 48 || l < 1)
    return 0;
  constexpr int64_t kMaxGroups = kOnePassChunks;
  const int64_t nblocks = v.P * ((v.S + 63) / 64);
  const int64_t rounds = (nblocks + kMaxGroups - 1) / kMaxGroups;
  return (int)((nblocks + rounds - 1) / rounds);
}

// ---------------------------------------------------------------------------
// Both products of a power step in one pass over X on the BF16 matrix cores:
// FP32 products through the three-piece split (NP = 3) or BF16 operands
// (NP = 1), n <= PS_NMAX. The partial layout and the chunk protocol are those
// of k_power_fused:
//   part[g][i][j] = sum over the column blocks b of chunk g of
//                   sum_{c in b} X_(k)[i, c] W[c, j],
//   W[c, j] = sum_i X_(k)[i, c] Q[i, j].
// A block is 32 consecutive columns s of one p, all n rows. It crosses HBM
// once and is staged in LDS in FP32: rows of 8 float4 slots, the slot index
// XOR-ed with bits 1..3 of the row (both read patterns below then spread over
// the banks); rows past n are zero. Four waves, one per SIMD: the Y tiles of
// all rows take 256 registers of every lane, kept in the accumulation
// registers across the chunk's blocks.
//  * W_b^T = Q^T X_b: wave h takes the 32-row k-steps of its quarter of the
//    rows, all j tiles and both 16-column tiles. k slot 8 g + e is row
//    32 ks + 4 e + g; column tile t holds columns 2 mm + t, so one 8-byte LDS
//    read per row serves both tiles. Q arrives as pieces already in that k
//    order (k_q_pieces), 16 bytes per lane, two k-steps ahead. The four
//    quarters' partials meet in LDS and are added in quarter order, split
//    once and shared as B-operand pieces.
//  * Y += X_b W_b: wave w owns the 16-row tiles w, w + 4, ... (k slot 8 g + e
//    is column 8 g + e: two 16-byte LDS reads per lane and tile).
// The next block's loads are issued when the second product starts and are
// in flight through it (128 registers). Loads take clamped addresses with no
// branch; clamped values are replaced by zeros or meet zero Q pieces.
// Requires S % 4 == 0 (a 4-column group of X is whole or absent).
// ---------------------------------------------------------------------------
constexpr int PS_NMAX = 1024;

__device__ __forceinline__ int ps_slot(int r, int s) { return s ^ ((r >> 1) & 7); }

template <int NP, int JT, int QN>
__global__ __launch_bounds__(256, 1) void k_power_split(const float* __restrict__ X, const __bf16* __restrict__ Qp,
                                                        int64_t n, int64_t S, int l, int64_t nbs,
                                                        int64_t nblocks, int nchunks, int* __restrict__ ctr, int base,
                                                        float* __restrict__ part, int* __restrict__ err) {
  constexpr int NR = 32 * QN;  // staged rows
  constexpr int KW = QN / 4;   // k-steps per wave in the first product
  constexpr int UR = QN / 2;   // row tiles per wave in the second
  constexpr int QD = NP == 1 ? 2 : 1;  // register sets for Q's pieces
  static_assert(QN % 4 == 0 && NR <= PS_NMAX && JT >= 1 && JT <= 4, "shape");
  using PR = BfProducts<NP>;
  typedef float fv4 __attribute__((ext_vector_type(4)));
  typedef float fv2 __attribute__((ext_vector_type(2)));
  // the block, then the quarter partials of W^T (whose space later holds W's
  // pieces and, between chunks, the chunk number)
  __shared__ __align__(16) float lds[NR * 32 + 4 * 64 * 32];
  float* Xs = lds;
  float* Pt = lds + NR * 32;
  bf16x8* Wp = reinterpret_cast<bf16x8*>(Pt);
  int* chunk_s = reinterpret_cast<int*>(Pt);

  const int tid = threadIdx.x, lane = tid & 63, w = wave_id();
  const int mm = lane & 15, g = lane >> 4;
  const int nks = (int)((n + 31) >> 5);
  const int64_t NC = nchunks;

  // thread (lf, lr) loads rows lr + 32 q, columns s0 + 4 lf .. + 3; its LDS
  // slot in those rows is the same for every q (bits 1..3 of lr + 32 q are
  // lr's). Rows past n take row n - 1 (they meet zero Q pieces in the first
  // product and feed unwritten rows in the second), columns past S the last
  // four (their W columns are set to zero before the second product).
  const int lf = tid & 7, lr = tid >> 3, nlast = (int)n - 1;
  float* const xst = Xs + 32 * lr + 4 * ps_slot(lr, lf);
  constexpr int QH = QN / 2;  // row groups per half block
  fv4 xr[QH];
  // half hh of block b: rows lr + 32 q for q in [QH hh, QH hh + QH)
  auto load_half = [&](int64_t b, int hh) {
    const int64_t p = b / nbs, s = (b - p * nbs) * 32 + 4 * lf;
    const float* src = X + p * n * S + (s < S ? s : S - 4);
    // the row stride, the last row and the lane's row made opaque here: the
    // row offsets are then formed at the loads (hoisted out of the block loop,
    // they would hold registers through the whole loop)
    int64_t rs = S;
    int il = nlast, ir = lr + 32 * QH * hh;
    __asm__ volatile("" : "+s"(rs), "+s"(il), "+v"(ir));
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const int i = min(ir + 32 * q, il);
      // streaming (non-temporal): X is read once, and in L2 it would evict
      // Q's pieces, which every block of the CU's XCD reads again
      const f4u_t v = __builtin_nontemporal_load(reinterpret_cast<const f4u_t*>(src + (int64_t)i * rs));
      xr[q] = fv4{v[0], v[1], v[2], v[3]};
      if ((q & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  };
  // (the half's LDS base made opaque: its rows then sit within the 64 KB
  // reach of the instructions' immediate offsets, with no address per row)
  auto stage_half = [&](int hh) {
    int off = 1024 * QH * hh;
    __asm__ volatile("" : "+v"(off));
    float* const dst = xst + off;
#pragma unroll
    for (int q = 0; q < QH; ++q) *reinterpret_cast<fv4*>(dst + 1024 * q) = xr[q];
  };
  // Q pieces of k-step ks (k-steps past the rows read the zero pieces of
  // k-step nks, so the staged copies of row n - 1 there add nothing): NP JT
  // 16-byte units per lane, one per (piece,
  // j tile), consecutive for a k-step. The lane offset is rewritten opaquely
  // for every block so that the unit addresses are formed where the loads are
  // issued (hoisted out of the block loop, they would hold two registers per load).
  const bf16x8* const qp8 = reinterpret_cast<const bf16x8*>(Qp);
  int qlane = lane;
  auto qload = [&](int ks, int jt0, int jt1, bf16x8 (&qv)[JT][NP]) {
    const bf16x8* src = qp8 + (int64_t)min(ks, nks) * (NP * JT * 64) + qlane;
#pragma unroll
    for (int jt = jt0; jt < jt1; ++jt)
#pragma unroll
      for (int c = 0; c < NP; ++c) qv[jt][c] = src[(c * JT + jt) * 64];
  };
  // first product's B operand: rows 32 ks + 4 e + g, columns 2 mm and 2 mm + 1
  // (bits 1..3 of the row are those of 4 e + g)
  auto xread = [&](int ks, fv2 (&xb)[8]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = 4 * e + g;
      xb[e] = *reinterpret_cast<const fv2*>(Xs + 32 * (32 * ks + r) + 4 * ps_slot(r, mm >> 1) + 2 * (mm & 1));
    }
  };
  auto bsplit = [&](const fv2 (&xb)[8], bf16x8 (&bp)[2][NP]) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const float f[8] = {xb[0][t], xb[1][t], xb[2][t], xb[3][t], xb[4][t], xb[5][t], xb[6][t], xb[7][t]};
      bf_pieces<NP>(f, bp[t]);
    }
  };
  // second product's A operand: row 16 rt + mm, columns 8 g .. 8 g + 7 (bits
  // 1..3 of the row are those of mm)
  const float* const xal = Xs + 32 * mm;
  const int sa0 = 4 * ps_slot(mm, 2 * g), sa1 = 4 * ps_slot(mm, 2 * g + 1);
  // tile w + 4 u of this wave, read from a base that is made opaque at the
  // start of each half (u0 = 0, UR / 2), so that the half's tiles sit within
  // the reach of immediate offsets
  const float* xa0 = xal;
  const float* xa1 = xal;
  int u0 = 0;
  auto abase = [&](int ub) {
    int off = 512 * (w + 4 * ub);
    __asm__ volatile("" : "+v"(off));
    xa0 = xal + off + sa0;
    xa1 = xal + off + sa1;
    u0 = ub;
  };
  auto aread = [&](int u, fv4 (&a)[2]) {
    a[0] = *reinterpret_cast<const fv4*>(xa0 + 2048 * (u - u0));
    a[1] = *reinterpret_cast<const fv4*>(xa1 + 2048 * (u - u0));
  };
  auto asplit = [&](const fv4 (&a)[2], bf16x8 (&ap)[NP]) {
    const float f[8] = {a[0][0], a[0][1], a[0][2], a[0][3], a[1][0], a[1][1], a[1][2], a[1][3]};
    bf_pieces<NP>(f, ap);
  };
  // issue order inside a pipeline step: the step's LDS reads, then each
  // product followed by VX vector instructions (the next step's split)
  auto interleave = [&](auto nreads, auto nmfma, auto vx) {
    constexpr int NRD = decltype(nreads)::value, NMF = decltype(nmfma)::value, VX = decltype(vx)::value;
    __builtin_amdgcn_sched_group_barrier(0x100, NRD, 0);
#pragma unroll
    for (int i = 0; i < NMF; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, VX, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };

  for (;;) {
    if (threadIdx.x == 0) *chunk_s = atomicAdd(ctr, 1) - base;
    lds_barrier();
    const int chunk = __builtin_amdgcn_readfirstlane(*chunk_s);
    if (chunk < 0 || chunk >= nchunks) {
      // a launch fetches exactly nchunks + gridDim.x numbers from base on; a
      // value outside that range means the counter and the host's base disagree
      if ((chunk < 0 || chunk >= nchunks + (int)gridDim.x) && err != nullptr && threadIdx.x == 0)
        atomicOr(err, TUCKER_INFO_INTERNAL);
      break;
    }
    // the Y tiles live in the accumulation registers (empty statements that
    // require them there, here and after every block: without them the
    // allocator moves some into vector registers and spills at n near 1024)
    floatx4 yacc[UR][JT];
#pragma unroll
    for (int u = 0; u < UR; ++u)
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) {
        yacc[u][jt] = floatx4{0.f, 0.f, 0.f, 0.f};
        __asm__ volatile("" : "+a"(yacc[u][jt]));
      }

    // the chunk's first block: its first half staged here, its second half in
    // flight into the loop
    int64_t b = chunk;
    load_half(b, 0);
    stage_half(0);
    load_half(b, 1);
    for (; b < nblocks; b += NC) {
      // Q pieces of this wave's first k-step, in flight while the block is staged
      const int ks0 = w * KW;
      __asm__ volatile("" : "+v"(qlane));
      bf16x8 qv[QD][JT][NP];
      qload(ks0, 0, JT, qv[0]);
      if (QD == 2 && KW > 1) qload(ks0 + 1, 0, JT, qv[QD - 1]);
      // 1. stage the block's second half (its first half was staged during the
      //    previous block's second product; that product and the chunk
      //    number's readers are done with the LDS)
      const int64_t scol = (b - (b / nbs) * nbs) * 32;  // the block's first column within its p
      lds_barrier();
      stage_half(1);
      lds_barrier();
      // 2. W_b^T over this wave's k-steps: step kk reads k-step kk + 1 from
      //    LDS and splits it while the matrix cores take k-step kk's pieces.
      //    Q's pieces stream from L2 (all of Q for every block: with three
      //    pieces they, not their latency, bound this product): with one
      //    piece, two register sets, each refilled two steps ahead; with
      //    three, one set, refilled by pairs of j tiles as soon as a pair's
      //    products are issued (each load a step ahead; a second set would
      //    push the kernel past the register file)
      floatx4 acc1[JT][2];
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) acc1[jt][0] = acc1[jt][1] = floatx4{0.f, 0.f, 0.f, 0.f};
      fv2 xb[8];
      bf16x8 bp[2][2][NP];
      xread(ks0, xb);
      bsplit(xb, bp[0]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int kk = 0; kk < KW; ++kk) {
        const int cur = kk & 1, nxt = cur ^ 1, qs = QD == 2 ? cur : 0;
        if (kk + 1 < KW) {
          xread(ks0 + kk + 1, xb);
          bsplit(xb, bp[nxt]);
        }
#pragma unroll
        for (int j0 = 0; j0 < JT; j0 += 2) {
          const int j1 = j0 + 2 < JT ? j0 + 2 : JT;
#pragma unroll
          for (int k = 0; k < PR::N; ++k)
#pragma unroll
            for (int jt = j0; jt < j1; ++jt)
#pragma unroll
              for (int t = 0; t < 2; ++t)
                acc1[jt][t] = mfma_bf16(qv[qs][jt][PR::A[k]], bp[cur][t][PR::B[k]], acc1[jt][t]);
          if (QD == 1 && kk + 1 < KW) qload(ks0 + kk + 1, j0, j1, qv[0]);
        }
        if (QD == 2 && kk + 2 < KW) qload(ks0 + kk + 2, 0, JT, qv[qs]);
        interleave(std::integral_constant<int, 8>{}, std::integral_constant<int, PR::N * JT * 2>{},
                   std::integral_constant<int, 2>{});
      }
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) __asm__ volatile("" : "+v"(acc1[jt][0]), "+v"(acc1[jt][1]));
      // 3. quarter partials Pt[w][j][c]: lane holds j = 16 jt + 4 g + v, c = 2 mm + t
#pragma unroll
      for (int jt = 0; jt < JT; ++jt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          *reinterpret_cast<fv2*>(Pt + (w * 64 + 16 * jt + 4 * g + v) * 32 + 2 * mm) =
              fv2{acc1[jt][0][v], acc1[jt][1][v]};
      lds_barrier();
      // wave w forms j tile w: lane (mm, g) sums W^T[16 w + mm][8 g .. 8 g + 7]
      // over the quarters in order and splits it (the B operand of the second
      // product: k slot 8 g + e is column 8 g + e)
      bf16x8 wown[NP];
      if (w < JT) {
        float sum[8];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const float* src = Pt + (h * 64 + 16 * w + mm) * 32 + 8 * g;
          const fv4 a = *reinterpret_cast<const fv4*>(src), c = *reinterpret_cast<const fv4*>(src + 4);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            sum[e] = h == 0 ? a[e] : sum[e] + a[e];
            sum[4 + e] = h == 0 ? c[e] : sum[4 + e] + c[e];
          }
        }
        // columns past S (the staged copies of the last four) contribute nothing
        const int64_t cvalid = S - scol - 8 * g;
#pragma unroll
        for (int e = 0; e < 8; ++e) sum[e] = e < cvalid ? sum[e] : 0.f;
        bf_pieces<NP>(sum, wown);
      }
      lds_barrier();
      if (w < JT)
#pragma unroll
        for (int c = 0; c < NP; ++c) Wp[(w * NP + c) * 64 + lane] = wown[c];
      lds_barrier();
      bf16x8 wq[JT][NP];
#pragma unroll
      for (int jt = 0; jt < JT; ++jt)
#pragma unroll
        for (int c = 0; c < NP; ++c) wq[jt][c] = Wp[(jt * NP + c) * 64 + lane];
      // 4. Y += X_b W_b over this wave's row tiles w + 4 u (rows past n are
      //    zero or copies of row n - 1 and feed unwritten rows): step u takes
      //    tile u's pieces, splits u + 1, reads u + 2. Tiles u < UR / 2 hold
      //    the first half of the rows: once every wave is past them, the next
      //    block's first half (its loads issued here) is staged over them and
      //    its second half's loads go out for the rest of the product.
      const int64_t bn = b + NC < nblocks ? b + NC : b;
      load_half(bn, 0);
      fv4 ar[2][2];
      bf16x8 ap[2][NP];
      abase(0);
      aread(0, ar[0]);
      if (UR > 1) aread(1, ar[1]);
      asplit(ar[0], ap[0]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int cur = u & 1, nxt = cur ^ 1;
        if (u == UR / 2) {
          lds_barrier();
          stage_half(0);
          load_half(bn, 1);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (u + 2 == UR / 2) abase(UR / 2);  // the first tile of the second half is read next
        if (u + 2 < UR) aread(u + 2, ar[cur]);
        if (u + 1 < UR) asplit(ar[nxt], ap[nxt]);
#pragma unroll
        for (int k = 0; k < PR::N; ++k)
#pragma unroll
          for (int jt = 0; jt < JT; ++jt) yacc[u][jt] = mfma_bf16(ap[cur][PR::A[k]], wq[jt][PR::B[k]], yacc[u][jt]);
        interleave(std::integral_constant<int, 2>{}, std::integral_constant<int, PR::N * JT>{},
                   std::integral_constant<int, 2>{});
      }
#pragma unroll
      for (int u = 0; u < UR; ++u)
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) __asm__ volatile("" : "+a"(yacc[u][jt]));
    }
    // lane holds rows 4 g + v of tile (u, jt): i = 16 (w + 4 u) + 4 g + v,
    // j = 16 jt + mm (n and l made opaque so that the row addresses are formed
    // here, not held from the kernel's start)
    int nn = (int)n, ll = l, i0 = 16 * w + 4 * g;
    __asm__ volatile("" : "+s"(nn), "+s"(ll), "+v"(i0));
    float* drow = part + ((int64_t)chunk * nn + i0) * ll + mm;
#pragma unroll
    for (int u = 0; u < UR; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (i0 + 64 * u + v < nn)
#pragma unroll
          for (int jt = 0; jt < JT; ++jt)
            if (16 * jt + mm < ll) drow[16 * jt] = yacc[u][jt][v];
        drow += ll;
      }
      drow += 60 * (int64_t)ll;  // the wave's next tile: 64 rows on
    }
    lds_barrier();  // the chunk number is rewritten next
  }
}

// Q's pieces in the first product's k order: 16-byte unit
// ((ks NP + c) JT + jt) 64 + 16 g + mm holds piece c of Q[32 ks + 4 e + g,
// 16 jt + mm], e = 0..7 (zero past n and past l), from Qt j-major; nks is the
// k-step count plus one (the last k-step all zero).
template <int NP>
__global__ __launch_bounds__(256) void k_q_pieces(const float* __restrict__ Qt, int64_t n, int l, int JT, int nks,
                                                  bf16x8* __restrict__ Qp) {
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (u >= (int64_t)nks * JT * 64) return;
  const int lane = (int)(u & 63), mm = lane & 15, g = lane >> 4;
  const int64_t r = u >> 6;
  const int jt = (int)(r % JT), ks = (int)(r / JT);
  const int64_t j = 16 * jt + mm;
  float f[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t i = 32 * (int64_t)ks + 4 * e + g;
    f[e] = (j < l && i < n) ? Qt[j * n + i] : 0.f;
  }
  bf16x8 p[NP];
  bf_pieces<NP>(f, p);
#pragma unroll
  for (int c = 0; c < NP; ++c) Qp[(((int64_t)ks * NP + c) * JT + jt) * 64 + lane] = p[c];
}

// The split one-pass kernel's chunks: the rule of power_fused_splits over
// 32-column blocks; 0 where the kernel does not apply (precision, S % 4,
// n > PS_NMAX, l > 64).
static int power_split_chunks(const View3& v, int l, tucker_precision prec) {
  if ((prec != TUCKER_FP32 && prec != TUCKER_BF16) || v.S < 32 || v.S % 4 != 0 || v.n > PS_NMAX || l < 1 || l > 64)
    return 0;
  constexpr int64_t kMaxGroups = kOnePassChunks;
  const int64_t nblocks = v.P * ((v.S + 31) / 32);
  const int64_t rounds = (nblocks + kMaxGroups - 1) / kMaxGroups;
  return (int)((nblocks + rounds - 1) / rounds);
}
static int64_t ps_nr32(int64_t n) { return (n + 31) / 32 * 32; }
// Q's pieces follow the partials in the same buffer.
static size_t ps_qp_offset(const View3& v, int l, int G) {
  return ((size_t)G * v.n * l * sizeof(float) + 255) / 256 * 256;
}
static size_t power_split_part_bytes(const View3& v, int l, tucker_precision prec) {
  const int G = power_split_chunks(v, l, prec);
  return G == 0 ? 0 : ps_qp_offset(v, l, G) + (size_t)3 * 64 * (ps_nr32(v.n) + 32) * sizeof(__bf16);
}

// Which pass a power step takes: the split one-pass kernel where it applies
// and the step's products run on the BF16 matrix cores, with BF16 operands at
// any n and FP32 products through the split at n > 256 (below, its 32-column
// blocks leave the matrix cores idle behind Q's stream and the two split
// kernels are faster: 120^4, 3.03 against 3.14 ms per solve); else the FP32
// one-pass kernel where it applies; else the row contraction and the column
// reduction.
enum PowerPass { PP_TWO = 0, PP_FUSED_F32 = 1, PP_SPLIT = 2 };
static PowerPass power_pass(const View3& v, int l, tucker_precision prec) {
  if ((prec == TUCKER_BF16 || (prec == TUCKER_FP32 && fp32_split_products() && v.n > 256)) &&
      power_split_chunks(v, l, prec) > 0)
    return PP_SPLIT;
  if (power_fused_splits(v, l, prec) > 0 && !(fp32_split_products() && v.n <= 256)) return PP_FUSED_F32;
  return PP_TWO;
}

// The FP32 one-pass kernel forms its products with FP32 instructions; where
// the split kernel does not apply and FP32 products go through the BF16 split
// with n <= 256 (one row group per wave, blocks too small to keep the FP32
// matrix cores busy), the two split kernels are faster despite their second
// pass over X. The partial layout covers every pass (power_fused_part_bytes
// does not depend on this choice).
int power_fused_launch_splits(const View3& v, int l, tucker_precision prec) {
  switch (power_pass(v, l, prec)) {
    case PP_SPLIT: return power_split_chunks(v, l, prec);
    case PP_FUSED_F32: return power_fused_splits(v, l, prec);
    default: return 0;
  }
}

size_t power_fused_part_bytes(const View3& v, int l, tucker_precision prec) {
  return std::max((size_t)power_fused_splits(v, l, prec) * v.n * l * sizeof(float),
                  power_split_part_bytes(v, l, prec == TUCKER_FP64 ? prec : TUCKER_FP32));
}

// Grid: the chunks plus four spare workgroups (at most one per CU), which
// take the chunks of workgroups that start late; at most 252 (see
// kOnePassChunks).
static int pf_grid(int NC) { return std::min<int>(kOnePassChunks + 4, NC + 4); }

template <int JT, int GW>
static void pf_launch(const View3& v, const float* X, const float* Qt, int l, float* part, int NC, int* ctr,
                      int base, int* err, hipStream_t st) {
  const int64_t nbs = (v.S + 63) / 64;
  TK_LAUNCH((k_power_fused<JT, GW>), dim3(pf_grid(NC)), dim3(512), 0, st, X, Qt, v.n, v.S, l, nbs, v.P * nbs, NC,
            ctr, base, part, err);
}

template <int JT>
static void pf_dispatch(const View3& v, const float* X, const float* Qt, int l, float* part, int NC, int* ctr,
                        int base, int* err, hipStream_t st) {
  const int gw = (int)(((v.n + 15) / 16 + 7) / 8);  // row groups per wave
  if (gw <= 1) pf_launch<JT, 1>(v, X, Qt, l, part, NC, ctr, base, err, st);
  else if (gw <= 2) pf_launch<JT, 2>(v, X, Qt, l, part, NC, ctr, base, err, st);
  else pf_launch<JT, 4>(v, X, Qt, l, part, NC, ctr, base, err, st);
}

template <int NP, int JT, int QN>
static void ps_launch(const View3& v, const float* X, const __bf16* Qp, int l, float* part, int NC, int* ctr,
                      int base, int* err, hipStream_t st) {
  const int64_t nbs = (v.S + 31) / 32;
  TK_LAUNCH((k_power_split<NP, JT, QN>), dim3(pf_grid(NC)), dim3(256), 0, st, X, Qp, v.n, v.S, l, nbs,
            v.P * nbs, NC, ctr, base, part, err);
}

template <int NP, int JT>
static void ps_dispatch_q(const View3& v, const float* X, const __bf16* Qp, int l, float* part, int NC, int* ctr,
                          int base, int* err, hipStream_t st) {
  const int64_t nq = (v.n + 31) / 32;  // staged 32-row groups: 4, 8, 16, 24 or 32
  if (NP == 1 && nq <= 4) ps_launch<NP, JT, 4>(v, X, Qp, l, part, NC, ctr, base, err, st);
  else if (NP == 1 && nq <= 8) ps_launch<NP, JT, 8>(v, X, Qp, l, part, NC, ctr, base, err, st);
  else if (nq <= 16) ps_launch<NP, JT, 16>(v, X, Qp, l, part, NC, ctr, base, err, st);
  else if (nq <= 24) ps_launch<NP, JT, 24>(v, X, Qp, l, part, NC, ctr, base, err, st);
  else ps_launch<NP, JT, 32>(v, X, Qp, l, part, NC, ctr, base, err, st);
}

template <int NP>
static hipError_t ps_run(const View3& v, const float* X, const float* qt, int l, float* part, int NC, int* ctr,
                         int base, int* err, hipStream_t st) {
  const int JT = (l + 15) / 16, nks = (int)((v.n + 31) / 32);
  __bf16* Qp = reinterpret_cast<__bf16*>(reinterpret_cast<char*>(part) + ps_qp_offset(v, l, NC));
  const int64_t units = (int64_t)(nks + 1) * JT * 64;
  hipLaunchKernelGGL(k_q_pieces<NP>, dim3((unsigned)((units + 255) / 256)), dim3(256), 0, st, qt, v.n, l, JT,
                     nks + 1, reinterpret_cast<bf16x8*>(Qp));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double N = (double)v.P * v.n * v.S;
  TimingScope ts(KC_POWERSTEP, st, 4.0 * (N + (double)v.n * l), 4.0 * N * l, true);
  switch (JT) {
    case 1: ps_dispatch_q<NP, 1>(v, X, Qp, l, part, NC, ctr, base, err, st); break;
    case 2: ps_dispatch_q<NP, 2>(v, X, Qp, l, part, NC, ctr, base, err, st); break;
    case 3: ps_dispatch_q<NP, 3>(v, X, Qp, l, part, NC, ctr, base, err, st); break;
    default: ps_dispatch_q<NP, 4>(v, X, Qp, l, part, NC, ctr, base, err, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_power_products(tucker_precision prec, const View3& v, const void* X, const void* qt, int l,
                                 void* z, void* part, int nsplit, int* ctr, int* fused_count, int* nsplit_used,
                                 hipStream_t st, int* err) {
  const PowerPass pp = power_pass(v, l, prec);
  if (pp == PP_TWO) {
    if (z == nullptr) return hipErrorInvalidValue;  // the two-kernel path needs Z's space
    *nsplit_used = nsplit;
    hipError_t e = launch_rowcontract(prec, v, X, qt, 1, v.n, l, z, true, st);
    if (e == hipSuccess) e = launch_colreduce(prec, v, X, z, l, part, nsplit, st);
    return e;
  }
  if (pp == PP_SPLIT) {
    const int G = power_split_chunks(v, l, prec);
    *nsplit_used = G;
    const int base = (*fused_count)++ * (G + pf_grid(G));
    return prec == TUCKER_BF16
               ? ps_run<1>(v, (const float*)X, (const float*)qt, l, (float*)part, G, ctr, base, err, st)
               : ps_run<3>(v, (const float*)X, (const float*)qt, l, (float*)part, G, ctr, base, err, st);
  }
  const int G = power_fused_splits(v, l, prec);
  *nsplit_used = G;
  const double N = (double)v.P * v.n * v.S;
  TimingScope ts(KC_POWERSTEP, st, 4.0 * (N + (double)v.n * l), 4.0 * N * l, true);
  const int base = (*fused_count)++ * (G + pf_grid(G));
  switch ((l + 15) / 16) {
    case 1: pf_dispatch<1>(v, (const float*)X, (const float*)qt, l, (float*)part, G, ctr, base, err, st); break;
    case 2: pf_dispatch<2>(v, (const float*)X, (const float*)qt, l, (float*)part, G, ctr, base, err, st); break;
    default: pf_dispatch<3>(v, (const float*)X, (const float*)qt, l, (float*)part, G, ctr, base, err, st); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gaussian fill.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void fill_gaussian_body(uint64_t seed, uint32_t mode, int64_t row0, int64_t rows,
                                                       int cols, int64_t ld, int jmajor, T* __restrict__ out, int bid) {
  const int groups = (cols + 3) / 4;
  const int64_t e = (int64_t)bid * 256 + threadIdx.x;
  if (e >= rows * groups) return;
  const int g = (int)(e / rows);
  const int64_t c = e - (int64_t)g * rows;
  T v[4];
  if constexpr (sizeof(T) == 8) {
    gaussian4_f64(seed, mode, (uint64_t)(row0 + c), (uint32_t)g, v);
  } else {
    gaussian4_f32(seed, mode, (uint64_t)(row0 + c), (uint32_t)g, v);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = 4 * g + q;
    if (j < cols) out[jmajor ? (int64_t)j * ld + c : c * cols + j] = v[q];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_gaussian(uint64_t seed, uint32_t mode, int64_t row0, int64_t rows,
                                                       int cols, int64_t ld, int jmajor, T* __restrict__ out) {
  fill_gaussian_body<T>(seed, mode, row0, rows, cols, ld, jmajor, out, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Test matrices of the other kinds (section 5): uniform [-1, 1] entries, and
// Khatri-Rao products whose entry [c, j] multiplies, in increasing mode
// order, the entries [c_i, j] of one small Gaussian or uniform factor per
// other mode (c_i: c in row-major order over those modes). Factor f of
// mode k is stream 4096 + 16 k + i (i its mode).
// ---------------------------------------------------------------------------
OmegaSpec omega_spec(int kind, int d, const int64_t* cur, int k) {
  OmegaSpec sp{};
  sp.kind = kind;
  for (int i = 0; i < d; ++i) {
    if (i == k) continue;
    sp.fdim[sp.nfac] = cur[i];
    sp.ftag[sp.nfac] = 4096u + 16u * (uint32_t)k + (uint32_t)i;
    ++sp.nfac;
  }
  return sp;
}

template <typename T>
__device__ __forceinline__ void omega4(int kr_uniform, uint64_t seed, uint32_t tag, uint64_t c, uint32_t g, T v[4]) {
  if constexpr (sizeof(T) == 8) {
    if (kr_uniform) uniform4_f64(seed, tag, c, g, v);
    else gaussian4_f64(seed, tag, c, g, v);
  } else {
    if (kr_uniform) uniform4_f32(seed, tag, c, g, v);
    else gaussian4_f32(seed, tag, c, g, v);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_omega(OmegaSpec sp, uint64_t seed, uint32_t mode, int64_t row0,
                                                    int64_t rows, int cols, int64_t ld, int jmajor, T* __restrict__ out) {
  const int groups = (cols + 3) / 4;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * groups) return;
  const int g = (int)(e / rows);
  const int64_t c = e - (int64_t)g * rows;
  const uint64_t row = (uint64_t)(row0 + c);
  T v[4];
  if (sp.kind == TUCKER_OMEGA_GAUSSIAN || sp.kind == TUCKER_OMEGA_UNIFORM) {
    omega4<T>(sp.kind == TUCKER_OMEGA_UNIFORM, seed, mode, row, (uint32_t)g, v);
  } else {
    const int uni = sp.kind == TUCKER_OMEGA_KR_UNIFORM;
    uint64_t ci[TUCKER_MAX_ORDER];
    uint64_t rem = row;
    for (int f = sp.nfac - 1; f >= 0; --f) {  // the last other mode varies fastest
      ci[f] = rem % (uint64_t)sp.fdim[f];
      rem /= (uint64_t)sp.fdim[f];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = T(1);
    for (int f = 0; f < sp.nfac; ++f) {
      T fv[4];
      omega4<T>(uni, seed, sp.ftag[f], ci[f], (uint32_t)g, fv);
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] *= fv[q];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = 4 * g + q;
    if (j < cols) out[jmajor ? (int64_t)j * ld + c : c * cols + j] = v[q];
  }
}

hipError_t launch_fill_omega(const OmegaSpec& sp, tucker_precision prec, uint64_t seed, uint32_t mode, int64_t row0,
                             int64_t rows, int cols, bool jmajor, void* out, hipStream_t st) {
  if (sp.kind == TUCKER_OMEGA_GAUSSIAN) return launch_fill_gaussian(prec, seed, mode, row0, rows, cols, jmajor, out, st);
  if (sp.kind < 0 || sp.kind > TUCKER_OMEGA_KR_UNIFORM || rows <= 0 || cols <= 0) return hipErrorInvalidValue;
  TimingScope ts(KC_FILL, st, (double)rows * cols * elem_bytes(prec), 0.0);
  const int64_t work = rows * ((cols + 3) / 4);
  const unsigned blocks = (unsigned)((work + 255) / 256);
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_fill_omega<double>), dim3(blocks), dim3(256), 0, st, sp, seed, mode, row0, rows, cols, rows,
                       jmajor ? 1 : 0, (double*)out);
  else
    hipLaunchKernelGGL((k_fill_omega<float>), dim3(blocks), dim3(256), 0, st, sp, seed, mode, row0, rows, cols, rows,
                       jmajor ? 1 : 0, (float*)out);
  return hipGetLastError();
}

hipError_t launch_fill_gaussian(tucker_precision prec, uint64_t seed, uint32_t mode, int64_t row0, int64_t rows,
                                int cols, bool jmajor, void* out, hipStream_t st) {
  const int64_t work = rows * (int64_t)((cols + 3) / 4);
  if (work == 0) return hipSuccess;
  TimingScope ts(KC_FILL, st, (double)rows * cols * elem_bytes(prec), 0.0);
  const unsigned blocks = (unsigned)((work + 255) / 256);
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_fill_gaussian<double>), dim3(blocks), dim3(256), 0, st, seed, mode, row0, rows, cols, rows,
                       jmajor ? 1 : 0, (double*)out);
  else
    hipLaunchKernelGGL((k_fill_gaussian<float>), dim3(blocks), dim3(256), 0, st, seed, mode, row0, rows, cols, rows,
                       jmajor ? 1 : 0, (float*)out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Frobenius norm squared, FP64 accumulation, two fixed-order stages.
// ---------------------------------------------------------------------------
int norm2_blocks(int64_t numel) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (numel + 4095) / 4096)); }

template <typename T>
__global__ __launch_bounds__(256) void k_norm2_part(const T* __restrict__ X, int64_t numel, double* part) {
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < numel; e += (int64_t)gridDim.x * 256) {
    const double v = (double)X[e];
    s = fma(v, v, s);
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_norm2_final(const double* part, int nb, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += part[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_norm2_final(const double* part, int nb, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2_final, dim3(1), dim3(256), 0, st, part, nb, out);
  return hipGetLastError();
}

// The relative error of section 5 through the orthogonal-projection identity
// ||A - Ahat||^2 = ||A||^2 - ||G||^2 (orthonormal factors, section 2.2).
__global__ void k_info_rel_error(tucker_info* info) {
  if (threadIdx.x != 0) return;
  const double a = info->normA2, gsq = info->normG2;
  info->rel_error = a > 0.0 ? sqrt(fmax(a - gsq, 0.0) / a) : 0.0;
}

hipError_t launch_info_rel_error(tucker_info* info, hipStream_t st) {
  hipLaunchKernelGGL(k_info_rel_error, dim3(1), dim3(64), 0, st, info);
  return hipGetLastError();
}

hipError_t launch_norm2(tucker_precision prec, const void* X, int64_t numel, double* part, double* out,
                        hipStream_t st) {
  const int nb = norm2_blocks(numel);
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_norm2_part<double>), dim3(nb), dim3(256), 0, st, (const double*)X, numel, part);
  else
    hipLaunchKernelGGL((k_norm2_part<float>), dim3(nb), dim3(256), 0, st, (const float*)X, numel, part);
  hipLaunchKernelGGL(k_norm2_final, dim3(1), dim3(256), 0, st, part, nb, out);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_to_f64(const T* __restrict__ src, int64_t count, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) dst[e] = (double)src[e];
}

hipError_t launch_convert_to_f64(tucker_precision prec, const void* src, int64_t count, double* dst,
                                 hipStream_t st) {
  if (count == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((count + 255) / 256);
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_to_f64<double>), dim3(blocks), dim3(256), 0, st, (const double*)src, count, dst);
  else
    hipLaunchKernelGGL((k_to_f64<float>), dim3(blocks), dim3(256), 0, st, (const float*)src, count, dst);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_from_f64(const double* __restrict__ src, int64_t count, T* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) dst[e] = (T)src[e];
}

hipError_t launch_convert_from_f64(tucker_precision prec, const double* src, int64_t count, void* dst,
                                   hipStream_t st) {
  if (count == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((count + 255) / 256);
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_from_f64<double>), dim3(blocks), dim3(256), 0, st, src, count, (double*)dst);
  else
    hipLaunchKernelGGL((k_from_f64<float>), dim3(blocks), dim3(256), 0, st, src, count, (float*)dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched persistent launches of the product kernels (FP32 storage; one
// instantiation per column class fits every shape and address).
// ---------------------------------------------------------------------------
void cr_geometry(const View3& v, int64_t* nsteps, int64_t* spp, int* nrblocks) {
  cr_geom(TUCKER_FP32, v, nsteps, spp, nrblocks);
}
// A batch's column reduction (S > 1) runs the split kernel's body: stages of
// 32 columns, items of 128 rows per split.
void cr_split_geometry(const View3& v, int64_t* nsteps, int64_t* spp, int* nrblocks) {
  *spp = (v.S + 31) / 32;
  *nsteps = v.P * *spp;
  *nrblocks = (int)((v.n + 127) / 128);
}
int64_t cr_split_items(int64_t n, int nsplit) { return (int64_t)nsplit * ((n + 127) / 128); }
int64_t cr_cols_items(int64_t n, int nsplit) { return (int64_t)nsplit * ((n + 255) / 256); }
// A batch's row contraction (S > 1): 32-column tiles, one per wave.
int64_t rc_split_tiles(const View3& v, int64_t* tpp) {
  *tpp = (v.S + RCS_COLS - 1) / RCS_COLS;
  return v.P * *tpp;
}

__device__ __forceinline__ void b_fill(const BFill& d, int bid) {
  fill_gaussian_body<float>(d.seed, d.mode, 0, d.rows, d.cols, d.ld, 1, d.out, bid);
}
// Request-local item -> (split, row block). Workgroups take items round robin
// and are dealt to the 8 XCDs round robin, so items whose local index agrees
// mod 8 run on one XCD whatever the request's first item; with a split count
// that is a multiple of 8 the row blocks of one split share an XCD (and its L2
// copy of the split's slice of the skinny operand).
__device__ __forceinline__ void batch_split_rb(int it, int nsplit, int nrb, int* split, int* rb) {
  if (nsplit % 8 == 0) {
    const int li = it >> 3;
    *rb = li % nrb;
    *split = (li / nrb) * 8 + (it & 7);
  } else {
    *split = it / nrb;
    *rb = it % nrb;
  }
}
// FP32 products through the three-piece split (the one-request path's
// default); EDGE 2 takes any S and row address.
template <int NJ>
__device__ __forceinline__ void b_cr_split(const BCrSplit& d, int bid) {
  int split, rb;
  batch_split_rb(bid, d.nsplit, d.nrb, &split, &rb);
  cr_split_body<3, NJ, 2, false>(d.X, d.Bt, d.n, d.S, d.l, d.m, d.spp, d.nsteps, d.nsplit, 0, d.part, nullptr, split,
                                 rb);
}
template <int NJ>
__device__ __forceinline__ void b_cr_cols(const BCrCols& d, int bid) {
  int split, rb;
  batch_split_rb(bid, d.nsplit, d.nrb, &split, &rb);
  cr_cols_body<MF_F32, NJ>(d.X, d.Bt, d.P, d.n, d.l, d.nsteps, d.nsplit, d.part, split, rb);
}
__device__ __forceinline__ void b_reduce(const BReduce& d, int bid) {
  reduce_splits_body<float, double>(d.part, d.nsplit, d.nl, d.qsub, d.alpha, d.Y, bid);
}
template <int NJ>
__device__ __forceinline__ void b_rc_split(const BRcSplit& d, int bid) {
  rc_split_body<3, NJ, true>(d.X, d.W, d.n, d.S, d.lw, d.wsi, d.wsj, d.tpp, d.ntiles, d.out, d.osp, d.osj, bid);
}
template <int NJ>
__device__ __forceinline__ void b_rc_cols(const BRcCols& d, int bid) {
  rc_cols_body<MF_F32, NJ, true>(d.X, d.W, d.P, d.n, d.lw, d.wsi, d.wsj, d.out, d.osp, d.osj, bid);
}

template <int NJ>
static hipError_t batch_ttm_nj(BatchKind kind, int* hdr, const void* desc, hipStream_t st) {
#define TK_PERSIST_N(D, F, MINB, CLAIM)                                                                       \
  {                                                                                                           \
    auto kern = k_persist<D, F, MINB, CLAIM>;                                                                 \
    TK_LAUNCH(kern, dim3(resident_grid(kern)), dim3(256), 0, st, hdr, (const D*)desc);                        \
  }                                                                                                           \
  break
#define TK_PERSIST(D, F) TK_PERSIST_N(D, F, 1, false)
  switch (kind) {
    case BK_FILL: TK_PERSIST(BFill, b_fill);
    case BK_CR_SPLIT: TK_PERSIST_N(BCrSplit, b_cr_split<NJ>, 2, true);  // the split kernel's occupancy
    case BK_CR_COLS: TK_PERSIST(BCrCols, b_cr_cols<NJ>);
    case BK_REDUCE: TK_PERSIST(BReduce, b_reduce);
    // three workgroups per CU as the one-request kernel; short items: claiming
    // would cost more than it evens out
    case BK_RC_SPLIT: TK_PERSIST_N(BRcSplit, b_rc_split<NJ>, 3, false);
    case BK_RC_COLS: TK_PERSIST(BRcCols, b_rc_cols<NJ>);
    default:
      return hipErrorInvalidValue;
  }
#undef TK_PERSIST
#undef TK_PERSIST_N
  return hipGetLastError();
}

hipError_t launch_batch_ttm(BatchKind kind, int lclass, int* hdr, const void* desc, hipStream_t st) {
  switch (lclass) {
    case 16: return batch_ttm_nj<1>(kind, hdr, desc, st);
    case 32: return batch_ttm_nj<2>(kind, hdr, desc, st);
    case 48: return batch_ttm_nj<3>(kind, hdr, desc, st);
    case 64: return batch_ttm_nj<4>(kind, hdr, desc, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tk
