// Mode-k products on the in-place unfolding X_(k)[i, p*S + s] = X[p, i, s].
//
// Two shapes of contraction cover the method's three products:
//  * column reduction  part = X_(k) B         (sketch Y = X_(k) Omega_k, and
//    the second half of the power step Y = X_(k) Z): a long reduction over
//    the m_k columns, split over workgroups and summed in a fixed order;
//  * row contraction   out = X_(k)^T W        (Z = X_(k)^T Q of the power step
//    and the core step X x_k U^T): a short reduction over n_k rows per
//    column tile, written in the [P, lw, S] layout of the result tensor.
// Both run on 16x16 matrix-core tiles: v_mfma_f32_16x16x4_f32 (FP32),
// v_mfma_f64_16x16x4_f64 (FP64) or v_mfma_f32_16x16x32_bf16 (BF16 operands,
// FP32 accumulation). Two load layouts: ROWS tiles run along s inside one p
// (contiguous rows of S elements), COLS handles S == 1 where each column of
// the unfolding is a contiguous n-vector.
#include "common.hpp"
#include "internal.hpp"

namespace tk {

template <int MK>
struct MfmaTraits;
template <>
struct MfmaTraits<MF_F32> {
  using lds_t = float;
  using acc_t = floatx4;
  using part_t = float;
  static constexpr int K = 4;
  static constexpr int PAD = 1;
};
template <>
struct MfmaTraits<MF_F64> {
  using lds_t = double;
  using acc_t = doublex4;
  using part_t = double;
  static constexpr int K = 4;
  static constexpr int PAD = 1;
};
template <>
struct MfmaTraits<MF_BF16> {
  using lds_t = unsigned short;
  using acc_t = floatx4;
  using part_t = float;
  static constexpr int K = 32;
  static constexpr int PAD = 8;  // keeps 16-byte alignment of 8-element rows
};

template <int MK, typename T>
__device__ __forceinline__ typename MfmaTraits<MK>::lds_t to_lds(T v) {
  if constexpr (MK == MF_BF16) {
    return f32_to_bf16_bits((float)v);
  } else {
    return (typename MfmaTraits<MK>::lds_t)v;
  }
}

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

// One K-step of a 16x16 tile: A row `arow`, B row `brow` (both stored with
// the contraction index contiguous), at contraction offset kk.
template <int MK>
__device__ __forceinline__ typename MfmaTraits<MK>::acc_t mfma_step(const typename MfmaTraits<MK>::lds_t* arow,
                                                                   const typename MfmaTraits<MK>::lds_t* brow,
                                                                   int kk, int lane,
                                                                   typename MfmaTraits<MK>::acc_t acc) {
  if constexpr (MK == MF_F32) {
    return mfma_f32(arow[kk + (lane >> 4)], brow[kk + (lane >> 4)], acc);
  } else if constexpr (MK == MF_F64) {
    return mfma_f64(arow[kk + (lane >> 4)], brow[kk + (lane >> 4)], acc);
  } else {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(arow + kk + 8 * (lane >> 4));
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(brow + kk + 8 * (lane >> 4));
    return mfma_bf16(a, b, acc);
  }
}

// ---------------------------------------------------------------------------
// Column reduction. Workgroup = 256 threads (4 waves) owning BM = 128 rows of
// the output and a contiguous range of column tiles (TC = 32 columns each).
// Wave w owns rows [32w, 32w+32) = 2 x 16-row blocks; NJ 16-column blocks.
// ---------------------------------------------------------------------------
constexpr int CR_BM = 128;
constexpr int CR_TC = 32;

template <typename T, int MK, int NJ, bool COLS>
__global__ __launch_bounds__(256) void k_colreduce(const T* __restrict__ X, const T* __restrict__ B, int64_t P,
                                                   int64_t n, int64_t S, int l, int64_t tiles_per_p,
                                                   int64_t ntiles, int nsplit,
                                                   typename MfmaTraits<MK>::part_t* __restrict__ part) {
  using Tr = MfmaTraits<MK>;
  using LT = typename Tr::lds_t;
  constexpr int BM = CR_BM, TC = CR_TC, LP = NJ * 16, STR = TC + Tr::PAD;
  __shared__ __attribute__((aligned(16))) LT Xs[BM * STR];
  __shared__ __attribute__((aligned(16))) LT Bs[LP * STR];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * BM;
  const int split = blockIdx.x;
  const int64_t t_begin = ntiles * split / nsplit;
  const int64_t t_end = ntiles * (split + 1) / nsplit;

  typename Tr::acc_t acc[2][NJ];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NJ; ++b) acc[a][b] = typename Tr::acc_t{0, 0, 0, 0};

  for (int64_t t = t_begin; t < t_end; ++t) {
    int64_t p, s0;
    int tw;
    if constexpr (COLS) {
      p = t * TC;
      s0 = 0;
      tw = (int)min<int64_t>(TC, P - p);
    } else {
      p = t / tiles_per_p;
      s0 = (t - p * tiles_per_p) * TC;
      tw = (int)min<int64_t>(TC, S - s0);
    }
    __syncthreads();
    if constexpr (!COLS) {
      const T* xb = X + (p * n) * S + s0;
      const int c = tid & (TC - 1);
#pragma unroll 4
      for (int it = 0; it < BM / 8; ++it) {
        const int r = (tid >> 5) + it * 8;
        const int64_t i = i0 + r;
        T v = (i < n && c < tw) ? xb[i * S + c] : T(0);
        Xs[r * STR + c] = to_lds<MK>(v);
      }
      const T* bb = B + ((int64_t)p * l) * S + s0;
#pragma unroll
      for (int it = 0; it < LP / 8; ++it) {
        const int j = (tid >> 5) + it * 8;
        T v = (j < l && c < tw) ? bb[(int64_t)j * S + c] : T(0);
        Bs[j * STR + c] = to_lds<MK>(v);
      }
    } else {
      const int r = tid & (BM - 1);
      const int64_t i = i0 + r;
#pragma unroll 4
      for (int it = 0; it < TC / 2; ++it) {
        const int c = (tid >> 7) + it * 2;
        T v = (i < n && c < tw) ? X[(p + c) * n + i] : T(0);
        Xs[r * STR + c] = to_lds<MK>(v);
      }
      for (int e = tid; e < TC * LP; e += 256) {
        const int c = e / LP, j = e - (e / LP) * LP;
        T v = (j < l && c < tw) ? B[(p + c) * l + j] : T(0);
        Bs[j * STR + c] = to_lds<MK>(v);
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TC; kk += Tr::K) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) {
        const LT* arow = Xs + (wave * 32 + mi * 16 + (lane & 15)) * STR;
#pragma unroll
        for (int nj = 0; nj < NJ; ++nj) {
          const LT* brow = Bs + (nj * 16 + (lane & 15)) * STR;
          acc[mi][nj] = mfma_step<MK>(arow, brow, kk, lane, acc[mi][nj]);
        }
      }
    }
  }
  // D[row = mfma_drow(lane, v)][col = lane % 16] of each 16x16 block
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < NJ; ++nj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = i0 + wave * 32 + mi * 16 + mfma_drow<MK>(lane, v);
        const int col = nj * 16 + (lane & 15);
        if (row < n && col < l) part[((int64_t)split * n + row) * l + col] = acc[mi][nj][v];
      }
}

static int64_t cr_tiles(const View3& v, int64_t* tiles_per_p) {
  if (v.S == 1) {
    *tiles_per_p = 0;
    return (v.P + CR_TC - 1) / CR_TC;
  }
  *tiles_per_p = (v.S + CR_TC - 1) / CR_TC;
  return v.P * *tiles_per_p;
}

int colreduce_splits(const View3& v, int l) {
  (void)l;
  int64_t tpp;
  const int64_t ntiles = cr_tiles(v, &tpp);
  const int64_t rowblocks = (v.n + CR_BM - 1) / CR_BM;
  // about 1024 workgroups in flight (4 per CU), at least 2 tiles each
  int64_t ns = (1024 + rowblocks - 1) / rowblocks;
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, ntiles / 2));
  return (int)std::max<int64_t>(1, ns);
}

size_t colreduce_part_bytes(const View3& v, int l, tucker_precision prec) {
  return (size_t)colreduce_splits(v, l) * (size_t)v.n * (size_t)l * elem_bytes(prec);
}

template <typename T, int MK, int NJ>
static hipError_t cr_launch(const View3& v, const void* X, const void* B, int l, void* part, int nsplit,
                            hipStream_t st) {
  int64_t tpp;
  const int64_t ntiles = cr_tiles(v, &tpp);
  dim3 grid((unsigned)nsplit, (unsigned)((v.n + CR_BM - 1) / CR_BM));
  using PT = typename MfmaTraits<MK>::part_t;
  if (v.S == 1)
    hipLaunchKernelGGL((k_colreduce<T, MK, NJ, true>), grid, dim3(256), 0, st, (const T*)X, (const T*)B, v.P,
                       v.n, v.S, l, tpp, ntiles, nsplit, (PT*)part);
  else
    hipLaunchKernelGGL((k_colreduce<T, MK, NJ, false>), grid, dim3(256), 0, st, (const T*)X, (const T*)B, v.P,
                       v.n, v.S, l, tpp, ntiles, nsplit, (PT*)part);
  return hipGetLastError();
}

template <typename T, int MK>
static hipError_t cr_dispatch(const View3& v, const void* X, const void* B, int l, void* part, int nsplit,
                              hipStream_t st) {
  const int nj = (l + 15) / 16;
  switch (nj) {
    case 1: return cr_launch<T, MK, 1>(v, X, B, l, part, nsplit, st);
    case 2: return cr_launch<T, MK, 2>(v, X, B, l, part, nsplit, st);
    case 3: return cr_launch<T, MK, 3>(v, X, B, l, part, nsplit, st);
    case 4: return cr_launch<T, MK, 4>(v, X, B, l, part, nsplit, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_colreduce(tucker_precision prec, const View3& v, const void* X, const void* B, int l,
                            void* part, int nsplit, hipStream_t st) {
  const double N = (double)v.P * v.n * v.S, es = (double)elem_bytes(prec);
  TimingScope ts(KC_COLREDUCE, st, N * es + N / v.n * l * es, 2.0 * N * l);
  switch (prec) {
    case TUCKER_FP64: return cr_dispatch<double, MF_F64>(v, X, B, l, part, nsplit, st);
    case TUCKER_FP32: return cr_dispatch<float, MF_F32>(v, X, B, l, part, nsplit, st);
    case TUCKER_BF16: return cr_dispatch<float, MF_BF16>(v, X, B, l, part, nsplit, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of the split partials, with the -alpha Q term.
// ---------------------------------------------------------------------------
template <typename PT, typename QT>
__global__ __launch_bounds__(256) void k_reduce_splits(const PT* __restrict__ part, int nsplit, int64_t nl,
                                                       const QT* __restrict__ qsub,
                                                       const double* __restrict__ alpha, double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nl) return;
  double s = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) s += (double)part[(int64_t)sp * nl + e];
  if (qsub != nullptr) s -= (*alpha) * (double)qsub[e];
  Y[e] = s;
}

hipError_t launch_reduce_splits(tucker_precision part_prec, const void* part, int nsplit, int64_t nl,
                                const void* qsub, tucker_precision qsub_prec, const double* alpha, double* Y,
                                hipStream_t st) {
  const unsigned blocks = (unsigned)((nl + 255) / 256);
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
// Row contraction. Workgroup = 256 threads owning TC = 64 columns of the
// unfolding (wave w: columns [16w, 16w+16)) and all lw outputs per column;
// it streams the n rows in chunks of BK = 32.
// ---------------------------------------------------------------------------
constexpr int RC_TC = 64;
constexpr int RC_BK = 32;

template <typename T, int MK, int NJ, bool COLS>
__global__ __launch_bounds__(256) void k_rowcontract(const T* __restrict__ X, const T* __restrict__ W, int64_t P,
                                                     int64_t n, int64_t S, int lw, int64_t tiles_per_p,
                                                     T* __restrict__ out) {
  using Tr = MfmaTraits<MK>;
  using LT = typename Tr::lds_t;
  constexpr int TC = RC_TC, BK = RC_BK, LP = NJ * 16, STR = BK + Tr::PAD;
  __shared__ __attribute__((aligned(16))) LT Xs[TC * STR];  // [c][i]
  __shared__ __attribute__((aligned(16))) LT Ws[LP * STR];  // [j][i]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t t = blockIdx.x;
  int64_t p, s0;
  int tw;
  if constexpr (COLS) {
    p = t * TC;
    s0 = 0;
    tw = (int)min<int64_t>(TC, P - p);
  } else {
    p = t / tiles_per_p;
    s0 = (t - p * tiles_per_p) * TC;
    tw = (int)min<int64_t>(TC, S - s0);
  }

  typename Tr::acc_t acc[NJ];
#pragma unroll
  for (int b = 0; b < NJ; ++b) acc[b] = typename Tr::acc_t{0, 0, 0, 0};

  for (int64_t i0 = 0; i0 < n; i0 += BK) {
    __syncthreads();
    if constexpr (!COLS) {
      const T* xb = X + (p * n) * S + s0;
      const int c = tid & (TC - 1);
#pragma unroll
      for (int it = 0; it < BK / 4; ++it) {
        const int r = (tid >> 6) + it * 4;
        const int64_t i = i0 + r;
        T v = (i < n && c < tw) ? xb[i * S + c] : T(0);
        Xs[c * STR + r] = to_lds<MK>(v);
      }
    } else {
      const int r = tid & (BK - 1);
      const int64_t i = i0 + r;
#pragma unroll
      for (int it = 0; it < TC / 8; ++it) {
        const int c = (tid >> 5) + it * 8;
        T v = (i < n && c < tw) ? X[(p + c) * n + i] : T(0);
        Xs[c * STR + r] = to_lds<MK>(v);
      }
    }
    for (int e = tid; e < BK * LP; e += 256) {
      const int r = e / LP, j = e - (e / LP) * LP;
      const int64_t i = i0 + r;
      T v = (i < n && j < lw) ? W[i * lw + j] : T(0);
      Ws[j * STR + r] = to_lds<MK>(v);
    }
    __syncthreads();
    const LT* arow = Xs + (wave * 16 + (lane & 15)) * STR;
#pragma unroll
    for (int kk = 0; kk < BK; kk += Tr::K) {
#pragma unroll
      for (int nj = 0; nj < NJ; ++nj) {
        const LT* brow = Ws + (nj * 16 + (lane & 15)) * STR;
        acc[nj] = mfma_step<MK>(arow, brow, kk, lane, acc[nj]);
      }
    }
  }
#pragma unroll
  for (int nj = 0; nj < NJ; ++nj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = wave * 16 + mfma_drow<MK>(lane, v);
      const int j = nj * 16 + (lane & 15);
      if (c < tw && j < lw) {
        if constexpr (COLS)
          out[(p + c) * lw + j] = (T)acc[nj][v];
        else
          out[(p * lw + j) * S + s0 + c] = (T)acc[nj][v];
      }
    }
}

template <typename T, int MK, int NJ>
static hipError_t rc_launch(const View3& v, const void* X, const void* W, int lw, void* out, hipStream_t st) {
  if (v.S == 1) {
    const int64_t tiles = (v.P + RC_TC - 1) / RC_TC;
    hipLaunchKernelGGL((k_rowcontract<T, MK, NJ, true>), dim3((unsigned)tiles), dim3(256), 0, st, (const T*)X,
                       (const T*)W, v.P, v.n, v.S, lw, (int64_t)0, (T*)out);
  } else {
    const int64_t tpp = (v.S + RC_TC - 1) / RC_TC;
    hipLaunchKernelGGL((k_rowcontract<T, MK, NJ, false>), dim3((unsigned)(v.P * tpp)), dim3(256), 0, st,
                       (const T*)X, (const T*)W, v.P, v.n, v.S, lw, tpp, (T*)out);
  }
  return hipGetLastError();
}

template <typename T, int MK>
static hipError_t rc_dispatch(const View3& v, const void* X, const void* W, int lw, void* out, hipStream_t st) {
  switch ((lw + 15) / 16) {
    case 1: return rc_launch<T, MK, 1>(v, X, W, lw, out, st);
    case 2: return rc_launch<T, MK, 2>(v, X, W, lw, out, st);
    case 3: return rc_launch<T, MK, 3>(v, X, W, lw, out, st);
    case 4: return rc_launch<T, MK, 4>(v, X, W, lw, out, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rowcontract(tucker_precision mk, const View3& v, const void* X, const void* W, int lw, void* out,
                              hipStream_t st) {
  const double N = (double)v.P * v.n * v.S, es = (double)elem_bytes(mk);
  TimingScope ts(KC_ROWCONTRACT, st, N * es + N / v.n * lw * es, 2.0 * N * lw);
  switch (mk) {
    case TUCKER_FP64: return rc_dispatch<double, MF_F64>(v, X, W, lw, out, st);
    case TUCKER_FP32: return rc_dispatch<float, MF_F32>(v, X, W, lw, out, st);
    case TUCKER_BF16: return rc_dispatch<float, MF_BF16>(v, X, W, lw, out, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Gaussian fill.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_fill_gaussian(uint64_t seed, uint32_t mode, int64_t row0, int64_t rows,
                                                       int cols, int64_t S, T* __restrict__ out) {
  const int groups = (cols + 3) / 4;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * groups) return;
  const int g = (int)(e / rows);
  const int64_t c = e - (int64_t)g * rows;
  T v[4];
  if constexpr (sizeof(T) == 8) {
    gaussian4_f64(seed, mode, (uint64_t)(row0 + c), (uint32_t)g, v);
  } else {
    gaussian4_f32(seed, mode, (uint64_t)(row0 + c), (uint32_t)g, v);
  }
  const int64_t pp = c / S, ss = c - pp * S;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = 4 * g + q;
    if (j < cols) out[(pp * cols + j) * S + ss] = v[q];
  }
}

hipError_t launch_fill_gaussian(tucker_precision prec, uint64_t seed, uint32_t mode, int64_t row0, int64_t rows,
                                int cols, int64_t S, void* out, hipStream_t st) {
  const int64_t work = rows * (int64_t)((cols + 3) / 4);
  if (work == 0) return hipSuccess;
  TimingScope ts(KC_FILL, st, (double)rows * cols * elem_bytes(prec), 0.0);
  const unsigned blocks = (unsigned)((work + 255) / 256);
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_fill_gaussian<double>), dim3(blocks), dim3(256), 0, st, seed, mode, row0, rows, cols, S,
                       (double*)out);
  else
    hipLaunchKernelGGL((k_fill_gaussian<float>), dim3(blocks), dim3(256), 0, st, seed, mode, row0, rows, cols, S,
                       (float*)out);
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

}  // namespace tk
