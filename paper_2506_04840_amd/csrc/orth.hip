// [Q, Sigma] = svd(Y, 'econ') for a tall-skinny FP64 iterate Y (n x l, l <= 64),
// the factorisation the paper applies after the sketch and after every
// shifted power step (Algorithms 2 and 3).
//
// Route, all in FP64:
//   pass 1  W = Y^T Y + s I, R1 = chol(W), Q1 = Y R1^-1        (shifted CholeskyQR,
//           s = 11 (n l + l (l+1)) u ||Y||_F^2, Fukaya et al. 2020)
//   pass 2  R2 = chol(Q1^T Q1), Q2 = Q1 R2^-1
//   pass 3  R3 = chol(Q2^T Q2), Q3 = Q2 R3^-1                   (re-orthogonalisation)
//   R = R3 R2 R1 (so Y = Q3 R), one-sided Jacobi on R^T: R^T J = B with
//   orthogonal columns, hence R = J diag(|B_j|) (B/|B|)^T and the left
//   singular vectors of Y are Q3 J. Columns sorted by descending Sigma.
// A Cholesky pivot below tau * max(diag) marks the column numerically
// dependent on the previous ones: its row of R is zero and the solve puts a
// random Gaussian direction in that column, which the next pass
// orthonormalises. Those columns end with Sigma = 0.
#include "common.hpp"
#include "internal.hpp"

namespace tk {

constexpr int OR_RB = 64;      // rows per workgroup in gram / solve kernels
constexpr int OR_LS = kMaxL + 1;  // LDS row stride for l x l matrices

size_t orth_ws_bytes(int64_t n, int l) {
  const size_t nl = (size_t)n * l * sizeof(double);
  const size_t nblk = (size_t)((n + OR_RB - 1) / OR_RB);
  size_t b = 0;
  b += align_up(nl);                                  // Qa
  b += align_up(nl);                                  // Qb
  b += align_up(nblk * l * l * sizeof(double));       // gram partials
  b += align_up(3 * (size_t)kMaxL * kMaxL * sizeof(double));  // R1..R3
  b += align_up((size_t)kMaxL * kMaxL * sizeof(double));      // Racc
  b += align_up((size_t)kMaxL * kMaxL * sizeof(double));      // Wm
  b += align_up(3 * kMaxL * sizeof(int));             // deficiency flags
  b += align_up(4 * sizeof(int));                     // status
  return b;
}

OrthWs carve_orth(void* base, int64_t n, int l) {
  char* p = (char*)base;
  const size_t nl = (size_t)n * l * sizeof(double);
  const size_t nblk = (size_t)((n + OR_RB - 1) / OR_RB);
  OrthWs w;
  w.Qa = (double*)p; p += align_up(nl);
  w.Qb = (double*)p; p += align_up(nl);
  w.part = (double*)p; p += align_up(nblk * l * l * sizeof(double));
  w.R = (double*)p; p += align_up(3 * (size_t)kMaxL * kMaxL * sizeof(double));
  w.Racc = (double*)p; p += align_up((size_t)kMaxL * kMaxL * sizeof(double));
  w.Wm = (double*)p; p += align_up((size_t)kMaxL * kMaxL * sizeof(double));
  w.defic = (int*)p; p += align_up(3 * kMaxL * sizeof(int));
  w.status = (int*)p; p += align_up(4 * sizeof(int));
  return w;
}

// Gram partials of a 64-row block: part[blk][a][b] = sum_r Y[r][a] Y[r][b].
__device__ __forceinline__ void block_gram(const double (*Zs)[OR_LS], int l, double* __restrict__ part_blk) {
  for (int e = threadIdx.x; e < l * l; e += 256) {
    const int a = e / l, b = e - (e / l) * l;
    double s = 0.0;
#pragma unroll 8
    for (int r = 0; r < OR_RB; ++r) s = fma(Zs[r][a], Zs[r][b], s);
    part_blk[e] = s;
  }
}

template <typename TIN>
__global__ __launch_bounds__(256) void k_gram(const TIN* __restrict__ Y, int64_t n, int l, double* __restrict__ part) {
  __shared__ double Zs[OR_RB][OR_LS];
  const int64_t r0 = (int64_t)blockIdx.x * OR_RB;
  for (int e = threadIdx.x; e < OR_RB * l; e += 256) {
    const int r = e / l, j = e - (e / l) * l;
    Zs[r][j] = (r0 + r < n) ? (double)Y[(r0 + r) * l + j] : 0.0;
  }
  __syncthreads();
  block_gram(Zs, l, part + (size_t)blockIdx.x * l * l);
}

// Q_out = Q_in R^-1 row by row (forward substitution on the upper factor);
// deficient columns get a Gaussian direction / sqrt(n). Optionally the Gram
// partials of Q_out for the next pass.
__global__ __launch_bounds__(256) void k_solve_gram(const double* __restrict__ Qin, int64_t n, int l,
                                                    const double* __restrict__ R, const int* __restrict__ defic,
                                                    uint64_t cseed, uint32_t ctag, double* __restrict__ Qout,
                                                    double* __restrict__ part) {
  __shared__ double Rs[kMaxL][OR_LS];
  __shared__ double Zs[OR_RB][OR_LS];
  __shared__ int dfs[kMaxL];
  const int64_t r0 = (int64_t)blockIdx.x * OR_RB;
  for (int e = threadIdx.x; e < l * l; e += 256) {
    const int a = e / l, b = e - (e / l) * l;
    Rs[a][b] = R[e];
  }
  if ((int)threadIdx.x < l) dfs[threadIdx.x] = defic[threadIdx.x];
  for (int e = threadIdx.x; e < OR_RB * l; e += 256) {
    const int r = e / l, j = e - (e / l) * l;
    Zs[r][j] = (r0 + r < n) ? Qin[(r0 + r) * l + j] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < OR_RB) {
    const int r = threadIdx.x;
    const int64_t i = r0 + r;
    if (i < n) {
      const double inv_sqrt_n = 1.0 / sqrt((double)n);
      for (int j = 0; j < l; ++j) {
        double z;
        if (dfs[j]) {
          double g4[4];
          gaussian4_f64(cseed, ctag, (uint64_t)i, (uint32_t)(j >> 2), g4);
          z = g4[j & 3] * inv_sqrt_n;
        } else {
          double s = Zs[r][j];
          for (int k = 0; k < j; ++k) s = fma(-Zs[r][k], Rs[k][j], s);
          z = s / Rs[j][j];
        }
        Zs[r][j] = z;
      }
      for (int j = 0; j < l; ++j) Qout[i * l + j] = Zs[r][j];
    }
  }
  if (part == nullptr) return;
  __syncthreads();
  block_gram(Zs, l, part + (size_t)blockIdx.x * l * l);
}

// Sum the Gram partials in block order, optionally shift, then Cholesky
// W = R^T R (R upper) with deficiency detection. Racc <- R * Racc (or R).
__global__ __launch_bounds__(256) void k_chol(const double* __restrict__ part, int nblk, int64_t n, int l,
                                              int shifted, double tau, double* __restrict__ Rout,
                                              int* __restrict__ defic, double* __restrict__ Racc, int accumulate,
                                              int* __restrict__ status) {
  __shared__ double W[kMaxL][OR_LS];
  __shared__ double Rl[kMaxL][OR_LS];
  __shared__ double Ra[kMaxL][OR_LS];
  __shared__ double red[256];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int e = tid; e < l * l; e += 256) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * l * l + e];
    const int a = e / l, c = e - (e / l) * l;
    W[a][c] = s;
    if (!isfinite(s)) bad = 1;
    if (accumulate) Ra[a][c] = Racc[e];
  }
  __syncthreads();
  double tr = 0.0;
  for (int a = tid; a < l; a += 256) tr += W[a][a];
  red[tid] = tr;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double trace = red[0];
  __syncthreads();
  if (shifted) {
    const double u = 1.1102230246251565e-16;
    const double s = 11.0 * ((double)n * l + (double)l * (l + 1)) * u * trace;
    for (int a = tid; a < l; a += 256) W[a][a] += s;
  }
  __syncthreads();
  double md = 0.0;
  for (int a = tid; a < l; a += 256) md = fmax(md, W[a][a]);
  red[tid] = md;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double maxdiag = red[0];
  const bool anybad = bad != 0;
  __syncthreads();
  int ndef = 0;
  for (int j = 0; j < l; ++j) {
    const double d = W[j][j];
    const bool dep = !(d > tau * maxdiag) || anybad;
    const double rjj = dep ? 0.0 : sqrt(d);
    for (int k = tid; k < l; k += 256) {
      double v = 0.0;
      if (!dep && k >= j) v = (k == j) ? rjj : W[j][k] / rjj;
      Rl[j][k] = v;
    }
    if (tid == 0) defic[j] = dep ? 1 : 0;
    ndef += dep ? 1 : 0;
    __syncthreads();
    const int m = l - j - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int a = j + 1 + e / m, b = j + 1 + (e - (e / m) * m);
      W[a][b] = fma(-Rl[j][a], Rl[j][b], W[a][b]);
    }
    __syncthreads();
  }
  for (int e = tid; e < l * l; e += 256) {
    const int a = e / l, c = e - (e / l) * l;
    Rout[e] = Rl[a][c];
    double s;
    if (accumulate) {
      s = 0.0;
      for (int k = a; k <= c; ++k) s = fma(Rl[a][k], Ra[k][c], s);
    } else {
      s = Rl[a][c];
    }
    Racc[e] = s;
  }
  if (tid == 0) {
    if (anybad) atomicOr(&status[0], TUCKER_INFO_NONFINITE);
    if (ndef) {
      atomicOr(&status[0], TUCKER_INFO_DEFICIENT);
      atomicMax(&status[1], ndef);
    }
  }
}

// One-sided Jacobi SVD of R^T (l x l, from Racc), then sort. Writes
// Wm = left singular vectors of R (columns, descending), sigma, the shift
// update and the info log. One workgroup; 8 threads per column pair.
__global__ __launch_bounds__(256) void k_small_svd(const double* __restrict__ Racc, int l, double* __restrict__ Wm,
                                                   double* __restrict__ sigma, double* __restrict__ alpha,
                                                   tucker_info* __restrict__ info, int mode, int step,
                                                   int* __restrict__ status) {
  __shared__ double A[kMaxL][OR_LS];  // A[a][x] = column a of R^T = row a of R
  __shared__ double J[kMaxL][OR_LS];  // J[a][x] = column a of the rotation
  __shared__ double sv[kMaxL];
  __shared__ int perm[kMaxL];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const int lp = (l + 1) & ~1;
  for (int e = tid; e < kMaxL * kMaxL; e += 256) {
    const int a = e / kMaxL, x = e - (e / kMaxL) * kMaxL;
    A[a][x] = (a < l && x < l) ? Racc[a * l + x] : 0.0;
    J[a][x] = (a == x) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int pair = tid >> 3, sub = tid & 7;
  const double tol = 2.220446049250313e-16 * l;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int rnd = 0; rnd < lp - 1; ++rnd) {
      if (pair < lp / 2) {
        // circle method: player 0 fixed, players 1..lp-1 rotate
        const int x0 = pair, x1 = lp - 1 - pair;
        const int a = (x0 == 0) ? 0 : 1 + (x0 - 1 + rnd) % (lp - 1);
        const int b = (x1 == 0) ? 0 : 1 + (x1 - 1 + rnd) % (lp - 1);
        double al = 0.0, be = 0.0, ga = 0.0;
        if (a < l && b < l) {
          for (int x = sub; x < l; x += 8) {
            const double u = A[a][x], v = A[b][x];
            al = fma(u, u, al);
            be = fma(v, v, be);
            ga = fma(u, v, ga);
          }
        }
#pragma unroll
        for (int off = 1; off < 8; off <<= 1) {
          al += __shfl_xor(al, off, 8);
          be += __shfl_xor(be, off, 8);
          ga += __shfl_xor(ga, off, 8);
        }
        if (a < l && b < l && ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          for (int x = sub; x < kMaxL; x += 8) {
            const double u = A[a][x], v = A[b][x];
            A[a][x] = c * u - s * v;
            A[b][x] = s * u + c * v;
            const double ju = J[a][x], jv = J[b][x];
            J[a][x] = c * ju - s * jv;
            J[b][x] = s * ju + c * jv;
          }
          if (sub == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  for (int a = tid; a < l; a += 256) {
    double s = 0.0;
    for (int x = 0; x < l; ++x) s = fma(A[a][x], A[a][x], s);
    sv[a] = isfinite(s) ? sqrt(s) : 0.0;
  }
  __syncthreads();
  for (int a = tid; a < l; a += 256) {
    int rank = 0;
    for (int b = 0; b < l; ++b) rank += (sv[b] > sv[a] || (sv[b] == sv[a] && b < a)) ? 1 : 0;
    perm[rank] = a;
  }
  __syncthreads();
  // Wm[x][j] = J[perm[j]][x]
  for (int e = tid; e < l * l; e += 256) {
    const int x = e / l, j = e - (e / l) * l;
    Wm[e] = J[perm[j]][x];
  }
  for (int j = tid; j < l; j += 256) sigma[j] = sv[perm[j]];
  if (tid == 0) {
    const double s1 = sv[perm[0]], sl = sv[perm[l - 1]];
    double al = 0.0;
    if (alpha != nullptr) {
      al = *alpha;
      if (sl > al) al = 0.5 * (sl + al);
      *alpha = al;
    }
    if (info != nullptr && mode >= 0 && mode < TUCKER_MAX_ORDER && step >= 0 && step <= TUCKER_MAX_Q) {
      info->sigma_1[mode][step] = s1;
      info->sigma_l[mode][step] = sl;
      info->alpha[mode][step] = al;
      info->flags |= status[0];
      info->deficient[mode] = status[1];
    }
  }
}

// Q = Q3 Wm, written in the storage precision (and optionally in FP64).
template <typename T>
__global__ __launch_bounds__(256) void k_rotate(const double* __restrict__ Q3, int64_t n, int l,
                                                const double* __restrict__ Wm, T* __restrict__ qout,
                                                double* __restrict__ q64) {
  __shared__ double Ws[kMaxL][OR_LS];
  for (int e = threadIdx.x; e < l * l; e += 256) {
    const int a = e / l, b = e - (e / l) * l;
    Ws[a][b] = Wm[e];
  }
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * l) return;
  const int64_t i = e / l;
  const int j = (int)(e - i * l);
  const double* row = Q3 + i * l;
  double s = 0.0;
  for (int k = 0; k < l; ++k) s = fma(row[k], Ws[k][j], s);
  qout[e] = (T)s;
  if (q64 != nullptr) q64[e] = s;
}

__global__ void k_clear_status(int* status) {
  if (threadIdx.x < 4) status[threadIdx.x] = 0;
}

hipError_t launch_orth(int64_t n, int l, const double* Y, tucker_precision prec, void* q_out, double* q64,
                       double* sigma, double* alpha, tucker_info* info, int mode, int step, const OrthWs& ws,
                       uint64_t cseed, hipStream_t st) {
  const int nblk = (int)((n + OR_RB - 1) / OR_RB);
  TimingScope ts(KC_ORTH, st, 8.0 * n * l * 8, 3.0 * 2.0 * n * l * l);
  // pass 1 carries the shift, so its pivots sit far above tau1; passes 2 and 3
  // flag a column whose pivot is below the rounding level of an n-row Gram
  const double tau1 = 1e-15, tau = fmax(1e-14, 4.0 * (double)n * 2.220446049250313e-16);
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, st, ws.status);
  // pass 1 (shifted)
  hipLaunchKernelGGL((k_gram<double>), dim3(nblk), dim3(256), 0, st, Y, n, l, ws.part);
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), 0, st, ws.part, nblk, n, l, 1, tau1, ws.R, ws.defic, ws.Racc, 0,
                     ws.status);
  hipLaunchKernelGGL(k_solve_gram, dim3(nblk), dim3(256), 0, st, Y, n, l, ws.R, ws.defic, cseed,
                     (uint32_t)(0x100 + 16 * step + 1), ws.Qa, ws.part);
  // pass 2
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), 0, st, ws.part, nblk, n, l, 0, tau, ws.R + kMaxL * kMaxL,
                     ws.defic + kMaxL, ws.Racc, 1, ws.status);
  hipLaunchKernelGGL(k_solve_gram, dim3(nblk), dim3(256), 0, st, ws.Qa, n, l, ws.R + kMaxL * kMaxL,
                     ws.defic + kMaxL, cseed, (uint32_t)(0x100 + 16 * step + 2), ws.Qb, ws.part);
  // pass 3
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), 0, st, ws.part, nblk, n, l, 0, tau, ws.R + 2 * kMaxL * kMaxL,
                     ws.defic + 2 * kMaxL, ws.Racc, 1, ws.status);
  hipLaunchKernelGGL(k_solve_gram, dim3(nblk), dim3(256), 0, st, ws.Qb, n, l, ws.R + 2 * kMaxL * kMaxL,
                     ws.defic + 2 * kMaxL, cseed, (uint32_t)(0x100 + 16 * step + 3), ws.Qa, (double*)nullptr);
  hipLaunchKernelGGL(k_small_svd, dim3(1), dim3(256), 0, st, ws.Racc, l, ws.Wm, sigma, alpha, info, mode, step,
                     ws.status);
  const unsigned rb = (unsigned)((n * l + 255) / 256);
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_rotate<double>), dim3(rb), dim3(256), 0, st, ws.Qa, n, l, ws.Wm, (double*)q_out, q64);
  else
    hipLaunchKernelGGL((k_rotate<float>), dim3(rb), dim3(256), 0, st, ws.Qa, n, l, ws.Wm, (float*)q_out, q64);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sign rule and truncation: one workgroup per kept column.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_signfix(const T* __restrict__ Q, int64_t n, int l, int r, T* __restrict__ U) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int j = blockIdx.x;
  double best = -1.0;
  int64_t bidx = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = fabs((double)Q[i * l + j]);
    if (v > best) {
      best = v;
      bidx = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double o = bv[threadIdx.x + w];
      const int64_t oi = bi[threadIdx.x + w];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const T sgn = (Q[bi[0] * l + j] < T(0)) ? T(-1) : T(1);
  for (int64_t i = threadIdx.x; i < n; i += 256) U[i * r + j] = sgn * Q[i * l + j];
}

hipError_t launch_signfix(tucker_precision prec, const void* Q, int64_t n, int l, int r, void* U, hipStream_t st) {
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_signfix<double>), dim3(r), dim3(256), 0, st, (const double*)Q, n, l, r, (double*)U);
  else
    hipLaunchKernelGGL((k_signfix<float>), dim3(r), dim3(256), 0, st, (const float*)Q, n, l, r, (float*)U);
  return hipGetLastError();
}

__global__ void k_info_init(tucker_info* info, int32_t l0, int32_t l1, int32_t l2, int32_t l3, int32_t l4, int32_t l5,
                            int32_t l6, int32_t l7, int d, int32_t flags) {
  char* p = (char*)info;
  for (size_t e = threadIdx.x; e < sizeof(tucker_info); e += blockDim.x) p[e] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int32_t ls[8] = {l0, l1, l2, l3, l4, l5, l6, l7};
    for (int k = 0; k < TUCKER_MAX_ORDER; ++k) info->l[k] = k < d ? ls[k] : 0;
    info->flags = flags;
  }
}

hipError_t launch_info_init(tucker_info* info, const int32_t* l, int d, int32_t flags, hipStream_t st) {
  int32_t ls[8] = {0};
  for (int k = 0; k < d && k < 8; ++k) ls[k] = l[k];
  hipLaunchKernelGGL(k_info_init, dim3(1), dim3(256), 0, st, info, ls[0], ls[1], ls[2], ls[3], ls[4], ls[5], ls[6],
                     ls[7], d, flags);
  return hipGetLastError();
}

__global__ void k_set_double(double* dst, double v) {
  if (threadIdx.x == 0) *dst = v;
}

hipError_t launch_set_double(double* dst, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, dst, v);
  return hipGetLastError();
}

}  // namespace tk
