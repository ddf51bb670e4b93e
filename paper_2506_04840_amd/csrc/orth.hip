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
//
// Launches per call: gram(Y), 3 x pass(p), svd, rotate. Each pass kernel sums
// the previous pass's Gram partials in block order and factors W itself (the
// same bits in every block), solves its 64 rows and writes the Gram partial
// of its output rows for the next pass.
#include "common.hpp"
#include "internal.hpp"

namespace tk {

constexpr int OR_RB = 64;         // rows per workgroup in the gram / pass kernels
constexpr int OR_LS = kMaxL + 1;  // LDS row stride for 64-wide matrices

size_t orth_ws_bytes(int64_t n, int l) {
  const size_t nl = (size_t)n * l * sizeof(double);
  const size_t nblk = (size_t)((n + OR_RB - 1) / OR_RB);
  size_t b = 0;
  b += align_up(nl);                                          // Qa
  b += align_up(nl);                                          // Qb
  b += 2 * align_up(nblk * l * l * sizeof(double));           // gram partials, ping-pong
  b += align_up(3 * (size_t)kMaxL * kMaxL * sizeof(double));  // R1..R3
  b += align_up((size_t)kMaxL * kMaxL * sizeof(double));      // Racc
  b += align_up((size_t)kMaxL * kMaxL * sizeof(double));      // Wm
  b += align_up(3 * kMaxL * sizeof(int));                     // deficiency flags
  b += align_up(4 * sizeof(int));                             // status
  return b;
}

OrthWs carve_orth(void* base, int64_t n, int l) {
  char* p = (char*)base;
  const size_t nl = (size_t)n * l * sizeof(double);
  const size_t nblk = (size_t)((n + OR_RB - 1) / OR_RB);
  OrthWs w;
  w.Qa = (double*)p; p += align_up(nl);
  w.Qb = (double*)p; p += align_up(nl);
  w.part = (double*)p; p += 2 * align_up(nblk * l * l * sizeof(double));
  w.R = (double*)p; p += align_up(3 * (size_t)kMaxL * kMaxL * sizeof(double));
  w.Racc = (double*)p; p += align_up((size_t)kMaxL * kMaxL * sizeof(double));
  w.Wm = (double*)p; p += align_up((size_t)kMaxL * kMaxL * sizeof(double));
  w.defic = (int*)p; p += align_up(3 * kMaxL * sizeof(int));
  w.status = (int*)p; p += align_up(4 * sizeof(int));
  return w;
}

// Full-precision reciprocal and reciprocal square root: hardware estimate plus
// two Newton steps (each squares the relative error).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * fma(-x, r, 2.0);
  r = r * fma(-x, r, 2.0);
  return r;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}

// Entry (row, col) of a completion direction for a deficient column: a value
// uniform in [-1, 1) from the splitmix64 finaliser of (seed, tag, row, col).
// Any direction in general position works: the next pass orthonormalises it.
__device__ __forceinline__ double completion_entry(uint64_t seed, uint32_t tag, uint64_t row, uint32_t col) {
  uint64_t z = seed ^ (row * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)col << 32) ^ ((uint64_t)tag << 48);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(int64_t)z * 1.0842021724855044e-19;  // 2^-63
}

// Sum over the 8 lanes of an aligned octet with DPP moves (no LDS traffic):
// xor-1 and xor-2 inside each quad, then the row half-mirror joins the quads.
__device__ __forceinline__ double dpp_f64(double v, int ctrl_sel) {
  const uint64_t u = __double_as_longlong(v);
  int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
  if (ctrl_sel == 0) {
    lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
  } else if (ctrl_sel == 1) {
    lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
  } else {
    lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false);
  }
  return __longlong_as_double(((int64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double octet_sum(double v) {
  v += dpp_f64(v, 0);
  v += dpp_f64(v, 1);
  v += dpp_f64(v, 2);
  return v;
}

// Gram of 64 rows held in LDS, for the 2-D thread grid (ta, tb) = (tid/16, tid%16):
// the thread owns W[ta + 16 i][tb + 16 j], i, j < LP/16.
template <int LP>
__device__ __forceinline__ void block_gram_store(const double (*Zs)[OR_LS], int l, double* __restrict__ part_blk) {
  constexpr int NB = LP / 16;
  const int ta = threadIdx.x >> 4, tb = threadIdx.x & 15;
  double acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = 0.0;
#pragma unroll 2
  for (int r = 0; r < OR_RB; ++r) {
    double za[NB], zb[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      za[i] = Zs[r][ta + 16 * i];
      zb[i] = Zs[r][tb + 16 * i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[i][j] = fma(za[i], zb[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int a = ta + 16 * i, b = tb + 16 * j;
      if (a < l && b < l) part_blk[a * l + b] = acc[i][j];
    }
}

template <int LP>
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ Y, int64_t n, int l, double* __restrict__ part) {
  __shared__ double Zs[OR_RB][OR_LS];
  const int64_t r0 = (int64_t)blockIdx.x * OR_RB;
  for (int e = threadIdx.x; e < OR_RB * LP; e += 256) {
    const int r = e / LP, j = e % LP;
    Zs[r][j] = (r0 + r < n && j < l) ? Y[(r0 + r) * l + j] : 0.0;
  }
  __syncthreads();
  block_gram_store<LP>(Zs, l, part + (size_t)blockIdx.x * l * l);
}

// One CholeskyQR pass over 64 rows per block.
//   W = sum_b part_in[b] (+ s I when shifted); R = chol(W) with deficiency
//   flags; Qout rows = Qin rows R^-1 (deficient columns: Gaussian / sqrt(n));
//   part_out[blk] = Gram of this block's Qout rows (if part_out != nullptr).
// Block 0 also writes R and the flags for the small SVD.
template <int LP>
__global__ __launch_bounds__(256) void k_pass(const double* __restrict__ Qin, int64_t n, int l,
                                              const double* __restrict__ part_in, int nblk, int shifted, double tau,
                                              uint64_t cseed, uint32_t ctag, double* __restrict__ Qout,
                                              double* __restrict__ part_out, double* __restrict__ Rg,
                                              int* __restrict__ defic_g, int* __restrict__ status) {
  constexpr int NB = LP / 16;
  __shared__ double Rl[kMaxL][OR_LS];
  __shared__ double Zs[OR_RB][OR_LS];
  __shared__ double rrow[kMaxL];
  __shared__ double inv_diag[kMaxL];
  __shared__ int dfs[kMaxL];
  __shared__ double red[2][16];
  __shared__ double piv;
  __shared__ int bad;

  const int tid = threadIdx.x;
  const int ta = tid >> 4, tb = tid & 15;
  if (tid == 0) bad = 0;
  __syncthreads();

  // 1. W in registers: thread owns W[ta + 16 i][tb + 16 j]; the partials are
  //    summed in block order, four blocks of loads in flight at a time
  double W[NB][NB];
  double mytr = 0.0, mymax = 0.0;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) W[i][j] = 0.0;
  for (int b0 = 0; b0 < nblk; b0 += 4) {
    double v[4][NB][NB];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const int a = ta + 16 * i, b = tb + 16 * j;
          v[q][i][j] = (b0 + q < nblk && a < l && b < l) ? part_in[(size_t)(b0 + q) * l * l + a * l + b] : 0.0;
        }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) W[i][j] += v[q][i][j];
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (!isfinite(W[i][j])) bad = 1;
  __syncthreads();
  const bool anybad = bad != 0;
  // trace (diagonal owners: ta == tb, i == j)
  if (ta == tb) {
#pragma unroll
    for (int i = 0; i < NB; ++i) mytr += W[i][i];
    red[0][ta] = mytr;
  }
  __syncthreads();
  double trace = 0.0;
#pragma unroll
  for (int t = 0; t < 16; ++t) trace += red[0][t];
  const double shift = shifted ? 11.0 * ((double)n * l + (double)l * (l + 1)) * 1.1102230246251565e-16 * trace : 0.0;
  if (ta == tb) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      W[i][i] += shift;
      mymax = fmax(mymax, W[i][i]);
    }
    red[1][ta] = mymax;
  }
  __syncthreads();
  double maxdiag = 0.0;
#pragma unroll
  for (int t = 0; t < 16; ++t) maxdiag = fmax(maxdiag, red[1][t]);

  // 2. right-looking Cholesky, W = R^T R, R upper
  int ndef = 0;
  for (int k = 0; k < l; ++k) {
    const int kt = k & 15, ki = k >> 4;
    if (ta == kt && tb == kt) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (i == ki) piv = W[i][i];
    }
    __syncthreads();
    const double d = piv;
    const bool dep = !(d > tau * maxdiag) || anybad;
    const double inv = dep ? 0.0 : rsq_nr(d);  // 1 / sqrt(d)
    const double rkk = d * inv;
    if (ta == kt) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (i == ki) {
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            const int b = tb + 16 * j;
            if (b < l) {
              double v = 0.0;
              if (!dep && b >= k) v = (b == k) ? rkk : W[i][j] * inv;
              rrow[b] = v;
              Rl[k][b] = v;
            }
          }
        }
    }
    if (tid == 0) {
      dfs[k] = dep ? 1 : 0;
      inv_diag[k] = inv;
    }
    ndef += dep ? 1 : 0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int a = ta + 16 * i;
      if (a > k && a < l) {
        const double ra = rrow[a];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const int b = tb + 16 * j;
          if (b > k && b < l) W[i][j] = fma(-ra, rrow[b], W[i][j]);
        }
      }
    }
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int e = tid; e < l * l; e += 256) Rg[e] = Rl[e / l][e % l];
    if (tid < l) defic_g[tid] = dfs[tid];
    if (tid == 0) {
      if (anybad) atomicOr(&status[0], TUCKER_INFO_NONFINITE);
      if (ndef) {
        atomicOr(&status[0], TUCKER_INFO_DEFICIENT);
        atomicMax(&status[1], ndef);
      }
    }
  }

  // 3. forward substitution z R = y for the block's 64 rows: 4 lanes per row
  //    (one quad), each summing a fixed quarter of the dot product, combined
  //    by two DPP exchanges; the row lives in LDS.
  const int64_t r0 = (int64_t)blockIdx.x * OR_RB;
  for (int e = tid; e < OR_RB * LP; e += 256) {
    const int r = e / LP, j = e % LP;
    Zs[r][j] = (r0 + r < n && j < l) ? Qin[(r0 + r) * l + j] : 0.0;
  }
  __syncthreads();
  {
    const int r = tid >> 2, t = tid & 3;
    const int64_t i = r0 + r;
    const double inv_sqrt_n = rsqrt((double)n);
    for (int j = 0; j < l; ++j) {
      double z;
      if (dfs[j]) {
        z = (i < n) ? completion_entry(cseed, ctag, (uint64_t)i, (uint32_t)j) * inv_sqrt_n : 0.0;
      } else {
        double s = 0.0, s2 = 0.0;
        int k = t;
        for (; k + 4 < j; k += 8) {
          s = fma(Zs[r][k], Rl[k][j], s);
          s2 = fma(Zs[r][k + 4], Rl[k + 4][j], s2);
        }
        if (k < j) s = fma(Zs[r][k], Rl[k][j], s);
        s += s2;
        s += dpp_f64(s, 0);
        s += dpp_f64(s, 1);
        z = (Zs[r][j] - s) * inv_diag[j];
      }
      if (t == 0) Zs[r][j] = z;
    }
  }
  __syncthreads();
  for (int e = tid; e < OR_RB * l; e += 256) {
    const int r = e / l, j = e % l;
    if (r0 + r < n) Qout[(r0 + r) * l + j] = Zs[r][j];
  }
  if (part_out == nullptr) return;
  __syncthreads();
  block_gram_store<LP>(Zs, l, part_out + (size_t)blockIdx.x * l * l);
}

// C = A B for 64-wide LDS matrices (full product; the zero triangles add
// exact zeros), thread grid (ta, tb) owning C[ta + 16 i][tb + 16 j].
__device__ __forceinline__ void tile_matmul(const double (*Am)[OR_LS], const double (*Bm)[OR_LS], int l,
                                            double (&c)[4][4]) {
  const int ta = threadIdx.x >> 4, tb = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) c[i][j] = 0.0;
#pragma unroll 2
  for (int k = 0; k < l; ++k) {
    double x[4], y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      x[i] = Am[ta + 16 * i][k];
      y[i] = Bm[k][tb + 16 * i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) c[i][j] = fma(x[i], y[j], c[i][j]);
  }
}

// Rotation (c, s) that orthogonalises two columns with squared norms al, be
// and inner product ga: t = sign(d) g / (|d| + sqrt(d^2 + g^2)), d = be - al,
// g = 2 ga. The angle is computed in FP32 on power-of-two-scaled inputs (any
// angle is a valid rotation; this one annihilates ga to ~1e-7 relative), then
// c = 1 / sqrt(1 + t^2) in FP64 by Newton, so c^2 + s^2 = 1 to rounding.
__device__ __forceinline__ void jacobi_rotation(double al, double be, double ga, double& c, double& s) {
  const double d = be - al, g = 2.0 * ga;
  const int e = ilogb(fmax(fabs(d), fabs(g)));
  const float df = (float)ldexp(d, -e), gf = (float)ldexp(g, -e);
  const float h = sqrtf(fmaf(df, df, gf * gf));
  const float tf = copysignf(1.0f, df) * gf * __builtin_amdgcn_rcpf(fabsf(df) + h);
  const double t = (double)tf;
  const double x = fma(t, t, 1.0);
  double y = (double)__builtin_amdgcn_rsqf((float)x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  c = y;
  s = y * t;
}

// Racc = R3 R2 R1, one-sided Jacobi on Racc^T, sort, shift update, log.
// Writes Wm (left singular vectors of R as columns, descending) and sigma.
// RPT = rows per lane (8 lanes per column pair cover 8 * RPT >= l rows).
template <int RPT>
__global__ __launch_bounds__(256) void k_small_svd(const double* __restrict__ Rg, int l, double* __restrict__ Wm,
                                                   double* __restrict__ sigma, double* __restrict__ alpha,
                                                   tucker_info* __restrict__ info, int mode, int step,
                                                   int* __restrict__ status) {
  __shared__ double A[kMaxL][OR_LS];  // A[a][x] = column a of R^T = row a of R
  __shared__ double J[kMaxL][OR_LS];  // J[a][x] = column a of the rotation
  __shared__ unsigned char sched[kMaxL - 1][kMaxL];  // pairs per round
  __shared__ double sv[kMaxL];
  __shared__ int perm[kMaxL];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const int ta = tid >> 4, tb = tid & 15;
  const int lp = (l + 1) & ~1;
  // R = R3 R2 R1 (upper triangular): J <- R1, A <- R2; c = A J; J <- c; A <- R3; c = A J
  for (int e = tid; e < kMaxL * kMaxL; e += 256) {
    const int r = e >> 6, x = e & 63;
    J[r][x] = (r < l && x < l) ? Rg[r * l + x] : 0.0;
    A[r][x] = (r < l && x < l) ? Rg[kMaxL * kMaxL + r * l + x] : 0.0;
  }
  __syncthreads();
  double c[4][4];
  tile_matmul(A, J, l, c);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) J[ta + 16 * i][tb + 16 * j] = c[i][j];
  for (int e = tid; e < kMaxL * kMaxL; e += 256) {
    const int r = e >> 6, x = e & 63;
    A[r][x] = (r < l && x < l) ? Rg[2 * kMaxL * kMaxL + r * l + x] : 0.0;
  }
  __syncthreads();
  tile_matmul(A, J, l, c);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = ta + 16 * i, x = tb + 16 * j;
      A[r][x] = c[i][j];
      J[r][x] = (r == x) ? 1.0 : 0.0;
    }
  // round-robin schedule (circle method: player 0 fixed, the others rotate);
  // for odd l the extra player is the zero column l, which never rotates
  for (int e = tid; e < (lp - 1) * (lp / 2); e += 256) {
    const int rnd = e / (lp / 2), pr = e % (lp / 2);
    const int x0 = pr, x1 = lp - 1 - pr;
    const int pa = (x0 == 0) ? 0 : 1 + (x0 - 1 + rnd) % (lp - 1);
    const int pb = (x1 == 0) ? 0 : 1 + (x1 - 1 + rnd) % (lp - 1);
    sched[rnd][2 * pr] = (unsigned char)pa;
    sched[rnd][2 * pr + 1] = (unsigned char)pb;
  }
  __syncthreads();

  // 8 lanes per column pair, lane `sub` owns rows sub + 8 q, q < RPT (rows
  // at or beyond l are zero in A and in the first l columns of J)
  const int pair = tid >> 3, sub = tid & 7;
  const double tol = 2.220446049250313e-16 * l;
  const double tol2 = tol * tol;
  int sweeps = 0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    sweeps = sweep + 1;
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int rnd = 0; rnd < lp - 1; ++rnd) {
      if (pair < lp / 2) {
        const int pa = sched[rnd][2 * pair], pb = sched[rnd][2 * pair + 1];
        double u[RPT], v[RPT], ju[RPT], jv[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          u[q] = A[pa][sub + 8 * q];
          v[q] = A[pb][sub + 8 * q];
          ju[q] = J[pa][sub + 8 * q];
          jv[q] = J[pb][sub + 8 * q];
        }
        double al0 = 0.0, be0 = 0.0, ga0 = 0.0, al1 = 0.0, be1 = 0.0, ga1 = 0.0;
#pragma unroll
        for (int q = 0; q < RPT; q += 2) {
          al0 = fma(u[q], u[q], al0);
          be0 = fma(v[q], v[q], be0);
          ga0 = fma(u[q], v[q], ga0);
          if (q + 1 < RPT) {
            al1 = fma(u[q + 1], u[q + 1], al1);
            be1 = fma(v[q + 1], v[q + 1], be1);
            ga1 = fma(u[q + 1], v[q + 1], ga1);
          }
        }
        const double al = octet_sum(al0 + al1), be = octet_sum(be0 + be1), ga = octet_sum(ga0 + ga1);
        if (ga * ga > tol2 * al * be) {
          double cs, sn;
          jacobi_rotation(al, be, ga, cs, sn);
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            A[pa][sub + 8 * q] = cs * u[q] - sn * v[q];
            A[pb][sub + 8 * q] = sn * u[q] + cs * v[q];
            J[pa][sub + 8 * q] = cs * ju[q] - sn * jv[q];
            J[pb][sub + 8 * q] = sn * ju[q] + cs * jv[q];
          }
          if (sub == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  for (int r = tid; r < l; r += 256) {
    double s2 = 0.0;
    for (int x = 0; x < l; ++x) s2 = fma(A[r][x], A[r][x], s2);
    sv[r] = isfinite(s2) ? sqrt(s2) : 0.0;
  }
  __syncthreads();
  for (int r = tid; r < l; r += 256) {
    int rank = 0;
    for (int q = 0; q < l; ++q) rank += (sv[q] > sv[r] || (sv[q] == sv[r] && q < r)) ? 1 : 0;
    perm[rank] = r;
  }
  __syncthreads();
  for (int e = tid; e < l * l; e += 256) {
    const int x = e / l, j = e % l;
    Wm[e] = J[perm[j]][x];
  }
  if (sigma != nullptr)
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
      info->jacobi_sweeps = max(info->jacobi_sweeps, sweeps);
    }
  }
}

// Q = Q3 Wm, written in the storage precision (and optionally in FP64).
template <typename T>
__global__ __launch_bounds__(256) void k_rotate(const double* __restrict__ Q3, int64_t n, int l,
                                                const double* __restrict__ Wm, T* __restrict__ qout,
                                                T* __restrict__ qt, double* __restrict__ q64) {
  __shared__ double Ws[kMaxL][OR_LS];
  for (int e = threadIdx.x; e < l * l; e += 256) Ws[e / l][e % l] = Wm[e];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * l) return;
  const int64_t i = e / l;
  const int j = (int)(e - i * l);
  const double* row = Q3 + i * l;
  double s = 0.0;
  for (int k = 0; k < l; ++k) s = fma(row[k], Ws[k][j], s);
  if (qout != nullptr) qout[e] = (T)s;
  if (qt != nullptr) qt[(int64_t)j * n + i] = (T)s;
  if (q64 != nullptr) q64[e] = s;
}

__global__ void k_clear_status(int* status) {
  if (threadIdx.x < 4) status[threadIdx.x] = 0;
}

template <int LP>
static void orth_passes(int64_t n, int l, const double* Y, const OrthWs& ws, uint64_t cseed, int step, hipStream_t st) {
  const int nblk = (int)((n + OR_RB - 1) / OR_RB);
  const size_t pstride = align_up((size_t)nblk * l * l * sizeof(double)) / sizeof(double);
  double* p0 = ws.part;
  double* p1 = ws.part + pstride;
  // pass 1 carries the shift, so its pivots sit far above tau1; passes 2 and 3
  // flag a column whose pivot is below the rounding level of an n-row Gram
  const double tau1 = 1e-15, tau = fmax(1e-14, 4.0 * (double)n * 2.220446049250313e-16);
  const uint32_t tag = 0x100u + 16u * (uint32_t)step;
  hipLaunchKernelGGL((k_gram<LP>), dim3(nblk), dim3(256), 0, st, Y, n, l, p0);
  hipLaunchKernelGGL((k_pass<LP>), dim3(nblk), dim3(256), 0, st, Y, n, l, p0, nblk, 1, tau1, cseed, tag + 1, ws.Qa, p1,
                     ws.R, ws.defic, ws.status);
  hipLaunchKernelGGL((k_pass<LP>), dim3(nblk), dim3(256), 0, st, ws.Qa, n, l, p1, nblk, 0, tau, cseed, tag + 2, ws.Qb,
                     p0, ws.R + kMaxL * kMaxL, ws.defic + kMaxL, ws.status);
  hipLaunchKernelGGL((k_pass<LP>), dim3(nblk), dim3(256), 0, st, ws.Qb, n, l, p0, nblk, 0, tau, cseed, tag + 3, ws.Qa,
                     (double*)nullptr, ws.R + 2 * kMaxL * kMaxL, ws.defic + 2 * kMaxL, ws.status);
}

hipError_t launch_orth(int64_t n, int l, const double* Y, tucker_precision prec, void* q_out, void* qt,
                       double* q64, double* sigma, double* alpha, tucker_info* info, int mode, int step,
                       const OrthWs& ws, uint64_t cseed, hipStream_t st) {
  TimingScope ts(KC_ORTH, st, 8.0 * n * l * 8, 3.0 * 2.0 * n * l * l);
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, st, ws.status);
  switch ((l + 15) / 16) {
    case 1: orth_passes<16>(n, l, Y, ws, cseed, step, st); break;
    case 2: orth_passes<32>(n, l, Y, ws, cseed, step, st); break;
    case 3: orth_passes<48>(n, l, Y, ws, cseed, step, st); break;
    case 4: orth_passes<64>(n, l, Y, ws, cseed, step, st); break;
    default: return hipErrorInvalidValue;
  }
  switch ((l + 15) / 16) {
    case 1: hipLaunchKernelGGL((k_small_svd<2>), dim3(1), dim3(256), 0, st, ws.R, l, ws.Wm, sigma, alpha, info, mode,
                               step, ws.status); break;
    case 2: hipLaunchKernelGGL((k_small_svd<4>), dim3(1), dim3(256), 0, st, ws.R, l, ws.Wm, sigma, alpha, info, mode,
                               step, ws.status); break;
    case 3: hipLaunchKernelGGL((k_small_svd<6>), dim3(1), dim3(256), 0, st, ws.R, l, ws.Wm, sigma, alpha, info, mode,
                               step, ws.status); break;
    default: hipLaunchKernelGGL((k_small_svd<8>), dim3(1), dim3(256), 0, st, ws.R, l, ws.Wm, sigma, alpha, info, mode,
                                step, ws.status); break;
  }
  const unsigned rb = (unsigned)((n * l + 255) / 256);
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_rotate<double>), dim3(rb), dim3(256), 0, st, ws.Qa, n, l, ws.Wm, (double*)q_out,
                       (double*)qt, q64);
  else
    hipLaunchKernelGGL((k_rotate<float>), dim3(rb), dim3(256), 0, st, ws.Qa, n, l, ws.Wm, (float*)q_out, (float*)qt,
                       q64);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sign rule and truncation: one workgroup per kept column.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_signfix(const double* __restrict__ Q, int64_t n, int l, int r,
                                                 T* __restrict__ U, T* __restrict__ Ut) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int j = blockIdx.x;
  double best = -1.0;
  int64_t bidx = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = fabs(Q[i * l + j]);
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
  const double sgn = (Q[bi[0] * l + j] < 0.0) ? -1.0 : 1.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const T v = (T)(sgn * Q[i * l + j]);
    U[i * r + j] = v;
    if (Ut != nullptr) Ut[(int64_t)j * n + i] = v;
  }
}

hipError_t launch_signfix(tucker_precision prec, const double* Q, int64_t n, int l, int r, void* U, void* Ut,
                          hipStream_t st) {
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_signfix<double>), dim3(r), dim3(256), 0, st, Q, n, l, r, (double*)U, (double*)Ut);
  else
    hipLaunchKernelGGL((k_signfix<float>), dim3(r), dim3(256), 0, st, Q, n, l, r, (float*)U, (float*)Ut);
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
