// [Q, Sigma] = svd(Y, 'econ') for a tall-skinny FP64 iterate Y (n x l, l <= 64),
// the factorisation the paper applies after the sketch and after every
// shifted power step (Algorithms 2 and 3).
//
// Route, all in FP64:
//   pass 1  D = 2^floor(log4 diag(Y^T Y)) (exact column scaling),
//           W = D^-1 Y^T Y D^-1 (+ s I), R~ = chol(W), Q1 = (Y D^-1) R~^-1, R1 = R~ D.
//           For an iterate formed by FP64 products this is shifted
//           CholeskyQR on Y D^-1 (s = 11 (n l + l (l+1)) u ||Y D^-1||_F^2,
//           Fukaya et al. 2020). For FP32 / BF16 products there is no shift;
//           a pivot below their rounding level marks the column dependent.
//   pass 2  R2 = chol(Q1^T Q1), Q2 = Q1 R2^-1, skipped (R2 = I) when Q1^T Q1
//           is already I to 1e-13 (FP64) / 1e-10 (FP32, BF16): the common
//           case for a power step's iterate, whose columns arrive turned to
//           the previous step's singular vectors, nearly orthogonal
//   pass 3  R3 = chol(Q2^T Q2), Q3 = Q2 R3^-1, skipped (R3 = I) when Q2^T Q2
//           is already I to the same level, or when pass 2 was skipped
//   R = R3 R2 R1 (so Y = Q3 R); one-sided Jacobi on R^T: R^T J = B with
//   orthogonal columns, hence R = J diag(|B_j|) (B/|B|)^T and the left
//   singular vectors of Y are Q3 J. Columns sorted by descending Sigma.
// The scaling makes pass 1 insensitive to graded column norms: the iterates
// of the power steps have nearly orthogonal columns of very different
// lengths, and for them two passes suffice.
// A Cholesky pivot below tau * max(diag) marks the column numerically
// dependent on the previous ones: its row of R is zero and the solve puts a
// random direction in that column, which the next pass orthonormalises.
// Those columns end with Sigma = 0.
//
// Launches: gram(Y) [optionally first Y <- Y Wm in place], 3 x pass, svd,
// rotate. Each pass kernel sums the previous Gram partials in block order and
// factors W itself (the same bits in every block), solves its 64 rows in
// place and writes the Gram partial of its output rows for the next pass.
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
  b += 2 * align_up(nblk * l * l * sizeof(double));           // gram partials, ping-pong
  b += align_up(3 * (size_t)kMaxL * kMaxL * sizeof(double));  // R1..R3
  b += align_up((size_t)kMaxL * kMaxL * sizeof(double));      // Wm
  b += align_up(3 * kMaxL * sizeof(int));                     // deficiency flags
  b += align_up(4 * sizeof(int));                             // status
  // the second set of R, flags and status (odd steps of a power iteration)
  b += align_up(3 * (size_t)kMaxL * kMaxL * sizeof(double));
  b += align_up(3 * kMaxL * sizeof(int));
  b += align_up(4 * sizeof(int));
  // the set of the sketch's factorisation when power steps follow (its small
  // SVD only feeds the logs and runs beside the power steps), with its own Wm
  b += align_up(3 * (size_t)kMaxL * kMaxL * sizeof(double));
  b += align_up(3 * kMaxL * sizeof(int));
  b += align_up(4 * sizeof(int));
  b += align_up((size_t)kMaxL * kMaxL * sizeof(double));
  return b;
}

OrthWs carve_orth(void* base, int64_t n, int l) {
  char* p = (char*)base;
  const size_t nl = (size_t)n * l * sizeof(double);
  const size_t nblk = (size_t)((n + OR_RB - 1) / OR_RB);
  OrthWs w;
  w.Qa = (double*)p; p += align_up(nl);
  w.part = (double*)p; p += 2 * align_up(nblk * l * l * sizeof(double));
  w.R = (double*)p; p += align_up(3 * (size_t)kMaxL * kMaxL * sizeof(double));
  w.Wm = (double*)p; p += align_up((size_t)kMaxL * kMaxL * sizeof(double));
  w.defic = (int*)p; p += align_up(3 * kMaxL * sizeof(int));
  w.status = (int*)p; p += align_up(4 * sizeof(int));
  w.pf_ctr = w.status + 8;  // in the same 256-byte block, past the 4 status words
  w.R_odd = (double*)p; p += align_up(3 * (size_t)kMaxL * kMaxL * sizeof(double));
  w.defic_odd = (int*)p; p += align_up(3 * kMaxL * sizeof(int));
  w.status_odd = (int*)p; p += align_up(4 * sizeof(int));
  w.R_log = (double*)p; p += align_up(3 * (size_t)kMaxL * kMaxL * sizeof(double));
  w.defic_log = (int*)p; p += align_up(3 * kMaxL * sizeof(int));
  w.status_log = (int*)p; p += align_up(4 * sizeof(int));
  w.Wm_log = (double*)p; p += align_up((size_t)kMaxL * kMaxL * sizeof(double));
  return w;
}

OrthWs orth_log_set(const OrthWs& w) {
  OrthWs o = w;
  o.R = w.R_log;
  o.defic = w.defic_log;
  o.status = w.status_log;
  o.Wm = w.Wm_log;
  return o;
}

OrthWs orth_step_set(const OrthWs& w, int step) {
  OrthWs o = w;
  if (step > 0 && (step & 1)) {
    o.R = w.R_odd;
    o.defic = w.defic_odd;
    o.status = w.status_odd;
  }
  return o;
}

// Full-precision reciprocal square root: hardware estimate plus two Newton
// steps (each squares the relative error).
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

// 64-bit DPP move of a double (two 32-bit halves, same control).
template <int CTRL>
__device__ __forceinline__ double dpp_mov_f64(double v) {
  const uint64_t u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((int64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 8 lanes of an aligned octet (no LDS traffic): xor-1 and xor-2
// inside each quad, then the row half-mirror joins the two quads. Every lane
// of the octet ends with the same bits.
__device__ __forceinline__ double octet_sum(double v) {
  v += dpp_mov_f64<0xB1>(v);
  v += dpp_mov_f64<0x4E>(v);
  v += dpp_mov_f64<0x141>(v);
  return v;
}

// Value of lane `src` (0..3, a compile-time constant after unrolling) of each quad.
__device__ __forceinline__ double quad_bcast(double v, int src) {
  switch (src) {
    case 0: return dpp_mov_f64<0x00>(v);
    case 1: return dpp_mov_f64<0x55>(v);
    case 2: return dpp_mov_f64<0xAA>(v);
    default: return dpp_mov_f64<0xFF>(v);
  }
}

// Gram Z^T Z of the 64 rows held in Zs, on the FP64 matrix cores: the upper
// 16 x 16 tiles are dealt round robin to the 4 waves (each tile a chain of 16
// k-steps over the rows) and stored to both triangles of part_blk (l x l).
template <int LP>
__device__ __forceinline__ void block_gram_mfma(const double (*Zs)[OR_LS], int l, double* __restrict__ part_blk) {
  constexpr int NB = LP / 16, NT = NB * (NB + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mm = lane & 15, g = lane >> 4;
  for (int tile = wave; tile < NT; tile += 4) {
    int I = 0, J = tile;
    while (J >= NB - I) {
      J -= NB - I;
      ++I;
    }
    J += I;
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < OR_RB; k0 += 4) acc = mfma_f64(Zs[k0 + g][16 * I + mm], Zs[k0 + g][16 * J + mm], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 16 * I + g + 4 * v, b = 16 * J + mm;
      if (a < l && b < l) {
        part_blk[a * l + b] = acc[v];
        if (I != J) part_blk[b * l + a] = acc[v];
      }
    }
  }
}

// Gram partials of Y, 64 rows per block. With Wm, the rows are first rotated
// in place, Y <- Y Wm (the basis change that turns the iterate of a power
// step run on an unrotated basis into the iterate of the rotated one).
template <int LP>
__device__ __forceinline__ void gram_body(double* __restrict__ Y, int64_t n, int l,
                                              const double* __restrict__ Wm, double* __restrict__ part,
                                              int* __restrict__ status, int bid) {
  constexpr int NB = LP / 16;
  __shared__ double Zs[OR_RB][OR_LS];
  __shared__ double Ws[kMaxL][OR_LS];
  const int tid = threadIdx.x;
  if (bid == 0 && tid < 4) status[tid] = 0;  // flags of this factorisation
  const int64_t r0 = (int64_t)bid * OR_RB;
  for (int e = tid; e < OR_RB * LP; e += 256) {
    const int r = e / LP, j = e % LP;
    Zs[r][j] = (r0 + r < n && j < l) ? Y[(r0 + r) * l + j] : 0.0;
  }
  if (Wm != nullptr)
    for (int e = tid; e < LP * LP; e += 256) {
      const int x = e / LP, j = e % LP;
      Ws[x][j] = (x < l && j < l) ? Wm[x * l + j] : 0.0;
    }
  __syncthreads();
  if (Wm != nullptr) {
    // wave w: rows 16 w .. 16 w + 15, all column tiles
    const int lane = tid & 63, w = tid >> 6, mm = lane & 15, g = lane >> 4;
    doublex4 acc[NB];
#pragma unroll
    for (int J = 0; J < NB; ++J) acc[J] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < LP; k0 += 4) {
      const double a = Zs[16 * w + mm][k0 + g];
#pragma unroll
      for (int J = 0; J < NB; ++J) acc[J] = mfma_f64(a, Ws[k0 + g][16 * J + mm], acc[J]);
    }
    __syncthreads();
#pragma unroll
    for (int J = 0; J < NB; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v) Zs[16 * w + g + 4 * v][16 * J + mm] = acc[J][v];
    __syncthreads();
    for (int e = tid; e < OR_RB * l; e += 256) {
      const int r = e / l, j = e % l;
      if (r0 + r < n) Y[(r0 + r) * l + j] = Zs[r][j];
    }
  }
  block_gram_mfma<LP>(Zs, l, part + (size_t)bid * l * l);
}

template <int LP>
__global__ __launch_bounds__(256) void k_gram(double* __restrict__ Y, int64_t n, int l,
                                              const double* __restrict__ Wm, double* __restrict__ part,
                                              int* __restrict__ status) {
  gram_body<LP>(Y, n, l, Wm, part, status, (int)blockIdx.x);
}

// One CholeskyQR pass over 64 rows per block (role 0: pass 1, scaled and
// shifted by shift_scale * trace; role 1: pass 2 and role 2: pass 3, each of
// which leaves at once when W is I to eps3, recording that in status[3] and
// status[2]; pass 3 also leaves when pass 2 did, since then its partials
// were never written).
//   W = sum_b part_in[b] (scaled and shifted for role 0); R = chol(W) with
//   deficiency flags; Qout rows = Qin rows R^-1 (deficient columns: random
//   direction / sqrt(n)); part_out[blk] = Gram of this block's Qout rows.
// Qout may alias Qin (each block reads its rows before writing them).
// The blocks write R between them (role 0: R~ D); block 0 the flags for the
// small SVD.
// Every pass that runs also writes Q j-major in the storage precision to qt
// (when not null): the last one that runs leaves the result.
template <int LP>
__device__ __forceinline__ void pass_body(const double* Qin, int64_t n, int l, const double* __restrict__ part_in,
                                              int nblk, int role, double tau, double shift_scale, double eps3,
                                              uint64_t cseed, uint32_t ctag, double* Qout, void* __restrict__ qt,
                                              int qt_f64,
                                              double* __restrict__ part_out, double* __restrict__ Rg,
                                              int* __restrict__ defic_g, int* __restrict__ status, int bid) {
  constexpr int NB = LP / 16, MW = LP / 4;
  constexpr int PF = 8;  // Gram partials in flight per thread (one round trip per 8 blocks)
  __shared__ double Zs[OR_RB][OR_LS];
  __shared__ double Rp[LP][4][MW];     // Rp[j][t][m] = R[j][t + 4 m]
  __shared__ double pbuf[2][4][LP];    // panel rows of the trailing matrix
  __shared__ double inv_diag[LP];
  __shared__ double red[2][16];
  __shared__ int esc[LP];
  __shared__ int flag_s, far_s;

  const int tid = threadIdx.x;
  const int ta = tid >> 4, tb = tid & 15;
  if (role == 2 && status[3] != 0) {  // pass 2 left: Q1 is the result
    if (bid == 0 && tid == 0) status[2] = 1;
    return;
  }
  if (tid == 0) {
    flag_s = 0;
    far_s = 0;
  }
  // the block's rows of Qin, loaded first so that they arrive while W is
  // summed and factored: 4 lanes per row (one quad), lane t holds columns
  // t + 4 m (role 0 scales them once the exponents are known)
  const int r = tid >> 2, t = tid & 3;
  const int64_t r0 = (int64_t)bid * OR_RB;
  const int64_t row = r0 + r;
  double y[MW], z[MW];
#pragma unroll
  for (int m = 0; m < MW; ++m) {
    const int b = t + 4 * m;
    y[m] = (row < n && b < l) ? Qin[row * l + b] : 0.0;
    z[m] = 0.0;
  }

  // 1. W in registers: thread owns W[ta + 16 i][tb + 16 j]; the partials are
  //    summed in block order
  double W[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) W[i][j] = 0.0;
  for (int b0 = 0; b0 < nblk; b0 += PF) {
    double v[PF][NB][NB];
#pragma unroll
    for (int q = 0; q < PF; ++q)
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const int a = ta + 16 * i, b = tb + 16 * j;
          v[q][i][j] = (b0 + q < nblk && a < l && b < l) ? part_in[(size_t)(b0 + q) * l * l + a * l + b] : 0.0;
        }
#pragma unroll
    for (int q = 0; q < PF; ++q)
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) W[i][j] += v[q][i][j];
  }
  __syncthreads();
  bool mybad = false, myfar = false;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int a = ta + 16 * i, b = tb + 16 * j;
      mybad = mybad || !isfinite(W[i][j]);
      myfar = myfar || (a < l && b < l && !(fabs(W[i][j] - (a == b ? 1.0 : 0.0)) <= eps3));
    }
  if (mybad) flag_s = 1;
  if (myfar) far_s = 1;
  if (ta == tb) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int a = ta + 16 * i;
      int e = 0;
      if (role == 0 && a < l && W[i][i] > 0.0 && isfinite(W[i][i])) e = ilogb(W[i][i]) >> 1;
      esc[a] = e;
    }
  }
  __syncthreads();
  const bool anybad = flag_s != 0;
  // passes 2 and 3: when the input's Gram is already I to eps3, the input is
  // the result (R = I); every block sees the same sums and leaves together
  if (role >= 1 && far_s == 0 && !anybad) {
    if (bid == 0 && tid == 0) status[role == 1 ? 3 : 2] = 1;
    return;
  }
  if (role == 0) {
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) W[i][j] = ldexp(W[i][j], -(esc[ta + 16 * i] + esc[tb + 16 * j]));
  }
  if (ta == tb) {
    double tr = 0.0, mx = 0.0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      tr += W[i][i];
      mx = fmax(mx, W[i][i]);
    }
    red[0][ta] = tr;
    red[1][ta] = mx;
  }
  __syncthreads();
  double trace = 0.0, maxdiag = 0.0;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    trace += red[0][t];
    maxdiag = fmax(maxdiag, red[1][t]);
  }
  const double shift = role == 0 ? shift_scale * trace : 0.0;
  maxdiag += shift;
  if (ta == tb) {
#pragma unroll
    for (int i = 0; i < NB; ++i)
      if (ta + 16 * i < l) W[i][i] += shift;
  }

  // 2. blocked right-looking Cholesky W = R^T R (R upper), panels of 4 rows
  //    and two barriers per panel. The panel's rows of the trailing matrix are
  //    published by their owners before the panel starts (double buffered).
  //    Phase A: the lanes of wave 0 (lane c < LP owns column c) factor the
  //    4 x 4 diagonal block (the same arithmetic in every lane) and form the
  //    panel rows of R at their column, into LDS. Phase B: every thread reads
  //    the panel rows at its rows and columns and applies the rank-4 update
  //    to the entries it owns, then publishes the next panel's rows.
  constexpr int PW = 4;
  __shared__ double rpan[PW][LP];  // the panel's rows of R (zero at and left of the diagonal)
  __shared__ unsigned long long dmask_s;
  __shared__ int ndef_s;
  if (ta < PW) {
#pragma unroll
    for (int j = 0; j < NB; ++j) pbuf[0][ta][tb + 16 * j] = W[0][j];
  }
  // rows l .. LP-1 of R stay zero, so the solve can run all LP steps
  for (int e = tid; e < (LP - l) * LP; e += 256) {
    const int j = l + e / LP, b = e % LP;
    Rp[j][b & 3][b >> 2] = 0.0;
  }
  if (tid >= l && tid < LP) inv_diag[tid] = 0.0;
  __syncthreads();
  uint64_t dmask = 0;  // kept by the lanes of phase A
  int ndef = 0;
  const int npan = (l + PW - 1) / PW;
  for (int pn = 0; pn < npan; ++pn) {
    const int k0 = PW * pn;
    const double (*buf)[LP] = pbuf[pn & 1];
    if (tid < LP) {
      // phase A, column c = tid
      double dg[PW][PW], col[PW];
#pragma unroll
      for (int q = 0; q < PW; ++q) {
#pragma unroll
        for (int c = 0; c < PW; ++c) dg[q][c] = buf[q][k0 + c];
        col[q] = buf[q][tid];
      }
      // diagonal block: pivots, inverse square roots, R[k0+q][k0+c]
      double inv[PW], piv[PW], rd[PW][PW];
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        double pv = dg[q][q];
#pragma unroll
        for (int pp = 0; pp < q; ++pp) pv = fma(-rd[pp][q], rd[pp][q], pv);
        const bool dep = !(pv > tau * maxdiag) || anybad;
        inv[q] = dep ? 0.0 : rsq_nr(fmax(pv, 1e-300));
        piv[q] = pv;
        const bool cnt = dep && k0 + q < l;
        dmask |= cnt ? (1ull << (k0 + q)) : 0ull;
        ndef += cnt ? 1 : 0;
#pragma unroll
        for (int c = 0; c < PW; ++c) {
          double v = dg[q][c];
#pragma unroll
          for (int pp = 0; pp < q; ++pp) v = fma(-rd[pp][q], rd[pp][c], v);
          rd[q][c] = c > q ? v * inv[q] : 0.0;
        }
      }
      // the panel rows of R at this column: R[k][c] for c > k, the diagonal
      // R[k][k] = pv^(1/2) (0 when dependent), zero left of it
      double rc[PW];
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int k = k0 + q;
        double v = col[q];
#pragma unroll
        for (int pp = 0; pp < q; ++pp) v = fma(-rd[pp][q], rc[pp], v);
        rc[q] = v * (tid > k && tid < l ? inv[q] : 0.0);
        rpan[q][tid] = rc[q];
        Rp[k][tid & 3][tid >> 2] = tid == k ? piv[q] * inv[q] : rc[q];  // inv = 0 when dep
      }
      if (tid < PW) {
        double v = inv[0];
#pragma unroll
        for (int q = 1; q < PW; ++q) v = tid == q ? inv[q] : v;
        inv_diag[k0 + tid] = v;
      }
    }
    __syncthreads();
    // phase B: rank-4 update of the entries this thread owns
    double ra[PW][NB], rb[PW][NB];
#pragma unroll
    for (int q = 0; q < PW; ++q) {
#pragma unroll
      for (int i = 0; i < NB; ++i) ra[q][i] = rpan[q][ta + 16 * i];
#pragma unroll
      for (int j = 0; j < NB; ++j) rb[q][j] = rpan[q][tb + 16 * j];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        double w = W[i][j];
#pragma unroll
        for (int q = 0; q < PW; ++q) w = fma(-ra[q][i], rb[q][j], w);
        W[i][j] = w;
      }
    // publish the next panel's rows
    const int k1 = k0 + PW;
    if (k1 < l && (ta >> 2) == ((k1 & 15) >> 2)) {
      const int i1 = k1 >> 4, q = ta - (k1 & 15);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        double v = W[0][j];
#pragma unroll
        for (int i = 1; i < NB; ++i) v = i1 == i ? W[i][j] : v;
        pbuf[(pn + 1) & 1][q][tb + 16 * j] = v;
      }
    }
    __syncthreads();
  }
  // the deficiency record of phase A, for every thread
  if (tid == 0) {
    dmask_s = dmask;
    ndef_s = ndef;
  }
  __syncthreads();
  dmask = dmask_s;
  ndef = ndef_s;
  // R to Rg: every block holds the same R, so the blocks share the copy
  for (int e = tid + 256 * bid; e < l * l; e += 256 * nblk) {
    const int a = e / l, b = e % l;
    const double v = Rp[a][b & 3][b >> 2];
    Rg[e] = role == 0 ? ldexp(v, esc[b]) : v;
  }
  if (bid == 0) {
    if (tid < l) defic_g[tid] = (int)((dmask >> tid) & 1ull);
    if (tid == 0) {
      if (anybad) atomicOr(&status[0], TUCKER_INFO_NONFINITE);
      if (ndef) {
        atomicOr(&status[0], TUCKER_INFO_DEFICIENT);
        atomicMax(&status[1], ndef);
      }
    }
  }
  // every pass that runs writes Q in the storage precision (a later pass
  // overwrites what an earlier one wrote)
  const bool emit = true;

  // 3. solve z R = y for the block's 64 rows (the rows loaded at the start):
  //    column j's value comes from its owner lane by a quad broadcast and
  //    updates the rest right-looking.
  if (role == 0) {
#pragma unroll
    for (int m = 0; m < MW; ++m) y[m] = ldexp(y[m], -esc[t + 4 * m]);
  }
  // A deficient column j has a zero row j in R (and inv_diag[j] = 0), so its
  // value never reaches later columns: the loop carries zero for it and the
  // completion direction is put in afterwards, off the dependency chain.
  // Row j + 1 of R (this lane's columns) and its pivot inverse are read
  // from LDS while step j runs, so no step waits for its own reads.
  double rrow[MW], rnext[MW], inv_j = inv_diag[0], inv_n;
#pragma unroll
  for (int m = 0; m < MW; ++m) rrow[m] = Rp[0][t][m];
#pragma unroll
  for (int j = 0; j < LP; ++j) {
    const int jt = j & 3, jm = j >> 2;
    if (j + 1 < LP) {
      inv_n = inv_diag[j + 1];
#pragma unroll
      for (int m = (j + 1) >> 2; m < MW; ++m) rnext[m] = Rp[j + 1][t][m];
    }
    double zj = quad_bcast(y[jm] * inv_j, jt);
    z[jm] = t == jt ? zj : z[jm];
#pragma unroll
    for (int m = jm; m < MW; ++m) y[m] = fma(-zj, rrow[m], y[m]);
    if (j + 1 < LP) {
      inv_j = inv_n;
#pragma unroll
      for (int m = (j + 1) >> 2; m < MW; ++m) rrow[m] = rnext[m];
    }
  }
#pragma unroll
  for (int m = 0; m < MW; ++m) Zs[r][t + 4 * m] = z[m];
  if (dmask != 0) {
    const double inv_sqrt_n = rsqrt((double)n);
    for (int j = t; j < l; j += 4)
      if ((dmask >> j) & 1ull)
        Zs[r][j] = row < n ? completion_entry(cseed, ctag, (uint64_t)row, (uint32_t)j) * inv_sqrt_n : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < OR_RB * l; e += 256) {
    const int rr = e / l, j = e % l;
    if (r0 + rr < n) Qout[(r0 + rr) * l + j] = Zs[rr][j];
  }
  if (emit && qt != nullptr) {
    for (int e = tid; e < OR_RB * l; e += 256) {
      const int j = e / OR_RB, rr = e % OR_RB;
      if (r0 + rr < n) {
        if (qt_f64)
          ((double*)qt)[(int64_t)j * n + r0 + rr] = Zs[rr][j];
        else
          ((float*)qt)[(int64_t)j * n + r0 + rr] = (float)Zs[rr][j];
      }
    }
  }
  if (part_out != nullptr) block_gram_mfma<LP>(Zs, l, part_out + (size_t)bid * l * l);
}

template <int LP>
__global__ __launch_bounds__(256) void k_pass(const double* Qin, int64_t n, int l, const double* __restrict__ part_in,
                                              int nblk, int role, double tau, double shift_scale, double eps3,
                                              uint64_t cseed, uint32_t ctag, double* Qout, void* __restrict__ qt,
                                              int qt_f64,
                                              double* __restrict__ part_out, double* __restrict__ Rg,
                                              int* __restrict__ defic_g, int* __restrict__ status) {
  pass_body<LP>(Qin, n, l, part_in, nblk, role, tau, shift_scale, eps3, cseed, ctag, Qout, qt, qt_f64, part_out, Rg, defic_g, status, (int)blockIdx.x);
}

// C = A B for 64-wide LDS matrices (full product; the zero triangles add
// exact zeros), thread grid (ta, tb) owning C[ta + 16 i][tb + 16 j].
template <int LS>
__device__ __forceinline__ void tile_matmul(const double (*Am)[LS], const double (*Bm)[LS], int l,
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
// and inner product ga: t = tan(theta) is the root of smallest magnitude of
// g t^2 + 2 d t - g = 0 (d = be - al, g = 2 ga). It is taken in FP32 on
// power-of-two-scaled inputs, t = sign(d) g / (|d| + sqrt(d^2 + g^2)), then
// refined by one FP64 Newton step (the FP32 start is within 1e-7, so one
// step reaches FP64 accuracy); c = 1 / sqrt(1 + t^2) in FP64 by Newton and
// s = c t, so c^2 + s^2 = 1 to rounding. Needs d or g nonzero.
__device__ __forceinline__ void jacobi_rotation(double al, double be, double ga, double& c, double& s) {
  const double d = be - al, g = 2.0 * ga;
  const int e = ilogb(fmax(fabs(d), fabs(g)));
  const double ds = ldexp(d, -e), gs = ldexp(g, -e);
  const float df = (float)ds, gf = (float)gs;
  const float h = __builtin_amdgcn_sqrtf(fmaf(df, df, gf * gf));
  const float tf = copysignf(1.0f, df) * gf * __builtin_amdgcn_rcpf(fabsf(df) + h);
  double t = (double)tf;
  const double f = fma(gs, fma(t, t, -1.0), 2.0 * ds * t);
  const double fp = 2.0 * fma(gs, t, ds);
  t -= f * (double)__builtin_amdgcn_rcpf((float)fp);
  const double x = fma(t, t, 1.0);
  double y = (double)__builtin_amdgcn_rsqf((float)x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  c = y;
  s = y * t;
}

// Racc = R3 R2 R1 (R3 = I when pass 3 did not run), one-sided Jacobi on
// Racc^T, sort, shift update, log. Writes Wm (left singular vectors of R as
// columns, descending), sigma and, when vright != nullptr, the right singular
// vectors of R (l x l, columns, descending): the rotated columns of Racc^T
// scaled to unit norm (a zero column stays zero). Columns of Racc^T left
// unrotated as noise (below negl) are orthogonal to the others only to that
// level.
// Pairs follow the circle method (player 0 fixed, the others rotate); a pair
// is left alone when its columns are orthogonal to tol relative to their
// norms or when either column is below negl times the largest (rounding
// noise of the iterate, whose directions carry no information: l u for FP64
// products, about the FP32 / BF16 rounding level otherwise). The iteration
// stops once a full cycle of rounds made no rotation.
// RPT = rows per lane (8 lanes per column pair cover 8 * RPT >= l rows).
template <int RPT>
__device__ __forceinline__ void small_svd_body(const double* __restrict__ Rg, int l,
                                                   const int* __restrict__ status, double tol, double negl,
                                                   double* __restrict__ Wm, double* __restrict__ sigma,
                                                   double* __restrict__ alpha, tucker_info* __restrict__ info,
                                                   int mode, int step, int pve_r, double pve_tol, double pve_floor,
                                                   const double* __restrict__ alpha_prev, double* __restrict__ sig_hat,
                                                   int* __restrict__ stop, double* __restrict__ vright, int bid,
                                                   bool last = true) {
  // Row stride of A and J: 72 doubles, 16 banks apart from row to row (of 32,
  // or of 64), so the column pairs of a round, whose rows run consecutively
  // through the circle, read and write their eight lanes' runs of row pa (and
  // of row pb) in disjoint banks. With a stride of 65 they shared banks, and
  // bank conflicts took about half of the kernel's LDS cycles.
  constexpr int SV_LS = kMaxL + 8;
  __shared__ double A[kMaxL][SV_LS];  // A[a][x] = column a of R^T = row a of R
  __shared__ double J[kMaxL][SV_LS];  // J[a][x] = column a of the rotation
  __shared__ double sv[kMaxL];
  __shared__ int perm[kMaxL];
  __shared__ int rotf[3];
  // issue priority over waves of other kernels sharing the CU: this one is a
  // latency-bound chain that often runs beside a bandwidth-bound product
  __builtin_amdgcn_s_setprio(3);
  const int tid = threadIdx.x;
  const int ta = tid >> 4, tb = tid & 15;
  const int lp = (l + 1) & ~1;
  const bool two = status[3] == 0, three = status[2] == 0;  // pass 3 runs only after pass 2
  // J <- R1, A <- R2; c = A J (R1 when pass 2 was skipped); then (pass 3
  // ran) J <- c, A <- R3, c = A J
  for (int e = tid; e < kMaxL * kMaxL; e += 256) {
    const int r = e >> 6, x = e & 63;
    J[r][x] = (r < l && x < l) ? Rg[r * l + x] : 0.0;
    A[r][x] = (r < l && x < l) ? Rg[kMaxL * kMaxL + r * l + x] : 0.0;
  }
  __syncthreads();
  double c[4][4];
  if (two) {
    tile_matmul(A, J, l, c);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) c[i][j] = J[ta + 16 * i][tb + 16 * j];
  }
  if (three) {
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
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = ta + 16 * i, x = tb + 16 * j;
      A[r][x] = c[i][j];
      J[r][x] = (r == x) ? 1.0 : 0.0;
    }
  if (tid < 3) rotf[tid] = 0;
  __syncthreads();
  for (int r = tid; r < l; r += 256) {
    double s2 = 0.0;
    for (int x = 0; x < l; ++x) s2 = fma(A[r][x], A[r][x], s2);
    sv[r] = s2;
  }
  __syncthreads();
  double big = 0.0;
  for (int r = 0; r < l; ++r) big = fmax(big, sv[r]);
  const double nu2 = negl * negl * big;
  const double tol2 = tol * tol;

  // 8 lanes per column pair, lane `sub` owns rows sub + 8 q, q < RPT (rows
  // at or beyond l are zero in A and in the first l columns of J)
  const int pair = tid >> 3, sub = tid & 7;
  const int np = lp / 2, nr = lp - 1;
  // players at positions x0 = pair, x1 = lp - 1 - pair; a moving player's
  // column at round rnd is 1 + (x - 1 + rnd) mod nr (player 0 stays column 0)
  int posa = pair == 0 ? 0 : pair - 1, posb = lp - 2 - pair;
  const int maxr = 40 * nr;
  int rnd = 0, quiet = 0, slot = 0;  // slot = rnd mod 3
  for (;;) {
    if (rnd > 0) {
      quiet = rotf[slot == 0 ? 2 : slot - 1] ? 0 : quiet + 1;
      if (quiet >= nr || rnd >= maxr) break;
    }
    if (tid == 0) rotf[slot == 2 ? 0 : slot + 1] = 0;
    if (pair < np) {
      const int pa = pair == 0 ? 0 : 1 + posa;
      const int pb = 1 + posb;
      double u[RPT], v[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        u[q] = A[pa][sub + 8 * q];
        v[q] = A[pb][sub + 8 * q];
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
      const bool rot = ga * ga > tol2 * al * be && fmin(al, be) > nu2;
      if (rot) {  // the same decision in all 8 lanes of the pair
        // J's columns only for a pair that turns (the rounds are bound by LDS
        // traffic); their reads go out before the rotation is formed
        double ju[RPT], jv[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          ju[q] = J[pa][sub + 8 * q];
          jv[q] = J[pb][sub + 8 * q];
        }
        double cs, sn;
        jacobi_rotation(al, be, ga, cs, sn);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          A[pa][sub + 8 * q] = cs * u[q] - sn * v[q];
          A[pb][sub + 8 * q] = sn * u[q] + cs * v[q];
          J[pa][sub + 8 * q] = cs * ju[q] - sn * jv[q];
          J[pb][sub + 8 * q] = sn * ju[q] + cs * jv[q];
        }
        if (sub == 0) rotf[slot] = 1;
      }
    }
    posa = posa + 1 == nr ? 0 : posa + 1;
    posb = posb + 1 == nr ? 0 : posb + 1;
    slot = slot == 2 ? 0 : slot + 1;
    ++rnd;
    __syncthreads();
  }
  const int sweeps = (rnd + nr - 1) / nr;
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
    if (vright != nullptr) {
      const double nv = sv[perm[j]];
      vright[e] = nv > 0.0 ? A[perm[j]][x] / nv : 0.0;
    }
  }
  if (sigma != nullptr)
    for (int j = tid; j < l; j += 256) sigma[j] = sv[perm[j]];
  if (tid == 0) {
    const double s1 = sv[perm[0]], sl = sv[perm[l - 1]];
    // per-vector-error test (Algorithm 4): before the shift update
    bool halt = false;
    if (pve_tol >= 0.0) {
      if (step == 0) {
        for (int i = 0; i < l; ++i) sig_hat[i] = 0.0;
        *stop = 0;
      } else {
        const double ap = alpha_prev != nullptr ? *alpha_prev : 0.0;
        double mx = 0.0;
        for (int i = 0; i < pve_r; ++i) mx = fmax(mx, fabs(sv[perm[i]] + ap - sig_hat[i]));
        halt = mx <= fmax(pve_tol * (sv[perm[min(pve_r, l - 1)]] + ap), pve_floor * (sv[perm[0]] + ap));
        *stop = halt ? 1 : 0;
        if (!halt)
          for (int i = 0; i < l; ++i) sig_hat[i] = sv[perm[i]] + ap;
      }
    }
    double al = 0.0;
    if (alpha != nullptr) {
      al = *alpha;
      if (sl > al && !halt) al = 0.5 * (sl + al);
      *alpha = al;
    }
    if (info != nullptr && mode >= 0 && mode < TUCKER_MAX_ORDER && step >= 0 && step <= TUCKER_MAX_Q) {
      info->sigma_1[mode][step] = s1;
      info->sigma_l[mode][step] = sl;
      info->alpha[mode][step] = al;
      atomicOr(&info->flags, status[0]);  // modes of a T-HOSVD may run concurrently
      if (last) info->deficient[mode] = status[1];
      // atomic: the sketch's SVD of a mode may run beside that mode's later ones
      if (status[0] & TUCKER_INFO_DEFICIENT) atomicOr(&info->deficient_steps[mode], 1 << step);
      atomicMax(&info->jacobi_sweeps, sweeps);
    }
  }
}

template <int RPT>
__global__ __launch_bounds__(256) void k_small_svd(const double* __restrict__ Rg, int l,
                                                   const int* __restrict__ status, double tol, double negl,
                                                   double* __restrict__ Wm, double* __restrict__ sigma,
                                                   double* __restrict__ alpha, tucker_info* __restrict__ info,
                                                   int mode, int step, int pve_r, double pve_tol, double pve_floor,
                                                   const double* __restrict__ alpha_prev, double* __restrict__ sig_hat,
                                                   int* __restrict__ stop, double* __restrict__ vright, int last) {
  small_svd_body<RPT>(Rg, l, status, tol, negl, Wm, sigma, alpha, info, mode, step, pve_r, pve_tol, pve_floor,
                      alpha_prev, sig_hat, stop, vright, (int)blockIdx.x, last != 0);
}

// Q = Q3 Wm, written in the storage precision (and optionally in FP64).
template <typename T>
__device__ __forceinline__ void rotate_body(const double* __restrict__ Q3, int64_t n, int l,
                                                const double* __restrict__ Wm, T* __restrict__ qout,
                                                T* __restrict__ qt, double* __restrict__ q64, int bid) {
  __shared__ double Ws[kMaxL][OR_LS];
  for (int e = threadIdx.x; e < l * l; e += 256) Ws[e / l][e % l] = Wm[e];
  __syncthreads();
  const int64_t e = (int64_t)bid * 256 + threadIdx.x;
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

template <typename T>
__global__ __launch_bounds__(256) void k_rotate(const double* __restrict__ Q3, int64_t n, int l,
                                                const double* __restrict__ Wm, T* __restrict__ qout,
                                                T* __restrict__ qt, double* __restrict__ q64) {
  rotate_body<T>(Q3, n, l, Wm, qout, qt, q64, (int)blockIdx.x);
}

template <int LP>
static void orth_passes(int64_t n, int l, double* Y, const double* Wrot, tucker_precision prec, const OrthWs& ws,
                        void* qt, int qt_f64, uint64_t cseed, int step, hipStream_t st) {
  const int nblk = (int)((n + OR_RB - 1) / OR_RB);
  const size_t pstride = align_up((size_t)nblk * l * l * sizeof(double)) / sizeof(double);
  double* p0 = ws.part;
  double* p1 = ws.part + pstride;
  // Pass 1 works on unit-scaled columns: a pivot below tau1 says the column
  // lies within sqrt(tau1) of the span of the previous ones, below what the
  // products that formed Y resolve (FP64: the shift keeps every pivot above
  // 1e-15; FP32 and BF16: their rounding level), so it is treated as
  // dependent. Passes 2 and 3 flag a column whose pivot is below the rounding
  // level of an n-row Gram.
  const double tau1 = prec == TUCKER_FP64 ? 1e-15 : prec == TUCKER_FP32 ? 1e-12 : 1e-6;
  const double tau = fmax(1e-14, 4.0 * (double)n * 2.220446049250313e-16);
  // the shift of pass 1 (FP64 only; the FP32 / BF16 threshold already keeps
  // every accepted pivot far above rounding)
  const double shift1 = prec == TUCKER_FP64 ? 11.0 * ((double)n * l + (double)l * (l + 1)) * 1.1102230246251565e-16 : 0.0;
  // passes 2 and 3 are skipped when their input is orthonormal to this (they
  // only re-orthogonalise)
  const double eps3 = prec == TUCKER_FP64 ? 1e-13 : 1e-10;
  const uint32_t tag = 0x100u + 16u * (uint32_t)step;
  hipLaunchKernelGGL((k_gram<LP>), dim3(nblk), dim3(256), 0, st, Y, n, l, Wrot, p0, ws.status);
  hipLaunchKernelGGL((k_pass<LP>), dim3(nblk), dim3(256), 0, st, (const double*)Y, n, l, (const double*)p0, nblk, 0,
                     tau1, shift1, 0.0, cseed, tag + 1, ws.Qa, qt, qt_f64, p1, ws.R, ws.defic, ws.status);
  hipLaunchKernelGGL((k_pass<LP>), dim3(nblk), dim3(256), 0, st, (const double*)ws.Qa, n, l, (const double*)p1, nblk,
                     1, tau, 0.0, eps3, cseed, tag + 2, ws.Qa, qt, qt_f64, p0, ws.R + kMaxL * kMaxL, ws.defic + kMaxL,
                     ws.status);
  hipLaunchKernelGGL((k_pass<LP>), dim3(nblk), dim3(256), 0, st, (const double*)ws.Qa, n, l, (const double*)p0, nblk,
                     2, tau, 0.0, eps3, cseed, tag + 3, ws.Qa, qt, qt_f64, (double*)nullptr, ws.R + 2 * kMaxL * kMaxL,
                     ws.defic + 2 * kMaxL, ws.status);
}

hipError_t launch_orth_qr(int64_t n, int l, double* Y, const double* Wrot, tucker_precision prec, void* qt,
                          const OrthWs& ws, uint64_t cseed, int step, hipStream_t st) {
  TimingScope ts(KC_ORTH, st, 8.0 * n * l * 8, 4.0 * 2.0 * n * l * l);
  const int f64 = prec == TUCKER_FP64 ? 1 : 0;
  switch ((l + 15) / 16) {
    case 1: orth_passes<16>(n, l, Y, Wrot, prec, ws, qt, f64, cseed, step, st); break;
    case 2: orth_passes<32>(n, l, Y, Wrot, prec, ws, qt, f64, cseed, step, st); break;
    case 3: orth_passes<48>(n, l, Y, Wrot, prec, ws, qt, f64, cseed, step, st); break;
    case 4: orth_passes<64>(n, l, Y, Wrot, prec, ws, qt, f64, cseed, step, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int RPT>
static void svd_launch(int l, const OrthWs& ws, double tol, double negl, double* sigma, double* alpha,
                       tucker_info* info, int mode, int step, const SvdPve& pv, double* vright, bool last,
                       hipStream_t st) {
  hipLaunchKernelGGL((k_small_svd<RPT>), dim3(1), dim3(256), 0, st, (const double*)ws.R, l, (const int*)ws.status,
                     tol, negl, ws.Wm, sigma, alpha, info, mode, step, pv.r, pv.tol, pv.floor, pv.alpha_prev,
                     pv.sig_hat, pv.stop, vright, last ? 1 : 0);
}

hipError_t launch_orth_svd(int l, tucker_precision prec, const OrthWs& ws, double* sigma, double* alpha,
                           tucker_info* info, int mode, int step, hipStream_t st, const SvdPve* pve,
                           double* vright, bool last) {
  const SvdPve off{0, -1.0, 0.0, nullptr, nullptr, nullptr};
  const SvdPve& pv = pve != nullptr ? *pve : off;
  // Rotation thresholds by the precision the iterate was formed in: FP64
  // converges to l u; FP32 and BF16 iterates carry rounding noise near 1e-7
  // and 1e-3 of their norm, which bounds what their singular values and
  // vectors can resolve.
  const double u = 2.220446049250313e-16;
  const double tol = prec == TUCKER_FP64 ? u * l : prec == TUCKER_FP32 ? 1e-8 : 1e-7;
  const double negl = prec == TUCKER_FP64 ? u * l : prec == TUCKER_FP32 ? 1e-6 : 1e-4;
  switch ((l + 7) / 8) {
    case 1: svd_launch<1>(l, ws, tol, negl, sigma, alpha, info, mode, step, pv, vright, last, st); break;
    case 2: svd_launch<2>(l, ws, tol, negl, sigma, alpha, info, mode, step, pv, vright, last, st); break;
    case 3: svd_launch<3>(l, ws, tol, negl, sigma, alpha, info, mode, step, pv, vright, last, st); break;
    case 4: svd_launch<4>(l, ws, tol, negl, sigma, alpha, info, mode, step, pv, vright, last, st); break;
    case 5: svd_launch<5>(l, ws, tol, negl, sigma, alpha, info, mode, step, pv, vright, last, st); break;
    case 6: svd_launch<6>(l, ws, tol, negl, sigma, alpha, info, mode, step, pv, vright, last, st); break;
    case 7: svd_launch<7>(l, ws, tol, negl, sigma, alpha, info, mode, step, pv, vright, last, st); break;
    case 8: svd_launch<8>(l, ws, tol, negl, sigma, alpha, info, mode, step, pv, vright, last, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_orth_rotate(int64_t n, int l, const OrthWs& ws, tucker_precision prec, void* q_out, void* qt,
                              double* q64, hipStream_t st) {
  const unsigned rb = (unsigned)((n * l + 255) / 256);
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_rotate<double>), dim3(rb), dim3(256), 0, st, (const double*)ws.Qa, n, l,
                       (const double*)ws.Wm, (double*)q_out, (double*)qt, q64);
  else
    hipLaunchKernelGGL((k_rotate<float>), dim3(rb), dim3(256), 0, st, (const double*)ws.Qa, n, l,
                       (const double*)ws.Wm, (float*)q_out, (float*)qt, q64);
  return hipGetLastError();
}

hipError_t launch_orth(int64_t n, int l, double* Y, tucker_precision prec, void* q_out, void* qt, double* q64,
                       double* sigma, double* alpha, tucker_info* info, int mode, int step, const OrthWs& ws,
                       uint64_t cseed, hipStream_t st) {
  hipError_t e = launch_orth_qr(n, l, Y, nullptr, prec, nullptr, ws, cseed, step, st);
  if (e == hipSuccess) e = launch_orth_svd(l, prec, ws, sigma, alpha, info, mode, step, st);
  if (e == hipSuccess) e = launch_orth_rotate(n, l, ws, prec, q_out, qt, q64, st);
  return e;
}

// ---------------------------------------------------------------------------
// Sign rule and truncation: one workgroup per kept column.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void signfix_body(const double* __restrict__ Q, int64_t n, int l, int r,
                                                 T* __restrict__ U, T* __restrict__ Ut, int bid) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int j = bid;
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

template <typename T>
__global__ __launch_bounds__(256) void k_signfix(const double* __restrict__ Q, int64_t n, int l, int r,
                                                 T* __restrict__ U, T* __restrict__ Ut) {
  signfix_body<T>(Q, n, l, r, U, Ut, (int)blockIdx.x);
}

hipError_t launch_signfix(tucker_precision prec, const double* Q, int64_t n, int l, int r, void* U, void* Ut,
                          hipStream_t st) {
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_signfix<double>), dim3(r), dim3(256), 0, st, Q, n, l, r, (double*)U, (double*)Ut);
  else
    hipLaunchKernelGGL((k_signfix<float>), dim3(r), dim3(256), 0, st, Q, n, l, r, (float*)U, (float*)Ut);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Holistic variants: the small tensor's unfoldings in FP64 and the factor
// assembly U_k = Q_k V_k.
// ---------------------------------------------------------------------------
// X viewed as P x n x S (storage T). trans: Y[(p S + s) n + i] = X[p, i, s]
// (the transposed mode unfolding, m x n); else Y[i m + p S + s] (the
// unfolding itself, n x m). m = P S.
template <typename T>
__global__ __launch_bounds__(256) void k_unfold64(const T* __restrict__ X, int64_t P, int64_t n, int64_t S, int trans,
                                                  double* __restrict__ Y) {
  const int64_t total = P * n * S;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t s = e % S, t = e / S;
    const int64_t i = t % n, p = t / n;
    const int64_t c = p * S + s;
    Y[trans ? c * n + i : i * (P * S) + c] = (double)X[e];
  }
}

hipError_t launch_unfold64(tucker_precision prec, const View3& v, const void* X, bool trans, double* Y,
                           hipStream_t st) {
  const int64_t total = v.P * v.n * v.S;
  const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_unfold64<double>), dim3(g), dim3(256), 0, st, (const double*)X, v.P, v.n, v.S, (int)trans,
                       Y);
  else
    hipLaunchKernelGGL((k_unfold64<float>), dim3(g), dim3(256), 0, st, (const float*)X, v.P, v.n, v.S, (int)trans,
                       Y);
  return hipGetLastError();
}

// Column c of U = sign_c Q V(:, c) (Q FP64 n x l, V FP64 l x ldv, columns
// c < r), with the sign rule of k_signfix (largest magnitude positive, lowest
// row on ties, +1 for a zero column); Vt row c = sign_c V(:, c) (j-major r x l).
// One workgroup per column; both passes form each entry by the same FMA chain.
template <typename T>
__global__ __launch_bounds__(256) void k_assemble(const double* __restrict__ Q, int64_t n, int l,
                                                  const double* __restrict__ V, int ldv, int r, T* __restrict__ U,
                                                  T* __restrict__ Vt) {
  __shared__ double vc[kMaxL];
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int c = blockIdx.x;
  for (int j = threadIdx.x; j < l; j += 256) vc[j] = V[(int64_t)j * ldv + c];
  __syncthreads();
  auto entry = [&](int64_t i) {
    double w = 0.0;
    for (int j = 0; j < l; ++j) w = fma(Q[i * l + j], vc[j], w);
    return w;
  };
  double best = -1.0;
  int64_t bidx = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double a = fabs(entry(i));
    if (a > best) {
      best = a;
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
  const double sgn = entry(bi[0]) < 0.0 ? -1.0 : 1.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) U[i * r + c] = (T)(sgn * entry(i));
  for (int j = threadIdx.x; j < l; j += 256) Vt[(int64_t)c * l + j] = (T)(sgn * vc[j]);
}

// Sign rule in place on the columns of Q (FP64 n x l, each column's largest
// magnitude positive, lowest row on ties), also written j-major (l x n) in
// the storage precision to Qt. One workgroup per column.
template <typename T>
__global__ __launch_bounds__(256) void k_signcols(double* __restrict__ Q, int64_t n, int l, T* __restrict__ Qt) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  __shared__ double sgn_s;
  const int c = blockIdx.x;
  double best = -1.0;
  int64_t bidx = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double a = fabs(Q[i * l + c]);
    if (a > best) {
      best = a;
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
  if (threadIdx.x == 0) sgn_s = Q[bi[0] * l + c] < 0.0 ? -1.0 : 1.0;
  __syncthreads();  // the sign is read before any entry of the column changes
  const double sgn = sgn_s;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = sgn * Q[i * l + c];
    Q[i * l + c] = v;
    Qt[(int64_t)c * n + i] = (T)v;
  }
}

hipError_t launch_signcols(tucker_precision prec, double* Q, int64_t n, int l, void* Qt, hipStream_t st) {
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_signcols<double>), dim3(l), dim3(256), 0, st, Q, n, l, (double*)Qt);
  else
    hipLaunchKernelGGL((k_signcols<float>), dim3(l), dim3(256), 0, st, Q, n, l, (float*)Qt);
  return hipGetLastError();
}

hipError_t launch_assemble(tucker_precision prec, const double* Q, int64_t n, int l, const double* V, int ldv, int r,
                           void* U, void* Vt, hipStream_t st) {
  if (prec == TUCKER_FP64)
    hipLaunchKernelGGL((k_assemble<double>), dim3(r), dim3(256), 0, st, Q, n, l, V, ldv, r, (double*)U, (double*)Vt);
  else
    hipLaunchKernelGGL((k_assemble<float>), dim3(r), dim3(256), 0, st, Q, n, l, V, ldv, r, (float*)U, (float*)Vt);
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

__global__ void k_mode_start(double* alpha, int* ctr) {
  if (threadIdx.x != 0) return;
  if (alpha != nullptr) *alpha = 0.0;
  *ctr = 0;
}

hipError_t launch_mode_start(double* alpha, int* ctr, hipStream_t st) {
  hipLaunchKernelGGL(k_mode_start, dim3(1), dim3(1), 0, st, alpha, ctr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched persistent launches of the orthonormalisation kernels.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void b_init(const BInit& d, int bid) {
  if (bid != 0) return;
  if (d.info != nullptr) {
    char* p = (char*)d.info;
    for (size_t e = threadIdx.x; e < sizeof(tucker_info); e += blockDim.x) p[e] = 0;
  }
  if ((int)threadIdx.x < d.d) d.alpha[threadIdx.x] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0 && d.info != nullptr) {
    for (int k = 0; k < TUCKER_MAX_ORDER; ++k) d.info->l[k] = k < d.d ? d.l[k] : 0;
    d.info->flags = d.flags;
  }
}
template <int LP>
__device__ __forceinline__ void b_gram(const BGram& d, int bid) {
  gram_body<LP>(d.Y, d.n, d.l, d.Wm, d.part, d.status, bid);
}
template <int LP>
__device__ __forceinline__ void b_pass(const BPass& d, int bid) {
  pass_body<LP>(d.Qin, d.n, d.l, d.part_in, d.nblk, d.role, d.tau, d.shift_scale, d.eps3, d.cseed, d.ctag, d.Qout,
                d.qt, 0, d.part_out, d.Rg, d.defic, d.status, bid);
}
template <int RPT>
__device__ __forceinline__ void b_svd(const BSvd& d, int bid) {
  small_svd_body<RPT>(d.Rg, d.l, d.status, d.tol, d.negl, d.Wm, d.sigma, d.alpha, d.info, d.mode, d.step, 0, -1.0,
                      0.0, nullptr, nullptr, nullptr, nullptr, bid);
}
__device__ __forceinline__ void b_rotate(const BRotate& d, int bid) {
  rotate_body<float>(d.Q3, d.n, d.l, d.Wm, (float*)nullptr, (float*)nullptr, d.q64, bid);
}
__device__ __forceinline__ void b_signfix(const BSignfix& d, int bid) {
  signfix_body<float>(d.Q, d.n, d.l, d.r, d.U, d.Ut, bid);
}

size_t batch_desc_bytes(BatchKind kind) {
  switch (kind) {
    case BK_INIT: return sizeof(BInit);
    case BK_FILL: return sizeof(BFill);
    case BK_CR_SPLIT: return sizeof(BCrSplit);
    case BK_CR_COLS: return sizeof(BCrCols);
    case BK_REDUCE: return sizeof(BReduce);
    case BK_RC_SPLIT: return sizeof(BRcSplit);
    case BK_RC_COLS: return sizeof(BRcCols);
    case BK_GRAM: return sizeof(BGram);
    case BK_PASS: return sizeof(BPass);
    case BK_SVD: return sizeof(BSvd);
    case BK_ROTATE: return sizeof(BRotate);
    case BK_SIGNFIX: return sizeof(BSignfix);
    default: return 0;
  }
}

template <int LP, int RPT>
static hipError_t batch_orth_lp(BatchKind kind, int* hdr, const void* desc, hipStream_t st) {
#define TK_PERSIST(D, F)                                                                                      \
  {                                                                                                           \
    auto kern = k_persist<D, F>;                                                                              \
    hipLaunchKernelGGL(kern, dim3(resident_grid(kern)), dim3(256), 0, st, hdr, (const D*)desc);               \
  }                                                                                                           \
  break
  switch (kind) {
    case BK_INIT: TK_PERSIST(BInit, b_init);
    case BK_GRAM: TK_PERSIST(BGram, b_gram<LP>);
    case BK_PASS: TK_PERSIST(BPass, b_pass<LP>);
    case BK_SVD: TK_PERSIST(BSvd, b_svd<RPT>);
    case BK_ROTATE: TK_PERSIST(BRotate, b_rotate);
    case BK_SIGNFIX: TK_PERSIST(BSignfix, b_signfix);
    default:
      return hipErrorInvalidValue;
  }
#undef TK_PERSIST
  return hipGetLastError();
}

hipError_t launch_batch_orth(BatchKind kind, int lclass, int* hdr, const void* desc, hipStream_t st) {
  switch (lclass) {
    case 16: return batch_orth_lp<16, 2>(kind, hdr, desc, st);
    case 32: return batch_orth_lp<32, 4>(kind, hdr, desc, st);
    case 48: return batch_orth_lp<48, 6>(kind, hdr, desc, st);
    case 64: return batch_orth_lp<64, 8>(kind, hdr, desc, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tk
