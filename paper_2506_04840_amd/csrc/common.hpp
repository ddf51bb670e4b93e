// Shared device helpers for the Tucker kernels (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tucker.h"

namespace tk {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short shortx8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;
constexpr int kMaxL = TUCKER_MAX_L;   // widest sketch handled by the kernels

// Which matrix-core instruction a product runs on.
enum MfmaKind { MF_F32 = 0, MF_F64 = 1, MF_BF16 = 2 };

// Tensor X viewed as row-major [P, n, S]; the mode-k unfolding is
// X_(k)[i, p*S + s] = X[p, i, s] (columns in row-major order of the other modes).
struct View {
  int64_t P, n, S;
};

// Round-to-nearest-even float -> bf16 bits (inputs are finite in this path;
// NaN keeps a quiet NaN pattern).
__device__ __forceinline__ unsigned short f32_to_bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma_f64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011) and the Box-Muller map that define
// the Gaussian test matrices Omega_k. Addressing of Omega_k[c, j]:
//   counter = (c mod 2^32, c div 2^32, j div 4, k), key = (seed lo, seed hi)
//   pair (w0,w1) for even j div 2, (w2,w3) for odd; u = (w + 1/2) 2^-32
//   value = sqrt(-2 ln u_a) * (cos 2 pi u_b for even j, sin 2 pi u_b for odd j)
// ---------------------------------------------------------------------------
struct U32x4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U32x4 philox4x32_10(U32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = U32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Four consecutive entries Omega[c, 4g .. 4g+3].
__device__ __forceinline__ void gaussian4_f64(uint64_t seed, uint32_t mode, uint64_t c, uint32_t g,
                                              double out[4]) {
  U32x4 w = philox4x32_10(U32x4{(uint32_t)c, (uint32_t)(c >> 32), g, mode}, (uint32_t)seed,
                          (uint32_t)(seed >> 32));
  const double sc = 2.3283064365386963e-10;  // 2^-32
  double ua = ((double)w.x + 0.5) * sc, ub = ((double)w.y + 0.5) * sc;
  double r = sqrt(-2.0 * log(ua)), sn, cs;
  sincospi(2.0 * ub, &sn, &cs);
  out[0] = r * cs;
  out[1] = r * sn;
  ua = ((double)w.z + 0.5) * sc;
  ub = ((double)w.w + 0.5) * sc;
  r = sqrt(-2.0 * log(ua));
  sincospi(2.0 * ub, &sn, &cs);
  out[2] = r * cs;
  out[3] = r * sn;
}

__device__ __forceinline__ void gaussian4_f32(uint64_t seed, uint32_t mode, uint64_t c, uint32_t g,
                                              float out[4]) {
  U32x4 w = philox4x32_10(U32x4{(uint32_t)c, (uint32_t)(c >> 32), g, mode}, (uint32_t)seed,
                          (uint32_t)(seed >> 32));
  const float sc = 2.3283064365386963e-10f;
  const float half = 1.16415321826934814e-10f;  // 2^-33
  float ua = fmaf((float)w.x, sc, half), ub = fmaf((float)w.y, sc, half);
  float r = sqrtf(-2.0f * logf(ua)), sn, cs;
  sincospif(2.0f * ub, &sn, &cs);
  out[0] = r * cs;
  out[1] = r * sn;
  ua = fmaf((float)w.z, sc, half);
  ub = fmaf((float)w.w, sc, half);
  r = sqrtf(-2.0f * logf(ua));
  sincospif(2.0f * ub, &sn, &cs);
  out[2] = r * cs;
  out[3] = r * sn;
}

// Uniform [-1, 1] entries of stream `tag` (the uniform bit 2^30 is added
// here): entry [c, 4g + q] = (w_q + 1/2) 2^-31 - 1 of the Philox block at
// counter (c lo, c hi, g, tag + 2^30). Formed exactly in FP64, rounded once
// for FP32.
__device__ __forceinline__ void uniform4_f64(uint64_t seed, uint32_t tag, uint64_t c, uint32_t g, double out[4]) {
  const U32x4 w = philox4x32_10(U32x4{(uint32_t)c, (uint32_t)(c >> 32), g, tag + (1u << 30)}, (uint32_t)seed,
                                (uint32_t)(seed >> 32));
  const double sc = 4.656612873077392578125e-10;  // 2^-31
  out[0] = ((double)w.x + 0.5) * sc - 1.0;
  out[1] = ((double)w.y + 0.5) * sc - 1.0;
  out[2] = ((double)w.z + 0.5) * sc - 1.0;
  out[3] = ((double)w.w + 0.5) * sc - 1.0;
}
__device__ __forceinline__ void uniform4_f32(uint64_t seed, uint32_t tag, uint64_t c, uint32_t g, float out[4]) {
  double d[4];
  uniform4_f64(seed, tag, c, g, d);
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = (float)d[q];
}

// Workgroup barrier that orders LDS only: global loads in flight (a
// prefetched stage) stay in flight across it, where __syncthreads would wait
// for every outstanding global access.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Persistent batched launch: the grid's workgroups loop over the work items
// of all requests in the table (hdr[0] = requests, hdr[1 + b] = first item of
// request b, hdr[1 + nreq] = total) and run the request's workgroup body F
// with the request-local block index. A workgroup starts with the item of its
// own index. With CLAIM (items long against an atomic's round trip: the
// product phases) it then claims the next unclaimed item of its residue class
// mod 8 (the class of the XCD it runs on, so items that share an operand
// through the index mod 8 keep sharing that XCD's L2) from the class's counter
// hdr[2 + nreq + class], which every upload of the table sets to zero:
// workgroups that drew short items take more, and the launch ends with the
// last item rather than with the longest static share. Without CLAIM it
// strides by the grid. The result of an item does not depend on which
// workgroup runs it. A workgroup's items only move forward, so the request of
// the previous item bounds the search for the next one. A barrier separates
// consecutive items so a body may leave some waves early and reuse LDS.
template <typename D, void (*F)(const D&, int), int MINB = 1, bool CLAIM = false>
__global__ __launch_bounds__(256, MINB) void k_persist(int* __restrict__ hdr, const D* __restrict__ desc) {
  __shared__ int next_s;
  const int nreq = hdr[0];
  const int total = hdr[1 + nreq];
  const int cls = (int)(blockIdx.x & 7);
  // the first item of the class past the static ones (indices below the grid)
  const int first = cls + 8 * (((int)gridDim.x - cls + 7) >> 3);
  int* const ctr = hdr + 2 + nreq + cls;
  int b = 0;
  int w = (int)blockIdx.x;
  while (w < total) {
    if (hdr[2 + b] <= w) {
      int lo = b + 1, hi = nreq - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (hdr[1 + mid] <= w)
          lo = mid;
        else
          hi = mid - 1;
      }
      b = lo;
    }
    F(desc[b], w - hdr[1 + b]);
    __syncthreads();
    if constexpr (CLAIM) {
      if (threadIdx.x == 0) next_s = first + 8 * atomicAdd(ctr, 1);
      __syncthreads();
      w = next_s;
    } else {
      w += (int)gridDim.x;
    }
  }
}

// Workgroups of a 256-thread kernel resident on the whole device at once
// (occupancy per CU x CUs), queried once per kernel and device: the grid of a
// persistent launch, so that every workgroup runs from the start.
template <typename Kern>
inline int resident_grid(Kern kernel) {
  static int cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int g = cache[dev];
  if (g == 0) {
    int per = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(kernel), 256, 0) !=
            hipSuccess || per < 1)
      per = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    g = per * cus;
    cache[dev] = g;
  }
  return g;
}

}  // namespace tk
