// Options of the sketch-truncate-ridge build (Sec. 2.3, 2.5; App. D):
//   k_philox_sketch : the Gaussian sketch S (T x k, N(0, 1/k)) drawn on the
//                     device from the Philox4x32-10 counter generator
//                     (Salmon et al., SC 2011), counter (t, j, 0, 0), key =
//                     seed; Box-Muller in float64 on two output words;
//   k_countsketch   : Y = L Phi for the CountSketch Phi(t, h(t)) = s(t):
//                     one workgroup per bucket gathers its periods in
//                     ascending t (deterministic) and sums s(t) L[:, t];
//   k_knee          : App. D knee rule, ell = max{i : lam_i/lam_1 >= tau,
//                     lam_{i+1}/lam_i <= rho} over the computed eigenvalues
//                     lam of G = Y^T Y (lam_i = sigma_i^2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"
#include "npga_sketch.h"

namespace npga {

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
  }
}

// S[t + j lds] for t < T, j < k.  `raw` (optional) receives the first two
// output words of each entry (t + j T) for bit-exact checks.
__global__ __launch_bounds__(256) void k_philox_sketch(uint64_t seed, int64_t T, int64_t k, float *S, int64_t lds,
                                                       uint32_t *raw) {
  const double inv_sqrt_k = 1.0 / sqrt((double)k);
  const int64_t total = T * k;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t j = e / T, t = e - j * T;
    uint32_t c[4] = {(uint32_t)t, (uint32_t)j, 0u, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = ((double)c[0] + 0.5) * 2.3283064365386963e-10;
    const double u2 = (double)c[1] * 2.3283064365386963e-10;
    const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    S[t + j * lds] = (float)(z * inv_sqrt_k);
    if (raw) {
      raw[2 * e] = c[0];
      raw[2 * e + 1] = c[1];
    }
  }
}

// Y[:, b] = sum_{t : h(t) = b} s(t) L[:, t], periods in ascending order.
// Workgroup b scans h in chunks of 256 periods; each wavefront's matches
// are a 64-bit ballot, combined in wavefront order through LDS.
__global__ __launch_bounds__(256) void k_countsketch(const float *L, int64_t ld, int64_t n, int64_t T,
                                                     const int32_t *h, const float *sgn, int64_t k, float *Y,
                                                     int64_t ldy, int32_t *bad) {
  constexpr int R = 32;  // rows per thread (n <= 8192)
  __shared__ unsigned long long masks[4];
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = 0.0;
  for (int64_t t0 = 0; t0 < T; t0 += 256) {
    const int64_t t = t0 + tid;
    int32_t ht = -1;
    if (t < T) {
      ht = h[t];
      if ((ht < 0 || ht >= k) && b == 0) *bad = 1;  // same value from every writer
    }
    const unsigned long long m = __ballot(ht == (int32_t)b);
    if (lane == 0) masks[wave] = m;
    __syncthreads();
    for (int w = 0; w < 4; ++w) {
      unsigned long long mw = masks[w];
      while (mw) {
        const int bit = __ffsll((long long)mw) - 1;
        mw &= mw - 1;
        const int64_t tt = t0 + 64 * w + bit;
        const double s = (double)sgn[tt];
        const float *col = L + tt * ld;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int64_t i = tid + 256 * q;
          if (i < n) acc[q] = fma(s, (double)col[i], acc[q]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int64_t i = tid + 256 * q;
    if (i < n) Y[i + b * ldy] = (float)acc[q];
  }
}

// ell by the knee rule over lam[0..m) (descending); 0 if no index qualifies.
__global__ __launch_bounds__(256) void k_knee(const double *lam, int64_t m, double tau, double rho, int64_t *ell) {
  __shared__ long long best[256];
  long long bi = 0;
  const double l1 = lam[0];
  for (int64_t i = threadIdx.x; i + 1 < m; i += 256) {
    // 1-based index i + 1: lam_{i+1}/lam_1 >= tau and lam_{i+2}/lam_{i+1} <= rho
    const double li = lam[i], ln = lam[i + 1];
    if (l1 > 0.0 && li >= tau * l1 && ln <= rho * li) bi = (long long)(i + 1);
  }
  best[threadIdx.x] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) best[threadIdx.x] = best[threadIdx.x] > best[threadIdx.x + s] ? best[threadIdx.x]
                                                                                          : best[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *ell = best[0];
}

int launch_philox_sketch(uint64_t seed, int64_t T, int64_t k, float *S, int64_t lds, uint32_t *raw,
                         hipStream_t s) {
  const int64_t blocks = (T * k + 255) / 256;
  const int g = (int)(blocks < 8192 ? blocks : 8192);
  hipLaunchKernelGGL(k_philox_sketch, dim3(g), dim3(256), 0, s, seed, T, k, S, lds, raw);
  return (int)hipGetLastError();
}

int launch_countsketch(const float *L, int64_t ld, int64_t n, int64_t T, const int32_t *h, const float *sgn,
                       int64_t k, float *Y, int64_t ldy, int32_t *bad, hipStream_t s) {
  if (n > 256 * 32) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_countsketch, dim3((unsigned)k), dim3(256), 0, s, L, ld, n, T, h, sgn, k, Y, ldy, bad);
  return (int)hipGetLastError();
}

int launch_knee(const double *lam, int64_t m, double tau, double rho, int64_t *ell, hipStream_t s) {
  hipLaunchKernelGGL(k_knee, dim3(1), dim3(256), 0, s, lam, m, tau, rho, ell);
  return (int)hipGetLastError();
}

}  // namespace npga
