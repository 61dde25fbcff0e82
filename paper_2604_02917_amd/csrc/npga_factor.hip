// Sample mean and centred covariance factor (paper Sec. 2.1):
//     mu = (1/T) R 1_T,   L = (R - mu 1_T^T) / sqrt(T - 1).
// Pass 1 streams R once: each wavefront owns whole columns and accumulates
// float64 row sums in registers; the four wavefronts of a workgroup are
// combined in a fixed order and each workgroup writes one partial vector.
// A row-block kernel then sums the partials in a fixed order (deterministic).
// Pass 2 streams R again and writes L (in place when L == R).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"

namespace npga {

template <int E>
__global__ __launch_bounds__(256) void k_rowsum(const float *R, int64_t n, int64_t T, int64_t ldr,
                                                double *part, int64_t ldp, double *badpart) {
  __shared__ double sh[256 * E * 4 / 4 + 4];  // one n-vector (256*E doubles) + 4 counters
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t W = (int64_t)gridDim.x * 4;
  double acc[4 * E];
  double bad = 0.0;
#pragma unroll
  for (int j = 0; j < 4 * E; ++j) acc[j] = 0.0;
  for (int64_t col = (int64_t)blockIdx.x * 4 + wave; col < T; col += W) {
    const f4 *p = reinterpret_cast<const f4 *>(R + col * ldr) + lane;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t row0 = 4 * lane + 256 * j;
      if (row0 < n) {
        const f4 c = __builtin_nontemporal_load(p + 64 * j);
        const float cc[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (row0 + e < n) {
            const float x = cc[e];
            if (isfinite(x))
              acc[4 * j + e] += (double)x;
            else
              bad += 1.0;
          }
        }
      }
    }
  }
  bad = wave_sum_f64(bad);
  // combine wavefronts 0..3 in order through one LDS vector
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int j = 0; j < E; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int idx = 4 * lane + 256 * j + e;
          sh[idx] = (w == 0) ? acc[4 * j + e] : sh[idx] + acc[4 * j + e];
        }
      if (lane == 0) sh[256 * E + w] = bad;
    }
    __syncthreads();
  }
  double *out = part + (int64_t)blockIdx.x * ldp;
  for (int idx = threadIdx.x; idx < 256 * E; idx += 256) out[idx] = sh[idx];
  if (threadIdx.x == 0)
    badpart[blockIdx.x] = ((sh[256 * E] + sh[256 * E + 1]) + sh[256 * E + 2]) + sh[256 * E + 3];
}

__global__ __launch_bounds__(256) void k_rowsum_reduce(const double *part, int G, int64_t ldp, int64_t n,
                                                       double invT, double *mu, const double *badpart,
                                                       double *nonfinite) {
  __shared__ double red[4][64];
  const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + r;
  double s = 0.0;
  if (i < n)
    for (int w = q; w < G; w += 4) s += part[(int64_t)w * ldp + i];
  red[q][r] = s;
  __syncthreads();
  if (q == 0 && i < n) mu[i] = (((red[0][r] + red[1][r]) + red[2][r]) + red[3][r]) * invT;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double b = 0.0;
    for (int w = 0; w < G; ++w) b += badpart[w];
    *nonfinite = b;
  }
}

template <int E>
__global__ __launch_bounds__(256) void k_center(const float *R, int64_t n, int64_t T, int64_t ldr,
                                                float *L, int64_t ldl, const double *mu, double scale) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t W = (int64_t)gridDim.x * 4;
  double m[4 * E];
#pragma unroll
  for (int j = 0; j < E; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = 4 * lane + 256 * j + e;
      m[4 * j + e] = (i < n) ? mu[i] : 0.0;
    }
  for (int64_t col = (int64_t)blockIdx.x * 4 + wave; col < T; col += W) {
    const f4 *p = reinterpret_cast<const f4 *>(R + col * ldr) + lane;
    f4 *q = reinterpret_cast<f4 *>(L + col * ldl) + lane;
    f4 c[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t row0 = 4 * lane + 256 * j;
      if (row0 < n) c[j] = __builtin_nontemporal_load(p + 64 * j);
    }
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t row0 = 4 * lane + 256 * j;
      if (row0 + 3 < n) {
        f4 o;
        o.x = (float)(((double)c[j].x - m[4 * j + 0]) * scale);
        o.y = (float)(((double)c[j].y - m[4 * j + 1]) * scale);
        o.z = (float)(((double)c[j].z - m[4 * j + 2]) * scale);
        o.w = (float)(((double)c[j].w - m[4 * j + 3]) * scale);
        __builtin_nontemporal_store(o, q + 64 * j);
      } else if (row0 < n) {
        float *qs = L + col * ldl + row0;
        const float cc[4] = {c[j].x, c[j].y, c[j].z, c[j].w};
        for (int e = 0; e < 4 && row0 + e < n; ++e)
          qs[e] = (float)(((double)cc[e] - m[4 * j + e]) * scale);
      }
    }
  }
}

// float32 -> bfloat16 with round-to-nearest-even (NaN kept quiet): the
// storage format of the reduced-precision factor.
__global__ __launch_bounds__(256) void k_to_bf16(const float *L, int64_t n, int64_t T, int64_t ld, uint16_t *Lb,
                                                 int64_t ldb) {
  const int64_t total = n * T;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
    const int64_t t = q / n, i = q - t * n;
    const uint32_t u = __float_as_uint(L[i + t * ld]);
    uint16_t b;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      b = (uint16_t)((u >> 16) | 0x40u);
    } else {
      const uint32_t lsb = (u >> 16) & 1u;
      b = (uint16_t)((u + 0x7fffu + lsb) >> 16);
    }
    Lb[i + t * ldb] = b;
  }
}

int launch_to_bf16(const float *L, int64_t n, int64_t T, int64_t ld, uint16_t *Lb, int64_t ldb, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(4096), dim3(256), 0, s, L, n, T, ld, Lb, ldb);
  return (int)hipGetLastError();
}

#define FACTOR_SLOT_SWITCH(slots, CALL) \
  switch (slots) {                     \
    case 1: CALL(1); break;            \
    case 2: CALL(2); break;            \
    case 4: CALL(4); break;            \
    case 8: CALL(8); break;            \
    case 12: CALL(12); break;          \
    case 16: CALL(16); break;          \
    case 22: CALL(22); break;          \
    case 28: CALL(28); break;          \
    case 32: CALL(32); break;          \
    default: return (int)hipErrorInvalidValue; \
  }

int launch_build_factor(const float *R, int64_t n, int64_t T, int64_t ldr, float *L, int64_t ldl,
                        double *mu_out, double *part, int grid, double *nonfinite, hipStream_t s) {
  const int slots = slots_for(n);
  const int64_t ldp = (int64_t)256 * slots;
  double *badpart = part + (int64_t)grid * ldp;
#define CALL(E) \
  hipLaunchKernelGGL(k_rowsum<E>, dim3(grid), dim3(256), 0, s, R, n, T, ldr, part, ldp, badpart)
  FACTOR_SLOT_SWITCH(slots, CALL)
#undef CALL
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
  hipLaunchKernelGGL(k_rowsum_reduce, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, part, grid, ldp,
                     n, 1.0 / (double)T, mu_out, badpart, nonfinite);
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
  const double scale = 1.0 / sqrt((double)(T - 1));
#define CALL(E) \
  hipLaunchKernelGGL(k_center<E>, dim3(grid), dim3(256), 0, s, R, n, T, ldr, L, ldl, mu_out, scale)
  FACTOR_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

}  // namespace npga
