// Float64 gradient at a refinement anchor x_a:
//     u_a = L^T x_a,   g_a = 2 L u_a      (eq. npga-unified-grad, ridge excluded)
// with float64 products and sums over the float32 factor.  Two streaming
// passes over L (u_a needs all of x_a before g_a can start).  The
// refinement phase then iterates on d = x - x_a with the float32 sweep:
// grad f(x) = g_a + 2 L (L^T d) + 2 gamma x, so the float32 rounding of the
// sweep scales with ||d|| instead of ||x|| (mixed-precision iterative
// refinement).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"

namespace npga {

template <int E, typename TL>
__device__ __forceinline__ void load_col_masked(const TL *L, int64_t ld, int64_t n, int64_t col, int lane,
                                                f4 (&c)[E]) {
  const TL *p = L + col * ld + 4 * lane;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t row0 = 4 * lane + 256 * j;
    f4 v = f4{0.f, 0.f, 0.f, 0.f};
    if (row0 < n) {
      v = load4_nt<TL>(p + 256 * j);
      if (row0 + 1 >= n) v.y = 0.f;
      if (row0 + 2 >= n) v.z = 0.f;
      if (row0 + 3 >= n) v.w = 0.f;
    }
    c[j] = v;
  }
}

template <int E, typename TL>
__global__ __launch_bounds__(256) void k_precise_u(const TL *L, int64_t ld, int64_t n, int64_t cols,
                                                   const double *x, double *u) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t W = (int64_t)gridDim.x * 4;
  double xr[4 * E];
#pragma unroll
  for (int j = 0; j < E; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = 4 * lane + 256 * j + e;
      xr[4 * j + e] = (i < n) ? x[i] : 0.0;
    }
  for (int64_t col = (int64_t)blockIdx.x * 4 + wave; col < cols; col += W) {
    f4 c[E];
    load_col_masked<E, TL>(L, ld, n, col, lane, c);
    double d = 0.0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      d = fma((double)c[j].x, xr[4 * j + 0], d);
      d = fma((double)c[j].y, xr[4 * j + 1], d);
      d = fma((double)c[j].z, xr[4 * j + 2], d);
      d = fma((double)c[j].w, xr[4 * j + 3], d);
    }
    d = wave_sum_f64(d);
    if (lane == 0) u[col] = d;
  }
}

template <int E, typename TL>
__global__ __launch_bounds__(256) void k_precise_g(const TL *L, int64_t ld, int64_t n, int64_t cols,
                                                   const double *u, double *part, int64_t ldp) {
  __shared__ double sh[256 * E];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t W = (int64_t)gridDim.x * 4;
  double g[4 * E];
#pragma unroll
  for (int j = 0; j < 4 * E; ++j) g[j] = 0.0;
  for (int64_t col = (int64_t)blockIdx.x * 4 + wave; col < cols; col += W) {
    f4 c[E];
    load_col_masked<E, TL>(L, ld, n, col, lane, c);
    const double uc = u[col];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      g[4 * j + 0] = fma((double)c[j].x, uc, g[4 * j + 0]);
      g[4 * j + 1] = fma((double)c[j].y, uc, g[4 * j + 1]);
      g[4 * j + 2] = fma((double)c[j].z, uc, g[4 * j + 2]);
      g[4 * j + 3] = fma((double)c[j].w, uc, g[4 * j + 3]);
    }
  }
  // combine wavefronts 0..3 in a fixed order
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int j = 0; j < E; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int idx = 4 * lane + 256 * j + e;
          sh[idx] = (w == 0) ? g[4 * j + e] : sh[idx] + g[4 * j + e];
        }
    }
    __syncthreads();
  }
  double *out = part + (int64_t)blockIdx.x * ldp;
  for (int idx = threadIdx.x; idx < 256 * E; idx += 256) out[idx] = sh[idx];
}

__global__ __launch_bounds__(256) void k_precise_reduce(const double *part, int G, int64_t ldp, int64_t n,
                                                        double *g) {
  __shared__ double red[4][64];
  const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + r;
  double s = 0.0;
  if (i < n)
    for (int w = q; w < G; w += 4) s += part[(int64_t)w * ldp + i];
  red[q][r] = s;
  __syncthreads();
  if (q == 0 && i < n) g[i] = 2.0 * (((red[0][r] + red[1][r]) + red[2][r]) + red[3][r]);
}

// H p = (2 L L^T p) + 2 gamma p for the float64 refinement steps.
__global__ __launch_bounds__(256) void k_add_ridge(SolveArgs a) {
  const DevState *st = a.st;
  if (st->done != kRunning) return;
  const double g2 = 2.0 * st->gamma;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * 256)
    a.gbuf0[i] = fma(g2, a.pvec[i], a.gbuf0[i]);
}

int launch_add_ridge(const SolveArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_add_ridge, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return (int)hipGetLastError();
}

#define PRECISE_SLOT_SWITCH(slots, CALL)         \
  switch (slots) {                               \
    case 1: CALL(1); break;                      \
    case 2: CALL(2); break;                      \
    case 4: CALL(4); break;                      \
    case 8: CALL(8); break;                      \
    case 12: CALL(12); break;                    \
    case 16: CALL(16); break;                    \
    case 22: CALL(22); break;                    \
    case 28: CALL(28); break;                    \
    case 32: CALL(32); break;                    \
    default: return (int)hipErrorInvalidValue;   \
  }

int launch_precise_gradient(const SolveArgs &a, const double *x, double *u_out, double *g_out,
                            double *part, int slots, hipStream_t s) {
  const int G = sweep_grid_for(a.cols);
  if (a.dtype == NPGA_BF16) {
    const bf16_t *L = static_cast<const bf16_t *>(a.L);
#define CALL(E) hipLaunchKernelGGL((k_precise_u<E, bf16_t>), dim3(G), dim3(256), 0, s, L, a.ld, a.n, a.cols, x, u_out)
    PRECISE_SLOT_SWITCH(slots, CALL)
#undef CALL
#define CALL(E) \
  hipLaunchKernelGGL((k_precise_g<E, bf16_t>), dim3(G), dim3(256), 0, s, L, a.ld, a.n, a.cols, u_out, part, a.ldp)
    PRECISE_SLOT_SWITCH(slots, CALL)
#undef CALL
  } else {
    const float *L = static_cast<const float *>(a.L);
#define CALL(E) hipLaunchKernelGGL((k_precise_u<E, float>), dim3(G), dim3(256), 0, s, L, a.ld, a.n, a.cols, x, u_out)
    PRECISE_SLOT_SWITCH(slots, CALL)
#undef CALL
#define CALL(E) \
  hipLaunchKernelGGL((k_precise_g<E, float>), dim3(G), dim3(256), 0, s, L, a.ld, a.n, a.cols, u_out, part, a.ldp)
    PRECISE_SLOT_SWITCH(slots, CALL)
#undef CALL
  }
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
  hipLaunchKernelGGL(k_precise_reduce, dim3((unsigned)((a.n + 63) / 64)), dim3(256), 0, s, part, G, a.ldp,
                     a.n, g_out);
  return (int)hipGetLastError();
}

}  // namespace npga
