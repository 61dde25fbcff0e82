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
    if (lane == 0 && u) u[col] = d;
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

// Both products in one pass over L, the order of the fused float32 sweep:
// per column t, u_t = L_t . x (float64 products and sums, all lanes hold it
// after the wave sum) and then g += L_t u_t (float64).  x lives in LDS
// (float64, 8 KB per slot), so g and two column buffers fit the registers
// and the next column loads while this one is used.  Per-workgroup float64
// partials of g as in k_precise_g.  Up to 22 slots (n <= 5632).
template <int E, typename TL>
__global__ __launch_bounds__(256) void k_precise_sweep(const TL *L, int64_t ld, int64_t n, int64_t cols,
                                                       const double *x, double *u, double *part,
                                                       int64_t ldp) {
  __shared__ double xsh[256 * E];  // x; after the sweep, the combine buffer
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t W = (int64_t)gridDim.x * 4;
  // entry 4 lane + 256 j + e of x at xsh[(4 j + e) 64 + lane]: a wavefront
  // reads 64 consecutive doubles per (j, e)
  for (int q = threadIdx.x; q < 256 * E; q += 256) {
    const int l = q & 63, je = q >> 6, j = je >> 2, e = je & 3;
    const int64_t i = 4 * l + 256 * j + e;
    xsh[q] = (i < n) ? x[i] : 0.0;
  }
  double g[4 * E];
#pragma unroll
  for (int j = 0; j < 4 * E; ++j) g[j] = 0.0;
  __syncthreads();
  // zero the compiler cannot see through (n < 2^62): the update below
  // widens the column again instead of keeping the float64 values of the
  // dot product live across its wave sum
  const unsigned int z = (unsigned int)((uint64_t)n >> 62);
  auto wide = [&](float v) { return (double)__uint_as_float(__float_as_uint(v) ^ z); };
  auto process = [&](const f4(&c)[E], int64_t col) {
    double d = 0.0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      d = fma((double)c[j].x, xsh[(4 * j + 0) * 64 + lane], d);
      d = fma((double)c[j].y, xsh[(4 * j + 1) * 64 + lane], d);
      d = fma((double)c[j].z, xsh[(4 * j + 2) * 64 + lane], d);
      d = fma((double)c[j].w, xsh[(4 * j + 3) * 64 + lane], d);
      __builtin_amdgcn_sched_barrier(0);  // keep the reads of x next to their use
    }
    d = wave_sum_f64(d);
    if (lane == 0 && u) u[col] = d;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      g[4 * j + 0] = fma(wide(c[j].x), d, g[4 * j + 0]);
      g[4 * j + 1] = fma(wide(c[j].y), d, g[4 * j + 1]);
      g[4 * j + 2] = fma(wide(c[j].z), d, g[4 * j + 2]);
      g[4 * j + 3] = fma(wide(c[j].w), d, g[4 * j + 3]);
    }
  };
  f4 c0[E], c1[E];
  int64_t col = (int64_t)blockIdx.x * 4 + wave;
  if (col < cols) load_col_masked<E, TL>(L, ld, n, col, lane, c0);
  while (col < cols) {
    const int64_t col1 = col + W;
    if (col1 < cols) load_col_masked<E, TL>(L, ld, n, col1, lane, c1);
    process(c0, col);
    if (col1 >= cols) break;
    const int64_t col2 = col1 + W;
    if (col2 < cols) load_col_masked<E, TL>(L, ld, n, col2, lane, c0);
    process(c1, col1);
    col = col2;
  }
  // combine wavefronts 0..3 in a fixed order (x is no longer needed)
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int j = 0; j < E; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int idx = 4 * lane + 256 * j + e;
          xsh[idx] = (w == 0) ? g[4 * j + e] : xsh[idx] + g[4 * j + e];
        }
    }
    __syncthreads();
  }
  double *out = part + (int64_t)blockIdx.x * ldp;
  for (int idx = threadIdx.x; idx < 256 * E; idx += 256) out[idx] = xsh[idx];
}

// The same pass with the rows of a column split over a pair of wavefronts
// (eight per workgroup, four column streams): each lane then keeps 2 E
// float64 accumulators instead of 4 E, which fit the vector registers (with
// 4 E = 88 at n = 5440 they sat in accumulation registers, moved in and out
// on every update, and the kernel was bound by its vector instructions).
// The pair's two partial dot products meet in LDS, one barrier per column
// step (slots alternate with the step's parity); every pair runs the step
// count of the workgroup's first pair so that the barriers match.
template <int E, typename TL>
__global__ __launch_bounds__(512) void k_precise_pair(const TL *L, int64_t ld, int64_t n, int64_t cols,
                                                      const double *x, double *u, double *part, int64_t ldp) {
  constexpr int E2 = (E + 1) / 2;
  __shared__ double xsh[256 * E];     // x; after the sweep, the combine buffer
  __shared__ double dsh[2][4][2];     // [step parity][pair][half]
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int pr = wave >> 1, hf = wave & 1;
  const int j0 = hf * E2;  // the half's first group of four rows
  const int64_t W = (int64_t)gridDim.x * 4;
  for (int q = threadIdx.x; q < 256 * E; q += 512) {
    const int l = q & 63, je = q >> 6, j = je >> 2, e = je & 3;
    const int64_t i = 4 * l + 256 * j + e;
    xsh[q] = (i < n) ? x[i] : 0.0;
  }
  double g[4 * E2];
#pragma unroll
  for (int q = 0; q < 4 * E2; ++q) g[q] = 0.0;
  __syncthreads();
  const unsigned int z = (unsigned int)((uint64_t)n >> 62);
  auto wide = [&](float v) { return (double)__uint_as_float(__float_as_uint(v) ^ z); };
  auto load = [&](f4(&c)[E2], int64_t col) {
    const TL *p = L + col * ld + 4 * lane;
#pragma unroll
    for (int jj = 0; jj < E2; ++jj) {
      const int j = j0 + jj;
      const int64_t row0 = 4 * lane + 256 * j;
      f4 v = f4{0.f, 0.f, 0.f, 0.f};
      if (col < cols && j < E && row0 < n) {
        v = load4_nt<TL>(p + 256 * j);
        if (row0 + 1 >= n) v.y = 0.f;
        if (row0 + 2 >= n) v.z = 0.f;
        if (row0 + 3 >= n) v.w = 0.f;
      }
      c[jj] = v;
    }
  };
  auto step = [&](const f4(&c)[E2], int64_t col, int64_t k) {
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
#pragma unroll
    for (int jj = 0; jj < E2; ++jj) {
      const int j = j0 + jj;
      if (j < E) {
        d0 = fma((double)c[jj].x, xsh[(4 * j + 0) * 64 + lane], d0);
        d1 = fma((double)c[jj].y, xsh[(4 * j + 1) * 64 + lane], d1);
        d2 = fma((double)c[jj].z, xsh[(4 * j + 2) * 64 + lane], d2);
        d3 = fma((double)c[jj].w, xsh[(4 * j + 3) * 64 + lane], d3);
      }
    }
    const double dp = wave_sum_f64((d0 + d1) + (d2 + d3));
    const int par = (int)(k & 1);
    if (lane == 0) dsh[par][pr][hf] = dp;
    __syncthreads();
    const double d = dsh[par][pr][0] + dsh[par][pr][1];
    if (hf == 0 && lane == 0 && u && col < cols) u[col] = d;
#pragma unroll
    for (int jj = 0; jj < E2; ++jj) {
      g[4 * jj + 0] = fma(wide(c[jj].x), d, g[4 * jj + 0]);
      g[4 * jj + 1] = fma(wide(c[jj].y), d, g[4 * jj + 1]);
      g[4 * jj + 2] = fma(wide(c[jj].z), d, g[4 * jj + 2]);
      g[4 * jj + 3] = fma(wide(c[jj].w), d, g[4 * jj + 3]);
    }
  };
  const int64_t c00 = (int64_t)blockIdx.x * 4;
  const int64_t K = (c00 < cols) ? (cols - c00 + W - 1) / W : 0;  // steps of the first pair (the most)
  f4 c0[E2], c1[E2];
  if (K > 0) load(c0, c00 + pr);
  for (int64_t k = 0; k < K; k += 2) {
    const int64_t ca = c00 + pr + k * W;
    if (k + 1 < K) load(c1, ca + W);
    step(c0, ca, k);
    if (k + 1 >= K) break;
    if (k + 2 < K) load(c0, ca + 2 * W);
    step(c1, ca + W, k + 1);
  }
  // combine the four pairs in a fixed order (x is no longer needed)
  __syncthreads();
  for (int p = 0; p < 4; ++p) {
    if (pr == p) {
#pragma unroll
      for (int jj = 0; jj < E2; ++jj) {
        const int j = j0 + jj;
        if (j < E) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int idx = 4 * lane + 256 * j + e;
            xsh[idx] = (p == 0) ? g[4 * jj + e] : xsh[idx] + g[4 * jj + e];
          }
        }
      }
    }
    __syncthreads();
  }
  double *out = part + (int64_t)blockIdx.x * ldp;
  for (int idx = threadIdx.x; idx < 256 * E; idx += 512) out[idx] = xsh[idx];
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
  if (slots <= 22) {
    // one pass over L
#define ONEPASS(E, TL)                                                                                       \
  hipLaunchKernelGGL((k_precise_sweep<E, TL>), dim3(G), dim3(256), 0, s, static_cast<const TL *>(a.L), a.ld, \
                     a.n, a.cols, x, u_out, part, a.ldp)
#define PAIRPASS(E, TL)                                                                                     \
  hipLaunchKernelGGL((k_precise_pair<E, TL>), dim3(G), dim3(512), 0, s, static_cast<const TL *>(a.L), a.ld, \
                     a.n, a.cols, x, u_out, part, a.ldp)
#define ONEPASS_SWITCH(TL)                     \
  switch (slots) {                             \
    case 1: ONEPASS(1, TL); break;             \
    case 2: ONEPASS(2, TL); break;             \
    case 4: ONEPASS(4, TL); break;             \
    case 8: ONEPASS(8, TL); break;             \
    case 12: ONEPASS(12, TL); break;           \
    case 16: PAIRPASS(16, TL); break;          \
    case 22: PAIRPASS(22, TL); break;          \
    default: return (int)hipErrorInvalidValue; \
  }
    if (a.dtype == NPGA_BF16) {
      ONEPASS_SWITCH(bf16_t)
    } else {
      ONEPASS_SWITCH(float)
    }
#undef ONEPASS_SWITCH
#undef ONEPASS
#undef PAIRPASS
  } else if (a.dtype == NPGA_BF16) {
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


// --------------------------------------------------------------------------
// Batched float64 anchor gradients: G_j = 2 L (L^T x_j) for every target j
// whose last phase converged (the others get G_j = 0), two float64 matrix-core
// GEMMs for the whole batch instead of two streaming passes over L per
// target.  Each product of a float32 (or bfloat16) entry of L with a float64
// entry is formed in float64 by v_mfma_f64_16x16x4f64, as in the per-target
// kernels above; only the order of the float64 sums differs.
//   U^T (m x T)  = X^T L      contraction over the n assets
//   G^T (m x n)  = U^T L^T    contraction over the T periods, split in
//                             ranges of kc periods, one float64 partial
//                             G^T per range, summed in range order
// Tiles of 64 targets x 64 periods (or assets), four wavefronts of 32 x 32
// (2 x 2 blocks of 16 x 16), 16-deep stages double-buffered in LDS.
// --------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int PT = 64;
constexpr int PK = 16;

// Four entries of column col of L from row i (i % 4 == 0), zero past n.
// i < n <= ld and ld % 4 == 0 keep the 16-byte (8-byte for bfloat16) load
// inside the column.
template <typename TL>
__device__ __forceinline__ f4 load_l4(const TL *L, int64_t ld, int64_t n, int64_t col, int64_t i) {
  f4 v = f4{0.f, 0.f, 0.f, 0.f};
  if (i < n) {
    v = load4_nt<TL>(L + col * ld + i);
    if (i + 1 >= n) v.y = 0.f;
    if (i + 2 >= n) v.z = 0.f;
    if (i + 3 >= n) v.w = 0.f;
  }
  return v;
}

// The 4 x 16 x 16 MFMA steps of one stage for a 32 x 32 wavefront tile:
// A rows (targets) from As, B columns from Bs, lane l supplying row or
// column l % 16 at contraction index kk + l / 16.
__device__ __forceinline__ void prec_stage(const double (*As)[PT + 1], const double (*Bs)[PT + 1], int lane,
                                           int wr, int wc, d4 (&acc)[2][2]) {
#pragma unroll
  for (int kk = 0; kk < PK; kk += 4) {
    const int kr = kk + (lane >> 4);
    double av[2], bv[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) av[p] = As[kr][wr * 32 + p * 16 + (lane & 15)];
#pragma unroll
    for (int q = 0; q < 2; ++q) bv[q] = Bs[kr][wc * 32 + q * 16 + (lane & 15)];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
  }
}

// U^T = X^T L.  Grid: (period tiles, target tiles).  Target j's column of X
// is read only when st[j].done == kConverged.
template <typename TL>
__global__ __launch_bounds__(256) void k_bprec_u(const TL *L, int64_t ld, int64_t n, int64_t T, const double *X,
                                                 int64_t ldxv, int32_t m, const DevState *st, double *Ut,
                                                 int64_t ldu) {
  __shared__ double Xs[2][PK][PT + 1];
  __shared__ double Ls[2][PK][PT + 1];
  const int j0 = blockIdx.y * PT;
  const int64_t t0 = (int64_t)blockIdx.x * PT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  // loader: column tid / 4 of each panel, rows 4 (tid % 4) .. +3 of a stage
  const int col = tid >> 2, fi = tid & 3;
  const int jl = j0 + col;
  const bool live = jl < m && st[jl].done == kConverged;
  const double *xc = X + (int64_t)jl * ldxv;
  const int64_t tl = t0 + col;
  double xr[4];
  f4 lr;
  auto gload = [&](int64_t i0) {
    const int64_t i = i0 + 4 * fi;
#pragma unroll
    for (int e = 0; e < 4; ++e) xr[e] = (live && i + e < n) ? xc[i + e] : 0.0;
    lr = (tl < T) ? load_l4<TL>(L, ld, n, tl, i) : f4{0.f, 0.f, 0.f, 0.f};
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) Xs[buf][4 * fi + e][col] = xr[e];
    Ls[buf][4 * fi + 0][col] = (double)lr.x;
    Ls[buf][4 * fi + 1][col] = (double)lr.y;
    Ls[buf][4 * fi + 2][col] = (double)lr.z;
    Ls[buf][4 * fi + 3][col] = (double)lr.w;
  };
  d4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t nst = (n + PK - 1) / PK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t s = 0; s < nst; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nst) gload((s + 1) * PK);
    prec_stage(Xs[buf], Ls[buf], lane, wr, wc, acc);
    if (s + 1 < nst) sstore(buf ^ 1);
    __syncthreads();
  }
  // float64 16 x 16 output: lane l, register v -> row l / 16 + 4 v, column l % 16
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = j0 + wr * 32 + p * 16 + (lane >> 4) + 4 * v;
        const int64_t t = t0 + wc * 32 + q * 16 + (lane & 15);
        if (j < m && t < T) Ut[(int64_t)j * ldu + t] = acc[p][q][v];
      }
}

// Partial G^T over periods [z kc, min(T, (z + 1) kc)).  Grid: (target tiles,
// asset tiles, period ranges).  Out: P[(z m + j) npad + i].
template <typename TL>
__global__ __launch_bounds__(256) void k_bprec_g(const TL *L, int64_t ld, int64_t n, int64_t T, const double *Ut,
                                                 int64_t ldu, int32_t m, int64_t kc, double *P, int64_t npad) {
  __shared__ double Us[2][PK][PT + 1];
  __shared__ double Ls[2][PK][PT + 1];
  const int j0 = blockIdx.x * PT;
  const int64_t i0 = (int64_t)blockIdx.y * PT;
  const int64_t tb = (int64_t)blockIdx.z * kc;
  const int64_t te = (tb + kc < T) ? tb + kc : T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  // U loader: target tid / 4, periods 4 (tid % 4) .. +3 of a stage;
  // L loader: period tid / 16 of a stage, assets 4 (tid % 16) .. +3
  const int col = tid >> 2, fi = tid & 3;
  const int ju = j0 + col;
  const double *uc = Ut + (int64_t)ju * ldu;
  const int kt = tid >> 4, i4 = 4 * (tid & 15);
  double ur[4];
  f4 lr;
  auto gload = [&](int64_t t) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t te4 = t + 4 * fi + e;
      ur[e] = (ju < m && te4 < te) ? uc[te4] : 0.0;
    }
    const int64_t tt = t + kt;
    lr = (tt < te) ? load_l4<TL>(L, ld, n, tt, i0 + i4) : f4{0.f, 0.f, 0.f, 0.f};
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) Us[buf][4 * fi + e][col] = ur[e];
    Ls[buf][kt][i4 + 0] = (double)lr.x;
    Ls[buf][kt][i4 + 1] = (double)lr.y;
    Ls[buf][kt][i4 + 2] = (double)lr.z;
    Ls[buf][kt][i4 + 3] = (double)lr.w;
  };
  d4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t nst = (te - tb + PK - 1) / PK;
  if (nst > 0) {
    gload(tb);
    sstore(0);
  }
  __syncthreads();
  for (int64_t s = 0; s < nst; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nst) gload(tb + (s + 1) * PK);
    prec_stage(Us[buf], Ls[buf], lane, wr, wc, acc);
    if (s + 1 < nst) sstore(buf ^ 1);
    __syncthreads();
  }
  double *out = P + (int64_t)blockIdx.z * m * npad;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = j0 + wr * 32 + p * 16 + (lane >> 4) + 4 * v;
        const int64_t i = i0 + wc * 32 + q * 16 + (lane & 15);
        if (j < m && i < n) out[(int64_t)j * npad + i] = acc[p][q][v];
      }
}

// G[j ldg + i] = 2 sum_z P[(z m + j) npad + i], ranges added in order.
__global__ __launch_bounds__(256) void k_bprec_reduce(const double *P, int32_t splits, int32_t m, int64_t npad,
                                                      int64_t n, double *G, int64_t ldg) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += P[((int64_t)z * m + j) * npad + i];
  G[(int64_t)j * ldg + i] = 2.0 * s;
}

PreciseBatchPlan precise_batch_plan(int64_t n, int64_t T, int32_t m) {
  PreciseBatchPlan p{};
  const int64_t tiles = ((m + PT - 1) / PT) * ((n + PT - 1) / PT);
  int64_t want = (512 + tiles - 1) / tiles;
  if (want > 32) want = 32;
  const int64_t cap = (T + 8 * PK - 1) / (8 * PK);  // ranges of at least 8 stages
  if (want > cap) want = cap;
  if (want < 1) want = 1;
  p.kc = ((T + want - 1) / want + PK - 1) / PK * PK;
  p.splits = (int32_t)((T + p.kc - 1) / p.kc);
  p.ldu = (T + 1) / 2 * 2;
  p.u_bytes = sizeof(double) * (size_t)m * (size_t)p.ldu;
  return p;
}

size_t precise_batch_bytes(int64_t n, int64_t T, int32_t m, int64_t npad) {
  const PreciseBatchPlan p = precise_batch_plan(n, T, m);
  return (p.u_bytes + 255) / 256 * 256 + sizeof(double) * (size_t)p.splits * (size_t)m * (size_t)npad;
}

int launch_precise_gradient_batched(const void *L, int32_t dtype, int64_t ld, int64_t n, int64_t T,
                                    const double *X, int64_t ldxv, int32_t m, const DevState *st, double *scratch,
                                    int64_t npad, double *G, int64_t ldg, hipStream_t s) {
  if (m < 1 || n < 1 || T < 1 || npad < n || ld < n || (ld % 4) != 0) return (int)hipErrorInvalidValue;
  const PreciseBatchPlan p = precise_batch_plan(n, T, m);
  double *Ut = scratch;
  double *P = scratch + (p.u_bytes + 255) / 256 * 256 / sizeof(double);
  if ((T + PT - 1) / PT > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  const dim3 gu((unsigned)((T + PT - 1) / PT), (unsigned)((m + PT - 1) / PT));
  const dim3 gg((unsigned)((m + PT - 1) / PT), (unsigned)((n + PT - 1) / PT), (unsigned)p.splits);
  if (dtype == NPGA_BF16) {
    const bf16_t *Lb = static_cast<const bf16_t *>(L);
    hipLaunchKernelGGL(k_bprec_u<bf16_t>, gu, dim3(256), 0, s, Lb, ld, n, T, X, ldxv, m, st, Ut, p.ldu);
    hipLaunchKernelGGL(k_bprec_g<bf16_t>, gg, dim3(256), 0, s, Lb, ld, n, T, Ut, p.ldu, m, p.kc, P, npad);
  } else {
    const float *Lf = static_cast<const float *>(L);
    hipLaunchKernelGGL(k_bprec_u<float>, gu, dim3(256), 0, s, Lf, ld, n, T, X, ldxv, m, st, Ut, p.ldu);
    hipLaunchKernelGGL(k_bprec_g<float>, gg, dim3(256), 0, s, Lf, ld, n, T, Ut, p.ldu, m, p.kc, P, npad);
  }
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
  hipLaunchKernelGGL(k_bprec_reduce, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0, s, P, p.splits, m,
                     npad, n, G, ldg);
  return (int)hipGetLastError();
}

}  // namespace npga
