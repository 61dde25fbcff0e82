// Explicit-covariance path (paper Sec. 3.1: grad f(x) = 2 Sigma x at O(n^2)
// per iteration).
//
// k_syrk: Sigma = L L^T with float32 MFMA (v_mfma_f32_32x32x2_f32).  One
// workgroup computes a 128 x 128 tile of the lower triangle (eight
// wavefronts, 32 x 64 each as 1 x 2 MFMA blocks) and also writes the
// mirrored tile, so Sigma is stored full.  Columns of L (periods) are the
// reduction dimension; 32-period slices of both row panels are staged in
// LDS (double buffered).  The float32 MFMA accumulators are flushed into
// float64 registers every 256 periods, which bounds the float32 rounding
// to partial sums of 256 products.
//
// k_symv_tail: g = 2 Sigma x + 2 gamma x.  Sigma is symmetric, so
// (Sigma x)_i is the dot product of column i with x; every wavefront owns
// whole columns (contiguous) and writes g_i directly.  The last workgroup
// (atomic ticket) then runs the same NPGA tail as the factor path.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"

namespace npga {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kTile = 128;
constexpr int kKB = 32;          // periods per LDS stage
constexpr int kFlushStages = 8;  // float32 -> float64 flush every 256 periods

__global__ __launch_bounds__(512) void k_syrk(const float *__restrict__ L, int64_t n, int64_t T, int64_t ld,
                                              float *__restrict__ S, int64_t lds, int nb) {
  __shared__ float As[2][kKB][kTile];
  __shared__ float Bs[2][kKB][kTile];
  // triangular tile index from blockIdx; the eight XCDs receive
  // consecutive workgroups round-robin, so give each XCD a contiguous
  // range of tiles (tiles sharing a row panel) for L2 reuse
  const int ntiles = nb * (nb + 1) / 2;
  const int b = blockIdx.x;
  const int per_xcd = (ntiles + 7) / 8;
  const int tix = (b % 8) * per_xcd + (b / 8);
  if (tix >= ntiles) return;  // the map is a bijection of [0, 8 per_xcd); skip the padding
  int bi = 0;
  while ((bi + 1) * (bi + 2) / 2 <= tix) ++bi;
  const int bj = tix - bi * (bi + 1) / 2;
  const int64_t row_a = (int64_t)bi * kTile;
  const int64_t row_b = (int64_t)bj * kTile;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;  // rows wr*32.., columns wc*64..

  v16f acc[2];
  double acc64[2][16];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      acc[q][v] = 0.f;
      acc64[q][v] = 0.0;
    }

  // global -> register staging: thread loads float4 index (tid % 32) of
  // columns (tid / 32) + 16 q, q = 0..1, for both panels
  const int f4i = tid & 31;
  const int colq = tid >> 5;
  f4 ra[2], rb[2];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int64_t t = k0 + colq + 16 * q;
      const int64_t ra0 = row_a + 4 * f4i;
      const int64_t rb0 = row_b + 4 * f4i;
      f4 za = f4{0.f, 0.f, 0.f, 0.f}, zb = za;
      if (t < T) {
        if (ra0 < n) {
          za = *reinterpret_cast<const f4 *>(L + t * ld + ra0);
          if (ra0 + 1 >= n) za.y = 0.f;
          if (ra0 + 2 >= n) za.z = 0.f;
          if (ra0 + 3 >= n) za.w = 0.f;
        }
        if (rb0 < n) {
          zb = *reinterpret_cast<const f4 *>(L + t * ld + rb0);
          if (rb0 + 1 >= n) zb.y = 0.f;
          if (rb0 + 2 >= n) zb.z = 0.f;
          if (rb0 + 3 >= n) zb.w = 0.f;
        }
      }
      ra[q] = za;
      rb[q] = zb;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      *reinterpret_cast<f4 *>(&As[buf][colq + 16 * q][4 * f4i]) = ra[q];
      *reinterpret_cast<f4 *>(&Bs[buf][colq + 16 * q][4 * f4i]) = rb[q];
    }
  };

  const int64_t nstages = (T + kKB - 1) / kKB;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t s = 0; s < nstages; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nstages) gload((s + 1) * kKB);
#pragma unroll
    for (int kk = 0; kk < kKB; kk += 2) {
      const int kr = kk + (lane >> 5);
      const float av = As[buf][kr][wr * 32 + (lane & 31)];
      float bv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) bv[q] = Bs[buf][kr][wc * 64 + q * 32 + (lane & 31)];
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[q], acc[q], 0, 0, 0);
    }
    if (((s + 1) % kFlushStages) == 0 || s + 1 == nstages) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          acc64[q][v] += (double)acc[q][v];
          acc[q][v] = 0.f;
        }
    }
    if (s + 1 < nstages) {
      sstore(buf ^ 1);
    }
    __syncthreads();
  }

  // write the tile and its mirror.  MFMA 32x32 output layout: lane l,
  // register v -> row 8 (v/4) + 4 (l/32) + (v%4), column l%32.
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t r = row_a + wr * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const int64_t c = row_b + wc * 64 + q * 32 + (lane & 31);
      if (r < n && c < n) {
        const float val = (float)acc64[q][v];
        S[r + c * lds] = val;
        if (bi != bj) S[c + r * lds] = val;
      }
    }
}

// g = 2 Sigma x (+ 2 gamma x); the serial tail runs as a separate launch.
// A wavefront per column, the next column's loads in flight while the
// current one is reduced (Sigma, 118 MB at n = 5440, stays in the MALL
// between iterations, so the loads are ordinary cached ones).
template <int E>
__global__ __launch_bounds__(256) void k_symv(SolveArgs a, const float *__restrict__ S, int64_t lds) {
  DevState *st = a.st;
  if (st->done != kRunning) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t n = a.n;
  const int64_t W = (int64_t)gridDim.x * 4;
  const bool ragged = (n & 3) != 0;
  f4 xr[E];
#pragma unroll
  for (int j = 0; j < E; ++j) xr[j] = *reinterpret_cast<const f4 *>(a.xs + 4 * lane + 256 * j);
  const int cur = (a.mode == kTailNpga) ? (st->iter & 1) : 0;
  const double *xk = cur ? a.xbuf1 : a.xbuf0;
  double *gk = (a.mode == kTailNpga) ? (cur ? a.gbuf1 : a.gbuf0) : a.gbuf0;
  const double *pv = a.pvec;
  auto load = [&](f4(&c)[E], int64_t col) {
    const f4 *p = reinterpret_cast<const f4 *>(S + col * lds) + lane;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t row0 = 4 * lane + 256 * j;
      c[j] = (row0 < n) ? p[64 * j] : f4{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto process = [&](f4(&c)[E], int64_t col) {
    float d = 0.f;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t row0 = 4 * lane + 256 * j;
      if (ragged) {
        if (row0 + 1 >= n) c[j].y = 0.f;
        if (row0 + 2 >= n) c[j].z = 0.f;
        if (row0 + 3 >= n) c[j].w = 0.f;
      }
      d = fmaf(c[j].x, xr[j].x, d);
      d = fmaf(c[j].y, xr[j].y, d);
      d = fmaf(c[j].z, xr[j].z, d);
      d = fmaf(c[j].w, xr[j].w, d);
    }
    d = wave_sum_f32(d);
    if (lane == 0) {
      if (a.mode == kTailPower || a.mode == kTailLanczos)
        gk[col] = (double)d;
      else if (a.mode == kTailCG || a.mode == kTailAdj)
        gk[col] = 2.0 * (double)d + 2.0 * st->gamma * pv[col];
      else
        gk[col] = 2.0 * (double)d + (a.ga ? a.ga[col] : 0.0) + 2.0 * st->gamma * xk[col];
    }
  };
  f4 c0[E], c1[E];
  int64_t col = (int64_t)blockIdx.x * 4 + wave;
  if (col < n) load(c0, col);
  while (col < n) {
    const int64_t col1 = col + W;
    if (col1 < n) load(c1, col1);
    process(c0, col);
    if (col1 >= n) break;
    const int64_t col2 = col1 + W;
    if (col2 < n) load(c0, col2);
    process(c1, col1);
    col = col2;
  }
}

int launch_syrk(const float *L, int64_t n, int64_t T, int64_t ld, float *Sigma, int64_t lds,
                hipStream_t s) {
  const int nb = (int)((n + kTile - 1) / kTile);
  const int ntiles = nb * (nb + 1) / 2;
  const int grid = ((ntiles + 7) / 8) * 8;
  hipLaunchKernelGGL(k_syrk, dim3(grid), dim3(512), 0, s, L, n, T, ld, Sigma, lds, nb);
  return (int)hipGetLastError();
}

#define SYMV_SLOT_SWITCH(slots, CALL)            \
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

int launch_symv(const SolveArgs &a, const float *Sigma, int64_t lds, int slots, hipStream_t s) {
#define CALL(E) hipLaunchKernelGGL(k_symv<E>, dim3(a.sweep_grid), dim3(256), 0, s, a, Sigma, lds)
  SYMV_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_symv_tail(const SolveArgs &a, const float *Sigma, int64_t lds, int slots, hipStream_t s) {
  if (launch_symv(a, Sigma, lds, slots, s)) return (int)hipErrorLaunchFailure;
  return launch_tail(a, slots, 1, s);
}

}  // namespace npga
