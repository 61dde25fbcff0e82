// Sketch-Truncate-Ridge factor build (paper Sec. 2.5; App. D):
//     Y = L S                      sketch stage (S T x k, N(0, 1/k) entries)
//     Y = U Sig V^T, keep ell      truncation stage (top-ell right singular space)
//     L_eff = Y V_ell = U_ell Sig_ell   (App. D, "STR as one sketch")
//     gamma = c trace(Y Y^T) / n   ridge stage with the untruncated sketch
//
// The right singular space of Y is the top-ell eigenspace of the Gram
// matrix G = Y^T Y (k x k).  It is computed by a dense symmetric
// eigensolver written for the GPU (float64 throughout):
//   1. G by float64 MFMA (exact products of the float32 entries of Y);
//   2. Householder tridiagonalisation G = Q T Q^T, one reflector per step
//      (a one-workgroup kernel forms the reflector, a grid kernel applies the
//      previous rank-2 update to the trailing columns and forms the next
//      symmetric matrix-vector product in the same pass);
//   3. the ell largest eigenvalues of T by bisection on Sturm counts;
//   4. their eigenvectors of T by inverse iteration (tridiagonal LU with
//      partial pivoting);
//   5. back-transformation V = Q Z by the stored reflectors.
// The products Y = L S and L_eff = Y V use float32 MFMA with float64
// accumulation across k-chunks.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"
#include "npga_sketch.h"

namespace npga {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));

// --------------------------------------------------------------------------
// float32 MFMA GEMM  C (M x N, column-major, ldc) = A B
//   A element (m, k): A[m + k lda] (rows contiguous, e.g. L or Y)
//   B element (k, n): B[k + n ldb] (k contiguous, e.g. S or V)
// 128 x 128 tiles, eight wavefronts of 32 x 64 (1 x 2 v_mfma_f32_32x32x2_f32
// blocks; the small per-wavefront accumulator set leaves room for two
// wavefronts per SIMD), 32-deep k slices double buffered in LDS, float64
// flush every 64 k.
// --------------------------------------------------------------------------
constexpr int GT = 128;
constexpr int GK = 32;
constexpr int GPAD = 129;

__global__ __launch_bounds__(512) void k_gemm_f32(const float *__restrict__ A, int64_t lda,
                                                  const float *__restrict__ B, int64_t ldb,
                                                  float *__restrict__ C, int64_t ldc, int64_t M,
                                                  int64_t N, int64_t K) {
  __shared__ float As[2][GK][GT];
  __shared__ float Bs[2][GK][GPAD];
  const int64_t nbm = (M + GT - 1) / GT;
  const int64_t bm = blockIdx.x % nbm;
  const int64_t bn = blockIdx.x / nbm;
  const int64_t m0 = bm * GT, n0 = bn * GT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
  // A loader (rows contiguous): float4 index (tid % 32) of k-columns tid/32 + 16 q
  // B loader (k contiguous): column tid/8 + 64 q, float4 index (tid % 8) along k
  f4 ra[2], rb[2];
  const bool bvec = (ldb % 4) == 0 && (reinterpret_cast<uintptr_t>(B) % 16) == 0;
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int64_t kk = k0 + (tid >> 5) + 16 * q;
      const int64_t mm = m0 + 4 * (tid & 31);
      f4 z = f4{0.f, 0.f, 0.f, 0.f};
      if (kk < K && mm < M) {
        z = *reinterpret_cast<const f4 *>(A + kk * lda + mm);
        if (mm + 1 >= M) z.y = 0.f;
        if (mm + 2 >= M) z.z = 0.f;
        if (mm + 3 >= M) z.w = 0.f;
      }
      ra[q] = z;
      const int64_t nn = n0 + (tid >> 3) + 64 * q;
      const int64_t kb = k0 + 4 * (tid & 7);
      f4 zb = f4{0.f, 0.f, 0.f, 0.f};
      if (nn < N) {
        const float *bp = B + nn * ldb + kb;
        if (bvec && kb + 3 < K) {
          zb = *reinterpret_cast<const f4 *>(bp);
        } else {
          if (kb < K) zb.x = bp[0];
          if (kb + 1 < K) zb.y = bp[1];
          if (kb + 2 < K) zb.z = bp[2];
          if (kb + 3 < K) zb.w = bp[3];
        }
      }
      rb[q] = zb;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      *reinterpret_cast<f4 *>(&As[buf][(tid >> 5) + 16 * q][4 * (tid & 31)]) = ra[q];
      const int c = (tid >> 3) + 64 * q;
      const int kb = 4 * (tid & 7);
      Bs[buf][kb + 0][c] = rb[q].x;
      Bs[buf][kb + 1][c] = rb[q].y;
      Bs[buf][kb + 2][c] = rb[q].z;
      Bs[buf][kb + 3][c] = rb[q].w;
    }
  };
  const int64_t nst = (K + GK - 1) / GK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t s = 0; s < nst; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nst) gload((s + 1) * GK);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 2) {
      const int kr = kk + (lane >> 5);
      const float av = As[buf][kr][wr * 32 + (lane & 31)];
      float bv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) bv[q] = Bs[buf][kr][wc * 64 + q * 32 + (lane & 31)];
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[q], acc[q], 0, 0, 0);
    }
    if ((s & 1) == 1 || s + 1 == nst) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          acc64[q][v] += (double)acc[q][v];
          acc[q][v] = 0.f;
        }
    }
    if (s + 1 < nst) sstore(buf ^ 1);
    __syncthreads();
  }
  // MFMA 32x32 output layout: lane l, register v -> row 8 (v/4) + 4 (l/32) + (v%4), column l%32
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t r = m0 + wr * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const int64_t c = n0 + wc * 64 + q * 32 + (lane & 31);
      if (r < M && c < N) C[r + c * ldc] = (float)acc64[q][v];
    }
}

// --------------------------------------------------------------------------
// float64 Gram matrix G = Y^T Y (k x k, column-major, leading dim k), both
// triangles, by v_mfma_f64_16x16x4_f64 on the float32 entries of Y (exact
// products).  64 x 64 tiles of the lower triangle; four wavefronts of
// 32 x 32 (2 x 2 MFMA blocks); 16-deep slices of Y in LDS.
// --------------------------------------------------------------------------
constexpr int HT = 64;
constexpr int HK = 16;

__global__ __launch_bounds__(256) void k_gram_f64(const float *__restrict__ Y, int64_t ldy, int64_t n,
                                                  int64_t k, double *__restrict__ G, int nb) {
  __shared__ double As[2][HK][HT + 1];
  __shared__ double Bs[2][HK][HT + 1];
  const int b = blockIdx.x;
  int bi = 0;
  while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
  const int bj = b - bi * (bi + 1) / 2;
  if (bi >= nb) return;
  const int64_t r0 = (int64_t)bi * HT, c0 = (int64_t)bj * HT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v4d acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = v4d{0.0, 0.0, 0.0, 0.0};
  // loader: column tid/4 of each panel, float4 index tid%4 along n
  const int col = tid >> 2, fi = tid & 3;
  f4 ra, rb;
  auto gload = [&](int64_t a0) {
    const int64_t aa = a0 + 4 * fi;
    ra = f4{0.f, 0.f, 0.f, 0.f};
    rb = ra;
    const int64_t ja = r0 + col, jb = c0 + col;
    if (ja < k) {
      const float *p = Y + ja * ldy + aa;
      if (aa + 3 < n) {
        ra = *reinterpret_cast<const f4 *>(p);
      } else {
        if (aa < n) ra.x = p[0];
        if (aa + 1 < n) ra.y = p[1];
        if (aa + 2 < n) ra.z = p[2];
      }
    }
    if (jb < k) {
      const float *p = Y + jb * ldy + aa;
      if (aa + 3 < n) {
        rb = *reinterpret_cast<const f4 *>(p);
      } else {
        if (aa < n) rb.x = p[0];
        if (aa + 1 < n) rb.y = p[1];
        if (aa + 2 < n) rb.z = p[2];
      }
    }
  };
  auto sstore = [&](int buf) {
    As[buf][4 * fi + 0][col] = (double)ra.x;
    As[buf][4 * fi + 1][col] = (double)ra.y;
    As[buf][4 * fi + 2][col] = (double)ra.z;
    As[buf][4 * fi + 3][col] = (double)ra.w;
    Bs[buf][4 * fi + 0][col] = (double)rb.x;
    Bs[buf][4 * fi + 1][col] = (double)rb.y;
    Bs[buf][4 * fi + 2][col] = (double)rb.z;
    Bs[buf][4 * fi + 3][col] = (double)rb.w;
  };
  const int64_t nst = (n + HK - 1) / HK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t s = 0; s < nst; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nst) gload((s + 1) * HK);
#pragma unroll
    for (int kk = 0; kk < HK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) av[p] = As[buf][kr][wr * 32 + p * 16 + (lane & 15)];
#pragma unroll
      for (int q = 0; q < 2; ++q) bv[q] = Bs[buf][kr][wc * 32 + q * 16 + (lane & 15)];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
    }
    if (s + 1 < nst) sstore(buf ^ 1);
    __syncthreads();
  }
  // float64 16x16 output layout: lane l, register v -> row (l/16) + 4 v, column l%16
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + wr * 32 + p * 16 + (lane >> 4) + 4 * v;
        const int64_t c = c0 + wc * 32 + q * 16 + (lane & 15);
        if (r < k && c < k) {
          G[r + c * k] = acc[p][q][v];
          if (bi != bj) G[c + r * k] = acc[p][q][v];
        }
      }
}

// ||Y||_F^2 = trace(Y^T Y) in float64 (one workgroup per column block, then
// a fixed-order sum).
__global__ __launch_bounds__(256) void k_frob_partial(const float *Y, int64_t ldy, int64_t n, int64_t k,
                                                      double *part) {
  __shared__ double buf[64];
  BlockReducer<5> red{buf, 0};
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t j = blockIdx.x; j < k; j += gridDim.x)
    for (int64_t a = threadIdx.x; a < n; a += 256) {
      const double y = Y[a + j * ldy];
      acc[0] = fma(y, y, acc[0]);
    }
  red.sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// --------------------------------------------------------------------------
// Householder tridiagonalisation, one reflector per step (float64).
// State (SketchState): A = G (k x k, lda k) is overwritten: the reflector
// of step i is kept in A[i+1:, i] (leading 1 explicit), d and e receive T.
//
// Step i, one workgroup of 1024 threads (k_tri_small):
//   w_{i-1} = p - (tau_{i-1}/2)(p^T v_{i-1}) v_{i-1}    (p = tau A v from the
//            previous grid kernel), then column i of the trailing block gets
//            the rank-2 update A <- A - v w^T - w v^T, d_i = A[i, i], and the
//            reflector of x = A[i+1:, i] (LAPACK dlarfg convention):
//            beta = -sign(x_0)||x||, tau = (beta - x_0)/beta,
//            v = [1, x_1:/(x_0 - beta)], e_i = beta.
// Step i, grid (k_tri_tiles): only the lower triangle r >= c > i of the
//   trailing block is kept.  It gets the pending update from step i-1, is
//   written back, and gives p = tau_i A v_i, where every stored entry adds
//   A[r, c] v_r to p_c and, below the diagonal, A[r, c] v_c to p_r.
//   The upper triangle is never read again.
// --------------------------------------------------------------------------
constexpr int kTriThreads = 1024;  // one-workgroup step: 16 wavefronts
constexpr int kTriRows = 8;        // rows per thread (k <= 8192)

// Sum over the 1024-thread workgroup; every thread gets the same bits (the
// sixteen wave totals are added in wave order).  buf: 2 x 16 doubles.
__device__ __forceinline__ double tri_block_sum(double v, double *buf, int &parity) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum_f64(v);
  double *b = buf + 16 * parity;
  if (lane == 0) b[wave] = v;
  __syncthreads();
  double t = b[0];
#pragma unroll
  for (int w = 1; w < 16; ++w) t += b[w];
  parity ^= 1;
  return t;
}

__global__ __launch_bounds__(kTriThreads) void k_tri_small(SketchState s, int64_t i) {
  __shared__ double buf[32];
  __shared__ double x0s, wis, vis;
  int parity = 0;
  const int64_t k = s.k;
  double *A = s.A;
  double *coli = A + i * k;
  const int tid = threadIdx.x;
  // thread t owns rows r_q = i + t + 1024 q of column i, held in registers
  // through every phase of the step
  double c[kTriRows], vp[kTriRows], wp[kTriRows];
#pragma unroll
  for (int q = 0; q < kTriRows; ++q) {
    const int64_t r = i + tid + (int64_t)kTriThreads * q;
    c[q] = (r < k) ? coli[r] : 0.0;
  }
  if (i > 0) {
    // w_{i-1} = p - (tau_{i-1}/2)(p^T v_{i-1}) v_{i-1} over rows >= i
    double pr[kTriRows], dot = 0.0;
#pragma unroll
    for (int q = 0; q < kTriRows; ++q) {
      const int64_t r = i + tid + (int64_t)kTriThreads * q;
      pr[q] = (r < k) ? s.p[r] : 0.0;
      vp[q] = (r < k) ? s.vcur[r] : 0.0;
      dot = fma(pr[q], vp[q], dot);
    }
    const double half = 0.5 * s.tau[i - 1] * tri_block_sum(dot, buf, parity);
#pragma unroll
    for (int q = 0; q < kTriRows; ++q) {
      const int64_t r = i + tid + (int64_t)kTriThreads * q;
      wp[q] = pr[q] - half * vp[q];
      if (r < k) {
        s.wprev[r] = wp[q];
        s.vprev[r] = vp[q];
      }
    }
    // rank-2 update of column i with the entries at row i (thread 0, q = 0)
    if (tid == 0) {
      wis = wp[0];
      vis = vp[0];
    }
    __syncthreads();
    const double wi = wis, vi = vis;
#pragma unroll
    for (int q = 0; q < kTriRows; ++q) {
      const int64_t r = i + tid + (int64_t)kTriThreads * q;
      c[q] -= vp[q] * wi + wp[q] * vi;
      if (r < k) coli[r] = c[q];
    }
  }
  if (tid == 0) s.d[i] = c[0];
  if (i >= k - 1) return;
  // reflector of x = A[i+1:, i] (x_0 is row i+1: thread 1, q = 0)
  if (tid == 1) x0s = c[0];
  double xn = 0.0;
#pragma unroll
  for (int q = 0; q < kTriRows; ++q) {
    const int64_t r = i + tid + (int64_t)kTriThreads * q;
    if (r >= i + 2 && r < k) xn = fma(c[q], c[q], xn);
  }
  const double xn2 = tri_block_sum(xn, buf, parity);  // its barrier also publishes x0s
  const double x0 = x0s;
  double tau = 0.0, beta = x0, scale = 0.0;
  if (xn2 > 0.0) {
    beta = -copysign(sqrt(x0 * x0 + xn2), x0);
    tau = (beta - x0) / beta;
    scale = 1.0 / (x0 - beta);
  }
#pragma unroll
  for (int q = 0; q < kTriRows; ++q) {
    const int64_t r = i + tid + (int64_t)kTriThreads * q;
    if (r >= i + 1 && r < k) {
      const double v = (r == i + 1) ? 1.0 : ((tau != 0.0) ? c[q] * scale : 0.0);
      s.vcur[r] = v;
      coli[r] = v;
    }
  }
  if (tid == 0) {
    s.e[i] = beta;
    s.tau[i] = tau;
  }
}

// k_tri_tiles: one workgroup per 64 x 64 tile (I, J), I >= J, of the
// trailing lower triangle; lane = row of the tile, wavefront w = columns
// 16 w .. 16 w + 15.  A tile writes its 64 column sums (for block J) and 64
// row sums (for block I) to `work`.  k_tri_reduce: one workgroup per block
// adds that block's partial sums in a fixed order and writes p for its
// rows.  (Letting the last tile of a block do its sum inside k_tri_tiles
// needs a device-scope release fence per tile, an L2 write-back on its XCD;
// measured, that costs four times the launch it saves.)
constexpr int kTT = 64;  // tile edge

__device__ __forceinline__ int64_t tri_tile_index(int64_t a, int64_t b) { return a * (a + 1) / 2 + b; }

size_t tri_scratch_bytes(int64_t k) {
  const int64_t nb = (k + kTT - 1) / kTT;
  return sizeof(double) * 2 * (size_t)(nb * (nb + 1) / 2) * kTT;
}

__global__ __launch_bounds__(256) void k_tri_tiles(SketchState s, int64_t i, int64_t tiles_max) {
  __shared__ double prod[kTT][kTT + 1];
  __shared__ double rowp[4][kTT], colp[4][kTT];
  __shared__ double cv[kTT], cvp[kTT], cwp[kTT];
  const int64_t k = s.k;
  double *A = s.A;
  double *prow = s.work;                   // tiles_max x 64 row sums
  double *pcol = s.work + tiles_max * kTT;  // tiles_max x 64 column sums
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t J0 = (i + 1) / kTT;
  // tile t = Ir (Ir + 1) / 2 + Jr of the block indices relative to J0
  const int64_t t = blockIdx.x;
  int64_t Ir = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (tri_tile_index(Ir + 1, 0) <= t) ++Ir;
  while (tri_tile_index(Ir, 0) > t) --Ir;
  const int64_t Jr = t - tri_tile_index(Ir, 0);
  const int64_t r0 = (J0 + Ir) * kTT, c0 = (J0 + Jr) * kTT;
  const bool upd = i > 0;
  if (tid < kTT) {
    const int64_t c = c0 + tid;
    const bool ok = c > i && c < k;
    cv[tid] = ok ? s.vcur[c] : 0.0;
    cvp[tid] = (ok && upd) ? s.vprev[c] : 0.0;
    cwp[tid] = (ok && upd) ? s.wprev[c] : 0.0;
  }
  const int64_t r = r0 + lane;
  const bool rok = r > i && r < k;
  const double rv = rok ? s.vcur[r] : 0.0;
  const double rvp = (rok && upd) ? s.vprev[r] : 0.0;
  const double rwp = (rok && upd) ? s.wprev[r] : 0.0;
  double a[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int64_t c = c0 + 16 * w + j;
    const bool ok = rok && c > i && r >= c;
    a[j] = ok ? A[r + c * k] : 0.0;
  }
  __syncthreads();  // cv, cvp, cwp
  double racc = 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int cl = 16 * w + j;
    const int64_t c = c0 + cl;
    const bool ok = rok && c > i && r >= c;
    if (upd && ok) {
      a[j] -= rvp * cwp[cl] + rwp * cvp[cl];
      A[r + c * k] = a[j];
    }
    prod[lane][cl] = a[j] * rv;                   // to p_c (diagonal included)
    if (r > c) racc = fma(a[j], cv[cl], racc);  // to p_r (a[j] = 0 off the triangle)
  }
  rowp[w][lane] = racc;
  __syncthreads();
  {
    const int cl = tid & 63, g = tid >> 6;
    double cs = 0.0;
#pragma unroll
    for (int l = 0; l < 16; ++l) cs += prod[16 * g + l][cl];
    colp[g][cl] = cs;
  }
  __syncthreads();
  if (tid < kTT) {
    prow[t * kTT + tid] = ((rowp[0][tid] + rowp[1][tid]) + rowp[2][tid]) + rowp[3][tid];
    pcol[t * kTT + tid] = ((colp[0][tid] + colp[1][tid]) + colp[2][tid]) + colp[3][tid];
  }
}

// Block X (relative to J0): row sums of tiles (X, 0..X), then column sums
// of tiles (X..nbr-1, X), in sixteen interleaved groups added in group
// order.
__global__ __launch_bounds__(1024) void k_tri_reduce(SketchState s, int64_t i, int64_t nbr, int64_t tiles_max) {
  __shared__ double part[16][kTT];
  const double *prow = s.work, *pcol = s.work + tiles_max * kTT;
  const int tid = threadIdx.x, lane = tid & 63, g = tid >> 6;
  const int64_t X = blockIdx.x;
  double acc = 0.0;
  for (int64_t q = g; q <= nbr; q += 16)
    acc += (q <= X) ? prow[tri_tile_index(X, q) * kTT + lane] : pcol[tri_tile_index(q - 1, X) * kTT + lane];
  part[g][lane] = acc;
  __syncthreads();
  if (tid < kTT) {
    const int64_t rr = ((i + 1) / kTT + X) * kTT + tid;
    double tot = part[0][tid];
#pragma unroll
    for (int u = 1; u < 16; ++u) tot += part[u][tid];
    if (rr > i && rr < s.k) s.p[rr] = s.tau[i] * tot;
  }
}

// --------------------------------------------------------------------------
// The ell largest eigenvalues of the symmetric tridiagonal T (d, e) by
// multisection on Sturm counts (number of eigenvalues below x from the
// signs of the LDL^T pivots).  One wavefront per eigenvalue: each round its
// 64 lanes count at 64 interior points of the current interval and the cell
// where the count passes the eigenvalue's index is kept, so a round shrinks
// the interval 65-fold where bisection halves it.  Four eigenvalues per
// workgroup share d and e^2 in LDS.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bisect(SketchState s, int64_t ell) {
  extern __shared__ double sm[];
  const int64_t k = s.k;
  double *dd = sm;
  double *ee = sm + k;  // e_i^2
  __shared__ double bnd[64];
  double lo = 1e308, hi = -1e308;
  for (int64_t i = threadIdx.x; i < k; i += 256) {
    dd[i] = s.d[i];
    const double el = (i > 0) ? fabs(s.e[i - 1]) : 0.0;
    const double er = (i + 1 < k) ? fabs(s.e[i]) : 0.0;
    if (i + 1 < k) ee[i] = s.e[i] * s.e[i];
    lo = fmin(lo, s.d[i] - el - er);
    hi = fmax(hi, s.d[i] + el + er);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    bnd[wave] = lo;
    bnd[4 + wave] = hi;
  }
  __syncthreads();
  lo = fmin(fmin(bnd[0], bnd[1]), fmin(bnd[2], bnd[3]));
  hi = fmax(fmax(bnd[4], bnd[5]), fmax(bnd[6], bnd[7]));
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pivmin = 1e-300 + 4.0 * 2.2250738585072014e-308 * tnorm;
  lo -= 2.2e-16 * tnorm + 1e-300;
  hi += 2.2e-16 * tnorm + 1e-300;
  const int64_t j = (int64_t)blockIdx.x * 4 + wave;
  if (j >= ell) return;  // whole wavefronts leave, after the last barrier
  const int64_t m = k - 1 - j;  // ascending index of the j-th largest
  double a = lo, b = hi;         // count(a) <= m < count(b)
  for (int round = 0; round < 64; ++round) {
    const double w = (b - a) / 65.0;
    const double x = a + w * (double)(lane + 1);
    int64_t cnt = 0;  // eigenvalues below x
    double q = dd[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
    for (int64_t i = 1; i < k; ++i) {
      q = dd[i] - x - ee[i - 1] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      if (q < 0.0) ++cnt;
    }
    // first lane whose point lies above the eigenvalue (64: none)
    const unsigned long long above = __ballot(cnt > m);
    const int l = above ? __ffsll((long long)above) - 1 : 64;
    const double na = a + w * (double)l;
    const double nb = (l == 64) ? b : a + w * (double)(l + 1);
    if (!(na > a || nb < b)) break;  // the cells no longer split at this precision
    a = na;
    b = nb;
    if (b - a <= 2.2e-16 * fmax(fabs(a), fabs(b)) + pivmin) break;
  }
  if (lane == 0) s.lam[j] = 0.5 * (a + b);
}

// --------------------------------------------------------------------------
// Eigenvectors of T for the computed eigenvalues by inverse iteration: LU
// of T - lambda I with partial pivoting (the LAPACK dgttrf/dgttrs scheme),
// three solves from a hashed start vector, normalisation.  One thread per
// eigenvalue; the factor arrays are interleaved across threads so each
// step is a coalesced access.  The recurrences carry the entries they pass
// from row to row in registers (the arrays are only written, or read ahead
// of the chain), so a step costs its arithmetic rather than a memory round
// trip; the U solve multiplies by reciprocal pivots kept by the factorisation.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mixh(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr int kIB = 16;  // rows whose inputs are loaded ahead of the recurrence

__global__ __launch_bounds__(64) void k_inverse_iter(SketchState s, int64_t ell, int64_t stride) {
  const int64_t k = s.k;
  const double *__restrict__ d = s.d;
  const double *__restrict__ e = s.e;
  // ||T||_inf bound (the same for every eigenvalue): the wavefront's lanes
  // split the rows, then a wave maximum
  double tnorm = 0.0;
  for (int64_t i = threadIdx.x; i < k; i += 64)
    tnorm = fmax(tnorm, fabs(d[i]) + ((i > 0) ? fabs(e[i - 1]) : 0.0) + ((i + 1 < k) ? fabs(e[i]) : 0.0));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) tnorm = fmax(tnorm, __shfl_xor(tnorm, off, 64));
  const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (j >= ell) return;
  const double lam = s.lam[j];
  double *__restrict__ frd = s.work;               // reciprocal of the U diagonal
  double *__restrict__ fu = s.work + stride * k;   // first superdiagonal of U
  double *__restrict__ fu2 = s.work + 2 * stride * k;
  double *__restrict__ fl = s.work + 3 * stride * k;  // multipliers
  double *__restrict__ bv = s.work + 4 * stride * k;  // right-hand side / solution
  uint8_t *__restrict__ piv = reinterpret_cast<uint8_t *>(s.work + 5 * stride * k);
#define IX(i) ((i) * stride + j)
  const double tiny = 2.2e-16 * tnorm + 1e-300;
  auto recip = [&](double u) {
    if (fabs(u) < tiny) u = (u < 0.0) ? -tiny : tiny;
    return 1.0 / u;
  };
  // factor T - lam I = P L U; dcur, ucur: row i of the partly eliminated
  // matrix.  One step, without branches: the row interchange (when the
  // subdiagonal entry is the larger pivot) is a selection.
  double dcur = d[0] - lam;
  double ucur = (k > 1) ? e[0] : 0.0;
  auto fstep = [&](int64_t i, double dnext, double li, double unext) {
    const bool np = fabs(dcur) >= fabs(li);
    const double dv = (dcur != 0.0) ? dcur : tiny;
    const double den = np ? dv : li;
    const double f = (np ? li : dcur) / den;
    frd[IX(i)] = recip(den);
    fl[IX(i)] = f;
    fu[IX(i)] = np ? ucur : dnext;
    fu2[IX(i)] = np ? 0.0 : unext;
    piv[IX(i)] = np ? 0 : 1;
    const double dn = np ? fma(-f, ucur, dnext) : fma(-f, dnext, ucur);
    ucur = np ? unext : -f * unext;
    dcur = dn;
  };
  int64_t i0 = 0;
  for (; i0 + kIB <= k - 1; i0 += kIB) {  // whole blocks: every row index below k - 1
    double dn[kIB], li[kIB], un[kIB];
#pragma unroll
    for (int u = 0; u < kIB; ++u) {
      const int64_t i = i0 + u;
      dn[u] = d[i + 1] - lam;
      li[u] = e[i];
      un[u] = (i + 2 < k) ? e[min(i + 1, k - 2)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kIB; ++u) fstep(i0 + u, dn[u], li[u], un[u]);
  }
  for (int64_t i = i0; i + 1 < k; ++i) fstep(i, d[i + 1] - lam, e[i], (i + 2 < k) ? e[i + 1] : 0.0);
  frd[IX(k - 1)] = recip((dcur != 0.0) ? dcur : tiny);
  // start vector
#pragma unroll 8
  for (int64_t i = 0; i < k; ++i) {
    const uint64_t h = mixh(0x5bd1e995ull * (uint64_t)(j + 1) + (uint64_t)i);
    bv[IX(i)] = ((double)(h >> 11) * (1.0 / 9007199254740992.0)) - 0.5;
  }
  double scale = 1.0;  // the previous solve's normalisation, applied as rows are read
  for (int iter = 0; iter < 3; ++iter) {
    // L solve with the row interchanges; bcur is row i of the running vector
    double bcur = bv[IX(0)] * scale;
    auto lstep = [&](int64_t i, double f, double bn, uint8_t pv) {
      const bool np = pv == 0;
      bv[IX(i)] = np ? bcur : bn;
      bcur = np ? fma(-f, bcur, bn) : fma(-f, bn, bcur);
    };
    int64_t i1 = 0;
    for (; i1 + kIB <= k - 1; i1 += kIB) {
      double f[kIB], bn[kIB];
      uint8_t pv[kIB];
#pragma unroll
      for (int u = 0; u < kIB; ++u) {
        const int64_t i = i1 + u;
        f[u] = fl[IX(i)];
        bn[u] = bv[IX(i + 1)] * scale;
        pv[u] = piv[IX(i)];
      }
#pragma unroll
      for (int u = 0; u < kIB; ++u) lstep(i1 + u, f[u], bn[u], pv[u]);
    }
    for (int64_t i = i1; i + 1 < k; ++i) lstep(i, fl[IX(i)], bv[IX(i + 1)] * scale, piv[IX(i)]);
    bv[IX(k - 1)] = bcur;
    // U solve from the last row, carrying the two rows below
    double b1 = 0.0, b2 = 0.0, nrm = 0.0;
    auto ustep = [&](int64_t i, double bb, double u1, double u2, double rd) {
      const double v = (bb - u1 * b1 - u2 * b2) * rd;
      bv[IX(i)] = v;
      nrm = fmax(nrm, fabs(v));
      b2 = b1;
      b1 = v;
    };
    // rows k-1 and k-2 have no second (and k-1 no first) superdiagonal entry
    int64_t i2 = k - 1;
    for (; i2 >= 0 && i2 + 2 >= k; --i2)
      ustep(i2, bv[IX(i2)], (i2 + 1 < k) ? fu[IX(i2)] : 0.0, 0.0, frd[IX(i2)]);
    for (; i2 + 1 >= kIB; i2 -= kIB) {  // whole blocks of rows i2, i2-1, ..., i2-kIB+1 >= 0
      double bb[kIB], u1[kIB], u2[kIB], rd[kIB];
#pragma unroll
      for (int u = 0; u < kIB; ++u) {
        const int64_t i = i2 - u;
        bb[u] = bv[IX(i)];
        u1[u] = fu[IX(i)];
        u2[u] = fu2[IX(i)];
        rd[u] = frd[IX(i)];
      }
#pragma unroll
      for (int u = 0; u < kIB; ++u) ustep(i2 - u, bb[u], u1[u], u2[u], rd[u]);
    }
    for (; i2 >= 0; --i2) ustep(i2, bv[IX(i2)], fu[IX(i2)], fu2[IX(i2)], frd[IX(i2)]);
    scale = (nrm > 0.0) ? 1.0 / nrm : 1.0;
  }
  double n2 = 0.0;
#pragma unroll 8
  for (int64_t i = 0; i < k; ++i) {
    const double v = bv[IX(i)] * scale;
    n2 = fma(v, v, n2);
  }
  const double inv = scale / sqrt(n2);
#pragma unroll 8
  for (int64_t i = 0; i < k; ++i) s.Z[i + j * k] = bv[IX(i)] * inv;
#undef IX
}

// --------------------------------------------------------------------------
// V = Q Z with Q = H_0 H_1 ... H_{k-2}, the reflectors taken kWY at a time
// in compact WY form (Schreiber-Van Loan; LAPACK dlarft, forward and
// columnwise): H_{i0} ... H_{i0+nb-1} = I - V_b T_b V_b^T with T_b upper
// triangular, T_b[j][j] = tau_j and T_b[0:j, j] = -tau_j T_b[0:j, 0:j]
// (V_b[:, 0:j]^T v_j).  The blocks are applied from the last to the first,
// Z <- Z - V_b (T_b (V_b^T Z)), which needs one workgroup reduction per
// block instead of one per reflector.
// --------------------------------------------------------------------------
constexpr int kWY = 32;

// Entry r of reflector i (stored below the diagonal of A with its leading 1).
__device__ __forceinline__ double refl(const SketchState &s, int64_t i, int64_t r) {
  return (r > i) ? s.A[r + i * s.k] : 0.0;
}

// T_b of every block (one workgroup per block): the Gram matrix of the
// block's reflectors, accumulated over 32-row slices staged in LDS, then the
// triangular recurrence.  Tall: kWY x kWY per block, column-major.
__global__ __launch_bounds__(256) void k_wy_t(SketchState s, double *Tall) {
  __shared__ double Vs[32][kWY + 1];
  __shared__ double G[kWY][kWY + 1];
  __shared__ double Ts[kWY][kWY + 1];
  const int64_t k = s.k;
  const int64_t i0 = (int64_t)blockIdx.x * kWY;
  const int nb = (int)min((int64_t)kWY, k - 1 - i0);
  const int tid = threadIdx.x;
  double g[4] = {0.0, 0.0, 0.0, 0.0};  // entries e = tid + 256 m: (e % 32, e / 32)
  for (int64_t r0 = i0 + 1; r0 < k; r0 += 32) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int rr = tid & 31, jj = (tid >> 5) + 8 * m;
      const int64_t r = r0 + rr;
      Vs[rr][jj] = (jj < nb && r < k) ? refl(s, i0 + jj, r) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int e = tid + 256 * m, p = e & 31, q = e >> 5;
      double acc = g[m];
#pragma unroll 8
      for (int rr = 0; rr < 32; ++rr) acc = fma(Vs[rr][p], Vs[rr][q], acc);
      g[m] = acc;
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int e = tid + 256 * m;
    G[e & 31][e >> 5] = g[m];
    Ts[e & 31][e >> 5] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double tj = s.tau[i0 + j];
    if (tid < j) {
      double acc = 0.0;
      for (int m = tid; m < j; ++m) acc = fma(Ts[tid][m], G[m][j], acc);
      Ts[tid][j] = -tj * acc;
    }
    if (tid == 0) Ts[j][j] = tj;
    __syncthreads();
  }
  double *T = Tall + (int64_t)blockIdx.x * kWY * kWY;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int e = tid + 256 * m;
    T[e] = Ts[e & 31][e >> 5];
  }
}

// Every workgroup owns two columns of Z (in LDS) and applies the blocks.
// Writes V in float32 (k x ell, leading dim k) for the final product.
__global__ __launch_bounds__(256) void k_backtransform(SketchState s, int64_t ell, const double *Tall,
                                                       float *V32) {
  extern __shared__ double zc[];  // 2 k doubles
  __shared__ double buf[2 * 4 * 2 * kWY];
  __shared__ double Tb[kWY * kWY];
  __shared__ double xs[2 * kWY], ys[2 * kWY];
  BlockReducer<2 * kWY> red{buf, 0};
  const int64_t k = s.k;
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * 2;
  const int ncol = (j0 + 1 < ell) ? 2 : 1;
  for (int64_t r = tid; r < k; r += 256) {
    zc[r] = s.Z[r + j0 * k];
    zc[k + r] = (ncol == 2) ? s.Z[r + (j0 + 1) * k] : 0.0;
  }
  const int64_t nblk = (k - 1 + kWY - 1) / kWY;
  for (int64_t b = nblk - 1; b >= 0; --b) {
    const int64_t i0 = b * kWY;
    const int nb = (int)min((int64_t)kWY, k - 1 - i0);
    for (int e = tid; e < kWY * kWY; e += 256) Tb[e] = Tall[b * kWY * kWY + e];
    __syncthreads();  // also orders the previous block's updates of zc
    // x = V_b^T z for both columns
    double x[2 * kWY];
#pragma unroll
    for (int q = 0; q < 2 * kWY; ++q) x[q] = 0.0;
    for (int64_t r = i0 + 1 + tid; r < k; r += 256) {
      const double z0 = zc[r], z1 = zc[k + r];
#pragma unroll
      for (int jj = 0; jj < kWY; ++jj) {
        const double v = (jj < nb) ? refl(s, i0 + jj, r) : 0.0;
        x[jj] = fma(v, z0, x[jj]);
        x[kWY + jj] = fma(v, z1, x[kWY + jj]);
      }
    }
    red.sum(x);
    if (tid == 0) {
#pragma unroll
      for (int q = 0; q < 2 * kWY; ++q) xs[q] = x[q];
    }
    __syncthreads();
    // y = T_b x (T_b upper triangular), one entry per thread
    if (tid < 2 * kWY) {
      const int c = tid / kWY, jrow = tid % kWY;
      double acc = 0.0;
      for (int l = jrow; l < kWY; ++l) acc = fma(Tb[jrow + l * kWY], xs[c * kWY + l], acc);
      ys[tid] = acc;
    }
    __syncthreads();
    // z <- z - V_b y
    for (int64_t r = i0 + 1 + tid; r < k; r += 256) {
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int jj = 0; jj < kWY; ++jj) {
        const double v = (jj < nb) ? refl(s, i0 + jj, r) : 0.0;
        d0 = fma(v, ys[jj], d0);
        d1 = fma(v, ys[kWY + jj], d1);
      }
      zc[r] -= d0;
      zc[k + r] -= d1;
    }
  }
  __syncthreads();
  for (int64_t r = tid; r < k; r += 256) {
    V32[r + j0 * k] = (float)zc[r];
    if (ncol == 2) V32[r + (j0 + 1) * k] = (float)zc[k + r];
  }
}

// gamma: coef tr(Y Y^T)/n (kappa_tar <= 0), or sigma_1^2/(kappa_tar - 1)
// (App. D, target condition number).
__global__ void k_finish_str(SketchState s, int64_t ell, int64_t n, double coef, const double *frob_part,
                             int nparts, float *sigma, double *gamma_dev, double kappa_tar) {
  __shared__ double buf[64];
  BlockReducer<5> red{buf, 0};
  double acc[5] = {0, 0, 0, 0, 0};
  for (int w = threadIdx.x; w < nparts; w += blockDim.x) acc[0] += frob_part[w];
  red.sum(acc);
  for (int64_t j = threadIdx.x; j < ell; j += blockDim.x) sigma[j] = (float)sqrt(fmax(s.lam[j], 0.0));
  if (threadIdx.x == 0) {
    gamma_dev[0] = (kappa_tar > 1.0) ? fmax(s.lam[0], 0.0) / (kappa_tar - 1.0) : coef * acc[0] / (double)n;
    gamma_dev[1] = acc[0];
  }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
int launch_gemm_f32(const float *A, int64_t lda, const float *B, int64_t ldb, float *C, int64_t ldc,
                    int64_t M, int64_t N, int64_t K, hipStream_t st) {
  const int64_t tiles = ((M + GT - 1) / GT) * ((N + GT - 1) / GT);
  hipLaunchKernelGGL(k_gemm_f32, dim3((unsigned)tiles), dim3(512), 0, st, A, lda, B, ldb, C, ldc, M, N, K);
  return (int)hipGetLastError();
}

int launch_gram_f64(const float *Y, int64_t ldy, int64_t n, int64_t k, double *G, hipStream_t st) {
  const int nb = (int)((k + HT - 1) / HT);
  const int tiles = nb * (nb + 1) / 2;
  hipLaunchKernelGGL(k_gram_f64, dim3(tiles), dim3(256), 0, st, Y, ldy, n, k, G, nb);
  return (int)hipGetLastError();
}

int launch_frob(const float *Y, int64_t ldy, int64_t n, int64_t k, double *part, int nparts,
                hipStream_t st) {
  hipLaunchKernelGGL(k_frob_partial, dim3(nparts), dim3(256), 0, st, Y, ldy, n, k, part);
  return (int)hipGetLastError();
}

int launch_tridiag(const SketchState &s, hipStream_t st) {
  const int64_t k = s.k;
  const int64_t nb = (k + kTT - 1) / kTT;
  const int64_t tiles_max = nb * (nb + 1) / 2;
  for (int64_t i = 0; i < k; ++i) {
    hipLaunchKernelGGL(k_tri_small, dim3(1), dim3(kTriThreads), 0, st, s, i);
    if (i + 1 < k) {
      const int64_t nbr = nb - (i + 1) / kTT;
      hipLaunchKernelGGL(k_tri_tiles, dim3((unsigned)(nbr * (nbr + 1) / 2)), dim3(256), 0, st, s, i, tiles_max);
      hipLaunchKernelGGL(k_tri_reduce, dim3((unsigned)nbr), dim3(1024), 0, st, s, i, nbr, tiles_max);
    }
  }
  return (int)hipGetLastError();
}

int launch_bisect(const SketchState &s, int64_t ell, hipStream_t st) {
  const int grid = (int)((ell + 3) / 4);
  const size_t lds = sizeof(double) * 2 * (size_t)s.k;
  hipLaunchKernelGGL(k_bisect, dim3(grid), dim3(256), lds, st, s, ell);
  return (int)hipGetLastError();
}

int launch_inverse_iter(const SketchState &s, int64_t ell, int64_t stride, hipStream_t st) {
  const int grid = (int)((ell + 63) / 64);
  hipLaunchKernelGGL(k_inverse_iter, dim3(grid), dim3(64), 0, st, s, ell, stride);
  return (int)hipGetLastError();
}

int launch_backtransform(const SketchState &s, int64_t ell, float *V32, hipStream_t st) {
  // the T factors go to the inverse-iteration work area, free by now
  double *Tall = s.work;
  const int nblk = (int)((s.k - 1 + kWY - 1) / kWY);
  if (nblk > 0) hipLaunchKernelGGL(k_wy_t, dim3(nblk), dim3(256), 0, st, s, Tall);
  const int grid = (int)((ell + 1) / 2);
  const size_t lds = sizeof(double) * 2 * (size_t)s.k;
  hipLaunchKernelGGL(k_backtransform, dim3(grid), dim3(256), lds, st, s, ell, (const double *)Tall, V32);
  return (int)hipGetLastError();
}

int launch_finish_str(const SketchState &s, int64_t ell, int64_t n, double coef, const double *frob_part,
                      int nparts, float *sigma, double *gamma_dev, double kappa_tar, hipStream_t st) {
  hipLaunchKernelGGL(k_finish_str, dim3(1), dim3(256), 0, st, s, ell, n, coef, frob_part, nparts, sigma,
                     gamma_dev, kappa_tar);
  return (int)hipGetLastError();
}

}  // namespace npga
