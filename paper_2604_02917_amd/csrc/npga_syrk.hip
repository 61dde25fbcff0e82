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
// k_symv: g = 2 Sigma x + 2 gamma x.  Sigma is symmetric, so (Sigma x)_i
// is the dot product of column i with x; every wavefront owns whole columns
// (contiguous) and writes g_i directly, so no partial sums are needed.  The
// serial tail (the same one as the factor path's) is the next launch on the
// stream.
#include <hip/hip_runtime.h>

#include <algorithm>
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

// --------------------------------------------------------------------------
// Sigma = L L^T on the bfloat16 matrix cores with three-plane operands.
//
// Every float32 entry is split exactly into three bfloat16 planes,
// v = v_h + v_m + v_l (v_h = bf16(v), v_m = bf16(v - v_h), v_l = bf16(v -
// v_h - v_m); each difference is exact in float32), which carries 24
// significant bits.  A product of two such entries keeps the six plane
// products whose weight is at least 2^-24 of the leading one (h h, h m,
// m h, h l, m m, l h); each is exact in float32, and
// v_mfma_f32_32x32x16_bf16 accumulates them in float32, flushed to float64
// every 256 periods like the float32 kernel.  Six bfloat16 products run at
// 2.5 PFLOP/s against one float32 product at 157 TFLOP/s.
//
// k_split_t: L (float32, column-major, ld) -> three planes stored
//   row-major, P_pl[i ldt + t], with zeros for t in [T, ldt); one 64 x 64
//   tile per workgroup, transposed through LDS.
// k_mm16<true>: 128 x 128 tiles of the lower triangle, eight wavefronts of
//   32 x 64; 32-period stages of both row panels (three planes each) in LDS,
//   double buffered; the mirrored tile is written too.  k_mm16<false>: the
//   same on all tiles of a general product C = A B (the sketch Y = L S).
// --------------------------------------------------------------------------
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

constexpr int kSplitTile = 64;
constexpr int kLDH = 40;  // LDS row length in bfloat16 (80 bytes, 16-byte aligned)

__device__ __forceinline__ uint32_t rne_bf16(float f) {  // finite inputs
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_f32(uint32_t h) { return __uint_as_float(h << 16); }

__global__ __launch_bounds__(256) void k_split_t(const float *__restrict__ L, int64_t n, int64_t T, int64_t ld,
                                                 uint16_t *__restrict__ P, int64_t ldt, int64_t plane) {
  __shared__ float tile[kSplitTile][kSplitTile + 1];  // [t][i]
  const int tid = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * kSplitTile, i0 = (int64_t)blockIdx.y * kSplitTile;
  const int il = 4 * (tid & 15);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int tl = (tid >> 4) + 16 * q;
    const int64_t t = t0 + tl, i = i0 + il;
    f4 v = f4{0.f, 0.f, 0.f, 0.f};
    if (t < T && i < n) {
      v = *reinterpret_cast<const f4 *>(L + t * ld + i);
      if (i + 1 >= n) v.y = 0.f;
      if (i + 2 >= n) v.z = 0.f;
      if (i + 3 >= n) v.w = 0.f;
    }
    tile[tl][il + 0] = v.x;
    tile[tl][il + 1] = v.y;
    tile[tl][il + 2] = v.z;
    tile[tl][il + 3] = v.w;
  }
  __syncthreads();
  // row i0 + (tid >> 2), periods t0 + 16 (tid & 3) .. +15: two 8-entry groups per plane
  const int ir = tid >> 2, ts = 16 * (tid & 3);
  const int64_t i = i0 + ir;
  if (i >= n) return;
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    uint32_t hw[4], mw[4], lw[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      uint32_t h2[2], m2[2], l2[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const float v = tile[ts + 8 * g + 2 * w + e][ir];
        h2[e] = rne_bf16(v);
        const float r1 = v - bf16_f32(h2[e]);
        m2[e] = rne_bf16(r1);
        l2[e] = rne_bf16(r1 - bf16_f32(m2[e]));
      }
      hw[w] = h2[0] | (h2[1] << 16);
      mw[w] = m2[0] | (m2[1] << 16);
      lw[w] = l2[0] | (l2[1] << 16);
    }
    const int64_t off = i * ldt + t0 + ts + 8 * g;
    *reinterpret_cast<u4v *>(P + off) = u4v{hw[0], hw[1], hw[2], hw[3]};
    *reinterpret_cast<u4v *>(P + plane + off) = u4v{mw[0], mw[1], mw[2], mw[3]};
    *reinterpret_cast<u4v *>(P + 2 * plane + off) = u4v{lw[0], lw[1], lw[2], lw[3]};
  }
}

// Three planes of a matrix whose rows are already contiguous along the
// contraction (column j of S: S[t + j lds], t < T): P_pl[j ldt + t], zeros
// for t in [T, ldt).  A thread splits 8 consecutive entries.
__global__ __launch_bounds__(256) void k_split_rows(const float *__restrict__ X, int64_t rows, int64_t T,
                                                    int64_t ldx, uint16_t *__restrict__ P, int64_t ldt,
                                                    int64_t plane) {
  const int64_t groups = ldt / 8;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < rows * groups; e += (int64_t)gridDim.x * 256) {
    const int64_t j = e / groups, t0 = 8 * (e % groups);
    uint32_t hw[4], mw[4], lw[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      uint32_t h2[2], m2[2], l2[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int64_t t = t0 + 2 * w + q;
        const float v = (t < T) ? X[j * ldx + t] : 0.f;
        h2[q] = rne_bf16(v);
        const float r1 = v - bf16_f32(h2[q]);
        m2[q] = rne_bf16(r1);
        l2[q] = rne_bf16(r1 - bf16_f32(m2[q]));
      }
      hw[w] = h2[0] | (h2[1] << 16);
      mw[w] = m2[0] | (m2[1] << 16);
      lw[w] = l2[0] | (l2[1] << 16);
    }
    const int64_t off = j * ldt + t0;
    *reinterpret_cast<u4v *>(P + off) = u4v{hw[0], hw[1], hw[2], hw[3]};
    *reinterpret_cast<u4v *>(P + plane + off) = u4v{mw[0], mw[1], mw[2], mw[3]};
    *reinterpret_cast<u4v *>(P + 2 * plane + off) = u4v{lw[0], lw[1], lw[2], lw[3]};
  }
}

__device__ __forceinline__ bf8 lds_bf8x(const uint16_t *p) {
  return __builtin_bit_cast(bf8, *reinterpret_cast<const u4v *>(p));
}

// SYM: C = P P^T over the lower-triangle tiles (A = B = P, n x n, mirrored);
// otherwise C (na x nb) = PA PB^T over all tiles.  Operands: three planes,
// row-major along the contraction (leading dim ldt, plane strides planeA,
// planeB); C column-major with leading dim ldc.
template <bool SYM>
__global__ __launch_bounds__(512) void k_mm16(const uint16_t *__restrict__ PA, const uint16_t *__restrict__ PB,
                                              int64_t na, int64_t nbr, int64_t ldt, int64_t planeA,
                                              int64_t planeB, float *__restrict__ S, int64_t lds, int tiles_a,
                                              int tiles_b) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][3][kTile * kLDH];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][3][kTile * kLDH];
  const int ntiles = SYM ? tiles_a * (tiles_a + 1) / 2 : tiles_a * tiles_b;
  const int b = blockIdx.x;
  const int per_xcd = (ntiles + 7) / 8;
  const int tix = (b % 8) * per_xcd + (b / 8);  // consecutive tiles on one XCD
  if (tix >= ntiles) return;
  int bi = 0, bj = 0;
  if (SYM) {
    while ((bi + 1) * (bi + 2) / 2 <= tix) ++bi;
    bj = tix - bi * (bi + 1) / 2;
  } else {
    bi = tix % tiles_a;
    bj = tix / tiles_a;
  }
  const int64_t row_a = (int64_t)bi * kTile, row_b = (int64_t)bj * kTile;
  const int64_t n = na, plane = planeA;
  const uint16_t *P = PA;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;  // rows wr*32.., columns wc*64..
  const int h = lane >> 5, r = lane & 31;

  // staging: thread tid loads, for each plane, the 8 periods 8 (tid & 3) ..
  // of panel row tid >> 2
  const int prow = tid >> 2, pseg = 8 * (tid & 3);
  const bool oka = row_a + prow < n, okb = row_b + prow < (SYM ? n : nbr);
  const uint16_t *pa = P + (row_a + prow) * ldt + pseg;
  const uint16_t *pb = (SYM ? P : PB) + (row_b + prow) * ldt + pseg;
  const int64_t planeb = SYM ? plane : planeB;
  u4v ra[3], rb[3];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int pl = 0; pl < 3; ++pl) {
      ra[pl] = oka ? *reinterpret_cast<const u4v *>(pa + pl * plane + k0) : u4v{0u, 0u, 0u, 0u};
      rb[pl] = okb ? *reinterpret_cast<const u4v *>(pb + pl * planeb + k0) : u4v{0u, 0u, 0u, 0u};
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int pl = 0; pl < 3; ++pl) {
      *reinterpret_cast<u4v *>(&As[buf][pl][prow * kLDH + pseg]) = ra[pl];
      *reinterpret_cast<u4v *>(&Bs[buf][pl][prow * kLDH + pseg]) = rb[pl];
    }
  };

  v16f acc[2];
  double acc64[2][16];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      acc[q][v] = 0.f;
      acc64[q][v] = 0.0;
    }
  const int64_t nstages = ldt / kKB;  // ldt is a multiple of 64
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t st = 0; st < nstages; ++st) {
    const int buf = (int)(st & 1);
    if (st + 1 < nstages) gload((st + 1) * kKB);
#pragma unroll
    for (int ks = 0; ks < kKB / 16; ++ks) {
      const int koff = 16 * ks + 8 * h;
      bf8 a[3], bb[2][3];
#pragma unroll
      for (int pl = 0; pl < 3; ++pl) a[pl] = lds_bf8x(&As[buf][pl][(wr * 32 + r) * kLDH + koff]);
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) bb[q][pl] = lds_bf8x(&Bs[buf][pl][(wc * 64 + 32 * q + r) * kLDH + koff]);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        // smallest terms first
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], bb[q][0], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], bb[q][1], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[q][2], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], bb[q][0], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[q][1], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[q][0], acc[q], 0, 0, 0);
      }
    }
    if (((st + 1) % kFlushStages) == 0 || st + 1 == nstages) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          acc64[q][v] += (double)acc[q][v];
          acc[q][v] = 0.f;
        }
    }
    if (st + 1 < nstages) sstore(buf ^ 1);
    __syncthreads();
  }
  // the tile and its mirror; 32 x 32 output layout: lane (h, r), register v
  // -> row 8 (v/4) + 4 h + (v%4), column r
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t rr = row_a + wr * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
      const int64_t cc = row_b + wc * 64 + 32 * q + r;
      if (SYM) {
        // the plane products of (i, j) and (j, i) are summed in different
        // orders, so a diagonal tile keeps its lower half and mirrors it
        if (rr < n && cc < n && (bi != bj || rr >= cc)) {
          const float val = (float)acc64[q][v];
          S[rr + cc * lds] = val;
          S[cc + rr * lds] = val;
        }
      } else if (rr < n && cc < nbr) {
        S[rr + cc * lds] = (float)acc64[q][v];
      }
    }
}

int64_t split_ldt(int64_t T) { return (T + kSplitTile - 1) / kSplitTile * kSplitTile; }

size_t syrk_split_bytes(int64_t n, int64_t T) { return (size_t)3 * (size_t)n * (size_t)split_ldt(T) * 2; }

int launch_syrk_split(const float *L, int64_t n, int64_t T, int64_t ld, uint16_t *planes, float *Sigma,
                      int64_t lds, hipStream_t s) {
  const int64_t ldt = split_ldt(T);
  const int64_t plane = n * ldt;
  hipLaunchKernelGGL(k_split_t, dim3((unsigned)(ldt / kSplitTile), (unsigned)((n + kSplitTile - 1) / kSplitTile)),
                     dim3(256), 0, s, L, n, T, ld, planes, ldt, plane);
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
  const int nb = (int)((n + kTile - 1) / kTile);
  const int ntiles = nb * (nb + 1) / 2;
  const int grid = ((ntiles + 7) / 8) * 8;
  hipLaunchKernelGGL(k_mm16<true>, dim3(grid), dim3(512), 0, s, planes, planes, n, n, ldt, plane, plane, Sigma,
                     lds, nb, nb);
  return (int)hipGetLastError();
}

size_t gemm_split_bytes(int64_t m, int64_t ncols, int64_t K) {
  return (size_t)3 * (size_t)(m + ncols) * (size_t)split_ldt(K) * 2;
}

int launch_split_rows(const float *X, int64_t rows, int64_t T, int64_t ldx, uint16_t *P, int64_t ldt,
                      int64_t plane, hipStream_t s) {
  if (ldt % 8 != 0 || ldt < T) return (int)hipErrorInvalidValue;
  const int64_t groups = rows * (ldt / 8);
  const int sgrid = (int)std::min<int64_t>((groups + 255) / 256, 65536);
  hipLaunchKernelGGL(k_split_rows, dim3(sgrid), dim3(256), 0, s, X, rows, T, ldx, P, ldt, plane);
  return (int)hipGetLastError();
}

int launch_gemm_split(const float *A, int64_t lda, const float *B, int64_t ldb, float *C, int64_t ldc, int64_t M,
                      int64_t N, int64_t K, uint16_t *planes, hipStream_t s) {
  const int64_t ldt = split_ldt(K);
  const int64_t planeA = M * ldt, planeB = N * ldt;
  uint16_t *PA = planes, *PB = planes + 3 * planeA;
  hipLaunchKernelGGL(k_split_t, dim3((unsigned)(ldt / kSplitTile), (unsigned)((M + kSplitTile - 1) / kSplitTile)),
                     dim3(256), 0, s, A, M, K, lda, PA, ldt, planeA);
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
  const int64_t groups = N * (ldt / 8);
  const int sgrid = (int)std::min<int64_t>((groups + 255) / 256, 65536);
  hipLaunchKernelGGL(k_split_rows, dim3(sgrid), dim3(256), 0, s, B, N, K, ldb, PB, ldt, planeB);
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
  const int ta = (int)((M + kTile - 1) / kTile), tb = (int)((N + kTile - 1) / kTile);
  const int grid = ((ta * tb + 7) / 8) * 8;
  hipLaunchKernelGGL(k_mm16<false>, dim3(grid), dim3(512), 0, s, PA, PB, M, N, ldt, planeA, planeB, C, ldc, ta,
                     tb);
  return (int)hipGetLastError();
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
      else if (a.mode == kTailCG || a.mode == kTailPdas || a.mode == kTailAdj)
        gk[col] = 2.0 * (double)d + 2.0 * st->gamma * pv[col];
      else
        npga_store_grad_step(a, st, col, 2.0 * (double)d + (a.ga ? a.ga[col] : 0.0) + 2.0 * st->gamma * xk[col]);
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
