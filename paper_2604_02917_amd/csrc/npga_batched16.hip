// Batched gradient GEMMs for a bfloat16 factor on the bfloat16 matrix cores
// (v_mfma_f32_32x32x16_bf16, float32 accumulation).
//
// The entries of L are exact in bfloat16.  The other operand (the float32
// iterates X, then the float32 product U) is split into three bfloat16
// planes, v = v_h + v_m + v_l with v_h = bf16(v), v_m = bf16(v - v_h),
// v_l = bf16(v - v_h - v_m) (each difference exact in float32), which
// represents v to about 2^-27 relative; three matrix-core products per tile
// then give L^T X and L U to float32 accuracy.  Both GEMMs read their
// operands contiguous along the contraction:
//   k_b16_u : U[c][t] = sum_i X[i][c] L[i][t]     (L column-major, X columns)
//   k_b16_g : P[s][i][c] = sum_{t in T_s} Lt[i][t] U[c][t]
// where Lt is a row-major copy of L made once per batched solve.  U is
// stored directly as its three bfloat16 planes.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"

namespace npga {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));

constexpr int KB16 = 32;          // contraction depth of one LDS stage
constexpr int LDH = KB16 + 8;     // LDS row length in bfloat16 (80 bytes)

// float32 -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint32_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_val(uint32_t h) { return __uint_as_float(h << 16); }

// Three-plane split of a float32 value.
__device__ __forceinline__ void split3(float v, uint32_t &h, uint32_t &m, uint32_t &l) {
  h = bf16_rne(v);
  const float r1 = v - bf16_val(h);
  m = bf16_rne(r1);
  const float r2 = r1 - bf16_val(m);
  l = bf16_rne(r2);
}

__device__ __forceinline__ bf8 lds_bf8(const uint16_t *p) {
  return __builtin_bit_cast(bf8, *reinterpret_cast<const u4v *>(p));
}

// --------------------------------------------------------------------------
// U = X^T L with X split in three planes.  Tile: BM GEMM columns c (rows of
// the product) x BN periods t; WM x WN wavefronts of PM x PN 32 x 32 blocks.
// Epilogue: U as three bfloat16 planes [c][t] and per-tile sums of U^2.
// --------------------------------------------------------------------------
template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(256) void k_b16_u(BatchArgs b) {
  constexpr int PM = BM / (32 * WM), PN = BN / (32 * WN);
  constexpr int QA = BM * KB16 / 4 / 256;  // float4 of X per thread per stage
  constexpr int QB = BN * KB16 / 8 / 256;  // 8 x bfloat16 of L per thread per stage
  static_assert(WM * WN == 4 && PM >= 1 && PN >= 1 && QA >= 1 && QB >= 1, "tile");
  __shared__ __attribute__((aligned(16))) uint16_t Ax[2][3][BM * LDH];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[2][BN * LDH];
  __shared__ double ush[WN * BM];
  const int64_t T = b.base.cols, n = b.base.n;
  const int ma = *b.mact;
  const int64_t t0 = (int64_t)blockIdx.x * BN;
  const int64_t c0 = (int64_t)blockIdx.y * BM;
  if (c0 >= ma) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WN, wc = wave % WN;
  const int h = lane >> 5, r = lane & 31;
  const uint16_t *L = static_cast<const uint16_t *>(b.base.L);
  const int64_t ld = b.base.ld;

  const float *xcol[QA];
#pragma unroll
  for (int q = 0; q < QA; ++q) {
    const int64_t c = c0 + (tid >> 3) + 32 * q;
    xcol[q] = (c < ma) ? b.base.xs + (int64_t)b.act[c] * b.ldx : nullptr;
  }
  f4 xa[QA];
  u4v lb[QB];
  auto gload = [&](int64_t k0) {
    const int64_t kx = k0 + 4 * (tid & 7);
#pragma unroll
    for (int q = 0; q < QA; ++q)
      xa[q] = (xcol[q] && kx < n) ? *reinterpret_cast<const f4 *>(xcol[q] + kx) : f4{0.f, 0.f, 0.f, 0.f};
    const int64_t kl = k0 + 8 * (tid & 3);
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int64_t t = t0 + (tid >> 2) + 64 * q;
      lb[q] = (t < T && kl < n) ? *reinterpret_cast<const u4v *>(L + t * ld + kl) : u4v{0u, 0u, 0u, 0u};
    }
  };
  auto sstore = [&](int buf, int64_t k0) {
    const int kx = 4 * (tid & 7);
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      uint32_t hh[4], mm[4], ll[4];
      split3(xa[q].x, hh[0], mm[0], ll[0]);
      split3(xa[q].y, hh[1], mm[1], ll[1]);
      split3(xa[q].z, hh[2], mm[2], ll[2]);
      split3(xa[q].w, hh[3], mm[3], ll[3]);
      const int off = ((tid >> 3) + 32 * q) * LDH + kx;
      *reinterpret_cast<u2v *>(&Ax[buf][0][off]) = u2v{hh[0] | (hh[1] << 16), hh[2] | (hh[3] << 16)};
      *reinterpret_cast<u2v *>(&Ax[buf][1][off]) = u2v{mm[0] | (mm[1] << 16), mm[2] | (mm[3] << 16)};
      *reinterpret_cast<u2v *>(&Ax[buf][2][off]) = u2v{ll[0] | (ll[1] << 16), ll[2] | (ll[3] << 16)};
    }
    const int64_t kl = k0 + 8 * (tid & 3);
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      u4v v = lb[q];
      // asset rows past n inside the group (ld may exceed n) are not data
      if (kl + 8 > n) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int64_t row = kl + 2 * w;
          const uint32_t keep = row + 1 < n ? 0xffffffffu : (row < n ? 0x0000ffffu : 0u);
          v[w] &= keep;
        }
      }
      *reinterpret_cast<u4v *>(&Bl[buf][((tid >> 2) + 64 * q) * LDH + 8 * (tid & 3)]) = v;
    }
  };

  v16f acc[PM][PN];
#pragma unroll
  for (int p = 0; p < PM; ++p)
#pragma unroll
    for (int q = 0; q < PN; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[p][q][v] = 0.f;

  const int64_t nk = (n + KB16 - 1) / KB16;
  gload(0);
  sstore(0, 0);
  __syncthreads();
  for (int64_t s = 0; s < nk; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nk) gload((s + 1) * KB16);
#pragma unroll
    for (int ks = 0; ks < KB16 / 16; ++ks) {
      const int koff = 16 * ks + 8 * h;
      bf8 a[PM][3], bb[PN];
#pragma unroll
      for (int p = 0; p < PM; ++p)
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) a[p][pl] = lds_bf8(&Ax[buf][pl][(wr * 32 * PM + 32 * p + r) * LDH + koff]);
#pragma unroll
      for (int q = 0; q < PN; ++q) bb[q] = lds_bf8(&Bl[buf][(wc * 32 * PN + 32 * q + r) * LDH + koff]);
#pragma unroll
      for (int p = 0; p < PM; ++p)
#pragma unroll
        for (int q = 0; q < PN; ++q) {
          acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[p][2], bb[q], acc[p][q], 0, 0, 0);
          acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[p][1], bb[q], acc[p][q], 0, 0, 0);
          acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[p][0], bb[q], acc[p][q], 0, 0, 0);
        }
    }
    if (s + 1 < nk) sstore(buf ^ 1, (s + 1) * KB16);
    __syncthreads();
  }

  // epilogue: U planes (coalesced along t) and row sums of U^2
  double rs[PM][16];
#pragma unroll
  for (int p = 0; p < PM; ++p)
#pragma unroll
    for (int v = 0; v < 16; ++v) rs[p][v] = 0.0;
#pragma unroll
  for (int p = 0; p < PM; ++p)
#pragma unroll
    for (int q = 0; q < PN; ++q) {
      const int64_t t = t0 + wc * 32 * PN + 32 * q + r;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t c = c0 + wr * 32 * PM + 32 * p + 8 * (v >> 2) + 4 * h + (v & 3);
        const float val = acc[p][q][v];
        if (c < ma && t < T) {
          uint32_t hh, mm, ll;
          split3(val, hh, mm, ll);
          uint16_t *u = b.U16 + c * b.ldu16 + t;
          u[0] = (uint16_t)hh;
          u[b.u16plane] = (uint16_t)mm;
          u[2 * b.u16plane] = (uint16_t)ll;
        }
        rs[p][v] = fma((double)val, (double)val, rs[p][v]);  // periods t >= T are zero
      }
    }
#pragma unroll
  for (int p = 0; p < PM; ++p)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      double x = rs[p][v];
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) x += __shfl_xor(x, off, 64);
      if (r == 0) ush[wc * BM + wr * 32 * PM + 32 * p + 8 * (v >> 2) + 4 * h + (v & 3)] = x;
    }
  __syncthreads();
  for (int cl = tid; cl < BM; cl += 256) {
    const int64_t c = c0 + cl;
    if (c >= ma) continue;
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < WN; ++w) sum += ush[w * BM + cl];
    b.usq_part[(int64_t)blockIdx.x * b.ldq + b.act[c]] = sum;
  }
}

// --------------------------------------------------------------------------
// P[s] = Lt_{:, T_s} U_{T_s}: BM assets x BN GEMM columns over the period
// range of split s; U's three planes give three products per step.
// --------------------------------------------------------------------------
template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(256) void k_b16_g(BatchArgs b) {
  constexpr int PM = BM / (32 * WM), PN = BN / (32 * WN);
  constexpr int NA = BM * KB16 / 8;            // 16-byte groups of an Lt stage
  constexpr int NB = BN * KB16 / 8;            // 16-byte groups of one U plane stage
  constexpr int QA = (NA + 255) / 256, QB = (NB + 255) / 256;
  static_assert(WM * WN == 4 && PM >= 1 && PN >= 1, "tile");
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LDH];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][3][BN * LDH];
  const int64_t T = b.base.cols, n = b.base.n;
  const int ma = *b.mact;
  const int64_t i0 = (int64_t)blockIdx.x * BM;
  const int64_t tb = (int64_t)blockIdx.y * b.kchunk;
  const int64_t te = (tb + b.kchunk < T) ? tb + b.kchunk : T;
  const int64_t c0 = (int64_t)blockIdx.z * BN;
  if (c0 >= ma) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WN, wc = wave % WN;
  const int h = lane >> 5, r = lane & 31;

  u4v ra[QA], rb[3][QB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int idx = tid + 256 * q;
      const int64_t i = i0 + (idx >> 2);
      const int64_t t = k0 + 8 * (idx & 3);
      ra[q] = (idx < NA && i < n && t < te) ? *reinterpret_cast<const u4v *>(b.Lt + i * b.ldlt + t)
                                           : u4v{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int idx = tid + 256 * q;
      const int64_t c = c0 + (idx >> 2);
      const int64_t t = k0 + 8 * (idx & 3);
      const bool ok = idx < NB && c < ma && t < te;
      const uint16_t *u = b.U16 + c * b.ldu16 + t;
#pragma unroll
      for (int pl = 0; pl < 3; ++pl)
        rb[pl][q] = ok ? *reinterpret_cast<const u4v *>(u + pl * b.u16plane) : u4v{0u, 0u, 0u, 0u};
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int idx = tid + 256 * q;
      if (idx < NA) *reinterpret_cast<u4v *>(&As[buf][(idx >> 2) * LDH + 8 * (idx & 3)]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int idx = tid + 256 * q;
      if (idx < NB)
#pragma unroll
        for (int pl = 0; pl < 3; ++pl)
          *reinterpret_cast<u4v *>(&Bs[buf][pl][(idx >> 2) * LDH + 8 * (idx & 3)]) = rb[pl][q];
    }
  };

  v16f acc[PM][PN];
#pragma unroll
  for (int p = 0; p < PM; ++p)
#pragma unroll
    for (int q = 0; q < PN; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[p][q][v] = 0.f;

  const int64_t nk = (te > tb) ? (te - tb + KB16 - 1) / KB16 : 0;
  if (nk > 0) {
    gload(tb);
    sstore(0);
  }
  __syncthreads();
  for (int64_t s = 0; s < nk; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nk) gload(tb + (s + 1) * KB16);
#pragma unroll
    for (int ks = 0; ks < KB16 / 16; ++ks) {
      const int koff = 16 * ks + 8 * h;
      bf8 a[PM], bb[PN][3];
#pragma unroll
      for (int p = 0; p < PM; ++p) a[p] = lds_bf8(&As[buf][(wr * 32 * PM + 32 * p + r) * LDH + koff]);
#pragma unroll
      for (int q = 0; q < PN; ++q)
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) bb[q][pl] = lds_bf8(&Bs[buf][pl][(wc * 32 * PN + 32 * q + r) * LDH + koff]);
#pragma unroll
      for (int p = 0; p < PM; ++p)
#pragma unroll
        for (int q = 0; q < PN; ++q) {
          acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[p], bb[q][2], acc[p][q], 0, 0, 0);
          acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[p], bb[q][1], acc[p][q], 0, 0, 0);
          acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[p], bb[q][0], acc[p][q], 0, 0, 0);
        }
    }
    if (s + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  float *P = b.P + (int64_t)blockIdx.y * n * b.ldpm;
#pragma unroll
  for (int p = 0; p < PM; ++p)
#pragma unroll
    for (int q = 0; q < PN; ++q) {
      const int64_t c = c0 + wc * 32 * PN + 32 * q + r;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t i = i0 + wr * 32 * PM + 32 * p + 8 * (v >> 2) + 4 * h + (v & 3);
        if (i < n && c < ma) P[i * b.ldpm + c] = acc[p][q][v];
      }
    }
}

// Lt[i][t] = L[i + t ld] for t < T, zero for T <= t < ldlt (64 x 64 tiles).
__global__ __launch_bounds__(256) void k_transpose16(const uint16_t *L, int64_t ld, int64_t n, int64_t T,
                                                     uint16_t *Lt, int64_t ldlt) {
  __shared__ uint16_t tile[64][66];
  const int64_t t0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int k = ty; k < 64; k += 4) {
    const int64_t t = t0 + k, i = i0 + tx;
    tile[k][tx] = (t < T && i < n) ? L[t * ld + i] : (uint16_t)0;
  }
  __syncthreads();
  for (int k = ty; k < 64; k += 4) {
    const int64_t i = i0 + k, t = t0 + tx;
    if (i < n && t < ldlt) Lt[i * ldlt + t] = tile[tx][k];
  }
}

int launch_b16_gemm(const BatchArgs &b, const BatchConfig &c, hipStream_t s) {
  const int64_t T = b.base.cols, n = b.base.n;
  const int bn = c.g_bn;  // width of the target tiles
  if (bn == 128) {
    const dim3 gu((unsigned)((T + 63) / 64), (unsigned)((b.m + 127) / 128));
    hipLaunchKernelGGL((k_b16_u<128, 64, 2, 2>), gu, dim3(256), 0, s, b);
  } else if (bn == 64) {
    const dim3 gu((unsigned)((T + 63) / 64), (unsigned)((b.m + 63) / 64));
    hipLaunchKernelGGL((k_b16_u<64, 64, 2, 2>), gu, dim3(256), 0, s, b);
  } else {
    const dim3 gu((unsigned)((T + 127) / 128), (unsigned)((b.m + 31) / 32));
    hipLaunchKernelGGL((k_b16_u<32, 128, 1, 4>), gu, dim3(256), 0, s, b);
  }
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
  const dim3 gg((unsigned)((n + 127) / 128), (unsigned)b.splits, (unsigned)((b.m + bn - 1) / bn));
  if (bn == 128)
    hipLaunchKernelGGL((k_b16_g<128, 128, 2, 2>), gg, dim3(256), 0, s, b);
  else if (bn == 64)
    hipLaunchKernelGGL((k_b16_g<128, 64, 2, 2>), gg, dim3(256), 0, s, b);
  else
    hipLaunchKernelGGL((k_b16_g<128, 32, 4, 1>), gg, dim3(256), 0, s, b);
  return (int)hipGetLastError();
}

int launch_transpose16(const uint16_t *L, int64_t ld, int64_t n, int64_t T, uint16_t *Lt, int64_t ldlt,
                       hipStream_t s) {
  const dim3 g((unsigned)((ldlt + 63) / 64), (unsigned)((n + 63) / 64));
  hipLaunchKernelGGL(k_transpose16, g, dim3(256), 0, s, L, ld, n, T, Lt, ldlt);
  return (int)hipGetLastError();
}

}  // namespace npga
