// Batched solves: m targets r_1..r_m on one factor L (points of the
// efficient frontier, Sec. 5), each running Algorithm 1 with its own state.
//
// One iteration of all targets is four launches:
//   k_bgemm_u : U^T = X^T L  (m x T): v_mfma_f32_32x32x2f32 over tiles of
//               periods t x targets j, both operands contiguous along the
//               asset index i (the contraction);
//   k_bgemm_g : P[s] = L_{:, T_s} U_{T_s, :}  (n x m) for the period range
//               T_s of split s: L tiles contiguous along the output rows i,
//               U^T tiles contiguous along the targets j;
//   k_breduce : g_j = 2 sum_s P[s][:, j] in a fixed order, plus the epilogue
//               of target j's mode (ridge term, anchor, CG direction);
//   k_btail   : one workgroup per target runs that target's serial tail
//               (stopping test, momentum, projection; or a face-CG step).
// L is read twice per iteration for all m targets instead of once per
// target, and the arithmetic moves from the vector ALUs to the matrix cores.
// The covariance form (Sigma = L L^T formed once) replaces the GEMM pair by
// one GEMM P[s] = Sigma[:, K_s] X[K_s, :] (k_cov16).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"
#include "npga_tail.h"

namespace npga {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

const BatchConfig kBatchConfigTable[kBatchConfigs] = {
    {128, 128, 128, 128, 16}, {128, 128, 128, 128, 32}, {64, 128, 128, 128, 32}, {64, 128, 64, 128, 32},
    {128, 64, 128, 64, 16},   {128, 64, 128, 64, 32},   {64, 64, 64, 64, 32},    {64, 64, 128, 64, 64},
    {128, 32, 128, 32, 16},   {128, 32, 128, 32, 32},   {128, 32, 128, 32, 64},  {64, 128, 128, 128, 64},
};

int batch_default_config(int64_t n, int64_t cols, int32_t m) {
  (void)cols;
  // widest target tile that m fills; split count so that the G GEMM has
  // about 2 workgroups per compute unit
  const int bn = m <= 32 ? 32 : (m <= 64 ? 64 : 128);
  const int64_t gt = ((n + 127) / 128) * ((m + bn - 1) / bn);
  const int want = (int)((512 + gt - 1) / gt);
  int best = -1, best_d = 1 << 30;
  for (int c = 0; c < kBatchConfigs; ++c) {
    const BatchConfig &k = kBatchConfigTable[c];
    if (k.u_bn != bn || k.g_bn != bn || k.g_bm != 128 || k.u_bm != 128) continue;
    const int d = k.splits > want ? k.splits - want : want - k.splits;
    if (d < best_d) {
      best_d = d;
      best = c;
    }
  }
  return best < 0 ? 0 : best;
}

// Per-target view of the batch: target j's state and vectors.
__device__ __forceinline__ SolveArgs target_args(const BatchArgs &b, int j) {
  SolveArgs a = b.base;
  const int64_t vs = (int64_t)j * b.vstride;
  const int64_t gs = (int64_t)j * b.gstride;
  a.st = b.base.st + j;
  a.xs = b.base.xs + (int64_t)j * b.ldx;
  a.xbuf0 = b.base.xbuf0 + vs;
  a.xbuf1 = b.base.xbuf1 + vs;
  a.gbuf0 = b.base.gbuf0 + gs;
  a.gbuf1 = b.base.gbuf1 ? b.base.gbuf1 + gs : nullptr;
  a.xa = b.base.xa ? b.base.xa + vs : nullptr;
  a.ga = b.base.ga ? b.base.ga + vs : nullptr;
  a.ua = nullptr;
  if (b.base.pvec) {
    a.pvec = b.base.pvec + vs;
    a.fvec = b.base.fvec + vs;
    a.gvec = b.base.gvec + vs;
  }
  return a;
}

// Four consecutive entries of L kept in their storage format until they are
// written to LDS, so the prefetch of the next tile never waits on its loads.
template <typename TL>
struct Raw4;
template <>
struct Raw4<float> {
  typedef f4 type;
  static __device__ __forceinline__ f4 load(const float *p) { return *reinterpret_cast<const f4 *>(p); }
  static __device__ __forceinline__ f4 zero() { return f4{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ f4 widen(f4 v) { return v; }
};
template <>
struct Raw4<bf16_t> {
  typedef u2v type;
  static __device__ __forceinline__ u2v load(const bf16_t *p) { return *reinterpret_cast<const u2v *>(p); }
  static __device__ __forceinline__ u2v zero() { return u2v{0u, 0u}; }
  static __device__ __forceinline__ f4 widen(u2v w) {
    return f4{__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xffff0000u), __uint_as_float(w.y << 16),
              __uint_as_float(w.y & 0xffff0000u)};
  }
};

constexpr int KB = 32;       // contraction depth of one LDS stage
constexpr int LDK = KB + 4;  // row length (floats) of contraction-contiguous LDS tiles

// --------------------------------------------------------------------------
// U^T = X^T L.  Tile: BM periods x BN targets; WM x WN wavefronts, each
// PM x PN blocks of 32 x 32.  Lane half h of a wavefront holds contraction
// indices 16h..16h+15 of a stage, read from LDS as four float4, so that MFMA
// step s pairs k = s (lanes 0-31) with k = 16 + s (lanes 32-63) on both
// operands.  Epilogue: U^T and per-tile column sums of U^2 (float64).
// --------------------------------------------------------------------------
// KSPLIT (covariance form, L := Sigma): the contraction is split over
// grid.z in ranges of b.kchunk rows, and each split writes its partial
// product into P[(z n + t) ldpm + j] (the layout k_breduce sums) instead
// of U^T; no column sums.
template <typename TL, int BM, int BN, int WM, int WN, bool KSPLIT = false>
__global__ __launch_bounds__(256) void k_bgemm_u(BatchArgs b) {
  constexpr int PM = BM / (32 * WM), PN = BN / (32 * WN);
  constexpr int QA = BM / 32, QB = BN / 32;
  static_assert(WM * WN == 4 && PM >= 1 && PN >= 1, "tile");
  typedef Raw4<TL> R;
  __shared__ float As[2][BM * LDK];
  __shared__ float Bs[2][BN * LDK];
  __shared__ double ush[WM * BN];
  const int64_t T = b.base.cols, n = b.base.n;
  const int m = b.m;
  const int64_t t0 = (int64_t)blockIdx.x * BM;
  const int64_t j0 = (int64_t)blockIdx.y * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WN, wc = wave % WN;
  const int h = lane >> 5, r = lane & 31;
  const TL *L = static_cast<const TL *>(b.base.L);
  const int64_t ld = b.base.ld;
  const float *X = b.base.xs;
  const int kq = 4 * (tid & 7);
  const int ma = *b.mact;
  if (j0 >= ma) return;
  (void)m;
  const int64_t kbeg = KSPLIT ? (int64_t)blockIdx.z * b.kchunk : 0;
  const int64_t kend = KSPLIT ? (kbeg + b.kchunk < n ? kbeg + b.kchunk : n) : n;
  // targets of this thread's X columns (column c -> target act[c])
  const float *xcol[QB];
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int64_t c = j0 + (tid >> 3) + 32 * q;
    xcol[q] = (c < ma) ? X + (int64_t)b.act[c] * b.ldx : nullptr;
  }

  typename R::type ra[QA];
  f4 rb[QB];
  // (a split's range starts and, except at n, ends on a multiple of 32, so
  // a float4 never straddles kend below n)
  auto gload = [&](int64_t k0) {
    const int64_t k = k0 + kq;
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int64_t t = t0 + (tid >> 3) + 32 * q;
      ra[q] = (t < T && k < kend) ? R::load(L + t * ld + k) : R::zero();
    }
#pragma unroll
    for (int q = 0; q < QB; ++q)
      rb[q] = (xcol[q] && k < kend) ? *reinterpret_cast<const f4 *>(xcol[q] + k) : f4{0.f, 0.f, 0.f, 0.f};
  };
  auto sstore = [&](int buf, int64_t k0) {
    const int64_t k = k0 + kq;
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      f4 v = R::widen(ra[q]);
      // rows past n inside the float4 (ld may exceed n): the contraction
      // must not see them
      if (k + 1 >= kend) v.y = 0.f;
      if (k + 2 >= kend) v.z = 0.f;
      if (k + 3 >= kend) v.w = 0.f;
      *reinterpret_cast<f4 *>(&As[buf][((tid >> 3) + 32 * q) * LDK + kq]) = v;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) *reinterpret_cast<f4 *>(&Bs[buf][((tid >> 3) + 32 * q) * LDK + kq]) = rb[q];
  };

  v16f acc[PM][PN];
#pragma unroll
  for (int p = 0; p < PM; ++p)
#pragma unroll
    for (int q = 0; q < PN; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[p][q][v] = 0.f;

  const int64_t nk = (kend - kbeg + KB - 1) / KB;
  gload(kbeg);
  sstore(0, kbeg);
  __syncthreads();
  for (int64_t s = 0; s < nk; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nk) gload(kbeg + (s + 1) * KB);
    float av[PM][16], bv[PN][16];
#pragma unroll
    for (int p = 0; p < PM; ++p) {
      const float *src = &As[buf][(wr * 32 * PM + 32 * p + r) * LDK + 16 * h];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const f4 t = *reinterpret_cast<const f4 *>(src + 4 * c);
        av[p][4 * c + 0] = t.x;
        av[p][4 * c + 1] = t.y;
        av[p][4 * c + 2] = t.z;
        av[p][4 * c + 3] = t.w;
      }
    }
#pragma unroll
    for (int q = 0; q < PN; ++q) {
      const float *src = &Bs[buf][(wc * 32 * PN + 32 * q + r) * LDK + 16 * h];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const f4 t = *reinterpret_cast<const f4 *>(src + 4 * c);
        bv[q][4 * c + 0] = t.x;
        bv[q][4 * c + 1] = t.y;
        bv[q][4 * c + 2] = t.z;
        bv[q][4 * c + 3] = t.w;
      }
    }
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
#pragma unroll
      for (int p = 0; p < PM; ++p)
#pragma unroll
        for (int q = 0; q < PN; ++q)
          acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[p][kk], bv[q][kk], acc[p][q], 0, 0, 0);
    if (s + 1 < nk) sstore(buf ^ 1, kbeg + (s + 1) * KB);
    __syncthreads();
  }

  if constexpr (KSPLIT) {
    float *Pz = b.P + (int64_t)blockIdx.z * n * b.ldpm;
#pragma unroll
    for (int p = 0; p < PM; ++p)
#pragma unroll
      for (int q = 0; q < PN; ++q) {
        const int64_t j = j0 + wc * 32 * PN + 32 * q + r;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t t = t0 + wr * 32 * PM + 32 * p + 8 * (v >> 2) + 4 * h + (v & 3);
          if (t < T && j < ma) Pz[t * b.ldpm + j] = acc[p][q][v];
        }
      }
    return;
  }

  // epilogue: U^T (coalesced along j) and column sums of U^2 over this tile
  double cs[PN];
#pragma unroll
  for (int q = 0; q < PN; ++q) cs[q] = 0.0;
#pragma unroll
  for (int p = 0; p < PM; ++p)
#pragma unroll
    for (int q = 0; q < PN; ++q) {
      const int64_t j = j0 + wc * 32 * PN + 32 * q + r;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t t = t0 + wr * 32 * PM + 32 * p + 8 * (v >> 2) + 4 * h + (v & 3);
        const float val = acc[p][q][v];
        if (t < T && j < ma) b.Ut[j + t * b.ldut] = val;
        cs[q] = fma((double)val, (double)val, cs[q]);  // rows t >= T are zero
      }
    }
#pragma unroll
  for (int q = 0; q < PN; ++q) cs[q] += __shfl_xor(cs[q], 32, 64);
  if (h == 0) {
#pragma unroll
    for (int q = 0; q < PN; ++q) ush[wr * BN + wc * 32 * PN + 32 * q + r] = cs[q];
  }
  __syncthreads();
  for (int c = tid; c < BN; c += 256) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < WM; ++w) sum += ush[w * BN + c];
    const int64_t cc = j0 + c;
    if (cc < ma) b.usq_part[(int64_t)blockIdx.x * b.ldq + b.act[cc]] = sum;
  }
}

// --------------------------------------------------------------------------
// P[s] = L_{:, T_s} U_{T_s, :}.  Tile: BM assets x BN targets over the
// period range of split s (grid.y).  Both LDS tiles are indexed [k][row];
// MFMA step s takes k = 2s + h.  Output rows i >= n and columns j >= m are
// never stored, so garbage there (padding of L or U^T) stays in unused
// accumulator entries; periods outside the range are zero in both tiles.
// --------------------------------------------------------------------------
template <typename TL, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(256) void k_bgemm_g(BatchArgs b) {
  constexpr int PM = BM / (32 * WM), PN = BN / (32 * WN);
  constexpr int LDA = BM + 4, LDB = BN + 4;
  constexpr int FA = BM / 4, FB = BN / 4;       // float4 per period row of a tile
  constexpr int QA = KB * FA / 256, QB = KB * FB / 256;
  static_assert(WM * WN == 4 && PM >= 1 && PN >= 1 && QA >= 1 && QB >= 1, "tile");
  typedef Raw4<TL> R;
  __shared__ float As[2][KB * LDA];
  __shared__ float Bs[2][KB * LDB];
  const int64_t T = b.base.cols, n = b.base.n;
  const int m = b.m;
  const int64_t i0 = (int64_t)blockIdx.x * BM;
  const int64_t tb = (int64_t)blockIdx.y * b.kchunk;
  const int64_t te = (tb + b.kchunk < T) ? tb + b.kchunk : T;
  const int64_t j0 = (int64_t)blockIdx.z * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WN, wc = wave % WN;
  const int h = lane >> 5, r = lane & 31;
  const TL *L = static_cast<const TL *>(b.base.L);
  const int64_t ld = b.base.ld;
  const float *Ut = b.Ut;
  const int ma = *b.mact;
  if (j0 >= ma) return;
  (void)m;

  typename R::type ra[QA];
  f4 rb[QB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int idx = tid + 256 * q;
      const int64_t t = k0 + idx / FA;
      const int64_t i = i0 + 4 * (idx % FA);
      ra[q] = (t < te && i < n) ? R::load(L + t * ld + i) : R::zero();
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int idx = tid + 256 * q;
      const int64_t t = k0 + idx / FB;
      const int64_t j = j0 + 4 * (idx % FB);
      rb[q] = (t < te && j < ma) ? *reinterpret_cast<const f4 *>(Ut + j + t * b.ldut) : f4{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int idx = tid + 256 * q;
      *reinterpret_cast<f4 *>(&As[buf][(idx / FA) * LDA + 4 * (idx % FA)]) = R::widen(ra[q]);
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int idx = tid + 256 * q;
      *reinterpret_cast<f4 *>(&Bs[buf][(idx / FB) * LDB + 4 * (idx % FB)]) = rb[q];
    }
  };

  v16f acc[PM][PN];
#pragma unroll
  for (int p = 0; p < PM; ++p)
#pragma unroll
    for (int q = 0; q < PN; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[p][q][v] = 0.f;

  const int64_t nk = (te > tb) ? (te - tb + KB - 1) / KB : 0;
  if (nk > 0) {
    gload(tb);
    sstore(0);
  }
  __syncthreads();
  for (int64_t s = 0; s < nk; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nk) gload(tb + (s + 1) * KB);
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 2 * kk + h;
      float av[PM], bv[PN];
#pragma unroll
      for (int p = 0; p < PM; ++p) av[p] = As[buf][k * LDA + wr * 32 * PM + 32 * p + r];
#pragma unroll
      for (int q = 0; q < PN; ++q) bv[q] = Bs[buf][k * LDB + wc * 32 * PN + 32 * q + r];
#pragma unroll
      for (int p = 0; p < PM; ++p)
#pragma unroll
        for (int q = 0; q < PN; ++q)
          acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[p], bv[q], acc[p][q], 0, 0, 0);
    }
    if (s + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  float *P = b.P + (int64_t)blockIdx.y * n * b.ldpm;
#pragma unroll
  for (int p = 0; p < PM; ++p)
#pragma unroll
    for (int q = 0; q < PN; ++q) {
      const int64_t j = j0 + wc * 32 * PN + 32 * q + r;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t i = i0 + wr * 32 * PM + 32 * p + 8 * (v >> 2) + 4 * h + (v & 3);
        if (i < n && j < ma) P[i * b.ldpm + j] = acc[p][q][v];
      }
    }
}

// --------------------------------------------------------------------------
// g_j = 2 sum_s P[s][:, j] (fixed order over s, float64) and the epilogue of
// the current mode.  A 16 x 32 tile (rows i x GEMM columns c) per
// workgroup: the partial reads run along c, eight splits in flight per
// thread; the tile is transposed through LDS so the per-target reads and
// writes run along i.
// --------------------------------------------------------------------------
constexpr int RB = 16;  // rows of a reduce tile

__global__ __launch_bounds__(256) void k_breduce(BatchArgs b) {
  __shared__ double tile[RB][33];
  const int64_t n = b.base.n;
  const int ma = *b.mact;
  const int64_t i0 = (int64_t)blockIdx.x * RB;
  const int c0 = blockIdx.y * 32;  // GEMM column block (running targets)
  const int tid = threadIdx.x;
  if (c0 >= ma) return;
  {
    const int cc = tid & 31, ii = tid >> 5;
    const int64_t split_stride = n * b.ldpm;
    const int S = b.splits;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t i = i0 + ii + 8 * h;
      double s = 0.0;
      if (i < n && c0 + cc < ma) {
        const float *p = b.P + i * b.ldpm + c0 + cc;
        int sp = 0;
        for (; sp + 8 <= S; sp += 8) {
          float v[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = p[(int64_t)(sp + e) * split_stride];
#pragma unroll
          for (int e = 0; e < 8; ++e) s += (double)v[e];
        }
        for (; sp < S; ++sp) s += (double)p[(int64_t)sp * split_stride];
      }
      tile[ii + 8 * h][cc] = s;
    }
  }
  __syncthreads();
  const int il = tid & 15, cq = tid >> 4;
  const int64_t i = i0 + il;
  if (i >= n) return;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int cl = cq + 16 * h;
    if (c0 + cl >= ma) continue;
    const SolveArgs a = target_args(b, b.act[c0 + cl]);
    const DevState *st = a.st;
    if (st->done != kRunning) continue;
    const double tot = tile[il][cl];
    if (a.mode == kTailNpga) {
      const double *xk = (st->iter & 1) ? a.xbuf1 : a.xbuf0;
      npga_store_grad_step(a, st, i, 2.0 * tot + (a.ga ? a.ga[i] : 0.0) + 2.0 * st->gamma * xk[i]);
    } else if (a.mode == kTailGrad) {
      a.gbuf0[i] = 2.0 * tot + 2.0 * st->gamma * a.xbuf0[i];
    } else if (a.mode == kTailCG) {
      a.gbuf0[i] = 2.0 * tot + 2.0 * st->gamma * a.pvec[i];
    }
  }
}

// One workgroup per target: the serial tail of that target's iteration.
template <int E>
__global__ __launch_bounds__(256) void k_btail(BatchArgs b) {
  const SolveArgs a = target_args(b, blockIdx.x);
  if (a.st->done != kRunning) return;
  __shared__ double redbuf[64];
  __shared__ double mbuf[8];
  __shared__ int64_t ibuf[8];
  double usq = -1.0;  // covariance form: f = x^T g / 2 in the tails
  if (!b.covariance && (a.mode == kTailNpga || a.mode == kTailGrad)) {
    BlockReducer<5> red5{redbuf, 0};
    double acc[5] = {0, 0, 0, 0, 0};
    for (int w = threadIdx.x; w < b.utiles; w += 256) acc[0] += b.usq_part[(int64_t)w * b.ldq + blockIdx.x];
    red5.sum(acc);
    usq = acc[0];
    __syncthreads();
  }
  if (a.mode == kTailNpga)
    tail_npga<E>(a, usq, redbuf);
  else if (a.mode == kTailCG)
    tail_cg<E>(a, redbuf, mbuf, ibuf);
  else if (a.mode == kTailGrad)
    tail_grad<E>(a, usq, redbuf);
}

template <int E>
__global__ __launch_bounds__(256) void k_bproject_init(BatchArgs b) {
  __shared__ double redbuf[64];
  const SolveArgs a = target_args(b, blockIdx.x);
  if (a.st->done != kRunning) return;
  project_init_body<E>(a, redbuf);
}

template <int E>
__global__ __launch_bounds__(256) void k_bcg_init(BatchArgs b) {
  __shared__ double redbuf[64];
  const SolveArgs a = target_args(b, blockIdx.x);
  if (a.st->done != kRunning) return;
  cg_init_body<E>(a, redbuf);
}

// X[:, j] = x_j (float32); grid (row blocks, m).
__global__ __launch_bounds__(256) void k_bfinalize(BatchArgs b, float *X, int64_t ldo) {
  const SolveArgs a = target_args(b, blockIdx.y);
  const double *x = (a.st->iter & 1) ? a.xbuf1 : a.xbuf0;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < a.n) X[(int64_t)blockIdx.y * ldo + i] = (float)x[i];
}

// x_j = X0[:, j] (or 1/n) in float64, the whole column of X zeroed first
// (rows n..ldx-1 stay zero for the U GEMM); grid (row blocks, m).
__global__ __launch_bounds__(256) void k_bset_x0(BatchArgs b, const float *X0, int64_t ldx0) {
  const SolveArgs a = target_args(b, blockIdx.y);
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < b.ldx) a.xs[i] = 0.0f;
  if (i < a.n) {
    const double v = X0 ? (double)X0[(int64_t)blockIdx.y * ldx0 + i] : 1.0 / (double)a.n;
    a.xbuf0[i] = v;
  }
}

// Float32 copy of X into the GEMM input and float64 copy into xbuf0 (the
// batched gradient entry point); grid (row blocks, m).
__global__ __launch_bounds__(256) void k_bload_x(BatchArgs b, const float *X, int64_t ldx_in) {
  const SolveArgs a = target_args(b, blockIdx.y);
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < b.ldx) {
    const float v = (i < a.n) ? X[(int64_t)blockIdx.y * ldx_in + i] : 0.0f;
    a.xs[i] = v;
    if (i < a.n) a.xbuf0[i] = (double)v;
  }
}

// Step size of the shared factor: alpha and L_f from the power-method state.
__global__ void k_bcopy_step(BatchArgs b, const DevState *src) {
  for (int j = threadIdx.x; j < b.m; j += blockDim.x) {
    b.base.st[j].alpha = src->alpha;
    b.base.st[j].lipschitz = src->lipschitz;
    b.base.st[j].rho2 = src->rho2;
    b.base.st[j].beta_const = src->beta_const;
    b.base.st[j].lz_m = src->lz_m;
  }
}

// Refinement phase: every target whose last phase converged runs again.
__global__ void k_bphase_reset(BatchArgs b, double tol, int32_t max_iter) {
  for (int j = threadIdx.x; j < b.m; j += blockDim.x) {
    DevState *st = b.base.st + j;
    if (st->done != kConverged) continue;
    st->done = kRunning;
    st->cg_window = 60;
    st->tol = tol;
    st->max_iter = max_iter;
    st->restart = 1;
    st->t = 1.0;
    st->beta = 0.0;
  }
}

// x_a = x_k for every target about to be refined (converged last phase).
__global__ __launch_bounds__(256) void k_bcopy_anchor(BatchArgs b) {
  const SolveArgs a = target_args(b, blockIdx.y);
  if (a.st->done != kConverged) return;
  const double *x = (a.st->iter & 1) ? a.xbuf1 : a.xbuf0;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < a.n) const_cast<double *>(a.xa)[i] = x[i];
}

// out[0] = number of running targets, out[1 + j] = done code of target j;
// act[0..mact) = the running targets in ascending order (GEMM columns of the
// next iterations).  One workgroup; target j = 4 tid + e (m <= 1024).
__global__ __launch_bounds__(256) void k_bstatus(BatchArgs b, int32_t *out, int32_t *act, int32_t *mact) {
  __shared__ int scan[256];
  const int tid = threadIdx.x;
  int run[4];
  int c = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int j = 4 * tid + e;
    run[e] = 0;
    if (j < b.m) {
      const int32_t d = b.base.st[j].done;
      out[1 + j] = d;
      run[e] = (d == kRunning) ? 1 : 0;
      c += run[e];
    }
  }
  // inclusive scan of the per-thread counts (Hillis-Steele)
  scan[tid] = c;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int v = (tid >= off) ? scan[tid - off] : 0;
    __syncthreads();
    scan[tid] += v;
    __syncthreads();
  }
  int pos = scan[tid] - c;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (run[e]) act[pos++] = 4 * tid + e;
  if (tid == 255) {
    out[0] = scan[255];
    *mact = scan[255];
  }
}

// Every target is a GEMM column (batched gradient, tuning).
__global__ __launch_bounds__(256) void k_bact_all(int32_t m, int32_t *act, int32_t *mact) {
  for (int j = threadIdx.x; j < m; j += 256) act[j] = j;
  if (threadIdx.x == 0) *mact = m;
}

// L32 = float32 values of a bfloat16 factor (the covariance form's SYRK
// reads float32); rows n..ld32-1 are written as zeros.
__global__ __launch_bounds__(256) void k_widen_bf16(const uint16_t *L, int64_t ld, int64_t n, int64_t T, float *L32,
                                                    int64_t ld32) {
  const int64_t total = ld32 * T;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t t = e / ld32, i = e - t * ld32;
    L32[e] = (i < n) ? __uint_as_float((uint32_t)L[i + t * ld] << 16) : 0.f;
  }
}

int launch_widen_bf16(const uint16_t *L, int64_t ld, int64_t n, int64_t T, float *L32, int64_t ld32, hipStream_t s) {
  hipLaunchKernelGGL(k_widen_bf16, dim3(2048), dim3(256), 0, s, L, ld, n, T, L32, ld32);
  return (int)hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero_f32(float *p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
    p[i] = 0.0f;
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
#define BATCH_SLOT_SWITCH(slots, CALL)     \
  switch (slots) {                         \
    case 1: CALL(1); break;                \
    case 2: CALL(2); break;                \
    case 4: CALL(4); break;                \
    case 8: CALL(8); break;                \
    case 12: CALL(12); break;              \
    case 16: CALL(16); break;              \
    case 22: CALL(22); break;              \
    case 28: CALL(28); break;              \
    case 32: CALL(32); break;              \
    default: return (int)hipErrorInvalidValue; \
  }

template <typename TL>
static int launch_bgemm_t(const BatchArgs &b, const BatchConfig &c, hipStream_t s) {
  const int64_t T = b.base.cols, n = b.base.n;
  const dim3 gu((unsigned)((T + c.u_bm - 1) / c.u_bm), (unsigned)((b.m + c.u_bn - 1) / c.u_bn));
  if (c.u_bm == 128 && c.u_bn == 128)
    hipLaunchKernelGGL((k_bgemm_u<TL, 128, 128, 2, 2>), gu, dim3(256), 0, s, b);
  else if (c.u_bm == 64 && c.u_bn == 128)
    hipLaunchKernelGGL((k_bgemm_u<TL, 64, 128, 1, 4>), gu, dim3(256), 0, s, b);
  else if (c.u_bm == 128 && c.u_bn == 64)
    hipLaunchKernelGGL((k_bgemm_u<TL, 128, 64, 2, 2>), gu, dim3(256), 0, s, b);
  else if (c.u_bm == 64 && c.u_bn == 64)
    hipLaunchKernelGGL((k_bgemm_u<TL, 64, 64, 2, 2>), gu, dim3(256), 0, s, b);
  else if (c.u_bm == 128 && c.u_bn == 32)
    hipLaunchKernelGGL((k_bgemm_u<TL, 128, 32, 4, 1>), gu, dim3(256), 0, s, b);
  else
    return (int)hipErrorInvalidValue;
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
  const dim3 gg((unsigned)((n + c.g_bm - 1) / c.g_bm), (unsigned)b.splits, (unsigned)((b.m + c.g_bn - 1) / c.g_bn));
  if (c.g_bm == 128 && c.g_bn == 128)
    hipLaunchKernelGGL((k_bgemm_g<TL, 128, 128, 2, 2>), gg, dim3(256), 0, s, b);
  else if (c.g_bm == 64 && c.g_bn == 128)
    hipLaunchKernelGGL((k_bgemm_g<TL, 64, 128, 1, 4>), gg, dim3(256), 0, s, b);
  else if (c.g_bm == 128 && c.g_bn == 64)
    hipLaunchKernelGGL((k_bgemm_g<TL, 128, 64, 2, 2>), gg, dim3(256), 0, s, b);
  else if (c.g_bm == 64 && c.g_bn == 64)
    hipLaunchKernelGGL((k_bgemm_g<TL, 64, 64, 2, 2>), gg, dim3(256), 0, s, b);
  else if (c.g_bm == 128 && c.g_bn == 32)
    hipLaunchKernelGGL((k_bgemm_g<TL, 128, 32, 4, 1>), gg, dim3(256), 0, s, b);
  else
    return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

// Covariance form on the bfloat16 matrix cores: P_z = Sigma[:, K_z] X[K_z, :]
// (the split-partial layout k_breduce sums) with Sigma given as three
// bfloat16 planes (split once per call) and each float32 column of X split
// into three planes as it is staged, v = v_h + v_m + v_l exactly; the six
// largest plane products (h h, h m, m h, h l, m m, l h: the dropped m l,
// l m and l l are below 2^-24 of the leading one) on
// v_mfma_f32_32x32x16_bf16 with float32 accumulation over the range, as the
// split SYRK does.  Tile: 64 rows of Sigma x 64 GEMM columns,
// four wavefronts of 32 x 32; 32-deep stages of both panels, double
// buffered.  Grid: (row tiles, column tiles, ranges).
constexpr int C16K = 32;            // contraction depth of one stage
constexpr int C16LD = C16K + 8;     // LDS row length in bfloat16 (80 bytes)

__global__ __launch_bounds__(256) void k_cov16(BatchArgs b) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][3][64 * C16LD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][3][64 * C16LD];
  const int64_t n = b.base.n;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int64_t j0 = (int64_t)blockIdx.y * 64;
  const int ma = *b.mact;
  if (j0 >= ma) return;
  const int64_t kbeg = (int64_t)blockIdx.z * b.kchunk;
  const int64_t kend = (kbeg + b.kchunk < n) ? kbeg + b.kchunk : n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int h = lane >> 5, r = lane & 31;
  // staging: row tid / 4 of each panel, contraction entries 8 (tid % 4) .. +7
  // of a stage
  const int prow = tid >> 2, pseg = 8 * (tid & 3);
  const bool oka = i0 + prow < n;
  const uint16_t *pa = b.Sp + (i0 + prow) * b.ldsp + pseg;
  const int64_t cb = j0 + prow;
  const float *xc = (cb < ma) ? b.base.xs + (int64_t)b.act[cb] * b.ldx + pseg : nullptr;
  u4v ra[3];
  f4 rx[2];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int pl = 0; pl < 3; ++pl)
      ra[pl] = oka ? *reinterpret_cast<const u4v *>(pa + pl * b.spplane + k0) : u4v{0u, 0u, 0u, 0u};
    // k0 + pseg + 8 <= ldx (X columns are padded to a multiple of 256), so
    // both loads stay in the column; entries at or past kend are masked at
    // the split
    rx[0] = xc ? *reinterpret_cast<const f4 *>(xc + k0) : f4{0.f, 0.f, 0.f, 0.f};
    rx[1] = xc ? *reinterpret_cast<const f4 *>(xc + k0 + 4) : f4{0.f, 0.f, 0.f, 0.f};
  };
  auto sstore = [&](int buf, int64_t k0) {
#pragma unroll
    for (int pl = 0; pl < 3; ++pl) *reinterpret_cast<u4v *>(&As[buf][pl][prow * C16LD + pseg]) = ra[pl];
    const float v[8] = {rx[0].x, rx[0].y, rx[0].z, rx[0].w, rx[1].x, rx[1].y, rx[1].z, rx[1].w};
    uint32_t hw[4], mw[4], lw[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      uint32_t h2[2], m2[2], l2[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const float x = (k0 + pseg + 2 * w + e < kend) ? v[2 * w + e] : 0.f;
        const uint32_t hb = (__float_as_uint(x) + 0x7fffu + ((__float_as_uint(x) >> 16) & 1u)) >> 16;
        const float r1 = x - __uint_as_float(hb << 16);
        const uint32_t mb = (__float_as_uint(r1) + 0x7fffu + ((__float_as_uint(r1) >> 16) & 1u)) >> 16;
        const float r2 = r1 - __uint_as_float(mb << 16);
        h2[e] = hb;
        m2[e] = mb;
        l2[e] = (__float_as_uint(r2) + 0x7fffu + ((__float_as_uint(r2) >> 16) & 1u)) >> 16;
      }
      hw[w] = h2[0] | (h2[1] << 16);
      mw[w] = m2[0] | (m2[1] << 16);
      lw[w] = l2[0] | (l2[1] << 16);
    }
    *reinterpret_cast<u4v *>(&Bs[buf][0][prow * C16LD + pseg]) = u4v{hw[0], hw[1], hw[2], hw[3]};
    *reinterpret_cast<u4v *>(&Bs[buf][1][prow * C16LD + pseg]) = u4v{mw[0], mw[1], mw[2], mw[3]};
    *reinterpret_cast<u4v *>(&Bs[buf][2][prow * C16LD + pseg]) = u4v{lw[0], lw[1], lw[2], lw[3]};
  };
  v16f acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  const int64_t nk = (kend - kbeg + C16K - 1) / C16K;
  gload(kbeg);
  sstore(0, kbeg);
  __syncthreads();
  for (int64_t st = 0; st < nk; ++st) {
    const int buf = (int)(st & 1);
    if (st + 1 < nk) gload(kbeg + (st + 1) * C16K);
#pragma unroll
    for (int ks = 0; ks < C16K / 16; ++ks) {
      const int koff = 16 * ks + 8 * h;
      bf16x8_t a[3], bb[3];
#pragma unroll
      for (int pl = 0; pl < 3; ++pl) {
        a[pl] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u4v *>(&As[buf][pl][(wr * 32 + r) * C16LD + koff]));
        bb[pl] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u4v *>(&Bs[buf][pl][(wc * 32 + r) * C16LD + koff]));
      }
      // smallest terms first
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], bb[0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], bb[1], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[2], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], bb[0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[1], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], bb[0], acc, 0, 0, 0);
    }
    if (st + 1 < nk) sstore(buf ^ 1, kbeg + (st + 1) * C16K);
    __syncthreads();
  }
  // 32 x 32 output layout: lane (h, r), register v -> row 8 (v / 4) + 4 h + v % 4, column r
  float *out = b.P + (int64_t)blockIdx.z * n * b.ldpm;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t row = i0 + wr * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
    const int64_t col = j0 + wc * 32 + r;
    if (row < n && col < ma) out[row * b.ldpm + col] = acc[v];
  }
}

// Covariance form: G = Sigma X split over the contraction (k_breduce sums
// the splits), by k_cov16 on Sigma's bfloat16 planes when they are given,
// else by the float32 U GEMM on L := Sigma (symmetric).
static int launch_bcov(const BatchArgs &b, const BatchConfig &c, hipStream_t s) {
  const int64_t n = b.base.n;
  const unsigned gy = (unsigned)((b.m + c.u_bn - 1) / c.u_bn);
  const dim3 g((unsigned)((n + c.u_bm - 1) / c.u_bm), gy, (unsigned)b.splits);
  if (b.Sp) {
    if (c.u_bm != 64 || c.u_bn != 64 || (b.kchunk % C16K) != 0) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cov16, g, dim3(256), 0, s, b);
    return (int)hipGetLastError();
  }
  if (c.u_bm == 128 && c.u_bn == 128)
    hipLaunchKernelGGL((k_bgemm_u<float, 128, 128, 2, 2, true>), g, dim3(256), 0, s, b);
  else if (c.u_bm == 128 && c.u_bn == 64)
    hipLaunchKernelGGL((k_bgemm_u<float, 128, 64, 2, 2, true>), g, dim3(256), 0, s, b);
  else if (c.u_bm == 128 && c.u_bn == 32)
    hipLaunchKernelGGL((k_bgemm_u<float, 128, 32, 4, 1, true>), g, dim3(256), 0, s, b);
  else if (c.u_bm == 64 && c.u_bn == 64)
    hipLaunchKernelGGL((k_bgemm_u<float, 64, 64, 2, 2, true>), g, dim3(256), 0, s, b);
  else if (c.u_bm == 64 && c.u_bn == 128)
    hipLaunchKernelGGL((k_bgemm_u<float, 64, 128, 1, 4, true>), g, dim3(256), 0, s, b);
  else
    return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

int launch_bgemm(const BatchArgs &b, const BatchConfig &c, hipStream_t s) {
  if (b.covariance) return launch_bcov(b, c, s);
  if (b.Lt) return launch_b16_gemm(b, c, s);
  if (b.base.dtype == NPGA_BF16) return launch_bgemm_t<bf16_t>(b, c, s);
  return launch_bgemm_t<float>(b, c, s);
}

int launch_breduce_tail(const BatchArgs &b, int slots, hipStream_t s) {
  const dim3 gr((unsigned)((b.base.n + RB - 1) / RB), (unsigned)((b.m + 31) / 32));
  hipLaunchKernelGGL(k_breduce, gr, dim3(256), 0, s, b);
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
#define CALL(E) hipLaunchKernelGGL(k_btail<E>, dim3((unsigned)b.m), dim3(256), 0, s, b)
  BATCH_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_bproject_init(const BatchArgs &b, int slots, hipStream_t s) {
#define CALL(E) hipLaunchKernelGGL(k_bproject_init<E>, dim3((unsigned)b.m), dim3(256), 0, s, b)
  BATCH_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_bcg_init(const BatchArgs &b, int slots, hipStream_t s) {
#define CALL(E) hipLaunchKernelGGL(k_bcg_init<E>, dim3((unsigned)b.m), dim3(256), 0, s, b)
  BATCH_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_bfinalize(const BatchArgs &b, float *X, int64_t ldx_out, hipStream_t s) {
  const dim3 g((unsigned)((b.base.n + 255) / 256), (unsigned)b.m);
  hipLaunchKernelGGL(k_bfinalize, g, dim3(256), 0, s, b, X, ldx_out);
  return (int)hipGetLastError();
}

int launch_bset_x0(const BatchArgs &b, const float *X0, int64_t ldx0, hipStream_t s) {
  const dim3 g((unsigned)((b.ldx + 255) / 256), (unsigned)b.m);
  hipLaunchKernelGGL(k_bset_x0, g, dim3(256), 0, s, b, X0, ldx0);
  return (int)hipGetLastError();
}

int launch_bload_x(const BatchArgs &b, const float *X, int64_t ldx_in, hipStream_t s) {
  const dim3 g((unsigned)((b.ldx + 255) / 256), (unsigned)b.m);
  hipLaunchKernelGGL(k_bload_x, g, dim3(256), 0, s, b, X, ldx_in);
  return (int)hipGetLastError();
}

int launch_bcopy_step(const BatchArgs &b, const DevState *src, hipStream_t s) {
  hipLaunchKernelGGL(k_bcopy_step, dim3(1), dim3(256), 0, s, b, src);
  return (int)hipGetLastError();
}

int launch_bphase_reset(const BatchArgs &b, double tol, int32_t max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_bphase_reset, dim3(1), dim3(256), 0, s, b, tol, max_iter);
  return (int)hipGetLastError();
}

int launch_bcopy_anchor(const BatchArgs &b, hipStream_t s) {
  const dim3 g((unsigned)((b.base.n + 255) / 256), (unsigned)b.m);
  hipLaunchKernelGGL(k_bcopy_anchor, g, dim3(256), 0, s, b);
  return (int)hipGetLastError();
}

int launch_bstatus(const BatchArgs &b, int32_t *out, int32_t *act, int32_t *mact, hipStream_t s) {
  if (b.m > 1024) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bstatus, dim3(1), dim3(256), 0, s, b, out, act, mact);
  return (int)hipGetLastError();
}

int launch_bact_all(const BatchArgs &b, int32_t *act, int32_t *mact, hipStream_t s) {
  hipLaunchKernelGGL(k_bact_all, dim3(1), dim3(256), 0, s, b.m, act, mact);
  return (int)hipGetLastError();
}

int launch_zero_f32(float *p, int64_t count, hipStream_t s) {
  const int64_t blocks = (count + 255) / 256;
  const int g = (int)(blocks < 1024 ? (blocks < 1 ? 1 : blocks) : 1024);
  hipLaunchKernelGGL(k_zero_f32, dim3(g), dim3(256), 0, s, p, count);
  return (int)hipGetLastError();
}

}  // namespace npga
