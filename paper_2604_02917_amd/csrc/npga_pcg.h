// Preconditioner of the refinement's face solves (paper Sec. 3.1: the
// float64 KKT refinement minimises f on a face of F by conjugate gradients).
//
// The face Hessian H_FF = 2 (L L^T)_FF of a factor model has a few large
// eigenvalues (the common factors) above a narrow bulk (the idiosyncratic
// part): plain CG spends about one iteration per outlier on every face and
// then converges at the rate of the bulk.  A randomized Nystrom
// approximation of H from one multi-vector product Y = H Omega (Omega:
// n x k signs, k = 32) gives the preconditioner on the face F
//     M_F = sigma I + Y_F S^{-1} Y_F^T,   S = Omega^T Y,
// with sigma the smallest eigenvalue of the Nystrom approximation on the
// face (the top of the bulk it leaves out), and by the Woodbury identity
//     M_F^{-1} v = (v - Y_F K^{-1} Y_F^T v) / sigma,   K = sigma S + Y_F^T Y_F.
// The face CG then runs preconditioned and projected onto the equality
// rows of the face in the M metric: z = M_F^{-1}(g - lam 1 - nu mu) with
// (lam, nu) such that 1^T z = mu^T z = 0, from a1 = M_F^{-1} 1_F and
// a2 = M_F^{-1} mu_F.  The preconditioner changes the path of the solve,
// not its result: the refinement stops on the same KKT test.
//
// All routines run in one workgroup of 8 wavefronts (thread t owns rows
// t + 512 j, j < E; with 256 registers per lane the per-row vectors stay in
// registers).  Y is stored in float32 twice: row-major (row i at pre_y +
// 32 i) for the Gram products on the matrix cores, and column-major
// (column c at pre_yt + c ldp) for the two passes of every application of
// M_F^{-1}, in which a load instruction then reads 64 consecutive rows of
// one column (with a row per thread and float4 loads, each instruction
// touched 64 cache lines and the passes took 18 us each at n = 5440).
// S, the Cholesky factor of K and the scalars live in pre_mat (float64).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"

namespace npga {

constexpr int kPcgWaves = 8;
constexpr int kPcgThreads = 64 * kPcgWaves;
constexpr int kPreKK = kPreK * kPreK;
static_assert(kPreKK % kPcgThreads == 0, "k x k entries per thread");

// Scalars of pre_mat after the two k x k blocks (S, the Cholesky factor).
constexpr int kPreSigma = 2 * kPreK * kPreK;
constexpr int kPreA11 = kPreSigma + 1;
constexpr int kPreA12 = kPreSigma + 2;
constexpr int kPreA22 = kPreSigma + 3;
constexpr int kPreOk = kPreSigma + 4;

// Sign draws of Omega: the splitmix64 finalizer of (32 i + c), low bit.
__device__ __forceinline__ float pre_omega(int64_t i, int c) {
  uint64_t z = (uint64_t)i * (uint64_t)kPreK + (uint64_t)c + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (z & 1u) ? 1.0f : -1.0f;
}

// LDS of the preconditioner routines (about 100 KB).  The k x k factors
// are kept with rows of kPreLd = k + 1 doubles, so that a lane per row
// reading one column hits distinct banks.
constexpr int kPreLd = kPreK + 1;
struct PcgShared {
  double part[kPcgWaves * kPreKK];        // per-wavefront k x k partial products (then S, padded)
  double kc[kPreK * kPreLd];               // K, then its Cholesky factor (lower)
  double m2[kPreK * kPreK];                // Y_F^T Y_F
  double m3[kPreK * kPreLd];               // Cholesky factor of Y_F^T Y_F
  double dinv[kPreK];                      // reciprocal pivots of kc's factor
  double dinv3[kPreK];                     // reciprocal pivots of m3's factor
  double t[kPcgWaves * kPreK];             // per-wavefront partial sums of Y^T v
  double s[kPreK];                         // K^{-1} Y^T v
  double s2[kPreK];                        // K^{-1} Y_F^T mu_F (a face change)
  double scal[8];                          // sigma, A11, A12, A22, ok (as pre_mat's scalars)
  int last;                                // this workgroup arrived last
};

// Sum over the wavefront of eight values per lane; lane l returns the total
// of column 4 b5 + 2 b4 + b3 (b = bits of l).  Fixed shuffle pattern, so
// every lane of a group gets the same bits.
__device__ __forceinline__ double wave_reduce8(double (&t)[8], int lane) {
  {
    const bool hi = (lane & 32) != 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double send = hi ? t[q] : t[q + 4];
      const double keep = hi ? t[q + 4] : t[q];
      t[q] = keep + __shfl_xor(send, 32);
    }
  }
  {
    const bool hi = (lane & 16) != 0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double send = hi ? t[q] : t[q + 2];
      const double keep = hi ? t[q + 2] : t[q];
      t[q] = keep + __shfl_xor(send, 16);
    }
  }
  {
    const bool hi = (lane & 8) != 0;
    const double send = hi ? t[0] : t[1];
    const double keep = hi ? t[1] : t[0];
    t[0] = keep + __shfl_xor(send, 8);
  }
  double r = t[0];
  r += __shfl_xor(r, 4);
  r += __shfl_xor(r, 2);
  r += __shfl_xor(r, 1);
  return r;
}

// Solves C C^T s = v in wavefront 0 (lanes 0..31 hold v_c, return s_c),
// C lower triangular in LDS (rows of kPreLd), dinv its reciprocal pivots.
__device__ __forceinline__ double chol_solve_lanes(const double *C, const double *dinv, double v, int lane) {
#pragma unroll 8
  for (int c = 0; c < kPreK; ++c) {
    const double yc = __shfl(v, c) * dinv[c];
    if (lane > c && lane < kPreK) v = fma(-C[lane * kPreLd + c], yc, v);
    if (lane == c) v = yc;
  }
#pragma unroll 8
  for (int c = kPreK - 1; c >= 0; --c) {
    const double sc = __shfl(v, c) * dinv[c];
    if (lane < c) v = fma(-C[c * kPreLd + lane], sc, v);
    if (lane == c) v = sc;
  }
  return v;
}

// out = sum_i w_i y_i^T over this workgroup's kPcgThreads rows (OMEGA:
// w_i = Omega row i over all rows, the block's part of S = Omega^T Y; else
// w_i = y_i on the face's rows, its part of Y_F^T Y_F), into global memory,
// on v_mfma_f64_16x16x4f64: the float32 entries of Y are exact in float64
// and so are their products, and the sums are float64 (float32 sums would
// bury the bulk of the spectrum, ~1e-7 of the factor part of Y^T Y, in
// rounding).  64 rows per wavefront, 2 x 2 blocks of 16 x 16; the
// wavefront partials added in a fixed order.
template <bool OMEGA>
__device__ __forceinline__ void pcg_gram_rows(const SolveArgs &a, PcgShared &sh, double *out) {
  typedef double pcg_d4 __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = a.n;
  const int64_t r0 = (int64_t)blockIdx.x * kPcgThreads + 64 * wave;
  const int64_t r1 = (r0 + 64 < n) ? r0 + 64 : n;
  const int c = lane & 15, kq = lane >> 4;
  pcg_d4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = pcg_d4{0.0, 0.0, 0.0, 0.0};
  // eight 4-row steps per batch, all loads issued before the products (a
  // load-then-multiply step per iteration waits on memory every time)
  constexpr int kB = 8;
  for (int64_t b0 = r0; b0 < r1; b0 += 4 * kB) {
    float yb[kB][2];
    bool kb[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int64_t i = b0 + 4 * u + kq;
      kb[u] = i < r1 && (OMEGA || a.fvec[i] > 0.0);
#pragma unroll
      for (int p = 0; p < 2; ++p) yb[u][p] = (i < r1) ? a.pre_y[i * kPreK + 16 * p + c] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int64_t i = b0 + 4 * u + kq;
      double yv[2], wv[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        yv[p] = (double)yb[u][p];
        wv[p] = OMEGA ? ((i < r1) ? (double)pre_omega(i, 16 * p + c) : 0.0) : (kb[u] ? yv[p] : 0.0);
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(wv[p], yv[q], acc[p][q], 0, 0, 0);
    }
  }
  // 16 x 16 output layout: lane (kq, c), register v -> row kq + 4 v, column c
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) sh.part[wave * kPreKK + (16 * p + kq + 4 * v) * kPreK + 16 * q + c] = acc[p][q][v];
  __syncthreads();
  for (int e = tid; e < kPreKK; e += kPcgThreads) {
    double ev = 0.0, od = 0.0;
#pragma unroll
    for (int w = 0; w < kPcgWaves; w += 2) {
      ev += sh.part[w * kPreKK + e];
      od += sh.part[(w + 1) * kPreKK + e];
    }
    out[e] = ev + od;
  }
  __syncthreads();
}

// out (LDS) = the sum over the row blocks, in block order, of their
// partial products (block b's at gp + (2 b + which) kPreKK).
__device__ __forceinline__ void pcg_gram_sum(const double *gp, int blocks, int which, double *out) {
  for (int e = threadIdx.x; e < kPreKK; e += kPcgThreads) {
    const double *g = gp + (int64_t)which * kPreKK + e;
    double acc = 0.0;
    for (int b0 = 0; b0 < blocks; b0 += 4) {
      double v[4];  // four loads in flight, then their sums in order
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = (b0 + u < blocks) ? g[(int64_t)(b0 + u) * 2 * kPreKK] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += v[u];
    }
    out[e] = acc;
  }
  __syncthreads();
}

// Y_F^T 1_F and Y_F^T mu_F over this workgroup's kPcgThreads rows (one per
// thread) into out[0, kPreK) and out[kPreK, 2 kPreK); tw: 2 kPcgWaves kPreK
// doubles of LDS.
__device__ __forceinline__ void pcg_face_ysum(const SolveArgs &a, double *tw, double *out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i = (int64_t)blockIdx.x * kPcgThreads + tid;
  const bool on = i < a.n && a.fvec[i] > 0.0;
  const double wmu = on ? a.mu[i] : 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int q = 0; q < kPreK / 8; ++q) {
      double t8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (on) {
        const float *yc = a.pre_yt + (int64_t)(8 * q) * a.ldp + i;
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) t8[cc] = h ? (double)yc[cc * a.ldp] * wmu : (double)yc[cc * a.ldp];
      }
      const double v = wave_reduce8(t8, lane);
      if ((lane & 7) == 0)
        tw[(h * kPcgWaves + wave) * kPreK + 8 * q + 4 * (lane >> 5) + 2 * ((lane >> 4) & 1) + ((lane >> 3) & 1)] = v;
    }
  }
  __syncthreads();
  if (tid < 2 * kPreK) {
    const double *th = tw + (tid >> 5) * kPcgWaves * kPreK + (tid & 31);
    double e = 0.0, o = 0.0;
#pragma unroll
    for (int w = 0; w < kPcgWaves; w += 2) {
      e += th[w * kPreK];
      o += th[(w + 1) * kPreK];
    }
    out[tid] = e + o;
  }
  __syncthreads();
}

// In-place lower Cholesky factor of the k x k matrix A in LDS (rows of
// kPreLd), its reciprocal pivots into dinv; false if a pivot is not
// positive (then A is left partly factored).
__device__ __forceinline__ bool pcg_cholesky(double *A, double *dinv) {
  const int tid = threadIdx.x;
  bool ok = true;
  for (int c = 0; c < kPreK; ++c) {
    const double d = A[c * kPreLd + c];
    ok = ok && d > 0.0;
    const double rd = (d > 0.0) ? sqrt(d) : 1.0;
    __syncthreads();
    if (tid >= c && tid < kPreK) A[tid * kPreLd + c] = (tid == c) ? rd : A[tid * kPreLd + c] / rd;
    if (tid == c) dinv[c] = 1.0 / rd;
    __syncthreads();
    for (int e = tid; e < kPreKK; e += kPcgThreads) {
      const int r = e >> 5, q = e & 31;
      if (q > c && r >= q) A[r * kPreLd + q] = fma(-A[r * kPreLd + c], A[q * kPreLd + c], A[r * kPreLd + q]);
    }
    __syncthreads();
  }
  return ok;
}

// z = fr (v - Y_F K^{-1} Y_F^T v) / sigma for v zero off the face; with
// lowrank false, z = v / sigma.  sh.kc holds the Cholesky factor of K.
template <int E>
__device__ __forceinline__ void pcg_apply(const SolveArgs &a, const double (&v)[E], const double (&fr)[E], double (&z)[E],
                          PcgShared &sh, double sigma, bool lowrank) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = a.n;
  if (lowrank) {
#pragma unroll
    for (int q = 0; q < kPreK / 8; ++q) {
      double t8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int64_t i = tid + kPcgThreads * j;
        if (i < n && fr[j] > 0.0) {
          // column-major Y: lanes read consecutive rows of one column
          const float *yc = a.pre_yt + (int64_t)(8 * q) * a.ldp + i;
#pragma unroll
          for (int cc = 0; cc < 8; ++cc) t8[cc] = fma((double)yc[cc * a.ldp], v[j], t8[cc]);
        }
      }
      const double r = wave_reduce8(t8, lane);
      if ((lane & 7) == 0) sh.t[wave * kPreK + 8 * q + 4 * (lane >> 5) + 2 * ((lane >> 4) & 1) + ((lane >> 3) & 1)] = r;
    }
    __syncthreads();
    if (wave == 0) {
      double tc = 0.0;
      if (lane < kPreK) {
        double e = 0.0, o = 0.0;
#pragma unroll
        for (int w = 0; w < kPcgWaves; w += 2) {
          e += sh.t[w * kPreK + lane];
          o += sh.t[(w + 1) * kPreK + lane];
        }
        tc = e + o;
      }
      tc = chol_solve_lanes(sh.kc, sh.dinv, tc, lane);
      if (lane < kPreK) sh.s[lane] = tc;
    }
    __syncthreads();
  }
  const double inv = 1.0 / sigma;
  // K^{-1} Y^T v in registers while the rows' vectors leave room (n <= 6144)
  constexpr bool kHoist = E <= 12;
  double sv[kHoist ? kPreK : 1];
  if constexpr (kHoist) {
#pragma unroll
    for (int c = 0; c < kPreK; ++c) sv[c] = lowrank ? sh.s[c] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + kPcgThreads * j;
    double w = v[j];
    if (lowrank && i < n && fr[j] > 0.0) {
      const float *yc = a.pre_yt + i;
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < kPreK; ++c) acc = fma((double)yc[c * a.ldp], kHoist ? sv[kHoist ? c : 0] : sh.s[c], acc);
      w -= acc;
    }
    z[j] = (i < n && fr[j] > 0.0) ? w * inv : 0.0;
  }
}

// Preconditioner for the face fr: K = sigma S + Y_F^T Y_F and its Cholesky
// factor (into sh.kc and pre_mat), then a1, a2 and the 2 x 2 metric of the
// equality rows.  The Gram products come from the row blocks' partials in
// pre_gpart (gblocks blocks).  INIT: S = Omega^T Y is formed and sigma
// estimated on this face (kept for the later faces and rounds of the
// solve).
template <int E, bool INIT>
__device__ __forceinline__ void pcg_face(const SolveArgs &a, const double (&fr)[E], const double (&mu)[E], PcgShared &sh,
                         BlockReducer<5, kPcgWaves> &red, int gblocks) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = a.n;
  double *pm = a.pre_mat;
  pcg_gram_sum(a.pre_gpart, gblocks, 0, sh.m2);
  double sigma;
  if constexpr (INIT) {
    pcg_gram_sum(a.pre_gpart, gblocks, 1, sh.part);
    // S symmetric up to rounding: keep its symmetric part (pre_mat, and
    // padded rows in kc for the matvecs below)
    double sym[kPreKK / kPcgThreads];
#pragma unroll
    for (int u = 0; u < kPreKK / kPcgThreads; ++u) {
      const int e = tid + kPcgThreads * u, r = e >> 5, q = e & 31;
      sym[u] = 0.5 * (sh.part[r * kPreK + q] + sh.part[q * kPreK + r]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPreKK / kPcgThreads; ++u) {
      const int e = tid + kPcgThreads * u, r = e >> 5, q = e & 31;
      pm[e] = sym[u];
      sh.m3[r * kPreLd + q] = sh.m2[e] + ((r == q) ? 1e-12 * sh.m2[r * kPreK + r] : 0.0);
      sh.kc[r * kPreLd + q] = sym[u];
    }
    __syncthreads();
    // sigma = smallest eigenvalue of S^{-1} G on the face: power iteration
    // on G^{-1} S (its largest eigenvalue is 1 / sigma); the ratio settles
    // inside the bulk cluster within a few steps, which is all the choice
    // needs
    const bool okg = pcg_cholesky(sh.m3, sh.dinv3);
    double ratio = 0.0;
    if (wave == 0 && okg) {
      double v = (lane < kPreK) ? 1.0 : 0.0;
      for (int it = 0; it < 16; ++it) {
        double w = 0.0;
#pragma unroll 8
        for (int c = 0; c < kPreK; ++c) {
          const double vc = __shfl(v, c);
          if (lane < kPreK) w = fma(sh.kc[lane * kPreLd + c], vc, w);
        }
        w = chol_solve_lanes(sh.m3, sh.dinv3, (lane < kPreK) ? w : 0.0, lane);
        const double wn = sqrt(wave_sum_f64((lane < kPreK) ? w * w : 0.0));
        const double vn = sqrt(wave_sum_f64((lane < kPreK) ? v * v : 0.0));
        ratio = (vn > 0.0) ? wn / vn : 0.0;
        v = (wn > 0.0 && lane < kPreK) ? w / wn : 0.0;
      }
    }
    if (tid == 0) sh.scal[0] = (ratio > 0.0 && isfinite(ratio)) ? 1.0 / ratio : 0.0;
    __syncthreads();
    sigma = sh.scal[0];
  } else {
    sigma = pm[kPreSigma];
    for (int e = tid; e < kPreKK; e += kPcgThreads) sh.kc[(e >> 5) * kPreLd + (e & 31)] = pm[e];
    __syncthreads();
  }
  // K = sigma S + G (+ a relative 1e-12 on the diagonal)
  for (int e = tid; e < kPreKK; e += kPcgThreads) {
    const int r = e >> 5, q = e & 31;
    sh.kc[r * kPreLd + q] = fma(sigma, sh.kc[r * kPreLd + q], sh.m2[e]) + ((r == q) ? 1e-12 * sh.m2[r * kPreK + r] : 0.0);
  }
  __syncthreads();
  bool ok = sigma > 0.0 && pcg_cholesky(sh.kc, sh.dinv);
  if (!(sigma > 0.0)) sigma = 1.0;  // no usable estimate: plain CG (the scale cancels)
  for (int e = tid; e < kPreKK; e += kPcgThreads) pm[kPreKK + e] = sh.kc[(e >> 5) * kPreLd + (e & 31)];
  if (tid == 0) {
    pm[kPreSigma] = sigma;
    pm[kPreOk] = ok ? 1.0 : 0.0;
    sh.scal[0] = sigma;
    sh.scal[4] = ok ? 1.0 : 0.0;
  }
  // a1 = M_F^{-1} 1_F, a2 = M_F^{-1} mu_F and their inner products: Y_F^T 1_F
  // and Y_F^T mu_F from the row blocks' partials (added in block order),
  // K^{-1} of each in its own wavefront, then one pass over Y for both
  if (ok) {
    if (wave < 2) {
      double tc = 0.0;
      if (lane < kPreK) {
        const double *tp = a.pre_gpart + kPreGpartT + wave * kPreK + lane;
        for (int b0 = 0; b0 < gblocks; b0 += 4) {
          double v[4];  // four loads in flight, then their sums in order
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = (b0 + u < gblocks) ? tp[(int64_t)(b0 + u) * 2 * kPreK] : 0.0;
#pragma unroll
          for (int u = 0; u < 4; ++u) tc += v[u];
        }
      }
      tc = chol_solve_lanes(sh.kc, sh.dinv, tc, lane);
      if (lane < kPreK) (wave ? sh.s2 : sh.s)[lane] = tc;
    }
    __syncthreads();
  }
  const double inv = 1.0 / sigma;
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + kPcgThreads * j;
    double w1 = 0.0, w2 = 0.0;
    if (i < n && fr[j] > 0.0) {
      double p1 = 0.0, p2 = 0.0;
      if (ok) {
        const float *yc = a.pre_yt + i;
#pragma unroll
        for (int c = 0; c < kPreK; ++c) {
          const double y = (double)yc[c * a.ldp];
          p1 = fma(y, sh.s[c], p1);
          p2 = fma(y, sh.s2[c], p2);
        }
      }
      w1 = (1.0 - p1) * inv;
      w2 = (mu[j] - p2) * inv;
    }
    acc[0] += w1;
    acc[1] = fma(mu[j], w1, acc[1]);
    acc[2] = fma(mu[j], w2, acc[2]);
    if (i < n) {
      a.pre_a1[i] = w1;
      a.pre_a2[i] = w2;
    }
  }
  red.sum(acc);
  if (tid == 0) {
    pm[kPreA11] = acc[0];
    pm[kPreA12] = acc[1];
    pm[kPreA22] = acc[2];
    sh.scal[1] = acc[0];
    sh.scal[2] = acc[1];
    sh.scal[3] = acc[2];
  }
  __syncthreads();
}

// Preconditioned projected gradient z of g on the face and rz = g^T z.
// fresh: pcg_face ran earlier in this launch (its factor and scalars are in
// LDS); else they are loaded from pre_mat.  lsq: the least-squares
// multipliers (lam0, nu0) of g on the face are given (the tail's), else
// formed here.
template <int E>
__device__ __forceinline__ void pcg_direction(const SolveArgs &a, const double (&g)[E], const double (&fr)[E],
                                              const double (&mu)[E], bool active, bool fresh, bool lsq,
                                              double lam0, double nu0, PcgShared &sh,
                                              BlockReducer<5, kPcgWaves> &red, double (&z)[E], double &rz) {
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  if (!fresh) {
    const double *pm = a.pre_mat;
    for (int e = tid; e < kPreKK; e += kPcgThreads) sh.kc[(e >> 5) * kPreLd + (e & 31)] = pm[kPreKK + e];
    if (tid < kPreK) sh.dinv[tid] = 1.0 / pm[kPreKK + tid * kPreK + tid];
    if (tid == 0) {
      sh.scal[0] = pm[kPreSigma];
      sh.scal[1] = pm[kPreA11];
      sh.scal[2] = pm[kPreA12];
      sh.scal[3] = pm[kPreA22];
      sh.scal[4] = pm[kPreOk];
    }
    __syncthreads();
  }
  const double sigma = sh.scal[0];
  const bool ok = sh.scal[4] > 0.5;
  // the residual r = g - lam0 1 - nu0 mu with the least-squares multipliers
  // first: near the solution g is almost all constraint part, so applying
  // M^{-1} to g and projecting afterwards (or forming g^T z) would cancel
  // most of the digits; r is small and M^{-1} r keeps them
  if (!lsq) {
    double acc0[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      acc0[0] += fr[j];
      acc0[1] = fma(fr[j], mu[j], acc0[1]);
      acc0[2] = fma(fr[j] * mu[j], mu[j], acc0[2]);
      acc0[3] = fma(fr[j], g[j], acc0[3]);
      acc0[4] = fma(fr[j] * mu[j], g[j], acc0[4]);
    }
    red.sum(acc0);
    lam0 = (acc0[0] > 0.0) ? acc0[3] / acc0[0] : 0.0;
    nu0 = 0.0;
    if (active && acc0[0] > 1.5) {
      const double det = acc0[0] * acc0[2] - acc0[1] * acc0[1];
      if (det > 1e-30 * acc0[0] * acc0[2]) {
        lam0 = (acc0[2] * acc0[3] - acc0[1] * acc0[4]) / det;
        nu0 = (acc0[0] * acc0[4] - acc0[1] * acc0[3]) / det;
      }
    }
  }
  double rv[E];
#pragma unroll
  for (int j = 0; j < E; ++j) rv[j] = (fr[j] > 0.0) ? g[j] - lam0 - nu0 * mu[j] : 0.0;
  pcg_apply<E>(a, rv, fr, z, sh, sigma, ok);
  // then the M-metric projection onto 1^T z = 0 (and mu^T z = 0), and
  // r^T z = r^T zr - lam r^T a1 - nu r^T a2 from the same reduction
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + kPcgThreads * j;
    const double a1 = (i < n) ? a.pre_a1[i] : 0.0;
    const double a2 = (i < n) ? a.pre_a2[i] : 0.0;
    acc[0] += z[j];
    acc[1] = fma(mu[j], z[j], acc[1]);
    acc[2] = fma(rv[j], z[j], acc[2]);
    acc[3] = fma(rv[j], a1, acc[3]);
    acc[4] = fma(rv[j], a2, acc[4]);
  }
  red.sum(acc);
  const double A11 = sh.scal[1], A12 = sh.scal[2], A22 = sh.scal[3];
  double lam = (A11 > 0.0) ? acc[0] / A11 : 0.0, nu = 0.0;
  if (active) {
    const double det = A11 * A22 - A12 * A12;
    if (det > 1e-30 * A11 * A22) {
      lam = (A22 * acc[0] - A12 * acc[1]) / det;
      nu = (A11 * acc[1] - A12 * acc[0]) / det;
    }
  }
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + kPcgThreads * j;
    if (i < n && fr[j] > 0.0) z[j] = fma(-nu, a.pre_a2[i], fma(-lam, a.pre_a1[i], z[j]));
    else z[j] = 0.0;
  }
  rz = acc[2] - lam * acc[3] - nu * acc[4];  // r^T z = g^T z, z being orthogonal to the equality rows
}

}  // namespace npga
