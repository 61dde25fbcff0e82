// NPGA solver kernels for gfx950 (paper Sec. 3.1, Algorithm 1).
//
// One NPGA iteration on the factor path is three launches on one stream:
//   k_sweep   : every wavefront streams whole columns of L_eff and computes
//               u_t = L_{:,t}^T x (wavefront sum), accumulates ||u||^2 and the
//               partial gradient sum_t L_{:,t} u_t in registers; each
//               workgroup writes one partial n-vector.  L_eff is read from
//               HBM exactly once per iteration.
//   k_reduce  : row blocks sum the partial vectors in a fixed order
//               (deterministic), giving g_k = 2 L(L^T x_k) + 2 gamma x_k.
//   k_tail_*  : one workgroup runs the serial tail of the current mode (for
//               NPGA: stopping test, momentum extrapolation, gradient step
//               and the exact projection).  The kernel boundaries order the
//               writes; no workgroup waits on another.
// In the refinement's active-set mode and the adjoint's face CG with the
// preconditioner set, a fourth launch (k_pcg_step) forms the next search
// direction after the tail.
//
// The sweep evaluates the gradient at the iterate x_k rather than at the
// extrapolated point y_k: the gradient is affine in x, so
//   grad f(y_k) = g_k + beta_{k-1} (g_k - g_{k-1}),  y_k = x_k + beta_{k-1}(x_k - x_{k-1}),
// which is Algorithm 1's gradient at y_k, and the stopping test of Sec. 3.1
// (which needs grad f(x_k)) costs one extra projection and no extra sweep.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"
#include "npga_tail.h"

namespace npga {

// --------------------------------------------------------------------------
// small kernels
// --------------------------------------------------------------------------

// Statistics of mu and a finiteness check of mu, one workgroup.
__global__ __launch_bounds__(256) void k_prepare(const double *mu, int64_t n, DevState *st) {
  __shared__ double sh[64];
  double mx = -1.0e308, amx = 0.0, bad = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double m = mu[i];
    if (!isfinite(m)) {
      bad += 1.0;
    } else {
      mx = fmax(mx, m);
      amx = fmax(amx, fabs(m));
    }
  }
  // max reductions by butterfly, then across waves
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off, 64));
    amx = fmax(amx, __shfl_xor(amx, off, 64));
    bad += __shfl_xor(bad, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wave * 3 + 0] = mx;
    sh[wave * 3 + 1] = amx;
    sh[wave * 3 + 2] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = sh[0], b = sh[1], c = sh[2];
    for (int w = 1; w < 4; ++w) {
      a = fmax(a, sh[w * 3 + 0]);
      b = fmax(b, sh[w * 3 + 1]);
      c += sh[w * 3 + 2];
    }
    st->mu_max = a;
    st->mu_absmax = b;
    st->n_nonfinite = c;
  }
}

// dst = src (float32 or float64) or fill; also the padded float32 copy xs.
__global__ __launch_bounds__(256) void k_set_vector(double *dst, const float *s32, const double *s64,
                                                    int64_t n, double fill, float *xs, int64_t npad) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < npad; i += (int64_t)gridDim.x * 256) {
    if (i < n) {
      const double v = s32 ? (double)s32[i] : (s64 ? s64[i] : fill);
      dst[i] = v;
      if (xs) xs[i] = (float)v;
    } else if (xs) {
      xs[i] = 0.0f;
    }
  }
}

// splitmix64 finaliser (Steele, Lea and Flood, 2014) as a counter hash.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// u = r / ||r||, r_i ~ N(0, 1) by Box-Muller on hashed counters (power-method start).
template <int E>
__global__ __launch_bounds__(256) void k_random_unit(double *u, float *xs, int64_t n, uint64_t seed) {
  __shared__ double sh[64];
  BlockReducer<5> red{sh, 0};
  double val[E];
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = threadIdx.x + 256 * j;
    val[j] = 0.0;
    if (i < n) {
      const uint64_t h1 = mix64(seed * 0x100000001B3ull + 2 * (uint64_t)i);
      const uint64_t h2 = mix64(seed * 0x100000001B3ull + 2 * (uint64_t)i + 1);
      const double a = ((double)(h1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
      const double b = (double)(h2 >> 11) * (1.0 / 9007199254740992.0);
      val[j] = sqrt(-2.0 * log(a)) * cos(6.283185307179586 * b);
      acc[0] = fma(val[j], val[j], acc[0]);
    }
  }
  red.sum(acc);
  const double inv = 1.0 / sqrt(acc[0]);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = threadIdx.x + 256 * j;
    if (i < n) {
      u[i] = val[j] * inv;
      xs[i] = (float)(val[j] * inv);
    } else {
      // the padding up to 256 E entries is read by the sweeps; later
      // writers of xs store only the first n entries
      xs[i] = 0.0f;
    }
  }
}

__global__ void k_set_tolphi(DevState *st, double proj_tol) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->tolphi = proj_tol * fmax(fabs(st->r), st->mu_absmax);
}

// alpha = 1 / (safety * L_f_hat), L_f_hat = 2 (rho^2 + gamma) (Sec. 3.1 "Fixed step").
// alpha = 1/(safety L_f_hat) with L_f_hat = 2 (rho2 + gamma), or the caller's
// alpha_fixed > 0 (L_f_hat then reports 1/alpha_fixed).
__global__ void k_set_alpha(DevState *st, double safety, double alpha_fixed) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (st->done == kConverged) st->done = kRunning;  // end of a Lanczos estimate
    if (alpha_fixed > 0.0) {
      st->alpha = alpha_fixed;
      st->lipschitz = 1.0 / alpha_fixed;
    } else {
      const double lf = 2.0 * (st->rho2 + st->gamma);
      st->lipschitz = lf;
      st->alpha = (lf > 0.0) ? 1.0 / (safety * lf) : 1.0;
    }
    // strongly convex specialization: m_f = 2 gamma
    const double q = sqrt(st->alpha * 2.0 * st->gamma);
    st->beta_const = (1.0 - q) / (1.0 + q);
  }
}

// Start of the refinement phase: momentum restarts from x_k (t = 1, beta = 0).
__global__ void k_phase_reset(DevState *st, double tol, int32_t max_iter, int32_t window) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->cg_window = window;
    st->done = kRunning;
    st->tol = tol;
    st->max_iter = max_iter;
    st->restart = 1;
    st->t = 1.0;
    st->beta = 0.0;
    st->pcg_arrive = 0;
  }
}

__global__ void k_phase(DevState *st, double tol, int32_t max_iter, int32_t restart) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->done = kRunning;
    st->tol = tol;
    st->max_iter = max_iter;
    st->restart = restart;
    st->pcg_arrive = 0;
  }
}

// --------------------------------------------------------------------------
// fused gradient sweep
// --------------------------------------------------------------------------
template <int E, typename TL>
__global__ __launch_bounds__(256) void k_sweep(SolveArgs a) {
  if (a.st->done != kRunning) return;
  __shared__ f4 sh[4 * 64 * E];
  __shared__ double shu[4];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t n = a.n;
  const int64_t W = (int64_t)gridDim.x * 4;
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave;
  const bool ragged = (n & 3) != 0;

  f4 xr[E], g[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    xr[j] = *reinterpret_cast<const f4 *>(a.xs + 4 * lane + 256 * j);
    g[j] = f4{0.f, 0.f, 0.f, 0.f};
  }
  double usq = 0.0;

  const TL *Lt = static_cast<const TL *>(a.L);
  auto load = [&](f4(&c)[E], int64_t col) {
    const TL *p = Lt + col * a.ld + 4 * lane;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t row0 = 4 * lane + 256 * j;
      c[j] = (row0 < n) ? load4_nt<TL>(p + 256 * j) : f4{0.f, 0.f, 0.f, 0.f};
    }
    if (ragged) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int64_t row0 = 4 * lane + 256 * j;
        if (row0 + 1 >= n) c[j].y = 0.f;
        if (row0 + 2 >= n) c[j].z = 0.f;
        if (row0 + 3 >= n) c[j].w = 0.f;
      }
    }
  };
  int64_t col_cur = 0;
  auto process = [&](const f4(&c)[E]) {
    float d = 0.f;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      d = fmaf(c[j].x, xr[j].x, d);
      d = fmaf(c[j].y, xr[j].y, d);
      d = fmaf(c[j].z, xr[j].z, d);
      d = fmaf(c[j].w, xr[j].w, d);
    }
    d = wave_sum_f32(d);
    // with a refinement anchor, u_t = (L^T x_a)_t + (L^T d)_t
    const double ut = a.ua ? a.ua[col_cur] + (double)d : (double)d;
    usq = fma(ut, ut, usq);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      g[j].x = fmaf(c[j].x, d, g[j].x);
      g[j].y = fmaf(c[j].y, d, g[j].y);
      g[j].z = fmaf(c[j].z, d, g[j].z);
      g[j].w = fmaf(c[j].w, d, g[j].w);
    }
  };

  f4 c0[E], c1[E];
  int64_t col = gw;
  if (col < a.cols) load(c0, col);
  while (col < a.cols) {
    const int64_t col1 = col + W;
    if (col1 < a.cols) load(c1, col1);
    col_cur = col;
    process(c0);
    if (col1 >= a.cols) break;
    const int64_t col2 = col1 + W;
    if (col2 < a.cols) load(c0, col2);
    col_cur = col1;
    process(c1);
    col = col2;
  }

  // combine the four wavefronts in a fixed order
#pragma unroll
  for (int j = 0; j < E; ++j) sh[wave * 64 * E + lane + 64 * j] = g[j];
  if (lane == 0) shu[wave] = usq;
  __syncthreads();
  float *out = a.partials + (int64_t)blockIdx.x * a.ldp;
  for (int q = threadIdx.x; q < 64 * E; q += 256) {
    f4 s = sh[q];
    s += sh[64 * E + q];
    s += sh[2 * 64 * E + q];
    s += sh[3 * 64 * E + q];
    *reinterpret_cast<f4 *>(out + 4 * q) = s;
  }
  if (threadIdx.x == 0) a.usq_part[blockIdx.x] = ((shu[0] + shu[1]) + shu[2]) + shu[3];
}

// Bfloat16 sweep with 16-byte loads: lane l holds rows 8l + 512j .. +7 of
// slot j, kept as raw 16-bit pairs in the double buffer (half the registers
// of converted values) and widened to float32 only when used.  Same partial
// layout as k_sweep: the float4 group q = 2l + h + 128j covers rows 4q..4q+3.
// Requires 16-byte alignment of L and ld % 8 == 0 (checked by the launcher);
// rows n..ld-1 of a column are read and masked to zero.
template <int E2, bool RAGGED, int NW>
__global__ __launch_bounds__(64 * NW) void k_sweep_b16(SolveArgs a) {
  static_assert(NW == 4 || NW == 8, "four or eight wavefronts");
  constexpr int E = 2 * E2;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  if (a.st->done != kRunning) return;
  __shared__ f4 sh[4 * 64 * E];
  __shared__ f4 xsh[64 * E];  // x, read by every wavefront; later the usq sums
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t n = a.n;
  const int64_t W = (int64_t)gridDim.x * NW;
  const int64_t gw = (int64_t)blockIdx.x * NW + wave;
  // zero that the compiler cannot see through (this kernel runs on bfloat16
  // factors only): the gradient update widens the raw column again instead
  // of keeping the widened values of the dot product live across its sum
  const unsigned int z = (unsigned int)(a.dtype - NPGA_BF16);

  // x in LDS (float4 2j + h of lane l at xsh[(2j + h) 64 + l]) leaves the
  // registers to g and two raw columns, so up to n = 5632 (7168 when n % 8
  // is 0) two wavefronts fit on a SIMD (NW = 8)
  for (int q = threadIdx.x; q < 64 * E; q += 64 * NW) {
    const int j2 = q >> 6, l = q & 63;
    xsh[q] = *reinterpret_cast<const f4 *>(a.xs + 8 * l + 512 * (j2 >> 1) + 4 * (j2 & 1));
  }
  f4 g[E];
#pragma unroll
  for (int j = 0; j < E; ++j) g[j] = f4{0.f, 0.f, 0.f, 0.f};
  double usq = 0.0;
  __syncthreads();

  const uint16_t *Lt = static_cast<const uint16_t *>(a.L);
  auto load = [&](u4(&c)[E2], int64_t col) {
    const uint16_t *p = Lt + col * a.ld + 8 * lane;
#pragma unroll
    for (int j = 0; j < E2; ++j) {
      const int64_t row0 = 8 * lane + 512 * j;
      c[j] = (row0 < n) ? __builtin_nontemporal_load(reinterpret_cast<const u4 *>(p + 512 * j)) : u4{0u, 0u, 0u, 0u};
    }
  };
  // rows past n inside a loaded 16-byte group (n % 8 != 0 only): masked at
  // use, so the mask never waits on a load still in flight
  auto keep = [&](int j, int w) -> unsigned int {
    if (!RAGGED) return 0xffffffffu;
    const int64_t row = 8 * lane + 512 * j + 2 * w;
    return row + 1 < n ? 0xffffffffu : (row < n ? 0x0000ffffu : 0u);
  };
  auto lo = [](unsigned int w) { return __uint_as_float(w << 16); };
  auto hi = [](unsigned int w) { return __uint_as_float(w & 0xffff0000u); };
  int64_t col_cur = 0;
  auto process = [&](const u4(&c)[E2]) {
    u4 m[E2];
#pragma unroll
    for (int j = 0; j < E2; ++j)
#pragma unroll
      for (int w = 0; w < 4; ++w) m[j][w] = c[j][w] & keep(j, w);
    float d0 = 0.f, d1 = 0.f;
#pragma unroll
    for (int j = 0; j < E2; ++j) {
      const f4 xa = xsh[(2 * j) * 64 + lane], xb = xsh[(2 * j + 1) * 64 + lane];
      d0 = fmaf(lo(m[j][0]), xa.x, d0);
      d1 = fmaf(hi(m[j][0]), xa.y, d1);
      d0 = fmaf(lo(m[j][1]), xa.z, d0);
      d1 = fmaf(hi(m[j][1]), xa.w, d1);
      d0 = fmaf(lo(m[j][2]), xb.x, d0);
      d1 = fmaf(hi(m[j][2]), xb.y, d1);
      d0 = fmaf(lo(m[j][3]), xb.z, d0);
      d1 = fmaf(hi(m[j][3]), xb.w, d1);
      __builtin_amdgcn_sched_barrier(0);  // keep the reads of x next to their use
    }
    const float d = wave_sum_f32(d0 + d1);
    const double ut = a.ua ? a.ua[col_cur] + (double)d : (double)d;
    usq = fma(ut, ut, usq);
#pragma unroll
    for (int j = 0; j < E2; ++j) {
      u4 r;
#pragma unroll
      for (int w = 0; w < 4; ++w) r[w] = (c[j][w] ^ z) & keep(j, w);
      g[2 * j].x = fmaf(lo(r[0]), d, g[2 * j].x);
      g[2 * j].y = fmaf(hi(r[0]), d, g[2 * j].y);
      g[2 * j].z = fmaf(lo(r[1]), d, g[2 * j].z);
      g[2 * j].w = fmaf(hi(r[1]), d, g[2 * j].w);
      g[2 * j + 1].x = fmaf(lo(r[2]), d, g[2 * j + 1].x);
      g[2 * j + 1].y = fmaf(hi(r[2]), d, g[2 * j + 1].y);
      g[2 * j + 1].z = fmaf(lo(r[3]), d, g[2 * j + 1].z);
      g[2 * j + 1].w = fmaf(hi(r[3]), d, g[2 * j + 1].w);
    }
  };

  u4 c0[E2], c1[E2];
  int64_t col = gw;
  if (col < a.cols) load(c0, col);
  while (col < a.cols) {
    const int64_t col1 = col + W;
    if (col1 < a.cols) load(c1, col1);
    col_cur = col;
    process(c0);
    if (col1 >= a.cols) break;
    const int64_t col2 = col1 + W;
    if (col2 < a.cols) load(c0, col2);
    col_cur = col1;
    process(c1);
    col = col2;
  }

  // combine the wavefronts in a fixed order (with eight: wavefront w + 4
  // into w first), then the four sums
  __syncthreads();  // every wavefront is done with x
  double *shu = reinterpret_cast<double *>(xsh);
  const int slot = wave & 3;
  if (NW == 4 || wave >= 4) {
#pragma unroll
    for (int j = 0; j < E2; ++j)
#pragma unroll
      for (int h = 0; h < 2; ++h) sh[slot * 64 * E + 2 * lane + h + 128 * j] = g[2 * j + h];
  }
  if (lane == 0) shu[wave] = usq;
  __syncthreads();
  if (NW == 8 && wave < 4) {
#pragma unroll
    for (int j = 0; j < E2; ++j)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        f4 &t = sh[slot * 64 * E + 2 * lane + h + 128 * j];
        t = g[2 * j + h] + t;
      }
  }
  if (NW == 8) __syncthreads();
  float *out = a.partials + (int64_t)blockIdx.x * a.ldp;
  for (int q = threadIdx.x; q < 64 * E; q += 64 * NW) {
    f4 s = sh[q];
    s += sh[64 * E + q];
    s += sh[2 * 64 * E + q];
    s += sh[3 * 64 * E + q];
    *reinterpret_cast<f4 *>(out + 4 * q) = s;
  }
  if (threadIdx.x == 0) {
    a.usq_part[blockIdx.x] =
        NW == 8 ? (((shu[0] + shu[4]) + (shu[1] + shu[5])) + (shu[2] + shu[6])) + (shu[3] + shu[7])
                : ((shu[0] + shu[1]) + shu[2]) + shu[3];
  }
}

// Row blocks of 64 sum the sweep partials in a fixed order (deterministic)
// and assemble the gradient of the current mode.  No cross-workgroup
// signalling: the serial tail is a separate one-workgroup launch, so the
// kernel boundary orders the writes (a per-workgroup device-scope fence
// costs more than that launch).
__global__ __launch_bounds__(1024) void k_reduce(SolveArgs a) {
  DevState *st = a.st;
  if (st->done != kRunning) return;
  // sixteen groups of 64 rows, so that each thread has at most 16 of the
  // (at most 256) partials to load and all of them are in flight at once
  __shared__ double red[16][64];
  const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
  if (blockIdx.x == 0) {
    // ||L^T x||^2 from the per-workgroup partials (one per sweep workgroup)
    __shared__ double ubuf[16];
    double u = threadIdx.x < a.sweep_grid ? a.usq_part[threadIdx.x] : 0.0;
    u = wave_sum_f64(u);
    if (r == 0) ubuf[q] = u;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = ubuf[0];
#pragma unroll
      for (int w = 1; w < 16; ++w) t += ubuf[w];
      st->usq_sweep = t;
    }
  }
  const int64_t i = (int64_t)blockIdx.x * 64 + r;
  const int G = a.sweep_grid;
  double s = 0.0;
  if (i < a.n) {
    const float *p = a.partials + i;
#pragma unroll 16
    for (int w = q; w < G; w += 16) s += (double)p[(int64_t)w * a.ldp];
  }
  red[q][r] = s;
  __syncthreads();
  if (q == 0 && i < a.n) {
    double tot = red[0][r];
#pragma unroll
    for (int u = 1; u < 16; ++u) tot += red[u][r];
    if (a.mode == kTailNpga) {
      const double *xk = (st->iter & 1) ? a.xbuf1 : a.xbuf0;
      npga_store_grad_step(a, st, i, 2.0 * tot + (a.ga ? a.ga[i] : 0.0) + 2.0 * st->gamma * xk[i]);
    } else if (a.mode == kTailGrad) {
      a.gbuf0[i] = 2.0 * tot + 2.0 * st->gamma * a.xbuf0[i];
    } else if (a.mode == kTailCG || a.mode == kTailPdas || a.mode == kTailAdj) {
      a.gbuf0[i] = 2.0 * tot + 2.0 * st->gamma * a.pvec[i];
    } else {
      a.gbuf0[i] = tot;
    }
  }
}

// The serial tails of one iteration, one kernel per mode (one workgroup
// each), so that each carries only its own mode's registers.  `covariance`
// selects the objective source: the sweep's ||L^T x||^2 partials on the
// factor path, 1/2 x^T g on the covariance path.  At the end of a chunk
// (a.host_done set) every tail stores the done word for the host.
__device__ __forceinline__ void store_host_done(const SolveArgs &a) {
  if (!a.host_done) return;
  __syncthreads();  // the tail's last state writes, by any thread
  if (threadIdx.x == 0) *a.host_done = a.st->done;
}

template <int E, int NW>
__global__ __launch_bounds__(64 * NW) void k_tail_npga(SolveArgs a, int covariance) {
  __shared__ double redbuf[red_buf_doubles<NW>()];
  DevState *st = a.st;
  if (st->done == kRunning) tail_npga<E, false, false, NW>(a, covariance ? -1.0 : st->usq_sweep, redbuf);
  store_host_done(a);
}

template <int E, int NW>
__global__ __launch_bounds__(64 * NW) void k_tail_cg(SolveArgs a) {
  __shared__ double redbuf[red_buf_doubles<NW>()];
  __shared__ double mbuf[2 * NW];
  __shared__ int64_t ibuf[2 * NW];
  if (a.st->done == kRunning) tail_cg<E, NW>(a, redbuf, mbuf, ibuf);
  store_host_done(a);
}

template <int E, int NW>
__global__ __launch_bounds__(64 * NW) void k_tail_pdas(SolveArgs a) {
  __shared__ double redbuf[red_buf_doubles<NW>()];
  if (a.st->done == kRunning) tail_pdas<E, NW>(a, redbuf);
  store_host_done(a);
}

// Preconditioned direction of the active-set refinement, launched after the
// tail (which left p alone and said in pcg_todo what follows): 1, the next
// CG direction p = -z + (g^T z / pcg_rz) p; 2, the first direction on the
// face the tail has just moved to (the face's factor first).  force = 2:
// the same at the start of a later round (after k_cg_init).  INIT (the
// start of the first round): S = Omega^T Y and sigma on the round's first
// face, its factor, p = -z.  Eight wavefronts.
// The next direction on an unchanged face (pcg_todo = 1) in three launches
// spread over row blocks, one row per thread, where k_pcg_step's single
// workgroup reads Y alone.  The arithmetic is pcg_direction's with
// r = g - lam0 1 - nu0 mu from the tail's multipliers:
//   k_pcg_step (one 512-thread workgroup per 512 rows): partial sums of
//     t = Y_F^T r per row block;
//   k_pcg_dir_z (one 256-thread workgroup per 256 rows): every workgroup
//     adds the partials in block order and solves K s = t (the same s in
//     each), z = (r - Y_F s) / sigma, and partial sums of 1^T z, mu^T z,
//     r^T z, r^T a1, r^T a2;
//   k_pcg_dir_p: every workgroup adds those in block order, projects z in
//     the M metric and writes p = -z + beta p; the last workgroup to
//     finish stores r^T z for the next step.
__device__ __forceinline__ bool pcg_dir_runs(const SolveArgs &a) {
  return a.st->done == kRunning && a.st->pcg_todo == 1;
}

__device__ __forceinline__ double pcg_dir_residual(const SolveArgs &a, int64_t i) {
  const DevState *st = a.st;
  return (i < a.n && a.fvec[i] > 0.0) ? a.gvec[i] - st->pcg_lam0 - st->pcg_nu0 * a.mu[i] : 0.0;
}

// Partial sums of Y_F^T r over this workgroup's kPcgThreads rows into
// pre_part (kPreK per block); tw: kPcgWaves x kPreK doubles of LDS.
__device__ __forceinline__ void pcg_dir_t(const SolveArgs &a, double *tw) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i = (int64_t)blockIdx.x * kPcgThreads + tid;
  const double r = pcg_dir_residual(a, i);
#pragma unroll
  for (int q = 0; q < kPreK / 8; ++q) {
    double t8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (r != 0.0) {
      // column-major Y: lanes read consecutive rows of one column
      const float *yc = a.pre_yt + (int64_t)(8 * q) * a.ldp + i;
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) t8[cc] = (double)yc[cc * a.ldp] * r;
    }
    const double v = wave_reduce8(t8, lane);
    if ((lane & 7) == 0) tw[wave * kPreK + 8 * q + 4 * (lane >> 5) + 2 * ((lane >> 4) & 1) + ((lane >> 3) & 1)] = v;
  }
  __syncthreads();
  if (tid < kPreK) {
    double e = 0.0, o = 0.0;
#pragma unroll
    for (int w = 0; w < kPcgWaves; w += 2) {
      e += tw[w * kPreK + tid];
      o += tw[(w + 1) * kPreK + tid];
    }
    a.pre_part[(int64_t)blockIdx.x * kPreK + tid] = e + o;
  }
}

// A solve's first round start: both partial Gram products (Y_F^T Y_F and
// Omega^T Y) and Y_F^T 1_F, Y_F^T mu_F of each block of kPcgThreads rows.
__global__ __launch_bounds__(kPcgThreads) void k_pcg_gram_init(SolveArgs a) {
  __shared__ PcgShared sh;
  if (a.st->done != kRunning) return;
  pcg_gram_rows<false>(a, sh, a.pre_gpart + (int64_t)blockIdx.x * 2 * kPreKK);
  pcg_gram_rows<true>(a, sh, a.pre_gpart + ((int64_t)blockIdx.x * 2 + 1) * kPreKK);
  pcg_face_ysum(a, sh.part, a.pre_gpart + kPreGpartT + (int64_t)blockIdx.x * 2 * kPreK);
}

template <int E, bool INIT>
__global__ __launch_bounds__(kPcgThreads) void k_pcg_step(SolveArgs a, int force, int gblocks) {
  __shared__ double redbuf[red_buf_doubles<kPcgWaves>()];
  __shared__ PcgShared sh;
  DevState *st = a.st;
  if (st->done != kRunning) return;
  const int todo = INIT ? 3 : (force ? force : st->pcg_todo);
  if (todo == 0) return;
  // a direction on an unchanged face: this launch's blocks take the first
  // of the row-block passes
  if (todo == 1) {
    pcg_dir_t(a, sh.t);
    return;
  }
  // a new face: every block forms its rows' partial Gram product (and
  // Y_F^T 1_F, Y_F^T mu_F); the last
  // block to arrive goes on alone with their sums (at a solve's first round
  // start k_pcg_gram_init has formed both partials and one block runs)
  if constexpr (!INIT) {
    pcg_gram_rows<false>(a, sh, a.pre_gpart + (int64_t)blockIdx.x * 2 * kPreKK);
    pcg_face_ysum(a, sh.part, a.pre_gpart + kPreGpartT + (int64_t)blockIdx.x * 2 * kPreK);
    __threadfence();  // the partials are visible device-wide before the block arrives
    __syncthreads();
    if (threadIdx.x == 0) sh.last = (atomicAdd(&st->pcg_arrive, 1) == (int)gridDim.x - 1) ? 1 : 0;
    __syncthreads();
    if (!sh.last) return;
    __threadfence();  // and read after every block has arrived
    gblocks = (int)gridDim.x;
  }
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  BlockReducer<5, kPcgWaves> red{redbuf, 0};
  double g[E], mu[E], fr[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + kPcgThreads * j;
    const bool ok = i < n;
    mu[j] = ok ? a.mu[i] : 0.0;
    fr[j] = ok ? a.fvec[i] : 0.0;
  }
  const bool active = st->cg_active != 0;
  if (INIT) pcg_face<E, true>(a, fr, mu, sh, red, gblocks);
  else if (todo == 2) pcg_face<E, false>(a, fr, mu, sh, red, gblocks);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + kPcgThreads * j;
    g[j] = (i < n) ? a.gvec[i] : 0.0;
  }
  double z[E], rz;
  // the tail's least-squares multipliers (none at a round's start)
  const bool lsq = force == 0 && !INIT;
  pcg_direction<E>(a, g, fr, mu, active, todo != 1, lsq, lsq ? st->pcg_lam0 : 0.0, lsq ? st->pcg_nu0 : 0.0, sh,
                   red, z, rz);
  const double beta = (todo == 1 && st->pcg_rz > 0.0) ? rz / st->pcg_rz : 0.0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + kPcgThreads * j;
    if (i < n) {
      const double p = (todo == 1) ? fma(beta, a.pvec[i], -z[j]) : -z[j];
      a.pvec[i] = p;
      a.xs[i] = (float)p;
    }
  }
  __syncthreads();  // every thread has read pcg_rz
  if (tid == 0) {
    st->pcg_rz = rz;
    st->pcg_todo = 0;
    st->pcg_arrive = 0;
    if (!isfinite(rz)) st->done = kNumeric;
  }
}

__global__ __launch_bounds__(256) void k_pcg_dir_z(SolveArgs a, int tblocks) {
  __shared__ double kc[kPreK * kPreLd];
  __shared__ double dinv[kPreK];
  __shared__ double sv[kPreK];
  __shared__ double tp[(kPreMaxRowBlocks / 2) * kPreK];
  __shared__ double redbuf[64];
  if (!pcg_dir_runs(a)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double *pm = a.pre_mat;
  const bool lowrank = pm[kPreOk] > 0.5;
  const double sigma = pm[kPreSigma];
  if (lowrank) {
    // every load in flight at once, then the sums from LDS
    for (int e = tid; e < kPreKK; e += 256) kc[(e >> 5) * kPreLd + (e & 31)] = pm[kPreKK + e];
    for (int e = tid; e < tblocks * kPreK; e += 256) tp[e] = a.pre_part[e];
    if (tid < kPreK) dinv[tid] = 1.0 / pm[kPreKK + tid * kPreK + tid];
    __syncthreads();
    if (wave == 0) {
      double tc = 0.0;
      if (lane < kPreK) {
        for (int b = 0; b < tblocks; ++b) tc += tp[b * kPreK + lane];
      }
      tc = chol_solve_lanes(kc, dinv, tc, lane);
      if (lane < kPreK) sv[lane] = tc;
    }
    __syncthreads();
  }
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  const double r = pcg_dir_residual(a, i);
  double z = 0.0;
  if (i < a.n && a.fvec[i] > 0.0) {
    double w = r;
    if (lowrank) {
      const float *yc = a.pre_yt + i;
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < kPreK; ++c) acc = fma((double)yc[c * a.ldp], sv[c], acc);
      w -= acc;
    }
    z = w * (1.0 / sigma);
  }
  const double a1 = (i < a.n) ? a.pre_a1[i] : 0.0;
  const double a2 = (i < a.n) ? a.pre_a2[i] : 0.0;
  const double mu = (i < a.n) ? a.mu[i] : 0.0;
  if (i < a.n) a.pre_z[i] = z;
  double acc[5] = {z, mu * z, r * z, r * a1, r * a2};
  BlockReducer<5> red{redbuf, 0};
  red.sum(acc);
  if (tid < 5) a.pre_part[(int64_t)kPreMaxRowBlocks * kPreK + (int64_t)blockIdx.x * 5 + tid] = acc[tid];
}

__global__ __launch_bounds__(256) void k_pcg_dir_p(SolveArgs a) {
  __shared__ double q5[kPreMaxRowBlocks * 5];
  __shared__ double s5[5];
  DevState *st = a.st;
  if (!pcg_dir_runs(a)) return;
  const int tid = threadIdx.x;
  if (tid < (int)gridDim.x * 5) q5[tid] = a.pre_part[(int64_t)kPreMaxRowBlocks * kPreK + tid];
  __syncthreads();
  if (tid < 5) {
    double v = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) v += q5[b * 5 + tid];
    s5[tid] = v;
  }
  __syncthreads();
  const double *pm = a.pre_mat;
  const double A11 = pm[kPreA11], A12 = pm[kPreA12], A22 = pm[kPreA22];
  double lam = (A11 > 0.0) ? s5[0] / A11 : 0.0, nu = 0.0;
  if (st->cg_active != 0) {
    const double det = A11 * A22 - A12 * A12;
    if (det > 1e-30 * A11 * A22) {
      lam = (A22 * s5[0] - A12 * s5[1]) / det;
      nu = (A11 * s5[1] - A12 * s5[0]) / det;
    }
  }
  const double rz = s5[2] - lam * s5[3] - nu * s5[4];
  const double rz_old = st->pcg_rz;
  const double beta = (rz_old > 0.0) ? rz / rz_old : 0.0;
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  if (i < a.n) {
    const double z = (a.fvec[i] > 0.0) ? fma(-nu, a.pre_a2[i], fma(-lam, a.pre_a1[i], a.pre_z[i])) : 0.0;
    const double p = fma(beta, a.pvec[i], -z);
    a.pvec[i] = p;
    a.xs[i] = (float)p;
  }
  // every workgroup has read pcg_rz and pcg_todo before it arrives; the
  // last one to arrive stores the new values
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    const int prev = atomicAdd(&st->pcg_arrive, 1);
    if (prev == (int)gridDim.x - 1) {
      st->pcg_arrive = 0;
      st->pcg_rz = rz;
      st->pcg_todo = 0;
      if (!isfinite(rz)) st->done = kNumeric;
    }
  }
}

// Omega's signs into the batched GEMM input (column c at X + c ldx, zeros
// past n up to ldx).
__global__ __launch_bounds__(256) void k_pre_omega(float *X, int64_t ldx, int64_t n) {
  const int64_t total = ldx * kPreK;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t c = e / ldx, i = e % ldx;
    X[e] = (i < n) ? pre_omega(i, (int)c) : 0.f;
  }
}

// Y[i][c] = 2 sum_s P[(s n + i) ldpm + c], the splits in order, stored
// row-major (Y) and column-major (Yt).
__global__ __launch_bounds__(256) void k_pre_reduce(const float *P, int64_t ldpm, int32_t splits, int64_t n,
                                                    float *Y, float *Yt, int64_t ldyt) {
  const int64_t total = n * kPreK;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / kPreK, c = e % kPreK;
    double acc = 0.0;
    for (int32_t sp = 0; sp < splits; ++sp) acc += (double)P[((int64_t)sp * n + i) * ldpm + c];
    const float y = (float)(2.0 * acc);
    Y[e] = y;
    Yt[c * ldyt + i] = y;
  }
}

template <int E>
__global__ __launch_bounds__(256) void k_tail_adj(SolveArgs a) {
  __shared__ double redbuf[64];
  if (a.st->done == kRunning) tail_adj<E>(a, redbuf);
  store_host_done(a);
}

template <int E>
__global__ __launch_bounds__(256) void k_tail_power(SolveArgs a, int covariance) {
  __shared__ double redbuf[64];
  DevState *st = a.st;
  if (st->done == kRunning) tail_power<E>(a, covariance ? -1.0 : st->usq_sweep, redbuf);
  store_host_done(a);
}

template <int E>
__global__ __launch_bounds__(256) void k_tail_lanczos(SolveArgs a) {
  __shared__ double redbuf[64];
  if (a.st->done == kRunning) tail_lanczos<E>(a, redbuf);
  store_host_done(a);
}

template <int E>
__global__ __launch_bounds__(256) void k_tail_grad(SolveArgs a, int covariance) {
  __shared__ double redbuf[64];
  DevState *st = a.st;
  if (st->done == kRunning) tail_grad<E>(a, covariance ? -1.0 : st->usq_sweep, redbuf);
  store_host_done(a);
}

// The NPGA tail with Dykstra's projections (options.projection = 1) and/or
// adaptive backtracking (options.backtrack_rho > 0).
template <int E, bool DYK, bool BT>
__global__ __launch_bounds__(256) void k_tail_var(SolveArgs a, int covariance) {
  __shared__ double redbuf[64];
  DevState *st = a.st;
  if (st->done == kRunning) tail_npga<E, DYK, BT>(a, covariance ? -1.0 : st->usq_sweep, redbuf);
  store_host_done(a);
}

template <int E>
__global__ __launch_bounds__(256) void k_project_init(SolveArgs a) {
  __shared__ double redbuf[64];
  if (a.dykstra)
    project_init_body<E, true>(a, redbuf);
  else
    project_init_body<E>(a, redbuf);
}

template <int E>
__global__ __launch_bounds__(256) void k_cg_init(SolveArgs a) {
  __shared__ double redbuf[64];
  cg_init_body<E>(a, redbuf);
}

// Standalone projection (npga_project entry point).
template <int E>
__global__ __launch_bounds__(256) void k_project_only(const double *vin, const double *muin, int64_t n,
                                                      double *xout, DevState *st) {
  __shared__ double redbuf[64];
  BlockReducer<5> red{redbuf, 0};
  const int tid = threadIdx.x;
  double mu[E], v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    mu[j] = (i < n) ? muin[i] : 0.0;
    v[j] = (i < n) ? vin[i] : -1.0e300;
  }
  const ProjResult pr = project_F<E>(v, mu, st->r, st->tolphi, 0.0, -1.0e300, red);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    if (i < n) xout[i] = v[j];
  }
  if (tid == 0) {
    st->nu = pr.nu;
    st->tau = pr.tau;
    st->proj_flags = pr.flags;
    st->iter = pr.passes;
  }
}

// Pi_F(v) by Dykstra's alternating projections alone (the fallback of the
// dual search), for checking it on its own.
template <int E>
__global__ __launch_bounds__(256) void k_project_dykstra(const double *vin, const double *muin, int64_t n,
                                                         double *xout, DevState *st, int max_iter,
                                                         double tol) {
  __shared__ double redbuf[64];
  BlockReducer<5> red{redbuf, 0};
  const int tid = threadIdx.x;
  double mu[E], v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    mu[j] = (i < n) ? muin[i] : 0.0;
    v[j] = (i < n) ? vin[i] : -1.0e300;
  }
  int flags = 0;
  double nu = 0.0, tau = 0.0;
  const int k = dykstra_F<E>(v, mu, st->r, max_iter, tol, red, flags, nu, tau);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    if (i < n) xout[i] = v[j];
  }
  if (tid == 0) {
    st->nu = nu;
    st->tau = tau;
    st->proj_flags = flags;
    st->iter = k;
  }
}

__global__ __launch_bounds__(256) void k_finalize(SolveArgs a, float *x_out) {
  const DevState *st = a.st;
  const double *x = (st->iter & 1) ? a.xbuf1 : a.xbuf0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * 256)
    x_out[i] = (float)x[i];
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
#define NPGA_SLOT_SWITCH(slots, CALL)                                 \
  switch (slots) {                                                   \
    case 1: CALL(1); break;                                          \
    case 2: CALL(2); break;                                          \
    case 4: CALL(4); break;                                          \
    case 8: CALL(8); break;                                          \
    case 12: CALL(12); break;                                        \
    case 16: CALL(16); break;                                        \
    case 22: CALL(22); break;                                        \
    case 28: CALL(28); break;                                        \
    case 32: CALL(32); break;                                        \
    default: return (int)hipErrorInvalidValue;                      \
  }

int slots_for(int64_t n) {
  const int64_t need = (n + 255) / 256;
  static const int buckets[] = {1, 2, 4, 8, 12, 16, 22, 28, 32};
  for (int b : buckets)
    if (need <= b) return b;
  return -1;
}

int launch_prepare(const SolveArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, s, a.mu, a.n, a.st);
  return (int)hipGetLastError();
}

int launch_set_vector(double *dst, const float *src32, const double *src64, int64_t n, double fill,
                      float *xs, hipStream_t s) {
  const int slots = slots_for(n);
  const int64_t npad = xs ? (int64_t)256 * slots : n;  // xs holds 256 * slots floats
  const int grid = (int)((npad + 255) / 256);
  hipLaunchKernelGGL(k_set_vector, dim3(grid), dim3(256), 0, s, dst, src32, src64, n, fill, xs,
                     npad);
  return (int)hipGetLastError();
}

int launch_random_unit(double *u, float *xs, int64_t n, uint64_t seed, hipStream_t s) {
  const int slots = slots_for(n);
#define CALL(E) hipLaunchKernelGGL(k_random_unit<E>, dim3(1), dim3(256), 0, s, u, xs, n, seed)
  NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_sweep(const SolveArgs &a, int slots, hipStream_t s) {
  if (a.dtype == NPGA_BF16) {
    const bool wide = slots >= 2 && (slots & 1) == 0 && (a.ld & 7) == 0 &&
                      (reinterpret_cast<uintptr_t>(a.L) & 15) == 0;
    if (wide) {
#define CALL(E2)                                                                          \
  do {                                                                                    \
    if (a.n & 7) {                                                                        \
      constexpr int NW = (E2 <= 11) ? 8 : 4;                                              \
      hipLaunchKernelGGL((k_sweep_b16<E2, true, NW>), dim3(a.sweep_grid), dim3(64 * NW), 0, s, a); \
    } else {                                                                              \
      constexpr int NW = (E2 <= 14) ? 8 : 4;                                              \
      hipLaunchKernelGGL((k_sweep_b16<E2, false, NW>), dim3(a.sweep_grid), dim3(64 * NW), 0, s, a); \
    }                                                                                     \
  } while (0)
      switch (slots / 2) {
        case 1: CALL(1); break;
        case 2: CALL(2); break;
        case 4: CALL(4); break;
        case 6: CALL(6); break;
        case 8: CALL(8); break;
        case 11: CALL(11); break;
        case 14: CALL(14); break;
        case 16: CALL(16); break;
        default: return (int)hipErrorInvalidValue;
      }
#undef CALL
    } else {
#define CALL(E) hipLaunchKernelGGL((k_sweep<E, bf16_t>), dim3(a.sweep_grid), dim3(256), 0, s, a)
      NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
    }
  } else {
#define CALL(E) hipLaunchKernelGGL((k_sweep<E, float>), dim3(a.sweep_grid), dim3(256), 0, s, a)
    NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
  }
  return (int)hipGetLastError();
}

int launch_reduce_tail(const SolveArgs &a, int slots, hipStream_t s) {
  const int grid = (int)((a.n + 63) / 64);
  hipLaunchKernelGGL(k_reduce, dim3(grid), dim3(1024), 0, s, a);
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
  return launch_tail(a, slots, 0, s);
}

// Wavefronts of the NPGA and CG tails for n > 1024 (thread t of the
// workgroup owns entries t + 64 NW j).  Four (one per SIMD) is the default:
// with eight the tails' reductions alone hold ~50 more registers per lane
// (the compiler keeps every wavefront's partials in flight) and the tails
// spill from 2816 assets up; with four, a 5440-asset tail keeps its vectors
// in registers and accumulation registers, with no scratch.
#ifndef NPGA_TAIL_WAVES
#define NPGA_TAIL_WAVES 4
#endif

// Per-thread entries of the NW-wavefront tails for the 256-thread slot count.
#define NPGA_WIDE_SLOT_SWITCH(slots, CALL)                                                     \
  switch (slots) {                                                                             \
    case 8: CALL((8 * 4 + NPGA_TAIL_WAVES - 1) / NPGA_TAIL_WAVES); break;                       \
    case 12: CALL((12 * 4 + NPGA_TAIL_WAVES - 1) / NPGA_TAIL_WAVES); break;                     \
    case 16: CALL((16 * 4 + NPGA_TAIL_WAVES - 1) / NPGA_TAIL_WAVES); break;                     \
    case 22: CALL((22 * 4 + NPGA_TAIL_WAVES - 1) / NPGA_TAIL_WAVES); break;                     \
    case 28: CALL((28 * 4 + NPGA_TAIL_WAVES - 1) / NPGA_TAIL_WAVES); break;                     \
    case 32: CALL((32 * 4 + NPGA_TAIL_WAVES - 1) / NPGA_TAIL_WAVES); break;                     \
    default: return (int)hipErrorInvalidValue;                                                 \
  }

// Per-thread rows of the 512-thread preconditioner kernel (n >= 2048).
#define NPGA_PCG_SLOT_SWITCH(slots, CALL)                     \
  switch (slots) {                                            \
    case 8: CALL(4); break;                                   \
    case 12: CALL(6); break;                                  \
    case 16: CALL(8); break;                                  \
    case 22: CALL(11); break;                                 \
    case 28: CALL(14); break;                                 \
    case 32: CALL(16); break;                                 \
    default: return (int)hipErrorInvalidValue;                \
  }

// Row blocks of the preconditioner's launches: 512-row blocks of k_pcg_step
// (0 if the buffers are missing or n is too large) and 256-row blocks of
// the direction kernels.
static int pcg_row_blocks(const SolveArgs &a, int *blocks) {
  if (!a.pre_y || !a.pre_yt || !a.pre_mat || !a.pre_a1 || !a.pre_a2 || !a.pre_z || !a.pre_part || !a.pre_gpart)
    return 0;
  const int tblocks = (int)((a.n + kPcgThreads - 1) / kPcgThreads);
  *blocks = (int)((a.n + 255) / 256);
  if (*blocks > kPreMaxRowBlocks || 2 * tblocks > kPreMaxRowBlocks) return 0;
  return tblocks;
}

int launch_pcg_init(const SolveArgs &a, int slots, bool first, hipStream_t s) {
  int blocks = 0;
  const int tblocks = pcg_row_blocks(a, &blocks);
  if (tblocks < 1) return (int)hipErrorInvalidValue;
  if (first) {
    hipLaunchKernelGGL(k_pcg_gram_init, dim3(tblocks), dim3(kPcgThreads), 0, s, a);
#define CALL(E) hipLaunchKernelGGL((k_pcg_step<E, true>), dim3(1), dim3(kPcgThreads), 0, s, a, 0, tblocks)
    NPGA_PCG_SLOT_SWITCH(slots, CALL)
#undef CALL
  } else {
#define CALL(E) hipLaunchKernelGGL((k_pcg_step<E, false>), dim3(tblocks), dim3(kPcgThreads), 0, s, a, 2, 0)
    NPGA_PCG_SLOT_SWITCH(slots, CALL)
#undef CALL
  }
  return (int)hipGetLastError();
}

int launch_pre_omega(float *X, int64_t ldx, int64_t n, hipStream_t s) {
  const int64_t total = ldx * kPreK;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pre_omega, dim3(grid), dim3(256), 0, s, X, ldx, n);
  return (int)hipGetLastError();
}

int launch_pre_reduce(const float *P, int64_t ldpm, int32_t splits, int64_t n, float *Y, float *Yt, int64_t ldyt,
                      hipStream_t s) {
  if (ldyt < n) return (int)hipErrorInvalidValue;
  const int64_t total = n * kPreK;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pre_reduce, dim3(grid), dim3(256), 0, s, P, ldpm, splits, n, Y, Yt, ldyt);
  return (int)hipGetLastError();
}

// The preconditioner's launches after a refinement or adjoint tail: a face
// change (k_pcg_step), else the direction on the same face over row blocks.
int launch_pcg_after_tail(const SolveArgs &a, int slots, hipStream_t s) {
  if (hipGetLastError() != hipSuccess) return (int)hipErrorLaunchFailure;
  int blocks = 0;
  const int tblocks = pcg_row_blocks(a, &blocks);
  if (tblocks < 1) return (int)hipErrorInvalidValue;
#define CALL(E) hipLaunchKernelGGL((k_pcg_step<E, false>), dim3(tblocks), dim3(kPcgThreads), 0, s, a, 0, 0)
  NPGA_PCG_SLOT_SWITCH(slots, CALL)
#undef CALL
  hipLaunchKernelGGL(k_pcg_dir_z, dim3(blocks), dim3(256), 0, s, a, tblocks);
  hipLaunchKernelGGL(k_pcg_dir_p, dim3(blocks), dim3(256), 0, s, a);
  return (int)hipGetLastError();
}

int launch_tail(const SolveArgs &a, int slots, int covariance, hipStream_t s) {
  if ((a.dykstra || a.backtrack) && a.mode == kTailNpga) {
    // the NPGA tail with Dykstra's projections and/or backtracking: own
    // instantiations, so the plain tail carries none of their registers
    if (a.dykstra && a.backtrack) {
#define CALL(E) hipLaunchKernelGGL((k_tail_var<E, true, true>), dim3(1), dim3(256), 0, s, a, covariance)
      NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
    } else if (a.dykstra) {
#define CALL(E) hipLaunchKernelGGL((k_tail_var<E, true, false>), dim3(1), dim3(256), 0, s, a, covariance)
      NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
    } else {
#define CALL(E) hipLaunchKernelGGL((k_tail_var<E, false, true>), dim3(1), dim3(256), 0, s, a, covariance)
      NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
    }
    return (int)hipGetLastError();
  }
  const bool wide = slots >= 8 && NPGA_TAIL_WAVES != 4;
  switch (a.mode) {
    case kTailNpga:
      if (wide) {
#define CALL(E) hipLaunchKernelGGL((k_tail_npga<E, NPGA_TAIL_WAVES>), dim3(1), dim3(64 * NPGA_TAIL_WAVES), 0, s, a, covariance)
        NPGA_WIDE_SLOT_SWITCH(slots, CALL)
#undef CALL
      } else {
#define CALL(E) hipLaunchKernelGGL((k_tail_npga<E, 4>), dim3(1), dim3(256), 0, s, a, covariance)
        NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
      }
      break;
    case kTailCG:
      if (wide) {
#define CALL(E) hipLaunchKernelGGL((k_tail_cg<E, NPGA_TAIL_WAVES>), dim3(1), dim3(64 * NPGA_TAIL_WAVES), 0, s, a)
        NPGA_WIDE_SLOT_SWITCH(slots, CALL)
#undef CALL
      } else {
#define CALL(E) hipLaunchKernelGGL((k_tail_cg<E, 4>), dim3(1), dim3(256), 0, s, a)
        NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
      }
      break;
    case kTailPdas:
      if (wide) {
#define CALL(E) hipLaunchKernelGGL((k_tail_pdas<E, NPGA_TAIL_WAVES>), dim3(1), dim3(64 * NPGA_TAIL_WAVES), 0, s, a)
        NPGA_WIDE_SLOT_SWITCH(slots, CALL)
#undef CALL
      } else {
#define CALL(E) hipLaunchKernelGGL((k_tail_pdas<E, 4>), dim3(1), dim3(256), 0, s, a)
        NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
      }
      if (a.pre_y) return launch_pcg_after_tail(a, slots, s);
      break;
    case kTailAdj:
#define CALL(E) hipLaunchKernelGGL(k_tail_adj<E>, dim3(1), dim3(256), 0, s, a)
      NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
      if (a.pre_y) return launch_pcg_after_tail(a, slots, s);
      break;
    case kTailPower:
#define CALL(E) hipLaunchKernelGGL(k_tail_power<E>, dim3(1), dim3(256), 0, s, a, covariance)
      NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
      break;
    case kTailLanczos:
#define CALL(E) hipLaunchKernelGGL(k_tail_lanczos<E>, dim3(1), dim3(256), 0, s, a)
      NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
      break;
    default:
#define CALL(E) hipLaunchKernelGGL(k_tail_grad<E>, dim3(1), dim3(256), 0, s, a, covariance)
      NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
      break;
  }
  return (int)hipGetLastError();
}

int launch_project_init(const SolveArgs &a, int slots, int /*use_x0*/, hipStream_t s) {
#define CALL(E) hipLaunchKernelGGL(k_project_init<E>, dim3(1), dim3(256), 0, s, a)
  NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_cg_init(const SolveArgs &a, int slots, hipStream_t s) {
#define CALL(E) hipLaunchKernelGGL(k_cg_init<E>, dim3(1), dim3(256), 0, s, a)
  NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_project_only(const double *v, const double *mu, int64_t n, double *x, DevState *st,
                        int slots, hipStream_t s) {
#define CALL(E) hipLaunchKernelGGL(k_project_only<E>, dim3(1), dim3(256), 0, s, v, mu, n, x, st)
  NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_project_dykstra(const double *v, const double *mu, int64_t n, double *x, DevState *st, int max_iter,
                           double tol, int slots, hipStream_t s) {
#define CALL(E) hipLaunchKernelGGL(k_project_dykstra<E>, dim3(1), dim3(256), 0, s, v, mu, n, x, st, max_iter, tol)
  NPGA_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_finalize(const SolveArgs &a, float *x_out, int /*slots*/, hipStream_t s) {
  const int grid = (int)((a.n + 255) / 256);
  hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(256), 0, s, a, x_out);
  return (int)hipGetLastError();
}

int launch_phase_reset(DevState *st, double tol, int32_t max_iter, int32_t window, hipStream_t s) {
  hipLaunchKernelGGL(k_phase_reset, dim3(1), dim3(64), 0, s, st, tol, max_iter, window);
  return (int)hipGetLastError();
}

int launch_set_tolphi(DevState *st, double proj_tol, hipStream_t s) {
  hipLaunchKernelGGL(k_set_tolphi, dim3(1), dim3(64), 0, s, st, proj_tol);
  return (int)hipGetLastError();
}

// Lanczos start: v_0 = xbuf0 (the random unit vector), v_{-1} = 0.
__global__ __launch_bounds__(256) void k_lanczos_init(SolveArgs a, double tol) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * 256) a.xbuf1[i] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.st->lz_m = 0;
    a.st->lz_theta = 0.0;
    a.st->lz_tol = tol;
  }
}

int launch_lanczos_init(const SolveArgs &a, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_lanczos_init, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, tol);
  return (int)hipGetLastError();
}

int launch_set_alpha(DevState *st, double step_safety, hipStream_t s, double alpha_fixed) {
  hipLaunchKernelGGL(k_set_alpha, dim3(1), dim3(64), 0, s, st, step_safety, alpha_fixed);
  return (int)hipGetLastError();
}

int launch_phase(DevState *st, int32_t /*phase_kind*/, double tol, int32_t max_iter, int32_t restart,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_phase, dim3(1), dim3(64), 0, s, st, tol, max_iter, restart);
  return (int)hipGetLastError();
}

}  // namespace npga
