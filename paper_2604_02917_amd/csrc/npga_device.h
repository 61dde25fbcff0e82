// Device helpers: deterministic wavefront/workgroup reductions and the
// exact projection onto F = {x >= 0, 1^T x = 1, mu^T x >= r} (paper Sec. 3.1).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "npga_internal.h"

namespace npga {

typedef float f4 __attribute__((ext_vector_type(4)));

// Element types of the factor L: float32, or bfloat16 kept as its 16 bits.
struct bf16_t {
  uint16_t bits;
};

// Four consecutive entries of a column as float32 (the address is 16-byte
// aligned for float32 and 8-byte aligned for bfloat16).
template <typename TL>
__device__ __forceinline__ f4 load4_nt(const TL *p);

template <>
__device__ __forceinline__ f4 load4_nt<float>(const float *p) {
  return __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p));
}

template <>
__device__ __forceinline__ f4 load4_nt<bf16_t>(const bf16_t *p) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  const u2 w = __builtin_nontemporal_load(reinterpret_cast<const u2 *>(p));
  f4 r;
  r.x = __uint_as_float(w.x << 16);
  r.y = __uint_as_float(w.x & 0xffff0000u);
  r.z = __uint_as_float(w.y << 16);
  r.w = __uint_as_float(w.y & 0xffff0000u);
  return r;
}

// Wavefront sums (all 64 lanes active).  Within each 16-lane row four DPP
// steps (swap neighbours, swap pairs, mirror the half-row, mirror the row)
// leave the row total in every lane of the row; the four row totals are
// read into scalar registers and added in a fixed order, so every lane gets
// the same bits.  DPP moves run in the vector ALU, without the LDS round
// trips of a ds_bpermute shuffle.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ float wave_sum_f32(float v) {
  v += dpp_f32<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f32<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f32<0x141>(v);  // row_half_mirror
  v += dpp_f32<0x140>(v);  // row_mirror
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return ((r0 + r1) + r2) + r3;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  return ((readlane_f64(v, 0) + readlane_f64(v, 16)) + readlane_f64(v, 32)) + readlane_f64(v, 48);
}

// Workgroup-wide sum of K doubles for a workgroup of NW wavefronts.  Every
// thread receives bitwise identical totals: the wave sums are uniform, and
// the NW wave totals are combined in a fixed order (sequentially for four
// wavefronts; beyond, the even and the odd wavefronts in two sequential
// chains, then their sum).  Two LDS buffers alternate so a single barrier
// per call suffices.
template <int NW>
__device__ __forceinline__ double combine_waves(const double *b, int stride) {
  if constexpr (NW == 4) {
    return ((b[0] + b[stride]) + b[2 * stride]) + b[3 * stride];
  } else {
    double e = b[0], o = b[stride];
#pragma unroll
    for (int w = 2; w < NW; w += 2) {
      e += b[w * stride];
      o += b[(w + 1) * stride];
    }
    return e + o;
  }
}

template <int K, int NW = 4>
struct BlockReducer {
  static constexpr int kWaves = NW;
  double *buf;  // shared: 2 * NW * K doubles
  int parity;

  __device__ __forceinline__ void sum(double (&a)[K]) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = wave_sum_f64(a[k]);
    double *b = buf + parity * (NW * K);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) b[wave * K + k] = a[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = combine_waves<NW>(b + k, K);
    parity ^= 1;
  }
};

// LDS doubles a reducer set of NW wavefronts needs: BlockReducer<5> (both
// halves) and the masked pass's BlockReducer<6> (one half).
template <int NW>
constexpr int red_buf_doubles() {
  return 2 * NW * 5 + NW * 6;
}

// Workgroup-wide minimum of (value, index) pairs; ties go to the smaller
// index, so every thread receives the same pair.
struct MinLoc {
  double v;
  int64_t i;
};

__device__ __forceinline__ MinLoc minloc_pick(MinLoc a, MinLoc b) {
  if (b.v < a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

// buf, ibuf: 2 * NW entries each
template <int NW = 4>
__device__ __forceinline__ MinLoc block_minloc(MinLoc m, double *buf, int64_t *ibuf, int &parity) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    MinLoc o;
    o.v = __shfl_xor(m.v, off, 64);
    o.i = __shfl_xor(m.i, off, 64);
    m = minloc_pick(m, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double *b = buf + parity * NW;
  int64_t *bi = ibuf + parity * NW;
  if (lane == 0) {
    b[wave] = m.v;
    bi[wave] = m.i;
  }
  __syncthreads();
  MinLoc r{b[0], bi[0]};
#pragma unroll
  for (int w = 1; w < NW; ++w) r = minloc_pick(r, MinLoc{b[w], bi[w]});
  parity ^= 1;
  return r;
}

// Sums over the support S = {i : v_i + nu mu_i > tau} of one pass.
struct PassSums {
  double c, sv, sm, smm, smv;
};

// Projection of the n-vector held in registers (thread t of the NW
// wavefronts owns entries i = t + 64 NW j, j < E; invalid entries carry
// v = -1e300, mu = 0).
//
// Pi_F(v) = Pi_Delta(v + nu mu) for the nu >= 0 that satisfies the
// complementarity of the return constraint (eq. projF-dualpath), with
// Pi_Delta(w)_i = max(w_i - tau, 0) and sum_i max(w_i - tau, 0) = 1
// (eq. simplex-tau / simplex-proj).
//
// tau(nu) is found without sorting by the monotone Newton (Michelot)
// iteration tau <- (sum_{w_i > tau} w_i - 1) / #{w_i > tau}: from a point
// left of the root it increases to the root in finitely many steps; from a
// point right of it the first step lands left of it.  The loop ends when
// the recomputed tau repeats bitwise, which happens exactly when the
// support is unchanged, so the final tau is the exact threshold of that
// support.  A correct guess costs one pass.
//
// The outer search solves phi(nu) = mu^T x(nu) = r.  phi is nondecreasing
// and affine between support changes: on a fixed support S,
// phi(nu) = sum_S mu v + nu sum_S mu^2 - tau(nu) sum_S mu with
// tau(nu) = (sum_S v + nu sum_S mu - 1)/|S|, so a Newton step from any
// evaluated point is exact if the support does not change.  Newton steps
// are safeguarded by the bracket lo < nu* <= hi (phi(lo) < r <= phi(hi))
// and replaced by bisection (or doubling while hi is unknown) when they
// leave it.  A positive nu with |phi(nu) - r| <= tolphi satisfies the KKT
// conditions of the projection, so the search can start from the previous
// call's nu without first evaluating nu = 0.
struct ProjResult {
  double nu, tau;
  int32_t passes;
  int32_t flags;  // bit 0: pass or sweep cap hit, bit 1: bracket failure, bit 2: Dykstra used
};

template <int E, int NW>
__device__ __forceinline__ PassSums proj_pass(const double (&v)[E], const double (&mu)[E], double nu,
                                              double tau, BlockReducer<5, NW> &red) {
  double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const double w = fma(nu, mu[j], v[j]);
    const double m = (w > tau) ? 1.0 : 0.0;
    a[0] += m;
    a[1] = fma(m, v[j], a[1]);
    a[2] = fma(m, mu[j], a[2]);
    a[3] = fma(m * mu[j], mu[j], a[3]);
    a[4] = fma(m * mu[j], v[j], a[4]);
  }
  red.sum(a);
  return PassSums{a[0], a[1], a[2], a[3], a[4]};
}

__device__ __forceinline__ double tau_of(const PassSums &s, double nu) {
  return (fma(nu, s.sm, s.sv) - 1.0) / s.c;
}

template <int E, int NW>
__device__ __forceinline__ double simplex_tau(const double (&v)[E], const double (&mu)[E], double nu,
                                              double guess, PassSums &s, BlockReducer<5, NW> &red,
                                              int &passes, int &flags) {
  double tau = guess;
  for (int it = 0; it < 96; ++it) {
    s = proj_pass<E, NW>(v, mu, nu, tau, red);
    ++passes;
    if (s.c < 0.5) {  // guess at or above max w: restart from the full set
      tau = -1.0e300;
      continue;
    }
    const double tn = tau_of(s, nu);
    if (tn == tau) return tau;
    tau = tn;
  }
  flags |= 1;
  return tau;
}

// One pass that also counts membership changes against the previous pass
// (per-thread bit masks, E <= 32).
// Whether the support {j : v_j + nu mu_j > tau} differs from mask in any
// thread (every thread gets the answer): one barrier and no sums, for the
// test that a Newton point keeps the support it was computed on.
template <int E>
__device__ __forceinline__ bool support_changes(const double (&v)[E], const double (&mu)[E], double nu, double tau,
                                                uint32_t mask) {
  uint32_t nm = 0u;
#pragma unroll
  for (int j = 0; j < E; ++j) nm |= ((fma(nu, mu[j], v[j]) > tau) ? 1u : 0u) << j;
  return __syncthreads_or(nm != mask ? 1 : 0) != 0;
}

template <int E, int NW>
__device__ __forceinline__ PassSums proj_pass_masked(const double (&v)[E], const double (&mu)[E], double nu,
                                                     double tau, uint32_t &mask, double &changed,
                                                     double *buf) {
  // buf holds red_buf_doubles<NW>() doubles: BlockReducer<5> uses the first
  // 10 NW; this pass uses the next 6 NW and is followed by a barrier before
  // its next use
  BlockReducer<6, NW> red6{buf + 10 * NW, 0};
  double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  uint32_t nm = 0u;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const double w = fma(nu, mu[j], v[j]);
    const bool in = w > tau;
    nm |= (in ? 1u : 0u) << j;
    const double m = in ? 1.0 : 0.0;
    a[0] += m;
    a[1] = fma(m, v[j], a[1]);
    a[2] = fma(m, mu[j], a[2]);
    a[3] = fma(m * mu[j], mu[j], a[3]);
    a[4] = fma(m * mu[j], v[j], a[4]);
  }
  a[5] = (double)__popc(nm ^ mask);
  mask = nm;
  red6.sum(a);
  changed = a[5];
  return PassSums{a[0], a[1], a[2], a[3], a[4]};
}

// Dykstra's alternating projections onto Delta and H = {mu^T x >= r}, the
// safeguarded fallback of Sec. 3.1 (Bauschke and Borwein, 1996): with x_0 = v
// and p_0 = q_0 = 0,
//   y_k = Pi_Delta(x_k + p_k),  p_{k+1} = x_k + p_k - y_k,
//   x_{k+1} = Pi_H(y_k + q_k),  q_{k+1} = y_k + q_k - x_{k+1},
// both converging to Pi_{Delta cap H}(v).  Stops when ||x_{k+1} - y_k||_2 and
// ||y_k - y_{k-1}||_2 are <= tol (after at least two sweeps) or after
// max_iter; v receives y (on the simplex exactly; 0 past n).  Returns the sweeps.
// Multipliers of the result (the dual search's nu and tau, for warm starts
// and the stopping test's KKT report) are fitted on the support S of y from
// y_i = v_i + nu mu_i - tau (the original v is x + p + q at every sweep).
template <int E, int NW>
__device__ int dykstra_F(double (&v)[E], const double (&mu)[E], double r, int max_iter, double tol,
                         BlockReducer<5, NW> &red, int &flags, double &nu_out, double &tau_out) {
  double a0[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) a0[0] = fma(mu[j], mu[j], a0[0]);  // invalid entries carry mu = 0
  red.sum(a0);
  const double mu2 = a0[0];
  bool valid[E];
  double pw[E], q[E], y[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    valid[j] = v[j] > -1.0e299;
    pw[j] = 0.0;
    q[j] = 0.0;
    y[j] = 0.0;
  }
  double tau = -1.0e300;
  int k = 0;
  for (k = 1; k <= max_iter; ++k) {
    // w = x + p (kept in pw), y = Pi_Delta(w), p = w - y
#pragma unroll
    for (int j = 0; j < E; ++j) pw[j] = valid[j] ? v[j] + pw[j] : -1.0e300;
    PassSums s;
    int passes = 0;
    tau = simplex_tau<E, NW>(pw, mu, 0.0, tau, s, red, passes, flags);
    double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const double yn = valid[j] ? fmax(pw[j] - tau, 0.0) : 0.0;
      acc[1] = fma(yn - y[j], yn - y[j], acc[1]);
      pw[j] = valid[j] ? pw[j] - yn : 0.0;
      y[j] = yn;
      acc[0] = fma(mu[j], yn + q[j], acc[0]);
    }
    red.sum(acc);
    // x = Pi_H(y + q), q = y + q - x
    const double shift = (acc[0] < r && mu2 > 0.0) ? (r - acc[0]) / mu2 : 0.0;
    double acc2[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const double z = y[j] + q[j];
      const double xn = valid[j] ? fma(shift, mu[j], z) : -1.0e300;
      if (valid[j]) {
        q[j] = z - xn;
        acc2[0] = fma(xn - y[j], xn - y[j], acc2[0]);
      }
      v[j] = xn;
    }
    red.sum(acc2);
    if (k > 1 && sqrt(acc2[0]) <= tol && sqrt(acc[1]) <= tol) break;
  }
  if (k > max_iter) {
    k = max_iter;
    flags |= 1;
  }
  // d = y - v_orig on S; sums for the 2 x 2 fit of (nu, tau)
  double f[5] = {0, 0, 0, 0, 0};  // |S|, sum d, sum mu d, sum mu, sum mu^2
  double g[5] = {0, 0, 0, 0, 0};  // mu^T y
#pragma unroll
  for (int j = 0; j < E; ++j) {
    if (valid[j] && y[j] > 0.0) {
      const double d = y[j] - (v[j] + pw[j] + q[j]);
      f[0] += 1.0;
      f[1] += d;
      f[2] = fma(mu[j], d, f[2]);
      f[3] += mu[j];
      f[4] = fma(mu[j], mu[j], f[4]);
    }
    g[0] = fma(mu[j], y[j], g[0]);
  }
  red.sum(f);
  red.sum(g);
  double nu = 0.0;
  const double den = f[4] - f[3] * (f[3] / fmax(f[0], 1.0));
  if (g[0] <= r * (1.0 + 1e-12) && den > 0.0) nu = fmax((f[2] - f[3] * (f[1] / fmax(f[0], 1.0))) / den, 0.0);
  nu_out = nu;
  tau_out = (nu * f[3] - f[1]) / fmax(f[0], 1.0);
  // entries past n leave as 0, like the dual search's result
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = valid[j] ? y[j] : 0.0;
  return k;
}

// DYK: Dykstra's alternating projections (dyk_iters sweeps, bit 2 of the
// flags) instead of the dual search; a separate instantiation, so the dual
// search's kernels carry none of its registers.
template <int E, bool DYK = false, int NW = 4>
__device__ ProjResult project_F(double (&v)[E], const double (&mu)[E], double r, double tolphi,
                                double nu_warm, double tau_warm, BlockReducer<5, NW> &red, int dyk_iters = 0) {
  ProjResult out{0.0, 0.0, 0, 0};
  int passes = 0, flags = 0;
  PassSums s;
  if constexpr (DYK) {
    out.passes = dykstra_F<E, NW>(v, mu, r, dyk_iters, 1e-14, red, flags, out.nu, out.tau);
    out.flags = flags | 4;
    return out;
  }
  // Fast path from a warm start with the return constraint binding: joint
  // Newton on (tau, nu).  On a support S the two conditions
  //   |S| tau - nu sum_S mu = sum_S v - 1,  tau sum_S mu - nu sum_S mu^2 = sum_S mu v - r
  // are linear; if the support at the solution (tau', nu') is again S and
  // nu' > 0, every KKT condition of the projection holds, so the point is
  // exact.  Otherwise the safeguarded search below takes over.
  if (nu_warm > 0.0) {
    uint32_t mask = 0u;
    double changed = 0.0;
    s = proj_pass_masked<E, NW>(v, mu, nu_warm, tau_warm, mask, changed, red.buf);
    ++passes;
    __syncthreads();
    for (int it = 0; it < 4; ++it) {
      if (s.c < 1.5) break;
      const double det = s.c * s.smm - s.sm * s.sm;
      if (!(det > 1e-30 * s.c * s.smm)) break;
      const double b1 = s.sv - 1.0, b2 = s.smv - r;
      const double tn = (b1 * s.smm - s.sm * b2) / det;
      const double nn = (s.sm * b1 - s.c * b2) / det;
      if (!(nn > 0.0) || !isfinite(tn)) break;
      ++passes;
      if (!support_changes<E>(v, mu, nn, tn, mask)) {
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = fmax(fma(nn, mu[j], v[j]) - tn, 0.0);
        out.nu = nn;
        out.tau = tn;
        out.passes = passes;
        out.flags = flags;
        return out;
      }
      // the support moved: its sums for the next Newton step
      s = proj_pass_masked<E, NW>(v, mu, nn, tn, mask, changed, red.buf);
      __syncthreads();
    }
  }
  const double INF = 1.0e308;
  double nu = (nu_warm > 0.0) ? nu_warm : 0.0;
  double tau = simplex_tau<E, NW>(v, mu, nu, tau_warm, s, red, passes, flags);
  double phi = fma(nu, s.smm, s.smv) - tau * s.sm;
  bool done = false;
  double lo = 0.0, hi = INF, tau_hi = 0.0;
  bool lo_known = false;
  if (nu == 0.0) {
    if (phi >= r - tolphi) done = true;
    lo_known = true;
  } else {
    if (fabs(phi - r) <= tolphi) {
      done = true;
    } else if (phi < r) {
      lo = nu;
      lo_known = true;
    } else {
      hi = nu;
      tau_hi = tau;
    }
  }
  for (int it = 0; it < 200 && !done; ++it) {
    const double slope = s.smm - s.sm * (s.sm / s.c);
    const double nun = (slope > 0.0) ? nu + (r - phi) / slope : -1.0;
    double cand;
    if (slope > 0.0 && nun > lo && nun < hi) {
      cand = nun;
    } else if (!lo_known) {
      cand = 0.0;
    } else if (hi < INF) {
      cand = 0.5 * (lo + hi);
    } else {
      cand = (nu > 0.0) ? 2.0 * nu : 1.0;
      if (cand > 1.0e300) {
        flags |= 2;
        break;
      }
    }
    // affine prediction of tau(cand) from the current support
    const double guess = tau_of(s, cand);
    tau = simplex_tau<E, NW>(v, mu, cand, guess, s, red, passes, flags);
    nu = cand;
    phi = fma(nu, s.smm, s.smv) - tau * s.sm;
    if (nu == 0.0) {
      lo_known = true;
      if (phi >= r - tolphi) {
        done = true;
        break;
      }
      lo = 0.0;
    } else if (fabs(phi - r) <= tolphi) {
      done = true;
      break;
    } else if (phi < r) {
      lo = nu;
      lo_known = true;
    } else {
      hi = nu;
      tau_hi = tau;
    }
    if (lo_known && hi < INF && (hi - lo) <= 4.0e-16 * hi) {
      // the bracket has collapsed to rounding: take the feasible end
      nu = hi;
      tau = tau_hi;
      done = true;
      break;
    }
  }
  if (!done && hi < INF) {  // iteration cap: return the feasible end
    nu = hi;
    tau = tau_hi;
    flags |= 1;
  } else if (!done) {
    flags |= 2;
  }
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = fmax(fma(nu, mu[j], v[j]) - tau, 0.0);
  out.nu = nu;
  out.tau = tau;
  out.passes = passes;
  out.flags = flags;
  return out;
}

// The element-wise part of an NPGA iteration at row i, done by the launch
// that produces the gradient: g_k into its slot and, without backtracking,
// the step input v = y - alpha grad f(y) with y = x_k + beta (x_k - x_{k-1})
// and grad f(y) = g_k + beta (g_k - g_{k-1}) (grad f is affine) into the
// g_{k-1} slot, which the serial tail reads instead of forming the step.
__device__ __forceinline__ void npga_store_grad_step(const SolveArgs &a, const DevState *st, int64_t i, double gi) {
  const int cur = st->iter & 1;
  const double *xk = cur ? a.xbuf1 : a.xbuf0;
  const double *xp = cur ? a.xbuf0 : a.xbuf1;
  double *gk = cur ? a.gbuf1 : a.gbuf0;
  double *gp = cur ? a.gbuf0 : a.gbuf1;
  gk[i] = gi;
  if (a.backtrack) return;
  const double x = xk[i];
  const double y = fma(st->beta, x - xp[i], x);
  const double gy = fma(st->beta, gi - gp[i], gi);
  gp[i] = fma(-st->alpha, gy, y);
}

}  // namespace npga
