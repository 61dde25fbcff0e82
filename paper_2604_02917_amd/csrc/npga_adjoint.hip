// Adjoint of the solution map x*(mu, L, r, gamma) of eq. mv: gradients of a
// loss l(x*) by implicit differentiation of the KKT system on the face of
// x* (support S, return constraint in the face or not).
//
//   k_adj_face   : float64 gradient at x*, support, whether the return row
//                  belongs to the face (slack below act_tol and nu >= 0), the
//                  multipliers (lam, nu) and a degeneracy flag (an x_i = 0
//                  with near-zero reduced cost, |S| = 1, or mu constant on S)
//   k_adj_init   : start of a projected-CG round for H a = rhs on the face
//   tail_adj     : one CG step per sweep (npga_tail.h)
//   k_adj_finish : adjoint multipliers from the float64 residual,
//                  dl/dmu_S = nu a - a_nu x_S, dl/dr = a_nu,
//                  dl/dgamma = -2 a^T x
//   k_adj_dL     : dl/dL = -2 (a u^T + x v^T), u = L^T x*, v = L^T a,
//                  written column by column (a write-only pass over n x T)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"
#include "npga_tail.h"

namespace npga {

template <int E>
__global__ __launch_bounds__(256) void k_adj_face(SolveArgs a, double act_tol) {
  __shared__ double redbuf[64];
  __shared__ double mbuf[8];
  __shared__ int64_t ibuf[8];
  DevState *st = a.st;
  BlockReducer<5> red{redbuf, 0};
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  double x[E], g[E], mu[E], fr[E];
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    const bool ok = i < n;
    x[j] = ok ? a.xbuf1[i] : 0.0;
    g[j] = ok ? a.ga[i] + 2.0 * st->gamma * x[j] : 0.0;
    mu[j] = ok ? a.mu[i] : 0.0;
    fr[j] = (ok && x[j] > 0.0) ? 1.0 : 0.0;
    acc[0] = fma(mu[j], x[j], acc[0]);
    acc[1] += fr[j];
    acc[2] = fma(fr[j], mu[j], acc[2]);
    acc[3] = fma(fr[j] * mu[j], mu[j], acc[3]);
    acc[4] = fma(g[j], g[j], acc[4]);
  }
  red.sum(acc);
  const double mx = acc[0], c = acc[1], sm = acc[2], smm = acc[3];
  const double gscale = sqrt(acc[4] / (double)n) + 1e-300;
  bool active = (mx - st->r) <= act_tol;
  double lam, nu;
  face_multipliers<E>(g, mu, fr, active, red, lam, nu);
  if (active && nu < 0.0) {
    active = false;
    face_multipliers<E>(g, mu, fr, false, red, lam, nu);
  }
  MinLoc dm{1.0e308, n};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    if (i < n && fr[j] == 0.0) dm = minloc_pick(dm, MinLoc{g[j] - lam - nu * mu[j], i});
  }
  int mpar = 0;
  dm = block_minloc(dm, mbuf, ibuf, mpar);
  const bool singular = active && (c * smm - sm * sm) <= 1e-12 * c * smm;
  const bool degenerate = dm.v < 1e-9 * gscale || c < 1.5 || singular;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    if (i < n) a.fvec[i] = fr[j];
  }
  if (tid == 0) {
    st->cg_active = active ? 1 : 0;
    st->nu_kkt = active ? nu : 0.0;
    st->lambda_kkt = lam;
    st->support = (int32_t)c;
    st->proj_flags = degenerate ? 4 : 0;
  }
}

template <int E>
__global__ __launch_bounds__(256) void k_adj_init(SolveArgs a, const double *rhs) {
  __shared__ double redbuf[64];
  DevState *st = a.st;
  BlockReducer<5> red{redbuf, 0};
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const bool active = st->cg_active != 0;
  double q[E], mu[E], fr[E];
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    const bool ok = i < n;
    const double gl = ok ? rhs[i] : 0.0;
    q[j] = -gl;
    mu[j] = ok ? a.mu[i] : 0.0;
    fr[j] = ok ? a.fvec[i] : 0.0;
    acc[0] = fma(fr[j] * gl, gl, acc[0]);
  }
  red.sum(acc);
  const double rr0 = acc[0];
  double lam, nu;
  face_multipliers<E>(q, mu, fr, active, red, lam, nu);
  double p[E];
  double acc2[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    p[j] = (fr[j] > 0.0) ? -(q[j] - lam - nu * mu[j]) : 0.0;
    acc2[0] = fma(p[j], p[j], acc2[0]);
  }
  red.sum(acc2);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    if (i < n) {
      a.xbuf0[i] = 0.0;
      a.gvec[i] = q[j];
      a.pvec[i] = p[j];
      a.xs[i] = (float)p[j];
    }
  }
  if (tid == 0) {
    st->cg_rr = acc2[0];
    st->cg_rr0 = rr0;
    st->cg_iter = 0;
    st->cg_best_rr = acc2[0];
    st->cg_best_it = 0;
    st->cg_kkt = 0;
    if (!(acc2[0] > 1e-24 * rr0)) st->done = kConverged;  // nothing to solve
  }
}

__global__ __launch_bounds__(256) void k_adj_rhs(int64_t n, double gamma, const double *gl, const double *abase,
                                                 const double *hab, double *rhs) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) rhs[i] = gl[i] - (hab[i] + 2.0 * gamma * abase[i]);
}

__global__ __launch_bounds__(256) void k_adj_accum(int64_t n, const double *a, double *abase) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) abase[i] += a[i];
}

template <int E>
__global__ __launch_bounds__(256) void k_adj_finish(SolveArgs a, const double *gl, const double *abase,
                                                    const double *hab, double *dl_dmu) {
  __shared__ double redbuf[64];
  DevState *st = a.st;
  BlockReducer<5> red{redbuf, 0};
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const bool active = st->cg_active != 0;
  const double gamma = st->gamma, nu = st->nu_kkt;
  double w[E], mu[E], fr[E], av[E], x[E];
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    const bool ok = i < n;
    av[j] = ok ? abase[i] : 0.0;
    x[j] = ok ? a.xbuf1[i] : 0.0;
    const double g = ok ? gl[i] : 0.0;
    w[j] = ok ? g - (hab[i] + 2.0 * gamma * av[j]) : 0.0;
    mu[j] = ok ? a.mu[i] : 0.0;
    fr[j] = ok ? a.fvec[i] : 0.0;
    acc[0] = fma(fr[j] * g, g, acc[0]);
    acc[1] = fma(fr[j] * av[j], x[j], acc[1]);
  }
  red.sum(acc);
  double alam, anu;
  face_multipliers<E>(w, mu, fr, active, red, alam, anu);
  double acc2[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const double e = fr[j] * (w[j] - alam - anu * mu[j]);
    acc2[0] = fma(e, e, acc2[0]);
    const int64_t i = tid + 256 * j;
    if (i < n) dl_dmu[i] = active ? fr[j] * (nu * av[j] - anu * x[j]) : 0.0;
  }
  red.sum(acc2);
  if (tid == 0) {
    st->adj_alam = alam;
    st->adj_anu = active ? anu : 0.0;
    st->adj_dgamma = -2.0 * acc[1];
    st->adj_res = (acc[0] > 0.0) ? sqrt(acc2[0] / acc[0]) : 0.0;
  }
}

// dl/dL[:, t] = -2 (a u_t + x v_t); one workgroup per column (grid-stride).
__global__ __launch_bounds__(256) void k_adj_dL(const double *ahat, const double *x, const double *u,
                                                const double *v, int64_t n, int64_t cols, float *dL, int64_t ldg) {
  for (int64_t t = blockIdx.x; t < cols; t += gridDim.x) {
    const double ut = u[t], vt = v[t];
    float *col = dL + t * ldg;
    for (int64_t i = threadIdx.x; i < n; i += 256) col[i] = (float)(-2.0 * fma(ahat[i], ut, x[i] * vt));
  }
}

#define ADJ_SLOT_SWITCH(slots, CALL)            \
  switch (slots) {                              \
    case 1: CALL(1); break;                     \
    case 2: CALL(2); break;                     \
    case 4: CALL(4); break;                     \
    case 8: CALL(8); break;                     \
    case 12: CALL(12); break;                   \
    case 16: CALL(16); break;                   \
    case 22: CALL(22); break;                   \
    case 28: CALL(28); break;                   \
    case 32: CALL(32); break;                   \
    default: return (int)hipErrorInvalidValue;  \
  }

int launch_adj_face(const SolveArgs &a, int slots, double act_tol, hipStream_t s) {
#define CALL(E) hipLaunchKernelGGL(k_adj_face<E>, dim3(1), dim3(256), 0, s, a, act_tol)
  ADJ_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_adj_init(const SolveArgs &a, const double *rhs, int slots, hipStream_t s) {
#define CALL(E) hipLaunchKernelGGL(k_adj_init<E>, dim3(1), dim3(256), 0, s, a, rhs)
  ADJ_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_adj_rhs(int64_t n, double gamma, const double *gl, const double *abase, const double *hab, double *rhs,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_adj_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, gamma, gl, abase, hab, rhs);
  return (int)hipGetLastError();
}

int launch_adj_accum(const SolveArgs &a, double *abase, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_accum, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a.n, a.xbuf0, abase);
  return (int)hipGetLastError();
}

int launch_adj_finish(const SolveArgs &a, const double *gl, const double *abase, const double *hab,
                      double *dl_dmu, int slots, hipStream_t s) {
#define CALL(E) hipLaunchKernelGGL(k_adj_finish<E>, dim3(1), dim3(256), 0, s, a, gl, abase, hab, dl_dmu)
  ADJ_SLOT_SWITCH(slots, CALL)
#undef CALL
  return (int)hipGetLastError();
}

int launch_adj_dL(const double *ahat, const double *x, const double *u, const double *v, int64_t n, int64_t cols,
                  float *dL, int64_t ldg, hipStream_t s) {
  const int grid = (int)(cols < 4096 ? cols : 4096);
  hipLaunchKernelGGL(k_adj_dL, dim3(grid), dim3(256), 0, s, ahat, x, u, v, n, cols, dL, ldg);
  return (int)hipGetLastError();
}

}  // namespace npga
