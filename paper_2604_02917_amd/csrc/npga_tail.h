// Serial tails of the NPGA iteration, run by the one workgroup that
// finishes a gradient launch last (paper Sec. 3.1, Algorithm 1).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"

namespace npga {

template <int E>
__device__ void tail_npga(const SolveArgs &a, double usq_total, double *redbuf) {
  DevState *st = a.st;
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const int k = st->iter;
  const int cur = k & 1;
  const double *xk_p = cur ? a.xbuf1 : a.xbuf0;
  double *xn_p = cur ? a.xbuf0 : a.xbuf1;  // holds x_{k-1}; receives x_{k+1}
  const double *gk_p = cur ? a.gbuf1 : a.gbuf0;
  const double *gp_p = cur ? a.gbuf0 : a.gbuf1;
  const double alpha = st->alpha, r = st->r, tolphi = st->tolphi;
  BlockReducer<5> red{redbuf, 0};

  double mu[E], xk[E], gk[E], v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    const bool ok = i < n;
    mu[j] = ok ? a.mu[i] : 0.0;
    xk[j] = ok ? xk_p[i] : 0.0;
    gk[j] = ok ? gk_p[i] : 0.0;
  }

  if (k % st->check_every == 0) {
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = (tid + 256 * j < n) ? fma(-alpha, gk[j], xk[j]) : -1.0e300;
    const ProjResult pr = project_F<E>(v, mu, r, tolphi, st->nu_c, st->tau_c, red);
    double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const double d = v[j] - xk[j];
      acc[0] = fma(d, d, acc[0]);
      acc[1] = fma(xk[j], xk[j], acc[1]);
      acc[2] += (xk[j] > 0.0) ? 1.0 : 0.0;
      acc[3] = fma(xk[j], gk[j], acc[3]);
    }
    red.sum(acc);
    const double res = sqrt(acc[0]);
    const bool finite = isfinite(res) && isfinite(acc[3]);
    const double fval = (usq_total >= 0.0) ? usq_total + st->gamma * acc[1] : 0.5 * acc[3];
    if (tid == 0) {
      st->residual = res;
      st->nu_c = pr.nu;
      st->tau_c = pr.tau;
      st->objective = fval;
      st->support = (int32_t)acc[2];
      st->lambda_kkt = -pr.tau / alpha;
      st->nu_kkt = pr.nu / alpha;
      st->proj_flags |= pr.flags;
      if (!finite) {
        st->done = kNumeric;
      } else if (res <= st->tol) {
        st->done = kConverged;
        st->stop_iter = k;
        st->stop_residual = res;
      } else if (pr.flags & 2) {
        st->done = kBracket;
      }
    }
    if (!finite || res <= st->tol || (pr.flags & 2)) return;
  }
  if (k >= st->max_iter) {
    if (tid == 0) st->done = kMaxIter;
    return;
  }
  const double beta = st->beta;
  double xp[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    const bool ok = i < n;
    xp[j] = ok ? xn_p[i] : 0.0;
    const double gp = ok ? gp_p[i] : 0.0;
    const double y = fma(beta, xk[j] - xp[j], xk[j]);
    const double gy = fma(beta, gk[j] - gp, gk[j]);
    v[j] = ok ? fma(-alpha, gy, y) : -1.0e300;
  }
  const ProjResult pr = project_F<E>(v, mu, r, tolphi, st->nu, st->tau, red);
  double t = st->t;
  int restarted = 0;
  if (st->restart) {
    double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const double y = fma(beta, xk[j] - xp[j], xk[j]);
      acc[0] = fma(y - v[j], v[j] - xk[j], acc[0]);
    }
    red.sum(acc);
    if (acc[0] > 0.0) {
      t = 1.0;
      restarted = 1;
    }
  }
  const double tn = 0.5 * (1.0 + sqrt(fma(4.0 * t, t, 1.0)));
  const double bn = (t - 1.0) / tn;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    if (i < n) {
      xn_p[i] = v[j];
      a.xs[i] = (float)(a.xa ? v[j] - a.xa[i] : v[j]);
    }
  }
  if (tid == 0) {
    st->iter = k + 1;
    st->t = tn;
    st->beta = bn;
    st->nu = pr.nu;
    st->tau = pr.tau;
    st->proj_flags |= pr.flags;
    st->n_restarts += restarted;
    if (pr.flags & 2) st->done = kBracket;
  }
}

template <int E>
__device__ void tail_grad(const SolveArgs &a, double usq_total, double *redbuf) {
  DevState *st = a.st;
  BlockReducer<5> red{redbuf, 0};
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = threadIdx.x + 256 * j;
    const double x = (i < a.n) ? a.xbuf0[i] : 0.0;
    acc[0] = fma(x, x, acc[0]);
  }
  red.sum(acc);
  if (threadIdx.x == 0) {
    st->usq = usq_total;
    st->objective = usq_total + st->gamma * acc[0];
  }
}

template <int E>
__device__ void tail_power(const SolveArgs &a, double usq_total, double *redbuf) {
  DevState *st = a.st;
  const int tid = threadIdx.x;
  BlockReducer<5> red{redbuf, 0};
  double w[E];
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    w[j] = (i < a.n) ? a.gbuf0[i] : 0.0;
    const double u = (i < a.n) ? a.xbuf0[i] : 0.0;
    acc[0] = fma(w[j], w[j], acc[0]);
    acc[1] = fma(u, w[j], acc[1]);  // u^T Sigma u on the covariance path
  }
  red.sum(acc);
  const double nrm = sqrt(acc[0]);
  if (tid == 0) st->rho2 = (usq_total >= 0.0) ? usq_total : acc[1];
  if (nrm > 0.0 && isfinite(nrm)) {
    const double inv = 1.0 / nrm;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + 256 * j;
      if (i < a.n) {
        a.xbuf0[i] = w[j] * inv;
        a.xs[i] = (float)(w[j] * inv);
      }
    }
  } else if (!isfinite(nrm) && tid == 0) {
    st->done = kNumeric;
  }
}

}  // namespace npga
