// Serial tails of the NPGA iteration (paper Sec. 3.1, Algorithm 1), each
// run by a one-workgroup launch after the gradient launches of an
// iteration.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "npga_device.h"
#include "npga_internal.h"
#include "npga_pcg.h"

namespace npga {

// DYK: step projections by Dykstra's method.  BT: adaptive backtracking
// (Sec. 3.1): each new iterate is a trial point; the next launch, which has
// its gradient, accepts it if f(x) <= f(y) + <grad f(y), x - y> +
// ||x - y||^2/(2 alpha), evaluated in the exact form of a quadratic f,
// (x - y)^T Q (x - y) <= ||x - y||^2/(2 alpha) with Q (x - y) = (grad f(x) -
// grad f(y))/2, plus an allowance for the float32 products of the sweep;
// otherwise alpha <- rho alpha and the trial is recomputed from the stored
// y and grad f(y).  NW: wavefronts of the workgroup (thread t owns entries
// t + 64 NW j, j < E).
template <int E, bool DYK = false, bool BT = false, int NW = 4>
__device__ void tail_npga(const SolveArgs &a, double usq_total, double *redbuf) {
  constexpr int NT = 64 * NW;
  DevState *st = a.st;
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const int k = st->iter;
  const int cur = k & 1;
  double *xk_p = cur ? a.xbuf1 : a.xbuf0;
  double *xn_p = cur ? a.xbuf0 : a.xbuf1;  // holds x_{k-1}; receives x_{k+1}
  const double *gk_p = cur ? a.gbuf1 : a.gbuf0;
  const double *gp_p = cur ? a.gbuf0 : a.gbuf1;
  const double alpha = st->alpha, r = st->r, tolphi = st->tolphi, beta = st->beta;
  BlockReducer<5, NW> red{redbuf, 0};

  // Without backtracking the gradient launch has already formed the step
  // input v = y - alpha grad f(y) in the g_{k-1} slot (an element-wise
  // update of its rows), so an iteration loads only mu and v here; x_k and
  // g_k are loaded for the stopping test and x_{k-1} for the restart test.
  // With backtracking the step is formed here, after the test of the
  // pending trial, which reads that trial's y and grad f(y) from ybt and
  // gybt; every vector it reads is then loaded up front.
  double mu[E], xk[E], gk[E], v[E], dx[E];
  bool have_xg = false;
  auto load_xg = [&]() {
    if (have_xg) return;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + NT * j;
      const bool ok = i < n;
      xk[j] = ok ? xk_p[i] : 0.0;
      gk[j] = ok ? gk_p[i] : 0.0;
    }
    have_xg = true;
  };
  auto form_step = [&](int j) {
    const int64_t i = tid + NT * j;
    const bool ok = i < n;
    const double xp = ok ? xn_p[i] : 0.0;
    const double gp = ok ? gp_p[i] : 0.0;
    dx[j] = xk[j] - xp;
    const double y = fma(beta, dx[j], xk[j]);
    const double gy = fma(beta, gk[j] - gp, gk[j]);
    v[j] = ok ? fma(-alpha, gy, y) : -1.0e300;
    if constexpr (BT) {
      if (ok) {
        a.ybt[i] = y;
        a.gybt[i] = gy;
      }
    }
  };
  if constexpr (!BT) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + NT * j;
      const bool ok = i < n;
      mu[j] = ok ? a.mu[i] : 0.0;
      v[j] = ok ? gp_p[i] : -1.0e300;
    }
  } else {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + NT * j;
      mu[j] = (i < n) ? a.mu[i] : 0.0;
    }
    load_xg();
  }
  if constexpr (BT) {
    if (st->bt_pending) {
      double acc[5] = {0, 0, 0, 0, 0};  // d^T Q d, ||d||^2, float32 allowance
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int64_t i = tid + NT * j;
        if (i < n) {
          const double yb = a.ybt[i], gyb = a.gybt[i];
          const double d = xk[j] - yb;
          acc[0] = fma(d, 0.5 * (gk[j] - gyb), acc[0]);
          acc[1] = fma(d, d, acc[1]);
          acc[2] = fma(fabs(d), fabs(gk[j]) + fabs(gyb), acc[2]);
        }
      }
      red.sum(acc);
      const bool accept = !(acc[1] > 0.0) || acc[0] <= acc[1] / (2.0 * alpha) + 1e-6 * acc[2] ||
                          st->bt_consec >= 40;
      if (!accept) {
        // alpha <- rho alpha; a new trial x^k = Pi_F(y - alpha grad f(y))
        const double an = alpha * st->bt_rho;
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const int64_t i = tid + NT * j;
          v[j] = (i < n) ? fma(-an, a.gybt[i], a.ybt[i]) : -1.0e300;
        }
        const ProjResult pr = project_F<E, DYK, NW>(v, mu, r, tolphi, st->nu, st->tau, red, st->dykstra_iters);
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const int64_t i = tid + NT * j;
          if (i < n) {
            xk_p[i] = v[j];
            a.xs[i] = (float)(a.xa ? v[j] - a.xa[i] : v[j]);
          }
        }
        if (tid == 0) {
          st->alpha = an;
          st->bt_rejections += 1;
          st->bt_consec += 1;
          st->nu = pr.nu;
          st->tau = pr.tau;
          st->proj_flags |= pr.flags;
          if (pr.flags & 2) st->done = kBracket;
        }
        return;
      }
      if (tid == 0) {
        st->bt_pending = 0;
        st->bt_consec = 0;
      }
    }
    // every thread has read ybt and gybt (the reduction's barrier) before
    // form_step overwrites its own entries; entries are per thread anyway
#pragma unroll
    for (int j = 0; j < E; ++j) form_step(j);
  }

  if (k % st->check_every == 0) {
    load_xg();
    double w[E];
    double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      w[j] = (tid + NT * j < n) ? fma(-alpha, gk[j], xk[j]) : -1.0e300;
      acc[1] = fma(xk[j], xk[j], acc[1]);
      acc[2] += (xk[j] > 0.0) ? 1.0 : 0.0;
      acc[3] = fma(xk[j], gk[j], acc[3]);
    }
    // warm start from the last step's projection (one iteration old, where
    // the last test's multipliers are check_every iterations old)
    const ProjResult pr = project_F<E, DYK, NW>(w, mu, r, tolphi, st->nu, st->tau, red, st->dykstra_iters);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const double d = w[j] - xk[j];
      acc[0] = fma(d, d, acc[0]);
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
  const ProjResult pr = project_F<E, DYK, NW>(v, mu, r, tolphi, st->nu, st->tau, red, st->dykstra_iters);
  double t = st->t;
  int restarted = 0;
  if (st->restart) {
    // gradient restart test (y - x_{k+1})^T (x_{k+1} - x_k) > 0 with
    // y - x_k = beta dx
    load_xg();
    if constexpr (!BT) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int64_t i = tid + NT * j;
        dx[j] = (i < n) ? xk[j] - xn_p[i] : 0.0;
      }
    }
    double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const double y = fma(beta, dx[j], xk[j]);
      acc[0] = fma(y - v[j], v[j] - xk[j], acc[0]);
    }
    red.sum(acc);
    if (acc[0] > 0.0) {
      t = 1.0;
      restarted = 1;
    }
  }
  const double tn = 0.5 * (1.0 + sqrt(fma(4.0 * t, t, 1.0)));
  const double bn = st->const_momentum ? st->beta_const : (t - 1.0) / tn;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + NT * j;
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
    if constexpr (BT) st->bt_pending = 1;
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


// Number of eigenvalues below x of the m x m symmetric tridiagonal T
// (diagonal al, off-diagonal be): negative pivots of T - x I = L D L^T.
__device__ inline int sturm_count(const double *al, const double *be, int m, double x) {
  int cnt = 0;
  double q = al[0] - x;
  cnt += q < 0.0;
  for (int i = 1; i < m; ++i) {
    const double qq = (fabs(q) < 1e-300) ? -1e-300 : q;
    q = al[i] - x - be[i - 1] * be[i - 1] / qq;
    cnt += q < 0.0;
  }
  return cnt;
}

// Largest eigenvalue of T by multisection with the whole workgroup: each
// round evaluates 256 Sturm counts across the bracket and keeps the cell
// where the count reaches m (8 rounds shrink the Gershgorin bracket by
// 257^8).  al, be in LDS; every thread returns the same value.
__device__ inline double tridiag_max_eig_block(const double *al, const double *be, int m, double *sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    double lo = 1e308, hi = -1e308;
    for (int i = 0; i < m; ++i) {
      const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i + 1 < m ? fabs(be[i]) : 0.0);
      lo = fmin(lo, al[i] - r);
      hi = fmax(hi, al[i] + r);
    }
    sh[0] = lo;
    sh[1] = hi;
  }
  __syncthreads();
  for (int round = 0; round < 8; ++round) {
    const double lo = sh[0], hi = sh[1];
    const double w = (hi - lo) / 257.0;
    const double x = lo + w * (double)(tid + 1);
    const bool above = sturm_count(al, be, m, x) == m;  // x exceeds the largest eigenvalue
    const unsigned long long mask = __ballot(above);
    if (lane == 0) sh[2 + wave] = mask ? (double)(wave * 64 + __ffsll((long long)mask) - 1) : 256.0;
    __syncthreads();
    if (tid == 0) {
      const int t = (int)fmin(fmin(sh[2], sh[3]), fmin(sh[4], sh[5]));
      const double nlo = (t == 0) ? lo : lo + w * (double)t;
      const double nhi = (t == 256) ? hi : lo + w * (double)(t + 1);
      sh[0] = nlo;
      sh[1] = nhi;
    }
    __syncthreads();
  }
  return sh[1];
}

// Last component of the unit eigenvector of the m x m tridiagonal T for its
// largest eigenvalue theta (an upper bound from the multisection), by two
// steps of inverse iteration with the shift theta (1 + 1e-12): T - shift I is
// negative definite, so its LDL^T recurrence needs no pivoting.  beta_m times
// this component is the residual norm ||A z - theta z|| of the Ritz pair.
__device__ inline double ritz_last_component(const double *al, const double *be, int m, double theta,
                                             double *w, double *y /* m scratch entries each */) {
  if (m == 1) return 1.0;
  const double shift = theta + 1e-12 * fabs(theta);
  for (int i = 0; i < m; ++i) y[i] = 1.0;
  double last = 1.0;
  for (int it = 0; it < 2; ++it) {
    // forward elimination (w: pivots), then back substitution, in place in y
    w[0] = al[0] - shift;
    for (int i = 1; i < m; ++i) {
      const double l = be[i - 1] / w[i - 1];
      w[i] = (al[i] - shift) - l * be[i - 1];
      y[i] -= l * y[i - 1];
    }
    y[m - 1] /= w[m - 1];
    for (int i = m - 2; i >= 0; --i) y[i] = (y[i] - be[i] * y[i + 1]) / w[i];
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm = fma(y[i], y[i], nrm);
    nrm = sqrt(nrm);
    if (!(nrm > 0.0) || !isfinite(nrm)) return 1.0;  // no estimate: not converged
    for (int i = 0; i < m; ++i) y[i] /= nrm;
    last = y[m - 1];
  }
  return last;
}

// One Lanczos step on A = L_eff L_eff^T (gbuf0 = A v from the sweep, v in
// xbuf0, the previous basis vector in xbuf1).  The largest Ritz value of
// T_m is a lower bound of ||L_eff||_2^2 that converges far faster than the
// power method's Rayleigh quotient on a clustered top spectrum.  The phase
// ends when the Ritz pair's residual beta_m |s_m| falls to lz_tol theta (an
// eigenvalue of A then lies within lz_tol theta of theta, and the Ritz
// value's own error is of the order of the squared residual) or the
// recurrence breaks down; rho2 receives theta.
template <int E>
__device__ void tail_lanczos(const SolveArgs &a, double *redbuf) {
  DevState *st = a.st;
  const int tid = threadIdx.x;
  BlockReducer<5> red{redbuf, 0};
  const int j = st->lz_m;
  const double bprev = (j > 0) ? st->lz_beta[j - 1] : 0.0;
  double w[E], v[E], vp[E];
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int64_t i = tid + 256 * q;
    const bool ok = i < a.n;
    w[q] = ok ? a.gbuf0[i] : 0.0;
    v[q] = ok ? a.xbuf0[i] : 0.0;
    vp[q] = ok ? a.xbuf1[i] : 0.0;
    acc[0] = fma(v[q], w[q], acc[0]);
  }
  red.sum(acc);
  const double al = acc[0];
  double acc2[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < E; ++q) {
    w[q] = w[q] - al * v[q] - bprev * vp[q];
    acc2[0] = fma(w[q], w[q], acc2[0]);
  }
  red.sum(acc2);
  const double be = sqrt(acc2[0]);
  __shared__ double tal[kLanczosMax], tbe[kLanczosMax], msh[8], lzw[kLanczosMax], lzy[kLanczosMax];
  if (tid < j) {
    tal[tid] = st->lz_alpha[tid];
    tbe[tid] = st->lz_beta[tid];
  }
  if (tid == 0) {
    tal[j] = al;
    tbe[j] = be;
    st->lz_alpha[j] = al;
    st->lz_beta[j] = be;
  }
  __syncthreads();
  const double theta = tridiag_max_eig_block(tal, tbe, j + 1, msh);
  if (tid == 0) msh[6] = (j > 0) ? be * fabs(ritz_last_component(tal, tbe, j + 1, theta, lzw, lzy)) : INFINITY;
  __syncthreads();
  const double ritz_res = msh[6];
  const bool conv = ritz_res <= st->lz_tol * theta || !(be > 1e-13 * theta) || j + 1 >= kLanczosMax;
  if (!conv) {
    const double inv = 1.0 / be;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int64_t i = tid + 256 * q;
      if (i < a.n) {
        a.xbuf1[i] = v[q];
        a.xbuf0[i] = w[q] * inv;
        a.xs[i] = (float)(w[q] * inv);
      }
    }
  }
  if (tid == 0) {
    st->lz_m = j + 1;
    st->lz_theta = theta;
    st->rho2 = theta;
    if (!isfinite(theta)) st->done = kNumeric;
    else if (conv) st->done = kConverged;
  }
}

// ---------------------------------------------------------------------------
// Float64 KKT refinement by conjugate gradients on the identified face.
//
// After the NPGA stopping test the support S of x and the state of the
// return constraint identify a face of F:
//     {x : x_i = 0 (i fixed), 1^T x = 1, mu^T x = r (if held)}.
// On that affine set f is a quadratic, minimised by conjugate gradients on
// the projected gradient r = -(g - lam 1 - nu mu) restricted to the free
// entries, where (lam, nu) are the least-squares multipliers of the free
// entries of g (the projector onto the face's direction space).  Active-set
// rules keep x in F and reach the KKT point of eq. mv:
//   * a step that would make a free x_i negative stops at x_i = 0 and fixes i;
//   * a step that would drop mu^T x below r stops there and holds the
//     return constraint;
//   * once the face problem is nearly solved, a fixed index with negative
//     reduced cost g_i - lam - nu mu_i is freed, and a held return
//     constraint with nu < 0 is released.
// Every change of the face restarts CG from the projected gradient.  The
// gradient is carried by linearity, g <- g + a H p, from a float64 anchor
// gradient; H p comes from the float32 sweep on the search direction.  The
// stopping test is the NPGA residual ||Pi_F(x - alpha g) - x|| of Sec. 3.1.
// ---------------------------------------------------------------------------
template <int E, int NW = 4>
__device__ __forceinline__ void face_multipliers(const double (&g)[E], const double (&mu)[E],
                                                 const double (&fr)[E], bool active, BlockReducer<5, NW> &red,
                                                 double &lam, double &nu) {
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    acc[0] += fr[j];
    acc[1] = fma(fr[j], mu[j], acc[1]);
    acc[2] = fma(fr[j] * mu[j], mu[j], acc[2]);
    acc[3] = fma(fr[j], g[j], acc[3]);
    acc[4] = fma(fr[j] * mu[j], g[j], acc[4]);
  }
  red.sum(acc);
  const double c = acc[0], sm = acc[1], smm = acc[2], sg = acc[3], smg = acc[4];
  lam = (c > 0.0) ? sg / c : 0.0;
  nu = 0.0;
  if (active && c > 1.5) {
    const double det = c * smm - sm * sm;
    if (det > 1e-30 * c * smm) {
      lam = (smm * sg - sm * smg) / det;
      nu = (c * smg - sm * sg) / det;
    }
  }
}

template <int E, int NW = 4>
__device__ void tail_cg(const SolveArgs &a, double *redbuf, double *mbuf, int64_t *ibuf) {
  constexpr int NT = 64 * NW;
  DevState *st = a.st;
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const int cur = st->iter & 1;
  double *x_p = cur ? a.xbuf1 : a.xbuf0;
  BlockReducer<5, NW> red{redbuf, 0};
  int mpar = 0;
  const double INF = 1.0e308;

  double x[E], g[E], p[E], hp[E], mu[E], fr[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + NT * j;
    const bool ok = i < n;
    x[j] = ok ? x_p[i] : 0.0;
    g[j] = ok ? a.gvec[i] : 0.0;
    p[j] = ok ? a.pvec[i] : 0.0;
    hp[j] = ok ? a.gbuf0[i] : 0.0;
    mu[j] = ok ? a.mu[i] : 0.0;
    fr[j] = ok ? a.fvec[i] : 0.0;
  }
  bool active = st->cg_active != 0;
  const double r = st->r;
  const double rr = st->cg_rr;
  double *xo_p = cur ? a.xbuf0 : a.xbuf1;  // the other iterate buffer (free in this phase)

  // (0) a pending projected-gradient step: x <- w, g <- g + H (w - x), and CG
  // restarts on the face of w
  if (st->cg_pg) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + NT * j;
      const bool ok = i < n;
      x[j] = ok ? xo_p[i] : 0.0;
      g[j] += hp[j];
      fr[j] = (ok && x[j] > 0.0) ? 1.0 : 0.0;
    }
    const bool act = st->cg_pg_nu > 0.0;
    double lam0, nu0;
    face_multipliers<E, NW>(g, mu, fr, act, red, lam0, nu0);
    double acc0[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      p[j] = (fr[j] > 0.0) ? -(g[j] - lam0 - nu0 * mu[j]) : 0.0;
      acc0[0] = fma(p[j], p[j], acc0[0]);
    }
    red.sum(acc0);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + NT * j;
      if (i < n) {
        x_p[i] = x[j];
        a.gvec[i] = g[j];
        a.pvec[i] = p[j];
        a.fvec[i] = fr[j];
        a.xs[i] = (float)p[j];
      }
    }
    if (tid == 0) {
      st->cg_pg = 0;
      st->cg_active = act ? 1 : 0;
      st->cg_rr = acc0[0];
      st->cg_rr0 = acc0[0];
      st->cg_cycles += 1;
      st->cg_iter += 1;
      st->cg_best_rr = acc0[0];  // a new face: restart the stagnation window
      st->cg_best_it = st->cg_iter;
      if (st->cg_iter >= st->max_iter) st->done = kMaxIter;
    }
    return;
  }

  // (1) step length along p, limited by x_i >= 0 and mu^T x >= r
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    acc[0] = fma(fr[j] * p[j], hp[j], acc[0]);
    acc[1] = fma(mu[j], p[j], acc[1]);
    acc[2] = fma(mu[j], x[j], acc[2]);
  }
  red.sum(acc);
  const double php = acc[0], mp = acc[1], mx = acc[2];
  double step = (php > 0.0 && rr > 0.0) ? rr / php : 0.0;
  MinLoc m{INF, n};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    if (fr[j] > 0.0 && p[j] < 0.0) m = minloc_pick(m, MinLoc{x[j] / (-p[j]), (int64_t)(tid + NT * j)});
  }
  m = block_minloc<NW>(m, mbuf, ibuf, mpar);
  int block = 0;
  if (m.v < step) {
    step = m.v;
    block = 1;
  }
  if (!active && mp < 0.0) {
    const double sr = fmax(mx - r, 0.0) / (-mp);
    if (sr < step) {
      step = sr;
      block = 2;
    }
  }
#pragma unroll
  for (int j = 0; j < E; ++j) {
    x[j] = fma(step, p[j], x[j]);
    g[j] = fma(step, hp[j], g[j]);
    if (block == 1 && (int64_t)(tid + NT * j) == m.i) {
      x[j] = 0.0;
      fr[j] = 0.0;
    }
    if (fr[j] == 0.0) x[j] = 0.0;
  }
  bool restart = block != 0;
  if (block == 2) active = true;

  // (2) multipliers, projected gradient, reduced costs of the fixed entries
  double lam, nu;
  face_multipliers<E, NW>(g, mu, fr, active, red, lam, nu);
  double rv[E];
  MinLoc dm{INF, n};
  double acc2[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + NT * j;
    const double d = g[j] - lam - nu * mu[j];
    rv[j] = (fr[j] > 0.0) ? -d : 0.0;
    acc2[0] = fma(rv[j], rv[j], acc2[0]);
    acc2[1] = fma(g[j], g[j], acc2[1]);
    if (i < n && fr[j] == 0.0) dm = minloc_pick(dm, MinLoc{d, i});
  }
#pragma unroll
  for (int j = 0; j < E; ++j) acc2[2] = fma(fr[j] * g[j], g[j], acc2[2]);
  red.sum(acc2);
  dm = block_minloc<NW>(dm, mbuf, ibuf, mpar);
  double rr_new = acc2[0];
  const double gscale = sqrt(acc2[1] / (double)n) + 1e-300;
  const double gs2 = acc2[2];  // ||g_S||^2 on the free entries

  // (3) face changes once the face problem is nearly solved (or the
  // violation dwarfs the face residual): a projected-gradient step
  // w = Pi_F(x - alpha g), which can free and fix many indices and the
  // return constraint at once (the gradient-projection phase of GPCG, More
  // and Toraldo 1991); the next sweep supplies H (w - x)
  const bool nearly = rr_new <= 1e-12 * st->cg_rr0;
  const bool want_pg = (dm.v < -1e-13 * gscale && (nearly || sqrt(rr_new) <= 1e-2 * (-dm.v))) ||
                       (active && nu < 0.0 && (nearly || sqrt(rr_new) <= 1e-2 * (-nu) * st->mu_absmax));
  if (want_pg) {
    const double alpha = st->alpha;
    double w[E];
#pragma unroll
    for (int j = 0; j < E; ++j) w[j] = (tid + NT * j < n) ? fma(-alpha, g[j], x[j]) : -1.0e300;
    const ProjResult pr = project_F<E, false, NW>(w, mu, r, st->tolphi, st->nu_c, st->tau_c, red);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + NT * j;
      if (i < n) {
        xo_p[i] = w[j];
        x_p[i] = x[j];
        a.gvec[i] = g[j];
        a.pvec[i] = w[j] - x[j];
        a.fvec[i] = fr[j];
        a.xs[i] = (float)(w[j] - x[j]);
      }
    }
    if (tid == 0) {
      st->cg_pg = 1;
      st->cg_pg_nu = pr.nu;
      st->cg_iter = st->cg_iter + 1;
      st->cg_released += 1;
      st->proj_flags |= pr.flags;
      if (block == 1) st->cg_blocked += 1;
      if (pr.flags & 2) st->done = kBracket;
      else if (st->cg_iter >= st->max_iter) st->done = kMaxIter;
    }
    return;
  }
  if (restart) {
    face_multipliers<E, NW>(g, mu, fr, active, red, lam, nu);
    double acc3[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const double d = g[j] - lam - nu * mu[j];
      rv[j] = (fr[j] > 0.0) ? -d : 0.0;
      acc3[0] = fma(rv[j], rv[j], acc3[0]);
    }
    red.sum(acc3);
    rr_new = acc3[0];
  }

  // (4) stopping tests: the KKT conditions hold to rounding on the face
  // (projected gradient below 1e-12 of the gradient, no fixed index with a
  // negative reduced cost, return multiplier of the right sign), or the
  // residual of Sec. 3.1 on the maintained gradient is below tol
  const int it = st->cg_iter + 1;
  const bool kkt = !restart && rr_new <= 1e-20 * gs2 && dm.v >= -1e-12 * gscale &&
                   !(active && nu < 0.0);
  // stagnation: no halving of ||r||^2 for cg_window iterations ends the
  // round (the host re-anchors the gradient in float64 and starts the next
  // round)
  double best = st->cg_best_rr;
  int best_it = st->cg_best_it;
  if (restart || rr_new < 0.5 * best) {
    best = rr_new;
    best_it = st->cg_iter + 1;
  }
  const bool stalled = (st->cg_iter + 1) - best_it > st->cg_window;
  bool stop = false;
  if (it % st->check_every == 0 || kkt || stalled) {
    double w[E];
    const double alpha = st->alpha;
#pragma unroll
    for (int j = 0; j < E; ++j) w[j] = (tid + NT * j < n) ? fma(-alpha, g[j], x[j]) : -1.0e300;
    const ProjResult pr = project_F<E, false, NW>(w, mu, r, st->tolphi, st->nu_c, st->tau_c, red);
    // objective from the float64 anchor as in tail_pdas (x^T g / 2 without one)
    double acc4[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + NT * j;
      const double d = w[j] - x[j];
      acc4[0] = fma(d, d, acc4[0]);
      acc4[2] += (x[j] > 0.0) ? 1.0 : 0.0;
      if (i < n) {
        const double xa = a.xa ? a.xa[i] : 0.0;
        const double gaf = a.xa ? a.ga[i] + 2.0 * st->gamma * xa : 0.0;
        acc4[1] = fma(xa, gaf, acc4[1]);
        acc4[3] = fma(x[j] - xa, g[j] + gaf, acc4[3]);
      }
    }
    red.sum(acc4);
    const double res = sqrt(acc4[0]);
    if (tid == 0) {
      st->residual = res;
      st->nu_c = pr.nu;
      st->tau_c = pr.tau;
      st->objective = 0.5 * acc4[1] + 0.5 * acc4[3];
      st->support = (int32_t)acc4[2];
      st->lambda_kkt = -pr.tau / alpha;
      st->nu_kkt = pr.nu / alpha;
      st->proj_flags |= pr.flags;
      if (!isfinite(res)) {
        st->done = kNumeric;
      } else if (kkt || stalled) {
        st->done = kConverged;
        st->cg_kkt = kkt ? 1 : 0;
      }
    }
    stop = !isfinite(res) || kkt || stalled;
  }
  if (!stop && it >= st->max_iter && tid == 0) st->done = kMaxIter;

  // (5) next direction
  const double beta = (!restart && rr > 0.0) ? rr_new / rr : 0.0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + NT * j;
    p[j] = fma(beta, p[j], rv[j]);
    if (i < n) {
      x_p[i] = x[j];
      a.gvec[i] = g[j];
      a.pvec[i] = p[j];
      a.fvec[i] = fr[j];
      a.xs[i] = (float)p[j];
    }
  }
  if (tid == 0) {
    st->cg_iter = it;
    st->cg_rr = rr_new;
    st->cg_best_rr = best;
    st->cg_best_it = best_it;
    if (restart) {
      st->cg_rr0 = rr_new;
      st->cg_cycles += 1;
    }
    if (block == 1) st->cg_blocked += 1;
    st->cg_active = active ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// Float64 KKT refinement by an inexact primal-dual active-set method.
//
// The face of eq. mv is a guess of the support S and of the state of the
// return constraint.  On a face, f restricted to {x_S : 1^T x_S = 1,
// mu_S^T x_S = r (if held)} is minimised by conjugate gradients on the
// projected gradient (multipliers by least squares, as in tail_cg), with no
// step limit: entries may turn negative.  Once the projected gradient has
// dropped by pdas_eta2 (or the face is settled and CG runs to the KKT
// tolerance), the face is updated by the sign conditions of the KKT system
// (the primal-dual active-set rule):
//   * a free x_i <= 0 leaves S (x_i := 0);
//   * a fixed index with reduced cost g_i - lam - nu mu_i < -1e-12 (the
//     gradient's root mean square) enters S;
//   * a held return row with nu < 0 is released, a free one with
//     mu^T x < r is held;
// and the equality rows are restored on the new face by adding c1 + c2 mu_i
// to its entries.  The step to the new point needs H (x' - x): it is the
// next sweep (pending step, as the projected-gradient step of tail_cg).
// Many indices change per update, where blocking steps change one.  The
// round ends when the face is unchanged, x > 0 on it and the projected
// gradient is below 1e-10 of the gradient on S (KKT to rounding), or on
// stagnation of the float32 products; after kPdasMaxOuter updates it
// projects x onto F and reports the fallback (pdas_failed).
// With the preconditioner set (a.pre_y), the search directions come from
// the preconditioner's launches after this tail (k_pcg_step, k_pcg_dir_z,
// k_pcg_dir_p; npga_pcg.h): the tail then leaves p alone, takes its step
// length from pcg_rz = g^T z and tells them in pcg_todo what follows (1:
// next direction, 2: the first direction on a new face); the tests keep
// using the plain projected gradient.
// ---------------------------------------------------------------------------
template <int E, int NW = 4>
__device__ void tail_pdas(const SolveArgs &a, double *redbuf) {
  constexpr int NT = 64 * NW;
  DevState *st = a.st;
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const int cur = st->iter & 1;
  double *x_p = cur ? a.xbuf1 : a.xbuf0;
  double *xo_p = cur ? a.xbuf0 : a.xbuf1;  // the pending point of a face update
  BlockReducer<5, NW> red{redbuf, 0};
  const double r = st->r;
  const bool pending = st->cg_pg != 0;

  double x[E], g[E], p[E], hp[E], mu[E], fr[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + NT * j;
    const bool ok = i < n;
    x[j] = ok ? (pending ? xo_p[i] : x_p[i]) : 0.0;
    g[j] = ok ? a.gvec[i] : 0.0;
    p[j] = ok ? a.pvec[i] : 0.0;
    hp[j] = ok ? a.gbuf0[i] : 0.0;
    mu[j] = ok ? a.mu[i] : 0.0;
    fr[j] = ok ? a.fvec[i] : 0.0;
  }
  bool active = st->cg_active != 0;

  if (pending) {
    // the face update is taken: x <- x', g <- g + H (x' - x); CG restarts
    // on the new face (fvec already holds it)
#pragma unroll
    for (int j = 0; j < E; ++j) g[j] += hp[j];
    double lam, nu;
    face_multipliers<E, NW>(g, mu, fr, active, red, lam, nu);
    double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      p[j] = (fr[j] > 0.0) ? -(g[j] - lam - nu * mu[j]) : 0.0;
      acc[0] = fma(p[j], p[j], acc[0]);
    }
    red.sum(acc);
    const bool pre = a.pre_y != nullptr;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + NT * j;
      if (i < n) {
        x_p[i] = x[j];
        a.gvec[i] = g[j];
        if (!pre) {
          a.pvec[i] = p[j];
          a.xs[i] = (float)p[j];
        }
      }
    }
    if (tid == 0) {
      st->pcg_todo = 2;
      st->pcg_lam0 = lam;
      st->pcg_nu0 = nu;
      st->cg_pg = 0;
      st->cg_rr = acc[0];
      st->cg_rr0 = acc[0];
      st->cg_best_rr = acc[0];
      st->cg_iter += 1;
      st->cg_best_it = st->cg_iter;
      if (st->cg_iter >= st->max_iter) st->done = kMaxIter;
    }
    return;
  }

  // (1) CG step on the face, not limited by x >= 0
  const double rr = a.pre_y ? st->pcg_rz : st->cg_rr;
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) acc[0] = fma(fr[j] * p[j], hp[j], acc[0]);
  red.sum(acc);
  const double php = acc[0];
  const double step = (php > 0.0 && rr > 0.0) ? rr / php : 0.0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    x[j] = fma(step * fr[j], p[j], x[j]);
    g[j] = fma(step, hp[j], g[j]);
  }
  // (2) multipliers and projected gradient
  double lam, nu;
  face_multipliers<E, NW>(g, mu, fr, active, red, lam, nu);
  double rv[E];
  double acc2[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    rv[j] = (fr[j] > 0.0) ? -(g[j] - lam - nu * mu[j]) : 0.0;
    acc2[0] = fma(rv[j], rv[j], acc2[0]);
    acc2[1] = fma(fr[j] * g[j], g[j], acc2[1]);
    acc2[2] = fma(g[j], g[j], acc2[2]);
  }
  red.sum(acc2);
  const double rr_new = acc2[0], gs2 = acc2[1];
  const double gscale = sqrt(acc2[2] / (double)n) + 1e-300;
  const int it = st->cg_iter + 1;
  double best = st->cg_best_rr;
  int best_it = st->cg_best_it;
  if (rr_new < 0.5 * best) {
    best = rr_new;
    best_it = it;
  }
  const bool stalled = it - best_it > st->cg_window;
  const bool tight = rr_new <= 1e-20 * gs2;
  const bool inner_done = tight || stalled || (!st->pdas_final && rr_new <= st->pdas_eta2 * st->cg_rr0);

  int face_change = 0;
  bool act_new = active;
  if (inner_done) {
    // (3) sign conditions of the KKT system on the current point
    double cnt[5] = {0, 0, 0, 0, 0};  // leaving, entering, mu^T x
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + NT * j;
      const double d = g[j] - lam - nu * mu[j];
      cnt[0] += (fr[j] > 0.0 && x[j] <= 0.0) ? 1.0 : 0.0;
      cnt[1] += (i < n && fr[j] == 0.0 && d < -1e-12 * gscale) ? 1.0 : 0.0;
      cnt[2] = fma(mu[j], x[j], cnt[2]);
    }
    red.sum(cnt);
    if (active && nu < 0.0) act_new = false;
    if (!active && cnt[2] < r - st->tolphi) act_new = true;
    face_change = (cnt[0] > 0.0 || cnt[1] > 0.0 || act_new != active) ? 1 : 0;
    if (face_change && st->pdas_outer < kPdasMaxOuter) {
      // (4) the new face and the point x' on it: leaving entries set to 0,
      // the equality rows restored by c1 + c2 mu_i on the new free set
      double fn[E], xn[E];
      double s[5] = {0, 0, 0, 0, 0};  // |S'|, sum mu, sum mu^2, sum x', sum mu x'
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int64_t i = tid + NT * j;
        const double d = g[j] - lam - nu * mu[j];
        const bool leave = fr[j] > 0.0 && x[j] <= 0.0;
        const bool enter = i < n && fr[j] == 0.0 && d < -1e-12 * gscale;
        fn[j] = ((fr[j] > 0.0 && !leave) || enter) ? 1.0 : 0.0;
        xn[j] = (fn[j] > 0.0) ? x[j] : 0.0;
        s[0] += fn[j];
        s[1] = fma(fn[j], mu[j], s[1]);
        s[2] = fma(fn[j] * mu[j], mu[j], s[2]);
        s[3] += xn[j];
        s[4] = fma(mu[j], xn[j], s[4]);
      }
      red.sum(s);
      const double b1 = 1.0 - s[3], b2 = r - s[4];
      double c1 = (s[0] > 0.0) ? b1 / s[0] : 0.0, c2 = 0.0;
      if (act_new && s[0] > 1.5) {
        const double det = s[0] * s[2] - s[1] * s[1];
        if (det > 1e-30 * s[0] * s[2]) {
          c1 = (s[2] * b1 - s[1] * b2) / det;
          c2 = (s[0] * b2 - s[1] * b1) / det;
        }
      }
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int64_t i = tid + NT * j;
        if (fn[j] > 0.0) xn[j] += c1 + c2 * mu[j];
        if (i < n) {
          xo_p[i] = xn[j];
          x_p[i] = x[j];
          a.gvec[i] = g[j];
          a.pvec[i] = xn[j] - x[j];
          a.fvec[i] = fn[j];
          a.xs[i] = (float)(xn[j] - x[j]);
        }
      }
      if (tid == 0) {
        st->pcg_todo = 0;
        st->cg_pg = 1;
        st->cg_active = act_new ? 1 : 0;
        st->pdas_outer += 1;
        st->pdas_final = 0;
        st->pdas_moved += (int32_t)(cnt[0] + cnt[1]);
        st->cg_iter = it;
        st->cg_rr = rr_new;
        if (it >= st->max_iter) st->done = kMaxIter;
      }
      return;
    }
  }

  // (5) end of the round: the KKT conditions hold on a settled face, the
  // float32 products stagnate, or too many face updates (fallback: project
  // x onto F and report it)
  const bool kkt = inner_done && !face_change && tight;
  const bool give_up = inner_done && face_change;  // kPdasMaxOuter reached
  const bool stop = kkt || (inner_done && stalled) || give_up;
  if (stop) {
    const double alpha = st->alpha;
    double w[E];
    ProjResult pr{0.0, 0.0, 0, 0};
    if (give_up) {
#pragma unroll
      for (int j = 0; j < E; ++j) x[j] = (tid + NT * j < n) ? x[j] : -1.0e300;
      pr = project_F<E, false, NW>(x, mu, r, st->tolphi, st->nu_c, st->tau_c, red);
    } else {
      // entries below float64 rounding of the largest are zeros (a face
      // that keeps an index the equality rows force to zero, e.g. at a
      // vertex, leaves ~1e-16 there)
      // largest entry: wave maxima, then the wave results through the last
      // NW doubles of redbuf (unused by the sum reductions outside a pass)
      double m2 = 0.0;
#pragma unroll
      for (int j = 0; j < E; ++j) m2 = fmax(m2, x[j]);
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) m2 = fmax(m2, __shfl_xor(m2, off, 64));
      double *mb = redbuf + red_buf_doubles<NW>() - NW;
      if ((tid & 63) == 0) mb[tid >> 6] = m2;
      __syncthreads();
      double xmax = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) xmax = fmax(xmax, mb[w2]);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < E; ++j) x[j] = (x[j] <= 1e-13 * xmax) ? 0.0 : x[j];
    }
#pragma unroll
    for (int j = 0; j < E; ++j) w[j] = (tid + NT * j < n) ? fma(-alpha, g[j], x[j]) : -1.0e300;
    pr = project_F<E, false, NW>(w, mu, r, st->tolphi, st->nu_c, st->tau_c, red);
    // f(x) = f(x_a) + (x - x_a)^T (g(x) + g(x_a))/2 for the quadratic f: the
    // float32 drift of the carried gradient g then enters through the small
    // move from the float64 anchor only (x^T g / 2 would take all of it).
    // ga = 2 L L^T x_a excludes the ridge.  Without an anchor (xa null)
    // this is x^T g / 2.
    double acc4[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + NT * j;
      const double d = w[j] - x[j];
      acc4[0] = fma(d, d, acc4[0]);
      acc4[2] += (x[j] > 0.0) ? 1.0 : 0.0;
      if (i < n) {
        const double xa = a.xa ? a.xa[i] : 0.0;
        const double gaf = a.xa ? a.ga[i] + 2.0 * st->gamma * xa : 0.0;
        acc4[1] = fma(xa, gaf, acc4[1]);
        acc4[3] = fma(x[j] - xa, g[j] + gaf, acc4[3]);
      }
    }
    red.sum(acc4);
    const double res = sqrt(acc4[0]);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int64_t i = tid + NT * j;
      if (i < n) {
        x_p[i] = x[j];
        a.gvec[i] = g[j];
      }
    }
    if (tid == 0) {
      st->residual = res;
      st->nu_c = pr.nu;
      st->tau_c = pr.tau;
      st->objective = 0.5 * acc4[1] + 0.5 * acc4[3];
      st->support = (int32_t)acc4[2];
      st->lambda_kkt = -pr.tau / alpha;
      st->nu_kkt = pr.nu / alpha;
      st->proj_flags |= pr.flags;
      st->cg_iter = it;
      st->cg_rr = rr_new;
      st->cg_active = active ? 1 : 0;
      st->cg_kkt = kkt ? 1 : 0;
      st->pdas_failed = give_up ? 1 : 0;
      st->done = isfinite(res) ? kConverged : kNumeric;
    }
    return;
  }
  if (inner_done && tid == 0) st->pdas_final = 1;  // settled face: solve it to the KKT tolerance

  // (6) next direction (by k_pcg_step when preconditioned)
  const bool pre = a.pre_y != nullptr;
  const double beta = (rr > 0.0) ? rr_new / rr : 0.0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + NT * j;
    p[j] = fma(beta, p[j], rv[j]);
    if (i < n) {
      x_p[i] = x[j];
      a.gvec[i] = g[j];
      if (!pre) {
        a.pvec[i] = p[j];
        a.xs[i] = (float)p[j];
      }
    }
  }
  if (tid == 0) {
    st->pcg_todo = 1;
    st->pcg_lam0 = lam;
    st->pcg_nu0 = nu;
    st->cg_iter = it;
    st->cg_rr = rr_new;
    st->cg_best_rr = best;
    st->cg_best_it = best_it;
    if (!isfinite(rr_new)) st->done = kNumeric;
    else if (it >= st->max_iter) st->done = kMaxIter;
  }
}

// x0 = Pi_F(xbuf0) (Algorithm 1 requires x^0 in F); initialises the iteration.
template <int E, bool DYK = false>
__device__ void project_init_body(const SolveArgs &a, double *redbuf) {
  DevState *st = a.st;
  BlockReducer<5> red{redbuf, 0};
  const int tid = threadIdx.x;
  double mu[E], v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    mu[j] = (i < a.n) ? a.mu[i] : 0.0;
    v[j] = (i < a.n) ? a.xbuf0[i] : -1.0e300;
  }
  const ProjResult pr = project_F<E, DYK>(v, mu, st->r, st->tolphi, 0.0, -1.0e300, red, st->dykstra_iters);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    if (i < a.n) {
      a.xbuf0[i] = v[j];
      a.xbuf1[i] = v[j];
      a.gbuf0[i] = 0.0;
      a.gbuf1[i] = 0.0;
      a.xs[i] = (float)v[j];
    }
  }
  if (tid == 0) {
    st->iter = 0;
    st->t = 1.0;
    st->beta = 0.0;
    st->nu = pr.nu;
    st->tau = pr.tau;
    st->nu_c = pr.nu;
    st->tau_c = pr.tau;
    st->proj_flags |= pr.flags;
    st->ticket = 0u;
    if (pr.flags & 2) st->done = kBracket;
  }
}

// Start of the face-CG refinement: x = x_k (= the anchor), g = g_a + 2 gamma x,
// free set = support of x, return constraint held if the last stopping-test
// projection had nu > 0; p = projected gradient.
template <int E>
__device__ void cg_init_body(const SolveArgs &a, double *redbuf) {
  DevState *st = a.st;
  BlockReducer<5> red{redbuf, 0};
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const double *x_p = (st->iter & 1) ? a.xbuf1 : a.xbuf0;
  double x[E], g[E], mu[E], fr[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    const bool ok = i < n;
    x[j] = ok ? x_p[i] : 0.0;
    g[j] = ok ? a.ga[i] + 2.0 * st->gamma * x[j] : 0.0;
    mu[j] = ok ? a.mu[i] : 0.0;
    fr[j] = (ok && x[j] > 0.0) ? 1.0 : 0.0;
  }
  const bool active = st->nu_c > 0.0;
  double lam, nu;
  face_multipliers<E>(g, mu, fr, active, red, lam, nu);
  double acc[5] = {0, 0, 0, 0, 0};
  double p[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    p[j] = (fr[j] > 0.0) ? -(g[j] - lam - nu * mu[j]) : 0.0;
    acc[0] = fma(p[j], p[j], acc[0]);
  }
  red.sum(acc);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    if (i < n) {
      a.gvec[i] = g[j];
      a.pvec[i] = p[j];
      a.fvec[i] = fr[j];
      a.xs[i] = (float)p[j];
    }
  }
  if (tid == 0) {
    st->cg_rr = acc[0];
    st->cg_rr0 = acc[0];
    st->cg_active = active ? 1 : 0;
    st->cg_iter = 0;
    st->cg_cycles = 0;
    st->cg_released = 0;
    st->cg_blocked = 0;
    st->cg_best_rr = acc[0];
    st->cg_best_it = 0;
    st->cg_kkt = 0;
    st->cg_pg = 0;
    st->ticket = 0u;
    st->pdas_outer = 0;
    st->pdas_final = 0;
    st->pdas_failed = 0;
    st->pdas_moved = 0;
    st->pdas_eta2 = 1e-6;  // inner solves to 1e-3 of their initial projected gradient
  }
}


// ---------------------------------------------------------------------------
// Adjoint of the solution map (implicit differentiation of the KKT system on
// the face of x*).  With H = 2 (L L^T + gamma I) restricted to the support S
// and the constraint rows 1^T (and mu_S^T when the return constraint is in
// the face), the adjoint a solves
//     H_SS a + a_lam 1 + a_nu mu_S = g_S,   1^T a = 0,   mu_S^T a = 0,
// i.e. a minimises 1/2 a^T H a - g^T a on that subspace.  Projected
// conjugate gradients: the projector is the least-squares multiplier fit of
// face_multipliers, the products H p come from the float32 sweep, and the
// gradient q = H a - g is carried by linearity.  State: a in xbuf0, q in
// gvec, p in pvec, free flags in fvec, H p in gbuf0.
// ---------------------------------------------------------------------------
template <int E>
__device__ void tail_adj(const SolveArgs &a, double *redbuf) {
  DevState *st = a.st;
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  BlockReducer<5> red{redbuf, 0};
  double x[E], q[E], p[E], hp[E], mu[E], fr[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    const bool ok = i < n;
    x[j] = ok ? a.xbuf0[i] : 0.0;
    q[j] = ok ? a.gvec[i] : 0.0;
    p[j] = ok ? a.pvec[i] : 0.0;
    hp[j] = ok ? a.gbuf0[i] : 0.0;
    mu[j] = ok ? a.mu[i] : 0.0;
    fr[j] = ok ? a.fvec[i] : 0.0;
  }
  const bool active = st->cg_active != 0;
  // with the preconditioner set (a.pre_y) the directions come from
  // k_pcg_step after this tail, and the step length from its g^T z
  const bool pre = a.pre_y != nullptr;
  const double rr = pre ? st->pcg_rz : st->cg_rr;
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) acc[0] = fma(fr[j] * p[j], hp[j], acc[0]);
  red.sum(acc);
  const double php = acc[0];
  const double step = (php > 0.0 && rr > 0.0) ? rr / php : 0.0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    x[j] = fma(step, p[j], x[j]);
    q[j] = fma(step, fr[j] * hp[j], q[j]);
  }
  double lam, nu;
  face_multipliers<E>(q, mu, fr, active, red, lam, nu);
  double rv[E];
  double acc2[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < E; ++j) {
    rv[j] = (fr[j] > 0.0) ? -(q[j] - lam - nu * mu[j]) : 0.0;
    acc2[0] = fma(rv[j], rv[j], acc2[0]);
  }
  red.sum(acc2);
  const double rr_new = acc2[0];
  const int it = st->cg_iter + 1;
  double best = st->cg_best_rr;
  int best_it = st->cg_best_it;
  if (rr_new < 0.5 * best) {
    best = rr_new;
    best_it = it;
  }
  // stop: projected residual below 1e-12 of the right-hand side, or no
  // halving for 60 iterations (the float32 products' floor; the host then
  // re-anchors in float64)
  const bool conv = rr_new <= 1e-24 * st->cg_rr0;
  const bool stalled = it - best_it > 60;
  const double beta = (rr > 0.0) ? rr_new / rr : 0.0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int64_t i = tid + 256 * j;
    p[j] = fma(beta, p[j], rv[j]);
    if (i < n) {
      a.xbuf0[i] = x[j];
      a.gvec[i] = q[j];
      if (!pre) {
        a.pvec[i] = p[j];
        a.xs[i] = (float)p[j];
      }
    }
  }
  if (tid == 0) {
    st->pcg_todo = 1;
    st->pcg_lam0 = lam;
    st->pcg_nu0 = nu;
    st->cg_iter = it;
    st->cg_rr = rr_new;
    st->cg_best_rr = best;
    st->cg_best_it = best_it;
    if (!isfinite(rr_new)) {
      st->done = kNumeric;
    } else if (conv || stalled) {
      st->done = kConverged;
      st->cg_kkt = conv ? 1 : 0;
    } else if (it >= st->max_iter) {
      st->done = kMaxIter;
    }
  }
}

}  // namespace npga
