// Host orchestration and the C ABI of libnpga (declared in include/npga.h).
//
// Every entry point validates its arguments before enqueuing anything,
// carves the caller's workspace, and enqueues HIP kernels on the caller's
// stream.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "npga.h"
#include "npga_internal.h"
#include "npga_sketch.h"

using npga::DevState;
using npga::SolveArgs;
using npga::SolveLayout;

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Pinned host mirrors of the device state, one set per host thread.  They
// are allocated on first use and kept for the life of the process.
constexpr int kStatusSlots = 4;
thread_local char *g_pin_dev = nullptr;  // device address of the pinned mirrors
DevState *pinned_status() {
  thread_local DevState *buf = nullptr;
  if (!buf) {
    void *p = nullptr, *d = nullptr;
    if (hipHostMalloc(&p, sizeof(DevState) * kStatusSlots, hipHostMallocDefault) != hipSuccess)
      return nullptr;
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess || !d) {
      (void)hipHostFree(p);
      return nullptr;
    }
    buf = static_cast<DevState *>(p);
    g_pin_dev = static_cast<char *>(d);
  }
  return buf;
}

// Device address of a word inside the pinned mirrors.
int32_t *pinned_dev(const DevState *pin, const int32_t *host_word) {
  return reinterpret_cast<int32_t *>(g_pin_dev + (reinterpret_cast<const char *>(host_word) -
                                                  reinterpret_cast<const char *>(pin)));
}

// A status word the device stores into pinned host memory is set to
// kStatusUnset by the host before the chunk is issued.  Once the chunk's
// event has completed the device's store is visible; should it not be
// (a platform that delays the store past the event), the host waits up to
// a millisecond for it and otherwise reports an error instead of reading
// a stale word.
constexpr int32_t kStatusUnset = -0x5eed;

bool read_status(const int32_t *word, int32_t *out) {
  const volatile int32_t *w = word;
  int32_t v = *w;
  if (v == kStatusUnset) {
    const auto t0 = std::chrono::steady_clock::now();
    while ((v = *w) == kStatusUnset &&
           std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(1)) {
    }
  }
  *out = v;
  return v != kStatusUnset;
}

#define HIPCHK(expr)                                   \
  do {                                                 \
    if ((expr) != hipSuccess) return NPGA_ERR_HIP;     \
  } while (0)
#define LAUNCHCHK(expr)                                \
  do {                                                 \
    if ((expr) != 0) return NPGA_ERR_HIP;              \
  } while (0)

bool is_fin(double v) { return std::isfinite(v); }

}  // namespace

namespace npga {

int sweep_grid_for(int64_t cols) {
  const int64_t waves_needed = cols;  // one wavefront per column at most
  const int64_t g = (waves_needed + 3) / 4;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 256));
}

SolveLayout solve_layout(int64_t n, int64_t cols, int path, bool pcg) {
  SolveLayout l{};
  l.slots = slots_for(n);
  const int64_t npad = (int64_t)256 * std::max(l.slots, 1);
  l.ldp = npad;
  l.sweep_grid = sweep_grid_for(path == NPGA_PATH_SYRK ? n : cols);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  l.off_state = take(sizeof(DevState));
  l.off_status_dev = take(sizeof(DevState));
  l.off_xs = take(sizeof(float) * npad);
  l.off_x0 = take(sizeof(double) * npad);
  l.off_x1 = take(sizeof(double) * npad);
  l.off_g0 = take(sizeof(double) * npad);
  l.off_g1 = take(sizeof(double) * npad);
  // partial vectors: float32 for the sweep, float64 for the anchor gradient
  const int gmax = sweep_grid_for(std::max(cols, n));
  l.off_part = take(sizeof(double) * (size_t)std::max(gmax, l.sweep_grid) * (size_t)l.ldp);
  l.off_usq = take(sizeof(double) * (size_t)l.sweep_grid);
  if (path == NPGA_PATH_SYRK) {
    const int64_t lds = (n + 3) / 4 * 4;
    l.off_sigma = take(sizeof(float) * (size_t)lds * (size_t)n);
    l.off_planes = take(syrk_split_bytes(n, cols));  // bfloat16 planes of L for the SYRK
  } else {
    l.off_sigma = 0;
    l.off_planes = 0;
  }
  l.off_vecs = take(sizeof(double) * npad * 4);
  l.off_bt = take(sizeof(double) * npad * 2);  // backtracking: y and grad f(y) of the pending trial
  l.off_xa = take(sizeof(double) * npad);
  l.off_ga = take(sizeof(double) * npad);
  l.off_ua = take(sizeof(double) * (size_t)cols);
  l.pcg = pcg;
  if (pcg) {
    l.off_pre_y = take(sizeof(float) * (size_t)npad * kPreK);
    l.off_pre_yt = take(sizeof(float) * (size_t)npad * kPreK);
    l.off_pre_mat = take(sizeof(double) * (size_t)kPreMatDoubles);
    l.off_pre_a1 = take(sizeof(double) * (size_t)npad);
    l.off_pre_a2 = take(sizeof(double) * (size_t)npad);
    l.off_pre_x = take(sizeof(float) * (size_t)npad * kPreK);
    l.off_pre_ut = take(sizeof(float) * (size_t)kPreK * (size_t)cols);
    l.off_pre_p = take(sizeof(float) * (size_t)kPreMaxSplits * (size_t)n * kPreK);
    l.off_pre_usq = take(sizeof(double) * (size_t)((cols + 31) / 32) * kPreK);
    l.off_pre_act = take(sizeof(int32_t) * (size_t)(kPreK + 1));
    l.off_pre_z = take(sizeof(double) * (size_t)npad);
    l.off_pre_part = take(sizeof(double) * (size_t)kPreMaxRowBlocks * (kPreK + 5));
    l.off_pre_gpart = take(sizeof(double) * (size_t)kPreGpartDoubles);
  }
  l.total = off;
  return l;
}

}  // namespace npga

namespace {

// NPGA_PATH_AUTO: the explicit covariance (Sigma = L L^T once, then one SYMV
// per iteration) when the factor has at least as many columns as rows and
// is float32, and its workspace (Sigma plus the bfloat16 planes of L the
// SYRK reads, about 1.5 times L) stays within kAutoSyrkMaxBytes; else the
// fused sweep.  Measured on MI355X over n = 64 ... 8192, T/n = 0.5 ... 16
// (solves to residual 1e-6 with the refinement): with T >= n the covariance
// path's whole solve is 1.1-2.9 times faster (n = 5440, T = 48374: 22.6
// against 38.4 ms) and its time to 1e-6 no slower; with T = n/2 the sweep
// reads half of Sigma's bytes per iteration and wins (n = 5440: 913 against
// 1044 ms).
constexpr size_t kAutoSyrkMaxBytes = (size_t)4 << 30;

int resolve_path(int requested, int64_t n, int64_t cols, int dtype = NPGA_F32) {
  if (requested == NPGA_PATH_GEMV || requested == NPGA_PATH_SYRK) return requested;
  if (dtype != NPGA_F32 || cols < n) return NPGA_PATH_GEMV;
  const SolveLayout l = npga::solve_layout(n, cols, NPGA_PATH_SYRK);
  return l.total <= kAutoSyrkMaxBytes ? NPGA_PATH_SYRK : NPGA_PATH_GEMV;
}

bool options_valid(const npga_options &o) {
  return is_fin(o.tol) && o.tol > 0 && o.check_every >= 1 && o.max_iter >= 1 && is_fin(o.proj_tol) &&
         o.proj_tol > 0 && o.power_iters >= 1 && is_fin(o.step_safety) && o.step_safety >= 1.0 &&
         (o.path == NPGA_PATH_AUTO || o.path == NPGA_PATH_GEMV || o.path == NPGA_PATH_SYRK) &&
         is_fin(o.refine_tol) && o.refine_tol > 0 && o.refine_max_iter >= 0 && o.batch_config >= -1 &&
         o.batch_config < npga::kBatchConfigs && (o.momentum == 0 || o.momentum == 1) &&
         (o.step_estimator == 0 || o.step_estimator == 1) && is_fin(o.alpha) && o.alpha >= 0.0 &&
         (o.projection == 0 || o.projection == 1) && o.dykstra_iters >= 1 && is_fin(o.backtrack_rho) &&
         o.backtrack_rho >= 0.0 && o.backtrack_rho < 1.0 && o.refine_method >= 0 && o.refine_method <= 2 &&
         (o.refine_plain_cg == 0 || o.refine_plain_cg == 1);
}

bool factor_valid(const npga_factor *f) {
  if (!f || !f->L || !f->mu) return false;
  if (f->n < 1 || f->n > NPGA_MAX_N || f->cols < 1) return false;
  if (f->ld < f->n || (f->ld % 4) != 0) return false;
  if (f->dtype != NPGA_F32 && f->dtype != NPGA_BF16) return false;
  if (!aligned(f->L, f->dtype == NPGA_F32 ? 16 : 8) || !aligned(f->mu, 8)) return false;
  if (!is_fin(f->gamma) || f->gamma < 0) return false;
  return true;
}

struct Carved {
  SolveArgs a;
  DevState *st;
  float *sigma;
  uint16_t *planes;  // SYRK path: three bfloat16 planes of L
  int64_t lds;
  bool precise = false;       // refinement steps with float64 products (H p by two float64 passes)
  double *uscratch = nullptr; // cols doubles for those passes
};

// Refinement method for refine_method = 0.  The primal-dual active-set
// updates need inner solves accurate enough for the sign of every entry; a
// factor with fewer columns than assets (the STR model, a short panel, with
// a ridge) gives a face Hessian with a large cluster at 2 gamma far below
// the rest, which the float32 products resolve poorly, and the face updates
// do not settle.  Measured on MI355X (parity-grade solve, ms): cols >= n
// favours the active-set updates (n = 5440: T = 48374 38 vs 66, T = 8160 27
// vs 101, T = 5440 35 vs 133), cols < n the blocking CG (STR with ell = 512:
// 8.8 vs 27.8; n = 1000, T = 500: 86 vs 141).
bool pdas_suits(int64_t n, int64_t cols) { return cols >= n; }

// The active-set method's face solves preconditioned by a rank-32 Nystrom
// sketch of H (npga_pcg.h) on the factor path from n = 2048 (the refinement
// then starts with one multi-vector product of 32 columns; on a 10-factor
// model the face Hessian has 10 outliers above a bulk of condition ~5, and
// a CPU simulation of the refinement from the C2 stopping point took 38
// face products instead of 84).
bool pcg_applies(const npga_options &o, int64_t n, int64_t cols, int path) {
  if (path != NPGA_PATH_GEMV || !o.refine || o.refine_max_iter <= 0 || o.refine_plain_cg) return false;
  if (n < 2048 || n > NPGA_MAX_N) return false;
  return o.refine_method == 1 || (o.refine_method == 0 && pdas_suits(n, cols));
}

int pcg_build(const npga_factor *f, const SolveLayout &l, char *base, hipStream_t s);

Carved carve(const npga_factor *f, const SolveLayout &l, void *ws, int path) {
  char *base = static_cast<char *>(ws);
  Carved c{};
  SolveArgs &a = c.a;
  a.L = f->L;
  a.dtype = f->dtype;
  a.ld = f->ld;
  a.n = f->n;
  a.cols = f->cols;
  a.mu = f->mu;
  a.xs = reinterpret_cast<float *>(base + l.off_xs);
  a.xbuf0 = reinterpret_cast<double *>(base + l.off_x0);
  a.xbuf1 = reinterpret_cast<double *>(base + l.off_x1);
  a.gbuf0 = reinterpret_cast<double *>(base + l.off_g0);
  a.gbuf1 = reinterpret_cast<double *>(base + l.off_g1);
  a.partials = reinterpret_cast<float *>(base + l.off_part);
  a.usq_part = reinterpret_cast<double *>(base + l.off_usq);
  a.ldp = l.ldp;
  a.sweep_grid = l.sweep_grid;
  a.mode = npga::kTailNpga;
  a.st = reinterpret_cast<DevState *>(base + l.off_state);
  c.st = a.st;
  c.lds = (f->n + 3) / 4 * 4;
  c.sigma = (path == NPGA_PATH_SYRK) ? reinterpret_cast<float *>(base + l.off_sigma) : nullptr;
  c.planes = (path == NPGA_PATH_SYRK) ? reinterpret_cast<uint16_t *>(base + l.off_planes) : nullptr;
  a.ybt = reinterpret_cast<double *>(base + l.off_bt);
  a.gybt = a.ybt + l.ldp;
  return c;
}

DevState initial_state(const npga_factor *f, double r, const npga_options &o) {
  DevState s;
  std::memset(&s, 0, sizeof(s));
  s.done = npga::kRunning;
  s.iter = 0;
  s.stop_iter = -1;
  s.max_iter = o.max_iter;
  s.check_every = o.check_every;
  s.restart = o.restart;
  s.t = 1.0;
  s.gamma = f->gamma;
  s.r = r;
  s.tol = o.tol;
  s.residual = INFINITY;
  s.stop_residual = INFINITY;
  s.const_momentum = o.momentum == 1 ? 1 : 0;
  s.dykstra_iters = o.dykstra_iters;
  s.bt_rho = o.backtrack_rho;
  return s;
}

// One gradient evaluation + tail, on either path.
int step(const Carved &c, int path, int slots, hipStream_t s) {
  if (c.precise) {
    // H p = 2 L (L^T p) + 2 gamma p with float64 products, then the tail
    int e = npga::launch_precise_gradient(c.a, c.a.pvec, c.uscratch, c.a.gbuf0,
                                          reinterpret_cast<double *>(c.a.partials), slots, s);
    if (e) return e;
    e = npga::launch_add_ridge(c.a, s);
    if (e) return e;
    return npga::launch_tail(c.a, slots, 0, s);
  }
  if (path == NPGA_PATH_SYRK) return npga::launch_symv_tail(c.a, c.sigma, c.lds, slots, s);
  int e = npga::launch_sweep(c.a, slots, s);
  if (e) return e;
  return npga::launch_reduce_tail(c.a, slots, s);
}

// ||L_eff||_2^2 by Lanczos on L_eff L_eff^T (default) or by the power method
// of the paper's Remark (power_iters sweeps); then alpha.  Lanczos stops at a
// Ritz residual of lz_tol theta.  For the step size that need only be a
// fraction of the safety margin: with alpha = 1/(step_safety 2 (theta +
// gamma)), lambda_max <= (1 + lz_tol) theta keeps alpha <= 1/L_f whenever
// lz_tol < step_safety - 1; a quarter of the margin, capped at 1e-2 (about
// eight sweeps on a factor spectrum), leaves room for rounding.
double step_lanczos_tol(const npga_options &o) {
  return std::min(1e-2, std::max(0.25 * (o.step_safety - 1.0), 1e-4));
}

int estimate_step(const Carved &c, int path, int slots, const npga_options &o, hipStream_t s, double lz_tol) {
  if (o.alpha > 0.0) return npga::launch_set_alpha(c.st, o.step_safety, s, o.alpha);  // given by the caller
  if (npga::launch_random_unit(c.a.xbuf0, c.a.xs, c.a.n, o.seed, s)) return 1;
  Carved cp = c;
  int steps = o.power_iters;
  if (o.step_estimator == 0) {
    cp.a.mode = npga::kTailLanczos;
    if (npga::launch_lanczos_init(cp.a, lz_tol, s)) return 1;
    steps = std::min(o.power_iters, npga::kLanczosMax);
  } else {
    cp.a.mode = npga::kTailPower;
  }
  for (int i = 0; i < steps; ++i)
    if (step(cp, path, slots, s)) return 1;
  return npga::launch_set_alpha(c.st, o.step_safety, s);
}

// Events that only take timestamps skip the system-scope fence (a cache
// writeback and invalidate) that a default event performs when recorded.
hipError_t timing_event(hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

// Owns up to N events; whatever was created is destroyed on every return
// path, including a failure part-way through creating the set.
template <int N>
struct EventSet {
  hipEvent_t ev[N];
  int made = 0;
  // one more event into *out: timestamp-only when `timing`, else a default
  // event (its completion also orders the host after earlier copies)
  hipError_t make(hipEvent_t *out, bool timing = true) {
    if (made == N) return hipErrorInvalidValue;
    const hipError_t e = timing ? timing_event(&ev[made]) : hipEventCreate(&ev[made]);
    if (e == hipSuccess) *out = ev[made++];
    return e;
  }
  ~EventSet() {
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
  }
};

int map_done(int done) {
  switch (done) {
    case npga::kConverged: return NPGA_OK;
    case npga::kMaxIter: return NPGA_ERR_NOT_CONVERGED;
    case npga::kNumeric: return NPGA_ERR_NUMERIC;
    case npga::kBracket: return NPGA_ERR_BRACKET;
    default: return NPGA_ERR_NOT_CONVERGED;
  }
}

// Runs chunks of `check_every` iterations until the device reports done.
// Two chunks are kept in flight; the status of chunk j is read while chunk
// j+1 runs.  Returns the final done code via *done_out and the GPU time
// from `ev0` to the end of the chunk in which the phase finished.
struct SweepTimer {
  hipEvent_t a[2], b[2];
  double total_ms = 0.0;
  int samples = 0;
};

int run_phase(const Carved &c, int path, int slots, int check_every, int64_t max_chunks, hipStream_t s,
              DevState *pin, hipEvent_t *evs, hipEvent_t ev0, int *done_out, double *phase_ms,
              SweepTimer *tm) {
  int64_t issued = 0, consumed = 0;
  // the last tail of a chunk stores the chunk's done word into its pinned slot
  Carved last = c;
  auto issue = [&](int slot) -> int {
    pin[slot].done = kStatusUnset;
    last.a.host_done = pinned_dev(pin, &pin[slot].done);
    for (int i = 0; i < check_every; ++i) {
      const Carved &ci = (i == check_every - 1) ? last : c;
      if (i == 0 && tm) {
        // time the first gradient launch of every chunk on this stream
        if (hipEventRecord(tm->a[slot], s) != hipSuccess) return NPGA_ERR_HIP;
        const int e = (path == NPGA_PATH_SYRK) ? npga::launch_symv(ci.a, ci.sigma, ci.lds, slots, s)
                                               : npga::launch_sweep(ci.a, slots, s);
        if (e) return NPGA_ERR_HIP;
        if (hipEventRecord(tm->b[slot], s) != hipSuccess) return NPGA_ERR_HIP;
        const int e2 = (path == NPGA_PATH_SYRK) ? npga::launch_tail(ci.a, slots, 1, s)
                                                : npga::launch_reduce_tail(ci.a, slots, s);
        if (e2) return NPGA_ERR_HIP;
        continue;
      }
      if (step(ci, path, slots, s)) return NPGA_ERR_HIP;
    }
    if (hipEventRecord(evs[slot], s) != hipSuccess) return NPGA_ERR_HIP;
    return NPGA_OK;
  };
  int e = issue(0);
  if (e) return e;
  ++issued;
  e = issue(1);
  if (e) return e;
  ++issued;
  for (;;) {
    const int slot = consumed & 1;
    if (hipEventSynchronize(evs[slot]) != hipSuccess) return NPGA_ERR_HIP;
    ++consumed;
    int32_t done = 0;
    if (!read_status(&pin[slot].done, &done)) return NPGA_ERR_HIP;
    if (tm && done == npga::kRunning) {  // only chunks that ran every launch in full
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, tm->a[slot], tm->b[slot]) == hipSuccess) {
        tm->total_ms += ms;
        tm->samples += 1;
      }
    }
    if (done != npga::kRunning) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev0, evs[slot]);
      *phase_ms = ms;
      *done_out = done;
      // drain the chunk still in flight (its kernels exit at once)
      if (hipStreamSynchronize(s) != hipSuccess) return NPGA_ERR_HIP;
      return NPGA_OK;
    }
    if (issued >= max_chunks) {
      // the device must have reported max_iter long before this; stop
      // rather than loop if it did not
      if (hipStreamSynchronize(s) != hipSuccess) return NPGA_ERR_HIP;
      *done_out = npga::kMaxIter;
      *phase_ms = 0.0;
      return NPGA_OK;
    }
    e = issue(slot);
    if (e) return e;
    ++issued;
  }
}

}  // namespace

extern "C" {

void npga_default_options(npga_options *o) {
  if (!o) return;
  o->tol = 1e-6;
  o->check_every = 5;
  o->max_iter = 200000;
  o->proj_tol = 1e-12;
  o->power_iters = 20;
  o->step_safety = 1.05;
  o->refine = 1;
  o->path = NPGA_PATH_AUTO;
  o->seed = 1;
  o->warm_start = 0;
  o->restart = 0;
  o->refine_tol = 1e-9;
  o->refine_max_iter = 20000;
  o->batch_config = -1;
  o->momentum = 0;
  o->step_estimator = 0;
  o->alpha = 0.0;
  o->projection = 0;
  o->dykstra_iters = 5000;
  o->backtrack_rho = 0.0;
  o->refine_method = 0;
  o->refine_plain_cg = 0;
}

size_t npga_struct_size(int32_t which) {
  switch (which) {
    case 0: return sizeof(npga_options);
    case 1: return sizeof(npga_result);
    case 2: return sizeof(npga_factor);
    case 3: return sizeof(npga_str_options);
    case 4: return sizeof(npga_backward_result);
    default: return 0;
  }
}

const char *npga_status_string(int status) {
  switch (status) {
    case NPGA_OK: return "ok";
    case NPGA_ERR_INVALID: return "invalid argument";
    case NPGA_ERR_INFEASIBLE: return "infeasible: target return exceeds max(mu)";
    case NPGA_ERR_NOT_CONVERGED: return "not converged within max_iter";
    case NPGA_ERR_BRACKET: return "dual search failed to bracket the return multiplier";
    case NPGA_ERR_NUMERIC: return "non-finite value in the data or the iteration";
    case NPGA_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case NPGA_ERR_HIP: return "HIP runtime error";
    case NPGA_ERR_UNSUPPORTED: return "not supported by the library";
    default: return "unknown status";
  }
}

int npga_auto_path(int64_t n, int64_t cols, int32_t dtype) {
  if (n < 1 || n > NPGA_MAX_N || cols < 1 || (dtype != NPGA_F32 && dtype != NPGA_BF16)) return -1;
  return resolve_path(NPGA_PATH_AUTO, n, cols, dtype);
}

size_t npga_solve_workspace_size(int64_t n, int64_t cols, const npga_options *opt) {
  if (n < 1 || n > NPGA_MAX_N || cols < 1) return 0;
  npga_options o;
  npga_default_options(&o);
  if (opt) o = *opt;
  const int path = resolve_path(o.path, n, cols);
  size_t t = npga::solve_layout(n, cols, path, pcg_applies(o, n, cols, path)).total;
  // AUTO: a bfloat16 factor takes the factor path
  if (o.path == NPGA_PATH_AUTO)
    t = std::max(t, npga::solve_layout(n, cols, NPGA_PATH_GEMV, pcg_applies(o, n, cols, NPGA_PATH_GEMV)).total);
  return t;
}

static int solve_once(const npga_factor *f, double r, const npga_options *opt, float *x, npga_result *res,
                      void *ws, size_t ws_bytes, hipStream_t stream) {
  const auto t0 = Clock::now();
  npga_options o;
  npga_default_options(&o);
  if (opt) o = *opt;
  if (!factor_valid(f) || !x || !is_fin(r) || !options_valid(o)) return NPGA_ERR_INVALID;
  if (o.momentum == 1 && !(f->gamma > 0.0)) return NPGA_ERR_INVALID;
  const int path = resolve_path(o.path, f->n, f->cols, f->dtype);
  if (path == NPGA_PATH_SYRK && f->dtype != NPGA_F32) return NPGA_ERR_UNSUPPORTED;
  const SolveLayout lay = npga::solve_layout(f->n, f->cols, path, pcg_applies(o, f->n, f->cols, path));
  if (!ws || !aligned(ws, 256) || ws_bytes < lay.total) return NPGA_ERR_WORKSPACE;
  DevState *pin = pinned_status();
  if (!pin) return NPGA_ERR_HIP;
  Carved c = carve(f, lay, ws, path);
  c.a.dykstra = o.projection == 1 ? 1 : 0;
  c.a.backtrack = o.backtrack_rho > 0.0 ? 1 : 0;
  const int slots = lay.slots;

  hipEvent_t ev0, evs[2], ev_setup;
  SweepTimer tm;
  EventSet<8> events;
  HIPCHK(events.make(&ev0));
  HIPCHK(events.make(&evs[0], false));
  HIPCHK(events.make(&evs[1], false));
  HIPCHK(events.make(&ev_setup));
  for (int i = 0; i < 2; ++i) {
    HIPCHK(events.make(&tm.a[i]));
    HIPCHK(events.make(&tm.b[i]));
  }

  HIPCHK(hipEventRecord(ev0, stream));
  // state, mu statistics and the feasibility check (the only sync before the loop)
  DevState init = initial_state(f, r, o);
  pin[2] = init;
  HIPCHK(hipMemcpyAsync(c.st, &pin[2], sizeof(DevState), hipMemcpyHostToDevice, stream));
  LAUNCHCHK(npga::launch_prepare(c.a, stream));
  HIPCHK(hipMemcpyAsync(&pin[3], c.st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (pin[3].n_nonfinite > 0) return NPGA_ERR_NUMERIC;
  if (r > pin[3].mu_max) return NPGA_ERR_INFEASIBLE;
  LAUNCHCHK(npga::launch_set_tolphi(c.st, o.proj_tol, stream));

  // explicit covariance (SYRK path): Sigma = L L^T once
  if (path == NPGA_PATH_SYRK)
    LAUNCHCHK(npga::launch_syrk_split(static_cast<const float *>(f->L), f->n, f->cols, f->ld, c.planes, c.sigma,
                                      c.lds, stream));

  // step size alpha = 1/(safety L_f_hat) from ||L_eff||_2^2 (Sec. 3.1 Remark)
  LAUNCHCHK(estimate_step(c, path, slots, o, stream, step_lanczos_tol(o)));

  // x^0 = Pi_F(x_in or 1/n)
  LAUNCHCHK(npga::launch_set_vector(c.a.xbuf0, o.warm_start ? x : nullptr, nullptr, f->n,
                                    1.0 / (double)f->n, c.a.xs, stream));
  LAUNCHCHK(npga::launch_project_init(c.a, slots, o.warm_start, stream));
  HIPCHK(hipEventRecord(ev_setup, stream));

  int done = 0;
  double tol_ms = 0.0;
  // refused backtracking trials take launches without advancing the iteration
  const int64_t main_chunks = ((int64_t)o.max_iter + (c.a.backtrack ? 4096 : 0)) / o.check_every + 4;
  int e = run_phase(c, path, slots, o.check_every, main_chunks, stream, pin, evs, ev0, &done, &tol_ms, &tm);
  if (e) return e;
  const int main_done = done;
  HIPCHK(hipMemcpyAsync(&pin[2], c.st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  const DevState after_main = pin[2];
  const double host_tol_ms = ms_since(t0);
  (void)host_tol_ms;

  int refined = 0;
  int refine_iters = 0;
  int refine_fallback = 0;
  if (main_done == npga::kConverged && o.refine && o.refine_max_iter > 0) {
    // float64 gradient at the stopping point, then the inexact primal-dual
    // active-set method (CG on a face, sign rules for the face) with the
    // gradient carried by linearity from there
    char *base = static_cast<char *>(ws);
    double *xa = reinterpret_cast<double *>(base + lay.off_xa);
    double *ga = reinterpret_cast<double *>(base + lay.off_ga);
    double *ua = reinterpret_cast<double *>(base + lay.off_ua);
    double *vecs = reinterpret_cast<double *>(base + lay.off_vecs);
    const int64_t npad = (int64_t)256 * slots;
    const double *xk = (after_main.iter & 1) ? c.a.xbuf1 : c.a.xbuf0;
    HIPCHK(hipMemcpyAsync(xa, xk, sizeof(double) * f->n, hipMemcpyDeviceToDevice, stream));
    LAUNCHCHK(npga::launch_precise_gradient(c.a, xa, ua, ga, reinterpret_cast<double *>(c.a.partials),
                                            slots, stream));
    c.a.ga = ga;
    c.a.xa = xa;  // read by the refinement tails only (the objective from the anchor)
    c.a.pvec = vecs;
    c.a.fvec = vecs + npad;
    c.a.gvec = vecs + 2 * npad;
    if (lay.pcg) {
      // Y = H Omega for the preconditioner of the face solves (one
      // multi-vector product, then set up per face on the device)
      LAUNCHCHK(pcg_build(f, lay, base, stream));
      c.a.pre_y = reinterpret_cast<const float *>(base + lay.off_pre_y);
      c.a.pre_yt = reinterpret_cast<const float *>(base + lay.off_pre_yt);
      c.a.pre_mat = reinterpret_cast<double *>(base + lay.off_pre_mat);
      c.a.pre_a1 = reinterpret_cast<double *>(base + lay.off_pre_a1);
      c.a.pre_a2 = reinterpret_cast<double *>(base + lay.off_pre_a2);
      c.a.pre_z = reinterpret_cast<double *>(base + lay.off_pre_z);
      c.a.pre_part = reinterpret_cast<double *>(base + lay.off_pre_part);
      c.a.pre_gpart = reinterpret_cast<double *>(base + lay.off_pre_gpart);
    }
    // rounds re-anchored in float64 at the previous round's result (removes
    // the drift of the gradient carried by linearity).  A round that ends
    // without the KKT test (stagnation of the float32 products, e.g. on a
    // badly conditioned face) switches the following rounds to float64
    // products; a round whose face updates do not settle (x then projected
    // onto F) switches them to the face CG with blocking steps.
    bool precise = false;
    bool blocking = o.refine_method == 2 || (o.refine_method == 0 && !pdas_suits(f->n, f->cols));
    bool pcg_ready = false;  // S and sigma formed (the first preconditioned round)
    for (int round = 0; round < 4; ++round) {
      if (round > 0) {
        HIPCHK(hipMemcpyAsync(xa, xk, sizeof(double) * f->n, hipMemcpyDeviceToDevice, stream));
        LAUNCHCHK(npga::launch_precise_gradient(c.a, xa, ua, ga,
                                                reinterpret_cast<double *>(c.a.partials), slots, stream));
      }
      // float32 products stagnate at their rounding floor within a few dozen
      // iterations; with float64 products a plateau means slow progress on a
      // badly conditioned face, so those rounds wait longer
      LAUNCHCHK(npga::launch_phase_reset(c.st, o.refine_tol, o.refine_max_iter, precise ? 1000 : 60, stream));
      LAUNCHCHK(npga::launch_cg_init(c.a, slots, stream));
      if (c.a.pre_y && !blocking) LAUNCHCHK(npga::launch_pcg_init(c.a, slots, !pcg_ready, stream));
      pcg_ready = pcg_ready || (c.a.pre_y && !blocking);
      double rms = 0.0;
      const int64_t ref_chunks = (int64_t)o.refine_max_iter / o.check_every + 4;
      Carved cr = c;
      cr.precise = precise;
      cr.uscratch = ua;
      cr.a.mode = blocking ? npga::kTailCG : npga::kTailPdas;
      e = run_phase(cr, path, slots, o.check_every, ref_chunks, stream, pin, evs, ev0, &done, &rms, nullptr);
      if (e) return e;
      HIPCHK(hipMemcpyAsync(&pin[2], c.st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
      HIPCHK(hipStreamSynchronize(stream));
      refine_iters += pin[2].cg_iter;
      if (done != npga::kConverged) break;
      if (!blocking && pin[2].pdas_failed) {
        blocking = true;
        refine_fallback = 1;
        continue;
      }
      if (pin[2].cg_kkt && round > 0) break;
      if (!pin[2].cg_kkt) precise = true;
    }
    refined = (done == npga::kConverged && pin[2].cg_kkt) ? 1 : 0;
  }
  LAUNCHCHK(npga::launch_finalize(c.a, x, slots, stream));
  HIPCHK(hipMemcpyAsync(&pin[3], c.st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  const DevState &fin = pin[3];

  int status = map_done(main_done);
  if (main_done == npga::kConverged && done != npga::kConverged && done != npga::kMaxIter)
    status = map_done(done);  // numeric or bracket failure during refinement
  if (res) {
    float setup_ms = 0.f;
    (void)hipEventElapsedTime(&setup_ms, ev0, ev_setup);
    std::memset(res, 0, sizeof(*res));
    res->status = status;
    res->iters = (main_done == npga::kConverged) ? after_main.stop_iter : after_main.iter;
    res->refine_iters = refine_iters;
    res->support = fin.support;
    res->return_active = fin.nu_c > 0.0 ? 1 : 0;
    res->refined = refined;
    res->path_used = path;
    res->step_sweeps = o.alpha > 0.0 ? 0 : (o.step_estimator == 0 ? after_main.lz_m : o.power_iters);
    res->residual = after_main.stop_residual;
    res->final_residual = fin.residual;
    res->objective = fin.objective;
    res->nu = fin.nu_kkt;
    res->lambda = fin.lambda_kkt;
    res->alpha = fin.alpha;
    res->lipschitz = fin.lipschitz;
    res->time_ms = ms_since(t0);
    res->time_to_tol_ms = tol_ms;
    res->setup_ms = setup_ms;
    res->sweep_ms = tm.samples ? tm.total_ms / tm.samples : 0.0;
    res->sweep_samples = tm.samples;
    res->dykstra_used = o.projection == 1 ? 1 : 0;
    res->backtracks = after_main.bt_rejections;
    res->refine_fallback = refine_fallback;
  }
  return status;
}

// Algorithm 1 with the exact dual-search projection; should that search fail
// to bracket the return multiplier (NPGA_ERR_BRACKET), the solve is run
// again with Dykstra's alternating projections, the safeguarded fallback of
// Sec. 3.1 (res->dykstra_used = 1).
int npga_solve(const npga_factor *f, double r, const npga_options *opt, float *x, npga_result *res,
               void *ws, size_t ws_bytes, hipStream_t stream) {
  npga_options o;
  npga_default_options(&o);
  if (opt) o = *opt;
  const int e = solve_once(f, r, &o, x, res, ws, ws_bytes, stream);
  if (e != NPGA_ERR_BRACKET || o.projection == 1) return e;
  o.projection = 1;
  return solve_once(f, r, &o, x, res, ws, ws_bytes, stream);
}

int npga_project(const double *v, const double *mu, int64_t n, double r, double *x, double *nu_tau,
                 void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!v || !mu || !x || n < 1 || n > NPGA_MAX_N || !is_fin(r)) return NPGA_ERR_INVALID;
  npga_options o;
  npga_default_options(&o);
  const SolveLayout lay = npga::solve_layout(n, 1, NPGA_PATH_GEMV);
  if (!ws || !aligned(ws, 256) || ws_bytes < lay.total) return NPGA_ERR_WORKSPACE;
  DevState *pin = pinned_status();
  if (!pin) return NPGA_ERR_HIP;
  DevState *st = reinterpret_cast<DevState *>(static_cast<char *>(ws) + lay.off_state);
  npga_factor f{n, 1, (n + 3) / 4 * 4, ws, mu, 0.0, NPGA_F32, 0};
  pin[2] = initial_state(&f, r, o);
  HIPCHK(hipMemcpyAsync(st, &pin[2], sizeof(DevState), hipMemcpyHostToDevice, stream));
  SolveArgs a{};
  a.mu = mu;
  a.n = n;
  a.st = st;
  LAUNCHCHK(npga::launch_prepare(a, stream));
  HIPCHK(hipMemcpyAsync(&pin[3], st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (pin[3].n_nonfinite > 0) return NPGA_ERR_NUMERIC;
  if (r > pin[3].mu_max) return NPGA_ERR_INFEASIBLE;
  LAUNCHCHK(npga::launch_set_tolphi(st, o.proj_tol, stream));
  LAUNCHCHK(npga::launch_project_only(v, mu, n, x, st, lay.slots, stream));
  HIPCHK(hipMemcpyAsync(&pin[3], st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (nu_tau) {
    nu_tau[0] = pin[3].nu;
    nu_tau[1] = pin[3].tau;
  }
  if (pin[3].proj_flags & 2) return NPGA_ERR_BRACKET;
  return NPGA_OK;
}

int npga_project_dykstra(const double *v, const double *mu, int64_t n, double r, int32_t max_iter, double tol,
                         double *x, double *nu_tau, int32_t *iters, void *ws, size_t ws_bytes,
                         hipStream_t stream) {
  if (!v || !mu || !x || n < 1 || n > NPGA_MAX_N || !is_fin(r) || max_iter < 1 || !is_fin(tol) || tol < 0)
    return NPGA_ERR_INVALID;
  npga_options o;
  npga_default_options(&o);
  const SolveLayout lay = npga::solve_layout(n, 1, NPGA_PATH_GEMV);
  if (!ws || !aligned(ws, 256) || ws_bytes < lay.total) return NPGA_ERR_WORKSPACE;
  DevState *pin = pinned_status();
  if (!pin) return NPGA_ERR_HIP;
  DevState *st = reinterpret_cast<DevState *>(static_cast<char *>(ws) + lay.off_state);
  npga_factor f{n, 1, (n + 3) / 4 * 4, ws, mu, 0.0, NPGA_F32, 0};
  pin[2] = initial_state(&f, r, o);
  HIPCHK(hipMemcpyAsync(st, &pin[2], sizeof(DevState), hipMemcpyHostToDevice, stream));
  SolveArgs a{};
  a.mu = mu;
  a.n = n;
  a.st = st;
  LAUNCHCHK(npga::launch_prepare(a, stream));
  HIPCHK(hipMemcpyAsync(&pin[3], st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (pin[3].n_nonfinite > 0) return NPGA_ERR_NUMERIC;
  if (r > pin[3].mu_max) return NPGA_ERR_INFEASIBLE;
  LAUNCHCHK(npga::launch_project_dykstra(v, mu, n, x, st, max_iter, tol, lay.slots, stream));
  HIPCHK(hipMemcpyAsync(&pin[3], st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (nu_tau) {
    nu_tau[0] = pin[3].nu;
    nu_tau[1] = pin[3].tau;
  }
  if (iters) *iters = pin[3].iter;
  return (pin[3].proj_flags & 1) ? NPGA_ERR_NOT_CONVERGED : NPGA_OK;
}

int npga_gradient(const npga_factor *f, const float *x, double *g, double *f_out, void *ws,
                  size_t ws_bytes, hipStream_t stream) {
  if (!factor_valid(f) || !x || !g) return NPGA_ERR_INVALID;
  if (!aligned(g, 8)) return NPGA_ERR_INVALID;
  const SolveLayout lay = npga::solve_layout(f->n, f->cols, NPGA_PATH_GEMV);
  if (!ws || !aligned(ws, 256) || ws_bytes < lay.total) return NPGA_ERR_WORKSPACE;
  DevState *pin = pinned_status();
  if (!pin) return NPGA_ERR_HIP;
  npga_options o;
  npga_default_options(&o);
  Carved c = carve(f, lay, ws, NPGA_PATH_GEMV);
  c.a.mode = npga::kTailGrad;
  c.a.gbuf0 = g;
  pin[2] = initial_state(f, 0.0, o);
  HIPCHK(hipMemcpyAsync(c.st, &pin[2], sizeof(DevState), hipMemcpyHostToDevice, stream));
  LAUNCHCHK(npga::launch_set_vector(c.a.xbuf0, x, nullptr, f->n, 0.0, c.a.xs, stream));
  LAUNCHCHK(npga::launch_sweep(c.a, lay.slots, stream));
  LAUNCHCHK(npga::launch_reduce_tail(c.a, lay.slots, stream));
  // always synchronise: the upload above reads the per-thread pinned buffer,
  // which the next call from this thread overwrites
  HIPCHK(hipMemcpyAsync(&pin[3], c.st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (f_out) *f_out = pin[3].objective;
  return NPGA_OK;
}

int npga_spectral_norm_sq(const npga_factor *f, int32_t iters, uint64_t seed, int32_t method, double *out,
                          int32_t *steps_out, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!factor_valid(f) || !out || iters < 1 || (method != 0 && method != 1)) return NPGA_ERR_INVALID;
  const SolveLayout lay = npga::solve_layout(f->n, f->cols, NPGA_PATH_GEMV);
  if (!ws || !aligned(ws, 256) || ws_bytes < lay.total) return NPGA_ERR_WORKSPACE;
  DevState *pin = pinned_status();
  if (!pin) return NPGA_ERR_HIP;
  npga_options o;
  npga_default_options(&o);
  o.power_iters = iters;
  o.seed = seed;
  o.step_estimator = method;
  Carved c = carve(f, lay, ws, NPGA_PATH_GEMV);
  pin[2] = initial_state(f, 0.0, o);
  HIPCHK(hipMemcpyAsync(c.st, &pin[2], sizeof(DevState), hipMemcpyHostToDevice, stream));
  LAUNCHCHK(estimate_step(c, NPGA_PATH_GEMV, lay.slots, o, stream, 1e-4));
  HIPCHK(hipMemcpyAsync(&pin[3], c.st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  *out = pin[3].rho2;
  if (steps_out) *steps_out = method == 0 ? pin[3].lz_m : iters;
  return NPGA_OK;
}

int npga_syrk(const float *L, int64_t n, int64_t T, int64_t ld, float *Sigma, int64_t lds,
              hipStream_t stream) {
  if (!L || !Sigma || n < 1 || T < 1 || ld < n || (ld % 4) != 0 || lds < n || (lds % 4) != 0)
    return NPGA_ERR_INVALID;
  if (!aligned(L, 16) || !aligned(Sigma, 16)) return NPGA_ERR_INVALID;
  LAUNCHCHK(npga::launch_syrk(L, n, T, ld, Sigma, lds, stream));
  return NPGA_OK;
}

size_t npga_syrk_split_workspace_size(int64_t n, int64_t T) {
  if (n < 1 || T < 1) return 0;
  return npga::syrk_split_bytes(n, T);
}

int npga_syrk_split(const float *L, int64_t n, int64_t T, int64_t ld, float *Sigma, int64_t lds, void *ws,
                    size_t ws_bytes, hipStream_t stream) {
  if (!L || !Sigma || n < 1 || T < 1 || ld < n || (ld % 4) != 0 || lds < n || !aligned(L, 16))
    return NPGA_ERR_INVALID;
  if (!ws || !aligned(ws, 256) || ws_bytes < npga::syrk_split_bytes(n, T)) return NPGA_ERR_WORKSPACE;
  LAUNCHCHK(npga::launch_syrk_split(L, n, T, ld, static_cast<uint16_t *>(ws), Sigma, lds, stream));
  return NPGA_OK;
}

int npga_to_bf16(const float *L, int64_t n, int64_t T, int64_t ld, uint16_t *Lb, int64_t ldb,
                 hipStream_t stream) {
  if (!L || !Lb || n < 1 || T < 1 || ld < n || ldb < n || (ld % 4) != 0 || (ldb % 4) != 0)
    return NPGA_ERR_INVALID;
  if (!aligned(L, 16) || !aligned(Lb, 8)) return NPGA_ERR_INVALID;
  LAUNCHCHK(npga::launch_to_bf16(L, n, T, ld, Lb, ldb, stream));
  return NPGA_OK;
}

size_t npga_build_factor_workspace_size(int64_t n, int64_t T) {
  if (n < 1 || n > NPGA_MAX_N || T < 2) return 0;
  const int slots = npga::slots_for(n);
  const int grid = npga::sweep_grid_for(T);
  return align_up(sizeof(double) * ((size_t)grid * 256 * slots + grid + 8), 256);
}

int npga_build_factor(const float *R, int64_t n, int64_t T, int64_t ldr, float *L, int64_t ldl,
                      double *mu_out, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!R || !L || !mu_out || n < 1 || n > NPGA_MAX_N || T < 2) return NPGA_ERR_INVALID;
  if (ldr < n || ldl < n || (ldr % 4) != 0 || (ldl % 4) != 0) return NPGA_ERR_INVALID;
  if (!aligned(R, 16) || !aligned(L, 16) || !aligned(mu_out, 8)) return NPGA_ERR_INVALID;
  if (R == L && ldr != ldl) return NPGA_ERR_INVALID;
  const size_t need = npga_build_factor_workspace_size(n, T);
  if (!ws || !aligned(ws, 256) || ws_bytes < need) return NPGA_ERR_WORKSPACE;
  DevState *pin = pinned_status();
  if (!pin) return NPGA_ERR_HIP;
  const int grid = npga::sweep_grid_for(T);
  const int slots = npga::slots_for(n);
  double *part = static_cast<double *>(ws);
  double *nonfinite = part + (size_t)grid * 256 * slots + grid;
  LAUNCHCHK(npga::launch_build_factor(R, n, T, ldr, L, ldl, mu_out, part, grid, nonfinite, stream));
  double *h = reinterpret_cast<double *>(&pin[3]);
  HIPCHK(hipMemcpyAsync(h, nonfinite, sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (*h > 0) return NPGA_ERR_NUMERIC;
  return NPGA_OK;
}

}  // extern "C"

namespace {

struct SketchLayout {
  size_t off_S, off_Y, off_A, off_vec, off_Z, off_work, off_V32, off_frob, off_gamma, off_planes, total;
  int64_t ldS, ldy, stride;
};

constexpr int kFrobParts = 256;

SketchLayout sketch_layout(int64_t n, int64_t T, int64_t k, int64_t ell, bool need_S, bool gemm = true) {
  SketchLayout l{};
  l.ldS = (T + 3) / 4 * 4;
  l.ldy = (n + 3) / 4 * 4;
  l.stride = (ell + 63) / 64 * 64;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  l.off_S = need_S ? take(sizeof(float) * (size_t)l.ldS * (size_t)k) : 0;
  l.off_Y = take(sizeof(float) * (size_t)l.ldy * (size_t)k);
  l.off_A = take(sizeof(double) * (size_t)k * (size_t)k);
  l.off_vec = take(sizeof(double) * (size_t)k * 8);
  l.off_Z = take(sizeof(double) * (size_t)k * (size_t)ell);
  l.off_work = take(std::max(sizeof(double) * 5 * (size_t)l.stride * (size_t)k + (size_t)l.stride * (size_t)k,
                             npga::tri_scratch_bytes(k)));
  l.off_V32 = take(sizeof(float) * (size_t)k * (size_t)ell);
  l.off_frob = take(sizeof(double) * kFrobParts);
  l.off_gamma = take(sizeof(double) * 4);
  // bfloat16 planes of L and S for the sketch product (Gaussian sketch)
  l.off_planes = gemm ? take(npga::gemm_split_bytes(n, k, T)) : 0;
  l.total = off;
  return l;
}

}  // namespace

extern "C" {

size_t npga_sketch_workspace_size(int64_t n, int64_t T, int64_t k, int64_t ell) {
  if (n < 1 || T < 1 || k < 1 || ell < 1 || ell > k || k > NPGA_MAX_N) return 0;
  return sketch_layout(n, T, k, ell, true).total;
}

void npga_default_str_options(npga_str_options *so) {
  if (!so) return;
  std::memset(so, 0, sizeof(*so));
  so->sketch = NPGA_SKETCH_GAUSSIAN;
  so->ell_rule = NPGA_ELL_FIXED;
  so->k = 4096;
  so->ell = 512;
  so->ridge_coef = 1e-4;
  so->kappa_tar = 0.0;
  so->knee_tau = 1e-3;
  so->knee_rho = 0.9;
  so->seed = 3;
}

size_t npga_sketch_ex_workspace_size(int64_t n, int64_t T, const npga_str_options *so) {
  if (!so) return 0;
  const int64_t k = so->k, ell = std::min(so->ell + 1, so->k);
  if (n < 1 || T < 1 || k < 1 || ell < 1 || k > NPGA_MAX_N) return 0;
  return sketch_layout(n, T, k, ell, true, so->sketch != NPGA_SKETCH_COUNT).total;
}

int npga_sketch_str_ex(const float *L, int64_t n, int64_t T, int64_t ldl, const npga_str_options *so, float *Leff,
                       int64_t ldle, float *sigma, int64_t *ell_out, double *gamma_out, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  if (!L || !so || !Leff || !sigma || !gamma_out) return NPGA_ERR_INVALID;
  const int64_t k = so->k, ell_cap = so->ell;
  if (n < 1 || n > NPGA_MAX_N || T < 1 || k < 2 || k > NPGA_MAX_N || ell_cap < 1 || ell_cap > k)
    return NPGA_ERR_INVALID;
  if (ldl < n || (ldl % 4) != 0 || ldle < n || (ldle % 4) != 0) return NPGA_ERR_INVALID;
  if (!aligned(L, 16) || !aligned(Leff, 16)) return NPGA_ERR_INVALID;
  if (!is_fin(so->ridge_coef) || so->ridge_coef < 0 || !is_fin(so->kappa_tar)) return NPGA_ERR_INVALID;
  if (so->sketch != NPGA_SKETCH_GAUSSIAN && so->sketch != NPGA_SKETCH_COUNT) return NPGA_ERR_INVALID;
  if (so->ell_rule != NPGA_ELL_FIXED && so->ell_rule != NPGA_ELL_KNEE) return NPGA_ERR_INVALID;
  if (so->ell_rule == NPGA_ELL_KNEE &&
      (!(so->knee_tau > 0) || !(so->knee_rho > 0) || !(so->knee_rho < 1) || ell_cap >= k))
    return NPGA_ERR_INVALID;
  if (so->sketch == NPGA_SKETCH_GAUSSIAN && so->S && so->lds < T) return NPGA_ERR_INVALID;
  if (so->sketch == NPGA_SKETCH_COUNT && (!so->cs_bucket || !so->cs_sign)) return NPGA_ERR_INVALID;
  // eigenpairs computed: ell (fixed), or ell_cap + 1 eigenvalues for the knee rule
  const int64_t m_eig = so->ell_rule == NPGA_ELL_KNEE ? ell_cap + 1 : ell_cap;
  const bool draw_S = so->sketch == NPGA_SKETCH_GAUSSIAN && !so->S;
  const SketchLayout lay = sketch_layout(n, T, k, m_eig, draw_S, so->sketch != NPGA_SKETCH_COUNT);
  if (!ws || !aligned(ws, 256) || ws_bytes < lay.total) return NPGA_ERR_WORKSPACE;
  char *base = static_cast<char *>(ws);
  float *Y = reinterpret_cast<float *>(base + lay.off_Y);
  double *vec = reinterpret_cast<double *>(base + lay.off_vec);
  npga::SketchState s{};
  s.k = k;
  s.A = reinterpret_cast<double *>(base + lay.off_A);
  s.d = vec;
  s.e = vec + k;
  s.tau = vec + 2 * k;
  s.vcur = vec + 3 * k;
  s.vprev = vec + 4 * k;
  s.wprev = vec + 5 * k;
  s.p = vec + 6 * k;
  s.lam = vec + 7 * k;
  s.Z = reinterpret_cast<double *>(base + lay.off_Z);
  s.work = reinterpret_cast<double *>(base + lay.off_work);
  float *V32 = reinterpret_cast<float *>(base + lay.off_V32);
  double *frob = reinterpret_cast<double *>(base + lay.off_frob);
  double *gdev = reinterpret_cast<double *>(base + lay.off_gamma);
  int64_t *ell_dev = reinterpret_cast<int64_t *>(gdev + 2);
  int32_t *bad_dev = reinterpret_cast<int32_t *>(gdev + 3);
  DevState *pin = pinned_status();
  if (!pin) return NPGA_ERR_HIP;
  // sketch stage: Y = L Phi
  if (so->sketch == NPGA_SKETCH_COUNT) {
    LAUNCHCHK(npga::launch_zero_f32(reinterpret_cast<float *>(bad_dev), 1, stream));
    LAUNCHCHK(npga::launch_countsketch(L, ldl, n, T, so->cs_bucket, so->cs_sign, k, Y, lay.ldy, bad_dev, stream));
  } else {
    const float *S = so->S;
    int64_t lds = so->lds;
    if (draw_S) {
      float *Sw = reinterpret_cast<float *>(base + lay.off_S);
      LAUNCHCHK(npga::launch_philox_sketch(so->seed, T, k, Sw, lay.ldS, nullptr, stream));
      S = Sw;
      lds = lay.ldS;
    }
    // Y = L S on the bfloat16 matrix cores with three-plane operands
    LAUNCHCHK(npga::launch_gemm_split(L, ldl, S, lds, Y, lay.ldy, n, k, T,
                                      reinterpret_cast<uint16_t *>(base + lay.off_planes), stream));
  }
  // truncation stage: eigenpairs of G = Y^T Y
  LAUNCHCHK(npga::launch_gram_f64(Y, lay.ldy, n, k, s.A, stream));
  LAUNCHCHK(npga::launch_frob(Y, lay.ldy, n, k, frob, kFrobParts, stream));
  LAUNCHCHK(npga::launch_tridiag(s, stream));
  LAUNCHCHK(npga::launch_bisect(s, m_eig, stream));
  int64_t ell = ell_cap;
  if (so->ell_rule == NPGA_ELL_KNEE || so->sketch == NPGA_SKETCH_COUNT) {
    if (so->ell_rule == NPGA_ELL_KNEE) LAUNCHCHK(npga::launch_knee(s.lam, m_eig, so->knee_tau, so->knee_rho, ell_dev, stream));
    double *h = reinterpret_cast<double *>(&pin[3]);
    HIPCHK(hipMemcpyAsync(h, gdev + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (so->sketch == NPGA_SKETCH_COUNT && *reinterpret_cast<int32_t *>(h + 1) != 0) return NPGA_ERR_INVALID;
    if (so->ell_rule == NPGA_ELL_KNEE) {
      ell = *reinterpret_cast<int64_t *>(h);
      if (ell_out) *ell_out = ell;
      if (ell < 1) return NPGA_ERR_INVALID;  // no index passes the knee rule
    }
  }
  if (ell_out) *ell_out = ell;
  LAUNCHCHK(npga::launch_inverse_iter(s, ell, lay.stride, stream));
  LAUNCHCHK(npga::launch_backtransform(s, ell, V32, stream));
  // L_eff = Y V_ell (n x ell)
  LAUNCHCHK(npga::launch_gemm_f32(Y, lay.ldy, V32, k, Leff, ldle, n, ell, k, stream));
  // ridge stage and singular values
  LAUNCHCHK(npga::launch_finish_str(s, ell, n, so->ridge_coef, frob, kFrobParts, sigma, gdev, so->kappa_tar,
                                    stream));
  double *h = reinterpret_cast<double *>(&pin[3]);
  HIPCHK(hipMemcpyAsync(h, gdev, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  *gamma_out = h[0];
  if (!is_fin(h[0])) return NPGA_ERR_NUMERIC;
  return NPGA_OK;
}

int npga_sketch_str(const float *L, int64_t n, int64_t T, int64_t ldl, int64_t k, int64_t ell,
                    double ridge_coef, uint64_t seed, const float *S_opt, int64_t lds_opt, float *Leff,
                    int64_t ldle, float *sigma, double *gamma_out, void *ws, size_t ws_bytes,
                    hipStream_t stream) {
  npga_str_options so;
  npga_default_str_options(&so);
  so.k = k;
  so.ell = ell;
  so.ridge_coef = ridge_coef;
  so.seed = seed;
  so.S = S_opt;
  so.lds = lds_opt;
  return npga_sketch_str_ex(L, n, T, ldl, &so, Leff, ldle, sigma, nullptr, gamma_out, ws, ws_bytes, stream);
}

int npga_philox_sketch(uint64_t seed, int64_t T, int64_t k, float *S, int64_t lds, uint32_t *raw,
                       hipStream_t stream) {
  if (!S || T < 1 || k < 1 || lds < T || T > 0xffffffffLL || k > 0xffffffffLL) return NPGA_ERR_INVALID;
  LAUNCHCHK(npga::launch_philox_sketch(seed, T, k, S, lds, raw, stream));
  return NPGA_OK;
}

}  // extern "C"

namespace {

// Workspace of a batched solve: a single-solve region (power method, float64
// anchors), then the per-target states and vectors and the GEMM buffers.
struct BatchLayout {
  SolveLayout single;
  size_t off_states, off_X, off_vec, off_Ut, off_P, off_usq, off_status, off_act, off_U16, off_Lt, off_sigma,
      off_planes, off_l32, off_prec, total;
  int64_t npad, ldx, ldut, ldpm, ldq, ldu16, ldlt, lds, ld32, ldsp;
  bool cov;
};

constexpr int kMaxSplits = 64;
// Tile of the covariance form's GEMM 2 Sigma X whatever the number of running
// targets: 64 x 64 (the table's 64 x 64 entry; measured at C4 with the
// float32 GEMM against the factor form's choice of 128 x m-wide tiles: 6535
// vs 5304 solves/s; the bfloat16 split-plane GEMM takes the same tile)
constexpr int kCovConfig = 6;
constexpr int kNumVec = 9;  // xbuf0, xbuf1, gbuf0, gbuf1, pvec, fvec, gvec, xa, ga

// cov: the covariance form (Sigma, the bfloat16 planes the SYRK reads, and a
// float32 copy for a bfloat16 factor) instead of the factor form's buffers.
BatchLayout batch_layout(int64_t n, int64_t cols, int32_t m, bool cov = false) {
  BatchLayout l{};
  l.cov = cov;
  l.single = npga::solve_layout(n, cols, NPGA_PATH_GEMV);
  l.npad = (int64_t)256 * l.single.slots;
  l.ldx = l.npad;
  l.ldut = (m + 3) / 4 * 4;
  l.ldpm = (m + 3) / 4 * 4;
  l.ldq = l.ldpm;
  size_t off = align_up(l.single.total, 256);
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  l.off_states = take(sizeof(DevState) * (size_t)m);
  l.off_X = take(sizeof(float) * (size_t)l.ldx * (size_t)m);
  l.off_vec = take(sizeof(double) * (size_t)kNumVec * (size_t)l.npad * (size_t)m);
  l.off_Ut = take(sizeof(float) * (size_t)l.ldut * (size_t)cols);
  l.off_P = take(sizeof(float) * (size_t)kMaxSplits * (size_t)n * (size_t)l.ldpm);
  const int64_t utiles_max = (cols + 63) / 64;
  l.off_usq = take(sizeof(double) * (size_t)utiles_max * (size_t)l.ldq);
  l.off_status = take(sizeof(int32_t) * (size_t)(2 * (m + 1)));
  l.off_act = take(sizeof(int32_t) * (size_t)(m + 1));
  // the refinement's batched float64 anchor gradients (U^T and the split partials)
  l.off_prec = take(npga::precise_batch_bytes(n, cols, m, l.npad));
  l.ldu16 = (cols + 7) / 8 * 8;
  l.ldlt = l.ldu16;
  l.lds = (n + 3) / 4 * 4;
  l.ld32 = l.lds;
  if (cov) {
    l.off_U16 = l.off_Lt = 0;
    l.off_sigma = take(sizeof(float) * (size_t)l.lds * (size_t)n);
    // the SYRK's planes of L, then (once Sigma is formed) Sigma's three
    // bfloat16 planes for the iteration GEMM
    l.ldsp = (n + 63) / 64 * 64;
    l.off_planes = take(std::max(npga::syrk_split_bytes(n, cols), sizeof(uint16_t) * 3 * (size_t)n * (size_t)l.ldsp));
    l.off_l32 = take(sizeof(float) * (size_t)l.ld32 * (size_t)cols);
  } else {
    // bfloat16 factors: U planes and the row-major copy of L
    l.off_U16 = take(sizeof(uint16_t) * 3 * (size_t)m * (size_t)l.ldu16);
    l.off_Lt = take(sizeof(uint16_t) * (size_t)n * (size_t)l.ldlt);
    l.off_sigma = l.off_planes = l.off_l32 = 0;
  }
  l.total = off;
  return l;
}

// The covariance form for a batch: asked for, or AUTO with the single
// solve's rule on the shape (cols >= n, Sigma and the SYRK planes within
// 4 GiB), for a float32 or a bfloat16 factor (Sigma is formed from its
// float32 values, which takes a float32 copy of a bfloat16 factor).
bool batch_uses_covariance(int requested, int64_t n, int64_t cols) {
  if (requested == NPGA_PATH_SYRK) return true;
  return requested == NPGA_PATH_AUTO && resolve_path(NPGA_PATH_AUTO, n, cols, NPGA_F32) == NPGA_PATH_SYRK;
}

// Split and tile counts of a configuration for this factor.
npga::BatchArgs with_config(npga::BatchArgs b, const npga::BatchConfig &cfg) {
  const int64_t cols = b.base.cols;
  if (b.covariance) {
    // Sigma X split over the contraction so that a launch has about 512
    // workgroups (chunks of whole 32-row stages; measured at n = 2000 with
    // 64 x 64 tiles and the split-plane GEMM: 256, 384, 512, 768 and 1024
    // workgroups took 20.5, 18.4, 16.0, 20.0 and 18.2 us per iteration)
    const int64_t n = b.base.n;
    const int64_t tiles = ((n + cfg.u_bm - 1) / cfg.u_bm) * ((b.m + cfg.u_bn - 1) / cfg.u_bn);
    int64_t want = std::max<int64_t>(1, std::min<int64_t>((512 + tiles - 1) / tiles, kMaxSplits));
    want = std::min<int64_t>(want, (n + 31) / 32);
    const int64_t kc = ((n + want - 1) / want + 31) / 32 * 32;
    b.kchunk = kc;
    b.splits = (int32_t)((n + kc - 1) / kc);
    b.utiles = 0;
    return b;
  }
  const int64_t kc = ((cols + cfg.splits - 1) / cfg.splits + 31) / 32 * 32;
  b.kchunk = kc;
  b.splits = (int32_t)((cols + kc - 1) / kc);
  if (b.Lt) {
    const int bt = cfg.g_bn == 32 ? 128 : 64;  // period tile of the bfloat16 U GEMM
    b.utiles = (int32_t)((cols + bt - 1) / bt);
  } else {
    b.utiles = (int32_t)((cols + cfg.u_bm - 1) / cfg.u_bm);
  }
  return b;
}

// The bfloat16 matrix-core path needs 16-byte groups along each column.
bool use_b16(const npga_factor *f) {
  return f->dtype == NPGA_BF16 && (f->ld % 8) == 0 && aligned(f->L, 16);
}

// Per-target vectors are laid out target-major inside each block: vector k
// of target j at v + k * (npad m) + j * npad.
npga::BatchArgs carve_batch(const npga_factor *f, const BatchLayout &l, void *ws, int32_t m,
                            const npga::BatchConfig &cfg) {
  char *base = static_cast<char *>(ws);
  npga::BatchArgs b{};
  SolveArgs &a = b.base;
  a.L = f->L;
  a.dtype = f->dtype;
  a.ld = f->ld;
  a.n = f->n;
  a.cols = f->cols;
  a.mu = f->mu;
  a.mode = npga::kTailNpga;
  a.st = reinterpret_cast<DevState *>(base + l.off_states);
  a.xs = reinterpret_cast<float *>(base + l.off_X);
  double *v = reinterpret_cast<double *>(base + l.off_vec);
  const int64_t blk = l.npad * (int64_t)m;
  a.xbuf0 = v;
  a.xbuf1 = v + blk;
  a.gbuf0 = v + 2 * blk;
  a.gbuf1 = v + 3 * blk;
  b.m = m;
  b.vstride = l.npad;
  b.gstride = l.npad;
  b.ldx = l.ldx;
  b.Ut = reinterpret_cast<float *>(base + l.off_Ut);
  b.ldut = l.ldut;
  b.P = reinterpret_cast<float *>(base + l.off_P);
  b.ldpm = l.ldpm;
  b.usq_part = reinterpret_cast<double *>(base + l.off_usq);
  b.ldq = l.ldq;
  int32_t *act = reinterpret_cast<int32_t *>(base + l.off_act);
  b.act = act;
  b.mact = act + m;
  if (use_b16(f)) {
    b.Lt = reinterpret_cast<const uint16_t *>(base + l.off_Lt);
    b.ldlt = l.ldlt;
    b.U16 = reinterpret_cast<uint16_t *>(base + l.off_U16);
    b.ldu16 = l.ldu16;
    b.u16plane = (int64_t)m * l.ldu16;
  }
  return with_config(b, cfg);
}

// Per-call preparation of the bfloat16 path: Lt = L row-major (zero past
// T) and zeroed U planes (their padding past T must read as zero).
int batch_prepare_b16(const npga::BatchArgs &b, const BatchLayout &l, hipStream_t s) {
  if (!b.Lt) return 0;
  const int64_t u16_floats = (int64_t)(3 * (size_t)b.m * (size_t)l.ldu16 * sizeof(uint16_t) / sizeof(float));
  if (npga::launch_zero_f32(reinterpret_cast<float *>(b.U16), u16_floats, s)) return 1;
  return npga::launch_transpose16(static_cast<const uint16_t *>(b.base.L), b.base.ld, b.base.n, b.base.cols,
                                  const_cast<uint16_t *>(b.Lt), b.ldlt, s);
}

void batch_refine_vectors(npga::BatchArgs &b, const BatchLayout &l, void *ws) {
  double *v = reinterpret_cast<double *>(static_cast<char *>(ws) + l.off_vec);
  const int64_t blk = l.npad * (int64_t)b.m;
  b.base.pvec = v + 4 * blk;
  b.base.fvec = v + 5 * blk;
  b.base.gvec = v + 6 * blk;
  b.base.xa = v + 7 * blk;
  b.base.ga = v + 8 * blk;
}

// Pinned host buffers of a batched call: m states and two status slots.
struct BatchPinned {
  DevState *states = nullptr;
  int32_t *status = nullptr;      // 2 slots of (m + 1)
  int32_t *status_dev = nullptr;  // its device address (written by k_bstatus)
  int32_t cap = 0;
};

BatchPinned *batch_pinned(int32_t m) {
  thread_local BatchPinned p;
  if (p.cap < m) {
    if (p.states) (void)hipHostFree(p.states);
    if (p.status) (void)hipHostFree(p.status);
    p.states = nullptr;
    p.status = nullptr;
    p.status_dev = nullptr;
    p.cap = 0;
    void *a = nullptr, *c = nullptr, *d = nullptr;
    if (hipHostMalloc(&a, sizeof(DevState) * (size_t)m, hipHostMallocDefault) != hipSuccess) return nullptr;
    if (hipHostMalloc(&c, sizeof(int32_t) * (size_t)(2 * (m + 1)), hipHostMallocDefault) != hipSuccess) {
      (void)hipHostFree(a);
      return nullptr;
    }
    if (hipHostGetDevicePointer(&d, c, 0) != hipSuccess || !d) {
      (void)hipHostFree(a);
      (void)hipHostFree(c);
      return nullptr;
    }
    p.states = static_cast<DevState *>(a);
    p.status = static_cast<int32_t *>(c);
    p.status_dev = static_cast<int32_t *>(d);
    p.cap = m;
  }
  return &p;
}

const npga::BatchConfig &batch_config_of(int32_t requested, int64_t n, int64_t cols, int32_t m) {
  const int id = (requested >= 0 && requested < npga::kBatchConfigs) ? requested
                                                                      : npga::batch_default_config(n, cols, m);
  return npga::kBatchConfigTable[id];
}

// Y = 2 L (L^T Omega) row-major in float32 for the refinement's
// preconditioner: Omega's signs as the 32 columns of the batched GEMM pair
// (the factor form, float32 matrix cores), then the split partials summed.
int pcg_build(const npga_factor *f, const SolveLayout &l, char *base, hipStream_t s) {
  npga::BatchArgs b{};
  SolveArgs &a = b.base;
  a.L = f->L;
  a.dtype = f->dtype;
  a.ld = f->ld;
  a.n = f->n;
  a.cols = f->cols;
  a.mu = f->mu;
  a.mode = npga::kTailGrad;
  a.xs = reinterpret_cast<float *>(base + l.off_pre_x);
  b.m = npga::kPreK;
  b.ldx = l.ldp;
  b.Ut = reinterpret_cast<float *>(base + l.off_pre_ut);
  b.ldut = npga::kPreK;
  b.P = reinterpret_cast<float *>(base + l.off_pre_p);
  b.ldpm = npga::kPreK;
  b.usq_part = reinterpret_cast<double *>(base + l.off_pre_usq);
  b.ldq = npga::kPreK;
  int32_t *act = reinterpret_cast<int32_t *>(base + l.off_pre_act);
  b.act = act;
  b.mact = act + npga::kPreK;
  const npga::BatchConfig &cfg = batch_config_of(-1, f->n, f->cols, npga::kPreK);
  b = with_config(b, cfg);
  if (b.splits > npga::kPreMaxSplits || b.utiles > (f->cols + 31) / 32) return 1;
  if (npga::launch_pre_omega(a.xs, l.ldp, f->n, s)) return 1;
  if (npga::launch_bact_all(b, act, act + npga::kPreK, s)) return 1;
  if (npga::launch_bgemm(b, cfg, s)) return 1;
  return npga::launch_pre_reduce(b.P, b.ldpm, b.splits, f->n, reinterpret_cast<float *>(base + l.off_pre_y),
                                 reinterpret_cast<float *>(base + l.off_pre_yt), l.ldp, s);
}

// Configuration for the chunk about to run: the requested one while it is
// not wider than the running targets need, else the built-in choice for
// the narrower tile (the host's count lags the device's by at most a
// chunk, and only ever over-counts, so the grid still covers every column).
const npga::BatchConfig &config_for_running(const npga::BatchConfig &req, int64_t n, int64_t cols,
                                            int32_t running) {
  const int need = running <= 32 ? 32 : (running <= 64 ? 64 : 128);
  if (req.u_bn <= need && req.g_bn <= need) return req;
  return npga::kBatchConfigTable[npga::batch_default_config(n, cols, need)];
}

// Runs chunks of check_every batched iterations until no target is running.
// t_done[j] receives the GPU time from ev0 to the end of the chunk in which
// target j stopped (unchanged for targets that stopped before the phase).
int run_batch_phase(const npga::BatchArgs &b0, const npga::BatchConfig &req, int slots, int check_every,
                    int64_t max_chunks, hipStream_t s, int32_t *dev_status, int32_t *pin_status,
                    int32_t *pin_status_dev, hipEvent_t *evs,
                    hipEvent_t ev0, double *t_done, SweepTimer *tm) {
  const int32_t m = b0.m;
  int32_t running = m;  // last count read back (an upper bound of the device's)
  int32_t *act = const_cast<int32_t *>(b0.act);
  int32_t *mact = const_cast<int32_t *>(b0.mact);
  // GEMM columns = targets running at the start of the phase
  if (npga::launch_bstatus(b0, dev_status, act, mact, s)) return NPGA_ERR_HIP;
  auto issue = [&](int slot) -> int {
    const npga::BatchConfig &cfg =
        b0.covariance ? req : config_for_running(req, b0.base.n, b0.base.cols, running);
    const npga::BatchArgs b = with_config(b0, cfg);
    for (int i = 0; i < check_every; ++i) {
      if (i == 0 && tm && hipEventRecord(tm->a[slot], s) != hipSuccess) return NPGA_ERR_HIP;
      if (npga::launch_bgemm(b, cfg, s)) return NPGA_ERR_HIP;
      if (i == 0 && tm && hipEventRecord(tm->b[slot], s) != hipSuccess) return NPGA_ERR_HIP;
      if (npga::launch_breduce_tail(b, slots, s)) return NPGA_ERR_HIP;
    }
    // running count and done codes, stored by the device into the pinned slot
    pin_status[(size_t)slot * (m + 1)] = kStatusUnset;
    if (npga::launch_bstatus(b, pin_status_dev + (size_t)slot * (m + 1), act, mact, s)) return NPGA_ERR_HIP;
    if (hipEventRecord(evs[slot], s) != hipSuccess) return NPGA_ERR_HIP;
    return NPGA_OK;
  };
  std::vector<char> seen(m, 0);
  int64_t issued = 0, consumed = 0;
  int e = issue(0);
  if (e) return e;
  ++issued;
  e = issue(1);
  if (e) return e;
  ++issued;
  for (;;) {
    const int slot = consumed & 1;
    if (hipEventSynchronize(evs[slot]) != hipSuccess) return NPGA_ERR_HIP;
    ++consumed;
    const int32_t *hs = pin_status + (size_t)slot * (m + 1);
    int32_t nrun = 0;
    if (!read_status(hs, &nrun)) return NPGA_ERR_HIP;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev0, evs[slot]);
    for (int32_t j = 0; j < m; ++j) {
      if (!seen[j] && hs[1 + j] != npga::kRunning) {
        seen[j] = 1;
        if (t_done[j] < 0) t_done[j] = ms;
      }
    }
    running = nrun;
    if (tm && nrun == m) {  // pairs over the full batch only
      float g = 0.f;
      if (hipEventElapsedTime(&g, tm->a[slot], tm->b[slot]) == hipSuccess) {
        tm->total_ms += g;
        tm->samples += 1;
      }
    }
    if (nrun == 0) {
      if (hipStreamSynchronize(s) != hipSuccess) return NPGA_ERR_HIP;
      return NPGA_OK;
    }
    if (issued >= max_chunks) {
      if (hipStreamSynchronize(s) != hipSuccess) return NPGA_ERR_HIP;
      return NPGA_OK;
    }
    e = issue(slot);
    if (e) return e;
    ++issued;
  }
}

}  // namespace

extern "C" {

size_t npga_batched_workspace_size(int64_t n, int64_t cols, int32_t m, const npga_options *opt) {
  if (n < 1 || n > NPGA_MAX_N || cols < 1 || m < 1 || m > NPGA_MAX_BATCH) return 0;
  npga_options o;
  npga_default_options(&o);
  if (opt) o = *opt;
  const size_t fac = batch_layout(n, cols, m).total;
  // the covariance form's buffers when that form would run; never less than
  // the factor form's (npga_gradient_batched and npga_batched_tune use it)
  return batch_uses_covariance(o.path, n, cols) ? std::max(fac, batch_layout(n, cols, m, true).total) : fac;
}

int npga_solve_batched(const npga_factor *f, const double *r_targets, int32_t m, const npga_options *opt,
                       float *X, int64_t ldx, npga_result *res, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  const auto t0 = Clock::now();
  npga_options o;
  npga_default_options(&o);
  if (opt) o = *opt;
  // per-target steps (backtracking) and Dykstra's projections are single-solve options
  if (o.backtrack_rho > 0.0 || o.projection != 0) return NPGA_ERR_INVALID;
  if (!factor_valid(f) || !r_targets || !X || m < 1 || m > NPGA_MAX_BATCH || ldx < f->n ||
      !options_valid(o) || !aligned(X, 4))
    return NPGA_ERR_INVALID;
  if (o.momentum == 1 && !(f->gamma > 0.0)) return NPGA_ERR_INVALID;
  for (int32_t j = 0; j < m; ++j)
    if (!is_fin(r_targets[j])) return NPGA_ERR_INVALID;
  const bool cov = batch_uses_covariance(o.path, f->n, f->cols);
  const BatchLayout lay = batch_layout(f->n, f->cols, m, cov);
  if (!ws || !aligned(ws, 256) || ws_bytes < lay.total) return NPGA_ERR_WORKSPACE;
  DevState *pin = pinned_status();
  BatchPinned *bp = batch_pinned(m);
  if (!pin || !bp) return NPGA_ERR_HIP;
  // the covariance form tiles by the batch width (batch_config tunes the
  // factor form's GEMM pair)
  const npga::BatchConfig &cfg = cov ? npga::kBatchConfigTable[kCovConfig]
                                     : batch_config_of(o.batch_config, f->n, f->cols, m);
  Carved c = carve(f, lay.single, ws, NPGA_PATH_GEMV);
  npga::BatchArgs b = carve_batch(f, lay, ws, m, cfg);
  const int slots = lay.single.slots;
  int32_t *dev_status = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + lay.off_status);

  hipEvent_t ev0, evs[2], ev_setup;
  SweepTimer tm;
  EventSet<8> events;
  HIPCHK(events.make(&ev0));
  HIPCHK(events.make(&evs[0], false));
  HIPCHK(events.make(&evs[1], false));
  HIPCHK(events.make(&ev_setup));
  for (int i = 0; i < 2; ++i) {
    HIPCHK(events.make(&tm.a[i]));
    HIPCHK(events.make(&tm.b[i]));
  }

  HIPCHK(hipEventRecord(ev0, stream));
  // mu statistics and feasibility of every target (one synchronisation)
  pin[2] = initial_state(f, r_targets[0], o);
  HIPCHK(hipMemcpyAsync(c.st, &pin[2], sizeof(DevState), hipMemcpyHostToDevice, stream));
  LAUNCHCHK(npga::launch_prepare(c.a, stream));
  HIPCHK(hipMemcpyAsync(&pin[3], c.st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (pin[3].n_nonfinite > 0) return NPGA_ERR_NUMERIC;
  const double mu_max = pin[3].mu_max, mu_absmax = pin[3].mu_absmax;
  for (int32_t j = 0; j < m; ++j)
    if (r_targets[j] > mu_max) return NPGA_ERR_INFEASIBLE;

  // shared step size from ||L||_2^2 (Sec. 3.1 Remark).  The few extra
  // Lanczos sweeps of the tight tolerance are negligible against m solves,
  // and the accurate estimate keeps the slowest target's count down.
  LAUNCHCHK(estimate_step(c, NPGA_PATH_GEMV, slots, o, stream, 1e-4));

  // per-target states, x^0 = Pi_F(x_in or 1/n)
  for (int32_t j = 0; j < m; ++j) {
    DevState s0 = initial_state(f, r_targets[j], o);
    s0.mu_max = mu_max;
    s0.mu_absmax = mu_absmax;
    s0.tolphi = o.proj_tol * std::max(std::fabs(r_targets[j]), mu_absmax);
    bp->states[j] = s0;
  }
  HIPCHK(hipMemcpyAsync(b.base.st, bp->states, sizeof(DevState) * (size_t)m, hipMemcpyHostToDevice, stream));
  LAUNCHCHK(npga::launch_bcopy_step(b, c.st, stream));
  if (cov) {
    // Sigma = L L^T once (split-plane SYRK on the float32 values of L);
    // every iteration then takes 2 Sigma X from one GEMM
    char *base = static_cast<char *>(ws);
    float *sigma = reinterpret_cast<float *>(base + lay.off_sigma);
    const float *L32 = static_cast<const float *>(f->L);
    int64_t ld32 = f->ld;
    if (f->dtype == NPGA_BF16) {
      float *w = reinterpret_cast<float *>(base + lay.off_l32);
      LAUNCHCHK(npga::launch_widen_bf16(static_cast<const uint16_t *>(f->L), f->ld, f->n, f->cols, w, lay.ld32,
                                        stream));
      L32 = w;
      ld32 = lay.ld32;
    }
    uint16_t *planes = reinterpret_cast<uint16_t *>(base + lay.off_planes);
    LAUNCHCHK(npga::launch_syrk_split(L32, f->n, f->cols, ld32, planes, sigma, lay.lds, stream));
    // Sigma's bfloat16 planes over the SYRK's (the SYRK is done with them
    // in stream order): the iteration GEMM runs on the bfloat16 matrix cores
    LAUNCHCHK(npga::launch_split_rows(sigma, f->n, f->n, lay.lds, planes, lay.ldsp, f->n * lay.ldsp, stream));
    b.Sp = planes;
    b.ldsp = lay.ldsp;
    b.spplane = f->n * lay.ldsp;
    b.base.L = sigma;
    b.base.ld = lay.lds;
    b.base.cols = f->n;
    b.base.dtype = NPGA_F32;
    b.Lt = nullptr;
    b.U16 = nullptr;
    b.covariance = 1;
    b = with_config(b, cfg);
  }
  LAUNCHCHK(batch_prepare_b16(b, lay, stream));
  LAUNCHCHK(npga::launch_bset_x0(b, o.warm_start ? X : nullptr, ldx, stream));
  LAUNCHCHK(npga::launch_bproject_init(b, slots, stream));
  HIPCHK(hipEventRecord(ev_setup, stream));

  std::vector<double> t_done(m, -1.0);
  const int64_t main_chunks = (int64_t)o.max_iter / o.check_every + 4;
  int e = run_batch_phase(b, cfg, slots, o.check_every, main_chunks, stream, dev_status, bp->status,
                          bp->status_dev, evs, ev0,
                          t_done.data(), &tm);
  if (e) return e;
  HIPCHK(hipMemcpyAsync(bp->states, b.base.st, sizeof(DevState) * (size_t)m, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  std::vector<DevState> after_main(bp->states, bp->states + m);

  std::vector<int32_t> refine_iters(m, 0), refined(m, 0), ref_done(m, npga::kConverged);
  bool any = false;
  for (int32_t j = 0; j < m; ++j) any = any || after_main[j].done == npga::kConverged;
  if (any && o.refine && o.refine_max_iter > 0) {
    batch_refine_vectors(b, lay, ws);
    npga::BatchArgs br = b;
    br.base.mode = npga::kTailCG;
    std::vector<double> t_unused(m, 0.0);
    for (int round = 0; round < 2; ++round) {
      // float64 anchor gradients of every target still converged (the
      // device's done flags are the ones copied to the host above)
      LAUNCHCHK(npga::launch_bcopy_anchor(br, stream));
      LAUNCHCHK(npga::launch_precise_gradient_batched(
          f->L, f->dtype, f->ld, f->n, f->cols, br.base.xa, br.vstride, m, br.base.st,
          reinterpret_cast<double *>(static_cast<char *>(ws) + lay.off_prec), lay.npad,
          const_cast<double *>(br.base.ga), br.vstride, stream));
      LAUNCHCHK(npga::launch_bphase_reset(br, o.refine_tol, o.refine_max_iter, stream));
      LAUNCHCHK(npga::launch_bcg_init(br, slots, stream));
      const int64_t ref_chunks = (int64_t)o.refine_max_iter / o.check_every + 4;
      e = run_batch_phase(br, cfg, slots, o.check_every, ref_chunks, stream, dev_status, bp->status,
                          bp->status_dev, evs, ev0,
                          t_unused.data(), nullptr);
      if (e) return e;
      HIPCHK(hipMemcpyAsync(bp->states, b.base.st, sizeof(DevState) * (size_t)m, hipMemcpyDeviceToHost,
                            stream));
      HIPCHK(hipStreamSynchronize(stream));
      for (int32_t j = 0; j < m; ++j) {
        const int32_t prev = round == 0 ? after_main[j].done : ref_done[j];
        if (prev != npga::kConverged) continue;
        refine_iters[j] += bp->states[j].cg_iter;
        ref_done[j] = bp->states[j].done;
        refined[j] = (bp->states[j].done == npga::kConverged && bp->states[j].cg_kkt) ? 1 : 0;
      }
    }
  }
  LAUNCHCHK(npga::launch_bfinalize(b, X, ldx, stream));
  HIPCHK(hipMemcpyAsync(bp->states, b.base.st, sizeof(DevState) * (size_t)m, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));

  float setup_ms = 0.f;
  (void)hipEventElapsedTime(&setup_ms, ev0, ev_setup);
  const double wall = ms_since(t0);
  int first_bad = NPGA_OK;
  for (int32_t j = 0; j < m; ++j) {
    const DevState &am = after_main[j];
    const DevState &fin = bp->states[j];
    int status = map_done(am.done);
    if (am.done == npga::kConverged && ref_done[j] != npga::kConverged && ref_done[j] != npga::kMaxIter)
      status = map_done(ref_done[j]);
    if (status != NPGA_OK && first_bad == NPGA_OK) first_bad = status;
    if (!res) continue;
    npga_result &rj = res[j];
    std::memset(&rj, 0, sizeof(rj));
    rj.status = status;
    rj.iters = (am.done == npga::kConverged) ? am.stop_iter : am.iter;
    rj.refine_iters = refine_iters[j];
    rj.support = fin.support;
    rj.return_active = fin.nu_c > 0.0 ? 1 : 0;
    rj.refined = refined[j];
    rj.path_used = cov ? NPGA_PATH_SYRK : NPGA_PATH_GEMV;
    rj.step_sweeps = o.alpha > 0.0 ? 0 : (o.step_estimator == 0 ? after_main[j].lz_m : o.power_iters);
    rj.residual = am.stop_residual;
    rj.final_residual = fin.residual;
    rj.objective = fin.objective;
    rj.nu = fin.nu_kkt;
    rj.lambda = fin.lambda_kkt;
    rj.alpha = fin.alpha;
    rj.lipschitz = fin.lipschitz;
    rj.time_ms = wall;
    rj.time_to_tol_ms = t_done[j];
    rj.setup_ms = setup_ms;
    rj.sweep_ms = tm.samples ? tm.total_ms / tm.samples : 0.0;
    rj.sweep_samples = tm.samples;
  }
  return first_bad;
}

int npga_gradient_batched(const npga_factor *f, const float *X, int64_t ldx, int32_t m, double *G, int64_t ldg,
                          double *f_out, int32_t config, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (!factor_valid(f) || !X || !G || m < 1 || m > NPGA_MAX_BATCH || ldx < f->n || ldg < f->n ||
      config < -1 || config >= npga::kBatchConfigs || !aligned(X, 4) || !aligned(G, 8))
    return NPGA_ERR_INVALID;
  const BatchLayout lay = batch_layout(f->n, f->cols, m);
  if (!ws || !aligned(ws, 256) || ws_bytes < lay.total) return NPGA_ERR_WORKSPACE;
  BatchPinned *bp = batch_pinned(m);
  if (!bp) return NPGA_ERR_HIP;
  npga_options o;
  npga_default_options(&o);
  const npga::BatchConfig &cfg = batch_config_of(config, f->n, f->cols, m);
  npga::BatchArgs b = carve_batch(f, lay, ws, m, cfg);
  b.base.mode = npga::kTailGrad;
  b.base.gbuf0 = G;
  b.base.gbuf1 = nullptr;
  b.gstride = ldg;
  for (int32_t j = 0; j < m; ++j) bp->states[j] = initial_state(f, 0.0, o);
  HIPCHK(hipMemcpyAsync(b.base.st, bp->states, sizeof(DevState) * (size_t)m, hipMemcpyHostToDevice, stream));
  LAUNCHCHK(batch_prepare_b16(b, lay, stream));
  LAUNCHCHK(npga::launch_bload_x(b, X, ldx, stream));
  LAUNCHCHK(npga::launch_bact_all(b, const_cast<int32_t *>(b.act), const_cast<int32_t *>(b.mact), stream));
  LAUNCHCHK(npga::launch_bgemm(b, cfg, stream));
  LAUNCHCHK(npga::launch_breduce_tail(b, lay.single.slots, stream));
  if (f_out) {
    HIPCHK(hipMemcpyAsync(bp->states, b.base.st, sizeof(DevState) * (size_t)m, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    for (int32_t j = 0; j < m; ++j) f_out[j] = bp->states[j].objective;
  }
  return NPGA_OK;
}

int npga_batched_tune(const npga_factor *f, int32_t m, int32_t reps, int32_t *best, float *ms_out, void *ws,
                      size_t ws_bytes, hipStream_t stream) {
  if (!factor_valid(f) || !best || m < 1 || m > NPGA_MAX_BATCH || reps < 1) return NPGA_ERR_INVALID;
  const BatchLayout lay = batch_layout(f->n, f->cols, m);
  if (!ws || !aligned(ws, 256) || ws_bytes < lay.total) return NPGA_ERR_WORKSPACE;
  hipEvent_t a, z;
  EventSet<2> events;
  HIPCHK(events.make(&a, false));
  HIPCHK(events.make(&z, false));
  {
    const npga::BatchConfig &c0 = npga::kBatchConfigTable[0];
    npga::BatchArgs b0 = carve_batch(f, lay, ws, m, c0);
    LAUNCHCHK(batch_prepare_b16(b0, lay, stream));
    LAUNCHCHK(npga::launch_bset_x0(b0, nullptr, 0, stream));  // zero GEMM input
    LAUNCHCHK(npga::launch_bact_all(b0, const_cast<int32_t *>(b0.act), const_cast<int32_t *>(b0.mact), stream));
  }
  float best_ms = 1e30f;
  int32_t best_id = 0;
  for (int c = 0; c < npga::kBatchConfigs; ++c) {
    const npga::BatchConfig &cfg = npga::kBatchConfigTable[c];
    npga::BatchArgs b = carve_batch(f, lay, ws, m, cfg);
    LAUNCHCHK(npga::launch_bgemm(b, cfg, stream));  // warm-up
    HIPCHK(hipEventRecord(a, stream));
    for (int r = 0; r < reps; ++r) LAUNCHCHK(npga::launch_bgemm(b, cfg, stream));
    HIPCHK(hipEventRecord(z, stream));
    HIPCHK(hipEventSynchronize(z));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, a, z));
    ms /= (float)reps;
    if (ms_out) ms_out[c] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best_id = c;
    }
  }
  *best = best_id;
  return NPGA_OK;
}

// The adjoint's face CG is preconditioned as the refinement's is (npga_pcg.h)
// for n >= 2048 and cols >= n (the factor shapes whose face Hessian has a
// few outliers above a narrow bulk).
bool adj_pcg(int64_t n, int64_t cols) { return n >= 2048 && n <= NPGA_MAX_N && cols >= n; }

size_t npga_backward_workspace_size(int64_t n, int64_t cols) {
  if (n < 1 || n > NPGA_MAX_N || cols < 1) return 0;
  const SolveLayout l = npga::solve_layout(n, cols, NPGA_PATH_GEMV, adj_pcg(n, cols));
  const size_t npad = (size_t)256 * l.slots;
  return align_up(l.total, 256) + align_up(sizeof(double) * (3 * npad + (size_t)cols), 256);
}

int npga_backward(const npga_factor *f, double r, const float *x_star, const float *dl_dx, double *dl_dmu,
                  float *dl_dL, int64_t ldg, npga_backward_result *res, void *ws, size_t ws_bytes,
                  hipStream_t stream) {
  const auto t0 = Clock::now();
  if (!factor_valid(f) || !x_star || !dl_dx || !dl_dmu || !is_fin(r) || !aligned(dl_dmu, 8)) return NPGA_ERR_INVALID;
  if (dl_dL && ldg < f->n) return NPGA_ERR_INVALID;
  const SolveLayout lay = npga::solve_layout(f->n, f->cols, NPGA_PATH_GEMV, adj_pcg(f->n, f->cols));
  if (!ws || !aligned(ws, 256) || ws_bytes < npga_backward_workspace_size(f->n, f->cols)) return NPGA_ERR_WORKSPACE;
  DevState *pin = pinned_status();
  if (!pin) return NPGA_ERR_HIP;
  npga_options o;
  npga_default_options(&o);
  Carved c = carve(f, lay, ws, NPGA_PATH_GEMV);
  const int slots = lay.slots;
  const int64_t npad = (int64_t)256 * slots;
  char *base = static_cast<char *>(ws);
  double *rhs = reinterpret_cast<double *>(base + lay.off_xa);
  double *G = reinterpret_cast<double *>(base + lay.off_ga);
  double *u = reinterpret_cast<double *>(base + lay.off_ua);
  double *vecs = reinterpret_cast<double *>(base + lay.off_vecs);
  double *extra = reinterpret_cast<double *>(base + align_up(lay.total, 256));
  double *gl = extra;
  double *abase = extra + npad;
  double *hab = extra + 2 * npad;
  double *v = extra + 3 * npad;  // cols doubles
  double *part = reinterpret_cast<double *>(c.a.partials);
  c.a.pvec = vecs;
  c.a.fvec = vecs + npad;
  c.a.gvec = vecs + 2 * npad;
  c.a.ga = G;

  pin[2] = initial_state(f, r, o);
  HIPCHK(hipMemcpyAsync(c.st, &pin[2], sizeof(DevState), hipMemcpyHostToDevice, stream));
  LAUNCHCHK(npga::launch_prepare(c.a, stream));
  HIPCHK(hipMemcpyAsync(&pin[3], c.st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (pin[3].n_nonfinite > 0) return NPGA_ERR_NUMERIC;
  const double act_tol = 1e-6 * std::max(std::fabs(r), pin[3].mu_absmax);

  // x* (float64) and the loss gradient; float64 gradient of f at x*
  LAUNCHCHK(npga::launch_set_vector(c.a.xbuf1, x_star, nullptr, f->n, 0.0, nullptr, stream));
  LAUNCHCHK(npga::launch_set_vector(gl, dl_dx, nullptr, f->n, 0.0, nullptr, stream));
  LAUNCHCHK(npga::launch_set_vector(abase, nullptr, nullptr, f->n, 0.0, nullptr, stream));
  LAUNCHCHK(npga::launch_precise_gradient(c.a, c.a.xbuf1, u, G, part, slots, stream));
  LAUNCHCHK(npga::launch_adj_face(c.a, slots, act_tol, stream));

  // projected CG on the face, two rounds: the second solves for the
  // correction from the float64 residual of the first
  Carved cg = c;
  cg.a.mode = npga::kTailAdj;
  cg.a.ga = nullptr;
  if (lay.pcg) {
    // the face CG preconditioned as in the refinement: Y = H Omega once
    LAUNCHCHK(pcg_build(f, lay, base, stream));
    cg.a.pre_y = reinterpret_cast<const float *>(base + lay.off_pre_y);
    cg.a.pre_yt = reinterpret_cast<const float *>(base + lay.off_pre_yt);
    cg.a.pre_mat = reinterpret_cast<double *>(base + lay.off_pre_mat);
    cg.a.pre_a1 = reinterpret_cast<double *>(base + lay.off_pre_a1);
    cg.a.pre_a2 = reinterpret_cast<double *>(base + lay.off_pre_a2);
    cg.a.pre_z = reinterpret_cast<double *>(base + lay.off_pre_z);
    cg.a.pre_part = reinterpret_cast<double *>(base + lay.off_pre_part);
    cg.a.pre_gpart = reinterpret_cast<double *>(base + lay.off_pre_gpart);
  }
  hipEvent_t evs[2], ev0;
  EventSet<3> events;
  HIPCHK(events.make(&ev0));
  HIPCHK(events.make(&evs[0], false));
  HIPCHK(events.make(&evs[1], false));
  HIPCHK(hipEventRecord(ev0, stream));
  int cg_iters = 0, done = npga::kConverged;
  const int max_iter = 4 * (int)std::min<int64_t>(f->n, 5000) + 100;
  for (int round = 0; round < 2; ++round) {
    const double *rr = gl;
    if (round > 0) {
      LAUNCHCHK(npga::launch_adj_rhs(f->n, f->gamma, gl, abase, hab, rhs, stream));
      rr = rhs;
    }
    LAUNCHCHK(npga::launch_phase(c.st, 0, 0.0, max_iter, 0, stream));
    LAUNCHCHK(npga::launch_adj_init(cg.a, rr, slots, stream));
    // first direction: S and sigma on the face in the first round, the
    // face's factor again in the second
    if (cg.a.pre_y) LAUNCHCHK(npga::launch_pcg_init(cg.a, slots, round == 0, stream));
    double ms = 0.0;
    const int64_t chunks = (int64_t)max_iter / o.check_every + 4;
    int e = run_phase(cg, NPGA_PATH_GEMV, slots, o.check_every, chunks, stream, pin, evs, ev0, &done, &ms, nullptr);
    if (e) return e;
    HIPCHK(hipMemcpyAsync(&pin[2], c.st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    cg_iters += pin[2].cg_iter;
    LAUNCHCHK(npga::launch_adj_accum(c.a, abase, stream));
    // float64 product H a_total for the next right-hand side and the finish
    LAUNCHCHK(npga::launch_precise_gradient(c.a, abase, v, hab, part, slots, stream));
    if (done != npga::kConverged) break;
  }
  LAUNCHCHK(npga::launch_adj_finish(c.a, gl, abase, hab, dl_dmu, slots, stream));
  if (dl_dL) LAUNCHCHK(npga::launch_adj_dL(abase, c.a.xbuf1, u, v, f->n, f->cols, dl_dL, ldg, stream));
  HIPCHK(hipMemcpyAsync(&pin[3], c.st, sizeof(DevState), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  const DevState &fin = pin[3];
  int status = NPGA_OK;
  if (done == npga::kNumeric) status = NPGA_ERR_NUMERIC;
  else if (done != npga::kConverged) status = NPGA_ERR_NOT_CONVERGED;
  if (res) {
    std::memset(res, 0, sizeof(*res));
    res->status = status;
    res->cg_iters = cg_iters;
    res->support = fin.support;
    res->return_active = fin.cg_active;
    res->degenerate = (fin.proj_flags & 4) ? 1 : 0;
    res->nu = fin.nu_kkt;
    res->lambda = fin.lambda_kkt;
    res->dl_dr = fin.adj_anu;
    res->dl_dgamma = fin.adj_dgamma;
    res->residual = fin.adj_res;
    res->time_ms = ms_since(t0);
  }
  return status;
}

}  // extern "C"
