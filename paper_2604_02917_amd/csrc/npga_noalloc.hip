// npga_gradient_noalloc: the fused gradient sweep of eq. npga-unified-grad
// (g = 2 L (L^T x) + 2 gamma x and f = ||L^T x||^2 + gamma ||x||^2) with its
// scratch space in a file-scope device array instead of a caller workspace,
// for callers that cannot allocate (code under HIP graph capture, serving
// loops that must not call the allocator).
//
// The array below is a host-side stand-in in host code: its device address
// is looked up once per device with hipGetSymbolAddress (the first call on
// that device, with the device current) and only that address is passed to
// kernels.  Each device holds its own copy until the process ends.  Every
// call on a device shares that device's copy: calls that overlap on one
// device (different streams or host threads) race.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "npga.h"
#include "npga_internal.h"

namespace npga {
namespace {

// Largest scratch the gradient needs: the solver state, the padded float32
// copy of x and its float64 copy, the per-workgroup ||L^T x||^2 partials and
// the float32 partial gradient vectors (at most 256 sweep workgroups of
// 256 * slots_for(NPGA_MAX_N) = 8192 rows each, 8 MiB).
constexpr size_t kScratchBytes = (size_t)8 * 1024 * 1024 + (size_t)256 * 1024;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the
// first call for that device).
int scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return NPGA_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return NPGA_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NPGA_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NPGA_OK;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct NoAllocLayout {
  size_t off_state, off_xs, off_x, off_usq, off_part, total;
  int32_t slots, grid;
  int64_t ldp;
};

NoAllocLayout noalloc_layout(int64_t n, int64_t cols) {
  NoAllocLayout l{};
  l.slots = slots_for(n);
  l.grid = sweep_grid_for(cols);
  l.ldp = (int64_t)256 * l.slots;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  l.off_state = take(sizeof(DevState));
  l.off_xs = take(sizeof(float) * (size_t)l.ldp);
  l.off_x = take(sizeof(double) * (size_t)l.ldp);
  l.off_usq = take(sizeof(double) * (size_t)l.grid);
  l.off_part = take(sizeof(float) * (size_t)l.grid * (size_t)l.ldp);
  l.total = off;
  return l;
}

// The largest layout (n = NPGA_MAX_N, the widest sweep grid) fits the array.
static_assert(sizeof(DevState) + (size_t)4 * 8192 + (size_t)8 * 8192 + (size_t)8 * 256 +
                      (size_t)4 * 256 * 8192 + (size_t)5 * 256 <=
                  kScratchBytes,
              "scratch array too small for the largest gradient");

// Clears the solver state the gradient kernels read (every word, so nothing
// left by an earlier call survives) and sets the running flag and the ridge.
__global__ __launch_bounds__(256) void k_noalloc_state(DevState *st, double gamma) {
  uint32_t *w = reinterpret_cast<uint32_t *>(st);
  for (size_t i = threadIdx.x; i < sizeof(DevState) / 4; i += 256) w[i] = 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    st->done = kRunning;
    st->gamma = gamma;
    st->check_every = 1;
  }
}

bool factor_ok(const npga_factor *f) {
  if (!f || !f->L || !f->mu) return false;
  if (f->n < 1 || f->n > NPGA_MAX_N || f->cols < 1) return false;
  if (f->ld < f->n || (f->ld % 4) != 0) return false;
  if (f->dtype != NPGA_F32 && f->dtype != NPGA_BF16) return false;
  const uintptr_t pl = reinterpret_cast<uintptr_t>(f->L);
  if (pl % (f->dtype == NPGA_F32 ? 16 : 8) != 0) return false;
  if (reinterpret_cast<uintptr_t>(f->mu) % 8 != 0) return false;
  if (!(f->gamma >= 0.0) || f->gamma > 1.0e308) return false;
  return true;
}

}  // namespace
}  // namespace npga

extern "C" size_t npga_gradient_noalloc_max_bytes(void) { return npga::kScratchBytes; }

extern "C" int npga_gradient_noalloc(const npga_factor *f, const float *x, double *g, double *f_out,
                                     hipStream_t stream) {
  using namespace npga;
  if (!factor_ok(f) || !x || !g || (reinterpret_cast<uintptr_t>(g) % 8) != 0) return NPGA_ERR_INVALID;
  const NoAllocLayout lay = noalloc_layout(f->n, f->cols);
  if (lay.slots < 1 || lay.total > kScratchBytes) return NPGA_ERR_WORKSPACE;
  void *ptr = nullptr;
  const int e = scratch_address(&ptr);
  if (e != NPGA_OK) return e;
  unsigned char *base = static_cast<unsigned char *>(ptr);
  SolveArgs a{};
  a.L = f->L;
  a.dtype = f->dtype;
  a.ld = f->ld;
  a.n = f->n;
  a.cols = f->cols;
  a.mu = f->mu;
  a.st = reinterpret_cast<DevState *>(base + lay.off_state);
  a.xs = reinterpret_cast<float *>(base + lay.off_xs);
  a.xbuf0 = reinterpret_cast<double *>(base + lay.off_x);
  a.gbuf0 = g;
  a.usq_part = reinterpret_cast<double *>(base + lay.off_usq);
  a.partials = reinterpret_cast<float *>(base + lay.off_part);
  a.ldp = lay.ldp;
  a.sweep_grid = lay.grid;
  a.mode = kTailGrad;
  hipLaunchKernelGGL(k_noalloc_state, dim3(1), dim3(256), 0, stream, a.st, f->gamma);
  if (hipGetLastError() != hipSuccess) return NPGA_ERR_HIP;
  if (launch_set_vector(a.xbuf0, x, nullptr, f->n, 0.0, a.xs, stream)) return NPGA_ERR_HIP;
  if (launch_sweep(a, lay.slots, stream)) return NPGA_ERR_HIP;
  if (launch_reduce_tail(a, lay.slots, stream)) return NPGA_ERR_HIP;
  if (f_out) {
    double h = 0.0;
    if (hipMemcpyAsync(&h, &a.st->objective, sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess)
      return NPGA_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return NPGA_ERR_HIP;
    *f_out = h;
  }
  return NPGA_OK;
}
