// Internal declarations of the sketch-truncate-ridge build (npga_sketch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace npga {

// Device buffers of the k x k symmetric eigensolver (all float64).
struct SketchState {
  int64_t k;
  double *A;      // k x k, leading dim k: G on entry, reflectors on exit
  double *d;      // diagonal of T (k)
  double *e;      // off-diagonal of T (k - 1)
  double *tau;    // reflector scalars (k)
  double *vcur;   // current reflector (k)
  double *vprev;  // previous reflector (k)
  double *wprev;  // previous rank-2 companion vector (k)
  double *p;      // tau A v of the current step (k)
  double *lam;    // wanted eigenvalues, descending (ell)
  double *Z;      // eigenvectors of T, then of G (k x ell, leading dim k)
  double *work;   // tridiagonalisation scratch, then inverse-iteration factors
                  // (5 stride k doubles + stride k bytes)
};

int launch_gemm_f32(const float *A, int64_t lda, const float *B, int64_t ldb, float *C, int64_t ldc,
                    int64_t M, int64_t N, int64_t K, hipStream_t st);
int launch_gram_f64(const float *Y, int64_t ldy, int64_t n, int64_t k, double *G, hipStream_t st);
int launch_frob(const float *Y, int64_t ldy, int64_t n, int64_t k, double *part, int nparts,
                hipStream_t st);
// Bytes of `work` the tridiagonalisation uses (partial sums and counters).
size_t tri_scratch_bytes(int64_t k);
int launch_tridiag(const SketchState &s, hipStream_t st);
int launch_bisect(const SketchState &s, int64_t ell, hipStream_t st);
int launch_inverse_iter(const SketchState &s, int64_t ell, int64_t stride, hipStream_t st);
int launch_backtransform(const SketchState &s, int64_t ell, float *V32, hipStream_t st);
int launch_finish_str(const SketchState &s, int64_t ell, int64_t n, double coef, const double *frob_part,
                      int nparts, float *sigma, double *gamma_dev, double kappa_tar, hipStream_t st);
int launch_philox_sketch(uint64_t seed, int64_t T, int64_t k, float *S, int64_t lds, uint32_t *raw,
                         hipStream_t s);
int launch_countsketch(const float *L, int64_t ld, int64_t n, int64_t T, const int32_t *h, const float *sgn,
                       int64_t k, float *Y, int64_t ldy, int32_t *bad, hipStream_t s);
int launch_knee(const double *lam, int64_t m, double tau, double rho, int64_t *ell, hipStream_t s);

}  // namespace npga
