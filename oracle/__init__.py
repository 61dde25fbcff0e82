"""FP64 CPU oracle for the NPGA mean-variance solver (test infrastructure).

This package is the independent checker of the HIP library.  It is plain,
slow and written to be read against the paper (arXiv 2604.02917, "Scalable
Mean-Variance Portfolio Optimization via Subspace Embeddings and
GPU-Friendly Nesterov-Accelerated Projected Gradient").  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the product path never does.  It shares no code, constants or helpers with
the HIP path; both sides read the same seeded inputs from ``gen``.

Every function states the passage it follows.  All arithmetic is float64.

Modules
  factor      sample mean and centered factor L            (Sec. 2.1)
  projection  simplex projection and the scalar dual search (Sec. 3.1)
  npga        power method and Algorithm 1 (NPGA)           (Sec. 3.1)
  qp          exact QP: brute force, active set, KKT checks (eq. mv; Sec. 3.1 stopping rule)
  sketch      Gaussian sketch, truncation, ridge (STR)      (Sec. 2.3-2.6, App. D)
  philox      Philox4x32-10 counter RNG + Box-Muller        (Salmon et al., SC'11)

Parity status: every function is pinned by a CPU test against a closed
form, brute force or an invariant; the NPGA iterate trajectory by a scalar
FISTA on the two-asset segment (projection = clamp).
"""
