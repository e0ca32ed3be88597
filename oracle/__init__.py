"""Plain FP64 CPU oracle for the autoencoder-compressed adjoint method.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, calls or
links this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it. It shares no code with the HIP library; the
only common dependency is the seeded input generator in `workloads`.

Modules
  wave      forward solve, misfit, exact discrete adjoint, gradient,
            incremental forward, Gauss-Newton and full-Newton Hv
            (paper Sec. 2, Eq. (model) and the MAP objective; Sec. 4
            for the Newton-CG use of gradient and Hv)
  ae        per-vector normalisation (Sec. 3.3.1), the dense autoencoder
            (Sec. 3.3, Eq. (single_layer)), its backward pass, Adam, and
            the patch layout of the space compression scheme (Sec. 3.1)
  rounding  bfloat16 and OCP FP8 E4M3FN round-to-nearest-even
  revolve   optimal binomial checkpointing cost (closed form and DP)
  inverse   BiLaplacian prior (Sec. 2) and the inexact Newton-CG loop for
            the MAP point (Sec. 4)
"""
