"""Plain FP64 CPU oracle for iterative Vecchia-Laplace inference.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle is written from the paper (Kuendig & Sigrist, "Iterative Methods
for Vecchia-Laplace Approximations for Latent Gaussian Process Models",
arXiv 2310.12000) in NumPy/SciPy, FP64 throughout, with no blocking, fusion or
reordering beyond what the paper's definitions and algorithms state.  Each
function cites the section / equation / algorithm it follows.

Modules
  rng       counter-based SplitMix64 probes (Rademacher, Gaussian)
  vecchia   nearest-earlier-neighbour sets, covariance, Vecchia factor B, D
            and its theta-derivatives (Sec. 2.1; App. "Derivatives of the
            Vecchia-approximated precision")
  laplace   likelihoods, preconditioned CG with Lanczos coefficients, Newton
            mode, SLQ negative log-marginal likelihood, STE gradient, LRAC
            preconditioner, simulation-based predictive variances (Sec. 2.2,
            3, App. A)

Parity status per function is listed in each module header.
"""
