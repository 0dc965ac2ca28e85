"""Plain, slow, FP64 CPU oracle for msMINRES-CIQ.

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it. The product path (the
HIP library and its Python binding) never imports, calls or links anything
in here, and this package never imports the product path.

What it computes (Pleiss et al., "Fast Matrix Square Roots with Applications
to Gaussian Processes and Bayesian Optimization", NeurIPS 2020):

* ``kernels``    -- K = o^2 k(X, X) + sigma^2 I for RBF / Matern-5/2
                    (isotropic or ARD) and the product K V, dense or blocked.
* ``quadrature`` -- Hale-Higham-Trefethen shifts t_q and weights w_q
                    (Appendix B, Alg. S2) through SciPy's elliptic routines.
* ``lanczos``    -- extreme-eigenvalue estimate (Appendix B.2).
* ``msminres``   -- multi-shift MINRES (Appendix C, Alg. S4), written from
                    the Lanczos + Givens-QR derivation of Appendix C.1.
* ``ciq``        -- the CIQ composition (Sec. 3, Alg. S1) and the exact
                    eigendecomposition references.
* ``precond``    -- the pivoted-Cholesky preconditioned form (Sec. 3.4,
                    Appendix D): partial pivoted Cholesky, P^{-1} and P^{1/2}
                    of P = Lbar Lbar^T + sigma^2 I, preconditioned CIQ.
* ``posterior``  -- the Gaussian-process posterior covariance at a candidate
                    set (Sec. 5.2, Thompson sampling) and its product.
* ``svgp``       -- the CIQ-whitened SVGP predictive distribution in natural
                    parameters (Sec. 5.1, App. E).
* ``adjoint``    -- the backward pass (Sec. 3.3) plus two independent
                    references: central finite differences and the
                    Daleckii-Krein divided-difference formula.

Every function is FP64 numpy / scipy; there is no blocking, fusion or
reordering beyond what the definitions need. Its correctness is pinned in
``tests/test_oracle_*.py`` against closed forms, library routines, brute
force and the paper's stated bounds. Parity status of every function: pinned.
"""
