"""CPU FP64 oracle for the condensed interior-point method (test infrastructure).

This package is test infrastructure. Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import, call or execute it; the product
path (the HIP library and its Python binding) never does.

It computes, slowly and plainly, what the GPU path computes:

* ``model``      polar AC optimal power flow: g, h, f and their dense/sparse
                 analytic derivatives G, A, grad f, W (state/control split of
                 the paper's state-control form, Section 2.1).
* ``reduction``  the sensitivity S = -G_x^{-1} G_u, the condensed matrix
                 K_cond = [I; S]^T K [I; S] (Theorems 1-2 and the batched
                 reduction identity of Section 3.3), the condensed right-hand
                 side and the step recovery, and the augmented system K_aug for
                 brute-force checks.
* ``cholesky``   inertia-corrected dense Cholesky of K_cond (Section 4.3 and
                 the inertia theorem of Section 2.2.1).
* ``powerflow``  Newton-Raphson solution of g(x, u) = 0 (implicit function
                 theorem, Section 2.3.1) used to pin S and K_cond by finite
                 differences.

Everything is float64. No code is shared with the GPU path.
"""
