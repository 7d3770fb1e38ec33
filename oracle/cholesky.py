"""Oracle: inertia-corrected Cholesky of K_cond (test infrastructure).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this.

Section 4.3: each iteration factorises K_cond with a dense Cholesky; if the
factorisation fails, a primal-dual regularisation is added until K_cond is
positive definite. By the inertia theorem (Section 2.2.1) Cholesky success is
exactly the inertia test of K_aug. The paper gives no constants; the reading
here is the published Ipopt rule that MadNLP follows: try delta = 0; else
delta = 1e-4 the first time (max(1e-20, delta_last / 3) later); multiply by 100
(first time) or 8 until the factorisation succeeds; give up above 1e40.
"""
from __future__ import annotations

import numpy as np


def try_cholesky(M):
    """Lower Cholesky factor of the lower triangle of M, or None."""
    try:
        return np.linalg.cholesky(np.tril(M) + np.tril(M, -1).T)
    except np.linalg.LinAlgError:
        return None


def factor_with_correction(Kc, delta_last=0.0, delta_max=1e40):
    """Returns (L, delta_w). L is None when no delta <= delta_max works."""
    L = try_cholesky(Kc)
    if L is not None:
        return L, 0.0
    n = Kc.shape[0]
    first = delta_last == 0.0
    delta = 1e-4 if first else max(1e-20, delta_last / 3.0)
    grow = 100.0 if first else 8.0
    while delta <= delta_max:
        L = try_cholesky(Kc + delta * np.eye(n))
        if L is not None:
            return L, delta
        delta *= grow
    return None, delta


def solve_with_factor(L, b):
    """x with L L^T x = b (plain triangular solves)."""
    import scipy.linalg as sla
    z = sla.solve_triangular(L, b, lower=True)
    return sla.solve_triangular(L.T, z, lower=False)
