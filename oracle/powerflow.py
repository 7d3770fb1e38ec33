"""Oracle: Newton-Raphson power flow and reduced-space functions (test
infrastructure; only tests, the smoke check and the benchmark's CPU-baseline
leg use this).

Section 2.3.1: under the implicit function theorem, g(x(u), u) = 0 defines
x(u) locally, its derivative is S = -G_x^{-1} G_u, and the reduced functions
f_r(u) = f(x(u), u), h_r(u) = h(x(u), u) have the reduced derivatives of the
reduced-derivatives theorem. These helpers evaluate x(u) by Newton-Raphson
(tolerance far below the paper's 1e-10) so that finite differences through
them pin S and K_cond independently of the condensation code.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def solve_pf(model, u, x0, tol=1e-13, max_iter=30):
    """x with g(x, u) = 0, Newton-Raphson from x0."""
    x = np.array(x0, dtype=float)
    nu = model.nu
    for _ in range(max_iter):
        g, _, _ = model.functions(x, u)
        if np.max(np.abs(g)) < tol:
            return x
        G, _, _ = model.jacobians(x, u)
        x = x - spla.spsolve(G[:, nu:].tocsc(), g)
    g, _, _ = model.functions(x, u)
    if np.max(np.abs(g)) > 1e3 * tol:
        raise RuntimeError("power flow did not converge")
    return x


def reduced_values(model, u, x0, y):
    """x(u), f_r(u), h_r(u) and L_r(u) = f_r + y^T h_r."""
    x = solve_pf(model, u, x0)
    _, h, f = model.functions(x, u)
    return x, f, h, f + y @ h


def reduced_gradient(model, u, x0, y):
    """grad_u L_r with L_r = f + y^T h along x(u), by the adjoint
    lambda = -G_x^{-T} grad_x (f + y^T h) (reduced-derivatives theorem)."""
    nu = model.nu
    x = solve_pf(model, u, x0)
    G, A, gf = model.jacobians(x, u)
    gl = gf + A.T @ y
    lam = -spla.spsolve(G[:, nu:].T.tocsc(), gl[nu:])
    return gl[:nu] + G[:, :nu].T @ lam, x, lam
