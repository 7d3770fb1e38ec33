"""Pins of the RedLin oracle (Algorithm 2, oracle.redlin):

* the reduced derivatives (eq. reduced:derivatives) equal central differences
  through power-flow solves: grad f_r, A_hat = d h_r / du, and W_hat = the
  derivative of grad L_r at fixed y (the adjoint absorbs the second-order
  state terms);
* the reduced KKT step (dense solve) equals its condensed form (Theorem 2),
  and equals the full-space condensation of oracle.reduction with the state
  bounds' Sigma placed on the bounded states and r4 = 0 (the mapping the
  library's RedLin driver uses);
* RedLin reaches the LinRed optimum (the two methods solve the same problem;
  LinRed's optimum is pinned against SciPy), with g = 0 to the projection
  tolerance at every iterate, and its answer is a KKT point of the full-space
  problem with the multipliers it carries.
"""
import numpy as np
import pytest

import synthnet
from oracle.ipm import LinRedIPM, IPMOptions, flat_start
from oracle.redlin import RedLinIPM
from oracle import reduction as R

NETS = {
    "syn9-1": lambda: synthnet.case9(1),
    "syn9-3": lambda: synthnet.case9(3),
    "syn5": lambda: synthnet.small(5, 7, 2, seed=1),
}


def _midpoint(name, iters=3):
    """A RedLin iterate a few steps in (interior, nonzero multipliers)."""
    rl = RedLinIPM(NETS[name](), IPMOptions(tol=1e-8))
    st = rl.initial_state(*flat_start(rl.M))
    for _ in range(iters):
        rl.iterate(st)
    return rl, st


@pytest.mark.parametrize("name", list(NETS))
def test_reduced_derivatives_match_differences(name):
    rl, st = _midpoint(name)
    D = rl.derivatives(st.u, st.x, st.y)
    nu, h = rl.nu, 1e-6
    fd_gf = np.zeros(nu)
    fd_A = np.zeros((rl.mr, nu))
    fd_W = np.zeros((nu, nu))
    for j in range(nu):
        vals = []
        for sgn in (1.0, -1.0):
            u = st.u.copy()
            u[j] += sgn * h
            rl.pf_tol, tol0 = 1e-13, rl.pf_tol
            x, _ = rl.project(u, st.x)
            rl.pf_tol = tol0
            Dp = rl.derivatives(u, x, st.y)
            vals.append((rl.objective(u, x), rl.h_r(u, x), Dp["grad_lr"]))
        fd_gf[j] = (vals[0][0] - vals[1][0]) / (2 * h)
        fd_A[:, j] = (vals[0][1] - vals[1][1]) / (2 * h)
        fd_W[:, j] = (vals[0][2] - vals[1][2]) / (2 * h)
    sc = lambda a: max(1.0, np.abs(a).max())
    assert np.abs(fd_gf - D["grad_fr"]).max() <= 1e-6 * sc(D["grad_fr"])
    assert np.abs(fd_A - D["A_hat"]).max() <= 1e-6 * sc(D["A_hat"])
    assert np.abs(fd_W - D["W_hat"]).max() <= 1e-5 * sc(D["W_hat"])


@pytest.mark.parametrize("name", list(NETS))
def test_reduced_step_equals_condensed_forms(name):
    rl, st = _midpoint(name)
    D = rl.derivatives(st.u, st.x, st.y)
    sig_u, sig_s = rl.sigmas(st)
    mu = st.mu
    r_u, r_s, r_y = rl.residuals(st, D, mu)
    nu, m, mr = rl.nu, rl.m, rl.mr
    p = np.linalg.solve(rl.kkt_matrix(D, sig_u, sig_s), -np.concatenate([r_u, r_s, r_y]))
    pu = p[:nu]
    # Theorem 2 on the reduced system
    Kc = rl.condensed(D, sig_u, sig_s)
    b = -(r_u + D["A_hat"].T @ (sig_s * r_y - r_s))
    np.testing.assert_allclose(np.linalg.solve(Kc, b), pu, rtol=0, atol=1e-9 * np.abs(pu).max())
    # the full-space condensation with Sigma_x on the bounded states and r4 = 0
    sig_x = np.zeros(rl.nx)
    sig_x[rl.xb] = sig_s[m:]
    B = R.kkt_blocks(rl.M, st.x, st.u, D["lam"], st.y[:m], sig_x, sig_u, sig_s[:m])
    Kf = R.symmetrize(R.condensed_matrix(B))
    np.testing.assert_allclose(Kf, Kc, rtol=0, atol=1e-9 * np.abs(Kc).max())
    x_part = np.zeros(rl.nx)
    x_part[rl.xb] = -(sig_s[m:] * r_y[m:] - r_s[m:])
    r_full = np.concatenate([r_u, x_part, r_s[:m], np.zeros(rl.nx), r_y[:m]])
    bf, _, _ = R.condensed_rhs(B, r_full)
    np.testing.assert_allclose(bf, b, rtol=0, atol=1e-9 * np.abs(b).max())
    # and the recovered state step is S p_u (r4 = 0)
    _, px, ps, _, _ = R.recover(B, r_full, pu)
    np.testing.assert_allclose(px, D["S"] @ pu, rtol=0, atol=1e-9 * max(1.0, np.abs(px).max()))
    np.testing.assert_allclose(ps, p[nu:nu + m], rtol=0, atol=1e-8 * max(1.0, np.abs(ps).max()))


@pytest.mark.parametrize("name", list(NETS))
def test_redlin_reaches_linred_optimum(name):
    net = NETS[name]()
    rl = RedLinIPM(net, IPMOptions(tol=1e-8))
    st, log, ok = rl.solve(*flat_start(rl.M))
    assert ok
    lin = LinRedIPM(net, IPMOptions(tol=1e-8))
    st2, log2, ok2 = lin.solve(*flat_start(lin.M))
    assert ok2
    f1 = rl.objective(st.u, st.x) / rl.sigma_f
    f2 = lin.evaluate(st2.w, st2.s)[2] / lin.sigma_f
    assert abs(f1 - f2) <= 1e-8 * abs(f2)
    np.testing.assert_allclose(st.u, st2.w[:rl.nu], rtol=0, atol=1e-5)
    # every accepted iterate satisfies the state equation
    g, _, _ = rl.M.functions(st.x, st.u)
    assert np.abs(g).max() <= rl.pf_tol
    assert sum(e["pf_iters"] for e in log) >= len(log) // 2


@pytest.mark.parametrize("name", list(NETS))
def test_redlin_answer_is_full_space_kkt_point(name):
    net = NETS[name]()
    rl = RedLinIPM(net, IPMOptions(tol=1e-8))
    st, _, ok = rl.solve(*flat_start(rl.M))
    assert ok
    m, nu = rl.m, rl.nu
    G, A, gf = rl.M.jacobians(st.x, st.u)
    gl = gf + G.T @ st.lam + A.T @ st.y[:m]
    # full-space bound multipliers: controls' own, states' from their slacks
    zl = np.concatenate([st.zl, np.zeros(rl.nx)])
    zu = np.concatenate([st.zu, np.zeros(rl.nx)])
    zl[nu + rl.xb] = st.zsl[m:]
    zu[nu + rl.xb] = st.zsu[m:]
    scale = max(1.0, np.abs(gf).max())
    assert np.abs(gl - zl + zu).max() <= 1e-6 * scale
    _, h, _ = rl.M.functions(st.x, st.u)
    hl, hu = rl.M.h_bounds()
    assert np.all(h >= hl - 1e-7) and np.all(h <= hu + 1e-7)
    assert np.all(st.u >= rl.ul - 1e-12) and np.all(st.u <= rl.uu + 1e-12)


def test_projection_fails_cleanly():
    rl = RedLinIPM(synthnet.case9(1), IPMOptions())
    x0, u0 = flat_start(rl.M)
    u = u0.copy()
    u[rl.M.ng:] *= 60.0          # far more generation than any flow can carry
    x, k = rl.project(u, x0)
    assert x is None and k >= 1
