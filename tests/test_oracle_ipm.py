"""Pins of the oracle interior-point method (Algorithm 1 with a filter line
search) against facts that do not come from its own code path:

* first-order optimality of the returned point, checked with the model's
  functions and Lagrangian gradient (both pinned elsewhere by finite
  differences): primal feasibility, bounds, complementarity, stationarity;
* the optimal objective agrees with SciPy's trust-region constrained solver
  (an unrelated method) on small networks.
"""
import numpy as np
import pytest
from scipy.optimize import minimize, NonlinearConstraint, Bounds

import synthnet
from oracle.model import Model
from oracle.ipm import LinRedIPM, flat_start, IPMOptions

NETS = [synthnet.case9(1), synthnet.case9(3), synthnet.small(5, 7, 2, seed=1)]


@pytest.mark.parametrize("net", NETS, ids=lambda n: f"{n.name}-{n.seed}")
def test_ipm_returns_a_kkt_point(net):
    ipm = LinRedIPM(net, IPMOptions(tol=1e-8))
    x0, u0 = flat_start(ipm.M)
    st, log, ok = ipm.solve(x0, u0)
    assert ok and len(log) < 60
    M = Model(net)                       # unscaled model, independent evaluation
    x, u = st.w[M.nu:], st.w[:M.nu]
    g, h, f = M.functions(x, u)
    hl, hu = M.h_bounds()
    xl, xu, ul, uu = M.var_bounds()
    assert np.abs(g).max() <= 1e-8
    assert np.all(h <= hu + 1e-8) and np.all(h >= hl - 1e-8)
    w = st.w
    wl, wu = np.concatenate([ul, xl]), np.concatenate([uu, xu])
    assert np.all(w <= wu + 1e-12) and np.all(w >= wl - 1e-12)
    # stationarity of the scaled Lagrangian with the returned multipliers
    sig = ipm.sigma_f
    _, _, gf = M.jacobians(x, u)
    G, A, _ = M.jacobians(x, u)
    r = sig * gf + G.T @ st.lam + A.T @ st.y - st.zl + st.zu
    assert np.abs(r).max() <= 1e-6 * max(1.0, np.abs(sig * gf).max())
    assert np.abs(st.y - st.zsl + st.zsu).max() <= 1e-6
    # complementarity near zero (mu ends at tol / 10)
    fin = np.isfinite(wl)
    assert np.abs((w - wl)[fin] * st.zl[fin]).max() <= 1e-7


@pytest.mark.parametrize("net", [synthnet.case9(3), synthnet.small(5, 7, 2, seed=1)],
                         ids=lambda n: f"{n.name}-{n.seed}")
def test_ipm_objective_matches_scipy(net):
    ipm = LinRedIPM(net, IPMOptions(tol=1e-8))
    x0, u0 = flat_start(ipm.M)
    st, log, ok = ipm.solve(x0, u0)
    assert ok
    M = Model(net)
    nu = M.nu
    xl, xu, ul, uu = M.var_bounds()
    hl, hu = M.h_bounds()
    sc = 1e-3

    def fun(w):
        return sc * float(np.real(M.functions(w[nu:], w[:nu])[2]))

    def jac(w):
        return sc * M.jacobians(w[nu:], w[:nu])[2]

    eq = NonlinearConstraint(lambda w: np.real(M.functions(w[nu:], w[:nu])[0]), 0.0, 0.0,
                             jac=lambda w: M.jacobians(w[nu:], w[:nu])[0].toarray())
    ineq = NonlinearConstraint(lambda w: np.real(M.functions(w[nu:], w[:nu])[1]), hl, hu,
                               jac=lambda w: M.jacobians(w[nu:], w[:nu])[1].toarray())
    w0 = st.w + 1e-3 * np.random.default_rng(0).normal(size=st.w.shape)
    w0 = np.clip(w0, np.concatenate([ul, xl]), np.concatenate([uu, xu]))
    res = minimize(fun, w0, jac=jac, method="trust-constr", constraints=[eq, ineq],
                   bounds=Bounds(np.concatenate([ul, xl]), np.concatenate([uu, xu])),
                   options={"gtol": 1e-10, "xtol": 1e-12, "maxiter": 3000})
    f_ipm = log[-1]["obj"]
    assert abs(res.fun / sc - f_ipm) <= 1e-5 * abs(f_ipm), (res.fun / sc, f_ipm, res.message)


@pytest.mark.parametrize("net", [synthnet.case9(3), synthnet.small(5, 7, 2, seed=1)],
                         ids=lambda n: f"{n.name}-{n.seed}")
def test_sparse_linear_solver_takes_the_same_iterations(net):
    """The oracle IPM with the sparse-LU solve of K_aug (its option for large
    networks) takes the dense solve's iterations: same count, barrier
    parameters, trials and inertia shifts, objectives within rounding."""
    runs = []
    for solver in ("dense", "sparse"):
        ipm = LinRedIPM(net, IPMOptions(tol=1e-8, linear_solver=solver))
        st, log, ok = ipm.solve(*flat_start(ipm.M))
        assert ok
        runs.append(log)
    a, b = runs
    assert len(a) == len(b)
    for p, q in zip(a, b):
        assert p["mu"] == q["mu"] and p["trials"] == q["trials"]
        assert (p["delta_w"] == 0.0) == (q["delta_w"] == 0.0)
        assert abs(p["obj"] - q["obj"]) <= 1e-9 * abs(q["obj"])
