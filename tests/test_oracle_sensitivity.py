"""Pins of the oracle's implicit differentiation of the OPF solution with
respect to the loads (oracle.sensitivity):

* the load Jacobian dF/dp equals central differences of the barrier
  residual rebuilt from networks with perturbed loads (F is at most
  quadratic in the loads, so the differences are exact up to rounding);
* the sensitivity -C K_aug^{-1} dF/dp equals central differences of the
  barrier solution itself, re-solved by Newton's method at fixed mu for loads
  p +- h e_i, at barrier parameters where differences are accurate (the
  identity does not depend on mu);
* the envelope theorem: the objective's gradient at the optimum equals the
  partial derivative of the Lagrangian in the loads, i.e. the balance
  multipliers (plus the y terms of Pg_ref and Qg at generator buses), up to
  O(mu);
* the gradient at the IPM's own final iterate (primal-dual Sigma) agrees with
  the exact barrier solution's.
"""
import numpy as np
import pytest

import synthnet
from oracle.ipm import LinRedIPM, IPMOptions, flat_start
from oracle import sensitivity as S

NETS = {
    # seed 5: the plain Newton re-solve of the barrier problem (no line search)
    # converges from the optimum to the rounding floor at mu = 1e-3 .. 1e-5;
    # on seed 1 it stalls near 1e-6 at mu = 1e-4
    "syn9-5": lambda: synthnet.case9(5),
    "syn5": lambda: synthnet.small(5, 7, 2, seed=1),
}

_SOLVED = {}


def solved(name, tol=1e-8):
    """The oracle IPM run to tol on a named network (cached)."""
    key = (name, tol)
    if key not in _SOLVED:
        ipm = LinRedIPM(NETS[name](), IPMOptions(tol=tol))
        x0, u0 = flat_start(ipm.M)
        st, _, ok = ipm.solve(x0, u0)
        assert ok
        _SOLVED[key] = (ipm, st)
    return _SOLVED[key]


def barrier_point(name, mu, floor=1e-8):
    """The barrier solution at mu, by Newton from the IPM's optimum (the
    residual floor grows as mu shrinks: rounding in the bound slacks)."""
    ipm, st = solved(name)
    w, s, lam, y, nrm = S.solve_barrier(ipm, st.w, st.s, st.lam, st.y, mu)
    assert nrm <= floor, nrm
    return ipm, (w, s, lam, y)


def _row_close(a, b, rel):
    """Each row of a equals the same row of b within rel of the row's max."""
    scale = np.maximum(np.abs(b).max(axis=1, keepdims=True), 1e-12)
    err = np.abs(a - b) / scale
    assert err.max() <= rel, (err.max(), np.unravel_index(err.argmax(), err.shape))


@pytest.mark.parametrize("name", list(NETS))
def test_barrier_newton_reaches_rounding_level(name):
    ipm, st = solved(name)
    w, s, lam, y, nrm = S.solve_barrier(ipm, st.w, st.s, st.lam, st.y, 1e-4)
    F0 = np.abs(S.barrier_residual(ipm, st.w, st.s, st.lam, st.y, 1e-4)).max()
    assert F0 > 1e-6          # the optimum is not the mu = 1e-4 barrier solution
    assert nrm <= 1e-11


@pytest.mark.parametrize("name", list(NETS))
def test_load_jacobian_matches_residual_differences(name):
    ipm, (w, s, lam, y) = barrier_point(name, 1e-4)
    net = ipm.net
    Fp = S.load_jacobian(ipm, w, s)
    h = 1e-3
    fd = np.zeros_like(Fp)
    for j in range(2 * net.nb):
        cols = []
        for sign in (1.0, -1.0):
            pd, qd = net.pd.copy(), net.qd.copy()
            (pd if j < net.nb else qd)[j % net.nb] += sign * h
            other = S.with_loads(ipm, pd, qd)
            cols.append(S.barrier_residual(other, w, s, lam, y, 1e-4))
        fd[:, j] = (cols[0] - cols[1]) / (2 * h)
    assert np.abs(fd - Fp).max() <= 1e-7 * max(1.0, np.abs(Fp).max())
    # every load reaches F somewhere
    assert (np.abs(Fp).sum(axis=0) > 0).all()


@pytest.mark.parametrize("name", list(NETS))
@pytest.mark.parametrize("mu", [1e-3, 1e-5])
def test_sensitivity_matches_differences_of_barrier_solution(name, mu):
    ipm, (w, s, lam, y) = barrier_point(name, mu)
    net = ipm.net
    sw, ss = S.barrier_sigmas(ipm, w, s, mu)
    J = S.output_sensitivity(ipm, w, s, lam, y, sw, ss)
    # the re-solves stop at a residual floor set by rounding in the bound
    # slacks (~1e-9 at these mu), so the difference error is ~ h^2 + floor / h
    h = 1e-5
    fd = np.zeros_like(J)
    for j in range(2 * net.nb):
        outs = []
        for sign in (1.0, -1.0):
            pd, qd = net.pd.copy(), net.qd.copy()
            (pd if j < net.nb else qd)[j % net.nb] += sign * h
            other = S.with_loads(ipm, pd, qd)
            wp, sp_, _, _, nrm = S.solve_barrier(other, w, s, lam, y, mu)
            assert nrm <= 1e-8
            pg, vm, f = S.outputs(other, wp, sp_)
            outs.append(np.concatenate([pg, vm, [f]]))
        fd[:, j] = (outs[0] - outs[1]) / (2 * h)
    _row_close(J, fd, 5e-6)
    assert np.abs(J).max() > 1.0


@pytest.mark.parametrize("name", list(NETS))
def test_objective_gradient_is_envelope(name):
    """df*/dPd_i = (lambda_P(i) + [i = ref] (y_0 + sigma df/dPg_ref)) / sigma,
    df*/dQd_i = (lambda_Q(i) + y_{1+g(i)}) / sigma at the optimum (mu -> 0)."""
    ipm, st = solved(name)
    M, net = ipm.M, ipm.net
    sw, ss = S.primal_dual_sigmas(ipm, st)
    gpd, gqd, _ = S.load_gradient(ipm, st.w, st.s, st.lam, st.y, sw, ss,
                                  np.zeros(M.ng), np.zeros(M.nb), 1.0)
    sig = ipm.sigma_f
    pg, _, _ = S.outputs(ipm, st.w, st.s)
    B = M.base
    epd = np.zeros(M.nb)
    eqd = np.zeros(M.nb)
    for k, i in enumerate(M.g_rows_p):
        epd[i] += st.lam[k]
    for k, i in enumerate(M.g_rows_q):
        eqd[i] += st.lam[len(M.g_rows_p) + k]
    rg = M.ref_gen
    epd[M.ref] += st.y[0] + sig * B * (2.0 * net.c2[rg] * B * pg[rg] + net.c1[rg])
    for g in range(M.ng):
        eqd[net.gen_bus[g]] += st.y[1 + g]
    epd /= sig
    eqd /= sig
    scale = np.abs(np.concatenate([epd, eqd])).max()
    assert scale > 100.0
    assert np.abs(gpd - epd).max() <= 1e-6 * scale
    assert np.abs(gqd - eqd).max() <= 1e-6 * scale


@pytest.mark.parametrize("name", list(NETS))
def test_primal_dual_sigma_matches_barrier_solution(name):
    ipm, st = solved(name)
    M = ipm.M
    rng = np.random.default_rng(5)
    dpg, dvm, df = rng.standard_normal(M.ng), rng.standard_normal(M.nb), 1e-3
    sw, ss = S.primal_dual_sigmas(ipm, st)
    a = S.load_gradient(ipm, st.w, st.s, st.lam, st.y, sw, ss, dpg, dvm, df)
    _, (w, s, lam, y) = barrier_point(name, st.mu, floor=1e-7)
    bw, bs = S.barrier_sigmas(ipm, w, s, st.mu)
    b = S.load_gradient(ipm, w, s, lam, y, bw, bs, dpg, dvm, df)
    scale = max(np.abs(b[0]).max(), np.abs(b[1]).max())
    assert np.abs(a[0] - b[0]).max() <= 1e-5 * scale
    assert np.abs(a[1] - b[1]).max() <= 1e-5 * scale


def test_gradient_is_adjoint_of_full_sensitivity():
    """The adjoint form equals the weights applied to the full Jacobian."""
    ipm, (w, s, lam, y) = barrier_point("syn9-5", 1e-5)
    M = ipm.M
    sw, ss = S.barrier_sigmas(ipm, w, s, 1e-5)
    J = S.output_sensitivity(ipm, w, s, lam, y, sw, ss)
    rng = np.random.default_rng(3)
    wt = rng.standard_normal(M.ng + M.nb + 1)
    gpd, gqd, _ = S.load_gradient(ipm, w, s, lam, y, sw, ss, wt[:M.ng], wt[M.ng:-1], wt[-1])
    ref = wt @ J
    np.testing.assert_allclose(np.concatenate([gpd, gqd]), ref, rtol=0,
                               atol=1e-10 * np.abs(ref).max())


def test_sparse_gradient_equals_dense():
    """load_gradient's sparse-LU solve (used for the 1354-bus reference) equals
    the dense solve."""
    ipm, st = solved("syn9-5")
    sw, ss = S.primal_dual_sigmas(ipm, st)
    rng = np.random.default_rng(3)
    args = (rng.standard_normal(ipm.net.ng), rng.standard_normal(ipm.net.nb), 1e-3)
    a = S.load_gradient(ipm, st.w, st.s, st.lam, st.y, sw, ss, *args)
    b = S.load_gradient(ipm, st.w, st.s, st.lam, st.y, sw, ss, *args, sparse=True)
    for p, q in zip(a, b):
        assert np.abs(p - q).max() <= 1e-9 * np.abs(p).max()
