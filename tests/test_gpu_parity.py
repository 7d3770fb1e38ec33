"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances: g, h, f 1e-12 relative; K_cond entry by entry, each entry (i, j)
within 1e-8 of sqrt(|K_ii K_jj|) (the accuracy target of the method's FP64
condensation, applied to every entry, so a wrong weak row or column fails),
and in the Frobenius norm; the condensed right-hand side 1e-8 of its largest
entry; every block of the step (p_u, p_x, p_s, p_lambda, p_y) within 1e-8 of
that block's own largest entry; the Cholesky factor row by row, each entry of
row i within 1e-8 of sqrt(K_ii) (which bounds every entry of that row of L).
At the interior-point method's own iterates, where K_cond is ill-conditioned,
the step is checked by its backward error in the oracle's augmented system.
The GPU path sums in a fixed order, so repeated calls and different panel
widths must agree bitwise."""
import os

import numpy as np
import pytest

import synthnet
from oracle.model import Model
from oracle import reduction as R, cholesky as OC
from helpers import (random_point, residual_vector, kcond_entry_error, step_block_errors)

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _net_api():
    from paper_2203_11875_amd import api
    return api


NETS = {
    "syn9": lambda: synthnet.case9(1),
    "syn5": lambda: synthnet.small(5, 7, 2, seed=1),
    "syn118": lambda: synthnet.case118(0),
    "syn300": lambda: synthnet.case300(0),
    "syn1354": lambda: synthnet.case1354(0),
    # 400 generators: nu = 799, 25 blocks of 32, between the one-pass (<= 544)
    # and the 9241-bus sizes of the backward substitution
    "syn1354g400": lambda: synthnet.make_network(1354, 1991, 400, seed=0, load_frac=0.6,
                                                 name="syn1354g400"),
}


def _t(a):
    return torch.as_tensor(np.asarray(a, np.float64), device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _linf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _factor_row_error(Lg, Kd):
    """Entries of row i of the Cholesky factor against sqrt(K_ii): the row's
    squares sum to K_ii, so that bounds every entry of the row."""
    Lo = np.linalg.cholesky(Kd)
    d = np.sqrt(np.abs(np.diag(Kd)))
    return float((np.abs(Lg - Lo) / d[:, None]).max())


def _check_step(got, want, nu, nx, m, tol=1e-8):
    errs = step_block_errors(got, want, nu, nx, m)
    for name, e in errs.items():
        assert e <= tol, (name, errs)
    return errs


@pytest.mark.parametrize("name", list(NETS))
def test_eval_residual(name):
    net = NETS[name]()
    M = Model(net)
    G = _net_api().Net(net)
    x, u, *_ = random_point(M, 0)
    g, h, f = G.eval_residual(_t(x), _t(u))
    torch.cuda.synchronize()
    go, ho, fo = M.functions(x, u)
    assert _rel(_np(g), go) <= 1e-12
    assert _rel(_np(h), ho) <= 1e-12
    assert abs(_np(f)[0] - fo) <= 1e-12 * abs(fo)


@pytest.mark.parametrize("name", list(NETS))
@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("refactor", [0, 1], ids=["wave", "staged"])
def test_condense_matches_oracle(name, seed, refactor):
    net = NETS[name]()
    M = Model(net)
    G = _net_api().Net(net, refactor=refactor)
    assert G.info["refactor_kernel"] == refactor
    x, u, lam, y, sx, su, ss = random_point(M, seed)
    r = residual_vector(M, seed)
    K, rhs = G.condense_reduced_hessian(*map(_t, (x, u, lam, y, sx, su, ss)), r=_t(r))
    torch.cuda.synchronize()
    B = R.kkt_blocks(M, x, u, lam, y, sx, su, ss)
    S, lu = R.sensitivity(B)
    Kc = R.symmetrize(R.condensed_matrix(B, S))
    b, _, _ = R.condensed_rhs(B, r, S, lu)
    Kg = _np(K).T          # column-major nu x nu
    assert kcond_entry_error(Kg, Kc) <= 1e-8, kcond_entry_error(Kg, Kc)
    assert _rel(Kg, Kc) <= 1e-8, _rel(Kg, Kc)
    assert np.array_equal(Kg, Kg.T)
    assert _linf(_np(rhs), b) <= 1e-8


@pytest.mark.parametrize("name,ordering", [("syn118", 1), ("syn118", 2), ("syn1354", 1)])
def test_condense_matches_oracle_under_other_orderings(name, ordering):
    """K_cond and the right-hand side entry by entry with G_x ordered by plain
    minimum degree or nested dissection instead of the default."""
    net = NETS[name]()
    M = Model(net)
    G = _net_api().Net(net, ordering=ordering)
    x, u, lam, y, sx, su, ss = random_point(M, 2)
    r = residual_vector(M, 2)
    K, rhs = G.condense_reduced_hessian(*map(_t, (x, u, lam, y, sx, su, ss)), r=_t(r))
    torch.cuda.synchronize()
    B = R.kkt_blocks(M, x, u, lam, y, sx, su, ss)
    S, lu = R.sensitivity(B)
    Kc = R.symmetrize(R.condensed_matrix(B, S))
    b, _, _ = R.condensed_rhs(B, r, S, lu)
    Kg = _np(K).T
    assert kcond_entry_error(Kg, Kc) <= 1e-8, kcond_entry_error(Kg, Kc)
    assert _linf(_np(rhs), b) <= 1e-8


@pytest.mark.parametrize("name", ["syn9", "syn118", "syn1354", "syn1354g400"])
@pytest.mark.parametrize("delta", [0.0, 10.0])
def test_solve_matches_oracle(name, delta):
    net = NETS[name]()
    M = Model(net)
    G = _net_api().Net(net)
    x, u, lam, y, sx, su, ss = random_point(M, 3, lam_scale=1.0, sig_range=(1.0, 1e3))
    r = residual_vector(M, 4)
    K, rhs = G.condense_reduced_hessian(*map(_t, (x, u, lam, y, sx, su, ss)), r=_t(r))
    B = R.kkt_blocks(M, x, u, lam, y, sx, su, ss)
    S, lu = R.sensitivity(B)
    Kc = R.symmetrize(R.condensed_matrix(B, S))
    # shift so that K_cond + delta I is positive definite (inertia correction)
    delta += max(0.0, -np.linalg.eigvalsh(Kc).min()) * 1.5
    Kc = Kc + delta * np.eye(M.nu)
    assert OC.try_cholesky(Kc) is not None
    b, _, _ = R.condensed_rhs(B, r, S, lu)
    p, code = G.solve_condensed_kkt(K, delta, rhs, _t(r))
    torch.cuda.synchronize()
    assert code == 0
    pu = np.linalg.solve(Kc, b)
    want = np.concatenate(R.recover(B, r, pu, S, lu))
    _check_step(_np(p), want, M.nu, M.nx, M.m)
    # the lower triangle of K now holds the Cholesky factor of K_cond + delta I
    Lg = np.tril(_np(K).T)
    assert _factor_row_error(Lg, Kc) <= 1e-8
    assert _rel(Lg, np.linalg.cholesky(Kc)) <= 1e-8


def test_cholesky_reports_indefinite():
    net = synthnet.case118(0)
    M = Model(net)
    G = _net_api().Net(net)
    for seed in range(6):
        x, u, lam, y, sx, su, ss = random_point(M, seed, lam_scale=400.0)
        B = R.kkt_blocks(M, x, u, lam, y, sx, su, ss)
        if OC.try_cholesky(R.symmetrize(R.condensed_matrix(B))) is None:
            break
    else:
        pytest.skip("no indefinite draw")
    r = residual_vector(M, 0)
    K, rhs = G.condense_reduced_hessian(*map(_t, (x, u, lam, y, sx, su, ss)), r=_t(r))
    _, code = G.solve_condensed_kkt(K, 0.0, rhs, _t(r))
    assert code == 1   # RH_NOT_POSDEF


def test_failed_solve_leaves_no_trace():
    """The factorisation's first launch clears the status word and reads the
    right-hand side: after a solve that meets a non-positive pivot, a solve
    with an inertia shift on the same handle succeeds, leaves the right-hand
    side as it was and equals the same solve on a fresh handle bit for bit."""
    net = synthnet.case118(0)
    M = Model(net)
    api = _net_api()
    for seed in range(6):
        x, u, lam, y, sx, su, ss = random_point(M, seed, lam_scale=400.0)
        Kc = R.symmetrize(R.condensed_matrix(R.kkt_blocks(M, x, u, lam, y, sx, su, ss)))
        if OC.try_cholesky(Kc) is None:
            break
    else:
        pytest.skip("no indefinite draw")
    delta = 1.5 * max(0.0, -np.linalg.eigvalsh(Kc).min()) + 1e-3
    r = residual_vector(M, 0)
    args = list(map(_t, (x, u, lam, y, sx, su, ss)))
    G = api.Net(net)
    K, rhs = G.condense_reduced_hessian(*args, r=_t(r))
    K0, rhs0 = K.clone(), rhs.clone()
    _, code = G.solve_condensed_kkt(K, 0.0, rhs, _t(r))
    assert code == 1   # RH_NOT_POSDEF
    K.copy_(K0)
    p, code = G.solve_condensed_kkt(K, delta, rhs, _t(r))
    assert code == 0
    assert torch.equal(rhs, rhs0)
    H = api.Net(net)
    K2, rhs2 = H.condense_reduced_hessian(*args, r=_t(r))
    p2, code2 = H.solve_condensed_kkt(K2, delta, rhs2, _t(r))
    torch.cuda.synchronize()
    assert code2 == 0
    assert torch.equal(p, p2)


@pytest.mark.parametrize("name", ["syn118", "syn1354"])
def test_bitwise_repeatable_and_width_independent(name):
    net = NETS[name]()
    M = Model(net)
    x, u, lam, y, sx, su, ss = random_point(M, 5)
    args = list(map(_t, (x, u, lam, y, sx, su, ss)))
    outs = []
    # (panel width, panels in LDS, waves per work-group, sweeps on all waves:
    # 0 the library's choice, else 1 + a mask over L, U, U^T, L^T)
    # (lds 2: the step metadata read from global memory, as for a panel that
    # fills the LDS)
    for width, lds, nw, grp in ((1, 1, 1, 0), (1, 1, 4, 1), (1, 1, 4, 16), (1, 1, 4, 1 + 5),
                                (1, 1, 8, 1), (1, 1, 8, 16), (1, 1, 2, 1), (1, 2, 2, 1),
                                (1, 2, 8, 16), (1, 2, 1, 0), (2, 1, 1, 0), (2, 1, 1, 0),
                                (3, 1, 1, 0), (2, 0, 1, 0), (4, 0, 1, 0)):
        G = _net_api().Net(net, panel_width=width, lds_panel=lds, cond_waves=nw,
                           sweep_grouping=grp)
        assert G.info["cond_waves"] == nw
        assert G.info["lds_panel"] == lds
        if nw > 1:
            assert G.info["sweep_grouped"] == grp - 1
        K, _ = G.condense_reduced_hessian(*args)
        torch.cuda.synchronize()
        outs.append((width, lds, nw, grp, G.info["lds_panel"], _np(K).copy()))
        G.close()
    for w, l, nw, grp, used, K in outs[1:]:
        assert np.array_equal(K, outs[0][5]), (w, l, nw, grp, used)


def test_set_loads_changes_residual():
    net = synthnet.case118(0)
    M = Model(net)
    G = _net_api().Net(net)
    x, u, *_ = random_point(M, 0)
    net2 = synthnet.scale_loads(net, 3)
    G.set_loads(_t(net2.pd), _t(net2.qd))
    g, h, f = G.eval_residual(_t(x), _t(u))
    torch.cuda.synchronize()
    go, ho, fo = Model(net2).functions(x, u)
    assert _rel(_np(g), go) <= 1e-12 and _rel(_np(h), ho) <= 1e-12


@pytest.mark.parametrize("name,width,nw,grp", [
    ("syn9", 1, 1, 0), ("syn1354", 1, 1, 0), ("syn1354", 1, 2, 0), ("syn1354", 1, 4, 0),
    ("syn1354", 1, 4, 16), ("syn1354", 1, 8, 0), ("syn1354", 1, 8, 16), ("syn118", 2, 1, 0),
    ("syn1354", 3, 1, 0)])
def test_solve_after_condensation_without_rhs(name, width, nw, grp):
    """Recovery by the single-column pass (condensation called without r),
    with the right-hand side condensed separately on the same factors; the
    pass reads the sweep records of the handle's panel width and runs the
    handle's waves per work-group."""
    net = NETS[name]()
    M = Model(net)
    G = _net_api().Net(net, panel_width=width, cond_waves=nw, sweep_grouping=grp)
    assert G.info["panel_width"] == width and G.info["cond_waves"] == nw
    x, u, lam, y, sx, su, ss = random_point(M, 3, lam_scale=1.0, sig_range=(10.0, 1e4))
    r = residual_vector(M, 4)
    args = list(map(_t, (x, u, lam, y, sx, su, ss)))
    _, rhs = G.condense_reduced_hessian(*args, r=_t(r))       # right-hand side only
    K, _ = G.condense_reduced_hessian(*args)                   # no stored RHS column
    B = R.kkt_blocks(M, x, u, lam, y, sx, su, ss)
    S, lu = R.sensitivity(B)
    Kc = R.symmetrize(R.condensed_matrix(B, S))
    delta = max(0.0, -np.linalg.eigvalsh(Kc).min()) * 1.5
    p, code = G.solve_condensed_kkt(K, delta, rhs, _t(r))
    torch.cuda.synchronize()
    assert code == 0
    b, _, _ = R.condensed_rhs(B, r, S, lu)
    pu = np.linalg.solve(Kc + delta * np.eye(M.nu), b)
    want = np.concatenate(R.recover(B, r, pu, S, lu))
    _check_step(_np(p), want, M.nu, M.nx, M.m)


def test_solve_9241_matches_oracle():
    """The 9241-bus network (nx 17036, nu 2889) in the launch shape the
    library picks: every entry of K_cond and the right-hand side against the
    oracle's sparse-LU columns, then the blocked Cholesky of the
    2889 x 2889 K_cond + delta I (the wide backward-substitution variant) and
    every block of the recovered step against the oracle's dense solve of
    its K_cond and its sparse-LU recovery."""
    net = synthnet.case9241(0)
    M = Model(net)
    print("solve syn9241", flush=True)
    G = _net_api().Net(net)
    x, u, lam, y, sx, su, ss = random_point(M, 3, lam_scale=1.0, sig_range=(1.0, 1e3))
    r = residual_vector(M, 4)
    K, rhs = G.condense_reduced_hessian(*map(_t, (x, u, lam, y, sx, su, ss)), r=_t(r))
    Kg = _np(K).T.copy()
    B = R.kkt_blocks(M, x, u, lam, y, sx, su, ss)
    Kc, splu = R.condensed_columns_sparse(B, range(M.nu))
    Kc = R.symmetrize(Kc)
    print(f"syn9241 K_cond entry error {kcond_entry_error(Kg, Kc):.2e}", flush=True)
    assert kcond_entry_error(Kg, Kc) <= 1e-8
    assert np.array_equal(Kg, Kg.T)
    b, _ = R.condensed_rhs_sparse(B, r, splu)
    assert _linf(_np(rhs), b) <= 1e-8
    delta = 1.0           # then x10 until K_cond + delta I has a Cholesky factor
    while OC.try_cholesky(Kc + delta * np.eye(M.nu)) is None:
        delta *= 10.0
    Kd = Kc + delta * np.eye(M.nu)
    p, code = G.solve_condensed_kkt(K, delta, rhs, _t(r))
    torch.cuda.synchronize()
    assert code == 0
    pu = np.linalg.solve(Kd, b)
    want = np.concatenate(R.recover_sparse(B, r, pu, splu))
    errs = _check_step(_np(p), want, M.nu, M.nx, M.m)
    print(f"syn9241 step block errors {errs}", flush=True)
    Lg = np.tril(_np(K).T)
    assert _factor_row_error(Lg, Kd) <= 1e-8


@pytest.mark.parametrize("tag", ["it0", "it10", "last"])
def test_condense_and_solve_at_ipm_iterates_1354(tag):
    """K_cond, the right-hand side and the step at the oracle interior-point
    method's own iterates on the 1354-bus network (iterations 0, 10 and the
    last one of a run to 1e-6, where Sigma spans many decades and K_cond is
    ill-conditioned), with the objective scale and the inertia shift the
    method used there. K_cond and the right-hand side entry by entry; the
    step by its backward error in the oracle's augmented system (a stable
    solve of an ill-conditioned system is only accurate in that sense), and
    by its forward error relative to the condition number."""
    z = np.load(os.path.join(GOLD, "iterates_syn1354.npz"))
    net = synthnet.case1354(0)
    sig = float(z[f"{tag}_obj_scale"])
    Ms = Model(net.copy(c2=net.c2 * sig, c1=net.c1 * sig, c0=net.c0 * sig))
    api = _net_api()
    G = api.Net(net)
    assert api.lib().rh_set_objective_scale(G.h, sig) == 0
    args = [z[f"{tag}_{k}"] for k in ("x", "u", "lam", "y", "sig_x", "sig_u", "sig_s")]
    r = z[f"{tag}_r"]
    delta = float(z[f"{tag}_delta_w"])
    print(f"syn1354 iterate {tag}: delta_w {delta:g}", flush=True)
    K, rhs = G.condense_reduced_hessian(*map(_t, args), r=_t(r))
    Kg = _np(K).T.copy()
    B = R.kkt_blocks(Ms, *args)
    S, lu = R.sensitivity(B)
    Kc = R.symmetrize(R.condensed_matrix(B, S))
    err = kcond_entry_error(Kg, Kc)
    print(f"  K_cond entry error {err:.2e}, cond {np.linalg.cond(Kc + delta * np.eye(Ms.nu)):.2e}",
          flush=True)
    assert err <= 1e-8
    b, _, _ = R.condensed_rhs(B, r, S, lu)
    assert _linf(_np(rhs), b) <= 1e-8
    p, code = G.solve_condensed_kkt(K, delta, rhs, _t(r))
    torch.cuda.synchronize()
    assert code == 0
    got = _np(p)
    Kaug = R.augmented_matrix_sparse(B, delta)
    res = np.abs(Kaug @ got + r).max()
    scale = np.abs(Kaug).max() * np.abs(got).max() + np.abs(r).max()
    print(f"  step backward error {res / scale:.2e}", flush=True)
    assert res <= 1e-12 * scale
    Kd = Kc + delta * np.eye(Ms.nu)
    want = np.concatenate(R.recover(B, r, np.linalg.solve(Kd, b), S, lu))
    errs = step_block_errors(got, want, Ms.nu, Ms.nx, Ms.m)
    print(f"  step block errors {errs}", flush=True)
    kappa = np.linalg.cond(Kd)
    for name, e in errs.items():
        assert e <= max(1e-8, 1e-14 * kappa), (name, e, kappa)
