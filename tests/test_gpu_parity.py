"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances: g, h, f 1e-12 relative; K_cond and the condensed right-hand side
1e-8 relative in the Frobenius / max norm (the accuracy target of the method's
FP64 condensation); the step 1e-8 relative to its largest entry. The GPU path
sums in a fixed order, so repeated calls and different panel widths must agree
bitwise."""
import numpy as np
import pytest

import synthnet
from oracle.model import Model
from oracle import reduction as R, cholesky as OC
from helpers import random_point, residual_vector

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
    "syn9": lambda: synthnet.case9(0),
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
    assert _rel(Kg, Kc) <= 1e-8, _rel(Kg, Kc)
    assert np.array_equal(Kg, Kg.T)
    assert _rel(_np(rhs), b) <= 1e-8


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
    got = _np(p)
    assert np.abs(got - want).max() <= 1e-8 * np.abs(want).max()
    # the lower triangle of K now holds the Cholesky factor of K_cond + delta I
    Lg = np.tril(_np(K).T)
    Lo = np.linalg.cholesky(Kc)
    assert _rel(Lg, Lo) <= 1e-8


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


@pytest.mark.parametrize("name", ["syn118", "syn1354"])
def test_bitwise_repeatable_and_width_independent(name):
    net = NETS[name]()
    M = Model(net)
    x, u, lam, y, sx, su, ss = random_point(M, 5)
    args = list(map(_t, (x, u, lam, y, sx, su, ss)))
    outs = []
    for width, lds in ((1, 1), (2, 1), (2, 1), (3, 1), (2, 0), (4, 0)):
        G = _net_api().Net(net, panel_width=width, lds_panel=lds)
        K, _ = G.condense_reduced_hessian(*args)
        torch.cuda.synchronize()
        outs.append((width, lds, G.info["lds_panel"], _np(K).copy()))
        G.close()
    for w, l, used, K in outs[1:]:
        assert np.array_equal(K, outs[0][3]), (w, l, used)


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


@pytest.mark.parametrize("name,width", [("syn9", 1), ("syn1354", 1), ("syn118", 2),
                                        ("syn1354", 3)])
def test_solve_after_condensation_without_rhs(name, width):
    """Recovery by the single-column pass (condensation called without r),
    with the right-hand side condensed separately on the same factors; the
    pass reads the sweep records of the handle's panel width."""
    net = NETS[name]()
    M = Model(net)
    G = _net_api().Net(net, panel_width=width)
    assert G.info["panel_width"] == width
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
    assert np.abs(_np(p) - want).max() <= 1e-8 * np.abs(want).max()


def test_condense_9241_sampled_columns():
    """The 9241-bus condensation (nx 17036, nu 2889) in the launch shape the
    library picks, against the oracle on sampled columns and the full
    right-hand side (sparse LU of G_x on the host)."""
    net = synthnet.case9241(0)
    M = Model(net)
    print("condense syn9241 (sampled columns)", flush=True)
    G = _net_api().Net(net)
    x, u, lam, y, sx, su, ss = random_point(M, 0)
    r = residual_vector(M, 1)
    K, rhs = G.condense_reduced_hessian(*map(_t, (x, u, lam, y, sx, su, ss)), r=_t(r))
    torch.cuda.synchronize()
    B = R.kkt_blocks(M, x, u, lam, y, sx, su, ss)
    cols = [0, 1, 700, 1444, 1445, 2000, M.nu - 1]
    want, splu = R.condensed_columns_sparse(B, cols)
    Kg = _np(K).T
    for k, j in enumerate(cols):
        # K is symmetrised: compare with the mean of column and row j
        wj = want[:, k]
        err = np.linalg.norm(0.5 * (Kg[:, j] + Kg[j, :]) - wj) / np.linalg.norm(wj)
        assert err <= 1e-8, (j, err)
        assert np.array_equal(Kg[:, j], Kg[j, :])
    b, _ = R.condensed_rhs_sparse(B, r, splu)
    assert _rel(_np(rhs), b) <= 1e-8


def test_solve_9241_matches_oracle():
    """The condensed solve at 9241 buses: blocked Cholesky of the 2889 x 2889
    K_cond + delta I (the wide backward-substitution variant) and the
    control step, against the oracle's K_cond from sparse-LU columns, factored
    and solved densely on the host."""
    net = synthnet.case9241(0)
    M = Model(net)
    print("solve syn9241", flush=True)
    G = _net_api().Net(net)
    x, u, lam, y, sx, su, ss = random_point(M, 3, lam_scale=1.0, sig_range=(1.0, 1e3))
    r = residual_vector(M, 4)
    K, rhs = G.condense_reduced_hessian(*map(_t, (x, u, lam, y, sx, su, ss)), r=_t(r))
    B = R.kkt_blocks(M, x, u, lam, y, sx, su, ss)
    Kc, splu = R.condensed_columns_sparse(B, range(M.nu))
    Kc = R.symmetrize(Kc)
    delta = max(0.0, -np.linalg.eigvalsh(Kc).min()) * 1.5 + 1.0
    Kd = Kc + delta * np.eye(M.nu)
    b, _ = R.condensed_rhs_sparse(B, r, splu)
    p, code = G.solve_condensed_kkt(K, delta, rhs, _t(r))
    torch.cuda.synchronize()
    assert code == 0
    pu = np.linalg.solve(Kd, b)
    got = _np(p)[:M.nu]
    assert np.abs(got - pu).max() <= 1e-8 * np.abs(pu).max()
    Lg = np.tril(_np(K).T)
    assert _rel(Lg, np.linalg.cholesky(Kd)) <= 1e-8
