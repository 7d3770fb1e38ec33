"""The interior-point driver on the GPU (rh_ipm_*) against the oracle's
Algorithm 1: the same iterations (barrier parameter, step lengths, inertia
shifts, objective) and the same final point. The oracle solves the augmented
KKT system densely, the library through the condensed matrix, so the steps
agree to rounding; the tolerances below (1e-6 relative on iterates, exact on
the discrete decisions) leave room for that."""
import json
import os

import numpy as np
import pytest

import synthnet
from oracle.model import Model
from oracle.ipm import LinRedIPM, flat_start, IPMOptions

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _api():
    from paper_2203_11875_amd import api
    return api


NETS = {
    "syn9-1": lambda: synthnet.case9(1),
    "syn9-3": lambda: synthnet.case9(3),
    "syn5": lambda: synthnet.small(5, 7, 2, seed=1),
    "syn118": lambda: synthnet.case118(0),
}


@pytest.mark.parametrize("name", list(NETS))
def test_ipm_iterates_match_oracle(name):
    net = NETS[name]()
    api = _api()
    G = api.Net(net)
    ipm = api.Ipm(G, tol=1e-6)
    orc = LinRedIPM(net, IPMOptions(tol=1e-6))
    x0, u0 = flat_start(orc.M)
    st, log, ok = orc.solve(x0, u0)
    assert ok
    glog = []
    for _ in range(len(log) + 5):
        code, info = ipm.step()
        assert code == 0, (code, info)
        if info["converged"]:
            break
        glog.append(info)
    assert info["converged"] == 1
    assert len(glog) == len(log)
    assert abs(info["obj_scale"] - orc.sigma_f) <= 1e-12 * orc.sigma_f
    for k, (a, b) in enumerate(zip(glog, log)):
        assert a["mu"] == pytest.approx(b["mu"], rel=1e-9), k
        assert a["alpha_pr"] == pytest.approx(b["alpha_pr"], rel=1e-6), k
        assert a["ls_trials"] == b["trials"], k
        assert (a["delta_w"] == 0.0) == (b["delta_w"] == 0.0), k
        assert a["obj"] == pytest.approx(b["obj"], rel=1e-8), k
    s = ipm.state()
    got_w = np.concatenate([s["u"].cpu().numpy(), s["x"].cpu().numpy()])
    assert np.abs(got_w - st.w).max() <= 1e-6 * max(1.0, np.abs(st.w).max())
    assert np.abs(s["s"].cpu().numpy() - st.s).max() <= 1e-6 * max(1.0, np.abs(st.s).max())
    ipm.close()
    G.close()


def test_objective_scale_scales_f():
    net = synthnet.case118(0)
    api = _api()
    G = api.Net(net)
    M = Model(net)
    x, u = flat_start(M)
    _, _, f1 = G.eval_residual(x, u)
    code = api.lib().rh_set_objective_scale(G.h, 0.25)
    assert code == 0
    _, _, f2 = G.eval_residual(x, u)
    assert float(f2.cpu()[0]) == pytest.approx(0.25 * float(f1.cpu()[0]), rel=1e-14)
    assert api.lib().rh_set_objective_scale(G.h, 0.0) != 0
    assert api.lib().rh_set_objective_scale(G.h, 1.0) == 0
    _, _, f3 = G.eval_residual(x, u)
    assert float(f3.cpu()[0]) == float(f1.cpu()[0])
    G.close()


def test_ipm_1354_matches_oracle():
    """The 1354-bus stand-in solved to 1e-6 on the GPU against the oracle's
    run of the same method from the same start (tests/golden/ipm_syn1354.json,
    written by the oracle alone): same iteration count, optimal objective
    within 1e-6 relative, optimal control within 1e-6; the final point is also
    checked with the oracle's model (feasibility and bounds)."""
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                       "golden", "ipm_syn1354.json")))["tol_1e-6"]
    net = synthnet.case1354(0)
    api = _api()
    G = api.Net(net)
    print("ipm syn1354 to 1e-6", flush=True)
    ipm = api.Ipm(G, tol=1e-6, max_iter=150)
    code, info = ipm.solve()
    assert code == 0 and info["converged"] == 1, info
    assert info["iter"] == gold["iterations"], (info["iter"], gold["iterations"])
    assert abs(info["obj"] - gold["objective"]) <= 1e-6 * abs(gold["objective"])
    assert abs(info["obj_scale"] - gold["obj_scale"]) <= 1e-12 * gold["obj_scale"]
    s = ipm.state()
    x, u = s["x"].cpu().numpy(), s["u"].cpu().numpy()
    uo = np.asarray(gold["u"])
    assert np.abs(u - uo).max() <= 1e-6 * max(1.0, np.abs(uo).max())
    M = Model(net)
    g, h, f = M.functions(x, u)
    hl, hu = M.h_bounds()
    assert np.abs(g).max() <= 1e-6
    assert np.all(h <= hu + 1e-6) and np.all(h >= hl - 1e-6)
    assert float(f) == pytest.approx(info["obj"], rel=1e-9)
    ipm.close()
    G.close()


def test_tiny_static_pivot_stops_the_step():
    """At a point where the static pivots of G_x fail (a lossless line
    carrying a 90-degree angle difference; the matrix itself is nonsingular,
    see test_host_symbolic.py), the solve reports RH_SMALL_PIVOT ahead of the
    Cholesky's outcome, and rh_ipm_step returns RH_SMALL_PIVOT without moving
    the iterate."""
    from oracle.model import BUS_PQ, BUS_REF
    net = synthnet.Network(
        nb=3, base_mva=100.0, bus_type=np.array([BUS_REF, BUS_PQ, BUS_PQ], np.int32),
        pd=np.array([0.0, 0.3, 0.2]), qd=np.array([0.0, 0.1, 0.05]),
        vmin=np.full(3, 0.9), vmax=np.full(3, 1.1),
        f=np.array([0, 1], np.int32), t=np.array([1, 2], np.int32),
        r=np.zeros(2), x=np.array([0.1, 0.1]), b=np.zeros(2), rate=np.zeros(2),
        gen_bus=np.array([0], np.int32), c2=np.array([0.02]), c1=np.array([20.0]),
        c0=np.array([0.0]), pmin=np.array([0.0]), pmax=np.array([2.0]),
        qmin=np.array([-2.0]), qmax=np.array([2.0]))
    api = _api()
    M = Model(net)
    x0, u0 = M.join(np.array([0.0, -np.pi / 2, -np.pi / 2]), np.ones(3), np.zeros(1))
    dev = torch.device("cuda", 0)
    T = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=dev)
    G = api.Net(net)
    ones = lambda n: T(np.ones(n))
    r = T(np.ones(M.nu + 2 * M.nx + 2 * M.m))
    K, rhs = G.condense_reduced_hessian(T(x0), T(u0), T(np.zeros(M.nx)), T(np.zeros(M.m)),
                                        ones(M.nx), ones(M.nu), ones(M.m), r=r)
    _, code = G.solve_condensed_kkt(K, 0.0, rhs, r)
    assert code == 2                       # RH_SMALL_PIVOT
    ipm = api.Ipm(G, x0=T(x0), u0=T(u0), tol=1e-6)
    before = {k: v.clone() for k, v in ipm.state().items()}
    code, info = ipm.step()
    assert code == 2, (code, info)
    after = ipm.state()
    for k in before:
        assert torch.equal(before[k], after[k]), k
    ipm.close()
    G.close()
