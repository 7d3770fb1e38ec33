"""The Newton-Raphson power flow (rh_power_flow) and the reduce-then-linearize
driver (rh_redlin_*, Algorithm 2) on the GPU against the oracle: the power
flow reaches the oracle's solution of g(x, u) = 0; RedLin takes the oracle
RedLin's iterations (barrier parameter, step lengths, trials, objective) and
reaches its final point; on the 1354-bus stand-in it reaches the GPU LinRed
optimum."""
import numpy as np
import pytest

import synthnet
from oracle.ipm import IPMOptions, flat_start
from oracle.redlin import RedLinIPM
from oracle import powerflow as PF

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


@pytest.mark.parametrize("name", ["syn9-1", "syn118", "syn1354"])
def test_power_flow_matches_oracle(name):
    net = synthnet.case1354(0) if name == "syn1354" else NETS[name]()
    print(f"power flow: {name}", flush=True)
    rl = RedLinIPM(net, IPMOptions())
    x0, u0 = flat_start(rl.M)
    u = u0.copy()
    u[: rl.M.ng] = 1.02                       # generator voltages
    want = PF.solve_pf(rl.M, u, x0)
    api = _api()
    G = api.Net(net)
    x, code, it, res = G.power_flow(u, x0, tol=1e-10, max_iter=20)
    assert code == 0 and res <= 1e-10 and 2 <= it <= 10, (code, it, res)
    np.testing.assert_allclose(x.cpu().numpy(), want, rtol=0, atol=1e-9)


def test_power_flow_reports_failure():
    net = synthnet.case9(1)
    rl = RedLinIPM(net, IPMOptions())
    x0, u0 = flat_start(rl.M)
    u = u0.copy()
    u[rl.M.ng:] *= 60.0            # far more generation than the lines can carry
    api = _api()
    G = api.Net(net)
    _, code, it, res = G.power_flow(u, x0, tol=1e-10, max_iter=20)
    assert code == 3 and not res <= 1e-10


@pytest.mark.parametrize("name", list(NETS))
def test_redlin_iterates_match_oracle(name):
    net = NETS[name]()
    print(f"redlin vs oracle: {name}", flush=True)
    orc = RedLinIPM(net, IPMOptions(tol=1e-6))
    st, log, ok = orc.solve(*flat_start(orc.M))
    assert ok
    api = _api()
    G = api.Net(net)
    rl = api.RedLin(G, tol=1e-6)
    assert rl.mr == orc.mr
    glog = []
    for _ in range(len(log) + 5):
        code, info = rl.step()
        assert code == 0, (code, info)
        if info["converged"]:
            break
        glog.append(info)
    assert info["converged"] == 1
    assert len(glog) == len(log)
    for k, (a, b) in enumerate(zip(glog, log)):
        assert a["mu"] == pytest.approx(b["mu"], rel=1e-9), k
        assert a["alpha_pr"] == pytest.approx(b["alpha_pr"], rel=1e-6), k
        assert a["ls_trials"] == b["trials"], k
        assert a["delta_w"] == pytest.approx(b["delta_w"], rel=1e-9, abs=0.0), k
        assert a["obj"] == pytest.approx(b["obj"], rel=1e-8), k
    s = {k: v.cpu().numpy() for k, v in rl.state().items()}
    np.testing.assert_allclose(s["u"], st.u, rtol=0, atol=1e-6)
    np.testing.assert_allclose(s["x"], st.x, rtol=0, atol=1e-6)
    np.testing.assert_allclose(s["s"], st.s, rtol=0, atol=1e-6)
    # every accepted point satisfies the state equation
    g, _, _ = G.eval_residual(rl.state()["x"], rl.state()["u"])
    assert np.abs(g.cpu().numpy()).max() <= 1e-10


def test_redlin_1354_reaches_linred_optimum():
    net = synthnet.case1354(0)
    print("redlin: syn1354", flush=True)
    api = _api()
    G = api.Net(net)
    rl = api.RedLin(G, tol=1e-6)
    code, info = rl.solve()
    assert code == 0 and info["converged"] == 1, (code, info)
    f_rl = info["obj"]
    rl.close()
    ipm = api.Ipm(G, tol=1e-6)
    code, info2 = ipm.solve()
    assert code == 0
    assert abs(f_rl - info2["obj"]) <= 1e-6 * abs(info2["obj"])
