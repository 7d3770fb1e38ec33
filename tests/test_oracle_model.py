"""Pins of the oracle's OPF model against things the oracle does not compute
itself: textbook closed forms, complex-phasor arithmetic, conservation,
complex-step derivatives of its own function values, and Table 1."""
import json
import os

import numpy as np
import pytest

import synthnet
from oracle.model import Model, BUS_PQ, BUS_PV, BUS_REF

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def two_bus(r, x, b, vg=1.0):
    """Bus 0 = reference generator, bus 1 = PQ load, one line."""
    return synthnet.Network(
        nb=2, base_mva=100.0, bus_type=np.array([BUS_REF, BUS_PQ], np.int32),
        pd=np.array([0.0, 0.5]), qd=np.array([0.0, 0.15]),
        vmin=np.full(2, 0.9), vmax=np.full(2, 1.1),
        f=np.array([0], np.int32), t=np.array([1], np.int32),
        r=np.array([r]), x=np.array([x]), b=np.array([b]), rate=np.array([2.0]),
        gen_bus=np.array([0], np.int32), c2=np.array([0.05]), c1=np.array([20.0]),
        c0=np.array([0.0]), pmin=np.array([0.0]), pmax=np.array([2.0]),
        qmin=np.array([-2.0]), qmax=np.array([2.0]))


def test_lossless_line_closed_form():
    gold = json.load(open(os.path.join(GOLD, "lossless_line.json")))
    for c in gold["cases"]:
        M = Model(two_bus(0.0, c["X"], 0.0))
        theta = np.array([c["d"], 0.0])      # bus 0 is the reference: shift both
        theta -= theta[0]
        vm = np.array([c["V1"], c["V2"]])
        P, Q = M.injections(theta, vm)
        Pf, Qf = M.line_flows(theta, vm, np.array([0]), "f")
        Pt, Qt = M.line_flows(theta, vm, np.array([0]), "t")
        for got, want in ((P[0], c["P12"]), (Q[0], c["Q12"]), (P[1], c["P21"]),
                          (Q[1], c["Q21"]), (Pf[0], c["P12"]), (Qf[0], c["Q12"]),
                          (Pt[0], c["P21"]), (Qt[0], c["Q21"])):
            assert abs(got - want) < 1e-10


def test_generator_cost_closed_form():
    """The objective f of a 2-bus network with generators at both buses
    against the cost closed form evaluated by hand (tests/golden/cost_2bus.json):
    pins the MW cost convention, c0, and the reference generator's output
    taken from the power balance."""
    gold = json.load(open(os.path.join(GOLD, "cost_2bus.json")))
    c = gold["network"]
    net = synthnet.Network(
        nb=2, base_mva=100.0, bus_type=np.array([BUS_REF, BUS_PV], np.int32),
        pd=np.array(c["pd"]), qd=np.array([0.0, 0.1]),
        vmin=np.full(2, 0.9), vmax=np.full(2, 1.1),
        f=np.array([0], np.int32), t=np.array([1], np.int32),
        r=np.array([0.0]), x=np.array([c["X"]]), b=np.array([0.0]), rate=np.array([0.0]),
        gen_bus=np.array([0, 1], np.int32), c2=np.array(c["c2"]), c1=np.array(c["c1"]),
        c0=np.array(c["c0"]), pmin=np.zeros(2), pmax=np.full(2, 3.0),
        qmin=np.full(2, -3.0), qmax=np.full(2, 3.0))
    M = Model(net)
    assert M.nx == 1 and M.nu == 3          # theta_1; Vm_0, Vm_1, Pg_1
    x, u = M.join(np.array([c["theta0"], c["theta1"]]), np.array([c["V0"], c["V1"]]),
                  np.array([0.0, c["pg1"]]))
    _, h, f = M.functions(x, u)
    assert abs(h[0] - gold["pg_ref"]) <= 1e-10           # h_0 = Pg_ref
    assert abs(float(np.real(f)) - gold["f"]) <= 1e-8 * gold["f"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_injections_match_complex_phasors(seed):
    """S_i = V_i conj(sum_k Y_ik V_k) with Y assembled here from r, x, b."""
    net = synthnet.small(6, 9, 2, seed=seed)
    M = Model(net)
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.2, net.nb)
    vm = rng.uniform(0.9, 1.1, net.nb)
    Y = np.zeros((net.nb, net.nb), complex)
    for l in range(net.nl):
        y = 1.0 / complex(net.r[l], net.x[l])
        f, t = net.f[l], net.t[l]
        Y[f, f] += y + 0.5j * net.b[l]
        Y[t, t] += y + 0.5j * net.b[l]
        Y[f, t] -= y
        Y[t, f] -= y
    V = vm * np.exp(1j * theta)
    S = V * np.conj(Y @ V)
    P, Q = M.injections(theta, vm)
    assert np.allclose(P, S.real, atol=1e-12) and np.allclose(Q, S.imag, atol=1e-12)
    # line flows from the line's own current
    for l in range(net.nl):
        f, t = net.f[l], net.t[l]
        y = 1.0 / complex(net.r[l], net.x[l])
        If = (y + 0.5j * net.b[l]) * V[f] - y * V[t]
        Sf = V[f] * np.conj(If)
        Pf, Qf = M.line_flows(theta, vm, np.array([l]), "f")
        assert abs(Pf[0] - Sf.real) < 1e-12 and abs(Qf[0] - Sf.imag) < 1e-12


def test_flows_sum_to_injections_and_losses_nonnegative():
    net = synthnet.case118(0)
    net = net.copy(b=np.zeros(net.nl))
    M = Model(net)
    rng = np.random.default_rng(3)
    theta = rng.normal(0, 0.1, net.nb)
    vm = rng.uniform(0.95, 1.05, net.nb)
    P, Q = M.injections(theta, vm)
    Pf, Qf = M.line_flows(theta, vm, None, "f")
    Pt, Qt = M.line_flows(theta, vm, None, "t")
    Ps = np.zeros(net.nb)
    Qs = np.zeros(net.nb)
    np.add.at(Ps, net.f, Pf)
    np.add.at(Ps, net.t, Pt)
    np.add.at(Qs, net.f, Qf)
    np.add.at(Qs, net.t, Qt)
    assert np.allclose(P, Ps, atol=1e-12) and np.allclose(Q, Qs, atol=1e-12)
    assert np.all(Pf + Pt >= -1e-14)      # series resistance only dissipates
    assert P.sum() > 0


def _complex_step_jac(M, x, u, which, lam=None, y=None):
    w = np.concatenate([u, x])
    h = 1e-30
    cols = []
    for j in range(w.shape[0]):
        wc = w.astype(complex)
        wc[j] += 1j * h
        xc, uc = wc[M.nu:], wc[:M.nu]
        if which == "grad_l":
            v = M.lagrangian_gradient(xc, uc, lam, y)
        else:
            g, hh, f = M.functions(xc, uc)
            v = {"g": g, "h": hh, "f": np.atleast_1d(f)}[which]
        cols.append(np.asarray(v).imag / h)
    return np.array(cols).T


@pytest.mark.parametrize("name,net", [("syn9", synthnet.case9(1)),
                                      ("syn12", synthnet.small(12, 18, 4, seed=3))])
def test_first_derivatives_complex_step(name, net):
    M = Model(net)
    rng = np.random.default_rng(7)
    x, u = M.join(rng.normal(0, 0.1, net.nb), rng.uniform(0.9, 1.1, net.nb),
                  rng.uniform(0, 1, net.ng))
    G, A, gf = M.jacobians(x, u)
    for which, ana in (("g", G.toarray()), ("h", A.toarray()), ("f", gf[None, :])):
        cs = _complex_step_jac(M, x, u, which)
        scale = max(1.0, np.abs(cs).max())
        assert np.abs(cs - ana).max() <= 1e-12 * scale, which


@pytest.mark.parametrize("name,net", [("syn9", synthnet.case9(3)),
                                      ("syn12", synthnet.small(12, 18, 4, seed=4))])
def test_hessian_complex_step_of_gradient(name, net):
    M = Model(net)
    rng = np.random.default_rng(8)
    x, u = M.join(rng.normal(0, 0.1, net.nb), rng.uniform(0.9, 1.1, net.nb),
                  rng.uniform(0, 1, net.ng))
    lam = rng.normal(0, 20, M.nx)
    y = rng.uniform(0, 5, M.m)
    W = M.hessian_lagrangian(x, u, lam, y).toarray()
    cs = _complex_step_jac(M, x, u, "grad_l", lam, y)
    assert np.abs(cs - W).max() <= 1e-12 * np.abs(W).max()
    assert np.abs(W - W.T).max() <= 1e-12 * np.abs(W).max()


def test_state_control_dimensions_match_table1():
    """The state/control split reproduces Table 1's n_x and n_u."""
    gold = json.load(open(os.path.join(GOLD, "table1_dims.json")))
    for c in gold["cases"]:
        net = synthnet.make_network(c["nb"], c["nl"], c["ng"], seed=0, load_frac=0.6)
        M = Model(net)
        assert (M.nx, M.nu) == (c["nx"], c["nu"]), c["case"]


def test_nine_bus_dimensions():
    M = Model(synthnet.case9(1))
    assert (M.nx, M.nu, M.m) == (14, 5, 4)


def test_index_maps_roundtrip():
    net = synthnet.case118(2)
    M = Model(net)
    rng = np.random.default_rng(0)
    th, vm, pg = rng.normal(size=net.nb), rng.uniform(size=net.nb), rng.uniform(size=net.ng)
    th[M.ref] = 0.0
    x, u = M.join(th, vm, pg)
    th2, vm2, pg2 = M.split(x, u)
    assert np.array_equal(th2, th) and np.array_equal(vm2, vm)
    mask = np.ones(net.ng, bool)
    mask[M.ref_gen] = False
    assert np.array_equal(pg2[mask], pg[mask])
    assert np.array_equal(M.x_bus[M.x_kind == 0], np.array(M.nonref))
