"""Host logic of the HIP library, run on the CPU: the C ABI loads and exports
every declared symbol; the symbolic analysis (index maps, patterns, ordering,
symbolic LU, level sets, refactorisation schedule) agrees with the oracle."""
import os
import re

import numpy as np
import pytest

import synthnet
from oracle.model import Model

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2203_11875_amd import api
    return api


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_2203_11875_amd import _abi
    header = open(os.path.join(ROOT, "include", "rhipm.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    names = set(re.findall(r"\b(rh_[a-z_]+)\s*\(", header))
    assert names, "no declarations parsed"
    lib = ctypes.CDLL(_abi.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert names == set(_abi.SIGNATURES), "binding and header disagree"


NETS = [synthnet.case9(1), synthnet.small(5, 7, 2, seed=1), synthnet.case118(0),
        synthnet.case300(0), synthnet.case1354(0)]


@pytest.mark.parametrize("net", NETS, ids=lambda n: n.name)
def test_dimensions_and_index_maps_match_oracle(net):
    S = _lib().Symbolic(net)
    M = Model(net)
    assert (S.info["nx"], S.info["nu"], S.info["m"]) == (M.nx, M.nu, M.m)
    xk, xb, uk, ur = S.index_maps()
    assert np.array_equal(xk, M.x_kind) and np.array_equal(xb, M.x_bus)
    assert np.array_equal(uk, M.u_kind) and np.array_equal(ur, M.u_ref)


@pytest.mark.parametrize("net", NETS, ids=lambda n: n.name)
def test_levels_valid(net):
    """Level sets, the sweep step schedule and the step lists of work-groups
    of 4 and 8 waves (every step once, a group's steps of one level, in
    schedule order) pass the host check (rh_symbolic_check_levels)."""
    S = _lib().Symbolic(net)
    assert S.check_levels() == 0
    assert S.info["levels_lower"] >= 1 and S.info["nnz_lu"] >= S.info["nnz_gx"]


def test_refactor_split_levels_1354():
    """The leading levels with many rows of the 1354-bus factorisation run as
    per-level launches; their tables (global U positions of every task step)
    agree with the wave-resident ones (checked by check_levels)."""
    S = _lib().Symbolic(synthnet.case1354(0))
    assert S.info["refactor_kernel"] == 0
    assert 1 <= S.info["refactor_split"] < S.info["levels_lower"]
    assert S.check_levels() == 0


@pytest.mark.parametrize("width", [1, 3])
@pytest.mark.parametrize("net", NETS[:4], ids=lambda n: n.name)
def test_condensation_records_emulated_match_dense(net, width):
    """The condensation kernel's device records (sweep steps, K and G_u^T
    streams with their byte offsets for the panel width, row orders and
    transcription lists), run lane by lane on the host as the wave runs them
    (FMA chains, DPP shift tree, flushes), give the columns of
    [I;S]^T K [I;S] and the right-hand-side column that a dense computation
    gives for random values (Section 3.3)."""
    S = _lib().Symbolic(net)
    for seed in (1, 2):
        err = S.check_condense(width=width, seed=seed)
        assert err <= 1e-11, (net.name, width, seed, err)


@pytest.mark.parametrize("refactor", [0, 1], ids=["wave", "staged"])
@pytest.mark.parametrize("net", NETS, ids=lambda n: n.name)
def test_patterns_cover_oracle_and_host_refactorisation_solves(net, refactor):
    """The G_x pattern holds every structural nonzero of the oracle's G_x, the
    pivot order is a permutation, and refactorising with the device schedule
    (wave-resident tasks emulated lane by lane, or the level-staged rows)
    then sweeping the level sets solves G_x z = b and G_x^T z = b."""
    S = _lib().Symbolic(net, refactor=refactor)
    assert S.info["refactor_kernel"] == refactor
    M = Model(net)
    rng = np.random.default_rng(0)
    x, u = M.join(rng.normal(0, .1, net.nb), rng.uniform(.95, 1.05, net.nb),
                  rng.uniform(0, 1, net.ng))
    G, _, _ = M.jacobians(x, u)
    Gx = G[:, M.nu:].tocsr()
    ptr, col, perm = S.gx_pattern()
    assert np.array_equal(np.sort(perm), np.arange(M.nx))
    pat = {(r, c) for r in range(M.nx) for c in col[ptr[r]:ptr[r + 1]]}
    Gc = Gx.tocoo()
    assert all((r, c) in pat for r, c in zip(Gc.row, Gc.col))
    vals = np.asarray(Gx[np.repeat(np.arange(M.nx), np.diff(ptr)), col]).ravel()
    Gd = Gx.toarray()
    for tr in (False, True):
        b = rng.normal(size=M.nx)
        z = S.host_solve(vals, b, transpose=tr)
        A = Gd.T if tr else Gd
        assert np.abs(A @ z - b).max() <= 1e-10 * max(1.0, np.abs(b).max()) * np.abs(Gd).max()


@pytest.mark.parametrize("ordering", [0, 1, 2], ids=["md_level", "md", "nd"])
@pytest.mark.parametrize("net", NETS, ids=lambda n: n.name)
def test_each_ordering_gives_a_valid_factorisation(net, ordering):
    """Every ordering of G_x (minimum degree with a level term, plain minimum
    degree, nested dissection) gives a permutation whose level tables check
    and whose host refactorisation solves G_x z = b. Nested dissection puts
    its separators last, whose dense rows exceed a sweep step on the larger
    networks: those are rejected with an argument error, not mis-solved."""
    api = _lib()
    if ordering == 2 and net.nb > 200:
        with pytest.raises(api.RhError):
            api.Symbolic(net, ordering=ordering)
        return
    S = api.Symbolic(net, ordering=ordering)
    assert S.check_levels() == 0
    M = Model(net)
    rng = np.random.default_rng(3)
    x, u = M.join(rng.normal(0, .1, net.nb), rng.uniform(.95, 1.05, net.nb),
                  rng.uniform(0, 1, net.ng))
    G, _, _ = M.jacobians(x, u)
    Gx = G[:, M.nu:].tocsr()
    ptr, col, perm = S.gx_pattern()
    assert np.array_equal(np.sort(perm), np.arange(M.nx))
    vals = np.asarray(Gx[np.repeat(np.arange(M.nx), np.diff(ptr)), col]).ravel()
    b = rng.normal(size=M.nx)
    z = S.host_solve(vals, b)
    assert np.abs(Gx @ z - b).max() <= 1e-10 * max(1.0, np.abs(b).max()) * np.abs(Gx).max()


def test_level_term_shortens_the_dependency_chain():
    """The level term of the default ordering: on the 1354-bus network it
    factors in about half the levels of plain minimum degree (22 against
    43) with at most 2% more LU entries."""
    api = _lib()
    net = synthnet.case1354(0)
    a, b = api.Symbolic(net, ordering=0).info, api.Symbolic(net, ordering=1).info
    assert a["levels_lower"] <= 0.6 * b["levels_lower"], (a["levels_lower"], b["levels_lower"])
    assert a["nnz_lu"] <= 1.02 * b["nnz_lu"]
    assert a["sweep_steps"] < b["sweep_steps"]


def test_launch_key_and_tuning_file(tmp_path):
    """The tuning cache's key follows the network structure only: load
    scenarios share it, another network does not; a saved table loads back."""
    api = _lib()
    a = synthnet.case118(0)
    assert api.launch_key(a) == api.launch_key(synthnet.scale_loads(a, 5))
    assert api.launch_key(a) != api.launch_key(synthnet.case300(0))
    saved = dict(api.TUNING)
    try:
        api.TUNING.clear()
        api.TUNING[api.launch_key(a)] = (2, 1, 1)
        path = tmp_path / "tuning.json"
        api.save_tuning(path)
        api.TUNING.clear()
        api.load_tuning(path)
        assert api.TUNING == {api.launch_key(a): (2, 1, 1)}
    finally:
        api.TUNING.clear()
        api.TUNING.update(saved)


def test_rejects_bad_networks():
    api = _lib()
    net = synthnet.case9(1)
    bad = net.copy(bus_type=np.full(net.nb, 1, np.int32))          # no reference bus
    with pytest.raises(RuntimeError, match="invalid argument"):
        api.Symbolic(bad)
    f = net.f.copy()
    f[0] = net.t[0]                                                  # self loop
    with pytest.raises(RuntimeError, match="invalid argument"):
        api.Symbolic(net.copy(f=f))
    iso = synthnet.make_network(6, 5, 2, seed=0, load_frac=0.5)      # tree
    f, t = iso.f.copy(), iso.t.copy()                                 # cut bus 5 off
    keep = (f != 5) & (t != 5)
    cut = iso.copy(f=f[keep], t=t[keep], r=iso.r[keep], x=iso.x[keep], b=iso.b[keep],
                   rate=iso.rate[keep])
    if 5 not in cut.gen_bus:
        with pytest.raises(RuntimeError, match="singular"):
            api.Symbolic(cut)


def test_nine_bus_sizes_and_9241_analysis():
    S = _lib().Symbolic(synthnet.case9241(0))
    assert (S.info["nx"], S.info["nu"]) == (17036, 2889)
    assert S.check_levels() == 0


def _line_pair(x01, x12):
    """Reference bus 0 (generator), PQ buses 1 and 2, lossless lines 0-1 and
    1-2 with reactances x01, x12."""
    from oracle.model import BUS_PQ, BUS_REF
    return synthnet.Network(
        nb=3, base_mva=100.0, bus_type=np.array([BUS_REF, BUS_PQ, BUS_PQ], np.int32),
        pd=np.array([0.0, 0.3, 0.2]), qd=np.array([0.0, 0.1, 0.05]),
        vmin=np.full(3, 0.9), vmax=np.full(3, 1.1),
        f=np.array([0, 1], np.int32), t=np.array([1, 2], np.int32),
        r=np.zeros(2), x=np.array([x01, x12]), b=np.zeros(2), rate=np.zeros(2),
        gen_bus=np.array([0], np.int32), c2=np.array([0.02]), c1=np.array([20.0]),
        c0=np.array([0.0]), pmin=np.array([0.0]), pmax=np.array([2.0]),
        qmin=np.array([-2.0]), qmax=np.array([2.0]))


def _gx_values(S, M, theta, vm):
    x, u = M.join(theta, vm, np.zeros(M.ng))
    G, _, _ = M.jacobians(x, u)
    Gx = G.tocsr()[:, M.nu:]
    ptr, col, _ = S.gx_pattern()
    return np.asarray(Gx[np.repeat(np.arange(M.nx), np.diff(ptr)), col]).ravel(), \
        Gx.toarray()


@pytest.mark.parametrize("case", ["quarter_turn", "near_zero_reactance"])
def test_static_pivot_flags_tiny_pivots(case):
    """The static-pivot refactorisation (host emulation of the device
    schedule) reports RH_SMALL_PIVOT when a pivot is not above 1e-14 of its
    row's largest entry, on two crafted G_x: (a) a lossless line carrying a
    90-degree angle difference, where dP/dtheta at its PQ end vanishes
    (cos(pi/2) = 0) while the matrix stays nonsingular; (b) a line of
    reactance 1e-16 p.u. between two PQ buses, whose eliminated pivot is the
    difference of two admittances of 1e16. The same networks at ordinary
    points solve to rounding."""
    S_cls = _lib().Symbolic
    if case == "quarter_turn":
        net = _line_pair(0.1, 0.1)
        bad = (np.array([0.0, -np.pi / 2, -np.pi / 2]), np.ones(3))
    else:
        net = _line_pair(0.1, 1e-16)
        bad = (np.array([0.0, -0.05, -0.05]), np.ones(3))
    good = (np.array([0.0, -0.05, -0.08]), np.array([1.0, 0.98, 0.97]))
    S = S_cls(net)
    M = Model(net)
    vals, Gd = _gx_values(S, M, *good)
    if case == "quarter_turn":
        b = np.arange(1.0, M.nx + 1)
        z = S.host_solve(vals, b)
        assert np.abs(Gd @ z - b).max() <= 1e-10 * np.abs(Gd).max() * np.abs(z).max()
    vals, Gd = _gx_values(S, M, *bad)
    assert np.linalg.matrix_rank(Gd) == M.nx or case != "quarter_turn"
    with pytest.raises(RuntimeError, match="small pivot"):
        S.host_solve(vals, np.ones(M.nx))
