"""Seeded synthetic power networks and random iterates.

This module only draws random numbers and builds topologies. It holds none of
the condensation method's arithmetic (no admittances, no power-flow equations,
no derivatives), so both the CPU oracle and the GPU path may take their inputs
from it.

Networks follow the shapes of the paper's benchmark instances (Table 1:
number of buses, lines and generators) but the MATPOWER/PGLIB case files are not
available, so each instance is a seeded stand-in:

* topology: a random recursive spanning tree over a random bus permutation, plus
  *local* chords obtained from 2-4 step random walks (real grids are nearly
  planar; uniformly random chords would give a sparse LU with ~10x more fill);
* line data, two recipes (per unit on a 100 MVA base):
  - "wide" (the 9-bus ring): r ~ U[0.005, 0.05], x ~ U[0.02, 0.3],
    b ~ U[0, 0.2], rate ~ U[1, 5] p.u. or none;
  - "transmission" (118 buses and up): x ~ U[0.005, 0.05], r = x U[0.1, 0.3],
    b ~ U[0, 0.1], rate ~ U[2, 8] p.u. or none. With the wide ranges and loads
    Pd ~ U[0.1, 2], most seeds of the 118- to 1354-bus meshes have no
    interior-point solution from the flat start (measured with the oracle),
    so the larger stand-ins use transmission-like line data and lighter loads;
* one generator per generator bus, the first one sits on the reference bus;
  quadratic cost c2 ~ U[0.01, 0.1] $/MW^2, c1 ~ U[10, 40] $/MW, c0 = 0;
* loads Pd ~ U[lo, hi] p.u. on a random fraction of the buses, Qd = 0.3 Pd;
* limits: Vm in [0.9, 1.1] at every bus, Pmin = 0, Pmax = 2 sum(Pd) / ng,
  Qmax = -Qmin = Pmax.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

BUS_PQ, BUS_PV, BUS_REF = 1, 2, 3


@dataclass
class Network:
    """Plain network description; every array is a numpy array (host)."""
    nb: int
    base_mva: float
    bus_type: np.ndarray   # int32[nb]: 3 ref, 2 PV (generator bus), 1 PQ
    pd: np.ndarray         # float64[nb] active load, p.u.
    qd: np.ndarray         # float64[nb] reactive load, p.u.
    vmin: np.ndarray       # float64[nb]
    vmax: np.ndarray       # float64[nb]
    f: np.ndarray          # int32[nl] from bus
    t: np.ndarray          # int32[nl] to bus
    r: np.ndarray          # float64[nl] series resistance, p.u.
    x: np.ndarray          # float64[nl] series reactance, p.u.
    b: np.ndarray          # float64[nl] total line charging, p.u.
    rate: np.ndarray       # float64[nl] apparent-power limit, p.u.; <= 0 means none
    gen_bus: np.ndarray    # int32[ng] bus of each generator (gen 0 is on the ref bus)
    c2: np.ndarray         # float64[ng] $/MW^2
    c1: np.ndarray         # float64[ng] $/MW
    c0: np.ndarray         # float64[ng] $
    pmin: np.ndarray       # float64[ng] p.u.
    pmax: np.ndarray       # float64[ng] p.u.
    qmin: np.ndarray       # float64[ng] p.u.
    qmax: np.ndarray       # float64[ng] p.u.
    name: str = ""
    seed: int = 0

    @property
    def nl(self) -> int:
        return int(self.f.shape[0])

    @property
    def ng(self) -> int:
        return int(self.gen_bus.shape[0])

    def copy(self, **changes) -> "Network":
        arrays = {k: (v.copy() if isinstance(v, np.ndarray) else v)
                  for k, v in self.__dict__.items()}
        arrays.update(changes)
        return Network(**arrays)


def _tree_plus_local_chords(rng: np.random.Generator, nb: int, nl: int):
    """Random recursive tree on a random permutation + local chords."""
    if nl < nb - 1:
        raise ValueError("need at least nb-1 lines for a spanning tree")
    perm = rng.permutation(nb)
    edges = []
    adj = [set() for _ in range(nb)]
    for k in range(1, nb):
        a = int(perm[k])
        b = int(perm[rng.integers(0, k)])
        edges.append((b, a))
        adj[a].add(b)
        adj[b].add(a)
    tries = 0
    while len(edges) < nl:
        tries += 1
        if tries > 200 * nl + 1000:
            raise RuntimeError("could not place the requested number of chords")
        start = int(rng.integers(0, nb))
        cur = start
        steps = int(rng.integers(2, 5))
        for _ in range(steps):
            nbrs = sorted(adj[cur])
            cur = nbrs[int(rng.integers(0, len(nbrs)))]
        if cur == start or cur in adj[start]:
            continue
        edges.append((start, cur))
        adj[start].add(cur)
        adj[cur].add(start)
    e = np.array(edges, dtype=np.int32)
    return e[:, 0].copy(), e[:, 1].copy()


def make_network(nb: int, nl: int, ng: int, *, seed: int, load_frac: float,
                 pd_range=(0.05, 0.5), rated: bool = True, name: str = "",
                 ring: bool = False, lines: str = "transmission") -> Network:
    """Seeded synthetic network (see module docstring for the recipe)."""
    if ng < 1 or ng > nb:
        raise ValueError("bad generator count")
    rng = np.random.default_rng(seed)
    if ring:
        if nl != nb:
            raise ValueError("a ring has nb lines")
        f = np.arange(nb, dtype=np.int32)
        t = ((np.arange(nb) + 1) % nb).astype(np.int32)
    else:
        f, t = _tree_plus_local_chords(rng, nb, nl)
    if lines == "wide":
        r = rng.uniform(0.005, 0.05, nl)
        x = rng.uniform(0.02, 0.3, nl)
        b = rng.uniform(0.0, 0.2, nl)
        rate = rng.uniform(1.0, 5.0, nl) if rated else np.zeros(nl)
    elif lines == "transmission":
        x = rng.uniform(0.005, 0.05, nl)
        r = x * rng.uniform(0.1, 0.3, nl)
        b = rng.uniform(0.0, 0.1, nl)
        rate = rng.uniform(2.0, 8.0, nl) if rated else np.zeros(nl)
    else:
        raise ValueError(f"unknown line recipe {lines}")

    gen_bus = rng.choice(nb, size=ng, replace=False).astype(np.int32)
    bus_type = np.full(nb, BUS_PQ, dtype=np.int32)
    bus_type[gen_bus] = BUS_PV
    bus_type[gen_bus[0]] = BUS_REF

    pd = np.zeros(nb)
    if ring:
        # loads at every non-generator bus
        load_buses = np.flatnonzero(bus_type == BUS_PQ)
    else:
        n_load = int(round(load_frac * nb))
        load_buses = rng.choice(nb, size=n_load, replace=False)
    pd[load_buses] = rng.uniform(pd_range[0], pd_range[1], load_buses.shape[0])
    qd = 0.3 * pd

    c2 = rng.uniform(0.01, 0.1, ng)
    c1 = rng.uniform(10.0, 40.0, ng)
    c0 = np.zeros(ng)
    pmax_each = 2.0 * pd.sum() / ng
    pmin = np.zeros(ng)
    pmax = np.full(ng, pmax_each)
    qmax = np.full(ng, pmax_each)
    qmin = -qmax
    return Network(nb=nb, base_mva=100.0, bus_type=bus_type, pd=pd, qd=qd,
                   vmin=np.full(nb, 0.9), vmax=np.full(nb, 1.1), f=f, t=t, r=r,
                   x=x, b=b, rate=rate, gen_bus=gen_bus, c2=c2, c1=c1, c0=c0,
                   pmin=pmin, pmax=pmax, qmin=qmin, qmax=qmax, name=name,
                   seed=seed)


# Named stand-ins (sizes from the paper's Table 1 where a case exists).
def case9(seed: int = 1) -> Network:
    """9-bus ring, 3 generator buses (1 reference), loads at the 6 PQ buses,
    Pd ~ U[0.5, 1.5] p.u., no line limits, wide line-data ranges. The default
    seed is the first one whose OPF the oracle's interior-point method solves
    from the flat start (seeds 0, 2, 4 and 7 end in a failed line search)."""
    return make_network(9, 9, 3, seed=seed, load_frac=1.0, pd_range=(0.5, 1.5),
                        rated=False, ring=True, name="syn9", lines="wide")


def case118(seed: int = 0) -> Network:
    return make_network(118, 186, 54, seed=seed, load_frac=0.6, name="syn118")


def case300(seed: int = 0) -> Network:
    return make_network(300, 411, 69, seed=seed, load_frac=0.6, name="syn300")


def case1354(seed: int = 0) -> Network:
    return make_network(1354, 1991, 260, seed=seed, load_frac=0.6, name="syn1354")


def case9241(seed: int = 0) -> Network:
    return make_network(9241, 16049, 1445, seed=seed, load_frac=0.7, name="syn9241")


def small(nb: int, nl: int, ng: int, seed: int = 0, rated: bool = True) -> Network:
    """Tiny networks for brute-force pins (2-, 3-, 5-bus ...)."""
    return make_network(nb, nl, ng, seed=seed, load_frac=0.8, pd_range=(0.2, 1.0),
                        rated=rated, name=f"syn{nb}")


def scale_loads(net: Network, seed: int, lo: float = 0.8, hi: float = 1.2) -> Network:
    """Load scenario: every bus load scaled independently by U[lo, hi]."""
    rng = np.random.default_rng(seed)
    s = rng.uniform(lo, hi, net.nb)
    return net.copy(pd=net.pd * s, qd=net.qd * s, seed=seed,
                    name=f"{net.name}-s{seed}")


@dataclass
class RandomIterate:
    """Random primal-dual point, drawn per bus/generator/constraint.

    theta[nb] (reference entry ignored), vm[nb], pg[ng], lam_p[nb], lam_q[nb]
    (entries of buses without the matching balance row are ignored), y[m],
    sig_theta/sig_vm[nb], sig_pg[ng], sig_s[m].
    """
    theta: np.ndarray
    vm: np.ndarray
    pg: np.ndarray
    lam_p: np.ndarray
    lam_q: np.ndarray
    y: np.ndarray
    sig_vm: np.ndarray
    sig_pg: np.ndarray
    sig_s: np.ndarray


def random_iterate(net: Network, m: int, seed: int, *, lam_scale: float = 50.0,
                   y_scale: float = 5.0, sig_range=(1e-2, 1e2)) -> RandomIterate:
    rng = np.random.default_rng(10_000 + seed)
    nb, ng = net.nb, net.ng
    lo, hi = np.log10(sig_range[0]), np.log10(sig_range[1])
    return RandomIterate(
        theta=rng.normal(0.0, 0.1, nb),
        vm=rng.uniform(0.95, 1.05, nb),
        pg=rng.uniform(net.pmin, np.maximum(net.pmax, net.pmin + 1e-3)),
        lam_p=rng.normal(0.0, lam_scale, nb),
        lam_q=rng.normal(0.0, lam_scale, nb),
        y=rng.uniform(0.0, y_scale, m),
        sig_vm=10.0 ** rng.uniform(lo, hi, nb),
        sig_pg=10.0 ** rng.uniform(lo, hi, ng),
        sig_s=10.0 ** rng.uniform(lo, hi, m),
    )


def random_vector(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    return np.random.default_rng(20_000 + seed).normal(0.0, scale, n)
