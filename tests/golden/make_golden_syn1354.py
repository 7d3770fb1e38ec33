"""Writes the oracle's reference results for the 1354-bus stand-in.

Calls only the oracle (and the seeded network generator): the oracle's
Algorithm 1 (dense model, sparse LU of the augmented system) solved from the
flat start, and its implicit differentiation of the solution in the loads.

Outputs, next to this file:
* ipm_syn1354.json: for tol 1e-6 the iteration count, the optimal objective and
  the optimal control u; for tol 1e-8 the outputs (Pg, Vm, f) and the gradient
  of dpg . Pg + dvm . Vm + df f in (Pd, Qd) for the weights drawn by
  numpy.random.default_rng(11) (dpg ~ N(0, 1) per generator, then dvm ~ N(0, 1)
  per bus) and df = 1e-3;
* iterates_syn1354.npz: the inputs of one condensation at iterations 0, 10 and
  the last iteration of the tol 1e-6 run (x, u, lambda, y, Sigma_x, Sigma_u,
  Sigma_s, the residual r of the augmented system and the inertia shift
  delta_w the method used there), for parity checks at late, ill-conditioned
  iterates.

Usage: python tests/golden/make_golden_syn1354.py   (about 3 minutes)
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthnet  # noqa: E402
from oracle.ipm import LinRedIPM, IPMOptions, flat_start  # noqa: E402
from oracle import sensitivity as S  # noqa: E402

KEEP = (0, 10)


def _inv(d):
    return np.where(np.isfinite(d), 1.0 / np.where(np.isfinite(d), d, 1.0), 0.0)


def condensation_inputs(o, st, delta):
    """The arguments of one condensation + solve at state st, as the oracle
    IPM's step builds them (natural variable order)."""
    nu = o.nu
    mu = st.mu
    w, s = st.w, st.s
    x, u = o.split(w)
    dwl, dwu, dsl, dsu = o.slacks(w, s)
    sig_w = st.zl * _inv(dwl) + st.zu * _inv(dwu)
    sig_s = st.zsl * _inv(dsl) + st.zsu * _inv(dsu)
    gl = o.M.lagrangian_gradient(x, u, st.lam, st.y)
    r_w = gl - mu * _inv(dwl) + mu * _inv(dwu)
    r3 = st.y - mu * _inv(dsl) + mu * _inv(dsu)
    g, h, _ = o.evaluate(w, s)
    r = np.concatenate([r_w, r3, g, h + s])
    return {"x": x.copy(), "u": u.copy(), "lam": st.lam.copy(), "y": st.y.copy(),
            "sig_x": sig_w[nu:].copy(), "sig_u": sig_w[:nu].copy(), "sig_s": sig_s.copy(),
            "r": r, "delta_w": np.float64(delta), "mu": np.float64(mu),
            "obj_scale": np.float64(o.sigma_f)}


def run(tol, keep=()):
    net = synthnet.case1354(0)
    o = LinRedIPM(net, IPMOptions(tol=tol, linear_solver="sparse"))
    st = o.initial_state(*flat_start(o.M))
    kept = {}
    log = []
    while o.optimality_error(st, 0.0) > tol:
        if len(log) >= o.opt.max_iter:
            raise RuntimeError("oracle IPM did not converge")
        k = len(log)
        before = {f: getattr(st, f).copy() for f in ("w", "s", "lam", "y", "zl", "zu",
                                                     "zsl", "zsu")}
        dl0 = st.delta_last
        info = o.iterate(st)
        log.append(info)
        print(f"tol {tol:g} iteration {k}: obj {info['obj']:.10g} mu {info['mu']:.1e}",
              flush=True)
        if keep == "all" or k in keep:
            # the state the iteration started from, with the barrier parameter
            # and inertia shift the iteration used
            from oracle.ipm import IPMState
            pre = IPMState(mu=info["mu"], delta_last=dl0, **before)
            kept[k] = condensation_inputs(o, pre, info["delta_w"])
    return o, st, log, kept


def main():
    o6, st6, log6, kept = run(1e-6, keep="all")
    last = len(log6) - 1
    iterates = {}
    for k in sorted(set(KEEP) | {last}):
        tag = "last" if k == last else f"it{k}"
        for key, v in kept[k].items():
            iterates[f"{tag}_{key}"] = v
    iterates["last_index"] = np.int64(last)
    np.savez_compressed(os.path.join(HERE, "iterates_syn1354.npz"), **iterates)

    o8, st8, log8, _ = run(1e-8)
    net = o8.net
    rng = np.random.default_rng(11)
    dpg, dvm, df = rng.standard_normal(net.ng), rng.standard_normal(net.nb), 1e-3
    sw, ss = S.primal_dual_sigmas(o8, st8)
    gpd, gqd, _ = S.load_gradient(o8, st8.w, st8.s, st8.lam, st8.y, sw, ss, dpg, dvm, df,
                                  sparse=True)
    pg, vm, f = S.outputs(o8, st8.w, st8.s)
    out = {
        "source": "oracle/ipm.py (Algorithm 1, sparse LU of the augmented system) and "
                  "oracle/sensitivity.py on synthnet.case1354(0) from the flat start; "
                  "written by tests/golden/make_golden_syn1354.py",
        "tol_1e-6": {"iterations": len(log6), "objective": log6[-1]["obj"],
                     "obj_scale": o6.sigma_f, "u": st6.w[:o6.nu].tolist()},
        "tol_1e-8": {"iterations": len(log8), "objective": log8[-1]["obj"],
                     "pg": pg.tolist(), "vm": vm.tolist(), "f": f,
                     "weights": "numpy.random.default_rng(11): dpg ~ N(0,1) (ng), "
                                "dvm ~ N(0,1) (nb); df = 1e-3",
                     "grad_pd": gpd.tolist(), "grad_qd": gqd.tolist()},
    }
    with open(os.path.join(HERE, "ipm_syn1354.json"), "w") as fh:
        json.dump(out, fh)
        fh.write("\n")
    print("written", flush=True)


if __name__ == "__main__":
    main()
