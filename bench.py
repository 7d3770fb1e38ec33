#!/usr/bin/env python
"""Throughput of the condensation hot path on one MI355X.

One step = one pass of the whole hot path on one synthetic iterate of the
1354-bus network: derivative values, refactorisation of G_x, K_cond (all nu
columns) with the condensed right-hand side, dense Cholesky + solve for p_u,
and the recovery of (p_x, p_s, p_lambda, p_y) -- what one iteration of the
linearize-then-reduce IPM spends on linear algebra (Algorithm 1). The value is
condensations per second with every input resident in HBM. The "ipm" entry
reports the second half of the metric: IPM iterations per second of the full
method (rh_ipm_step) solving the same network from the flat start; "batched"
the batched form (rh_batch_*) over 112 instances of uneven size.

Prints ONE JSON line (rank 0). Runs on one GPU only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("reduced-Hessian condensations/s + IPM iters/s, 1354-bus FP64; "
          "plain vs batched/adjoint")
FP64_PEAK_TFLOPS = 78.6          # MI355X dense FP64 (MFMA)
HBM_PEAK_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_condense_syn1354_pmc.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2203_11875_amd", "csrc", "kernels.hip")
# Paper context (V100, Table 3, 1354pegase: 40 iterations, 0.29 s reduction)
PAPER_CONTEXT = {"hardware": "NVIDIA V100 (paper, Table 3)", "case": "1354pegase",
                 "condensations_per_s_derived": 138.0}


def workload(name):
    import synthnet
    if name == "syn1354":
        return synthnet.case1354(0)
    if name == "syn9241":
        return synthnet.case9241(0)
    if name == "syn118":
        return synthnet.case118(0)
    if name == "syn9":
        return synthnet.case9(1)
    raise SystemExit(f"unknown workload {name}")


def iterate(G, net, seed=0):
    """Seeded iterate in the library's variable order (rh_get_index_maps).
    Multipliers and barrier terms of a late-stage iterate: K_cond is positive
    definite, so each step factorises once (an IPM step with delta_w = 0)."""
    import numpy as np
    import synthnet
    xk, xb, uk, ur = G.index_maps()
    it = synthnet.random_iterate(net, G.m, seed, lam_scale=1.0, sig_range=(10.0, 1e4))
    x = np.where(xk == 0, it.theta[xb], it.vm[xb])
    lam = np.where(xk == 0, it.lam_p[xb], it.lam_q[xb])
    sx = np.where(xk == 0, 0.0, it.sig_vm[xb])
    u = np.where(uk == 1, it.vm[np.minimum(ur, net.nb - 1)], it.pg[np.minimum(ur, net.ng - 1)])
    su = np.where(uk == 1, it.sig_vm[np.minimum(ur, net.nb - 1)],
                  it.sig_pg[np.minimum(ur, net.ng - 1)])
    r = synthnet.random_vector(G.nu + 2 * G.nx + 2 * G.m, seed + 1)
    return x, u, lam, it.y.copy(), sx, su, it.sig_s.copy(), r


def batched_run(api, torch, steps, warmup):
    """Batched condensation (rh_batch_*): 64 load scenarios of the 1354-bus
    network (every bus load scaled by U[0.8, 1.2]), 32 synthetic 118-bus and
    16 synthetic 300-bus networks in one batch; a step is one batched
    condensation (all columns with the right-hand side) plus one batched
    solve with recovery, every kernel one launch for all 112 instances."""
    import numpy as np
    import synthnet
    base = synthnet.case1354(0)
    nets = ([synthnet.scale_loads(base, s) for s in range(1, 65)]
            + [synthnet.case118(s) for s in range(32)]
            + [synthnet.case300(s) for s in range(16)])
    dev = torch.device("cuda", 0)
    T = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=dev)
    Gs = [api.Net(n) for n in nets]
    pts = [tuple(map(T, iterate(G, n, seed=i))) for i, (G, n) in enumerate(zip(Gs, nets))]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    B = api.Batch(Gs, stream=stream)
    delta = np.zeros(len(nets))

    def step():
        Ks, rhss = B.condense(pts)
        _, st = B.solve(Ks, delta, rhss, [p[7] for p in pts])
        return st

    with torch.cuda.stream(stream):
        for _ in range(max(1, warmup)):
            st = step()
            for _ in range(20):       # inertia correction per instance, as in an IPM iteration
                bad = [i for i, c in enumerate(st) if c == 1]
                if not bad:
                    break
                for i in bad:
                    delta[i] = 1e-4 if delta[i] == 0.0 else delta[i] * 8.0
                st = step()
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        stream.synchronize()
        el = time.perf_counter() - t0
        # the same step captured in a HIP graph and replayed
        B.capture(pts, delta)
        for _ in range(5):
            B.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            B.replay()
        stream.synchronize()
        el_graph = time.perf_counter() - t0
        # each replay on its own, timed with events on the batch stream
        import numpy as np
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(max(steps, 10))]
        for a, b in evs:
            a.record(stream)
            B.replay()
            b.record(stream)
            stream.synchronize()
        per = np.array([a.elapsed_time(b) for a, b in evs])
    B.close()
    n = len(nets)
    return {"instances": n, "condensations_per_s": n * steps / el,
            "ms_per_batch_step": 1e3 * el / steps,
            "graph_condensations_per_s": n * steps / el_graph,
            "graph_ms_per_batch_step": 1e3 * el_graph / steps, "steps": steps,
            "graph_replay_ms": {"p10": float(np.percentile(per, 10)),
                                "p50": float(np.median(per)),
                                "p90": float(np.percentile(per, 90))},
            "graph_condensations_per_s_median": n / (float(np.median(per)) * 1e-3),
            "composition": "64 x syn1354 load scenarios (nu 519), 32 x syn118 (nu 107), "
                           "16 x syn300 (nu 137)",
            "step": "batched eval + refactor + condense + symmetrize + Cholesky + solve + "
                    "recovery, one launch per kernel for all instances",
            "delta_w_nonzero": int((delta > 0).sum())}


def differentiated_run(api, torch, count=16):
    """Differentiated OPF (api.OPFLayer): load scenarios of the 1354-bus
    network (every bus load scaled by U[0.8, 1.2], scenario seeds 1..count),
    each solved to a scaled KKT error of 1e-8 (forward) and differentiated
    (backward: gradient of Pg . w_pg + Vm . w_vm + f in (Pd, Qd), one adjoint
    solve through the condensed KKT system)."""
    import numpy as np
    import synthnet
    base = synthnet.case1354(0)
    dev = torch.device("cuda", 0)
    layer = api.OPFLayer(base, tol=1e-8)
    rng = np.random.default_rng(0)
    w_pg = torch.as_tensor(rng.standard_normal(base.ng), device=dev)
    w_vm = torch.as_tensor(rng.standard_normal(base.nb), device=dev)
    scen = [synthnet.scale_loads(base, s) for s in range(1, count + 1)]
    loads = [(torch.as_tensor(n.pd, device=dev), torch.as_tensor(n.qd, device=dev)) for n in scen]
    # one untimed scenario (first use of every kernel)
    pd = loads[0][0].clone().requires_grad_(True)
    pg, vm, f = layer(pd, loads[0][1])
    ((pg * w_pg).sum() + (vm * w_vm).sum() + f).backward()
    torch.cuda.synchronize()
    t_fwd = t_bwd = 0.0
    iters = 0
    for pdv, qdv in loads:
        pd = pdv.clone().requires_grad_(True)
        qd = qdv.clone().requires_grad_(True)
        t0 = time.perf_counter()
        pg, vm, f = layer(pd, qd)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ((pg * w_pg).sum() + (vm * w_vm).sum() + f).backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_fwd += t1 - t0
        t_bwd += t2 - t1
        iters += int(layer.last_info["iter"])
    return {"scenarios": count, "scenarios_per_s": count / (t_fwd + t_bwd),
            "forward_ms": 1e3 * t_fwd / count, "backward_ms": 1e3 * t_bwd / count,
            "ipm_iterations_mean": iters / count, "tol": 1e-8,
            "step": "forward: IPM from the flat start to 1e-8; backward: evaluation, "
                    "condensation with the adjoint right-hand side, Cholesky, recovery, "
                    "load-gradient scatter"}


def concurrent_scenarios(api, torch, count=16, workers=4):
    """The differentiated OPF scenarios of differentiated_run solved by
    `workers` host threads at once, each with its own network handle and HIP
    stream (the solver is latency-bound: one scenario leaves most of the chip
    idle). Reports the aggregate rate and checks every gradient against a
    one-at-a-time solve bit for bit."""
    import threading
    import numpy as np
    import synthnet
    base = synthnet.case1354(0)
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(0)
    w_pg = torch.as_tensor(rng.standard_normal(base.ng), device=dev)
    w_vm = torch.as_tensor(rng.standard_normal(base.nb), device=dev)
    scen = [synthnet.scale_loads(base, s) for s in range(1, count + 1)]
    layers = [api.OPFLayer(base, tol=1e-8, stream=torch.cuda.Stream()) for _ in range(workers)]
    out = [None] * count
    iters = [0] * count

    def run(layer, k):
        with torch.cuda.stream(layer.net.stream):
            pd = torch.as_tensor(scen[k].pd, device=dev).requires_grad_(True)
            qd = torch.as_tensor(scen[k].qd, device=dev).requires_grad_(True)
            pg, vm, f = layer(pd, qd)
            iters[k] = int(layer.last_info["iter"])
            ((pg * w_pg).sum() + (vm * w_vm).sum() + f).backward()
            layer.net.stream.synchronize()
            out[k] = (pd.grad.cpu().numpy(), qd.grad.cpu().numpy())

    def worker(w):
        for k in range(w, count, workers):
            run(layers[w], k)

    for w in range(workers):          # untimed first use of every handle
        run(layers[w], w)
    ref = [out[w] for w in range(workers)]
    torch.cuda.synchronize()
    threads = [threading.Thread(target=worker, args=(w,)) for w in range(workers)]
    t0 = time.perf_counter()
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    same = all(np.array_equal(out[w][0], ref[w][0]) and np.array_equal(out[w][1], ref[w][1])
               for w in range(workers))
    return {"scenarios": count, "workers": workers, "scenarios_per_s": count / el,
            "ipm_iters_per_s": sum(iters) / el, "ipm_iterations_mean": sum(iters) / count,
            "repeatable": bool(same),
            "step": "forward (IPM to 1e-8) + backward per scenario, scenarios spread over "
                    "host threads with one handle and stream each"}


def batched_scenarios(api, torch, count=16):
    """The differentiated OPF scenarios of differentiated_run as one
    api.OPFBatchLayer call: the forward solves all scenarios in lockstep with
    one batched condensation and solve per round; the backward batches the
    adjoint solves of all scenarios."""
    import numpy as np
    import synthnet
    base = synthnet.case1354(0)
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(0)
    w_pg = torch.as_tensor(rng.standard_normal(base.ng), device=dev)
    w_vm = torch.as_tensor(rng.standard_normal(base.nb), device=dev)
    scen = [synthnet.scale_loads(base, s) for s in range(1, count + 1)]
    layer = api.OPFBatchLayer(base, count, tol=1e-8)
    pd0 = torch.as_tensor(np.stack([n.pd for n in scen]), device=dev)
    qd0 = torch.as_tensor(np.stack([n.qd for n in scen]), device=dev)

    def run():
        pd = pd0.clone().requires_grad_(True)
        qd = qd0.clone().requires_grad_(True)
        t0 = time.perf_counter()
        pg, vm, f = layer(pd, qd)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ((pg * w_pg).sum() + (vm * w_vm).sum() + f.sum()).backward()
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1

    run()                               # untimed first use of every handle
    tf, tb = run()
    iters = sum(int(i["iter"]) for i in layer.last_infos)
    return {"scenarios": count, "scenarios_per_s": count / (tf + tb),
            "forward_ms": 1e3 * tf, "backward_ms": 1e3 * tb,
            "ipm_iters_per_s_forward": iters / tf, "ipm_iterations_mean": iters / count,
            "step": "forward: all scenarios in lockstep to 1e-8 (rh_ipm_batch_step); "
                    "backward: the adjoint solves of all scenarios in one batched "
                    "condensation and solve (rh_ipm_batch_backward)"}


def _progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def other_stages(info, phases, steps):
    """The step's other large stages and what bounds them: the refactorisation
    is one work-group walking the level sets of L (a dependency chain, not a
    bandwidth or MFMA limit); the Cholesky of the nu x nu condensed matrix is
    n^3 / 3 flops on FP64 MFMA in one launch per 32-column panel, then one
    matrix-vector product per inverse super-block (and one between two of
    them) for the backward substitution."""
    nu = info["nu"]
    ref_us = 1e3 * phases["refactor"][0] / steps
    chol_us = 1e3 * phases["cholesky"][0] / steps
    flops = nu ** 3 / 3.0
    tf = flops / (chol_us * 1e-6) / 1e12
    return {"refactor": {"us": ref_us, "bound": "latency", "levels": info["levels_lower"],
                         "us_per_level": ref_us / max(1, info["levels_lower"])},
            "cholesky": {"us": chol_us, "bound": "mfma", "flops": flops, "achieved": tf,
                         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFLOPS,
                         "launches": chol_launches(nu)}}


def chol_launches(n):
    """Kernel launches of one Cholesky + solve of order n: one per 32-column
    panel, 2 s - 1 for the backward substitution over s super-blocks (one
    super-block up to 24 panels, 16-panel super-blocks above), and the
    status clear."""
    nbk = (n + 31) // 32
    sb = nbk if nbk <= 24 else 16
    return nbk + 2 * ((nbk + sb - 1) // sb) - 1 + 1


def algorithmic_bytes(info, ncols):
    """Paper-dataflow bytes of one condensation launch: every stage reads its
    input panel and writes its output panel (8 (12 nx + 5 nu) bytes per
    column) plus one pass over the matrix data per stage (12 bytes per
    stored nonzero: value + index)."""
    nx, nu = info["nx"], info["nu"]
    per_col = 8 * (12 * nx + 5 * nu)
    matrix = 12 * (2 * info["nnz_lu"] + info["nnz_k"] + 2 * info["nnz_gu"])
    return per_col * ncols + matrix, per_col


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source (else None)."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    txt = open(PMC_SUMMARY).read()
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    m_sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_sha or not m_b or m_sha.group(1) != sha:
        return None
    return float(m_b.group(1))


def ipm_run(api, net, torch, max_iter):
    """IPM iterations per second: Algorithm 1 (rh_ipm_step) from the flat
    start to a scaled KKT error of 1e-6, every iteration timed (evaluation,
    condensation, Cholesky with inertia correction, recovery, filter line
    search)."""
    G = api.Net(net)
    ipm = api.Ipm(G, tol=1e-6, max_iter=max_iter)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, code, info, trace = 0, 0, {}, []
    while iters <= max_iter:
        code, info = ipm.step()
        trace.append(float(f"{info['err']:.3g}"))
        if code != 0 or info["converged"]:
            break
        iters += 1
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ipm.close()
    G.close()
    return {"iters_per_s": iters / el if iters else 0.0, "iterations": iters,
            "ms_per_iter": 1e3 * el / max(1, iters), "converged": bool(info.get("converged")),
            "status": int(code), "objective": info.get("obj"), "kkt_error": info.get("err"),
            "tol": 1e-6, "start": "flat (theta 0, Vm 1, Pg mid-range)",
            "kkt_error_per_iteration": trace}


def ipm_batched_run(api, torch, count=16, max_iter=150):
    """Algorithm 1 on `count` load scenarios of the 1354-bus network (every bus
    load scaled by U[0.8, 1.2], seeds 1..count) stepped in lockstep
    (rh_ipm_batch_step: batched condensation and solve, per-scenario line
    searches on their own streams) from the flat start to 1e-6; aggregate
    IPM iterations per second."""
    import synthnet
    base = synthnet.case1354(0)
    nets = [synthnet.scale_loads(base, s) for s in range(1, count + 1)]
    Gs = [api.Net(n, stream=torch.cuda.Stream()) for n in nets]
    ipms = [api.Ipm(G, tol=1e-6, max_iter=max_iter) for G in Gs]
    B = api.Batch(Gs, stream=torch.cuda.Stream())
    IB = api.IpmBatch(B, ipms)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = [0] * count
    done = [False] * count
    codes = [0] * count
    rounds = 0
    while not all(done) and rounds <= max_iter:
        rounds += 1
        for i, (code, info) in enumerate(IB.step()):
            if done[i]:
                continue
            codes[i] = code
            if code != 0 or info["converged"]:
                done[i] = True
            else:
                iters[i] += 1
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    B.close()
    return {"scenarios": count, "iters_per_s": sum(iters) / el, "lockstep_rounds": rounds,
            "iterations_total": sum(iters), "converged": sum(1 for c in codes if c == 0),
            "ms_per_round": 1e3 * el / max(1, rounds), "tol": 1e-6,
            "step": "per round: every scenario's evaluation, one batched condensation + "
                    "solve for all, per-scenario inertia retries and filter line search"}


def redlin_run(api, net, torch, max_iter):
    """RedLin (Algorithm 2, rh_redlin_step) from the flat start to a scaled
    KKT error of 1e-6: iterations per second, with the projection's
    Newton-Raphson steps and its share of the time."""
    G = api.Net(net)
    rl = api.RedLin(G, tol=1e-6, max_iter=max_iter)
    G.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, code, info, pf, trace = 0, 0, {}, 0, []
    while iters <= max_iter:
        code, info = rl.step()
        trace.append(float(f"{info['err']:.3g}"))
        if code != 0 or info["converged"]:
            break
        iters += 1
        pf += info["pf_iters"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phases = G.profile_read()
    rl.close()
    G.close()
    return {"iters_per_s": iters / el if iters else 0.0, "iterations": iters,
            "ms_per_iter": 1e3 * el / max(1, iters), "converged": bool(info.get("converged")),
            "status": int(code), "objective": info.get("obj"), "pf_newton_steps": pf,
            "projection_ms_per_iter": phases["project"][0] / max(1, iters),
            "phases_ms_per_iter": {k: v[0] / max(1, iters) for k, v in phases.items()},
            "tol": 1e-6, "start": "flat (theta 0, Vm 1, Pg mid-range), projected",
            "kkt_error_per_iteration": trace}


def cpu_baseline(net, args_np, seconds):
    """The oracle's full step (dense LU of G_x, explicit K_cond, RHS, Cholesky,
    recovery) on the host, repeated for a bounded time."""
    import numpy as np
    from oracle.model import Model
    from oracle import reduction as R, cholesky as OC
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    M = Model(net)
    x, u, lam, y, sx, su, ss, r = args_np
    done = 0
    t0 = time.perf_counter()
    while True:
        B = R.kkt_blocks(M, x, u, lam, y, sx, su, ss)
        S, lu = R.sensitivity(B)
        Kc = R.symmetrize(R.condensed_matrix(B, S))
        b, _, _ = R.condensed_rhs(B, r, S, lu)
        L, delta = OC.factor_with_correction(Kc)
        pu = OC.solve_with_factor(L, b)
        R.recover(B, r, pu, S, lu)
        done += 1
        el = time.perf_counter() - t0
        if el >= seconds or done >= 200:
            break
    # one iteration of the oracle's Algorithm 1 (sparse LU of K_aug) from the
    # flat start, a few times
    from oracle.ipm import LinRedIPM, IPMOptions, flat_start
    o = LinRedIPM(net, IPMOptions(tol=1e-6, linear_solver="sparse"))
    st = o.initial_state(*flat_start(o.M))
    t1 = time.perf_counter()
    its = 0
    while its < 3 and time.perf_counter() - t1 < seconds:
        o.iterate(st)
        its += 1
    ipm_s = (time.perf_counter() - t1) / its
    return {"value": done / el, "unit": "condensations/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"{done} full steps of the oracle on {net.name} (numpy/scipy FP64, "
                      f"{el:.1f} s); then {its} iterations of its Algorithm 1",
            "cpu_model": _cpu_model(), "blas": _blas_info(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "ipm_iters_per_s": 1.0 / ipm_s,
            "ipm_iteration": "oracle Algorithm 1 from the flat start: model derivatives, "
                             "inertia test on the dense K_cond, sparse LU solve of K_aug, "
                             "filter line search"}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _blas_info():
    try:
        from threadpoolctl import threadpool_info
        return [{k: t.get(k) for k in ("internal_api", "version", "threading_layer",
                                       "num_threads", "architecture")}
                for t in threadpool_info() if t.get("user_api") == "blas"]
    except Exception as e:       # threadpoolctl missing or failing: say so
        return f"unavailable ({type(e).__name__})"


def workload_name(net, key):
    if key == "syn1354":
        return (f"{net.name}: seeded synthetic 1354-bus stand-in for 1354pegase (nb {net.nb}, "
                f"nl {net.nl}, ng {net.ng}; transmission-like line data x ~ U[0.005, 0.05], "
                f"r = x U[0.1, 0.3], b ~ U[0, 0.1], rate ~ U[2, 8], loads Pd ~ U[0.05, 0.5] "
                f"on 60% of buses)")
    if key == "syn9241":
        return (f"{net.name}: seeded synthetic 9241-bus stand-in for 9241pegase (nb {net.nb}, "
                f"nl {net.nl}, ng {net.ng}; line data as syn1354, loads on 70% of buses)")
    return net.name


def single_instance(api, torch, net, steps, warmup, width=0, lds=1, key="syn1354", waves=0):
    """One instance, one step = eval + refactor + condense (nu + 1 columns) +
    symmetrize + Cholesky + solve + recovery on a seeded iterate; timed over
    `steps` steps after `warmup`, with per-phase HIP events on the library's
    stream and a per-step spread; the condensation kernel's roofline."""
    import numpy as np
    dev = torch.device("cuda", 0)
    G = api.Net(net, panel_width=width, lds_panel=lds, cond_waves=waves)
    args_np = iterate(G, net)
    T = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=dev)
    x, u, lam, y, sx, su, ss, r = map(T, args_np)
    nu = G.nu
    K = torch.empty((nu, nu), dtype=torch.float64, device=dev)
    rhs = torch.empty(nu, dtype=torch.float64, device=dev)

    def step(delta):
        G.condense_reduced_hessian(x, u, lam, y, sx, su, ss, r=r, K=K, rhs=rhs)
        p, code = G.solve_condensed_kkt(K, delta, rhs, r)
        return code

    delta = 0.0
    for _ in range(max(1, warmup)):
        code = step(delta)
        while code == 1:        # inertia correction as in an IPM iteration
            delta = 1e-4 if delta == 0.0 else delta * 8.0
            code = step(delta)
        if code != 0:
            raise SystemExit(f"solve failed with status {code}")
    torch.cuda.synchronize()
    G.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(delta)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phases = G.profile_read()
    G.profile_enable(False)
    # per-step spread: the same step timed one at a time with events on the
    # library's stream (outside the timed region above)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(max(steps, 10))]
    for a, b in evs:
        a.record(G.stream)
        step(delta)
        b.record(G.stream)
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in evs])
    spread = {"p10": float(np.percentile(per, 10)), "p50": float(np.median(per)),
              "p90": float(np.percentile(per, 90))}
    graph = graph_replay(api, torch, G, (x, u, lam, y, sx, su, ss, r), delta,
                         reps=max(50, steps))
    cond_ms, cond_calls = phases["condense"]
    kern_s = cond_ms / 1e3 / max(1, cond_calls)
    ncols = nu + 1
    alg_bytes, per_col = algorithmic_bytes(G.info, ncols)
    achieved = alg_bytes / kern_s / 1e9
    traffic = measured_traffic() if key == "syn1354" else None
    return {
        "_net": G, "_args": args_np,
        "value": steps / el,
        "ms_per_step": 1e3 * el / steps,
        "config": {"workload": workload_name(net, key),
                   "nx": G.nx, "nu": nu, "m": G.m,
                   "step": "eval + refactor + condense (nu+1 columns) + symmetrize + "
                           "Cholesky + solve + recovery",
                   "panel_width": G.info["panel_width"], "lds_panel": G.info["lds_panel"],
                   "cond_waves": G.info["cond_waves"],
                   "ordering": "minimum degree with a level term (2 degree + level)",
                   "levels": G.info["levels_lower"], "nnz_lu": G.info["nnz_lu"],
                   "delta_w": delta},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "k_condense", "kernel_avg_us": kern_s * 1e6,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "bytes_per_column": per_col, "columns_per_launch": ncols},
        "phases_ms_per_step": {k: v[0] / steps for k, v in phases.items()},
        "step_ms_spread": spread,
        "graph_replay": graph,
        "condensation_only_per_s": 1e3 / sum(phases[k][0] / steps
                                              for k in ("eval", "refactor", "condense",
                                                        "symmetrize")),
        "other_stages": other_stages(G.info, phases, steps),
    }


def graph_replay(api, torch, G, point, delta, reps=50, warmup=5):
    """The same step (evaluation, refactorisation, condensation with the
    right-hand side, Cholesky, solve, recovery) captured once in a HIP graph,
    as a one-member batch (the
    batched kernels run the single-instance bodies: same results bit for
    bit), and replayed: `warmup` replays, then `reps` replays each timed with
    HIP events on the batch's stream. Milliseconds p10 / p50 / p90 and the
    rate at the median."""
    import numpy as np
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    B = api.Batch([G], stream=stream)
    with torch.cuda.stream(stream):
        B.capture([point], np.array([delta]))
        for _ in range(warmup):
            B.replay()
        stream.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for a, b in evs:
            a.record(stream)
            B.replay()
            b.record(stream)
        stream.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in evs])
    B.close()
    p50 = float(np.median(per))
    return {"replays": reps, "ms_p10": float(np.percentile(per, 10)), "ms_p50": p50,
            "ms_p90": float(np.percentile(per, 90)), "condensations_per_s_p50": 1e3 / p50,
            "step": "eval + refactor + condense (nu+1 columns) + symmetrize + Cholesky + solve "
                    "+ recovery as one captured graph (a one-member batch)"}


def large_block(api, torch, steps, warmup):
    """The 9241-bus stand-in (nx 17036, nu 2889): one instance, the same step;
    condensations per second, the condensation kernel's HBM roofline and the
    dense Cholesky's FP64-MFMA roofline at n = 2889."""
    import synthnet
    net = synthnet.case9241(0)
    one = single_instance(api, torch, net, steps, warmup, key="syn9241")
    G = one.pop("_net")
    one.pop("_args")
    G.close()
    out = {"value": one["value"], "unit": "condensations/s",
           "ms_per_step": one["ms_per_step"], "steps": steps, "warmup": warmup}
    out.update({k: v for k, v in one.items() if k not in ("value", "ms_per_step")})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="syn1354")
    ap.add_argument("--width", type=int, default=0)
    ap.add_argument("--lds", type=int, default=1)
    ap.add_argument("--waves", type=int, default=0,
                    help="waves per condensation work-group (0: the library's choice)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ipm", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-diff", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 9241-bus block")
    ap.add_argument("--large-steps", type=int, default=5)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--ipm-iters", type=int, default=150)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one device copy of 512 MiB first (a plain copy kernel of known "
                         "size that scales the rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the condensation of one instance runs on a "
              "single MI355X (multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    from paper_2203_11875_amd import api

    net = workload(args.workload)
    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    one = single_instance(api, torch, net, args.steps, args.warmup, args.width, args.lds,
                          key=args.workload, waves=args.waves)
    G, args_np = one.pop("_net"), one.pop("_args")
    line = {
        "metric": METRIC,
        "value": one["value"],
        "unit": "condensations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": one["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": one["config"],
        "roofline": one["roofline"],
    }
    line.update({k: v for k, v in one.items() if k not in line and k != "value"})
    line["paper_context"] = PAPER_CONTEXT
    x, u, lam, y, sx, su, ss, r = (torch.as_tensor(np.asarray(a, np.float64), device=dev)
                                   for a in args_np)
    _progress("single-instance steps done")
    if not args.no_large:
        line["syn9241"] = large_block(api, torch, args.large_steps, 2)
        _progress("syn9241 done")
    if not args.no_ipm:
        line["ipm"] = ipm_run(api, net, torch, args.ipm_iters)
        _progress("ipm done")
    if not args.no_batch:
        line["batched"] = batched_run(api, torch, args.batch_steps, 2)
        _progress("batched condensation done")
        best, times = api.autotune(net, (x, u, lam, y, sx, su, ss, r), widths=(1, 2, 4),
                                   lds=(1, 0), reps=3, record=False)
        line["autotune"] = {"best": {"panel_width": best[0], "lds_panel": best[1],
                                     "cond_waves": best[2]},
                            "condensation_us": {f"w{w}_lds{l}_nw{nw}": round(v, 1)
                                                for (w, l, nw), v in times.items()}}
    if not args.no_ipm:
        line["redlin"] = redlin_run(api, net, torch, args.ipm_iters)
        _progress("redlin done")
    if not args.no_ipm and not args.no_batch:
        line["ipm_batched"] = ipm_batched_run(api, torch, 16, args.ipm_iters)
        _progress("lockstep ipm done")
    if not args.no_diff:
        line["differentiated"] = differentiated_run(api, torch)
        line["differentiated"]["concurrent"] = concurrent_scenarios(api, torch, 16,
                                                                    args.workers)
        line["differentiated"]["batched"] = batched_scenarios(api, torch, 16)
        _progress("differentiated done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(net, args_np, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
