"""Shared test helpers: turn seeded per-bus draws into (x, u, lambda, y, Sigma)
vectors in the natural variable order that both the oracle and the C ABI use."""
from __future__ import annotations

import numpy as np

import synthnet


def iterate_vectors(M, it):
    """(x, u, lam, y, sig_x, sig_u, sig_s) from a synthnet.RandomIterate."""
    net = M.net
    x, u = M.join(it.theta, it.vm, it.pg)
    lam = np.concatenate([it.lam_p[M.nonref], it.lam_q[M.pq]])
    sx = np.zeros(M.nx)
    vmx = M.x_kind == 1
    sx[vmx] = it.sig_vm[M.x_bus[vmx]]
    su = np.concatenate([it.sig_vm[np.asarray(net.gen_bus)],
                         it.sig_pg[M.nonref_gens]])
    return x, u, lam, it.y.copy(), sx, su, it.sig_s.copy()


def random_point(M, seed, **kw):
    it = synthnet.random_iterate(M.net, M.m, seed, **kw)
    return iterate_vectors(M, it)


def balanced_control(M, vg=1.02):
    """A control near which the power flow is solvable: generator voltages vg,
    non-reference generators share the total load evenly."""
    net = M.net
    pg = np.full(M.ng, net.pd.sum() / M.ng)
    theta = np.zeros(M.nb)
    vm = np.ones(M.nb)
    vm[np.asarray(net.gen_bus)] = vg
    return M.join(theta, vm, pg)


def residual_vector(M, seed, scale=1.0):
    return synthnet.random_vector(M.nu + 2 * M.nx + 2 * M.m, seed, scale)


def kcond_entry_error(Kg, Kc):
    """Largest entrywise error of K_cond, each entry (i, j) measured against
    sqrt(|K_ii K_jj|) of the reference (the scale a symmetric matrix's
    entries are bounded by when it is definite)."""
    d = np.sqrt(np.abs(np.diag(Kc)))
    scale = np.outer(d, d)
    scale = np.where(scale > 0, scale, np.abs(Kc).max())
    return float((np.abs(np.asarray(Kg) - Kc) / scale).max())


STEP_BLOCKS = ("p_u", "p_x", "p_s", "p_lambda", "p_y")


def step_block_errors(got, want, nu, nx, m):
    """Error of each block of a packed step (p_u, p_x, p_s, p_lambda, p_y)
    relative to that block's own largest entry."""
    o = np.cumsum([0, nu, nx, m, nx, m])
    got, want = np.asarray(got), np.asarray(want)
    out = {}
    for k, name in enumerate(STEP_BLOCKS):
        g, w = got[o[k]:o[k + 1]], want[o[k]:o[k + 1]]
        if w.size == 0:
            continue
        ref = np.abs(w).max()
        out[name] = float(np.abs(g - w).max() / ref) if ref > 0 else float(np.abs(g).max())
    return out
