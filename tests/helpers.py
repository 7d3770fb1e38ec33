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
