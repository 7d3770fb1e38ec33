"""Oracle: derivatives of the OPF solution with respect to the loads
(test infrastructure).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this.

At a fixed barrier parameter mu, with the bound multipliers eliminated
(z = mu / bound slack), the barrier problem's first-order conditions are
F(w, s, lambda, y; p) = 0 with
    F_w      = grad f + G^T lambda + A^T y - mu / (w - wl) + mu / (wu - w)
    F_s      = y - mu / (s - sl) + mu / (su - s)
    F_lambda = g
    F_y      = h + s
and p = (Pd, Qd) the loads. The Jacobian of F in (w, s, lambda, y) is the
augmented matrix K_aug of eq. kktmatrix:normal (Section 2.2.1; the +I reading
of its (s, y) blocks, see oracle.reduction) with Sigma = mu / slack^2. By the
implicit function theorem the barrier solution z*(p) has
    dz*/dp = -K_aug^{-1} dF/dp,
and a scalar function L of outputs o(z) has
    dL/dp = -xi^T dF/dp,   xi = K_aug^{-1} (do/dz)^T dL/do
(K_aug is symmetric): one more solve with the matrix an iteration of
Algorithm 1 builds, so the reduction and condensation of Theorems 1 and 2
apply to it unchanged.

Where the loads enter F (the model of oracle.model):
* P balance at a non-reference bus i carries +Pd_i, Q balance at a PQ bus i
  carries +Qd_i;
* h_0 = Pg_ref = P_ref + Pd_ref carries +Pd_ref; h_{1+g} = Qg_g = Q_b + Qd_b
  at b = gen_bus[g] carries +Qd_b;
* F_w through grad f: the cost of Pg_ref contributes
  (2 c2_ref base^2 Pg_ref + c1_ref base) grad h_0, whose derivative in Pd_ref
  is 2 c2_ref base^2 grad h_0 (scaled costs, as the IPM's f).

The outputs are Pg of every generator (Pg_ref = -s_0, equal to h_0 at a
solution), Vm of every bus and the objective f with the network's own
(unscaled) costs, all functions of (w, s) only.

Readings: the derivative is that of the barrier solution at the IPM's final
mu (the problem is smooth there; at mu -> 0 it tends to the sensitivity of the
optimum where strict complementarity holds). At the IPM's final iterate the
primal-dual Sigma = z / slack stands for mu / slack^2 (they agree to the
solver's tolerance).
"""
from __future__ import annotations

import numpy as np

from . import reduction as R


def _inv(d):
    return np.where(np.isfinite(d), 1.0 / np.where(np.isfinite(d), d, 1.0), 0.0)


def offsets(ipm):
    """Start of each block of the unknowns (u, x, s, lambda, y) and the total."""
    nu, nx, m = ipm.nu, ipm.nx, ipm.m
    return np.cumsum([0, nu, nx, m, nx, m])


def barrier_residual(ipm, w, s, lam, y, mu):
    """F at (w, s, lambda, y) for barrier parameter mu, rows (w, s, lambda, y)."""
    x, u = ipm.split(w)
    gl = ipm.M.lagrangian_gradient(x, u, lam, y)
    dwl, dwu, dsl, dsu = ipm.slacks(w, s)
    g, h, _ = ipm.evaluate(w, s)
    return np.concatenate([gl - mu * _inv(dwl) + mu * _inv(dwu),
                           y - mu * _inv(dsl) + mu * _inv(dsu), g, h + s])


def barrier_sigmas(ipm, w, s, mu):
    """Sigma_w, Sigma_s of the barrier problem: mu / slack^2 on finite bounds."""
    dwl, dwu, dsl, dsu = ipm.slacks(w, s)
    return mu * (_inv(dwl) ** 2 + _inv(dwu) ** 2), mu * (_inv(dsl) ** 2 + _inv(dsu) ** 2)


def primal_dual_sigmas(ipm, st):
    """Sigma_w, Sigma_s of an IPM state: bound multiplier / bound slack."""
    dwl, dwu, dsl, dsu = ipm.slacks(st.w, st.s)
    return (st.zl * _inv(dwl) + st.zu * _inv(dwu), st.zsl * _inv(dsl) + st.zsu * _inv(dsu))


def kkt_matrix(ipm, w, s, lam, y, sig_w, sig_s):
    """Dense K_aug at the point (unknown order u, x, s, lambda, y)."""
    x, u = ipm.split(w)
    nu = ipm.nu
    B = R.kkt_blocks(ipm.M, x, u, lam, y, sig_w[nu:], sig_w[:nu], sig_s)
    return R.augmented_matrix(B)


def solve_barrier(ipm, w, s, lam, y, mu, max_iter=60):
    """Newton's method on F = 0 at fixed mu from a nearby point, with a
    fraction-to-the-boundary rule (0.995) keeping the bound slacks positive.
    Runs until the residual stops decreasing; returns (w, s, lam, y, |F|_inf)."""
    o = offsets(ipm)
    w, s, lam, y = (np.array(v, float) for v in (w, s, lam, y))
    F = barrier_residual(ipm, w, s, lam, y, mu)
    nrm = np.abs(F).max()
    for _ in range(max_iter):
        sw, ss = barrier_sigmas(ipm, w, s, mu)
        dz = np.linalg.solve(kkt_matrix(ipm, w, s, lam, y, sw, ss), -F)
        dw = dz[o[0]:o[2]]
        ds = dz[o[2]:o[3]]
        alpha = 1.0
        for d, step, sign in zip(ipm.slacks(w, s), (dw, dw, ds, ds), (1, -1, 1, -1)):
            q = sign * step
            sel = np.isfinite(d) & (q < 0)
            if sel.any():
                alpha = min(alpha, float(np.min(-0.995 * d[sel] / q[sel])))
        wn, sn = w + alpha * dw, s + alpha * ds
        lamn = lam + alpha * dz[o[3]:o[4]]
        yn = y + alpha * dz[o[4]:o[5]]
        Fn = barrier_residual(ipm, wn, sn, lamn, yn, mu)
        nn = np.abs(Fn).max()
        if not nn < nrm:
            break
        w, s, lam, y, F, nrm = wn, sn, lamn, yn, Fn, nn
    return w, s, lam, y, nrm


def outputs(ipm, w, s):
    """(Pg per generator, Vm per bus, f) at (w, s); f with unscaled costs."""
    M, net = ipm.M, ipm.net
    x, u = ipm.split(w)
    _, vm, pg = M.split(x, u)
    pg = np.array(pg, float)
    pg[M.ref_gen] = -s[0]
    B = M.base
    f = float(np.sum(net.c2 * (B * pg) ** 2 + net.c1 * (B * pg) + net.c0))
    return pg, np.array(vm, float), f


def output_jacobian(ipm, w, s):
    """d(Pg, Vm, f)/d(u, x, s, lambda, y): (ng + nb + 1) x n dense."""
    M, net = ipm.M, ipm.net
    o = offsets(ipm)
    ng, nb = M.ng, M.nb
    C = np.zeros((ng + nb + 1, o[-1]))
    pg, _, _ = outputs(ipm, w, s)
    B = M.base
    dcost = B * (2.0 * net.c2 * B * pg + net.c1)       # df / dPg_g
    for g in range(ng):
        if g == M.ref_gen:
            C[g, o[2]] = -1.0                            # Pg_ref = -s_0
            C[ng + nb, o[2]] = -dcost[g]
        else:
            C[g, M.u_pg[g]] = 1.0
            C[ng + nb, M.u_pg[g]] = dcost[g]
    for i in range(nb):
        k = M.u_vm[i] if M.u_vm[i] >= 0 else M.nu + M.x_vm[i]
        C[ng + i, k] = 1.0
    return C


def load_jacobian(ipm, w, s):
    """dF/d(Pd, Qd): n x 2 nb dense (columns Pd_0 .. Pd_{nb-1}, Qd_0 ..)."""
    M = ipm.M
    o = offsets(ipm)
    nb = M.nb
    Fp = np.zeros((o[-1], 2 * nb))
    x, u = ipm.split(w)
    _, A, _ = M.jacobians(x, u)
    a0 = np.asarray(A[[0], :].todense()).ravel()
    for k, i in enumerate(M.g_rows_p):
        Fp[o[3] + k, i] = 1.0
    for k, i in enumerate(M.g_rows_q):
        Fp[o[3] + len(M.g_rows_p) + k, nb + i] = 1.0
    Fp[o[4] + 0, M.ref] = 1.0
    Fp[o[0]:o[2], M.ref] = 2.0 * M.net.c2[M.ref_gen] * M.base ** 2 * a0
    for g in range(M.ng):
        Fp[o[4] + 1 + g, nb + M.net.gen_bus[g]] = 1.0
    return Fp


def output_sensitivity(ipm, w, s, lam, y, sig_w, sig_s):
    """d(Pg, Vm, f)/d(Pd, Qd) = -C K_aug^{-1} dF/dp: (ng + nb + 1) x 2 nb."""
    K = kkt_matrix(ipm, w, s, lam, y, sig_w, sig_s)
    return -output_jacobian(ipm, w, s) @ np.linalg.solve(K, load_jacobian(ipm, w, s))


def load_gradient(ipm, w, s, lam, y, sig_w, sig_s, dpg, dvm, df, sparse=False):
    """Gradient of L = dpg . Pg + dvm . Vm + df f with respect to (Pd, Qd):
    the adjoint xi = K_aug^{-1} C^T [dpg; dvm; df], then -dF/dp^T xi.
    Returns (grad_Pd, grad_Qd, xi) with xi in (u, x, s, lambda, y) order.
    sparse: solve with K_aug by a sparse LU (large networks) instead of a
    dense one."""
    c = output_jacobian(ipm, w, s).T @ np.concatenate([dpg, dvm, [df]])
    if sparse:
        import scipy.sparse.linalg as spla
        x, u = ipm.split(w)
        nu = ipm.nu
        B = R.kkt_blocks(ipm.M, x, u, lam, y, sig_w[nu:], sig_w[:nu], sig_s)
        lu = spla.splu(R.augmented_matrix_sparse(B), permc_spec="COLAMD",
                       diag_pivot_thresh=1.0)
        xi = lu.solve(c)
    else:
        xi = np.linalg.solve(kkt_matrix(ipm, w, s, lam, y, sig_w, sig_s), c)
    gp = -load_jacobian(ipm, w, s).T @ xi
    nb = ipm.M.nb
    return gp[:nb], gp[nb:], xi


def with_loads(ipm, pd, qd):
    """A copy of the solver on the same network with loads (pd, qd) and the
    same objective scale."""
    from .ipm import LinRedIPM
    other = LinRedIPM(ipm.net.copy(pd=np.array(pd, float), qd=np.array(qd, float)), ipm.opt)
    other.set_objective_scale(ipm.sigma_f)
    return other
