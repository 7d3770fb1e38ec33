"""Oracle: the linearize-then-reduce interior-point method (test infrastructure).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this.

Algorithm 1 of the paper (LinRed): at every iteration evaluate the
derivatives, solve the augmented KKT system (eq. kktmatrix:normal) for the
step (p_u, p_x, p_s, p_lambda, p_y), regularising until the inertia is right
(Section 4.3: K_cond positive definite, else delta_w is raised), and move
along the step with a filter line search. The paper delegates the line
search, the barrier update and the initial point to MadNLP / Ipopt; the
reading used here is the textbook filter line-search method of Waechter and
Biegler (2006) without second-order correction and without the restoration
phase (a failing line search ends the run), with a monotone barrier update.
Every constant is listed in IPMOptions.

The objective is scaled as in those methods: f is multiplied by
sigma_f = min(1, 100 / max|grad f(w0)|) at the initial point w0 (after it is
pushed inside the bounds), by scaling the generator cost coefficients; the
reported objective is f itself.

Problem (Section 2.1, with the two-sided bounds of the OPF model):
    min f(w)  s.t.  g(w) = 0,  h(w) + s = 0,  wl <= w <= wu,  sl <= s <= su
with w = [u; x] and s = -h at a feasible point (sl = -h_hi, su = -h_lo).
The barrier terms of eq. kktmatrix:normal generalise to two-sided bounds:
Sigma = zl / (w - wl) + zu / (wu - w) and the residuals carry
-mu / (w - wl) + mu / (wu - w).

The step is computed here by a direct solve of the augmented system (the
oracle does not condense): a dense LU, or for large networks a sparse LU with
partial pivoting of the same matrix; the library computes the same step
through the condensed matrix.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import reduction as R


@dataclass
class IPMOptions:
    tol: float = 1e-6          # stop when the scaled optimality error E_0 <= tol
    max_iter: int = 200
    mu_init: float = 0.1
    kappa_eps: float = 10.0    # barrier subproblem solved when E_mu <= kappa_eps mu
    kappa_mu: float = 0.2      # mu <- max(tol / 10, min(kappa_mu mu, mu^theta_mu))
    theta_mu: float = 1.5
    tau_min: float = 0.99      # fraction to the boundary: tau = max(tau_min, 1 - mu)
    s_max: float = 100.0       # scaling of the optimality error
    kappa_sigma: float = 1e10  # bound multipliers kept within [mu/(k s), k mu/s]
    bound_push: float = 1e-2   # initial point pushed inside the bounds
    bound_frac: float = 1e-2
    # inertia correction (delta_w on the control block of K_aug)
    delta_w0: float = 1e-4
    delta_min: float = 1e-20
    delta_max: float = 1e40
    kappa_w_minus: float = 1.0 / 3.0
    kappa_w_plus: float = 8.0
    kappa_w_plus_bar: float = 100.0
    # filter line search
    gamma_theta: float = 1e-5
    gamma_phi: float = 1e-8
    delta_sw: float = 1.0
    s_theta: float = 1.1
    s_phi: float = 2.3
    eta_phi: float = 1e-8
    gamma_alpha: float = 0.05
    obj_scale: float = 0.0     # 0: automatic (see above)
    # "dense": K_aug factored densely; "sparse": the same system by a sparse
    # LU with partial pivoting (networks whose dense K_aug is too large)
    linear_solver: str = "dense"


@dataclass
class IPMState:
    w: np.ndarray
    s: np.ndarray
    lam: np.ndarray
    y: np.ndarray
    zl: np.ndarray
    zu: np.ndarray
    zsl: np.ndarray
    zsu: np.ndarray
    mu: float
    delta_last: float = 0.0
    filt: list = field(default_factory=list)
    it: int = 0


def _push(v, lo, hi, opt):
    """Moves v strictly inside [lo, hi] (finite sides only)."""
    v = np.array(v, float)
    fl, fu = np.isfinite(lo), np.isfinite(hi)
    both = fl & fu
    pl = np.where(fl, opt.bound_push * np.maximum(1.0, np.abs(np.where(fl, lo, 0.0))), 0.0)
    pu = np.where(fu, opt.bound_push * np.maximum(1.0, np.abs(np.where(fu, hi, 0.0))), 0.0)
    width = np.where(both, np.where(both, hi, 0.0) - np.where(both, lo, 0.0), np.inf)
    pl = np.where(both, np.minimum(pl, opt.bound_frac * width), pl)
    pu = np.where(both, np.minimum(pu, opt.bound_frac * width), pu)
    v = np.where(fl, np.maximum(v, np.where(fl, lo, 0.0) + pl), v)
    v = np.where(fu, np.minimum(v, np.where(fu, hi, 0.0) - pu), v)
    return v


class LinRedIPM:
    """Algorithm 1 on the oracle model of a network (dense linear algebra)."""

    def __init__(self, net, options=None):
        from .model import Model
        self.net = net
        self.M = Model(net)
        self.sigma_f = 1.0
        model = self.M
        self.opt = options or IPMOptions()
        xl, xu, ul, uu = model.var_bounds()
        self.wl = np.concatenate([ul, xl])
        self.wu = np.concatenate([uu, xu])
        hl, hu = model.h_bounds()
        self.sl = -hu
        self.su = -hl
        self.fwl, self.fwu = np.isfinite(self.wl), np.isfinite(self.wu)
        self.fsl, self.fsu = np.isfinite(self.sl), np.isfinite(self.su)
        self.nu, self.nx, self.m = model.nu, model.nx, model.m

    # ------------------------------------------------------------ pieces
    def split(self, w):
        return w[self.nu:], w[:self.nu]          # x, u

    def evaluate(self, w, s):
        x, u = self.split(w)
        g, h, f = self.M.functions(x, u)
        return np.asarray(g, float), np.asarray(h, float), float(np.real(f))

    def slacks(self, w, s):
        dwl = np.where(self.fwl, w - np.where(self.fwl, self.wl, 0.0), np.inf)
        dwu = np.where(self.fwu, np.where(self.fwu, self.wu, 0.0) - w, np.inf)
        dsl = np.where(self.fsl, s - np.where(self.fsl, self.sl, 0.0), np.inf)
        dsu = np.where(self.fsu, np.where(self.fsu, self.su, 0.0) - s, np.inf)
        return dwl, dwu, dsl, dsu

    def barrier_obj(self, f, w, s, mu):
        """phi = f - mu sum log(bound slacks) over finite bounds."""
        dwl, dwu, dsl, dsu = self.slacks(w, s)
        logs = sum(np.log(d[np.isfinite(d)]).sum() for d in (dwl, dwu, dsl, dsu))
        return f - mu * logs

    def set_objective_scale(self, sigma):
        from .model import Model
        net = self.net
        self.sigma_f = float(sigma)
        self.M = Model(net.copy(c2=net.c2 * sigma, c1=net.c1 * sigma, c0=net.c0 * sigma))

    def initial_state(self, x0, u0):
        opt = self.opt
        w = _push(np.concatenate([u0, x0]), self.wl, self.wu, opt)
        x, u = self.split(w)
        if opt.obj_scale > 0.0:
            self.set_objective_scale(opt.obj_scale)
        else:
            from .model import Model
            _, _, gf = Model(self.net).jacobians(x, u)
            self.set_objective_scale(min(1.0, 100.0 / max(np.abs(gf).max(), 1e-300)))
        _, h, _ = self.M.functions(x, u)
        s = _push(-np.asarray(h, float), self.sl, self.su, opt)
        one = lambda mask: np.where(mask, 1.0, 0.0)
        return IPMState(w=w, s=s, lam=np.zeros(self.nx), y=np.zeros(self.m),
                        zl=one(self.fwl), zu=one(self.fwu), zsl=one(self.fsl),
                        zsu=one(self.fsu), mu=opt.mu_init)

    def optimality_error(self, st, mu):
        """Scaled KKT error E_mu (dual infeasibility, primal infeasibility,
        complementarity), as in the Waechter-Biegler method."""
        opt = self.opt
        w, s = st.w, st.s
        x, u = self.split(w)
        g, h, _ = self.evaluate(w, s)
        gl = self.M.lagrangian_gradient(x, u, st.lam, st.y)
        rd_w = gl - st.zl + st.zu
        rd_s = st.y - st.zsl + st.zsu
        dwl, dwu, dsl, dsu = self.slacks(w, s)
        comp = []
        for d, z, msk in ((dwl, st.zl, self.fwl), (dwu, st.zu, self.fwu),
                          (dsl, st.zsl, self.fsl), (dsu, st.zsu, self.fsu)):
            comp.append(np.abs(d[msk] * z[msk] - mu))
        comp = np.concatenate(comp) if comp else np.zeros(0)
        nz = int(self.fwl.sum() + self.fwu.sum() + self.fsl.sum() + self.fsu.sum())
        zsum = np.abs(st.zl).sum() + np.abs(st.zu).sum() + np.abs(st.zsl).sum() + np.abs(st.zsu).sum()
        sd = max(opt.s_max, (np.abs(st.lam).sum() + np.abs(st.y).sum() + zsum) /
                 max(1, self.nx + self.m + nz)) / opt.s_max
        sc = max(opt.s_max, zsum / max(1, nz)) / opt.s_max
        e_dual = max(np.abs(rd_w).max(), np.abs(rd_s).max() if self.m else 0.0) / sd
        e_prim = max(np.abs(g).max(), np.abs(h + s).max() if self.m else 0.0)
        e_comp = (comp.max() if comp.size else 0.0) / sc
        return max(e_dual, e_prim, e_comp)

    def step(self, st, mu, delta):
        """Residuals, sigmas and the solve of K_aug(delta) p = -r."""
        w, s = st.w, st.s
        x, u = self.split(w)
        dwl, dwu, dsl, dsu = self.slacks(w, s)
        inv = lambda d: np.where(np.isfinite(d), 1.0 / d, 0.0)
        sig_w = st.zl * inv(dwl) + st.zu * inv(dwu)
        sig_s = st.zsl * inv(dsl) + st.zsu * inv(dsu)
        gl = self.M.lagrangian_gradient(x, u, st.lam, st.y)
        r_w = gl - mu * inv(dwl) + mu * inv(dwu)
        r3 = st.y - mu * inv(dsl) + mu * inv(dsu)
        g, h, _ = self.evaluate(w, s)
        r = np.concatenate([r_w, r3, g, h + s])          # r1, r2 (= r_w), r3, r4, r5
        B = R.kkt_blocks(self.M, x, u, st.lam, st.y, sig_w[self.nu:], sig_w[:self.nu], sig_s)
        solve = R.solve_augmented_sparse if self.opt.linear_solver == "sparse" else R.solve_augmented
        p = solve(B, r, delta_w=delta)                  # [p_u, p_x, p_s, p_lambda, p_y]
        return B, r, p, sig_w, sig_s

    def inertia_ok(self, st, sig_w, sig_s, delta):
        x, u = self.split(st.w)
        B = R.kkt_blocks(self.M, x, u, st.lam, st.y, sig_w[self.nu:], sig_w[:self.nu], sig_s)
        Kc = R.symmetrize(R.condensed_matrix(B)) + delta * np.eye(self.nu)
        try:
            np.linalg.cholesky(Kc)
            return True
        except np.linalg.LinAlgError:
            return False

    # -------------------------------------------------------------- iterate
    def iterate(self, st):
        """One iteration of Algorithm 1; returns a dict of the iteration's
        scalars (as rh_ipm_info), or raises RuntimeError on a failed line
        search."""
        opt = self.opt
        nu, nx, m = self.nu, self.nx, self.m
        # barrier update (monotone): decrease mu while the subproblem is solved
        for _ in range(10):
            if self.optimality_error(st, st.mu) > opt.kappa_eps * st.mu:
                break
            new_mu = max(opt.tol / 10.0, min(opt.kappa_mu * st.mu, st.mu ** opt.theta_mu))
            if new_mu == st.mu:
                break
            st.mu = new_mu
            st.filt = []
        mu = st.mu
        w, s = st.w, st.s
        dwl, dwu, dsl, dsu = self.slacks(w, s)
        inv = lambda d: np.where(np.isfinite(d), 1.0 / d, 0.0)
        sig_w = st.zl * inv(dwl) + st.zu * inv(dwu)
        sig_s = st.zsl * inv(dsl) + st.zsu * inv(dsu)
        # inertia correction on K_cond + delta I
        delta = 0.0
        if not self.inertia_ok(st, sig_w, sig_s, 0.0):
            delta = (opt.delta_w0 if st.delta_last == 0.0
                     else max(opt.delta_min, opt.kappa_w_minus * st.delta_last))
            while not self.inertia_ok(st, sig_w, sig_s, delta):
                delta *= opt.kappa_w_plus_bar if st.delta_last == 0.0 else opt.kappa_w_plus
                if delta > opt.delta_max:
                    raise RuntimeError("inertia correction failed")
            st.delta_last = delta
        B, r, p, _, _ = self.step(st, mu, delta)
        pu, px, ps, plam, py = p
        pw = np.concatenate([pu, px])
        # bound multiplier steps
        pzl = np.where(self.fwl, mu * inv(dwl) - st.zl - st.zl * inv(dwl) * pw, 0.0)
        pzu = np.where(self.fwu, mu * inv(dwu) - st.zu + st.zu * inv(dwu) * pw, 0.0)
        pzsl = np.where(self.fsl, mu * inv(dsl) - st.zsl - st.zsl * inv(dsl) * ps, 0.0)
        pzsu = np.where(self.fsu, mu * inv(dsu) - st.zsu + st.zsu * inv(dsu) * ps, 0.0)
        # fraction to the boundary
        tau = max(opt.tau_min, 1.0 - mu)

        def amax(d, pd, mask, sign):
            # largest a in (0, 1] with d + sign a pd >= (1 - tau) d
            q = sign * pd
            sel = mask & (q < 0)
            if not sel.any():
                return 1.0
            return min(1.0, float(np.min(-tau * d[sel] / q[sel])))

        a_pri = min(amax(dwl, pw, self.fwl, 1.0), amax(dwu, pw, self.fwu, -1.0),
                    amax(dsl, ps, self.fsl, 1.0), amax(dsu, ps, self.fsu, -1.0))

        def zmax(z, pz, mask):
            sel = mask & (pz < 0)
            if not sel.any():
                return 1.0
            return min(1.0, float(np.min(-tau * z[sel] / pz[sel])))

        a_dual = min(zmax(st.zl, pzl, self.fwl), zmax(st.zu, pzu, self.fwu),
                     zmax(st.zsl, pzsl, self.fsl), zmax(st.zsu, pzsu, self.fsu))
        # filter line search
        g, h, f = self.evaluate(w, s)
        theta = np.abs(g).sum() + np.abs(h + s).sum()
        phi = self.barrier_obj(f, w, s, mu)
        x, u = self.split(w)
        _, _, gf = self.M.jacobians(x, u)
        dphi = (gf @ pw - mu * (inv(dwl) @ pw - inv(dwu) @ pw)
                - mu * (inv(dsl) @ ps - inv(dsu) @ ps))
        if st.it == 0 and not hasattr(self, "theta0"):
            self.theta0 = theta
        th0 = getattr(self, "theta0", theta)
        theta_max = 1e4 * max(1.0, th0)
        theta_min = 1e-4 * max(1.0, th0)
        if dphi < 0:
            a_min = opt.gamma_theta
            a_min = min(a_min, opt.gamma_phi * theta / -dphi)
            if theta <= theta_min:
                a_min = min(a_min, opt.delta_sw * theta ** opt.s_theta / (-dphi) ** opt.s_phi)
        else:
            a_min = opt.gamma_theta
        a_min *= opt.gamma_alpha
        alpha = a_pri
        trials = 0
        while True:
            if alpha < a_min:
                raise RuntimeError("line search failed (restoration not implemented)")
            wt, stt = w + alpha * pw, s + alpha * ps
            gt, ht, ft = self.evaluate(wt, stt)
            th_t = np.abs(gt).sum() + np.abs(ht + stt).sum()
            ph_t = self.barrier_obj(ft, wt, stt, mu)
            trials += 1
            ok = np.isfinite(ph_t) and th_t <= theta_max
            if ok:
                ok = not any(th_t >= tf and ph_t >= pf for tf, pf in st.filt)
            ftype = False
            if ok:
                switching = dphi < 0 and alpha * (-dphi) ** opt.s_phi > opt.delta_sw * theta ** opt.s_theta
                if switching and theta <= theta_min:
                    ok = ph_t <= phi + opt.eta_phi * alpha * dphi
                    ftype = True
                else:
                    ok = th_t <= (1 - opt.gamma_theta) * theta or ph_t <= phi - opt.gamma_phi * theta
            if ok:
                break
            alpha *= 0.5
        if not ftype:
            st.filt.append(((1 - opt.gamma_theta) * theta, phi - opt.gamma_phi * theta))
        # update
        st.w = w + alpha * pw
        st.s = s + alpha * ps
        st.lam = st.lam + alpha * plam
        st.y = st.y + alpha * py
        st.zl = st.zl + a_dual * pzl
        st.zu = st.zu + a_dual * pzu
        st.zsl = st.zsl + a_dual * pzsl
        st.zsu = st.zsu + a_dual * pzsu
        # keep the bound multipliers near mu / slack
        dwl, dwu, dsl, dsu = self.slacks(st.w, st.s)
        k = opt.kappa_sigma
        for zname, d, msk in (("zl", dwl, self.fwl), ("zu", dwu, self.fwu),
                              ("zsl", dsl, self.fsl), ("zsu", dsu, self.fsu)):
            z = getattr(st, zname)
            dd = np.where(msk, d, 1.0)
            z = np.where(msk, np.clip(z, mu / (k * dd), k * mu / dd), 0.0)
            setattr(st, zname, z)
        st.it += 1
        gn, hn, fnew = self.evaluate(st.w, st.s)
        return {"iter": st.it, "obj": fnew / self.sigma_f, "mu": mu, "alpha_pr": alpha,
                "alpha_du": a_dual, "delta_w": delta, "trials": trials,
                "inf_pr": max(np.abs(gn).max(), np.abs(hn + st.s).max() if self.m else 0.0)}

    def solve(self, x0, u0):
        """Runs to E_0 <= tol. Returns (state, per-iteration list, converged)."""
        st = self.initial_state(x0, u0)
        log = []
        for _ in range(self.opt.max_iter):
            if self.optimality_error(st, 0.0) <= self.opt.tol:
                return st, log, True
            log.append(self.iterate(st))
        return st, log, self.optimality_error(st, 0.0) <= self.opt.tol


def flat_start(model):
    """theta = 0, Vm = 1, Pg at the middle of its range (pushed inside the
    bounds by the method)."""
    net = model.net
    x = np.zeros(model.nx)
    u = np.zeros(model.nu)
    for i in model.pq:
        x[model.x_vm[i]] = 1.0
    for g in range(model.ng):
        u[g] = 1.0
    for g in model.nonref_gens:
        u[model.u_pg[g]] = 0.5 * (net.pmin[g] + net.pmax[g])
    return x, u
