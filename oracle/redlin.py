"""Oracle: the reduce-then-linearize interior-point method (test infrastructure).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this.

Algorithm 2 of the paper (RedLin, Section 2.3): the state is removed from the
problem by the implicit function theorem, x = x(u) with g(x(u), u) = 0, and
the reduced problem
    min f_r(u)  s.t.  h_r(u) + s = 0,  ul <= u <= uu,  sl <= s <= su,
    f_r(u) = f(x(u), u),  h_r(u) = [h(x(u), u); -x_b(u)]
is solved by an interior-point method. x_b are the states with bounds (Vm at
PQ buses; angles are free), whose bounds move into h_r (Section 2.3.1,
difference (ii)); their slacks are s_x = x_b with bounds [xl, xu].

Every iteration:
* projection: Newton-Raphson on g(x, u) = 0 (tolerance 1e-10, the paper's);
* adjoint: lambda = -G_x^{-T} grad_x (f + y_h^T h - y_x^T x_b);
* reduced derivatives (eq. reduced:derivatives): grad L_r = [I; S]^T grad_w L
  (S = -G_x^{-1} G_u), A_hat = [A_u + A_x S; -S_b],
  W_hat = [I; S]^T W [I; S] with W the Hessian of f + lambda^T g + y_h^T h;
* the reduced KKT system (eq. reduced:kktsystem) in (p_u, p_s, p_y), solved
  densely here, with K_cond = W_hat + Sigma_u + A_hat^T Sigma_s A_hat made
  positive definite by the inertia correction of Algorithm 1;
* filter line search on (u, s, y), every trial point projected first (a trial
  whose projection fails is rejected like one the filter refuses).

Readings (the paper prints no constants or details for RedLin):
* the reduced KKT matrix is printed with -I in its (s, y) blocks; as for
  eq. kktmatrix:normal (oracle.reduction) the Lagrangian gives +I, used here;
* the barrier update, filter, inertia correction, bound handling and
  objective scaling are those of the LinRed oracle (oracle.ipm), applied to
  (u, s) with the dual infeasibility grad L_r - zl + zu; the objective scale
  is taken at the projected initial point;
* the projection warm-starts from x + alpha S p_u (the linearised state step)
  and fails after 20 Newton iterations or a non-finite residual.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .ipm import IPMOptions, LinRedIPM, _push


@dataclass
class RedLinState:
    u: np.ndarray
    x: np.ndarray
    s: np.ndarray
    y: np.ndarray
    zl: np.ndarray
    zu: np.ndarray
    zsl: np.ndarray
    zsu: np.ndarray
    mu: float
    lam: np.ndarray = None
    delta_last: float = 0.0
    filt: list = field(default_factory=list)
    it: int = 0
    pf_iters: int = 0


class RedLinIPM:
    """Algorithm 2 on the oracle model of a network (dense linear algebra)."""

    def __init__(self, net, options=None, pf_tol=1e-10, pf_max_iter=20):
        self.lin = LinRedIPM(net, options or IPMOptions())
        self.net = net
        self.opt = self.lin.opt
        nu, nx, m = self.lin.nu, self.lin.nx, self.lin.m
        self.nu, self.nx, self.m = nu, nx, m
        xl, xu = self.lin.wl[nu:], self.lin.wu[nu:]
        self.xb = np.flatnonzero(np.isfinite(xl) | np.isfinite(xu))
        self.ul, self.uu = self.lin.wl[:nu], self.lin.wu[:nu]
        self.sl = np.concatenate([self.lin.sl, xl[self.xb]])
        self.su = np.concatenate([self.lin.su, xu[self.xb]])
        self.mr = m + self.xb.shape[0]
        self.ful, self.fuu = np.isfinite(self.ul), np.isfinite(self.uu)
        self.fsl, self.fsu = np.isfinite(self.sl), np.isfinite(self.su)
        self.pf_tol, self.pf_max_iter = pf_tol, pf_max_iter

    @property
    def M(self):
        return self.lin.M

    @property
    def sigma_f(self):
        return self.lin.sigma_f

    # ------------------------------------------------------------ pieces
    def project(self, u, x0):
        """Newton-Raphson on g(x, u) = 0 from x0; (x, iterations) or
        (None, iterations) if it does not reach the tolerance."""
        x = np.array(x0, float)
        nu = self.nu
        for k in range(self.pf_max_iter + 1):
            g, _, _ = self.M.functions(x, u)
            g = np.asarray(g, float)
            if not np.all(np.isfinite(g)):
                return None, k
            if np.abs(g).max() <= self.pf_tol:
                return x, k
            if k == self.pf_max_iter:
                break
            G, _, _ = self.M.jacobians(x, u)
            x = x - np.linalg.solve(G[:, nu:].toarray(), g)
        return None, self.pf_max_iter

    def h_r(self, u, x):
        _, h, _ = self.M.functions(x, u)
        return np.concatenate([np.asarray(h, float), -x[self.xb]])

    def objective(self, u, x):
        _, _, f = self.M.functions(x, u)
        return float(np.real(f))

    def slacks(self, u, s):
        inf = np.inf
        dul = np.where(self.ful, u - np.where(self.ful, self.ul, 0.0), inf)
        duu = np.where(self.fuu, np.where(self.fuu, self.uu, 0.0) - u, inf)
        dsl = np.where(self.fsl, s - np.where(self.fsl, self.sl, 0.0), inf)
        dsu = np.where(self.fsu, np.where(self.fsu, self.su, 0.0) - s, inf)
        return dul, duu, dsl, dsu

    def barrier_obj(self, f, u, s, mu):
        logs = sum(np.log(d[np.isfinite(d)]).sum() for d in self.slacks(u, s))
        return f - mu * logs

    def derivatives(self, u, x, y):
        """Adjoint, reduced gradients and matrices at (u, x(u)) for multipliers y."""
        nu, m = self.nu, self.m
        G, A, gf = self.M.jacobians(x, u)
        G, A = G.toarray(), A.toarray()
        Gx, Gu = G[:, nu:], G[:, :nu]
        lu = sla.lu_factor(Gx)
        S = -sla.lu_solve(lu, Gu)
        yh, yx = y[:m], y[m:]
        gx = gf[nu:] + A[:, nu:].T @ yh
        gx[self.xb] -= yx
        lam = -sla.lu_solve(lu, gx, trans=1)
        T = np.vstack([np.eye(nu), S])
        gl = gf + A.T @ yh + G.T @ lam
        grad_lr = gl[:nu]                                  # = [I; S]^T grad_w L
        grad_fr = T.T @ gf
        A_hat = np.vstack([A[:, :nu] + A[:, nu:] @ S, -S[self.xb]])
        W = self.M.hessian_lagrangian(x, u, lam, yh).toarray()
        W_hat = T.T @ W @ T
        return {"lam": lam, "S": S, "grad_lr": grad_lr, "grad_fr": grad_fr, "A_hat": A_hat,
                "W_hat": W_hat, "gf": gf}

    def sigmas(self, st):
        inv = lambda d: np.where(np.isfinite(d), 1.0 / d, 0.0)
        dul, duu, dsl, dsu = self.slacks(st.u, st.s)
        return (st.zl * inv(dul) + st.zu * inv(duu), st.zsl * inv(dsl) + st.zsu * inv(dsu))

    def residuals(self, st, D, mu):
        inv = lambda d: np.where(np.isfinite(d), 1.0 / d, 0.0)
        dul, duu, dsl, dsu = self.slacks(st.u, st.s)
        r_u = D["grad_lr"] - mu * inv(dul) + mu * inv(duu)
        r_s = st.y - mu * inv(dsl) + mu * inv(dsu)
        r_y = self.h_r(st.u, st.x) + st.s
        return r_u, r_s, r_y

    def condensed(self, D, sig_u, sig_s, delta=0.0):
        """K_cond of the reduced system (Theorem 2 applied to eq. reduced:kktsystem)."""
        Ah = D["A_hat"]
        K = D["W_hat"] + np.diag(sig_u + delta) + Ah.T @ (sig_s[:, None] * Ah)
        return 0.5 * (K + K.T)

    def kkt_matrix(self, D, sig_u, sig_s, delta=0.0):
        """Dense reduced KKT matrix in (p_u, p_s, p_y), +I reading."""
        nu, mr = self.nu, self.mr
        n = nu + 2 * mr
        K = np.zeros((n, n))
        K[:nu, :nu] = D["W_hat"] + np.diag(sig_u + delta)
        K[:nu, nu + mr:] = D["A_hat"].T
        K[nu + mr:, :nu] = D["A_hat"]
        K[nu:nu + mr, nu:nu + mr] = np.diag(sig_s)
        K[nu:nu + mr, nu + mr:] = np.eye(mr)
        K[nu + mr:, nu:nu + mr] = np.eye(mr)
        return K

    def optimality_error(self, st, mu, D=None):
        opt = self.opt
        if D is None:
            D = self.derivatives(st.u, st.x, st.y)
        rd_u = D["grad_lr"] - st.zl + st.zu
        rd_s = st.y - st.zsl + st.zsu
        prim = self.h_r(st.u, st.x) + st.s
        comp = []
        for d, z, msk in zip(self.slacks(st.u, st.s), (st.zl, st.zu, st.zsl, st.zsu),
                             (self.ful, self.fuu, self.fsl, self.fsu)):
            comp.append(np.abs(d[msk] * z[msk] - mu))
        comp = np.concatenate(comp)
        nz = int(self.ful.sum() + self.fuu.sum() + self.fsl.sum() + self.fsu.sum())
        zsum = np.abs(st.zl).sum() + np.abs(st.zu).sum() + np.abs(st.zsl).sum() + np.abs(st.zsu).sum()
        sd = max(opt.s_max, (np.abs(st.y).sum() + zsum) / max(1, self.mr + nz)) / opt.s_max
        sc = max(opt.s_max, zsum / max(1, nz)) / opt.s_max
        e_dual = max(np.abs(rd_u).max(), np.abs(rd_s).max()) / sd
        e_prim = np.abs(prim).max()
        e_comp = (comp.max() if comp.size else 0.0) / sc
        return max(e_dual, e_prim, e_comp)

    def initial_state(self, x0, u0):
        opt = self.opt
        u = _push(np.asarray(u0, float), self.ul, self.uu, opt)
        x, k = self.project(u, x0)
        if x is None:
            raise RuntimeError("projection of the initial point failed")
        if opt.obj_scale > 0.0:
            self.lin.set_objective_scale(opt.obj_scale)
        else:
            from .model import Model
            _, _, gf = Model(self.net).jacobians(x, u)
            self.lin.set_objective_scale(min(1.0, 100.0 / max(np.abs(gf).max(), 1e-300)))
        s = _push(-self.h_r(u, x), self.sl, self.su, opt)
        one = lambda mask: np.where(mask, 1.0, 0.0)
        return RedLinState(u=u, x=x, s=s, y=np.zeros(self.mr), zl=one(self.ful), zu=one(self.fuu),
                           zsl=one(self.fsl), zsu=one(self.fsu), mu=opt.mu_init, pf_iters=k)

    # -------------------------------------------------------------- iterate
    def iterate(self, st):
        """One iteration of Algorithm 2 (the projection of the current point was
        done when it was accepted); returns the iteration's scalars."""
        opt = self.opt
        nu, mr = self.nu, self.mr
        D = self.derivatives(st.u, st.x, st.y)
        st.lam = D["lam"]
        for _ in range(10):
            if self.optimality_error(st, st.mu, D) > opt.kappa_eps * st.mu:
                break
            new_mu = max(opt.tol / 10.0, min(opt.kappa_mu * st.mu, st.mu ** opt.theta_mu))
            if new_mu == st.mu:
                break
            st.mu = new_mu
            st.filt = []
        mu = st.mu
        sig_u, sig_s = self.sigmas(st)

        def pd(delta):
            try:
                np.linalg.cholesky(self.condensed(D, sig_u, sig_s, delta))
                return True
            except np.linalg.LinAlgError:
                return False

        delta = 0.0
        if not pd(0.0):
            delta = (opt.delta_w0 if st.delta_last == 0.0
                     else max(opt.delta_min, opt.kappa_w_minus * st.delta_last))
            while not pd(delta):
                delta *= opt.kappa_w_plus_bar if st.delta_last == 0.0 else opt.kappa_w_plus
                if delta > opt.delta_max:
                    raise RuntimeError("inertia correction failed")
            st.delta_last = delta
        r_u, r_s, r_y = self.residuals(st, D, mu)
        p = np.linalg.solve(self.kkt_matrix(D, sig_u, sig_s, delta),
                            -np.concatenate([r_u, r_s, r_y]))
        pu, ps, py = p[:nu], p[nu:nu + mr], p[nu + mr:]
        px = D["S"] @ pu
        inv = lambda d: np.where(np.isfinite(d), 1.0 / d, 0.0)
        dul, duu, dsl, dsu = self.slacks(st.u, st.s)
        pzl = np.where(self.ful, mu * inv(dul) - st.zl - st.zl * inv(dul) * pu, 0.0)
        pzu = np.where(self.fuu, mu * inv(duu) - st.zu + st.zu * inv(duu) * pu, 0.0)
        pzsl = np.where(self.fsl, mu * inv(dsl) - st.zsl - st.zsl * inv(dsl) * ps, 0.0)
        pzsu = np.where(self.fsu, mu * inv(dsu) - st.zsu + st.zsu * inv(dsu) * ps, 0.0)
        tau = max(opt.tau_min, 1.0 - mu)

        def amax(d, step, mask, sign):
            q = sign * step
            sel = mask & (q < 0)
            return 1.0 if not sel.any() else min(1.0, float(np.min(-tau * d[sel] / q[sel])))

        def zmax(z, pz, mask):
            sel = mask & (pz < 0)
            return 1.0 if not sel.any() else min(1.0, float(np.min(-tau * z[sel] / pz[sel])))

        a_pri = min(amax(dul, pu, self.ful, 1.0), amax(duu, pu, self.fuu, -1.0),
                    amax(dsl, ps, self.fsl, 1.0), amax(dsu, ps, self.fsu, -1.0))
        a_dual = min(zmax(st.zl, pzl, self.ful), zmax(st.zu, pzu, self.fuu),
                     zmax(st.zsl, pzsl, self.fsl), zmax(st.zsu, pzsu, self.fsu))
        # filter line search on the reduced problem (trial points projected)
        f0 = self.objective(st.u, st.x)
        theta = np.abs(r_y).sum()
        phi = self.barrier_obj(f0, st.u, st.s, mu)
        dphi = (D["grad_fr"] @ pu - mu * (inv(dul) @ pu - inv(duu) @ pu)
                - mu * (inv(dsl) @ ps - inv(dsu) @ ps))
        if st.it == 0 and not hasattr(self, "theta0"):
            self.theta0 = theta
        th0 = getattr(self, "theta0", theta)
        theta_max = 1e4 * max(1.0, th0)
        theta_min = 1e-4 * max(1.0, th0)
        a_min = opt.gamma_theta
        if dphi < 0:
            a_min = min(a_min, opt.gamma_phi * theta / -dphi)
            if theta <= theta_min:
                a_min = min(a_min, opt.delta_sw * theta ** opt.s_theta / (-dphi) ** opt.s_phi)
        a_min *= opt.gamma_alpha
        alpha = a_pri
        trials = pf_total = 0
        while True:
            if alpha < a_min:
                raise RuntimeError("line search failed (restoration not implemented)")
            ut, stt = st.u + alpha * pu, st.s + alpha * ps
            xt, k = self.project(ut, st.x + alpha * px)
            trials += 1
            pf_total += k
            ok, ftype = xt is not None, False
            if ok:
                th_t = np.abs(self.h_r(ut, xt) + stt).sum()
                ph_t = self.barrier_obj(self.objective(ut, xt), ut, stt, mu)
                ok = np.isfinite(ph_t) and th_t <= theta_max
                if ok:
                    ok = not any(th_t >= tf and ph_t >= pf for tf, pf in st.filt)
                if ok:
                    switching = (dphi < 0 and alpha * (-dphi) ** opt.s_phi
                                 > opt.delta_sw * theta ** opt.s_theta)
                    if switching and theta <= theta_min:
                        ok = ph_t <= phi + opt.eta_phi * alpha * dphi
                        ftype = True
                    else:
                        ok = (th_t <= (1 - opt.gamma_theta) * theta
                              or ph_t <= phi - opt.gamma_phi * theta)
            if ok:
                break
            alpha *= 0.5
        if not ftype:
            st.filt.append(((1 - opt.gamma_theta) * theta, phi - opt.gamma_phi * theta))
        st.u, st.x, st.s = ut, xt, stt
        st.y = st.y + alpha * py
        st.zl = st.zl + a_dual * pzl
        st.zu = st.zu + a_dual * pzu
        st.zsl = st.zsl + a_dual * pzsl
        st.zsu = st.zsu + a_dual * pzsu
        dul, duu, dsl, dsu = self.slacks(st.u, st.s)
        kk = opt.kappa_sigma
        for zname, d, msk in (("zl", dul, self.ful), ("zu", duu, self.fuu),
                              ("zsl", dsl, self.fsl), ("zsu", dsu, self.fsu)):
            z = getattr(st, zname)
            dd = np.where(msk, d, 1.0)
            setattr(st, zname, np.where(msk, np.clip(z, mu / (kk * dd), kk * mu / dd), 0.0))
        st.it += 1
        st.pf_iters += pf_total
        return {"iter": st.it, "obj": self.objective(st.u, st.x) / self.sigma_f, "mu": mu,
                "alpha_pr": alpha, "alpha_du": a_dual, "delta_w": delta, "trials": trials,
                "pf_iters": pf_total,
                "inf_pr": float(np.abs(self.h_r(st.u, st.x) + st.s).max())}

    def solve(self, x0, u0):
        """Runs to E_0 <= tol. Returns (state, per-iteration list, converged)."""
        st = self.initial_state(x0, u0)
        log = []
        for _ in range(self.opt.max_iter):
            if self.optimality_error(st, 0.0) <= self.opt.tol:
                st.lam = self.derivatives(st.u, st.x, st.y)["lam"]
                return st, log, True
            log.append(self.iterate(st))
        return st, log, self.optimality_error(st, 0.0) <= self.opt.tol
