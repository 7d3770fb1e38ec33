"""Oracle: polar AC-OPF model in state-control form (test infrastructure).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this.

The paper states the problem abstractly (Section 2.1: min f(x,u) s.t.
g(x,u) = 0 with nx equations, h(x,u) <= 0, bounds; Lagrangian with multipliers
lambda for g and y for h + s = 0) and uses AC optimal power flow as its
application without writing the model out. The reading taken here is the
standard polar formulation:

* bus injections  P_i = sum_k V_i V_k (G_ik cos t_ik + B_ik sin t_ik),
                  Q_i = sum_k V_i V_k (G_ik sin t_ik - B_ik cos t_ik),
  t_ik = theta_i - theta_k, with the admittance matrix of pi-model lines
  (series 1/(r + j x), half the charging b at each end);
* state x  = (theta at non-reference buses, Vm at PQ buses),
  control u = (Vm at generator buses, Pg at non-reference generators);
  this split reproduces the nx/nu columns of Table 1;
* g = (P balance at non-reference buses, Q balance at PQ buses): nx rows;
* h = (Pg_ref, Qg of every generator, |S_from|^2 and |S_to|^2 of limited lines);
* f = sum over generators of c2 (base Pg)^2 + c1 (base Pg) + c0, Pg in MW;
  the reference generator's Pg_ref = P_ref(x, u) + Pd_ref is a function of
  the state, so it enters f, grad f and W.

Derivatives are analytic. Every power quantity is a sum of terms
T = V_a V_b phi(theta_a - theta_b) with phi(t) = G cos t + B sin t (for P) or
G sin t - B cos t (for Q); the gradient and Hessian of one term follow from
the product and chain rules, and sums of terms are scattered into
(theta, Vm)-space and then mapped to the (u, x) variables.

Vector ordering used by the oracle (the paper's block order):
  w = [u; x],   u = [Vm at gen buses (gen order); Pg at non-ref gens (gen order)],
                x = [theta at non-ref buses (bus order); Vm at PQ buses (bus order)].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

BUS_PQ, BUS_PV, BUS_REF = 1, 2, 3


class Model:
    """Index maps, admittances and dense/sparse derivative builders."""

    def __init__(self, net):
        self.net = net
        nb, ng = net.nb, net.ng
        bt = np.asarray(net.bus_type)
        refs = np.flatnonzero(bt == BUS_REF)
        if refs.shape[0] != 1:
            raise ValueError("exactly one reference bus required")
        self.ref = int(refs[0])
        gb = np.asarray(net.gen_bus)
        if len(set(gb.tolist())) != ng:
            raise ValueError("one generator per generator bus required")
        if set(np.flatnonzero(bt != BUS_PQ).tolist()) != set(gb.tolist()):
            raise ValueError("generator buses must be exactly the PV/ref buses")
        self.ref_gen = int(np.flatnonzero(gb == self.ref)[0])
        self.nb, self.ng = nb, ng
        self.base = float(net.base_mva)

        # ---- variable split (state/control) ------------------------------
        nonref = [i for i in range(nb) if i != self.ref]
        pq = [i for i in range(nb) if bt[i] == BUS_PQ]
        self.nonref, self.pq = nonref, pq
        self.nx = len(nonref) + len(pq)
        self.nu = ng + (ng - 1)
        self.nonref_gens = [g for g in range(ng) if g != self.ref_gen]
        nu, nx = self.nu, self.nx
        # position of each variable in x and in u (-1: not a variable of that kind)
        self.x_theta = -np.ones(nb, dtype=np.int64)
        self.x_vm = -np.ones(nb, dtype=np.int64)
        self.u_vm = -np.ones(nb, dtype=np.int64)
        self.u_pg = -np.ones(ng, dtype=np.int64)
        for k, i in enumerate(nonref):
            self.x_theta[i] = k
        for k, i in enumerate(pq):
            self.x_vm[i] = len(nonref) + k
        for g in range(ng):
            self.u_vm[gb[g]] = g
        for k, g in enumerate(self.nonref_gens):
            self.u_pg[g] = ng + k
        # exported kinds (same convention as the C ABI's index maps)
        self.x_kind = np.array([0] * len(nonref) + [1] * len(pq), dtype=np.int32)
        self.x_bus = np.array(nonref + pq, dtype=np.int32)
        self.u_kind = np.array([1] * ng + [2] * (ng - 1), dtype=np.int32)
        self.u_ref = np.array(list(gb) + self.nonref_gens, dtype=np.int32)

        # bus-space (theta_0..theta_{nb-1}, V_0..V_{nb-1}) -> w = [u; x] index
        self.bus2w = -np.ones(2 * nb, dtype=np.int64)
        for i in range(nb):
            if self.x_theta[i] >= 0:
                self.bus2w[i] = nu + self.x_theta[i]
            if self.x_vm[i] >= 0:
                self.bus2w[nb + i] = nu + self.x_vm[i]
            if self.u_vm[i] >= 0:
                self.bus2w[nb + i] = self.u_vm[i]

        # ---- constraints -------------------------------------------------
        self.g_rows_p = nonref            # row k <-> P balance at nonref[k]
        self.g_rows_q = pq                # row len(nonref)+k <-> Q balance at pq[k]
        rate = np.asarray(net.rate)
        self.lim = np.flatnonzero(rate > 0)
        self.m = 1 + ng + 2 * self.lim.shape[0]

        # ---- admittances (pi-model lines) ---------------------------------
        z = np.asarray(net.r) + 1j * np.asarray(net.x)
        ys = 1.0 / z
        bc = np.asarray(net.b)
        self.y_ff = ys + 0.5j * bc       # = y_tt
        self.y_ft = -ys                  # = y_tf
        rows, cols, vals = [], [], []
        for l in range(net.nl):
            fb, tb = int(net.f[l]), int(net.t[l])
            rows += [fb, tb, fb, tb]
            cols += [fb, tb, tb, fb]
            vals += [self.y_ff[l], self.y_ff[l], self.y_ft[l], self.y_ft[l]]
        Y = sp.coo_matrix((np.array(vals, dtype=complex), (rows, cols)),
                          shape=(nb, nb)).tocsr()
        Y.sum_duplicates()
        Y = Y.tocoo()
        self.Ybus = Y
        self.y_i, self.y_k = Y.row.astype(np.int64), Y.col.astype(np.int64)
        self.y_G, self.y_B = Y.data.real.copy(), Y.data.imag.copy()

    # ------------------------------------------------------------------ state
    def split(self, x, u):
        """(x, u) -> per-bus theta, Vm and per-generator Pg (ref Pg = nan)."""
        net = self.net
        dt = np.result_type(x, u, float)
        theta = np.zeros(self.nb, dtype=dt)
        vm = np.zeros(self.nb, dtype=dt)
        for i in range(self.nb):
            if self.x_theta[i] >= 0:
                theta[i] = x[self.x_theta[i]]
            if self.x_vm[i] >= 0:
                vm[i] = x[self.x_vm[i]]
            if self.u_vm[i] >= 0:
                vm[i] = u[self.u_vm[i]]
        pg = np.full(self.ng, np.nan, dtype=dt)
        for g in self.nonref_gens:
            pg[g] = u[self.u_pg[g]]
        return theta, vm, pg

    def join(self, theta, vm, pg):
        """Inverse of split (ref theta and ref Pg are dropped)."""
        x = np.zeros(self.nx)
        u = np.zeros(self.nu)
        for i in range(self.nb):
            if self.x_theta[i] >= 0:
                x[self.x_theta[i]] = theta[i]
            if self.x_vm[i] >= 0:
                x[self.x_vm[i]] = vm[i]
            if self.u_vm[i] >= 0:
                u[self.u_vm[i]] = vm[i]
        for g in self.nonref_gens:
            u[self.u_pg[g]] = pg[g]
        return x, u

    # ------------------------------------------------------ term primitives
    @staticmethod
    def _phi(kind, G, B, t):
        """phi and its first two derivatives; kind 'c' (P) or 'd' (Q)."""
        c, s = np.cos(t), np.sin(t)
        if kind == "c":   # G cos t + B sin t
            return G * c + B * s, -G * s + B * c, -G * c - B * s
        return G * s - B * c, G * c + B * s, -G * s + B * c   # G sin t - B cos t

    def _terms(self, kind, a, b, G, B, theta, vm):
        """Values, gradients (4) and Hessians (4x4) of T = V_a V_b phi(th_a - th_b).

        Local variable order: (theta_a, theta_b, V_a, V_b)."""
        t = theta[a] - theta[b]
        va, vb = vm[a], vm[b]
        p, dp, ddp = self._phi(kind, G, B, t)
        val = va * vb * p
        grad = np.stack([va * vb * dp, -va * vb * dp, vb * p, va * p], axis=1)
        n = a.shape[0]
        H = np.zeros((n, 4, 4), dtype=np.result_type(val, float))
        H[:, 0, 0] = va * vb * ddp
        H[:, 0, 1] = -va * vb * ddp
        H[:, 1, 1] = va * vb * ddp
        H[:, 0, 2] = vb * dp
        H[:, 0, 3] = va * dp
        H[:, 1, 2] = -vb * dp
        H[:, 1, 3] = -va * dp
        H[:, 2, 3] = p
        for r in range(4):
            for c in range(r):
                H[:, r, c] = H[:, c, r]
        loc = np.stack([a, b, self.nb + a, self.nb + b], axis=1)  # bus-space ids
        return val, grad, H, loc

    # ------------------------------------------------------------ injections
    def injections(self, theta, vm):
        """P_i, Q_i by the polar formula summed over admittance entries."""
        vp = self._terms("c", self.y_i, self.y_k, self.y_G, self.y_B, theta, vm)[0]
        vq = self._terms("d", self.y_i, self.y_k, self.y_G, self.y_B, theta, vm)[0]
        dt = np.result_type(vp, float)
        P = np.zeros(self.nb, dtype=dt)
        Q = np.zeros(self.nb, dtype=dt)
        np.add.at(P, self.y_i, vp)
        np.add.at(Q, self.y_i, vq)
        return P, Q

    def _flow_terms(self, end, ll):
        """Terms of the flow at one end of lines ll: 'f' or 't'."""
        net = self.net
        f = np.asarray(net.f, dtype=np.int64)[ll]
        t = np.asarray(net.t, dtype=np.int64)[ll]
        a, b = (f, t) if end == "f" else (t, f)
        yff, yft = self.y_ff[ll], self.y_ft[ll]
        # self term (a, a) with Y_aa and mutual term (a, b) with Y_ab
        A = np.concatenate([a, a])
        Bb = np.concatenate([a, b])
        G = np.concatenate([yff.real, yft.real])
        B = np.concatenate([yff.imag, yft.imag])
        owner = np.concatenate([np.arange(ll.shape[0])] * 2)
        return owner, A, Bb, G, B

    def line_flows(self, theta, vm, ll=None, end="f"):
        """P and Q leaving bus `end` of each line in ll."""
        if ll is None:
            ll = np.arange(self.net.nl)
        owner, a, b, G, B = self._flow_terms(end, ll)
        vp = self._terms("c", a, b, G, B, theta, vm)[0]
        vq = self._terms("d", a, b, G, B, theta, vm)[0]
        dt = np.result_type(vp, float)
        P = np.zeros(ll.shape[0], dtype=dt)
        Q = np.zeros(ll.shape[0], dtype=dt)
        np.add.at(P, owner, vp)
        np.add.at(Q, owner, vq)
        return P, Q

    # ------------------------------------------------------------- functions
    def functions(self, x, u):
        """g (nx), h (m), f (scalar); works for complex inputs (complex step)."""
        net = self.net
        theta, vm, pg = self.split(x, u)
        P, Q = self.injections(theta, vm)
        dt = P.dtype
        pg_bus = np.zeros(self.nb, dtype=dt)
        for g in self.nonref_gens:
            pg_bus[net.gen_bus[g]] = pg[g]
        g = np.concatenate([
            np.array([P[i] - pg_bus[i] + net.pd[i] for i in self.g_rows_p], dtype=dt),
            np.array([Q[i] + net.qd[i] for i in self.g_rows_q], dtype=dt)])
        pg_ref = P[self.ref] + net.pd[self.ref]
        qg = np.array([Q[net.gen_bus[gi]] + net.qd[net.gen_bus[gi]]
                       for gi in range(self.ng)], dtype=dt)
        Pf, Qf = self.line_flows(theta, vm, self.lim, "f")
        Pt, Qt = self.line_flows(theta, vm, self.lim, "t")
        h = np.concatenate([np.array([pg_ref], dtype=dt), qg,
                            Pf * Pf + Qf * Qf, Pt * Pt + Qt * Qt])
        B = self.base
        fval = 0.0 + 0.0 * pg_ref
        for gi in range(self.ng):
            p = pg_ref if gi == self.ref_gen else pg[gi]
            fval = fval + net.c2[gi] * (B * p) ** 2 + net.c1[gi] * (B * p) + net.c0[gi]
        return g, h, fval

    def h_bounds(self):
        """Lower/upper bounds of h (Pg_ref, Qg, flows)."""
        net = self.net
        rg = self.ref_gen
        lo = np.concatenate([[net.pmin[rg]], net.qmin,
                             np.full(2 * self.lim.shape[0], -np.inf)])
        r2 = np.asarray(net.rate)[self.lim] ** 2
        hi = np.concatenate([[net.pmax[rg]], net.qmax, r2, r2])
        return lo, hi

    def var_bounds(self):
        """Bounds of x and u (theta free)."""
        net = self.net
        xl = np.full(self.nx, -np.inf)
        xu = np.full(self.nx, np.inf)
        ul = np.zeros(self.nu)
        uu = np.zeros(self.nu)
        for i in self.pq:
            xl[self.x_vm[i]] = net.vmin[i]
            xu[self.x_vm[i]] = net.vmax[i]
        for g in range(self.ng):
            b = net.gen_bus[g]
            ul[g] = net.vmin[b]
            uu[g] = net.vmax[b]
        for g in self.nonref_gens:
            ul[self.u_pg[g]] = net.pmin[g]
            uu[self.u_pg[g]] = net.pmax[g]
        return xl, xu, ul, uu

    # ----------------------------------------------------------- derivatives
    def _bus_jac(self, kind, owner, nrow, val, grad, loc):
        rows = np.repeat(owner, 4)
        cols = loc.reshape(-1)
        return sp.coo_matrix((grad.reshape(-1), (rows, cols)),
                             shape=(nrow, 2 * self.nb)).tocsr()

    def _inj_derivs(self, theta, vm):
        """Bus-space Jacobians of P and Q (nb x 2nb) and term Hessians."""
        out = {}
        for kind in ("c", "d"):
            val, grad, H, loc = self._terms(kind, self.y_i, self.y_k, self.y_G,
                                            self.y_B, theta, vm)
            J = self._bus_jac(kind, self.y_i, self.nb, val, grad, loc)
            out[kind] = (J, H, loc)
        return out

    def _flow_derivs(self, theta, vm, end):
        ll = self.lim
        owner, a, b, G, B = self._flow_terms(end, ll)
        res = {}
        for kind in ("c", "d"):
            val, grad, H, loc = self._terms(kind, a, b, G, B, theta, vm)
            v = np.zeros(ll.shape[0], dtype=np.result_type(val, float))
            np.add.at(v, owner, val)
            J = self._bus_jac(kind, owner, ll.shape[0], val, grad, loc)
            res[kind] = (v, J, H, loc, owner)
        return res

    def _to_w_cols(self, Jbus):
        """Bus-space Jacobian columns -> w = [u; x] columns (theta_ref dropped)."""
        Jbus = Jbus.tocoo()
        c = self.bus2w[Jbus.col]
        keep = c >= 0
        return sp.coo_matrix((Jbus.data[keep], (Jbus.row[keep], c[keep])),
                             shape=(Jbus.shape[0], self.nu + self.nx)).tocsr()

    def jacobians(self, x, u):
        """G = d g / d w (nx x (nu+nx)), A = d h / d w (m x (nu+nx)),
        grad f (nu+nx); all in w = [u; x] order, sparse CSR."""
        net = self.net
        theta, vm, pg = self.split(x, u)
        P, Q = self.injections(theta, vm)
        inj = self._inj_derivs(theta, vm)
        JP = self._to_w_cols(inj["c"][0])
        JQ = self._to_w_cols(inj["d"][0])
        nw = self.nu + self.nx
        # g rows
        Gm = sp.vstack([JP[self.g_rows_p, :], JQ[self.g_rows_q, :]]).tolil()
        for k, i in enumerate(self.g_rows_p):
            gens = np.flatnonzero(np.asarray(net.gen_bus) == i)
            for gi in gens:
                if gi != self.ref_gen:
                    Gm[k, self.u_pg[gi]] += -1.0
        Gm = Gm.tocsr()
        # h rows
        rows = [JP[[self.ref], :], JQ[list(np.asarray(net.gen_bus)), :]]
        for end in ("f", "t"):
            fd = self._flow_derivs(theta, vm, end)
            Pv, JPf = fd["c"][0], self._to_w_cols(fd["c"][1])
            Qv, JQf = fd["d"][0], self._to_w_cols(fd["d"][1])
            rows.append(sp.diags(2.0 * Pv) @ JPf + sp.diags(2.0 * Qv) @ JQf)
        Am = sp.vstack(rows).tocsr()
        # grad f
        B = self.base
        gf = np.zeros(nw, dtype=np.result_type(P, float))
        for g in self.nonref_gens:
            gf[self.u_pg[g]] = 2.0 * net.c2[g] * B * B * pg[g] + net.c1[g] * B
        rg = self.ref_gen
        pg_ref = P[self.ref] + net.pd[self.ref]
        dcost = 2.0 * net.c2[rg] * B * B * pg_ref + net.c1[rg] * B
        gf += dcost * np.asarray(JP[self.ref, :].todense()).ravel()
        return Gm, Am, gf

    def hessian_lagrangian(self, x, u, lam, y):
        """W = grad^2 f + sum_r lam_r grad^2 g_r + sum_j y_j grad^2 h_j,
        (nu+nx)^2 sparse, w = [u; x] order (Section 2.1's W)."""
        net = self.net
        theta, vm, pg = self.split(x, u)
        P, Q = self.injections(theta, vm)
        B = self.base
        rg = self.ref_gen
        nb = self.nb
        # weight of grad^2 P_i and grad^2 Q_i in W
        wP = np.zeros(nb)
        wQ = np.zeros(nb)
        for k, i in enumerate(self.g_rows_p):         # lam: P balance rows
            wP[i] += lam[k]
        for k, i in enumerate(self.g_rows_q):         # lam: Q balance rows
            wQ[i] += lam[len(self.g_rows_p) + k]
        wP[self.ref] += y[0]                          # h_0 = Pg_ref = P_ref + Pd_ref
        for gi in range(self.ng):                     # h_{1+g} = Qg
            wQ[net.gen_bus[gi]] += y[1 + gi]
        pg_ref = P[self.ref] + net.pd[self.ref]
        wP[self.ref] += 2.0 * net.c2[rg] * B * B * pg_ref + net.c1[rg] * B  # f
        rr, cc, vv = [], [], []

        def add_terms(weight_per_term, H, loc):
            rr.append(np.repeat(loc, 4, axis=1).reshape(-1))
            cc.append(np.tile(loc, (1, 4)).reshape(-1))
            vv.append((H * weight_per_term[:, None, None]).reshape(-1))

        for kind, wt in (("c", wP), ("d", wQ)):
            _, _, H, loc = self._terms(kind, self.y_i, self.y_k, self.y_G,
                                       self.y_B, theta, vm)
            add_terms(wt[self.y_i], H, loc)
        # grad f's rank-one part from Pg_ref^2: 2 c2 B^2 grad P_ref grad P_ref^T
        inj = self._inj_derivs(theta, vm)
        gP = np.asarray(inj["c"][0][self.ref, :].todense()).ravel()
        nzr = np.flatnonzero(gP)
        coef = 2.0 * net.c2[rg] * B * B
        rr.append(np.repeat(nzr, nzr.shape[0]))
        cc.append(np.tile(nzr, nzr.shape[0]))
        vv.append(coef * np.outer(gP[nzr], gP[nzr]).reshape(-1))
        # line flows: grad^2 (P^2 + Q^2) = 2 (gP gP^T + P H_P + gQ gQ^T + Q H_Q)
        nlim = self.lim.shape[0]
        for e, end in enumerate(("f", "t")):
            yl = y[1 + self.ng + e * nlim: 1 + self.ng + (e + 1) * nlim]
            fd = self._flow_derivs(theta, vm, end)
            for kind in ("c", "d"):
                v, J, H, loc, owner = fd[kind]
                add_terms(2.0 * yl[owner] * v[owner], H, loc)
                Jc = J.tocsr()
                for l in range(nlim):
                    row = Jc.getrow(l)
                    idx, dat = row.indices, row.data
                    rr.append(np.repeat(idx, idx.shape[0]))
                    cc.append(np.tile(idx, idx.shape[0]))
                    vv.append(2.0 * yl[l] * np.outer(dat, dat).reshape(-1))
        r = np.concatenate(rr)
        c = np.concatenate(cc)
        v = np.concatenate(vv)
        Hb = sp.coo_matrix((v, (r, c)), shape=(2 * nb, 2 * nb)).tocsr()
        Hb.sum_duplicates()
        Hb = Hb.tocoo()
        wr, wc = self.bus2w[Hb.row], self.bus2w[Hb.col]
        keep = (wr >= 0) & (wc >= 0)
        nw = self.nu + self.nx
        W = sp.coo_matrix((Hb.data[keep], (wr[keep], wc[keep])), shape=(nw, nw)).tolil()
        for g in self.nonref_gens:                    # f: c2 (B Pg)^2 of controls
            W[self.u_pg[g], self.u_pg[g]] += 2.0 * net.c2[g] * B * B
        return W.tocsr()

    def lagrangian_gradient(self, x, u, lam, y):
        """grad_w (f + lam^T g + y^T h) (the s, bound terms excluded)."""
        G, A, gf = self.jacobians(x, u)
        return gf + G.T @ lam + A.T @ y
