"""Thin Python binding of the C ABI (include/rhipm.h): same names, argument
marshalling only. Every step of the hot path runs in the HIP library; torch is
used for device memory and streams."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi
from ._abi import RhError

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = _abi.load()
    return _LIB


def _check(code, where):
    if code != _abi.RH_OK:
        raise _abi.RhError(code, where, lib())


class _Desc:
    """Keeps numpy copies alive while the C struct points at them."""

    def __init__(self, net):
        self.arrays = {}

        def a(name, dtype):
            v = np.ascontiguousarray(getattr(net, name), dtype=dtype)
            self.arrays[name] = v
            return v.ctypes.data_as(_abi.i32p if dtype == np.int32 else _abi.f64p)

        d = _abi.rh_network_desc()
        d.nb, d.nl, d.ng = int(net.nb), int(net.nl), int(net.ng)
        d.base_mva = float(net.base_mva)
        d.bus_type = a("bus_type", np.int32)
        for n in ("pd", "qd", "vmin", "vmax", "r", "x", "b", "rate", "c2", "c1", "c0",
                  "pmin", "pmax", "qmin", "qmax"):
            setattr(d, n, a(n, np.float64))
        d.from_ = a("f", np.int32)
        d.to = a("t", np.int32)
        d.gen_bus = a("gen_bus", np.int32)
        self.desc = d


# Launch shapes chosen by autotune(), by network structure (launch_key): Net
# takes them when its caller leaves the shape options unset.
TUNING = {}


def launch_key(net):
    """Structure of a network that its launch shape depends on (the sizes and
    the bus, branch and generator incidence; not the loads or line values),
    as a hex digest: load scenarios of one network share a key."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.asarray([int(net.nb), int(net.nl), int(net.ng)], np.int64).tobytes())
    for name in ("bus_type", "f", "t", "gen_bus"):
        h.update(np.ascontiguousarray(getattr(net, name), dtype=np.int32).tobytes())
    return h.hexdigest()


def save_tuning(path):
    """Writes TUNING as JSON ({key: [panel_width, lds_panel, cond_waves]})."""
    import json
    with open(path, "w") as f:
        json.dump({k: list(v) for k, v in TUNING.items()}, f, indent=1, sort_keys=True)


def load_tuning(path):
    """Adds the entries of a file written by save_tuning to TUNING."""
    import json
    with open(path) as f:
        for k, v in json.load(f).items():
            TUNING[str(k)] = tuple(int(x) for x in v)


def _opts(panel_width=0, lds_panel=1, refactor=0, cond_waves=0, sweep_grouping=0, ordering=0):
    o = _abi.rh_options()
    o.panel_width = int(panel_width)
    o.ordering = int(ordering)
    o.lds_panel = int(lds_panel)
    o.refactor = int(refactor)
    o.cond_waves = int(cond_waves)
    o.sweep_grouping = int(sweep_grouping)
    return o


def _info_dict(info):
    return {name: int(getattr(info, name)) for name, _ in _abi.rh_info._fields_}


class Symbolic:
    """Host-only symbolic analysis (rh_analyze_network); needs no GPU."""

    def __init__(self, net, panel_width=0, lds_panel=1, refactor=0, cond_waves=0, ordering=0):
        self._desc = _Desc(net)
        h = C.c_void_p()
        o = _opts(panel_width, lds_panel, refactor, cond_waves, 0, ordering)
        _check(lib().rh_analyze_network(C.byref(self._desc.desc), C.byref(o), C.byref(h)),
               "rh_analyze_network")
        self.h = h
        info = _abi.rh_info()
        _check(lib().rh_symbolic_info(self.h, C.byref(info)), "rh_symbolic_info")
        self.info = _info_dict(info)

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.rh_destroy_symbolic(self.h)
        self.h = None

    def index_maps(self):
        nx, nu = self.info["nx"], self.info["nu"]
        xk, xb = np.zeros(nx, np.int32), np.zeros(nx, np.int32)
        uk, ur = np.zeros(nu, np.int32), np.zeros(nu, np.int32)
        p = lambda v: v.ctypes.data_as(_abi.i32p)
        _check(lib().rh_symbolic_index_maps(self.h, p(xk), p(xb), p(uk), p(ur)),
               "rh_symbolic_index_maps")
        return xk, xb, uk, ur

    def gx_pattern(self):
        nx, nnz = self.info["nx"], self.info["nnz_gx"]
        ptr, col, perm = np.zeros(nx + 1, np.int32), np.zeros(nnz, np.int32), np.zeros(nx, np.int32)
        p = lambda v: v.ctypes.data_as(_abi.i32p)
        _check(lib().rh_symbolic_gx_pattern(self.h, p(ptr), p(col), p(perm)),
               "rh_symbolic_gx_pattern")
        return ptr, col, perm

    def host_solve(self, gx_values, b, transpose=False):
        v = np.ascontiguousarray(gx_values, np.float64)
        bb = np.ascontiguousarray(b, np.float64)
        z = np.zeros_like(bb)
        p = lambda a: a.ctypes.data_as(_abi.f64p)
        code = lib().rh_symbolic_host_solve(self.h, p(v), p(bb), p(z), 1 if transpose else 0)
        _check(code, "rh_symbolic_host_solve")
        return z

    def check_levels(self):
        return lib().rh_symbolic_check_levels(self.h)

    def check_condense(self, width=1, seed=0):
        """Host emulation of the condensation kernel on its device records
        (rh_symbolic_check_condense): largest relative error against a dense
        computation of three columns."""
        err = C.c_double(0.0)
        _check(lib().rh_symbolic_check_condense(self.h, int(width), int(seed), C.byref(err)),
               "rh_symbolic_check_condense")
        return err.value


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Net:
    """Device handle (rh_init_network). Inputs are float64 CUDA tensors.

    panel_width, lds_panel and cond_waves left as None take the shape that
    autotune() recorded for this network's structure (TUNING), else the
    library's choice (0, 1, 0)."""

    def __init__(self, net, panel_width=None, lds_panel=None, stream=None, refactor=0,
                 cond_waves=None, sweep_grouping=0, ordering=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("rhipm.Net needs a HIP device")
        if panel_width is None and lds_panel is None and cond_waves is None:
            panel_width, lds_panel, cond_waves = TUNING.get(launch_key(net), (0, 1, 0))
        panel_width = 0 if panel_width is None else panel_width
        lds_panel = 1 if lds_panel is None else lds_panel
        cond_waves = 0 if cond_waves is None else cond_waves
        self.tuned = (panel_width, lds_panel, cond_waves)
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._desc = _Desc(net)
        h = C.c_void_p()
        o = _opts(panel_width, lds_panel, refactor, cond_waves, sweep_grouping, ordering)
        _check(lib().rh_init_network(C.byref(self._desc.desc), C.byref(o),
                                     C.c_void_p(self.stream.cuda_stream), C.byref(h)),
               "rh_init_network")
        self.h = h
        info = _abi.rh_info()
        _check(lib().rh_get_info(self.h, C.byref(info)), "rh_get_info")
        self.info = _info_dict(info)
        self.nx, self.nu, self.m = self.info["nx"], self.info["nu"], self.info["m"]

    def close(self):
        if getattr(self, "h", None) and _LIB is not None:
            if getattr(self, "_ipm", None) is not None:
                self._ipm.close()
            _LIB.rh_destroy_network(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _t(self, a, n=None):
        t = self.torch
        if isinstance(a, t.Tensor):
            v = a.to(device=self.device, dtype=t.float64).contiguous()
        else:
            v = t.as_tensor(np.ascontiguousarray(a, np.float64), device=self.device)
        if n is not None and v.numel() != n:
            raise ValueError(f"expected {n} entries, got {v.numel()}")
        return v

    def index_maps(self):
        nx, nu = self.nx, self.nu
        xk, xb = np.zeros(nx, np.int32), np.zeros(nx, np.int32)
        uk, ur = np.zeros(nu, np.int32), np.zeros(nu, np.int32)
        p = lambda v: v.ctypes.data_as(_abi.i32p)
        _check(lib().rh_get_index_maps(self.h, p(xk), p(xb), p(uk), p(ur)), "rh_get_index_maps")
        return xk, xb, uk, ur

    def set_loads(self, pd, qd):
        pd, qd = self._t(pd), self._t(qd)
        _check(lib().rh_set_loads(self.h, _ptr(pd), _ptr(qd)), "rh_set_loads")
        self._keep = (pd, qd)

    def power_flow(self, u, x0, tol=1e-10, max_iter=20):
        """Newton-Raphson power flow (rh_power_flow): returns (x, status,
        iterations, max |g|); x starts at x0."""
        u = self._t(u, self.nu)
        x = self._t(x0, self.nx).clone()
        it, res = C.c_int32(0), C.c_double(0.0)
        code = lib().rh_power_flow(self.h, _ptr(u), _ptr(x), float(tol), int(max_iter),
                                   C.byref(it), C.byref(res))
        if code < 0:
            _check(code, "rh_power_flow")
        return x, code, it.value, res.value

    def eval_residual(self, x, u):
        t = self.torch
        x, u = self._t(x, self.nx), self._t(u, self.nu)
        g = t.empty(self.nx, dtype=t.float64, device=self.device)
        h = t.empty(self.m, dtype=t.float64, device=self.device)
        f = t.empty(1, dtype=t.float64, device=self.device)
        _check(lib().rh_eval_residual(self.h, _ptr(x), _ptr(u), _ptr(g), _ptr(h), _ptr(f)),
               "rh_eval_residual")
        return g, h, f

    def condense_reduced_hessian(self, x, u, lam, y, sig_x, sig_u, sig_s, r=None, K=None,
                                 rhs=None):
        t = self.torch
        nx, nu, m = self.nx, self.nu, self.m
        args = [self._t(x, nx), self._t(u, nu), self._t(lam, nx), self._t(y, m),
                self._t(sig_x, nx), self._t(sig_u, nu), self._t(sig_s, m)]
        rr = self._t(r, nu + 2 * nx + 2 * m) if r is not None else None
        if K is None:
            K = t.empty((nu, nu), dtype=t.float64, device=self.device)
        if rr is not None and rhs is None:
            rhs = t.empty(nu, dtype=t.float64, device=self.device)
        # K is column-major nu x nu with ld = nu: a contiguous (nu, nu) tensor
        # read as row-major holds K^T; K is symmetric after the call.
        code = lib().rh_condense_reduced_hessian(self.h, *[_ptr(a) for a in args], _ptr(rr),
                                                 _ptr(K), nu, _ptr(rhs) if rr is not None else None)
        _check(code, "rh_condense_reduced_hessian")
        self._keep = (args, rr)
        return K, rhs

    def profile_enable(self, on=True):
        _check(lib().rh_profile_enable(self.h, 1 if on else 0), "rh_profile_enable")

    def profile_read(self):
        n = len(_abi.PHASES)
        ms = (C.c_double * n)()
        calls = (C.c_int64 * n)()
        _check(lib().rh_profile_read(self.h, ms, calls), "rh_profile_read")
        return {name: (float(ms[k]), int(calls[k])) for k, name in enumerate(_abi.PHASES)}

    def profile_kernel_trace(self):
        t = (C.c_int64 * 512)()
        _check(lib().rh_profile_kernel_trace(self.h, t), "rh_profile_kernel_trace")
        names = ["start", "filled", "L", "U", "hvp", "UT", "LT", "written", "zstored", "kstream",
                 "entry"]
        out = {names[k]: (t[k] - t[0]) / 100.0 for k in range(11)}   # microseconds
        # Cholesky factorisation launches: [start, panel k-1 applied, factored,
        # stores issued] of the diagonal work-group, microseconds from launch 0
        chol = []
        for k in range(24):
            v = [t[256 + 8 * k + j] for j in range(4)]
            if v[0] == 0:
                break
            chol.append([(x - t[256]) / 100.0 for x in v])
        out["cholesky"] = chol
        return out

    def solve_condensed_kkt(self, K, delta_w, rhs, r):
        """Returns (p, status) where status is the rh_status integer; raises on
        hard errors only."""
        t = self.torch
        nx, nu, m = self.nx, self.nu, self.m
        rr = self._t(r, nu + 2 * nx + 2 * m)
        rhs = self._t(rhs, nu)
        p = t.empty(nu + 2 * nx + 2 * m, dtype=t.float64, device=self.device)
        # the status comes back as the return code (no device copy wanted)
        code = lib().rh_solve_condensed_kkt(self.h, _ptr(K), nu, float(delta_w), _ptr(rhs),
                                            _ptr(rr), _ptr(p), None)
        if code < 0:
            _check(code, "rh_solve_condensed_kkt")
        return p, code


def cholesky_solve_noalloc(K, delta_w, b, x, status, stream=None):
    """rh_cholesky_solve_noalloc: K (n x n float64 CUDA tensor, read as
    column-major with leading dimension n: a row-major symmetric K is the same
    matrix) factored in place, x = (K + delta_w I)^{-1} b, status (int32[2]
    on the device) as in the header. Enqueued on `stream` (a torch stream,
    default: the current one); the call allocates nothing and does not
    synchronise."""
    import torch
    n = int(b.shape[0])
    for t_, shape, dt in ((K, (n, n), torch.float64), (b, (n,), torch.float64),
                          (x, (n,), torch.float64), (status, (2,), torch.int32)):
        if tuple(t_.shape) != shape or t_.dtype != dt or not t_.is_cuda or not t_.is_contiguous():
            raise ValueError("cholesky_solve_noalloc: K (n, n), b, x (n,) float64 and status (2,) "
                             "int32, contiguous device tensors")
    s = stream if stream is not None else torch.cuda.current_stream(K.device)
    _check(lib().rh_cholesky_solve_noalloc(_ptr(K), n, n, float(delta_w), _ptr(b), _ptr(x),
                                           _ptr(status), C.c_void_p(s.cuda_stream)),
           "rh_cholesky_solve_noalloc")


def autotune(net, point, widths=(1, 2, 4), lds=(1, 0), waves=(1, 2, 4, 8), reps=3, record=True):
    """Launch-shape autotuner: times the condensation (all columns with the
    right-hand side) of `net` at `point` = (x, u, lam, y, sig_x, sig_u,
    sig_s, r) for each panel width, panel placement (lds 1: in LDS, with the
    sweep metadata in global memory where the panel fills the LDS) and waves
    per work-group (several only for one column in LDS), and returns
    (best (width, lds, waves), {(width, lds, waves): microseconds}).
    Configurations the device cannot hold are skipped. With record, the
    best shape goes into TUNING under the network's launch_key, so that Net
    handles of this network (any loads) created without shape options use
    it; save_tuning / load_tuning keep it across processes."""
    import time
    import torch
    times = {}
    for w in widths:
        for l in lds:
            for nw in waves:
                if nw != 1 and (w != 1 or not l):
                    continue
                try:
                    G = Net(net, panel_width=w, lds_panel=l, cond_waves=nw)
                except RhError:
                    continue
                got = (int(G.info["panel_width"]), int(G.info["lds_panel"]) != 0,
                       int(G.info["cond_waves"]))
                if got != (w, bool(l), nw):
                    G.close()
                    continue
                G.condense_reduced_hessian(*point[:7], r=point[7])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    G.condense_reduced_hessian(*point[:7], r=point[7])
                torch.cuda.synchronize()
                times[(w, l, nw)] = 1e6 * (time.perf_counter() - t0) / reps
                G.close()
    best = min(times, key=times.get)
    if record:
        TUNING[launch_key(net)] = tuple(int(v) for v in best)
    return best, times


class Batch:
    """Several device network handles condensed and solved together
    (rh_batch_*): one launch per kernel for all instances."""

    def __init__(self, nets, stream=None):
        import torch
        self.torch = torch
        self.nets = list(nets)
        arr = (C.c_void_p * len(self.nets))(*[n.h for n in self.nets])
        h = C.c_void_p()
        st = stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream
        _check(lib().rh_batch_create(arr, len(self.nets), C.c_void_p(st), C.byref(h)),
               "rh_batch_create")
        self.h = h
        self._keep = None

    def condense(self, points):
        """points: per instance (x, u, lam, y, sig_x, sig_u, sig_s, r); returns
        lists of K (nu x nu, column-major as in Net) and rhs."""
        t = self.torch
        items = (_abi.rh_batch_condense_item * len(self.nets))()
        keep, Ks, rhss = [], [], []
        for i, (G, pt) in enumerate(zip(self.nets, points)):
            nx, nu, m = G.nx, G.nu, G.m
            x, u, lam, y, sx, su, ss, r = pt
            a = [G._t(x, nx), G._t(u, nu), G._t(lam, nx), G._t(y, m), G._t(sx, nx),
                 G._t(su, nu), G._t(ss, m), G._t(r, nu + 2 * nx + 2 * m)]
            K = t.empty((nu, nu), dtype=t.float64, device=G.device)
            rhs = t.empty(nu, dtype=t.float64, device=G.device)
            it = items[i]
            for name, v in zip(("x", "u", "lam", "y", "sig_x", "sig_u", "sig_s", "r"), a):
                setattr(it, name, _ptr(v))
            it.K, it.ldk, it.rhs = _ptr(K), nu, _ptr(rhs)
            keep.append(a)
            Ks.append(K)
            rhss.append(rhs)
        _check(lib().rh_batch_condense(self.h, items), "rh_batch_condense")
        self._keep = keep
        return Ks, rhss

    def solve(self, Ks, delta_w, rhss, rs):
        """Returns (list of p, list of status codes)."""
        t = self.torch
        items = (_abi.rh_batch_solve_item * len(self.nets))()
        ps, keep = [], []
        for i, G in enumerate(self.nets):
            nx, nu, m = G.nx, G.nu, G.m
            rr = G._t(rs[i], nu + 2 * nx + 2 * m)
            rhs = G._t(rhss[i], nu)
            p = t.empty(nu + 2 * nx + 2 * m, dtype=t.float64, device=G.device)
            it = items[i]
            it.K, it.ldk = _ptr(Ks[i]), nu
            it.delta_w = float(delta_w[i] if hasattr(delta_w, "__len__") else delta_w)
            it.rhs, it.r, it.p = _ptr(rhs), _ptr(rr), _ptr(p)
            keep.append((rr, rhs))
            ps.append(p)
        st = (C.c_int32 * len(self.nets))()
        code = lib().rh_batch_solve(self.h, items, st)
        if code < 0 and not any(int(v) for v in st):
            _check(code, "rh_batch_solve")
        self._keep = keep
        return ps, [int(v) for v in st]

    def _items(self, points, delta_w):
        t = self.torch
        ci = (_abi.rh_batch_condense_item * len(self.nets))()
        si = (_abi.rh_batch_solve_item * len(self.nets))()
        keep, Ks, rhss, ps = [], [], [], []
        for i, (G, pt) in enumerate(zip(self.nets, points)):
            nx, nu, m = G.nx, G.nu, G.m
            x, u, lam, y, sx, su, ss, r = pt
            a = [G._t(x, nx), G._t(u, nu), G._t(lam, nx), G._t(y, m), G._t(sx, nx),
                 G._t(su, nu), G._t(ss, m), G._t(r, nu + 2 * nx + 2 * m)]
            K = t.empty((nu, nu), dtype=t.float64, device=G.device)
            rhs = t.empty(nu, dtype=t.float64, device=G.device)
            p = t.empty(nu + 2 * nx + 2 * m, dtype=t.float64, device=G.device)
            for name, v in zip(("x", "u", "lam", "y", "sig_x", "sig_u", "sig_s", "r"), a):
                setattr(ci[i], name, _ptr(v))
            ci[i].K, ci[i].ldk, ci[i].rhs = _ptr(K), nu, _ptr(rhs)
            si[i].K, si[i].ldk, si[i].rhs, si[i].r, si[i].p = _ptr(K), nu, _ptr(rhs), _ptr(a[7]), _ptr(p)
            si[i].delta_w = float(delta_w[i] if hasattr(delta_w, "__len__") else delta_w)
            keep.append(a)
            Ks.append(K)
            rhss.append(rhs)
            ps.append(p)
        return ci, si, keep, Ks, rhss, ps

    def capture(self, points, delta_w=0.0):
        """Capture one batched step (condensation + solve) into a HIP graph
        (rh_batch_capture); replay() runs it again on the same buffers."""
        ci, si, keep, Ks, rhss, ps = self._items(points, delta_w)
        _check(lib().rh_batch_capture(self.h, ci, si), "rh_batch_capture")
        self._graph = (ci, si, keep, Ks, rhss, ps)

    def replay(self):
        """Returns (Ks, rhss, ps, status codes) of the captured step's buffers."""
        ci, si, keep, Ks, rhss, ps = self._graph
        st = (C.c_int32 * len(self.nets))()
        code = lib().rh_batch_replay(self.h, None, None, st)
        if code < 0 and not any(int(v) for v in st):
            _check(code, "rh_batch_replay")
        return Ks, rhss, ps, [int(v) for v in st]

    def close(self):
        if getattr(self, "h", None) is not None and _LIB is not None:
            lib().rh_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _info_ipm(info):
    return {name: (float(getattr(info, name)) if isinstance(getattr(info, name), float)
                   else int(getattr(info, name)))
            for name, _ in _abi.rh_ipm_info._fields_}


class Ipm:
    """Interior-point solver on a device network handle (rh_ipm_*)."""

    def __init__(self, net, x0=None, u0=None, tol=1e-6, max_iter=200, mu_init=0.1,
                 obj_scale=0.0):
        if not isinstance(net, Net):
            raise TypeError("Ipm needs an api.Net")
        self.net = net
        o = _abi.rh_ipm_options()
        _check(lib().rh_ipm_default_options(C.byref(o)), "rh_ipm_default_options")
        o.tol, o.max_iter, o.mu_init, o.obj_scale = float(tol), int(max_iter), float(mu_init), \
            float(obj_scale)
        xs = net._t(x0, net.nx) if x0 is not None else None
        us = net._t(u0, net.nu) if u0 is not None else None
        h = C.c_void_p()
        _check(lib().rh_ipm_create(net.h, C.byref(o), _ptr(xs), _ptr(us), C.byref(h)),
               "rh_ipm_create")
        self.h = h
        net._ipm = self

    def close(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.rh_ipm_destroy(self.h)
        self.h = None
        if getattr(self, "net", None) is not None and getattr(self.net, "_ipm", None) is self:
            self.net._ipm = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self):
        """One iteration; returns (status, info dict)."""
        info = _abi.rh_ipm_info()
        code = lib().rh_ipm_step(self.h, C.byref(info))
        if code < 0:
            _check(code, "rh_ipm_step")
        return code, _info_ipm(info)

    def solve(self):
        info = _abi.rh_ipm_info()
        code = lib().rh_ipm_solve(self.h, C.byref(info))
        if code < 0:
            _check(code, "rh_ipm_solve")
        return code, _info_ipm(info)

    def state(self):
        t = self.net.torch
        n = self.net
        out = [t.empty(k, dtype=t.float64, device=n.device) for k in (n.nx, n.nu, n.m, n.nx, n.m)]
        _check(lib().rh_ipm_get_state(self.h, *[_ptr(a) for a in out]), "rh_ipm_get_state")
        return dict(zip(("x", "u", "s", "lam", "y"), out))

    def outputs(self):
        """(Pg per generator, Vm per bus, f) at the current point
        (rh_ipm_outputs)."""
        t, n = self.net.torch, self.net
        pg = t.empty(n.info["ng"], dtype=t.float64, device=n.device)
        vm = t.empty(n.info["nb"], dtype=t.float64, device=n.device)
        f = t.empty(1, dtype=t.float64, device=n.device)
        _check(lib().rh_ipm_outputs(self.h, _ptr(pg), _ptr(vm), _ptr(f)), "rh_ipm_outputs")
        return pg, vm, f[0]

    def backward(self, dpg=None, dvm=None, df=None, want_xi=False):
        """Gradient of dpg . Pg + dvm . Vm + df f in (Pd, Qd) (rh_ipm_backward);
        returns (grad_pd, grad_qd[, xi])."""
        t, n = self.net.torch, self.net
        nb, ng = n.info["nb"], n.info["ng"]
        a = n._t(dpg, ng) if dpg is not None else None
        b = n._t(dvm, nb) if dvm is not None else None
        c = n._t(t.as_tensor(df, dtype=t.float64).reshape(1), 1) if df is not None else None
        gpd = t.empty(nb, dtype=t.float64, device=n.device)
        gqd = t.empty(nb, dtype=t.float64, device=n.device)
        xi = (t.empty(n.nu + 2 * n.nx + 2 * n.m, dtype=t.float64, device=n.device)
              if want_xi else None)
        code = lib().rh_ipm_backward(self.h, _ptr(a), _ptr(b), _ptr(c), _ptr(gpd), _ptr(gqd),
                                     _ptr(xi))
        _check(code, "rh_ipm_backward")
        return (gpd, gqd, xi) if want_xi else (gpd, gqd)


class IpmBatch:
    """Solvers on the networks of a batch stepped in lockstep
    (rh_ipm_batch_step): the condensation and the first solve of every
    iteration are one batched launch each over all instances."""

    def __init__(self, batch, ipms):
        if len(ipms) != len(batch.nets):
            raise ValueError("one solver per network of the batch")
        self.batch, self.ipms = batch, list(ipms)
        self._h = (C.c_void_p * len(ipms))(*[i.h.value for i in ipms])

    def step(self):
        """One lockstep iteration; returns [(status, info dict)] per solver."""
        n = len(self.ipms)
        infos = (_abi.rh_ipm_info * n)()
        codes = (C.c_int32 * n)()
        _check(lib().rh_ipm_batch_step(self.batch.h, C.cast(self._h, C.c_void_p),
                                       C.cast(infos, C.c_void_p), C.cast(codes, C.c_void_p)),
               "rh_ipm_batch_step")
        return [(int(codes[i]), _info_ipm(infos[i])) for i in range(n)]

    def backward(self, dpg=None, dvm=None, df=None):
        """Gradients in (Pd, Qd) of every converged solver at once
        (rh_ipm_batch_backward); dpg (S, ng), dvm (S, nb), df (S) device
        tensors or None. Returns (grad_pd (S, nb), grad_qd (S, nb), codes)."""
        t = self.batch.torch
        n0 = self.ipms[0].net
        S, nb = len(self.ipms), n0.info["nb"]
        dev = n0.device

        def rows(a, width):
            if a is None:
                return None, None
            a = a.to(device=dev, dtype=t.float64).reshape(S, width).contiguous()
            arr = (C.c_void_p * S)(*[a[i].data_ptr() for i in range(S)])
            return a, arr

        keep = [rows(dpg, n0.info["ng"]), rows(dvm, nb), rows(df, 1)]
        gpd = t.empty((S, nb), dtype=t.float64, device=dev)
        gqd = t.empty((S, nb), dtype=t.float64, device=dev)
        gp = (C.c_void_p * S)(*[gpd[i].data_ptr() for i in range(S)])
        gq = (C.c_void_p * S)(*[gqd[i].data_ptr() for i in range(S)])
        codes = (C.c_int32 * S)()
        arg = lambda k: C.cast(k[1], C.c_void_p) if k[1] is not None else None
        _check(lib().rh_ipm_batch_backward(self.batch.h, C.cast(self._h, C.c_void_p),
                                           arg(keep[0]), arg(keep[1]), arg(keep[2]),
                                           C.cast(gp, C.c_void_p), C.cast(gq, C.c_void_p),
                                           C.cast(codes, C.c_void_p)),
               "rh_ipm_batch_backward")
        return gpd, gqd, [int(codes[i]) for i in range(S)]


class RedLin:
    """Reduce-then-linearize solver (Algorithm 2) on a device network handle
    (rh_redlin_*)."""

    def __init__(self, net, x0=None, u0=None, tol=1e-6, max_iter=200, mu_init=0.1,
                 obj_scale=0.0):
        if not isinstance(net, Net):
            raise TypeError("RedLin needs an api.Net")
        self.net = net
        o = _abi.rh_ipm_options()
        _check(lib().rh_ipm_default_options(C.byref(o)), "rh_ipm_default_options")
        o.tol, o.max_iter, o.mu_init, o.obj_scale = float(tol), int(max_iter), float(mu_init), \
            float(obj_scale)
        xs = net._t(x0, net.nx) if x0 is not None else None
        us = net._t(u0, net.nu) if u0 is not None else None
        h = C.c_void_p()
        _check(lib().rh_redlin_create(net.h, C.byref(o), _ptr(xs), _ptr(us), C.byref(h)),
               "rh_redlin_create")
        self.h = h
        mr, nxb = C.c_int64(0), C.c_int64(0)
        _check(lib().rh_redlin_dims(self.h, C.byref(mr), C.byref(nxb)), "rh_redlin_dims")
        self.mr, self.nxb = mr.value, nxb.value

    def close(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.rh_redlin_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self):
        info = _abi.rh_ipm_info()
        code = lib().rh_redlin_step(self.h, C.byref(info))
        if code < 0:
            _check(code, "rh_redlin_step")
        return code, _info_ipm(info)

    def solve(self):
        info = _abi.rh_ipm_info()
        code = lib().rh_redlin_solve(self.h, C.byref(info))
        if code < 0:
            _check(code, "rh_redlin_solve")
        return code, _info_ipm(info)

    def state(self):
        t, n = self.net.torch, self.net
        out = [t.empty(k, dtype=t.float64, device=n.device)
               for k in (n.nx, n.nu, self.mr, n.nx, self.mr)]
        _check(lib().rh_redlin_get_state(self.h, *[_ptr(a) for a in out]), "rh_redlin_get_state")
        return dict(zip(("x", "u", "s", "lam", "y"), out))


class OPFLayer:
    """Differentiable AC optimal power flow: loads (Pd, Qd) -> (Pg, Vm, f).

    The forward pass sets the loads on the layer's device network and runs
    the interior-point method to tol; the backward pass differentiates the
    solution by the implicit function theorem (rh_ipm_backward: one adjoint
    solve with the condensed KKT system at the final iterate). Each forward
    call keeps its solver for its backward pass; the loads are set again
    before differentiating, so several forward calls may precede the
    backward ones."""

    def __init__(self, net, tol=1e-8, max_iter=200, **net_kw):
        self.net = net if isinstance(net, Net) else Net(net, **net_kw)
        self.tol, self.max_iter = float(tol), int(max_iter)

    def __call__(self, pd, qd):
        return _OPFFunction.apply(pd, qd, self)

    def _solve(self, pd, qd):
        n = self.net
        n.set_loads(pd, qd)
        ipm = Ipm(n, tol=self.tol, max_iter=self.max_iter)
        n._ipm = None       # the solver belongs to the autograd graph
        code, info = ipm.solve()
        if code != _abi.RH_OK:
            _check(code, "rh_ipm_solve")
        self.last_info = info
        return ipm, info


class OPFBatchLayer:
    """OPFLayer over a batch of load scenarios of one network: (Pd, Qd) of
    shape (S, nb) -> (Pg (S, ng), Vm (S, nb), f (S)). The forward pass solves
    all scenarios in lockstep (rh_ipm_batch_step: one batched condensation
    and solve per round, each scenario on its own handle and stream); the
    backward pass differentiates each scenario as OPFLayer does. Gradients
    equal those of OPFLayer scenario by scenario, bit for bit."""

    def __init__(self, net, count, tol=1e-8, max_iter=200, **net_kw):
        import torch
        self.torch = torch
        self.count, self.tol, self.max_iter = int(count), float(tol), int(max_iter)
        self.nets = [Net(net, stream=torch.cuda.Stream(), **net_kw) for _ in range(self.count)]
        self.batch = Batch(self.nets, stream=torch.cuda.Stream())
        self.nb, self.ng = self.nets[0].info["nb"], self.nets[0].info["ng"]

    def __call__(self, pd, qd):
        return _OPFBatchFunction.apply(pd, qd, self)

    def _solve(self, pd, qd):
        self._fork()
        ipms = []
        for i, G in enumerate(self.nets):
            G.set_loads(pd[i], qd[i])
            ipm = Ipm(G, tol=self.tol, max_iter=self.max_iter)
            G._ipm = None        # the solvers belong to the autograd graph
            ipms.append(ipm)
        ib = IpmBatch(self.batch, ipms)
        self._ib = ib
        done = [False] * self.count
        infos = [None] * self.count
        for _ in range(self.max_iter + 2):
            for i, (code, info) in enumerate(ib.step()):
                if done[i]:
                    continue
                if code != _abi.RH_OK:
                    _check(code, "rh_ipm_batch_step")
                if info["converged"]:
                    done[i], infos[i] = True, info
            if all(done):
                break
        if not all(done):
            _check(_abi.RH_NOT_CONVERGED, "rh_ipm_batch_step")
        self.last_infos = infos
        return ipms, ib

    def _fork(self):
        """Every handle's stream waits for the caller's (inputs ready)."""
        cur = self.torch.cuda.current_stream()
        for G in self.nets:
            G.stream.wait_stream(cur)

    def _join(self):
        """The caller's stream waits for every handle's (outputs ready)."""
        cur = self.torch.cuda.current_stream()
        for G in self.nets:
            cur.wait_stream(G.stream)


def _make_opf_function():
    import torch

    class _OPF(torch.autograd.Function):
        @staticmethod
        def forward(ctx, pd, qd, layer):
            n = layer.net
            pdd, qdd = n._t(pd, n.info["nb"]), n._t(qd, n.info["nb"])
            ipm, info = layer._solve(pdd, qdd)
            pg, vm, f = ipm.outputs()
            ctx.ipm, ctx.layer, ctx.loads, ctx.info = ipm, layer, (pdd, qdd), info
            ctx.devices = (torch.as_tensor(pd).device, torch.as_tensor(qd).device)
            return pg, vm, f

        @staticmethod
        def backward(ctx, gpg, gvm, gf):
            n = ctx.layer.net
            n.set_loads(*ctx.loads)
            gpd, gqd = ctx.ipm.backward(gpg, gvm, gf)
            return gpd.to(ctx.devices[0]), gqd.to(ctx.devices[1]), None

    class _OPFBatch(torch.autograd.Function):
        @staticmethod
        def forward(ctx, pd, qd, layer):
            S, nb = layer.count, layer.nb
            n0 = layer.nets[0]
            pdd = n0._t(pd).reshape(S, nb).contiguous()
            qdd = n0._t(qd).reshape(S, nb).contiguous()
            ipms, ib = layer._solve(pdd, qdd)
            outs = [ipm.outputs() for ipm in ipms]
            layer._join()
            ctx.ipms, ctx.ib, ctx.layer, ctx.loads = ipms, ib, layer, (pdd, qdd)
            ctx.devices = (torch.as_tensor(pd).device, torch.as_tensor(qd).device)
            ctx.shapes = (torch.as_tensor(pd).shape, torch.as_tensor(qd).shape)
            return (torch.stack([o[0] for o in outs]), torch.stack([o[1] for o in outs]),
                    torch.stack([o[2] for o in outs]))

        @staticmethod
        def backward(ctx, gpg, gvm, gf):
            layer = ctx.layer
            pdd, qdd = ctx.loads
            S, dev = layer.count, layer.nets[0].device

            def dense(a, width):
                # on the caller's stream, before the handles' streams wait for it
                if a is None:
                    return None
                return a.to(device=dev, dtype=torch.float64).reshape(S, width).contiguous()

            gpg, gvm, gf = dense(gpg, layer.ng), dense(gvm, layer.nb), dense(gf, 1)
            layer._fork()
            for i, G in enumerate(layer.nets):
                G.set_loads(pdd[i], qdd[i])
            gp, gq, codes = ctx.ib.backward(gpg, gvm, gf)
            for c in codes:
                _check(c, "rh_ipm_batch_backward")
            layer._join()
            return (gp.reshape(ctx.shapes[0]).to(ctx.devices[0]),
                    gq.reshape(ctx.shapes[1]).to(ctx.devices[1]), None)

    return _OPF, _OPFBatch


class _Lazy:
    def __init__(self, which):
        self.which, self.fn = which, None

    def apply(self, *a):
        if self.fn is None:
            self.fn = _make_opf_function()[self.which]
        return self.fn.apply(*a)


_OPFFunction = _Lazy(0)
_OPFBatchFunction = _Lazy(1)
