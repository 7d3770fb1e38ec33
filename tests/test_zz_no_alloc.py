"""rh_cholesky_solve_noalloc (workspaces in the library's static device array)
against the Cholesky stage of rh_solve_condensed_kkt: the same factor and
the same p_u, bit for bit, on two calls in a row, the second of smaller
order; the right-hand side is left unchanged."""
import numpy as np
import pytest
import torch

import synthnet
from helpers import random_point, residual_vector
from oracle.model import Model

pytestmark = pytest.mark.gpu


def _solve_both(api, net, seed):
    M = Model(net)
    G = api.Net(net)
    dev = torch.device("cuda", 0)
    T = lambda a: torch.as_tensor(np.asarray(a, np.float64), device=dev)
    x, u, lam, y, sx, su, ss = random_point(M, seed, sig_range=(10.0, 1e4))
    r = T(residual_vector(M, seed + 1))
    K, rhs = G.condense_reduced_hessian(*map(T, (x, u, lam, y, sx, su, ss)), r=r)
    K0, rhs0 = K.clone(), rhs.clone()
    delta = 0.0
    while True:
        K.copy_(K0)
        p, code = G.solve_condensed_kkt(K, delta, rhs, r)
        if code != 1:
            break
        delta = 1e-4 if delta == 0.0 else 8.0 * delta
    assert code == 0
    nu = G.nu
    K2 = K0.clone()
    xs = torch.full((nu,), np.nan, dtype=torch.float64, device=dev)
    st = torch.full((2,), -7, dtype=torch.int32, device=dev)
    api.cholesky_solve_noalloc(K2, delta, rhs, xs, st)
    torch.cuda.synchronize()
    G.close()
    return nu, delta, K0, K, K2, rhs, rhs0, p[:nu], xs, st


@pytest.mark.parametrize("first,second", [("syn1354", "syn118")])
def test_noalloc_solve_equals_condensed_solve(first, second):
    from paper_2203_11875_amd import api
    nets = {"syn1354": synthnet.case1354(0), "syn118": synthnet.case118(0)}
    orders = []
    for k, name in enumerate((first, second)):
        print(f"noalloc solve {name}", flush=True)
        nu, delta, K0, K, K2, rhs, rhs0, pu, xs, st = _solve_both(api, nets[name], 30 + k)
        orders.append(nu)
        assert st.cpu().tolist() == [0, 0]
        assert torch.equal(rhs, rhs0)                       # b is not modified
        assert torch.equal(xs, pu)                          # same p_u bit for bit
        Lk = torch.tril(K.T)                                # column-major lower triangle
        L2 = torch.tril(K2.T)
        assert torch.equal(Lk, L2)                          # same factor bit for bit
        Kd = K0.cpu().numpy().T + delta * np.eye(nu)
        want = np.linalg.solve(np.tril(Kd) + np.tril(Kd, -1).T, rhs0.cpu().numpy())
        assert np.abs(xs.cpu().numpy() - want).max() <= 1e-8 * np.abs(want).max()
    assert orders[1] < orders[0]


def test_noalloc_reports_indefinite_and_rejects_large_orders():
    from paper_2203_11875_amd import api
    from paper_2203_11875_amd._abi import RhError
    dev = torch.device("cuda", 0)
    n = 300
    rng = np.random.default_rng(3)
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    ev = np.linspace(1.0, 2.0, n)
    ev[117] = -0.5                                         # one negative eigenvalue
    A = torch.as_tensor((Q * ev) @ Q.T, device=dev)
    b = torch.ones(n, dtype=torch.float64, device=dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    st = torch.zeros(2, dtype=torch.int32, device=dev)
    print("noalloc indefinite n=300", flush=True)
    api.cholesky_solve_noalloc(A.clone(), 0.0, b, x, st)
    torch.cuda.synchronize()
    assert int(st[0]) == 1 and 0 <= int(st[1]) < n
    print("noalloc same matrix shifted", flush=True)
    api.cholesky_solve_noalloc(A.clone(), 1.0, b, x, st)
    torch.cuda.synchronize()
    assert int(st[0]) == 0
    want = np.linalg.solve((Q * (ev + 1.0)) @ Q.T, np.ones(n))
    assert np.abs(x.cpu().numpy() - want).max() <= 1e-10 * np.abs(want).max()
    big = torch.zeros((1025, 1025), dtype=torch.float64, device=dev)
    bb = torch.zeros(1025, dtype=torch.float64, device=dev)
    with pytest.raises(RhError):
        api.cholesky_solve_noalloc(big, 0.0, bb, bb.clone(), st)
