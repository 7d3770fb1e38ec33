"""Pins of the oracle's reduction/condensation against brute force, finite
differences through Newton power-flow solves, and the inertia theorem."""
import numpy as np
import pytest

import synthnet
from oracle.model import Model
from oracle import reduction as R, powerflow as PF, cholesky as C
from helpers import random_point, balanced_control, residual_vector

NETS = [("syn5", lambda: synthnet.small(5, 7, 2, seed=1)),
        ("syn9", lambda: synthnet.case9(3)),
        ("syn12", lambda: synthnet.small(12, 18, 4, seed=3))]


def _blocks(M, seed, **kw):
    x, u, lam, y, sx, su, ss = random_point(M, seed, **kw)
    return R.kkt_blocks(M, x, u, lam, y, sx, su, ss)


@pytest.mark.parametrize("name,mk", NETS)
@pytest.mark.parametrize("seed", [0, 1])
def test_kcond_is_inverse_of_kaug_inverse_uu_block(name, mk, seed):
    """Theorems 1-2: K_cond^{-1} = [K_aug^{-1}]_uu (dense brute force)."""
    M = Model(mk())
    B = _blocks(M, seed)
    Kc = R.condensed_matrix(B)
    inv_uu = np.linalg.inv(R.augmented_matrix(B))[:M.nu, :M.nu]
    assert np.abs(np.linalg.inv(inv_uu) - Kc).max() <= 1e-9 * np.abs(Kc).max()


@pytest.mark.parametrize("name,mk", NETS)
@pytest.mark.parametrize("delta", [0.0, 3.0])
def test_condensed_solve_equals_augmented_solve(name, mk, delta):
    M = Model(mk())
    B = _blocks(M, 2)
    S, lu = R.sensitivity(B)
    Kc = R.condensed_matrix(B, S) + delta * np.eye(M.nu)
    r = residual_vector(M, 5)
    b, _, _ = R.condensed_rhs(B, r, S, lu)
    pu = np.linalg.solve(R.symmetrize(Kc), b)
    got = R.recover(B, r, pu, S, lu)
    want = R.solve_augmented(B, r, delta_w=delta)
    for g, w in zip(got, want):
        assert np.abs(g - w).max() <= 1e-9 * max(1.0, np.abs(w).max())


@pytest.mark.parametrize("name,mk", NETS[1:])
def test_sensitivity_is_derivative_of_power_flow(name, mk):
    """Implicit function theorem: dx(u)/du = S = -G_x^{-1} G_u."""
    M = Model(mk())
    x0, u = balanced_control(M)
    x0 = PF.solve_pf(M, u, x0)
    B = R.kkt_blocks(M, x0, u, np.zeros(M.nx), np.zeros(M.m), np.zeros(M.nx),
                     np.zeros(M.nu), np.zeros(M.m))
    S, _ = R.sensitivity(B)
    h = 1e-6
    Sfd = np.zeros_like(S)
    for j in range(M.nu):
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        Sfd[:, j] = (PF.solve_pf(M, up, x0) - PF.solve_pf(M, um, x0)) / (2 * h)
    assert np.abs(S - Sfd).max() <= 1e-7 * np.abs(S).max()


@pytest.mark.parametrize("name,mk", NETS[1:])
def test_kcond_is_reduced_lagrangian_hessian(name, mk):
    """Reduced-derivatives theorem: with the adjoint multiplier and Sigma = 0,
    K_cond equals the Hessian of L_r(u) = f(x(u), u) + y^T h(x(u), u),
    obtained here by central differences of the adjoint reduced gradient."""
    M = Model(mk())
    x0, u = balanced_control(M)
    rng = np.random.default_rng(4)
    y = rng.uniform(0, 5, M.m)
    g0, xs, lam = PF.reduced_gradient(M, u, x0, y)
    B = R.kkt_blocks(M, xs, u, lam, y, np.zeros(M.nx), np.zeros(M.nu), np.zeros(M.m))
    Kc = R.condensed_matrix(B)
    h = 1e-5
    H = np.zeros_like(Kc)
    for j in range(M.nu):
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        H[:, j] = (PF.reduced_gradient(M, up, xs, y)[0]
                   - PF.reduced_gradient(M, um, xs, y)[0]) / (2 * h)
    assert np.abs(H - Kc).max() <= 1e-6 * np.abs(Kc).max()


@pytest.mark.parametrize("name,mk", NETS[1:])
def test_slack_term_is_reduced_jacobian_gram(name, mk):
    """K_cond(Sigma_s) - K_cond(0) = A_hat^T Sigma_s A_hat with the reduced
    Jacobian A_hat = d h(x(u), u)/du taken by differences of PF solves."""
    M = Model(mk())
    x0, u = balanced_control(M)
    x0 = PF.solve_pf(M, u, x0)
    rng = np.random.default_rng(6)
    ss = 10 ** rng.uniform(-1, 1, M.m)
    z = np.zeros
    B0 = R.kkt_blocks(M, x0, u, z(M.nx), z(M.m), z(M.nx), z(M.nu), z(M.m))
    B1 = R.kkt_blocks(M, x0, u, z(M.nx), z(M.m), z(M.nx), z(M.nu), ss)
    h = 1e-6
    Ahat = np.zeros((M.m, M.nu))
    for j in range(M.nu):
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        hp = M.functions(PF.solve_pf(M, up, x0), up)[1]
        hm = M.functions(PF.solve_pf(M, um, x0), um)[1]
        Ahat[:, j] = (hp - hm) / (2 * h)
    D = R.condensed_matrix(B1) - R.condensed_matrix(B0)
    want = Ahat.T @ (ss[:, None] * Ahat)
    assert np.abs(D - want).max() <= 1e-6 * np.abs(want).max()


@pytest.mark.parametrize("name,mk", NETS)
def test_symmetry(name, mk):
    M = Model(mk())
    Kc = R.condensed_matrix(_blocks(M, 3))
    assert np.abs(Kc - Kc.T).max() <= 1e-11 * np.abs(Kc).max()


@pytest.mark.parametrize("name,mk", NETS)
def test_inertia_theorem(name, mk):
    """Cholesky of K_cond succeeds iff I(K_aug) = (nx+nu+m, nx+m, 0)."""
    M = Model(mk())
    want = (M.nx + M.nu + M.m, M.nx + M.m, 0)
    seen = set()
    for seed in range(12):
        kw = {"sig_range": (1e-1, 1e3)} if seed % 2 else {"lam_scale": 400.0}
        B = _blocks(M, seed, **kw)
        Kc = R.symmetrize(R.condensed_matrix(B))
        pd = C.try_cholesky(Kc) is not None
        assert pd == (R.inertia(R.augmented_matrix(B)) == want)
        seen.add(pd)
    assert seen == {True, False}, "pick draws that exercise both outcomes"


def test_inertia_correction_reaches_positive_definite():
    M = Model(synthnet.case9(1))
    B = _blocks(M, 0, lam_scale=400.0)
    Kc = R.symmetrize(R.condensed_matrix(B))
    L, delta = C.factor_with_correction(Kc)
    assert L is not None and delta > 0
    assert np.linalg.eigvalsh(Kc + delta * np.eye(M.nu)).min() > 0
    assert np.linalg.eigvalsh(Kc + delta / 100 * np.eye(M.nu)).min() <= 0
    bb = np.arange(M.nu, dtype=float)
    xs = C.solve_with_factor(L, bb)
    assert np.allclose((Kc + delta * np.eye(M.nu)) @ xs, bb, rtol=1e-10, atol=1e-10)


def test_sparse_columns_match_dense():
    M = Model(synthnet.case118(0))
    B = _blocks(M, 1)
    Kc = R.condensed_matrix(B)
    cols = [0, 5, 53, 54, 106]
    Ks, _ = R.condensed_columns_sparse(B, cols)
    assert np.abs(Ks - Kc[:, cols]).max() <= 1e-9 * np.abs(Kc).max()


@pytest.mark.parametrize("seed", [0, 1])
def test_sparse_condensation_equals_dense(seed):
    """The sparse-LU forms (used at 9241 buses) equal the dense definitions."""
    net = synthnet.case118(0)
    M = Model(net)
    x, u, lam, y, sx, su, ss = random_point(M, seed)
    B = R.kkt_blocks(M, x, u, lam, y, sx, su, ss)
    Kc = R.condensed_matrix(B)
    cols = [0, 5, M.nu - 1]
    got, splu = R.condensed_columns_sparse(B, cols)
    np.testing.assert_allclose(got, Kc[:, cols], rtol=0, atol=1e-9 * np.abs(Kc).max())
    r = residual_vector(M, seed)
    b, _, _ = R.condensed_rhs(B, r)
    bs, _ = R.condensed_rhs_sparse(B, r, splu)
    np.testing.assert_allclose(bs, b, rtol=0, atol=1e-9 * np.abs(b).max())


@pytest.mark.parametrize("delta", [0.0, 3.0])
def test_sparse_augmented_solve_and_recovery_equal_dense(delta):
    """The sparse-LU solve of K_aug (the oracle IPM's large-network option)
    and the sparse-LU recovery (used at 9241 buses) equal the dense forms on
    118 buses: the same system, a different factorisation."""
    M = Model(synthnet.case118(0))
    x, u, lam, y, sx, su, ss = random_point(M, 2)
    B = R.kkt_blocks(M, x, u, lam, y, sx, su, ss)
    r = residual_vector(M, 3)
    want = np.concatenate(R.solve_augmented(B, r, delta_w=delta))
    got = np.concatenate(R.solve_augmented_sparse(B, r, delta_w=delta))
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()
    np.testing.assert_array_equal(R.augmented_matrix_sparse(B, delta).toarray(),
                                  R.augmented_matrix(B, delta))
    S, lu = R.sensitivity(B)
    pu = want[:M.nu]
    dense = np.concatenate(R.recover(B, r, pu, S, lu))
    sparse = np.concatenate(R.recover_sparse(B, r, pu))
    assert np.abs(sparse - dense).max() <= 1e-9 * np.abs(dense).max()
