"""Oracle: reduction and condensation of the KKT system (test infrastructure).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this.

Definitions followed (paper, Section 2.2.1 and Section 3.3):

* augmented system K_aug p = -r (eq. kktmatrix:normal), unknowns
  p = (p_u, p_x, p_s, p_lambda, p_y), Sigma_u, Sigma_x, Sigma_s diagonal;
* Theorem 1 (reduction through the invertible G_x) and Theorem 2 (condensation
  through the nonsingular Sigma_s), taken in the order K_aug -> K_cond -> K_red
  that the discussion after Theorem 2 recommends;
* the batched reduction identity (eq. algo:reduction):
      K_cond = [I; S]^T K [I; S],  S = -G_x^{-1} G_u,
  with K = W + diag(Sigma_u, Sigma_x) + A^T Sigma_s A.

Readings (the paper is inconsistent or silent on these points):

* The printed K_aug carries -I in its (s, y) and (y, s) blocks, which does not
  follow from the Lagrangian f + lambda^T g + y^T (h + s) - z^T s. Linearising
  that Lagrangian's stationarity in s and the constraint h + s = 0 gives +I;
  this oracle uses +I. K_cond does not depend on the choice (A^T Sigma_s A is
  sign-free); the right-hand side and the recovery do, and they are pinned by
  a direct solve of the same K_aug.
* Theorem 2 and the reduction identity print K without the Sigma_u / Sigma_x
  terms that Theorem 1 carries; K here includes them, as Theorem 1 requires.
* The product in the reduction's third step needs G_u^T (not G_u).
* Regularisation delta_w is added to the control block only, i.e.
  K_cond + delta_w I, which is K_aug with W_uu + delta_w I.

Vectors are in w = [u; x] order (see oracle.model).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def _dense(M):
    return M.toarray() if sp.issparse(M) else np.asarray(M)


def kkt_blocks(model, x, u, lam, y, sig_x, sig_u, sig_s):
    """Derivative blocks at (x, u, lam, y) and the matrix
    K = W + diag(Sigma_u, Sigma_x) + A^T diag(Sigma_s) A (sparse)."""
    G, A, gf = model.jacobians(x, u)
    W = model.hessian_lagrangian(x, u, lam, y)
    sig = np.concatenate([sig_u, sig_x])
    K = W + sp.diags(sig) + A.T @ sp.diags(sig_s) @ A
    return {"G": G.tocsr(), "A": A.tocsr(), "gf": gf, "W": W.tocsr(),
            "K": K.tocsr(), "nu": model.nu, "nx": model.nx, "m": model.m,
            "sig_x": np.asarray(sig_x, float), "sig_u": np.asarray(sig_u, float),
            "sig_s": np.asarray(sig_s, float)}


def sensitivity(blocks):
    """S = -G_x^{-1} G_u by a dense LU with partial pivoting (nx x nu)."""
    nu = blocks["nu"]
    G = blocks["G"]
    Gx = _dense(G[:, nu:])
    Gu = _dense(G[:, :nu])
    lu = sla.lu_factor(Gx)
    return -sla.lu_solve(lu, Gu), lu


def condensed_matrix(blocks, S=None):
    """K_cond = [I; S]^T K [I; S] (dense nu x nu), not symmetrised."""
    nu = blocks["nu"]
    if S is None:
        S, _ = sensitivity(blocks)
    T = np.vstack([np.eye(nu), S])
    K = blocks["K"]
    return T.T @ (K @ T)


def symmetrize(Kc):
    return 0.5 * (Kc + Kc.T)


def condensed_rhs(blocks, r, S=None, lu=None):
    """Condensed right-hand side b with K_cond p_u = b.

    r = (r1, r2, r3, r4, r5) packed as [r1 (nu), r2 (nx), r3 (m), r4 (nx), r5 (m)].
    Eliminating p_s = -r5 - A p and p_y = -r3 - Sigma_s p_s from K_aug gives
        K p + G^T p_lambda = -rt,   rt = [r1; r2] + A^T (Sigma_s r5 - r3);
    then p = [I; S] p_u + [0; d] with d = -G_x^{-1} r4 (G p = -r4), and
    multiplying by [I; S]^T (which annihilates G^T) gives
        K_cond p_u = -([I; S]^T rt + [I; S]^T K [0; d]).
    """
    nu, nx, m = blocks["nu"], blocks["nx"], blocks["m"]
    if S is None or lu is None:
        S, lu = sensitivity(blocks)
    r1, r2, r3, r4, r5 = unpack(r, nu, nx, m)
    A, K, sig_s = blocks["A"], blocks["K"], blocks["sig_s"]
    rt = np.concatenate([r1, r2]) + A.T @ (sig_s * r5 - r3)
    d = -sla.lu_solve(lu, r4)
    Kd = K @ np.concatenate([np.zeros(nu), d])
    T = np.vstack([np.eye(nu), S])
    return -(T.T @ rt + T.T @ Kd), rt, d


def recover(blocks, r, pu, S=None, lu=None):
    """Full step (p_u, p_x, p_s, p_lambda, p_y) from p_u (Theorems 1-2):
    p_x = S p_u + d, p_lambda = -G_x^{-T}(rt_x + (K p)_x), p_s = -r5 - A p,
    p_y = -r3 - Sigma_s p_s."""
    nu, nx, m = blocks["nu"], blocks["nx"], blocks["m"]
    if S is None or lu is None:
        S, lu = sensitivity(blocks)
    r1, r2, r3, r4, r5 = unpack(r, nu, nx, m)
    _, rt, d = condensed_rhs(blocks, r, S, lu)
    px = S @ pu + d
    p = np.concatenate([pu, px])
    Kp = blocks["K"] @ p
    plam = -sla.lu_solve(lu, rt[nu:] + Kp[nu:], trans=1)
    ps = -r5 - blocks["A"] @ p
    py = -r3 - blocks["sig_s"] * ps
    return pu, px, ps, plam, py


def unpack(r, nu, nx, m):
    r = np.asarray(r, float)
    o = np.cumsum([0, nu, nx, m, nx, m])
    if r.shape[0] != o[-1]:
        raise ValueError("bad residual length")
    return [r[o[i]:o[i + 1]] for i in range(5)]


def augmented_matrix(blocks, delta_w=0.0):
    """Dense K_aug (eq. kktmatrix:normal, +I reading of the s/y blocks),
    unknown order (p_u, p_x, p_s, p_lambda, p_y)."""
    nu, nx, m = blocks["nu"], blocks["nx"], blocks["m"]
    W = _dense(blocks["W"]).copy()
    W[np.arange(nu), np.arange(nu)] += blocks["sig_u"] + delta_w
    W[nu + np.arange(nx), nu + np.arange(nx)] += blocks["sig_x"]
    G = _dense(blocks["G"])
    A = _dense(blocks["A"])
    n = nu + nx + m + nx + m
    K = np.zeros((n, n))
    iw = slice(0, nu + nx)
    i_s = slice(nu + nx, nu + nx + m)
    il = slice(nu + nx + m, nu + 2 * nx + m)
    iy = slice(nu + 2 * nx + m, n)
    K[iw, iw] = W
    K[iw, il] = G.T
    K[il, iw] = G
    K[iw, iy] = A.T
    K[iy, iw] = A
    K[i_s, i_s] = np.diag(blocks["sig_s"])
    K[i_s, iy] = np.eye(m)
    K[iy, i_s] = np.eye(m)
    return K


def solve_augmented(blocks, r, delta_w=0.0):
    """Brute-force step: dense solve of K_aug p = -r."""
    nu, nx, m = blocks["nu"], blocks["nx"], blocks["m"]
    p = np.linalg.solve(augmented_matrix(blocks, delta_w), -np.asarray(r, float))
    o = np.cumsum([0, nu, nx, m, nx, m])
    return [p[o[i]:o[i + 1]] for i in range(5)]


def augmented_matrix_sparse(blocks, delta_w=0.0):
    """K_aug of augmented_matrix as a sparse matrix (same blocks, same order)."""
    nu, nx, m = blocks["nu"], blocks["nx"], blocks["m"]
    sig = np.concatenate([blocks["sig_u"] + delta_w, blocks["sig_x"]])
    W = blocks["W"] + sp.diags(sig)
    G, A = blocks["G"], blocks["A"]
    I = sp.identity(m, format="csr")
    return sp.bmat([[W, None, G.T, A.T],
                    [None, sp.diags(blocks["sig_s"]), None, I],
                    [G, None, None, None],
                    [A, I, None, None]], format="csc")


def solve_augmented_sparse(blocks, r, delta_w=0.0):
    """The step of solve_augmented (K_aug p = -r) by a sparse LU with partial
    pivoting (SuperLU) instead of a dense one: for networks whose dense K_aug
    is too large to factor at every iteration."""
    import scipy.sparse.linalg as spla
    nu, nx, m = blocks["nu"], blocks["nx"], blocks["m"]
    lu = spla.splu(augmented_matrix_sparse(blocks, delta_w), permc_spec="COLAMD",
                   diag_pivot_thresh=1.0)
    p = lu.solve(-np.asarray(r, float))
    o = np.cumsum([0, nu, nx, m, nx, m])
    return [p[o[i]:o[i + 1]] for i in range(5)]


def inertia(M, tol=None):
    """(n+, n-, n0) of a symmetric matrix by its eigenvalues."""
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    if tol is None:   # eigenvalue error bound of a backward-stable solver
        tol = M.shape[0] * np.finfo(float).eps * np.abs(ev).max()
    return int((ev > tol).sum()), int((ev < -tol).sum()), int((np.abs(ev) <= tol).sum())


def condensed_columns_sparse(blocks, cols, splu=None):
    """Selected columns of K_cond with a sparse LU of G_x (for networks where
    dense G_x is too large): column j = [I; S]^T K [e_j; S e_j], with
    S e_j = -G_x^{-1} G_u e_j and S^T v = -G_u^T G_x^{-T} v."""
    import scipy.sparse.linalg as spla
    nu = blocks["nu"]
    G = blocks["G"].tocsc()
    Gx, Gu = G[:, nu:].tocsc(), G[:, :nu].tocsc()
    if splu is None:
        splu = spla.splu(Gx, permc_spec="COLAMD", diag_pivot_thresh=1.0)
    K = blocks["K"]
    out = np.zeros((nu, len(cols)))
    for k, j in enumerate(cols):
        ej = np.zeros(nu)
        ej[j] = 1.0
        sj = -splu.solve(Gu @ ej)
        q = K @ np.concatenate([ej, sj])
        out[:, k] = q[:nu] - Gu.T @ splu.solve(q[nu:], trans="T")
    return out, splu


def condensed_rhs_sparse(blocks, r, splu=None):
    """condensed_rhs with a sparse LU of G_x (large networks): d = -G_x^{-1} r4
    and [I; S]^T v = v_u - G_u^T G_x^{-T} v_x."""
    import scipy.sparse.linalg as spla
    nu, nx, m = blocks["nu"], blocks["nx"], blocks["m"]
    G = blocks["G"].tocsc()
    Gx, Gu = G[:, nu:].tocsc(), G[:, :nu].tocsc()
    if splu is None:
        splu = spla.splu(Gx, permc_spec="COLAMD", diag_pivot_thresh=1.0)
    r1, r2, r3, r4, r5 = unpack(r, nu, nx, m)
    A, K, sig_s = blocks["A"], blocks["K"], blocks["sig_s"]
    rt = np.concatenate([r1, r2]) + A.T @ (sig_s * r5 - r3)
    d = -splu.solve(r4)
    v = rt + K @ np.concatenate([np.zeros(nu), d])
    return -(v[:nu] - Gu.T @ splu.solve(v[nu:], trans="T")), splu


def recover_sparse(blocks, r, pu, splu=None):
    """recover() with a sparse LU of G_x: p_x = -G_x^{-1}(G_u p_u + r4),
    p_lambda = -G_x^{-T}(rt_x + (K p)_x), p_s = -r5 - A p,
    p_y = -r3 - Sigma_s p_s."""
    import scipy.sparse.linalg as spla
    nu, nx, m = blocks["nu"], blocks["nx"], blocks["m"]
    G = blocks["G"].tocsc()
    Gx, Gu = G[:, nu:].tocsc(), G[:, :nu].tocsc()
    if splu is None:
        splu = spla.splu(Gx, permc_spec="COLAMD", diag_pivot_thresh=1.0)
    r1, r2, r3, r4, r5 = unpack(r, nu, nx, m)
    A, K, sig_s = blocks["A"], blocks["K"], blocks["sig_s"]
    pu = np.asarray(pu, float)
    rt = np.concatenate([r1, r2]) + A.T @ (sig_s * r5 - r3)
    px = -splu.solve(Gu @ pu + r4)
    p = np.concatenate([pu, px])
    Kp = K @ p
    plam = -splu.solve(rt[nu:] + Kp[nu:], trans="T")
    ps = -r5 - A @ p
    py = -r3 - sig_s * ps
    return pu, px, ps, plam, py
