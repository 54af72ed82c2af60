"""Pins of the oracle's adjoint (Sec. 2, eq. adj) and of its implicit-Euler heat rollout (Sec. A.1).

Every check leans on something other than the oracle's own formulas: finite differences of
element matrices built by independent quadrature (tests/indep.py), invariance of the bilinear
forms under rigid motions and their homogeneity under scaling, the closed-form compliance
sensitivity (the analogue of the SIMP expression in the supplementary inverse-design experiment),
and finite differences of the
rollout loss.
"""
from __future__ import annotations

import numpy as np
import pytest

import indep
import meshgen
import oracle


def _rand_simplex(rng, dim, min_vol=0.02):
    while True:
        X = rng.random((dim + 1, dim))
        if indep.simplex_volume(X) > min_vol:
            return X


def _phi_indep(X, c, lam, u, w, mass):
    K, _ = indep.laplace_element(X, c, 0.0)
    M = indep.mass_element(X)
    A = K + M if mass else K
    return lam @ A @ u - lam @ M @ w


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mass", [False, True])
def test_element_adjoint_matches_fd_of_independent_matrices(dim, mass):
    rng = np.random.default_rng(10 + dim)
    h = 1e-6
    for _ in range(3):
        X = _rand_simplex(rng, dim)
        c = float(np.exp(rng.standard_normal()))
        lam, u, w = (rng.standard_normal(dim + 1) for _ in range(3))
        dlogc, dx = oracle.p1_adjoint_element(X, c, lam, u, w, mass=mass)
        K, _ = indep.laplace_element(X, c, 0.0)
        assert dlogc == pytest.approx(lam @ K @ u, rel=1e-12, abs=1e-13)
        fd = np.zeros_like(dx)
        for a in range(dim + 1):
            for i in range(dim):
                Xp, Xm = X.copy(), X.copy()
                Xp[a, i] += h
                Xm[a, i] -= h
                fd[a, i] = (_phi_indep(Xp, c, lam, u, w, mass) - _phi_indep(Xm, c, lam, u, w, mass)) / (2 * h)
        assert np.abs(dx - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_element_adjoint_invariants(dim):
    """Translation and rotation leave Phi unchanged; scaling by s multiplies the stiffness part by
    s^(d-2) and the mass part by s^d, so sum_a x_a . dPhi/dx_a = (d-2) Phi_K + d Phi_M."""
    rng = np.random.default_rng(20 + dim)
    for _ in range(4):
        X = _rand_simplex(rng, dim)
        c = 0.7
        lam, u, w = (rng.standard_normal(dim + 1) for _ in range(3))
        _, dx = oracle.p1_adjoint_element(X, c, lam, u, w, mass=True)
        assert np.abs(dx.sum(axis=0)).max() < 1e-12 * np.abs(dx).max() * 10
        R = X.T @ dx  # sum_a x_a dx_a^T: symmetric for a rotation-invariant Phi
        assert np.abs(R - R.T).max() < 1e-11 * np.abs(R).max()
        K, _ = indep.laplace_element(X, c, 0.0)
        M = indep.mass_element(X)
        phi_k = lam @ K @ u
        phi_m = lam @ M @ (u - w)
        assert np.sum(X * dx) == pytest.approx((dim - 2) * phi_k + dim * phi_m, rel=1e-10, abs=1e-12)


def test_element_adjoint_without_w_and_degenerate():
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    d1 = oracle.p1_adjoint_element(X, 1.0, np.ones(3), np.arange(3.0), None, mass=True)
    d2 = oracle.p1_adjoint_element(X, 1.0, np.ones(3), np.arange(3.0), np.zeros(3), mass=True)
    assert d1[0] == d2[0] and np.array_equal(d1[1], d2[1])
    with pytest.raises(oracle.OracleError):
        oracle.p1_adjoint_element(np.array([[0.0, 0.0], [1.0, 1.0], [2.0, 2.0]]), 1.0,
                                  np.ones(3), np.ones(3), None)


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_global_adjoint_matches_fd_of_dense_independent_assembly(dim, n):
    """Reduce onto nodes: the global coordinate gradient equals central differences of
    lam^T (K + M) u - lam^T M w assembled densely from independent element matrices."""
    d = meshgen.poisson_inputs(dim, n, seed=3)
    coords, conn, a = d["coords"], d["conn"], d["a"]
    rng = np.random.default_rng(4)
    nv = coords.shape[0]
    lam, u, w = (rng.standard_normal(nv) for _ in range(3))

    def phi(xy):
        A = np.zeros((nv, nv))
        M = np.zeros((nv, nv))
        for e, g in enumerate(conn):
            K, _ = indep.laplace_element(xy[g], a[e], 0.0)
            Me = indep.mass_element(xy[g])
            A[np.ix_(g, g)] += K + Me
            M[np.ix_(g, g)] += Me
        return lam @ A @ u - lam @ M @ w

    dlogc, dx = oracle.p1_adjoint(coords, conn, a, lam, u, w, mass=True)
    h = 1e-6
    for v in rng.choice(nv, size=min(nv, 6), replace=False):
        for i in range(dim):
            xp, xm = coords.copy(), coords.copy()
            xp[v, i] += h
            xm[v, i] -= h
            fd = (phi(xp) - phi(xm)) / (2 * h)
            assert dx[v, i] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    for e in rng.choice(conn.shape[0], size=5, replace=False):
        K, _ = indep.laplace_element(coords[conn[e]], a[e], 0.0)
        assert dlogc[e] == pytest.approx(lam[conn[e]] @ K @ u[conn[e]], rel=1e-12)


def test_compliance_closed_form():
    """Compliance C = F^T u with K(a) u = F: dC/da_e = -u_e^T (K_e / a_e) u_e (the analogue of the
    SIMP sensitivity of the supplementary inverse-design experiment), i.e. dC/dlog a_e = -u_e^T K_e u_e; checked against central
    differences of C computed by assembly and a direct solve."""
    d = meshgen.poisson_inputs(2, 6, seed=5)
    coords, conn, a, f = d["coords"], d["conn"], d["a"], d["f"]
    bnd = meshgen.boundary_vertices(coords)

    def compliance(log_a):
        A = oracle.assemble_p1(coords, conn, np.exp(log_a), f)
        u = oracle.condensed_solve(A, bnd)
        return A.rhs @ u, u

    C0, u = compliance(np.log(a))
    # adjoint of C = F^T u: lam = -u (eq. adj sign), dC/dlog a = lam^T (dK/dlog a) u = -u^T K_e u
    dlogc, _ = oracle.p1_adjoint(coords, conn, a, u, u)
    closed = np.array([-(u[g] @ indep.laplace_element(coords[g], a[e], 0.0)[0] @ u[g]) for e, g in enumerate(conn)])
    np.testing.assert_allclose(-dlogc, closed, rtol=1e-10, atol=1e-14)
    h = 1e-6
    for e in [0, 17, 40, 71]:
        lp, lm = np.log(a), np.log(a)
        lp[e] += h
        lm[e] -= h
        fd = (compliance(lp)[0] - compliance(lm)[0]) / (2 * h)
        assert closed[e] == pytest.approx(fd, rel=1e-6, abs=1e-12)


def test_heat_rollout_and_adjoint_fd():
    """End-to-end: the rollout's gradient (log a, coordinates, initial state) equals central
    differences of L = ||u^N - target||^2 through the rollout."""
    d = meshgen.heat_inputs(5, seed=0)
    coords, conn, log_a = d["coords"], d["conn"], d["log_a"]
    bnd = meshgen.boundary_vertices(coords)
    dt, N = 1e-2, 6
    u0 = np.sin(np.pi * coords[:, 0]) * np.sin(np.pi * coords[:, 1])
    target = np.random.default_rng(1).standard_normal(coords.shape[0]) * 0.1

    def loss(c, la, w0):
        U = oracle.heat_rollout(c, conn, la, w0, dt, N, bnd)
        return np.sum((U[-1] - target) ** 2), U

    L0, U = loss(coords, log_a, u0)
    assert np.all(U[1:, bnd] == 0.0)
    gla, gx, gu0 = oracle.heat_adjoint(coords, conn, log_a, U, dt, 2 * (U[-1] - target), bnd)
    h = 1e-6
    for e in [0, 9, 23, 44]:
        p, m = log_a.copy(), log_a.copy()
        p[e] += h
        m[e] -= h
        fd = (loss(coords, p, u0)[0] - loss(coords, m, u0)[0]) / (2 * h)
        assert gla[e] == pytest.approx(fd, rel=1e-5, abs=1e-11)
    interior = np.setdiff1d(np.arange(coords.shape[0]), bnd)
    for v in interior[[0, 3, 7]]:
        for i in range(2):
            p, m = coords.copy(), coords.copy()
            p[v, i] += h
            m[v, i] -= h
            fd = (loss(p, log_a, u0)[0] - loss(m, log_a, u0)[0]) / (2 * h)
            assert gx[v, i] == pytest.approx(fd, rel=1e-5, abs=1e-10)
    for v in [interior[2], bnd[1]]:
        p, m = u0.copy(), u0.copy()
        p[v] += h
        m[v] -= h
        fd = (loss(coords, log_a, p)[0] - loss(coords, log_a, m)[0]) / (2 * h)
        assert gu0[v] == pytest.approx(fd, rel=1e-5, abs=1e-10)
