"""Pins of the oracle's implicit-Euler heat rollout and its adjoint (SM A.1, method of lines;
Sec. 2, eq. adj) that do not reuse the oracle's time-step matrices.

The stiffness and mass matrices here come from the independent quadrature route
(tests/indep.py), assembled densely.  Two facts fix where dt enters the step
(M + dt K) u^{n+1} = M u^n:

* a generalised eigenvector K v = mu M v of the free block decays by exactly
  (1 + dt mu)^{-1} per step, and its discrete adjoint carries the same factor;
* with a = 1 on the unit square, the rollout from sin(pi x) sin(pi y) approaches
  exp(-2 pi^2 t) sin(pi x) sin(pi y) at the rate O(h^2 + dt).

Doubling dt, dropping M from the right-hand side, or stepping with K alone fails them.
"""
from __future__ import annotations

import numpy as np
import pytest
import scipy.linalg

import indep
import meshgen
import oracle


def _dense_km(coords, conn, a):
    nv = coords.shape[0]
    K = np.zeros((nv, nv))
    M = np.zeros((nv, nv))
    for e, g in enumerate(conn):
        Ke, _ = indep.laplace_element(coords[g], a[e], 0.0)
        K[np.ix_(g, g)] += Ke
        M[np.ix_(g, g)] += indep.mass_element(coords[g])
    return K, M


def _modes(n=4, seed=2):
    d = meshgen.heat_inputs(n, seed=seed)
    coords, conn, log_a = d["coords"], d["conn"], d["log_a"]
    bnd = meshgen.boundary_vertices(coords)
    free = np.setdiff1d(np.arange(coords.shape[0]), bnd)
    K, M = _dense_km(coords, conn, np.exp(log_a))
    mu, V = scipy.linalg.eigh(K[np.ix_(free, free)], M[np.ix_(free, free)])
    return coords, conn, log_a, bnd, free, K, M, mu, V


@pytest.mark.parametrize("dt,nsteps", [(1e-2, 5), (1e-3, 20)])
def test_rollout_decays_generalised_eigenmodes(dt, nsteps):
    coords, conn, log_a, bnd, free, K, M, mu, V = _modes()
    nv = coords.shape[0]
    for j in (0, len(mu) // 2, len(mu) - 1):
        u0 = np.zeros(nv)
        u0[free] = V[:, j]
        U = oracle.heat_rollout(coords, conn, log_a, u0, dt, nsteps, bnd)
        r = 1.0 / (1.0 + dt * mu[j])
        for n in range(nsteps + 1):
            np.testing.assert_allclose(U[n], r ** n * u0, rtol=0, atol=1e-12 * np.max(np.abs(u0)))
    # a mixture of modes decays mode by mode
    c = np.random.default_rng(0).standard_normal(len(mu))
    u0 = np.zeros(nv)
    u0[free] = V @ c
    U = oracle.heat_rollout(coords, conn, log_a, u0, dt, nsteps, bnd)
    expect = np.zeros(nv)
    expect[free] = V @ (c / (1.0 + dt * mu) ** nsteps)
    np.testing.assert_allclose(U[-1], expect, rtol=0, atol=1e-12 * np.max(np.abs(u0)))


def test_adjoint_of_a_mode_in_closed_form():
    """L = (M v)^T u^N from u^0 = v, with K v = mu M v and r = 1 / (1 + dt mu):
    u^n = r^n v and the adjoint states are lam^n = r^(N - n + 1) v, so
    dL/du^0 = r^N M v and dL/dlog a_e = -dt N r^(N+1) v_e^T K_e v_e."""
    coords, conn, log_a, bnd, free, K, M, mu, V = _modes(seed=5)
    nv = coords.shape[0]
    dt, N = 1e-2, 6
    a = np.exp(log_a)
    for j in (1, len(mu) - 2):
        v = np.zeros(nv)
        v[free] = V[:, j]
        r = 1.0 / (1.0 + dt * mu[j])
        U = oracle.heat_rollout(coords, conn, log_a, v, dt, N, bnd)
        g = M @ v
        g[bnd] = 0.0
        gla, _, gu0 = oracle.heat_adjoint(coords, conn, log_a, U, dt, g, bnd)
        np.testing.assert_allclose(gu0, r ** N * (M @ v), rtol=0, atol=1e-12 * np.max(np.abs(M @ v)))
        expect = np.array([-dt * N * r ** (N + 1) * (v[gi] @ indep.laplace_element(coords[gi], a[e], 0.0)[0] @ v[gi])
                           for e, gi in enumerate(conn)])
        np.testing.assert_allclose(gla, expect, rtol=1e-10, atol=1e-14 * np.max(np.abs(expect)))


def _separable_error(n, dt, nsteps):
    d = meshgen.heat_inputs(n, seed=0, jitter=0.0)
    coords, conn = d["coords"], d["conn"]
    bnd = meshgen.boundary_vertices(coords)
    u0 = np.sin(np.pi * coords[:, 0]) * np.sin(np.pi * coords[:, 1])
    U = oracle.heat_rollout(coords, conn, np.zeros(conn.shape[0]), u0, dt, nsteps, bnd)
    exact = np.exp(-2 * np.pi ** 2 * dt * nsteps) * u0
    return np.max(np.abs(U[-1] - exact)) / np.max(np.abs(exact))


def test_rollout_converges_to_the_separable_solution():
    """a = 1 on the unjittered grid: u(t) = exp(-2 pi^2 t) sin(pi x) sin(pi y).  At t = 0.02,
    refining h by 2 and dt by 4 cuts the error about fourfold (first order in dt, second in h)."""
    e1 = _separable_error(8, 4e-3, 5)
    e2 = _separable_error(16, 1e-3, 20)
    e3 = _separable_error(32, 2.5e-4, 80)
    assert e3 < 5e-4, e3
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)
    assert 3.0 < e2 / e3 < 5.0, (e2, e3)
