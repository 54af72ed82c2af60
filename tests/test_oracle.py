"""Pins of the FP64 oracle against facts fixed outside it (no GPU).

Each test checks the oracle against something it does not compute itself:
hand-derived reference elements (tests/golden), an independent Vandermonde +
collapsed-Gauss route (tests/indep.py), the cotangent formulas, invariants of
the continuous operators (zero row sums, symmetry, rigid modes, partition of
unity), patch tests, and brute-force dense assembly on tiny meshes.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import meshgen
import oracle
import indep

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "p1_reference_elements.txt")


def _read_golden():
    out, name = {}, None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            name = line[1:-1]
            out[name] = []
            continue
        out[name].append([float(Fraction(t)) for t in line.split()])
    return {k: np.array(v) for k, v in out.items()}


def _rand_simplex(rng, dim, min_vol=0.02):
    while True:
        X = rng.random((dim + 1, dim))
        if indep.simplex_volume(X) > min_vol:
            return X


# ------------------------------------------------------------------ elements

@pytest.mark.parametrize("shape", ["triangle", "tet"])
def test_reference_elements_golden(shape):
    g = _read_golden()
    X = g[f"{shape}_vertices"]
    K, F = oracle.p1_laplace_element(X, 1.0, 1.0)
    np.testing.assert_allclose(K, g[f"{shape}_K"], atol=1e-15)
    np.testing.assert_allclose(F, g[f"{shape}_F"].ravel(), atol=1e-16)
    np.testing.assert_allclose(oracle.p1_mass_element(X), g[f"{shape}_M"], atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
def test_p1_matches_independent_quadrature(dim):
    rng = np.random.default_rng(10 + dim)
    for _ in range(20):
        X = _rand_simplex(rng, dim)
        a, f = np.exp(rng.standard_normal()), rng.uniform(-1, 1)
        K, F = oracle.p1_laplace_element(X, a, f)
        Ki, Fi = indep.laplace_element(X, a, f)
        np.testing.assert_allclose(K, Ki, atol=1e-12 * np.abs(Ki).max())
        np.testing.assert_allclose(F, Fi, atol=1e-14)
        np.testing.assert_allclose(oracle.p1_mass_element(X), indep.mass_element(X), atol=1e-15)


def test_cotangent_formulas():
    rng = np.random.default_rng(3)
    for _ in range(20):
        X = _rand_simplex(rng, 2)
        np.testing.assert_allclose(oracle.p1_laplace_element(X)[0], indep.cot_laplace_triangle(X), atol=1e-12)
        X = _rand_simplex(rng, 3)
        np.testing.assert_allclose(oracle.p1_laplace_element(X)[0], indep.cot_laplace_tet(X), atol=1e-12)


def test_equilateral_and_regular():
    s3 = np.sqrt(3.0)
    X = np.array([[0, 0], [1, 0], [0.5, s3 / 2]])
    K = oracle.p1_laplace_element(X)[0]
    np.testing.assert_allclose(np.diag(K), 1 / s3, rtol=1e-14)
    np.testing.assert_allclose(K[0, 1], -1 / (2 * s3), rtol=1e-14)
    L = 2.0  # regular tet of edge L: off-diagonal -L/(12 sqrt 2), diagonal L/(4 sqrt 2)
    X = L / np.sqrt(8.0) * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float)
    K = oracle.p1_laplace_element(X)[0]
    np.testing.assert_allclose(np.diag(K), L / (4 * np.sqrt(2)), rtol=1e-13)
    off = K[~np.eye(4, dtype=bool)]
    np.testing.assert_allclose(off, -L / (12 * np.sqrt(2)), rtol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_invariance_and_scaling(dim):
    rng = np.random.default_rng(5)
    X = _rand_simplex(rng, dim)
    K, F = oracle.p1_laplace_element(X, 1.3, 0.4)
    # translation + rotation
    Q, _ = np.linalg.qr(rng.standard_normal((dim, dim)))
    K2, F2 = oracle.p1_laplace_element(X @ Q.T + rng.standard_normal(dim), 1.3, 0.4)
    np.testing.assert_allclose(K2, K, atol=1e-12)
    np.testing.assert_allclose(F2, F, atol=1e-14)
    # relabelling permutes rows and columns
    p = rng.permutation(dim + 1)
    K3, F3 = oracle.p1_laplace_element(X[p], 1.3, 0.4)
    np.testing.assert_allclose(K3, K[np.ix_(p, p)], atol=1e-12)
    np.testing.assert_allclose(F3, F[p], atol=1e-15)
    # scaling: K ~ s^(d-2), F ~ s^d
    K4, F4 = oracle.p1_laplace_element(2.5 * X, 1.3, 0.4)
    np.testing.assert_allclose(K4, K * 2.5 ** (dim - 2), atol=1e-12)
    np.testing.assert_allclose(F4, F * 2.5 ** dim, atol=1e-14)


def test_degenerate_element_rejected():
    X = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0]], dtype=float)
    with pytest.raises(oracle.OracleError):
        oracle.p1_laplace_element(X)
    with pytest.raises(oracle.OracleError):
        oracle.p2_elasticity_element(X, 1.0, 1.0)


def test_monomial_rule_against_quadrature():
    rng = np.random.default_rng(7)
    X = _rand_simplex(rng, 3)
    g, vol = oracle.simplex_geometry(X)
    pts, wts = indep.simplex_quadrature(X, 6)
    lam = np.linalg.solve(np.vstack([np.ones(4), X.T]), np.vstack([np.ones(len(pts)), pts.T]))  # [4, Q]
    for e in [(1, 0, 0, 0), (2, 0, 0, 0), (1, 1, 0, 0), (0, 2, 1, 0), (1, 1, 1, 1), (3, 0, 0, 2)]:
        ref = np.sum(wts * np.prod(lam ** np.array(e)[:, None], axis=0))
        assert abs(oracle.monomial_integral(3, e, vol) - ref) < 1e-14


def test_p2_elasticity_matches_independent_hooke():
    rng = np.random.default_rng(11)
    for _ in range(4):
        X = _rand_simplex(rng, 3, 0.03)
        lam, mu = rng.uniform(0.5, 2.0, 2)
        b = rng.standard_normal(3)
        K, F = oracle.p2_elasticity_element(X, lam, mu, b)
        Ki, Fi = indep.elasticity_element(X, lam, mu, b)
        np.testing.assert_allclose(K, Ki, atol=1e-11 * np.abs(Ki).max())
        np.testing.assert_allclose(F, Fi, atol=1e-13)


def test_p2_rigid_modes_rank_symmetry_load():
    rng = np.random.default_rng(12)
    X = _rand_simplex(rng, 3, 0.03)
    K, F = oracle.p2_elasticity_element(X, 1.1, 0.8, (1.0, 2.0, 3.0))
    np.testing.assert_allclose(K, K.T, atol=1e-13 * np.abs(K).max())
    R = indep.rigid_modes(indep.p2_local_nodes(X))
    assert np.abs(K @ R.T).max() < 1e-12 * np.abs(K).max()
    assert np.linalg.matrix_rank(K, tol=1e-9 * np.abs(K).max()) == 24
    vol = indep.simplex_volume(X)
    Fn = F.reshape(10, 3)
    np.testing.assert_allclose(Fn[:4], -vol / 20 * np.array([1.0, 2.0, 3.0])[None, :].repeat(4, 0), atol=1e-15)
    np.testing.assert_allclose(Fn[4:], vol / 5 * np.array([1.0, 2.0, 3.0])[None, :].repeat(6, 0), atol=1e-15)


# ------------------------------------------------------------------ global assembly

def _dense_bruteforce(n, conn, elements):
    A = np.zeros((n, n))
    for g, Ke in zip(conn, elements):
        A[np.ix_(g, g)] += Ke
    return A


@pytest.mark.parametrize("dim,n", [(2, 1), (2, 3), (3, 1), (3, 2)])
def test_assembly_equals_dense_bruteforce(dim, n):
    d = meshgen.poisson_inputs(dim, n, seed=4)
    A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
    locs = [oracle.p1_laplace_element(d["coords"][g], a, f) for g, a, f in zip(d["conn"], d["a"], d["f"])]
    ref = _dense_bruteforce(d["coords"].shape[0], d["conn"], [K for K, _ in locs])
    np.testing.assert_allclose(A.scipy().toarray(), ref, atol=1e-14)
    rhs = np.zeros(d["coords"].shape[0])
    for g, (_, Fe) in zip(d["conn"], locs):
        rhs[g] += Fe
    np.testing.assert_allclose(A.rhs, rhs, atol=1e-16)
    # the pattern is exactly the set of vertex pairs that share an element
    mask = _dense_bruteforce(d["coords"].shape[0], d["conn"], [np.ones((dim + 1, dim + 1))] * len(d["conn"])) > 0
    S = A.scipy()
    S.data[:] = 1
    assert (S.toarray() > 0).tolist() == mask.tolist()


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 6)])
def test_global_laplace_invariants(dim, n):
    d = meshgen.poisson_inputs(dim, n, seed=0)
    A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
    K = A.scipy()
    absrow = abs(K) @ np.ones(A.n)
    assert np.all(np.abs(K @ np.ones(A.n)) <= 64 * np.finfo(float).eps * absrow)
    assert abs(K - K.T).max() == 0.0
    # PSD with a one-dimensional kernel (dense check on a small case)
    w = np.linalg.eigvalsh(K.toarray())
    assert w[0] > -1e-12 * w[-1] and abs(w[0]) < 1e-12 * w[-1] and w[1] > 1e-8 * w[-1]
    # sum F = sum_e f_e |T_e| = int f (partition of unity); |T_e| computed independently
    vols = np.array([indep.simplex_volume(d["coords"][g]) for g in d["conn"]])
    assert abs(A.rhs.sum() - np.dot(d["f"], vols)) < 1e-14
    ones = oracle.assemble_p1(d["coords"], d["conn"], d["a"], np.ones(len(d["conn"])))
    assert abs(ones.rhs.sum() - 1.0) < 1e-13


@pytest.mark.parametrize("dim,n", [(2, 12), (3, 5)])
def test_linear_patch_test(dim, n):
    d = meshgen.poisson_inputs(dim, n, seed=2)
    E = d["conn"].shape[0]
    A = oracle.assemble_p1(d["coords"], d["conn"], np.full(E, 1.7), np.zeros(E))
    u = d["coords"] @ np.arange(1.0, dim + 1.0) + 0.3
    interior = np.setdiff1d(np.arange(A.n), meshgen.boundary_vertices(d["coords"]))
    r = A.scipy() @ u
    assert np.abs(r[interior]).max() < 1e-12
    # the Dirichlet-condensed solve with g = u on the boundary reproduces u
    bnd = meshgen.boundary_vertices(d["coords"])
    ug = np.zeros(A.n)
    ug[bnd] = u[bnd]
    rhs = -(A.scipy() @ ug)
    sol = oracle.condensed_solve(A, bnd, rhs)
    np.testing.assert_allclose(sol[interior], u[interior], atol=1e-12)


def test_mass_global():
    d = meshgen.poisson_inputs(3, 4, seed=1)
    M = oracle.assemble_p1(d["coords"], d["conn"], form="mass").scipy()
    assert abs(M.sum() - 1.0) < 1e-13  # sum of all entries = |Omega|
    assert abs(M - M.T).max() == 0.0


def test_shuffled_numbering_gives_permuted_matrix():
    d = meshgen.poisson_inputs(3, 3, seed=6)
    A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"]).scipy().toarray()
    c2, t2, vperm, eperm, a2, f2 = meshgen.shuffle_numbering(d["coords"], d["conn"], 9, d["a"], d["f"])
    B = oracle.assemble_p1(c2, t2, a2, f2)
    P = np.zeros((len(vperm), len(vperm)))
    P[vperm, np.arange(len(vperm))] = 1
    np.testing.assert_allclose(B.scipy().toarray(), P @ A @ P.T, atol=1e-13)


def test_p2_global_rigid_and_quadratic_patch():
    d = meshgen.elasticity_inputs(2, seed=3)
    E = d["conn"].shape[0]
    lam, mu = 1.3, 0.6
    A = oracle.assemble_p2_elasticity(d["coords"], d["conn"], np.full(E, lam), np.full(E, mu))
    nodes = oracle.p2_node_coords(d["coords"], d["conn"], A.nodes10, A.n_nodes)
    K = A.scipy()
    assert abs(K - K.T).max() <= 1e-15 * abs(K).max()
    R = indep.rigid_modes(nodes)
    assert np.abs(K @ R.T).max() < 1e-12 * abs(K).max()
    # quadratic displacement u_l = 1/2 x^T H_l x + c_l . x: -div sigma = b (constant)
    rng = np.random.default_rng(0)
    H = rng.standard_normal((3, 3, 3))
    H = 0.5 * (H + H.transpose(0, 2, 1))
    C = rng.standard_normal((3, 3))
    U = np.stack([0.5 * np.einsum("ni,ij,nj->n", nodes, H[l], nodes) + nodes @ C[l] for l in range(3)], axis=1)
    b = -np.array([(lam + mu) * sum(H[m][l, m] for m in range(3)) + mu * np.trace(H[l]) for l in range(3)])
    Ab = oracle.assemble_p2_elasticity(d["coords"], d["conn"], np.full(E, lam), np.full(E, mu), np.tile(b, (E, 1)))
    on_bnd = np.any((nodes == 0.0) | (nodes == 1.0), axis=1)
    interior = np.flatnonzero(np.repeat(~on_bnd, 3))
    r = K @ U.ravel() - Ab.rhs
    assert np.abs(r[interior]).max() < 1e-11 * np.abs(Ab.rhs).max()


def test_p2_numbering_counts():
    for n in (1, 2, 3):
        c, t = meshgen.structured_mesh(3, n)
        nodes, nn = oracle.p2_numbering(c.shape[0], t)
        assert nn == (2 * n + 1) ** 3
        assert nodes.max() == nn - 1


def test_condensed_solve_residual():
    d = meshgen.poisson_inputs(3, 6, seed=0)
    A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
    bnd = meshgen.boundary_vertices(d["coords"])
    u = oracle.condensed_solve(A, bnd)
    assert oracle.relres_lin(A, u, bnd) < 1e-12
    assert np.all(u[bnd] == 0.0)


@pytest.mark.parametrize("dim,n", [(2, 9), (3, 5)])
def test_parallel_oracle_bitwise_equals_serial(dim, n):
    """The multi-core CPU baseline (OpenMP Map, per-row sums in ascending element order) gives the serial
    element loop's values and load bit for bit, at any thread count."""
    d = meshgen.poisson_inputs(dim, n, seed=3)
    A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
    inc_ptr, inc = oracle.p1_incidence(len(d["coords"]), d["conn"])
    for threads in (1, 3, 8):
        v, r = oracle.assemble_p1_values_parallel(d["coords"], d["conn"], d["a"], d["f"], A.row_ptr, A.col_idx,
                                                  inc_ptr, inc, threads)
        assert np.array_equal(v, A.vals) and np.array_equal(r, A.rhs)
