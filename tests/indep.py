"""Independent numerical routes used to pin the oracle.

Nothing here shares arithmetic with the oracle: basis functions come from a
monomial Vandermonde system solved on the physical element (no barycentric
coordinates, no reference Jacobian), integrals from a collapsed (Duffy)
tensor Gauss-Legendre rule, and the elasticity form from strains and Hooke's
law written out directly.
"""
from __future__ import annotations

import itertools

import numpy as np


def _gl01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def simplex_quadrature(X, n=6):
    """Points [Q, d] and weights [Q] of a collapsed Gauss rule on the simplex X [d+1, d]."""
    X = np.asarray(X, dtype=np.float64)
    dim = X.shape[1]
    u, wu = _gl01(n)
    pts, wts = [], []
    if dim == 2:
        for (a, wa), (b, wb) in itertools.product(zip(u, wu), zip(u, wu)):
            xi = np.array([a, b * (1 - a)])
            pts.append(xi)
            wts.append(wa * wb * (1 - a))
    else:
        for (a, wa), (b, wb), (c, wc) in itertools.product(zip(u, wu), zip(u, wu), zip(u, wu)):
            xi = np.array([a, b * (1 - a), c * (1 - a) * (1 - b)])
            pts.append(xi)
            wts.append(wa * wb * wc * (1 - a) ** 2 * (1 - b))
    pts, wts = np.array(pts), np.array(wts)
    A = (X[1:] - X[0]).T  # reference -> physical
    phys = X[0] + pts @ A.T
    return phys, wts * abs(np.linalg.det(A))


def _monomials(dim, degree):
    exps = [e for e in itertools.product(range(degree + 1), repeat=dim) if sum(e) <= degree]
    exps.sort(key=lambda e: (sum(e), [-v for v in e]))
    return exps


def lagrange_basis(nodes, degree):
    """Callables (values, gradients) of the Lagrange basis on `nodes` [k, d], from a Vandermonde solve."""
    nodes = np.asarray(nodes, dtype=np.float64)
    dim = nodes.shape[1]
    exps = _monomials(dim, degree)
    assert len(exps) == nodes.shape[0]

    def mono(x):
        return np.array([np.prod([x[i] ** e[i] for i in range(dim)]) for e in exps])

    def dmono(x):
        out = np.zeros((len(exps), dim))
        for j, e in enumerate(exps):
            for i in range(dim):
                if e[i] == 0:
                    continue
                ee = list(e)
                ee[i] -= 1
                out[j, i] = e[i] * np.prod([x[t] ** ee[t] for t in range(dim)])
        return out

    V = np.array([mono(p) for p in nodes])
    C = np.linalg.solve(V, np.eye(len(exps)))  # column i = coefficients of phi_i

    def values(x):
        return mono(x) @ C

    def grads(x):
        return (dmono(x).T @ C).T  # [k, d]

    return values, grads


def p2_local_nodes(X):
    X = np.asarray(X, dtype=np.float64)
    edges = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
    return np.vstack([X] + [0.5 * (X[p] + X[q]) for p, q in edges])


def laplace_element(X, a=1.0, f=1.0, n=5):
    X = np.asarray(X, dtype=np.float64)
    val, grad = lagrange_basis(X, 1)
    pts, wts = simplex_quadrature(X, n)
    k = X.shape[0]
    K, F = np.zeros((k, k)), np.zeros(k)
    for x, w in zip(pts, wts):
        G = grad(x)
        K += w * a * G @ G.T
        F += w * f * val(x)
    return K, F


def mass_element(X, n=5):
    X = np.asarray(X, dtype=np.float64)
    val, _ = lagrange_basis(X, 1)
    pts, wts = simplex_quadrature(X, n)
    k = X.shape[0]
    M = np.zeros((k, k))
    for x, w in zip(pts, wts):
        v = val(x)
        M += w * np.outer(v, v)
    return M


def elasticity_element(X, lam, mu, b=(0.0, 0.0, 0.0), n=5):
    """P2 tetrahedron: a(u, v) = int sigma(u) : eps(v), sigma = lam tr(eps) I + 2 mu eps."""
    nodes = p2_local_nodes(X)
    val, grad = lagrange_basis(nodes, 2)
    pts, wts = simplex_quadrature(X, n)
    K, F = np.zeros((30, 30)), np.zeros(30)
    b = np.asarray(b, dtype=np.float64)
    I3 = np.eye(3)
    for x, w in zip(pts, wts):
        G = grad(x)
        phi = val(x)
        # eps of the vector basis function phi_a e_c: grad u = e_c grad(phi_a)^T
        eps = np.zeros((30, 3, 3))
        for a in range(10):
            for c in range(3):
                gu = np.outer(I3[c], G[a])
                eps[3 * a + c] = 0.5 * (gu + gu.T)
        sig = lam * np.trace(eps, axis1=1, axis2=2)[:, None, None] * I3 + 2 * mu * eps
        # row = test (v), column = trial (u): K[r, s] = sigma(u_s) : eps(v_r)
        K += w * np.einsum("sij,rij->rs", sig, eps)
        for a in range(10):
            for c in range(3):
                F[3 * a + c] += w * b[c] * phi[a]
    return K, F


def cot_laplace_triangle(X):
    """K_ab = -1/2 cot(theta_c), theta_c the angle at the third vertex (cotangent formula)."""
    X = np.asarray(X, dtype=np.float64)
    K = np.zeros((3, 3))
    for a, b in ((0, 1), (0, 2), (1, 2)):
        c = 3 - a - b
        u, v = X[a] - X[c], X[b] - X[c]
        cot = np.dot(u, v) / abs(u[0] * v[1] - u[1] * v[0])
        K[a, b] = K[b, a] = -0.5 * cot
    for a in range(3):
        K[a, a] = -K[a].sum()
    return K


def cot_laplace_tet(X):
    """K_ab = -(1/6) l_cd cot(theta_cd), {c,d} the opposite edge, theta_cd its dihedral angle."""
    X = np.asarray(X, dtype=np.float64)
    K = np.zeros((4, 4))
    for a, b in itertools.combinations(range(4), 2):
        c, d = [i for i in range(4) if i not in (a, b)]
        t = X[d] - X[c]
        ell = np.linalg.norm(t)
        t = t / ell
        ua = X[a] - X[c] - np.dot(X[a] - X[c], t) * t
        ub = X[b] - X[c] - np.dot(X[b] - X[c], t) * t
        cot = np.dot(ua, ub) / np.linalg.norm(np.cross(ua, ub))
        K[a, b] = K[b, a] = -ell * cot / 6.0
    for a in range(4):
        K[a, a] = -K[a].sum()
    return K


def simplex_volume(X):
    X = np.asarray(X, dtype=np.float64)
    d = X.shape[1]
    return abs(np.linalg.det((X[1:] - X[0]).T)) / (2.0 if d == 2 else 6.0)


def rigid_modes(nodes):
    """6 rigid-body displacement fields of 3D points [k, 3], flattened with DoF 3*node + c."""
    nodes = np.asarray(nodes, dtype=np.float64)
    k = nodes.shape[0]
    modes = []
    for c in range(3):
        u = np.zeros((k, 3))
        u[:, c] = 1.0
        modes.append(u.ravel())
    for axis in np.eye(3):
        modes.append(np.cross(axis, nodes).ravel())
    return np.array(modes)
