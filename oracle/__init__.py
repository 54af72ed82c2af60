"""FP64 CPU oracle for batched Galerkin assembly (TensorGalerkin, arXiv 2602.05052).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The library never imports it, and it
imports nothing from the library.  It shares with the HIP path only the seeded
inputs from `meshgen`.

The element arithmetic lives in `tg_oracle.c` (plain C, FP64, closed-form
simplex integrals, serial scatter-add in ascending element order, Sec. 2
eq. scatter_add).  This module compiles it with gcc, calls it through ctypes,
and adds the pieces that are library primitives on top: Dirichlet
condensation (Sec. B.1.2, the condensed system) solved with scipy's sparse
direct solver, and the two verification metrics of Sec. B.1.3 (eq. relerr and
eq. linres).

Parity unpinned: nothing (every function has a pin in tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile tg_oracle.c into liboracle.so (gcc -O3, OpenMP for the multi-core baseline, no fast-math)."""
    with _lock:
        if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            tmp = _LIB + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC,
                                   "-lm"])
            os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.oracle_monomial.restype = ctypes.c_double
        lib.oracle_monomial.argtypes = [ctypes.c_int, _i32p, ctypes.c_double]
        lib.oracle_simplex_geometry.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        lib.oracle_p1_laplace_element.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _dp, _dp]
        lib.oracle_p1_mass_element.argtypes = [ctypes.c_int, _dp, _dp]
        lib.oracle_p2_elasticity_element.argtypes = [_dp, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
        lib.oracle_p2_numbering.argtypes = [ctypes.c_int64, ctypes.c_int64, _i32p, _i64p, _i64p]
        lib.oracle_csr_pattern.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, _i64p, _i64p,
                                           ctypes.POINTER(_i64p), _i64p]
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_assemble_p1.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _dp, ctypes.c_int64, _i32p,
                                           _dp, _dp, _i64p, _i64p, _dp, _dp, _i64p]
        lib.oracle_assemble_p1_parallel.argtypes = [ctypes.c_int, ctypes.c_int64, _dp, ctypes.c_int64, _i32p, _dp,
                                                    _dp, _i64p, _i64p, _i64p, _i64p, _dp, _dp, _dp, _dp, ctypes.c_int,
                                                    _i64p]
        lib.oracle_assemble_p2_elasticity.argtypes = [ctypes.c_int64, _dp, ctypes.c_int64, _i32p, _i64p, _dp, _dp,
                                                      _dp, _i64p, _i64p, _dp, _dp, _i64p]
        lib.oracle_p1_adjoint_element.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp, _dp, _dp, ctypes.c_int,
                                                  _dp, _dp]
        lib.oracle_p1_adjoint.argtypes = [ctypes.c_int, ctypes.c_int64, _dp, ctypes.c_int64, _i32p, ctypes.c_int,
                                          _dp, _dp, _dp, _dp, _dp, _dp, _i64p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None, typ):
    if a is None:
        return ctypes.cast(None, typ)
    return a.ctypes.data_as(typ)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc: int, what: str, bad: int | None = None):
    if rc == -2:
        raise OracleError(f"{what}: degenerate element" + (f" {bad}" if bad is not None else ""))
    if rc != 0:
        raise OracleError(f"{what}: error {rc}")


# ---------------------------------------------------------------- elements

def monomial_integral(dim: int, exps, vol: float) -> float:
    """int_T prod lambda_i^{e_i} = d! prod e_i! / (d + sum e_i)! |T| (barycentric monomial rule)."""
    e = np.zeros(4, dtype=np.int32)
    e[: dim + 1] = exps
    return _load().oracle_monomial(dim, _ptr(e, _i32p), float(vol))


def simplex_geometry(X):
    """Barycentric gradients [d+1, d] and volume of the affine simplex X [d+1, d] (Sec. 2 Alg. 1, Geometry)."""
    X = _f64(X)
    dim = X.shape[1]
    g = np.zeros((dim + 1, dim))
    vol = ctypes.c_double()
    _check(_load().oracle_simplex_geometry(dim, _ptr(X, _dp), _ptr(g, _dp), ctypes.byref(vol)), "geometry")
    return g, vol.value


def p1_laplace_element(X, a: float = 1.0, f: float = 1.0):
    """(K_e, F_e) of -div(a grad u) = f on one P1 simplex (SM A.2, eq. matlclquad, exact integrals)."""
    X = _f64(X)
    dim = X.shape[1]
    K = np.zeros((dim + 1, dim + 1))
    F = np.zeros(dim + 1)
    _check(_load().oracle_p1_laplace_element(dim, _ptr(X, _dp), a, f, _ptr(K, _dp), _ptr(F, _dp)), "p1 element")
    return K, F


def p1_mass_element(X):
    """M_e with (M_e)_ab = int_T lambda_a lambda_b (SM A.1 mass inner product)."""
    X = _f64(X)
    dim = X.shape[1]
    M = np.zeros((dim + 1, dim + 1))
    _check(_load().oracle_p1_mass_element(dim, _ptr(X, _dp), _ptr(M, _dp)), "mass element")
    return M


def p2_elasticity_element(X, lam: float, mu: float, b=(0.0, 0.0, 0.0)):
    """(K_e [30,30], F_e [30]) of P2 linear elasticity on one tetrahedron (Sec. B.1.1 Hooke's law).

    Local DoF 3*node + component; local nodes are the 4 vertices then the
    edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3).
    """
    X = _f64(X)
    b = _f64(b)
    K = np.zeros((30, 30))
    F = np.zeros(30)
    _check(_load().oracle_p2_elasticity_element(_ptr(X, _dp), lam, mu, _ptr(b, _dp), _ptr(K, _dp), _ptr(F, _dp)),
           "p2 element")
    return K, F


# ---------------------------------------------------------------- numbering / pattern

P2_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def p2_numbering(nv: int, conn):
    """Global P2 nodes per element [E, 10] and the node count (vertices, then edges by (min, max))."""
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    E = conn.shape[0]
    nodes = np.zeros((E, 10), dtype=np.int64)
    nn = ctypes.c_int64()
    _check(_load().oracle_p2_numbering(nv, E, _ptr(conn, _i32p), _ptr(nodes, _i64p), ctypes.byref(nn)), "p2 numbering")
    return nodes, nn.value


def p2_node_coords(coords, conn, nodes10, n_nodes):
    """Coordinates of the P2 nodes: vertices, then edge midpoints (straight edges)."""
    coords = _f64(coords)
    out = np.zeros((n_nodes, 3))
    out[: coords.shape[0]] = coords
    for m, (p, q) in enumerate(P2_EDGES):
        out[nodes10[:, 4 + m]] = 0.5 * (coords[conn[:, p]] + coords[conn[:, q]])
    return out


def csr_pattern(ndof: int, dofs):
    """(row_ptr, col_idx) int64 of the matrix coupling the DoFs of each row of dofs [E, kd]."""
    dofs = np.ascontiguousarray(dofs, dtype=np.int64)
    E, kd = dofs.shape
    row_ptr = np.zeros(ndof + 1, dtype=np.int64)
    cols = _i64p()
    nnz = ctypes.c_int64()
    lib = _load()
    _check(lib.oracle_csr_pattern(ndof, E, kd, _ptr(dofs, _i64p), _ptr(row_ptr, _i64p), ctypes.byref(cols),
                                  ctypes.byref(nnz)), "csr pattern")
    col_idx = np.ctypeslib.as_array(cols, shape=(nnz.value,)).copy() if nnz.value else np.zeros(0, np.int64)
    lib.oracle_free(cols)
    return row_ptr, col_idx


# ---------------------------------------------------------------- global assembly

class Assembled:
    """A CSR matrix (int64 indices, FP64 values) and its right-hand side."""

    def __init__(self, row_ptr, col_idx, vals, rhs):
        self.row_ptr, self.col_idx, self.vals, self.rhs = row_ptr, col_idx, vals, rhs

    @property
    def n(self):
        return self.row_ptr.shape[0] - 1

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.col_idx, self.row_ptr), shape=(self.n, self.n))


def assemble_p1(coords, conn, a=None, f=None, form: str = "laplace") -> Assembled:
    """Scatter-add assembly of P1 Laplace (K, F) or mass (M) on a triangle/tet mesh."""
    coords = _f64(coords)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    nv, dim = coords.shape
    E = conn.shape[0]
    row_ptr, col_idx = csr_pattern(nv, conn)
    vals = np.zeros(col_idx.shape[0])
    fm = 0 if form == "laplace" else 1
    rhs = np.zeros(nv)
    coef = _f64(a) if (fm == 0) else None
    load = _f64(f) if (fm == 0 and f is not None) else None
    bad = ctypes.c_int64(-1)
    rc = _load().oracle_assemble_p1(dim, fm, nv, _ptr(coords, _dp), E, _ptr(conn, _i32p), _ptr(coef, _dp),
                                    _ptr(load, _dp), _ptr(row_ptr, _i64p), _ptr(col_idx, _i64p), _ptr(vals, _dp),
                                    _ptr(rhs, _dp), ctypes.byref(bad))
    _check(rc, "assemble_p1", bad.value)
    return Assembled(row_ptr, col_idx, vals, rhs)


def assemble_p1_values(coords, conn, a, f, row_ptr, col_idx):
    """Value and load assembly only (Laplace), on a CSR pattern built beforehand by csr_pattern."""
    coords = _f64(coords)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    nv, dim = coords.shape
    vals = np.zeros(col_idx.shape[0])
    rhs = np.zeros(nv)
    bad = ctypes.c_int64(-1)
    rc = _load().oracle_assemble_p1(dim, 0, nv, _ptr(coords, _dp), conn.shape[0], _ptr(conn, _i32p),
                                    _ptr(_f64(a), _dp), _ptr(_f64(f), _dp), _ptr(row_ptr, _i64p),
                                    _ptr(col_idx, _i64p), _ptr(vals, _dp), _ptr(rhs, _dp), ctypes.byref(bad))
    _check(rc, "assemble_p1_values", bad.value)
    return vals, rhs


def p1_incidence(nv: int, conn):
    """(inc_ptr [nv+1], inc): every vertex's (element e, local node a) pairs as codes e*k + a, in ascending e."""
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    E, k = conn.shape
    codes = np.arange(E * k, dtype=np.int64)
    order = np.argsort(conn.reshape(-1), kind="stable")  # stable: ascending code (so e) within a vertex
    inc_ptr = np.zeros(nv + 1, dtype=np.int64)
    np.cumsum(np.bincount(conn.reshape(-1), minlength=nv), out=inc_ptr[1:])
    return inc_ptr, codes[order]


def assemble_p1_values_parallel(coords, conn, a, f, row_ptr, col_idx, inc_ptr, inc, threads: int = 0):
    """assemble_p1_values on several threads (OpenMP Map over elements, then per-row sums in ascending element
    order): bitwise the same values and load as the serial element loop."""
    coords = _f64(coords)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    nv, dim = coords.shape
    E, k = conn.shape
    vals = np.empty(col_idx.shape[0])
    rhs = np.empty(nv)
    ke, fe = np.empty(E * k * k), np.empty(E * k)
    bad = ctypes.c_int64(-1)
    rc = _load().oracle_assemble_p1_parallel(dim, nv, _ptr(coords, _dp), E, _ptr(conn, _i32p), _ptr(_f64(a), _dp),
                                             _ptr(_f64(f), _dp), _ptr(row_ptr, _i64p), _ptr(col_idx, _i64p),
                                             _ptr(inc_ptr, _i64p), _ptr(inc, _i64p), _ptr(ke, _dp), _ptr(fe, _dp),
                                             _ptr(vals, _dp), _ptr(rhs, _dp), int(threads), ctypes.byref(bad))
    _check(rc, "assemble_p1_values_parallel", bad.value)
    return vals, rhs


def assemble_p2_elasticity(coords, conn, lam, mu, b=None) -> Assembled:
    """Scatter-add assembly of P2 linear elasticity (3 DoFs per node, DoF = 3*node + c)."""
    coords = _f64(coords)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    nv = coords.shape[0]
    E = conn.shape[0]
    nodes10, n_nodes = p2_numbering(nv, conn)
    dofs = (3 * nodes10[:, :, None] + np.arange(3)[None, None, :]).reshape(E, 30)
    ndof = 3 * n_nodes
    row_ptr, col_idx = csr_pattern(ndof, dofs)
    vals = np.zeros(col_idx.shape[0])
    rhs = np.zeros(ndof)
    bad = ctypes.c_int64(-1)
    bb = _f64(b) if b is not None else None
    rc = _load().oracle_assemble_p2_elasticity(nv, _ptr(coords, _dp), E, _ptr(conn, _i32p), _ptr(nodes10, _i64p),
                                               _ptr(_f64(lam), _dp), _ptr(_f64(mu), _dp), _ptr(bb, _dp),
                                               _ptr(row_ptr, _i64p), _ptr(col_idx, _i64p), _ptr(vals, _dp),
                                               _ptr(rhs, _dp), ctypes.byref(bad))
    _check(rc, "assemble_p2_elasticity", bad.value)
    out = Assembled(row_ptr, col_idx, vals, rhs)
    out.nodes10, out.n_nodes = nodes10, n_nodes
    return out


# ---------------------------------------------------------------- adjoint

def p1_adjoint_element(X, c, lam, u, w=None, mass=False):
    """(dPhi/dlog c, dPhi/dx [d+1, d]) of Phi = lam^T (A u - M w) on one P1 simplex (A = K(c) [+ M])."""
    X = _f64(X)
    dim = X.shape[1]
    dlogc = ctypes.c_double()
    dx = np.zeros((dim + 1, dim))
    ww = _f64(w) if w is not None else None
    _check(_load().oracle_p1_adjoint_element(dim, _ptr(X, _dp), float(c), _ptr(_f64(lam), _dp), _ptr(_f64(u), _dp),
                                             _ptr(ww, _dp), int(mass), ctypes.byref(dlogc), _ptr(dx, _dp)), "adjoint")
    return dlogc.value, dx


def p1_adjoint(coords, conn, c, lam, u, w=None, mass=False):
    """Global (dPhi/dlog c [E], dPhi/dcoords [nv, d]) of Phi = lam^T (A(c) u - M w), elements in order."""
    coords = _f64(coords)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    nv, dim = coords.shape
    E = conn.shape[0]
    dlogc = np.zeros(E)
    dcoords = np.zeros((nv, dim))
    bad = ctypes.c_int64(-1)
    ww = _f64(w) if w is not None else None
    rc = _load().oracle_p1_adjoint(dim, nv, _ptr(coords, _dp), E, _ptr(conn, _i32p), int(mass), _ptr(_f64(c), _dp),
                                   _ptr(_f64(lam), _dp), _ptr(_f64(u), _dp), _ptr(ww, _dp), _ptr(dlogc, _dp),
                                   _ptr(dcoords, _dp), ctypes.byref(bad))
    _check(rc, "p1_adjoint", bad.value)
    return dlogc, dcoords


# ---------------------------------------------------------------- implicit-Euler heat rollout and its adjoint

def heat_matrices(coords, conn, log_a, dt):
    """(A, M) as scipy CSR: M the P1 mass matrix (Sec. A.1, mass inner product), A = M + dt K(exp(log_a))."""
    a = np.exp(_f64(log_a))
    K = assemble_p1(coords, conn, dt * a, np.zeros_like(a), form="laplace").scipy()
    M = assemble_p1(coords, conn, form="mass").scipy()
    return (M + K).tocsr(), M


class _InteriorSolver:
    """Direct solves with the free-DoF block A[mask][:, mask] (one sparse LU factorisation)."""

    def __init__(self, A, mask):
        import scipy.sparse.linalg as spla
        self.mask = mask
        self.n = A.shape[0]
        self.lu = spla.splu(A[mask][:, mask].tocsc()) if mask.any() else None

    def __call__(self, b):
        x = np.zeros(self.n)
        if self.lu is not None:
            x[self.mask] = self.lu.solve(np.ascontiguousarray(b[self.mask]))
        return x


def heat_rollout(coords, conn, log_a, u0, dt, nsteps, constrained):
    """States U [nsteps+1, nv] of implicit Euler for M U' + K U = 0 (Sec. A.1, method of lines)
    with U = 0 on the constrained vertices:  A u^{n+1} = M u^n on the free rows, A = M + dt K."""
    A, M = heat_matrices(coords, conn, log_a, dt)
    mask = np.ones(A.shape[0], dtype=bool)
    mask[np.asarray(constrained, dtype=np.int64)] = False
    U = np.zeros((nsteps + 1, A.shape[0]))
    U[0] = _f64(u0)
    solve = _InteriorSolver(A, mask)
    for n in range(nsteps):
        U[n + 1] = solve(M @ U[n])
    return U


def heat_adjoint(coords, conn, log_a, U, dt, g, constrained):
    """Discrete adjoint (Sec. 2, eq. adj) of the rollout for a loss with dL/du^N = g.

    lam^N solves A lam^N = g and lam^n solves A lam^n = M lam^{n+1} on the free rows (A symmetric).
    With Phi_n = lam^n^T (A u^n - M u^{n-1}), every parameter gradient is -sum_n dPhi_n; the
    element terms come from p1_adjoint.  Returns (dL/dlog_a [E], dL/dcoords [nv, d], dL/du0 [nv]).
    """
    N = U.shape[0] - 1
    if N == 0:  # u^N = u^0
        return np.zeros(conn.shape[0]), np.zeros_like(_f64(coords)), _f64(g).copy()
    A, M = heat_matrices(coords, conn, log_a, dt)
    mask = np.ones(A.shape[0], dtype=bool)
    mask[np.asarray(constrained, dtype=np.int64)] = False
    c = dt * np.exp(_f64(log_a))
    solve = _InteriorSolver(A, mask)
    lam = solve(_f64(g))
    dloga = np.zeros(conn.shape[0])
    dcoords = np.zeros_like(_f64(coords))
    for n in range(N, 0, -1):
        dl, dx = p1_adjoint(coords, conn, c, lam, U[n], U[n - 1], mass=True)
        dloga -= dl
        dcoords -= dx
        if n > 1:
            lam = solve(M @ lam)
    du0 = M @ lam
    return dloga, dcoords, du0


# ---------------------------------------------------------------- condensed solve and metrics

def condensed_solve(A: Assembled, constrained_dofs, rhs=None):
    """Solve the condensed system (Dirichlet rows/columns removed, u = 0 on them; Sec. B.1.2).

    Returns the full-length solution with zeros at constrained DoFs, using
    scipy's sparse direct solver on the interior block.
    """
    import scipy.sparse.linalg as spla
    n = A.n
    mask = np.ones(n, dtype=bool)
    mask[np.asarray(constrained_dofs, dtype=np.int64)] = False
    K = A.scipy()
    b = A.rhs if rhs is None else rhs
    Kii = K[mask][:, mask].tocsc()
    u = np.zeros(n)
    if Kii.shape[0]:
        u[mask] = spla.spsolve(Kii, b[mask])
    return u


def relres_lin(A: Assembled, u, constrained_dofs, rhs=None) -> float:
    """||K u - f|| / ||f|| on the condensed system (Sec. B.1.3, eq. linres)."""
    n = A.n
    mask = np.ones(n, dtype=bool)
    mask[np.asarray(constrained_dofs, dtype=np.int64)] = False
    b = A.rhs if rhs is None else rhs
    r = (A.scipy() @ np.where(mask, u, 0.0) - b)[mask]
    nb = np.linalg.norm(b[mask])
    return float(np.linalg.norm(r) / nb) if nb > 0 else float(np.linalg.norm(r))


def relerr(u, u_ref) -> float:
    """||u - u_ref|| / ||u_ref|| (Sec. B.1.3, eq. relerr)."""
    return float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))
