"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module builds meshes and draws coefficients; it holds none of the
assembly arithmetic.  Both sides of every parity test read the arrays it
returns, so neither side generates its own inputs.

Meshes are structured grids of the unit square / unit cube whose cells are
split into simplices, with interior vertices jittered so the result is an
unstructured simplicial mesh with the shapes of the paper's analytic
benchmarks (Poisson on the unit cube, Section B.1.1; the 2D elliptic example
of Section A.2).

Conventions (fixed so that pattern sizes are reproducible):
  * vertex id is x-fastest: v = i + (n+1)*(j + (n+1)*k);
  * 2D: every cell is cut along the diagonal v00-v11 into the triangles
    (v00, v10, v11) and (v00, v11, v01); element id = 2*cell + s;
  * 3D: Kuhn/Freudenthal split, 6 tetrahedra per cube
    {v000, v000+e_p1, v000+e_p1+e_p2, v111} for the axis permutations p in
    lexicographic order; element id = 6*cell + s;  every cube is split the
    same way, so the mesh is conforming;
  * jitter: each coordinate of each interior vertex moves by U(-delta*h,
    delta*h); vertices with any coordinate equal to 0 or 1 stay put, so the
    domain is exactly the unit square / cube;
  * random draws use numpy's PCG64 (default_rng(seed)) in a fixed order:
    jitter (n_interior, dim), then the coefficient arrays in the order each
    generator documents.
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = [
    "structured_mesh",
    "poisson_inputs",
    "elasticity_inputs",
    "heat_inputs",
    "boundary_vertices",
    "shuffle_numbering",
]

# the six axis permutations of the Kuhn split, lexicographic order
_KUHN_PERMS = list(itertools.permutations(range(3)))


def _grid_vertices(dim: int, n: int) -> np.ndarray:
    t = np.linspace(0.0, 1.0, n + 1)
    if dim == 2:
        yy, xx = np.meshgrid(t, t, indexing="ij")
        return np.stack([xx.ravel(), yy.ravel()], axis=1)
    zz, yy, xx = np.meshgrid(t, t, t, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)


def _connectivity(dim: int, n: int) -> np.ndarray:
    m = n + 1
    if dim == 2:
        j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        v00 = (i + m * j).ravel()
        v10, v01 = v00 + 1, v00 + m
        v11 = v01 + 1
        tri = np.empty((n * n, 2, 3), dtype=np.int64)
        tri[:, 0] = np.stack([v00, v10, v11], axis=1)
        tri[:, 1] = np.stack([v00, v11, v01], axis=1)
        return tri.reshape(-1, 3).astype(np.int32)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    v000 = (i + m * (j + m * k)).ravel()
    step = (1, m, m * m)  # vertex-id increment along x, y, z
    tets = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for s, p in enumerate(_KUHN_PERMS):
        a = v000
        b = a + step[p[0]]
        c = b + step[p[1]]
        d = c + step[p[2]]
        tets[:, s] = np.stack([a, b, c, d], axis=1)
    return tets.reshape(-1, 4).astype(np.int32)


def _on_boundary(coords: np.ndarray) -> np.ndarray:
    return np.any((coords == 0.0) | (coords == 1.0), axis=1)


def structured_mesh(dim: int, n: int, jitter: float | None = None,
                    rng: np.random.Generator | None = None):
    """Jittered structured simplicial mesh of the unit square (dim=2) or cube (dim=3).

    Returns (coords [Nv, dim] float64 C-order, conn [E, dim+1] int32).
    `jitter` is the fraction delta of the grid spacing h (defaults 0.2 in 2D,
    0.15 in 3D); draws come from `rng` (no jitter if rng is None).
    """
    if dim not in (2, 3) or n < 1:
        raise ValueError("dim must be 2 or 3 and n >= 1")
    if jitter is None:
        jitter = 0.2 if dim == 2 else 0.15
    coords = _grid_vertices(dim, n)
    conn = _connectivity(dim, n)
    if rng is not None and jitter > 0.0:
        h = 1.0 / n
        interior = ~_on_boundary(coords)
        d = rng.uniform(-jitter * h, jitter * h, size=(int(interior.sum()), dim))
        coords[interior] += d
    return np.ascontiguousarray(coords), np.ascontiguousarray(conn)


def poisson_inputs(dim: int, n: int, seed: int = 0, jitter: float | None = None):
    """Poisson workload: mesh, a = exp(N(0,1)) and f = U(-1,1) per element.

    Draw order: jitter, a, f.  Returns dict(coords, conn, a, f).
    """
    rng = np.random.default_rng(seed)
    coords, conn = structured_mesh(dim, n, jitter, rng)
    E = conn.shape[0]
    a = np.exp(rng.standard_normal(E))
    f = rng.uniform(-1.0, 1.0, size=E)
    return {"coords": coords, "conn": conn, "a": a, "f": f}


def elasticity_inputs(n: int, seed: int = 0, jitter: float | None = None):
    """3D linear-elasticity workload: lambda, mu ~ U(0.5, 2), b ~ N(0,1)^3 per element.

    Draw order: jitter, lambda (E), mu (E), b (E, 3).  Returns
    dict(coords, conn, lam, mu, b).
    """
    rng = np.random.default_rng(seed)
    coords, conn = structured_mesh(3, n, jitter, rng)
    E = conn.shape[0]
    lam = rng.uniform(0.5, 2.0, size=E)
    mu = rng.uniform(0.5, 2.0, size=E)
    b = rng.standard_normal((E, 3))
    return {"coords": coords, "conn": conn, "lam": lam, "mu": mu, "b": b}


def heat_inputs(n: int, seed: int = 0, jitter: float | None = None):
    """2D heat workload: mesh and log a ~ N(0,1) per element.  Draw order: jitter, log a."""
    rng = np.random.default_rng(seed)
    coords, conn = structured_mesh(2, n, jitter, rng)
    log_a = rng.standard_normal(conn.shape[0])
    return {"coords": coords, "conn": conn, "log_a": log_a}


def boundary_vertices(coords: np.ndarray) -> np.ndarray:
    """Vertices on the boundary of the unit square / cube (a coordinate equal to 0 or 1)."""
    return np.flatnonzero(_on_boundary(coords)).astype(np.int32)


def shuffle_numbering(coords: np.ndarray, conn: np.ndarray, seed: int,
                      *elem_arrays: np.ndarray):
    """Randomly renumber vertices and elements and rotate each element's vertex list.

    Returns (coords', conn', vperm, eperm, *elem_arrays') where vertex v of the
    input is vertex vperm[v] of the output and output element i is input element
    eperm[i].  Rotating the local vertex list keeps the element's orientation
    class irrelevant: assembly uses |det J|.
    """
    rng = np.random.default_rng(seed)
    nv, ne = coords.shape[0], conn.shape[0]
    vperm = rng.permutation(nv)
    eperm = rng.permutation(ne)
    new_coords = np.empty_like(coords)
    new_coords[vperm] = coords
    new_conn = vperm[conn[eperm]].astype(np.int32)
    shift = rng.integers(0, conn.shape[1], size=ne)
    rows = np.arange(ne)[:, None]
    cols = (np.arange(conn.shape[1])[None, :] + shift[:, None]) % conn.shape[1]
    new_conn = np.ascontiguousarray(new_conn[rows, cols])
    out = [np.ascontiguousarray(a[eperm]) for a in elem_arrays]
    return (np.ascontiguousarray(new_coords), new_conn, vperm, eperm, *out)
