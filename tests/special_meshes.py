"""Synthetic meshes whose row blocks go past the assembly kernels' thread counts (test inputs only).

- sphere_star: one vertex joined to every face of the convex hull of random points on the unit sphere;
  with 255 points the centre's row holds 506 (element, node) pairs, 256 CSR entries and 256 distinct
  vertices: the most a P1 block stages, beyond the 256 threads of the P1 kernel for pairs, entries and
  routing units.
- disjoint_simplices: elements with vertices of their own (every vertex in one element), interleaved so
  that element e owns vertices e, e + E, ..., e + d E: consecutive vertex rows belong to different
  elements, so a row block gathers many rows (P1: 256 rows of one pair each) and, in P2, many staged
  vertices and node entries.
- private_star: m tets that share one vertex and nothing else: the shared vertex's row (m pairs, one
  block of its own) stages 1 + 3 m distinct vertices and, in P2, holds 1 + 9 m node entries.
- polar_disk: a 2D disk of `rings` rings of m vertices around a centre of valence m: one long CSR row
  (m + 1 entries) among rows of about 7, so the CG iterations' sliced-ELL slices keep lengths of their
  own (padding every slice to the longest would cost far more than 1/32).
"""
import numpy as np


def _coefficients(m, rng):
    return {"a": np.exp(rng.standard_normal(m)), "f": rng.uniform(-1, 1, m),
            "lam": rng.uniform(0.5, 2.0, m), "mu": rng.uniform(0.5, 2.0, m), "b": rng.standard_normal((m, 3))}


def sphere_star(n_pts: int, seed: int):
    from scipy.spatial import ConvexHull

    rng = np.random.default_rng(seed)
    p = rng.standard_normal((n_pts, 3))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    hull = ConvexHull(p)
    coords = np.ascontiguousarray(np.concatenate([np.zeros((1, 3)), p]))
    conn = np.concatenate([np.zeros((len(hull.simplices), 1), np.int64), hull.simplices + 1], axis=1)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    return {"coords": coords, "conn": conn, **_coefficients(len(conn), rng)}


def disjoint_simplices(dim: int, E: int, seed: int):
    rng = np.random.default_rng(seed)
    ref = np.vstack([np.zeros(dim), np.eye(dim)])  # the reference simplex
    coords = np.zeros(((dim + 1) * E, dim))
    conn = np.zeros((E, dim + 1), dtype=np.int32)
    for e in range(E):
        x = ref + rng.uniform(-0.15, 0.15, ref.shape)
        x[:, 0] += 3.0 * e
        for a in range(dim + 1):
            conn[e, a] = e + a * E
            coords[e + a * E] = x[a]
    return {"coords": coords, "conn": conn, **_coefficients(E, rng)}


def block_shapes(pat):
    """Per row block of a pattern: (rows, pairs, node entries, staged vertices)."""
    r = pat.routing()
    br, ip, rp = r["blk_row"], r["inc_ptr"], r["node_rp"]
    vptr, _, _ = pat.block_vertices()
    return np.diff(br), ip[br[1:]] - ip[br[:-1]], rp[br[1:]] - rp[br[:-1]], np.diff(vptr)


def private_star(m: int, seed: int):
    rng = np.random.default_rng(seed)
    coords = np.zeros((1 + 3 * m, 3))
    conn = np.zeros((m, 4), dtype=np.int32)
    for t in range(m):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        u = np.cross(d, rng.standard_normal(3))
        u /= np.linalg.norm(u)
        w = np.cross(d, u)
        coords[1 + 3 * t:4 + 3 * t] = [2.0 * d, 2.0 * d + 0.5 * u, 2.0 * d + 0.5 * w]
        conn[t] = [0, 1 + 3 * t, 2 + 3 * t, 3 + 3 * t]
    return {"coords": coords, "conn": conn, **_coefficients(m, rng)}


def polar_disk(m: int, rings: int, seed: int):
    rng = np.random.default_rng(seed)
    pts = [np.zeros(2)]
    for k in range(1, rings + 1):
        ang = 2 * np.pi * (np.arange(m) + 0.5 * (k % 2)) / m
        pts.append(np.stack([np.cos(ang), np.sin(ang)], 1) * (k / rings))
    coords = np.ascontiguousarray(np.vstack(pts))
    ring = lambda k, j: 1 + (k - 1) * m + (j % m)  # noqa: E731
    tri = [[0, ring(1, j), ring(1, j + 1)] for j in range(m)]
    for k in range(1, rings):
        for j in range(m):
            tri.append([ring(k, j), ring(k + 1, j), ring(k + 1, j + 1)])
            tri.append([ring(k, j), ring(k + 1, j + 1), ring(k, j + 1)])
    conn = np.ascontiguousarray(np.array(tri, dtype=np.int32))
    return {"coords": coords, "conn": conn, **_coefficients(len(conn), rng)}
