"""GPU parity of the fused Map+Reduce kernels against the FP64 oracle (through the C ABI).

Bar (normwise, max absolute row sum): ||K - K*||_inf / ||K*||_inf and
||F - F*||_inf / ||F*||_inf <= 1e-12 in FP64 and <= 1e-5 in FP32; the CSR
pattern must be identical.  Sizes span one element up to the full 64^3 tet mesh
(several row blocks and a ragged last block in every case).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
import oracle
import special_meshes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
tg = pytest.importorskip("paper_2602_05052_amd")

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def _norm_rel(K, Kref):
    num = np.abs(K - Kref) @ np.ones(K.shape[1]) if sp.issparse(K) else np.abs(K - Kref).sum(axis=1)
    den = np.abs(Kref) @ np.ones(Kref.shape[1]) if sp.issparse(Kref) else np.abs(Kref).sum(axis=1)
    return float(np.max(num) / np.max(den))


def _vec_rel(v, vref):
    return float(np.max(np.abs(v - vref)) / max(np.max(np.abs(vref)), 1e-300))


def _gpu_poisson(d, dtype, form=tg.LAPLACE, pat=None):
    pat = pat or tg.Pattern(d["conn"], len(d["coords"]))
    coords = torch.from_numpy(d["coords"]).cuda()
    if form == tg.MASS:
        vals, rhs = tg.assemble(pat, tg.MASS, coords, dtype=dtype)
    else:
        a = torch.from_numpy(d["a"]).to(dtype).cuda()
        f = torch.from_numpy(d["f"]).to(dtype).cuda()
        vals, rhs = tg.assemble(pat, tg.LAPLACE, coords, a, f)
    torch.cuda.synchronize()
    return pat, vals.double().cpu().numpy(), (rhs.double().cpu().numpy() if rhs is not None else None)


def _check_p1(d, dtype, form=tg.LAPLACE):
    print(f"p1 parity E={len(d['conn'])} dim={d['coords'].shape[1]} dtype={dtype} form={form}", flush=True)
    pat, vals, rhs = _gpu_poisson(d, dtype, form)
    if form == tg.MASS:
        A = oracle.assemble_p1(d["coords"], d["conn"], form="mass")
    else:
        A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
    rp, ci = pat.csr()
    np.testing.assert_array_equal(rp, A.row_ptr)
    np.testing.assert_array_equal(ci, A.col_idx)
    K = sp.csr_matrix((vals, ci, rp), shape=(A.n, A.n))
    err = _norm_rel(K, A.scipy())
    assert err <= TOL[dtype], err
    if form != tg.MASS:
        ferr = _vec_rel(rhs, A.rhs)
        assert ferr <= TOL[dtype], ferr
    return err


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dim,n", [(2, 1), (2, 7), (2, 64), (3, 1), (3, 5), (3, 17)])
def test_p1_laplace_parity(dim, n, dtype):
    _check_p1(meshgen.poisson_inputs(dim, n, seed=0), dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_p1_full_64cube_parity(dtype):
    """The 64^3 Kuhn mesh (1,572,864 tets) the benchmark times, checked entry by entry."""
    _check_p1(meshgen.poisson_inputs(3, 64, seed=0), dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dim,n", [(2, 9), (3, 6)])
def test_p1_mass_parity(dim, n, dtype):
    _check_p1(meshgen.poisson_inputs(dim, n, seed=3), dtype, form=tg.MASS)


def _fan_inputs(dim, m, seed):
    """A node shared by m elements (more than the one-byte routing holds for m > 256 / (dim + 1)):
    2D a fan of m triangles around the origin; 3D m tets joining a bottom apex, a ring edge and a top apex."""
    rng = np.random.default_rng(seed)
    ang = np.linspace(0, 2 * np.pi, m, endpoint=False)
    if dim == 2:
        coords = np.concatenate([[[0.0, 0.0]], np.stack([np.cos(ang), np.sin(ang)], 1)])
        conn = np.array([[0, 1 + i, 1 + (i + 1) % m] for i in range(m)], dtype=np.int32)
    else:
        ring = np.stack([np.cos(ang), np.sin(ang), 0.1 * np.sin(3 * ang)], 1)
        coords = np.concatenate([[[0.0, 0.0, -1.0], [0.0, 0.0, 1.0]], ring])
        conn = np.array([[0, 2 + i, 2 + (i + 1) % m, 1] for i in range(m)], dtype=np.int32)
    return {"coords": np.ascontiguousarray(coords), "conn": conn, "a": np.exp(rng.standard_normal(m)),
            "f": rng.uniform(-1, 1, m)}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dim,m", [(2, 85), (3, 64)])
def test_p1_compact_routing_at_its_limit(dim, m, dtype):
    """The largest valence the one-byte routing holds (256 / (dim + 1) elements at a node)."""
    d = _fan_inputs(dim, m, seed=dim + 10)
    assert tg.Pattern(d["conn"], len(d["coords"]), host_only=True).compact_routing() is not None
    _check_p1(d, dtype)
    _check_p1(d, dtype, form=tg.MASS)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dim,m", [(2, 86), (2, 100), (3, 65), (3, 80)])
def test_p1_wide_routing_parity(dim, m, dtype):
    """High-valence nodes: the pattern keeps the wide routing (its own kernel instance)."""
    d = _fan_inputs(dim, m, seed=dim)
    assert tg.Pattern(d["conn"], len(d["coords"]), host_only=True).compact_routing() is None
    _check_p1(d, dtype)
    _check_p1(d, dtype, form=tg.MASS)
    # batched members on the wide routing equal single calls bitwise
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    coords = torch.from_numpy(d["coords"]).cuda()
    rng = np.random.default_rng(9)
    a = torch.from_numpy(np.exp(rng.standard_normal((3, m)))).to(dtype).cuda()
    f = torch.from_numpy(rng.uniform(-1, 1, (3, m))).to(dtype).cuda()
    vb, rb = tg.assemble_batched(pat, tg.LAPLACE, coords, a, f)
    for b in range(3):
        v, r = tg.assemble(pat, tg.LAPLACE, coords, a[b].contiguous(), f[b].contiguous())
        assert torch.equal(vb[b], v) and torch.equal(rb[b], r)


@pytest.mark.parametrize("dim", [2, 3])
def test_single_element(dim):
    rng = np.random.default_rng(dim)
    X = rng.random((dim + 1, dim))
    d = {"coords": X, "conn": np.arange(dim + 1, dtype=np.int32)[None, :], "a": np.array([2.5]), "f": np.array([-0.7])}
    _check_p1(d, torch.float64)


def test_shuffled_numbering_parity():
    d = meshgen.poisson_inputs(3, 9, seed=8)
    c2, t2, _, _, a2, f2 = meshgen.shuffle_numbering(d["coords"], d["conn"], 4, d["a"], d["f"])
    _check_p1({"coords": c2, "conn": t2, "a": a2, "f": f2}, torch.float64)


def test_bitwise_deterministic_across_repeats_and_streams():
    d = meshgen.poisson_inputs(3, 20, seed=1)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    coords = torch.from_numpy(d["coords"]).cuda()
    a = torch.from_numpy(d["a"]).cuda()
    f = torch.from_numpy(d["f"]).cuda()
    v0, r0 = tg.assemble(pat, tg.LAPLACE, coords, a, f)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for i in range(10):
        with torch.cuda.stream(s if i % 2 else torch.cuda.current_stream()):
            noise = torch.randn(1 << 20, device="cuda").sum()  # concurrent unrelated work
            v, r = tg.assemble(pat, tg.LAPLACE, coords, a, f, stream=s if i % 2 else None)
        torch.cuda.synchronize()
        assert torch.equal(v, v0) and torch.equal(r, r0)
    del noise


def test_status_degenerate_and_nonfinite():
    d = meshgen.poisson_inputs(2, 6, seed=0)
    coords = d["coords"].copy()
    # collapse element 17: move its third vertex onto its first
    g = d["conn"][17]
    coords[g[2]] = coords[g[0]]
    pat = tg.Pattern(d["conn"], len(coords))
    st = tg.new_status()
    tg.assemble(pat, tg.LAPLACE, torch.from_numpy(coords).cuda(), torch.from_numpy(d["a"]).cuda(),
                torch.from_numpy(d["f"]).cuda(), status=st)
    bad = tg.check_status(st)
    # elements holding both merged vertices have two coincident vertices: det J == 0 in any formula.
    # Others that hold the moved vertex may be near-collinear; whether their det rounds to exactly 0
    # depends on the formula, so they may be flagged too, but only if nearly degenerate.
    exact = np.flatnonzero(np.any(d["conn"] == g[2], axis=1) & np.any(d["conn"] == g[0], axis=1))
    assert 17 in exact
    assert bad <= exact.min()
    if bad != exact.min():
        X = coords[d["conn"][bad]]
        assert abs(np.linalg.det(X[1:] - X[0])) < 1e-12
    a = d["a"].copy()
    a[40] = np.nan
    a[41] = np.inf
    st = tg.new_status()
    tg.assemble(pat, tg.LAPLACE, torch.from_numpy(d["coords"]).cuda(), torch.from_numpy(a).cuda(),
                torch.from_numpy(d["f"]).cuda(), status=st)
    assert tg.check_status(st) == 40
    st = tg.new_status()
    tg.assemble(pat, tg.LAPLACE, torch.from_numpy(d["coords"]).cuda(), torch.from_numpy(d["a"]).cuda(),
                torch.from_numpy(d["f"]).cuda(), status=st)
    assert tg.check_status(st) is None


def test_argument_checks_on_device_pattern():
    d = meshgen.poisson_inputs(2, 3, seed=0)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    coords = torch.from_numpy(d["coords"]).cuda()
    with pytest.raises(tg.TGError, match="ELASTICITY needs"):
        tg.assemble(pat, tg.ELASTICITY, coords, torch.ones(2, pat.n_elements, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        tg.assemble(pat, tg.LAPLACE, coords, torch.ones(3, device="cuda", dtype=torch.float64))


# ---------------------------------------------------------------- P2 elasticity

def _gpu_elasticity(d, dtype):
    pat = tg.Pattern(d["conn"], len(d["coords"]), order=2, ncomp=3)
    coords = torch.from_numpy(d["coords"]).cuda()
    coef = torch.from_numpy(np.stack([d["lam"], d["mu"]])).to(dtype).cuda()
    load = torch.from_numpy(d["b"]).to(dtype).cuda()
    vals, rhs = tg.assemble(pat, tg.ELASTICITY, coords, coef, load)
    torch.cuda.synchronize()
    return pat, vals.double().cpu().numpy(), rhs.double().cpu().numpy()


def _check_p2(d, dtype):
    pat, vals, rhs = _gpu_elasticity(d, dtype)
    A = oracle.assemble_p2_elasticity(d["coords"], d["conn"], d["lam"], d["mu"], d["b"])
    rp, ci = pat.csr()
    np.testing.assert_array_equal(rp, A.row_ptr)
    np.testing.assert_array_equal(ci, A.col_idx)
    K = sp.csr_matrix((vals, ci, rp), shape=(A.n, A.n))
    err = _norm_rel(K, A.scipy())
    assert err <= TOL[dtype], err
    assert _vec_rel(rhs, A.rhs) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [1, 2, 5])
def test_p2_elasticity_parity(n, dtype):
    print(f"p2 parity n={n} dtype={dtype}", flush=True)
    _check_p2(meshgen.elasticity_inputs(n, seed=0), dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_p2_shuffled_numbering_parity(dtype):
    """Random vertex and element numbering and rotated local vertex lists: every pair frame (the
    pair's node first) starts from an arbitrary local order."""
    print(f"p2 shuffled dtype={dtype}", flush=True)
    d = meshgen.elasticity_inputs(4, seed=3)
    c2, t2, _, _, lam, mu, b = meshgen.shuffle_numbering(d["coords"], d["conn"], 7, d["lam"], d["mu"], d["b"])
    _check_p2({"coords": c2, "conn": t2, "lam": lam, "mu": mu, "b": b}, dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m", [7, 40, 64])
def test_p2_high_valence_parity(m, dtype):
    """Nodes shared by m tets (both apexes and their edge): 64 pairs in one row is the P2 block capacity."""
    print(f"p2 fan m={m} dtype={dtype}", flush=True)
    d = _fan_inputs(3, m, seed=m)
    rng = np.random.default_rng(m)
    d.update(lam=rng.uniform(0.5, 2.0, m), mu=rng.uniform(0.5, 2.0, m), b=rng.standard_normal((m, 3)))
    _check_p2(d, dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_p2_full_32cube_sampled_rows(dtype):
    """The 32^3 P2 mesh (196,608 tets, 69M nonzeros): 300 sampled DoF rows rebuilt by the oracle element by element."""
    d = meshgen.elasticity_inputs(32, seed=0)
    print(f"p2 full sampled dtype={dtype}", flush=True)
    pat, vals, rhs = _gpu_elasticity(d, dtype)
    rp, ci = pat.csr()
    nodes10 = pat.element_nodes()
    ref_nodes, _ = oracle.p2_numbering(len(d["coords"]), d["conn"])
    np.testing.assert_array_equal(nodes10, ref_nodes)
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([rng.choice(pat.n_dofs, 298, replace=False), [0, pat.n_dofs - 1]]))
    node_rows = set((rows // 3).tolist())
    inc = {}
    for e in range(len(d["conn"])):
        for a, nd in enumerate(nodes10[e]):
            if nd in node_rows:
                inc.setdefault(int(nd), []).append((e, a))
    worst = 0.0
    for r in rows:
        node, c = divmod(int(r), 3)
        row = {}
        F = 0.0
        for e, a in inc[node]:
            Ke, Fe = oracle.p2_elasticity_element(d["coords"][d["conn"][e]], d["lam"][e], d["mu"][e], d["b"][e])
            for bn in range(10):
                for cc in range(3):
                    col = 3 * int(nodes10[e][bn]) + cc
                    row[col] = row.get(col, 0.0) + Ke[3 * a + c, 3 * bn + cc]
            F += Fe[3 * a + c]
        cols = np.array(sorted(row))
        np.testing.assert_array_equal(ci[rp[r]:rp[r + 1]], cols)
        ref = np.array([row[j] for j in cols])
        got = vals[rp[r]:rp[r + 1]]
        worst = max(worst, np.abs(got - ref).sum() / np.abs(ref).sum())
        assert abs(rhs[r] - F) <= TOL[dtype] * max(abs(F), 1e-3)
    assert worst <= TOL[dtype], worst


def test_p2_symmetry_and_rigid_modes_on_gpu():
    d = meshgen.elasticity_inputs(4, seed=1)
    pat, vals, _ = _gpu_elasticity(d, torch.float64)
    rp, ci = pat.csr()
    K = sp.csr_matrix((vals, ci, rp), shape=(pat.n_dofs, pat.n_dofs))
    assert abs(K - K.T).max() <= 1e-14 * abs(K).max()
    nodes10 = pat.element_nodes()
    xyz = oracle.p2_node_coords(d["coords"], d["conn"], nodes10, pat.n_nodes)
    import indep
    R = indep.rigid_modes(xyz)
    assert np.abs(K @ R.T).max() < 1e-11 * abs(K).max()


# ---------------------------------------------------------------- batched coefficients, M + K(c)

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dim,n", [(2, 20), (3, 9)])
def test_batched_members_equal_solo_bitwise(dim, n, dtype):
    d = meshgen.poisson_inputs(dim, n, seed=2)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    coords = torch.from_numpy(d["coords"]).cuda()
    rng = np.random.default_rng(5)
    B, E = 5, len(d["conn"])
    a = torch.from_numpy(np.exp(rng.standard_normal((B, E)))).to(dtype).cuda()
    f = torch.from_numpy(rng.uniform(-1, 1, (B, E))).to(dtype).cuda()
    vb, rb = tg.assemble_batched(pat, tg.LAPLACE, coords, a, f)
    for b in range(B):
        v, r = tg.assemble(pat, tg.LAPLACE, coords, a[b].contiguous(), f[b].contiguous())
        assert torch.equal(vb[b], v) and torch.equal(rb[b], r)
    # and one member against the oracle
    A = oracle.assemble_p1(d["coords"], d["conn"], a[3].double().cpu().numpy(), f[3].double().cpu().numpy())
    rp, ci = pat.csr()
    K = sp.csr_matrix((vb[3].double().cpu().numpy(), ci, rp), shape=(A.n, A.n))
    assert _norm_rel(K, A.scipy()) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dim,n", [(2, 16), (3, 6)])
def test_mass_laplace_parity(dim, n, dtype):
    d = meshgen.poisson_inputs(dim, n, seed=7)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    c = 1e-3 * d["a"]
    vals, rhs = tg.assemble(pat, tg.MASS_LAPLACE, torch.from_numpy(d["coords"]).cuda(),
                            torch.from_numpy(c).to(dtype).cuda(), torch.from_numpy(d["f"]).to(dtype).cuda())
    M = oracle.assemble_p1(d["coords"], d["conn"], form="mass").scipy()
    A = oracle.assemble_p1(d["coords"], d["conn"], c, d["f"])
    rp, ci = pat.csr()
    K = sp.csr_matrix((vals.double().cpu().numpy(), ci, rp), shape=(A.n, A.n))
    assert _norm_rel(K, M + A.scipy()) <= TOL[dtype]
    assert _vec_rel(rhs.double().cpu().numpy(), A.rhs) <= TOL[dtype]


def test_batched_argument_errors():
    d = meshgen.poisson_inputs(2, 3, seed=0)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    coords = torch.from_numpy(d["coords"]).cuda()
    with pytest.raises(ValueError):
        tg.assemble_batched(pat, tg.MASS, coords, torch.ones(2, pat.n_elements, dtype=torch.float64, device="cuda"))
    st = tg._lib.tg_assemble_batched(pat.handle, tg.LAPLACE, tg.F64, 0, coords.data_ptr(), 8, None, 8, None, None,
                                     None)
    assert st == tg.TG_E_ARG


# ---------------------------------------------------------------- blocks past the kernels' thread counts

def _special(name):
    return {"star255": lambda: special_meshes.sphere_star(255, 1),
            "star170": lambda: special_meshes.sphere_star(170, 2),
            "disjoint2": lambda: special_meshes.disjoint_simplices(2, 600, 3),
            "disjoint3": lambda: special_meshes.disjoint_simplices(3, 400, 4)}[name]()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("mesh", ["star255", "star170", "disjoint2", "disjoint3"])
def test_p1_blocks_beyond_thread_counts_parity(mesh, dtype):
    """A row with 506 / 336 pairs, 256 CSR entries and more than 256 routing units (sphere stars: the Map of
    pairs past the 256th thread and the routing and segment copies past it), and blocks of many one-pair
    rows: Laplace, mass, M + K(c) and batched members against the oracle."""
    d = _special(mesh)
    print(f"p1 beyond-threads mesh={mesh} dtype={dtype}", flush=True)
    _check_p1(d, dtype)
    _check_p1(d, dtype, form=tg.MASS)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    coords = torch.from_numpy(d["coords"]).cuda()
    c = 1e-2 * d["a"]
    vals, rhs = tg.assemble(pat, tg.MASS_LAPLACE, coords, torch.from_numpy(c).to(dtype).cuda(),
                            torch.from_numpy(d["f"]).to(dtype).cuda())
    M = oracle.assemble_p1(d["coords"], d["conn"], form="mass").scipy()
    A = oracle.assemble_p1(d["coords"], d["conn"], c, d["f"])
    rp, ci = pat.csr()
    K = sp.csr_matrix((vals.double().cpu().numpy(), ci, rp), shape=(A.n, A.n))
    assert _norm_rel(K, M + A.scipy()) <= TOL[dtype]
    E = len(d["conn"])
    rng = np.random.default_rng(11)
    a = torch.from_numpy(np.exp(rng.standard_normal((3, E)))).to(dtype).cuda()
    f = torch.from_numpy(rng.uniform(-1, 1, (3, E))).to(dtype).cuda()
    vb, rb = tg.assemble_batched(pat, tg.LAPLACE, coords, a, f)
    for b in range(3):
        v, r = tg.assemble(pat, tg.LAPLACE, coords, a[b].contiguous(), f[b].contiguous())
        assert torch.equal(vb[b], v) and torch.equal(rb[b], r)
    A2 = oracle.assemble_p1(d["coords"], d["conn"], a[2].double().cpu().numpy(), f[2].double().cpu().numpy())
    K2 = sp.csr_matrix((vb[2].double().cpu().numpy(), ci, rp), shape=(A2.n, A2.n))
    assert _norm_rel(K2, A2.scipy()) <= TOL[dtype]
    assert _vec_rel(rb[2].double().cpu().numpy(), A2.rhs) <= TOL[dtype]


@pytest.mark.parametrize("mesh", ["disjoint", "star"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_p2_blocks_beyond_thread_counts_parity(dtype, mesh):
    """P2 row blocks with 480 (disjoint tets) or 577 (a star of 64 tets sharing one vertex) node entries
    and 193 staged vertices (the star): the copies past 2 x 192 entries and past 192 vertices."""
    print(f"p2 beyond-threads mesh={mesh} dtype={dtype}", flush=True)
    d = special_meshes.disjoint_simplices(3, 120, 5) if mesh == "disjoint" else special_meshes.private_star(64, 6)
    _check_p2(d, dtype)


_P2_32 = {}


def _p2_32cube_oracle():
    if not _P2_32:
        d = meshgen.elasticity_inputs(32, seed=0)
        print("p2 32^3: the FP64 oracle assembly (about a minute on the host) ...", flush=True)
        _P2_32["d"] = d
        _P2_32["A"] = oracle.assemble_p2_elasticity(d["coords"], d["conn"], d["lam"], d["mu"], d["b"])
    return _P2_32["d"], _P2_32["A"]


@pytest.mark.timeout(600)  # the oracle's serial assembly of 69M entries takes about a minute on the host
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_p2_full_32cube_every_row(dtype):
    """The 32^3 P2 matrix (69,108,489 entries) and load the elasticity benchmark times, against the oracle
    normwise over every row (max absolute row sum), with an identical pattern."""
    d, A = _p2_32cube_oracle()
    print(f"p2 32^3 every row dtype={dtype}", flush=True)
    pat, vals, rhs = _gpu_elasticity(d, dtype)
    rp, ci = pat.csr()
    np.testing.assert_array_equal(rp, A.row_ptr)
    np.testing.assert_array_equal(ci, A.col_idx)
    row = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    err = np.bincount(row, np.abs(vals - A.vals)).max() / np.bincount(row, np.abs(A.vals)).max()
    print(f"p2 32^3 {dtype}: normwise {err:.3e}", flush=True)
    assert err <= TOL[dtype], err
    assert _vec_rel(rhs, A.rhs) <= TOL[dtype]
