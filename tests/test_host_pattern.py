"""Host logic of libtg, no GPU: exports, CSR pattern, routing, Dirichlet sets, argument errors.

The routing check replays Stage II (Sec. 2 Alg. 2) on the CPU: the oracle's own
element matrices are pushed through the library's S_mat / S_vec segments in
their stored order, and the result must equal the oracle's scatter-add
assembly bit for bit (both sum every entry in ascending element order).
"""
import ctypes
import os
import re

import numpy as np
import pytest

import meshgen
import oracle
import special_meshes

tg = pytest.importorskip("paper_2602_05052_amd")

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "tg.h")


def test_library_exports_every_declared_symbol():
    decl = set(re.findall(r"^(?:const char \*|tg_status |void )(tg_[a-z0-9_]+)\(", open(HEADER).read(), re.M))
    assert decl, "no declarations found"
    lib = ctypes.CDLL(tg.library_path())
    for name in decl:
        assert hasattr(lib, name), name
    assert decl == set(tg.EXPORTED)


def _sequential_segment_sum(contrib, seg_ptr):
    """out[z] = contrib[seg[z]] + contrib[seg[z]+1] + ... summed left to right, starting from 0."""
    lens = np.diff(seg_ptr)
    out = np.zeros(len(lens))
    for t in range(int(lens.max()) if len(lens) else 0):
        m = lens > t
        out[m] = out[m] + contrib[seg_ptr[:-1][m] + t]
    return out


def _pair_of_slot(r, k):
    """Global pair index and local column b of every slot, in stored order."""
    nodes = len(r["inc_ptr"]) - 1
    blk_first_pair = r["inc_ptr"][r["blk_row"][:-1]]
    row_blk = np.searchsorted(r["blk_row"], np.arange(nodes), side="right") - 1
    node_of_entry = np.repeat(np.arange(nodes), np.diff(r["node_rp"]))
    seg_len = np.diff(r["seg_ptr"])
    slot_entry = np.repeat(np.arange(len(seg_len)), seg_len)
    assert len(r["slot"]) % 4 == 0 and len(r["slot"]) - r["seg_ptr"][-1] < 4  # padded to 4-slot units
    slot = r["slot"][:r["seg_ptr"][-1]].astype(np.int64)
    blk = row_blk[node_of_entry[slot_entry]]
    blk_pairs = (r["inc_ptr"][r["blk_row"][1:]] - r["inc_ptr"][r["blk_row"][:-1]])[blk]
    pair = blk_first_pair[blk] + slot % blk_pairs
    return pair, slot // blk_pairs


@pytest.mark.parametrize("dim,n", [(2, 1), (2, 7), (3, 1), (3, 4)])
def test_p1_pattern_routing_equals_oracle(dim, n):
    _replay_p1_against_oracle(meshgen.poisson_inputs(dim, n, seed=1), compact=True)


@pytest.mark.parametrize("mesh", ["star255", "star170", "disjoint2", "disjoint3"])
def test_p1_routing_beyond_thread_counts(mesh):
    """Blocks past the P1 kernel's 256 threads: a row with 506 or 336 pairs and (506 pairs) 256 CSR
    entries (257 wide segment pointers) and more than 256 four-slot routing units (sphere stars, the wide
    routing); blocks of 85 and 63 one-pair rows (disjoint simplices, the compact routing).  The routing still reproduces the
    oracle's scatter-add bit for bit."""
    d = {"star255": lambda: special_meshes.sphere_star(255, 1), "star170": lambda: special_meshes.sphere_star(170, 2),
         "disjoint2": lambda: special_meshes.disjoint_simplices(2, 600, 3),
         "disjoint3": lambda: special_meshes.disjoint_simplices(3, 400, 4)}[mesh]()
    pat = tg.Pattern(d["conn"], len(d["coords"]), host_only=True)
    rows, pairs, ents, verts = special_meshes.block_shapes(pat)
    assert verts.max() <= 256 and ents.max() <= 256
    if mesh.startswith("star"):
        k = 4
        slot_units = -(-pairs.max() * (k - 1) // 4) + 1
        assert pairs.max() > 256
        if mesh == "star255":  # nent + 1 = 257 wide segment pointers, over 256 routing units
            assert ents.max() == 256 and slot_units > 256
    _replay_p1_against_oracle(d, compact=not mesh.startswith("star"))


def _replay_p1_against_oracle(d, compact):
    dim = d["coords"].shape[1]
    pat = tg.Pattern(d["conn"], len(d["coords"]), host_only=True)
    A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
    rp, ci = pat.csr()
    np.testing.assert_array_equal(rp, A.row_ptr)
    np.testing.assert_array_equal(ci, A.col_idx)
    k = dim + 1
    r = pat.routing()
    assert r["slot"].max() < tg_block_cap(1) * k
    pairs_per_block = r["inc_ptr"][r["blk_row"][1:]] - r["inc_ptr"][r["blk_row"][:-1]]
    assert pairs_per_block.max() <= tg_block_cap(1)
    assert r["blk_row"][0] == 0 and r["blk_row"][-1] == pat.n_nodes
    # oracle element matrices, replayed through S_mat and S_vec
    Kl = np.zeros((len(d["conn"]), k, k))
    Fl = np.zeros((len(d["conn"]), k))
    for e, g in enumerate(d["conn"]):
        Kl[e], Fl[e] = oracle.p1_laplace_element(d["coords"][g], d["a"][e], d["f"][e])
    pair, b = _pair_of_slot(r, k)
    code = r["inc"][pair]
    vals = _sequential_segment_sum(Kl[code // k, code % k, b], r["seg_ptr"])
    # diagonal entries carry no slots: each sums its row's pairs' K_e[a][a] in S_vec order
    node_of_entry = np.repeat(np.arange(pat.n_nodes), np.diff(r["node_rp"]))
    diag = np.flatnonzero(ci == node_of_entry)
    assert len(diag) == pat.n_nodes and np.all(np.diff(r["seg_ptr"])[diag] == 0)
    assert np.all(np.diff(r["seg_ptr"])[np.setdiff1d(np.arange(len(ci)), diag)] > 0)
    vals[diag] = _sequential_segment_sum(Kl[r["inc"] // k, r["inc"] % k, r["inc"] % k], r["inc_ptr"])
    assert np.array_equal(vals, A.vals)  # bitwise
    # the compact routing the kernel reads names the same slots in the same order
    assert (pat.compact_routing() is not None) == compact
    if compact:
        cvals = _compact_replay(pat, r, Kl, k)
        cvals[diag] = vals[diag]
        assert np.array_equal(cvals, A.vals)
    rhs = _sequential_segment_sum(Fl[r["inc"] // k, r["inc"] % k], r["inc_ptr"])
    assert np.array_equal(rhs, A.rhs)
    # pairs ascending by element inside every node
    for i in range(pat.n_nodes):
        seg = r["inc"][r["inc_ptr"][i]:r["inc_ptr"][i + 1]] // k
        assert np.all(np.diff(seg) > 0)


def _compact_replay(pat, r, Kl, k):
    """Decode the one-byte P1 routing (tg_pattern_copy_compact_routing) on its own terms and sum the
    local matrices through it: entry z of node i sums slot8[start(z) .. start(z+1)), start(z) =
    inc_ptr[i] (k-1) + (ent16[z] & 255), code c -> pair inc_ptr[i] + c // k, column c % k."""
    ent, s8 = pat.compact_routing()
    inc_ptr, inc, node_rp, blk_row = r["inc_ptr"], r["inc"], r["node_rp"], r["blk_row"]
    vals = np.zeros(len(ent))
    for b in range(len(blk_row) - 1):
        for i in range(blk_row[b], blk_row[b + 1]):
            for z in range(node_rp[i], node_rp[i + 1]):
                assert ent[z] >> 8 == i - blk_row[b]
                start = inc_ptr[i] * (k - 1) + (ent[z] & 255)
                end = inc_ptr[i + 1] * (k - 1) if z + 1 == node_rp[i + 1] else inc_ptr[i] * (k - 1) + (ent[z + 1] & 255)
                acc = 0.0
                for g in range(start, end):
                    t, col = inc_ptr[i] + s8[g] // k, s8[g] % k
                    assert inc_ptr[i] <= t < inc_ptr[i + 1]
                    acc += Kl[inc[t] // k, inc[t] % k, col]
                vals[z] = acc
    return vals


def tg_block_cap(order):
    return 512 if order == 1 else 64


P2_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def _p2_frame(a):
    """The P2 kernel's frame of a pair whose node is local node a: the element's vertices ordered as a's
    vertex (or a's edge's two vertices), then the other vertices in local order; returns, for frame nodes
    0..9 (vertices, then the edges of P2_EDGES between frame vertices), the element's local node."""
    order = [a] if a < 4 else list(P2_EDGES[a - 4])
    order += [v for v in range(4) if v not in order]
    edges = [4 + P2_EDGES.index(tuple(sorted((order[i], order[j])))) for i, j in P2_EDGES]
    return np.array(order + edges)


P2_FRAME = np.stack([_p2_frame(a) for a in range(10)])


def test_p2_frame_rule():
    """Each frame is a permutation of the 10 local nodes that keeps vertex and edge nodes apart and puts
    the pair's own node first (vertex 0, or edge (0, 1) = frame node 4)."""
    for a in range(10):
        f = P2_FRAME[a]
        assert sorted(f) == list(range(10)) and np.all(f[:4] < 4)
        assert f[0 if a < 4 else 4] == a
    assert list(P2_FRAME[2]) == [2, 0, 1, 3, 5, 7, 9, 4, 6, 8]  # vertex 2: order (2, 0, 1, 3)
    assert list(P2_FRAME[8]) == [1, 3, 0, 2, 8, 4, 7, 6, 9, 5]  # edge (1, 3): order (1, 3, 0, 2)


@pytest.mark.parametrize("shuffle", [False, True])
def test_p2_pattern_routing_equals_oracle(shuffle):
    d = meshgen.elasticity_inputs(2, seed=2)
    if shuffle:  # arbitrary local vertex orders: every pair frame is a different permutation
        c2, t2, _, _, lam, mu, b = meshgen.shuffle_numbering(d["coords"], d["conn"], 5, d["lam"], d["mu"], d["b"])
        d = {"coords": c2, "conn": t2, "lam": lam, "mu": mu, "b": b}
    pat = tg.Pattern(d["conn"], len(d["coords"]), order=2, ncomp=3, host_only=True)
    A = oracle.assemble_p2_elasticity(d["coords"], d["conn"], d["lam"], d["mu"], d["b"])
    np.testing.assert_array_equal(pat.element_nodes(), A.nodes10)
    assert pat.n_nodes == A.n_nodes and pat.n_dofs == 3 * A.n_nodes
    rp, ci = pat.csr()
    np.testing.assert_array_equal(rp, A.row_ptr)
    np.testing.assert_array_equal(ci, A.col_idx)
    r = pat.routing()
    k = 10
    Kl = np.zeros((len(d["conn"]), 10, 3, 10, 3))
    Fl = np.zeros((len(d["conn"]), 10, 3))
    for e, g in enumerate(d["conn"]):
        Ke, Fe = oracle.p2_elasticity_element(d["coords"][g], d["lam"][e], d["mu"][e], d["b"][e])
        Kl[e], Fl[e] = Ke.reshape(10, 3, 10, 3), Fe.reshape(10, 3)
    pair, bf = _pair_of_slot(r, k)
    code = r["inc"][pair]
    e, a = code // k, code % k
    b = P2_FRAME[a, bf]  # slots name the column in the pair's frame
    # diagonal entries carry no slots: each sums its row's pairs' blocks (a, a) in S_vec order
    node_rp = r["node_rp"]
    node_of_entry = np.repeat(np.arange(pat.n_nodes), np.diff(node_rp))
    node_ci = np.concatenate([ci[9 * node_rp[i]:9 * node_rp[i] + 3 * (node_rp[i + 1] - node_rp[i]):3] // 3
                              for i in range(pat.n_nodes)])
    diag = np.flatnonzero(node_ci == node_of_entry)
    assert len(diag) == pat.n_nodes and np.all(np.diff(r["seg_ptr"])[diag] == 0)
    assert np.all(np.diff(r["seg_ptr"])[np.setdiff1d(np.arange(len(node_ci)), diag)] > 0)
    pe, pa = r["inc"] // k, r["inc"] % k
    # scalar value of node entry z, components (c, c') -> CSR position
    vals = np.zeros(pat.nnz)
    for c in range(3):
        for cc in range(3):
            v = _sequential_segment_sum(Kl[e, a, c, b, cc], r["seg_ptr"])
            v[diag] = _sequential_segment_sum(Kl[pe, pa, c, pa, cc], r["inc_ptr"])
            for i in range(pat.n_nodes):
                m = node_rp[i + 1] - node_rp[i]
                base = 9 * node_rp[i] + c * 3 * m
                vals[base + 3 * np.arange(m) + cc] = v[node_rp[i]:node_rp[i + 1]]
    assert np.array_equal(vals, A.vals)
    for c in range(3):
        rhs_c = _sequential_segment_sum(Fl[r["inc"] // k, r["inc"] % k, c], r["inc_ptr"])
        assert np.array_equal(rhs_c, A.rhs[c::3])


@pytest.mark.parametrize("dim", [2, 3])
def test_p1_boundary_dofs(dim):
    d = meshgen.poisson_inputs(dim, 5, seed=0)
    pat = tg.Pattern(d["conn"], len(d["coords"]), host_only=True)
    np.testing.assert_array_equal(pat.constrained_dofs(), meshgen.boundary_vertices(d["coords"]))
    explicit = np.array([0, 3, 7], dtype=np.int32)
    pat2 = tg.Pattern(d["conn"], len(d["coords"]), dirichlet=explicit, host_only=True)
    np.testing.assert_array_equal(pat2.constrained_dofs(), explicit)
    assert tg.Pattern(d["conn"], len(d["coords"]), dirichlet=None, host_only=True).n_constrained == 0


def test_p2_boundary_dofs_are_geometric_boundary():
    d = meshgen.elasticity_inputs(3, seed=0)
    pat = tg.Pattern(d["conn"], len(d["coords"]), order=2, ncomp=3, host_only=True)
    nodes10, nn = oracle.p2_numbering(len(d["coords"]), d["conn"])
    xyz = oracle.p2_node_coords(d["coords"], d["conn"], nodes10, nn)
    on = np.flatnonzero(np.any((xyz == 0.0) | (xyz == 1.0), axis=1))
    expect = (3 * on[:, None] + np.arange(3)[None, :]).ravel()
    np.testing.assert_array_equal(pat.constrained_dofs(), expect)


def test_shuffled_mesh_pattern():
    d = meshgen.poisson_inputs(3, 3, seed=5)
    c2, t2, *_ = meshgen.shuffle_numbering(d["coords"], d["conn"], 3)
    pat = tg.Pattern(t2, len(c2), host_only=True)
    A = oracle.assemble_p1(c2, t2, np.ones(len(t2)), np.ones(len(t2)))
    rp, ci = pat.csr()
    np.testing.assert_array_equal(rp, A.row_ptr)
    np.testing.assert_array_equal(ci, A.col_idx)


def test_argument_errors():
    c, t = meshgen.structured_mesh(2, 2)
    with pytest.raises(tg.TGError, match="TG_E_ARG"):
        tg.Pattern(t, len(c), order=2, ncomp=3, host_only=True)  # P2 needs dim 3
    bad = t.copy()
    bad[0, 0] = len(c)
    with pytest.raises(tg.TGError, match="out of range"):
        tg.Pattern(bad, len(c), host_only=True)
    rep = t.copy()
    rep[1, 1] = rep[1, 0]
    with pytest.raises(tg.TGError, match="repeats"):
        tg.Pattern(rep, len(c), host_only=True)
    with pytest.raises(tg.TGError, match="used by no element"):
        tg.Pattern(t, len(c) + 1, host_only=True)
    with pytest.raises(tg.TGError, match="out of range"):
        tg.Pattern(t, len(c), dirichlet=np.array([-1]), host_only=True)
    # a host-only pattern refuses device work (checked before any GPU call)
    pat = tg.Pattern(t, len(c), host_only=True)
    st = tg._lib.tg_assemble(pat.handle, tg.LAPLACE, tg.F64, 8, 8, 8, 8, 8, None, None)
    assert st == tg.TG_E_STATE
    assert tg._lib.tg_pcg(pat.handle, tg.F64, 8, 8, 8, 1e-8, 10, 1, None, None, None) == tg.TG_E_STATE
    assert tg._lib.tg_adjoint_p1(pat.handle, tg.LAPLACE, tg.F64, 1, 8, 8, 8, 8, None, 8, 1.0, 8, 8, None,
                                 None) == tg.TG_E_STATE
    assert tg._lib.tg_heat_rollout(pat.handle, tg.F64, 8, 8, 1e-3, 2, 8, 8, 1e-8, 10, 1, None, None, None,
                                   None) == tg.TG_E_STATE
    assert tg._lib.tg_heat_adjoint(pat.handle, tg.F64, 8, 8, 1e-3, 2, 8, 8, 8, 8, 8, 1e-8, 10, 1, None, None,
                                   None, None) == tg.TG_E_STATE
    # NULL pattern
    assert tg._lib.tg_adjoint_p1(None, tg.LAPLACE, tg.F64, 1, 8, 8, 8, 8, None, 8, 1.0, 8, 8, None,
                                 None) == tg.TG_E_ARG


def test_valence_over_capacity_rejected():
    # a fan of 600 triangles around vertex 0 exceeds the P1 block capacity
    m = 600
    ang = np.linspace(0, 2 * np.pi, m, endpoint=False)
    conn = np.array([[0, 1 + i, 1 + (i + 1) % m] for i in range(m)], dtype=np.int32)
    with pytest.raises(tg.TGError, match="block capacity"):
        tg.Pattern(conn, m + 1, host_only=True)


@pytest.mark.parametrize("dim,n,shuffle", [(3, 12, False), (3, 6, True), (2, 64, False), (2, 20, True)])
def test_block_vertex_staging_in_bounds(dim, n, shuffle):
    """The P1 kernel stages each block's vertices in LDS: every pair's local ids must lie inside its
    block's list (at most 256 entries) and name exactly its element's vertices in local order."""
    d = meshgen.poisson_inputs(dim, n, seed=0)
    coords, conn = d["coords"], d["conn"]
    if shuffle:
        coords, conn = meshgen.shuffle_numbering(coords, conn, seed=3)[:2]
    pat = tg.Pattern(conn, len(coords), host_only=True)
    vptr, vert, lv = pat.block_vertices()
    r = pat.routing()
    k = dim + 1
    assert vptr[0] == 0 and vptr[-1] == len(vert) and np.all(np.diff(vptr) >= 1)
    assert np.diff(vptr).max() <= 256
    pair_block = np.repeat(np.arange(pat.n_blocks), np.diff(r["inc_ptr"][r["blk_row"]]))
    e = r["inc"] // k
    for a in range(k):
        loc = (lv >> (8 * a)) & 255
        assert np.all(loc < np.diff(vptr)[pair_block])
        np.testing.assert_array_equal(vert[vptr[pair_block] + loc], conn[e, a])
    if k == 3:
        assert np.all(lv >> 24 == 0)
    for b in range(pat.n_blocks):  # ascending and distinct within a block
        seg = vert[vptr[b]:vptr[b + 1]]
        assert np.all(np.diff(seg) > 0)
    # the kernel copies each block's slots in whole 4-slot units from s0 rounded down to 4:
    # the units stay inside the padded slot list and inside the LDS slot array (mp (k-1) + 8)
    mp = int(np.diff(r["inc_ptr"][r["blk_row"]]).max())
    s0 = r["seg_ptr"][r["node_rp"][r["blk_row"][:-1]]]
    s1 = r["seg_ptr"][r["node_rp"][r["blk_row"][1:]]]
    sb = s0 & ~3
    nu = (s1 - sb + 3) // 4
    assert np.all(nu >= 1) and np.all(sb + 4 * nu <= len(r["slot"]))
    assert np.all(4 * nu <= mp * (k - 1) + 8)


@pytest.mark.parametrize("n", [1, 3])
def test_block_vertex_staging_p2(n):
    """P2 blocks stage the 4 vertex nodes of their elements the same way, each pair's in its frame."""
    d = meshgen.elasticity_inputs(n, seed=0)
    pat = tg.Pattern(d["conn"], len(d["coords"]), dim=3, order=2, ncomp=3, host_only=True)
    vptr, vert, lv = pat.block_vertices()
    r = pat.routing()
    nodes = pat.element_nodes()
    assert np.diff(vptr).max() <= 256 and np.all(np.diff(vptr) >= 1)
    pair_block = np.repeat(np.arange(pat.n_blocks), np.diff(r["inc_ptr"][r["blk_row"]]))
    e, a = r["inc"] // 10, r["inc"] % 10
    np.testing.assert_array_equal(nodes[:, :4], d["conn"])
    for kf in range(4):  # frame vertex kf of each pair
        loc = (lv >> (8 * kf)) & 255
        assert np.all(loc < np.diff(vptr)[pair_block])
        np.testing.assert_array_equal(vert[vptr[pair_block] + loc], nodes[e, P2_FRAME[a, kf]])


def test_p1_wide_routing_for_a_high_valence_node():
    """A node with more than 256 / k elements keeps the wide (uint16) routing; the routing still
    replays the oracle bitwise."""
    m = 100  # fan of m triangles around vertex 0
    ang = np.linspace(0, 2 * np.pi, m, endpoint=False)
    coords = np.concatenate([[[0.0, 0.0]], np.stack([np.cos(ang), np.sin(ang)], 1)])
    conn = np.array([[0, 1 + i, 1 + (i + 1) % m] for i in range(m)], dtype=np.int32)
    a = np.exp(np.random.default_rng(0).standard_normal(m))
    f = np.random.default_rng(1).uniform(-1, 1, m)
    pat = tg.Pattern(conn, m + 1, host_only=True)
    assert pat.compact_routing() is None
    r = pat.routing()
    A = oracle.assemble_p1(coords, conn, a, f)
    Kl = np.stack([oracle.p1_laplace_element(coords[g], a[e], f[e])[0] for e, g in enumerate(conn)])
    pair, b = _pair_of_slot(r, 3)
    code = r["inc"][pair]
    vals = _sequential_segment_sum(Kl[code // 3, code % 3, b], r["seg_ptr"])
    rp, ci = pat.csr()
    node_of_entry = np.repeat(np.arange(pat.n_nodes), np.diff(rp))
    diag = np.flatnonzero(ci == node_of_entry)
    vals[diag] = _sequential_segment_sum(Kl[r["inc"] // 3, r["inc"] % 3, r["inc"] % 3], r["inc_ptr"])
    assert np.array_equal(vals, A.vals)


@pytest.mark.parametrize("m,compact", [(64, True), (65, False)])
def test_p1_compact_routing_limit(m, compact):
    """3D: two apexes shared by m tets each.  m = 64 = 256 / 4 is the largest valence whose one-byte
    slot codes ((pair offset) * 4 + b <= 255) fit; one more element switches the pattern to the wide
    form.  At the limit the compact codes still replay the oracle bitwise."""
    ang = np.linspace(0, 2 * np.pi, m, endpoint=False)
    ring = np.stack([np.cos(ang), np.sin(ang), 0.1 * np.sin(3 * ang)], 1)
    coords = np.ascontiguousarray(np.concatenate([[[0.0, 0.0, -1.0], [0.0, 0.0, 1.0]], ring]))
    conn = np.array([[0, 2 + i, 2 + (i + 1) % m, 1] for i in range(m)], dtype=np.int32)
    rng = np.random.default_rng(m)
    a, f = np.exp(rng.standard_normal(m)), rng.uniform(-1, 1, m)
    pat = tg.Pattern(conn, m + 2, host_only=True)
    assert (pat.compact_routing() is not None) == compact
    if not compact:
        return
    ent, s8 = pat.compact_routing()
    assert s8[:m * 4 * 3].max() == 255  # the apex rows use the full byte range
    r = pat.routing()
    A = oracle.assemble_p1(coords, conn, a, f)
    Kl = np.stack([oracle.p1_laplace_element(coords[g], a[e], f[e])[0] for e, g in enumerate(conn)])
    vals = _compact_replay(pat, r, Kl, 4)
    rp, ci = pat.csr()
    node_of_entry = np.repeat(np.arange(pat.n_nodes), np.diff(rp))
    diag = np.flatnonzero(ci == node_of_entry)
    vals[diag] = _sequential_segment_sum(Kl[r["inc"] // 4, r["inc"] % 4, r["inc"] % 4], r["inc_ptr"])
    assert np.array_equal(vals, A.vals)


@pytest.mark.parametrize("m,ok", [(64, True), (65, False)])
def test_p2_block_capacity(m, ok):
    """P2 kernels hold a node's pairs in one wave: a node may belong to at most 64 elements."""
    conn = np.array([[0, 2 + i, 2 + (i + 1) % m, 1] for i in range(m)], dtype=np.int32)
    if ok:
        pat = tg.Pattern(conn, m + 2, order=2, ncomp=3, host_only=True)
        assert pat.n_nodes == m + 2 + 2 * m + m + 1  # vertices, 2m apex-ring edges, m ring edges, the apex edge
    else:
        with pytest.raises(tg.TGError, match="block capacity"):
            tg.Pattern(conn, m + 2, order=2, ncomp=3, host_only=True)


def test_p2_blocks_beyond_thread_counts():
    """P2 row blocks with more node entries than two per thread of the 192-thread kernel (interleaved
    disjoint tets: 480; a star of 64 tets sharing one vertex: 577) and more staged vertices than threads
    (the star: 193)."""
    d = special_meshes.disjoint_simplices(3, 120, 5)
    pat = tg.Pattern(d["conn"], len(d["coords"]), order=2, ncomp=3, host_only=True)
    rows, pairs, ents, verts = special_meshes.block_shapes(pat)
    assert ents.max() > 2 * 192 - 1 and pairs.max() <= 64
    d = special_meshes.private_star(64, 6)
    pat = tg.Pattern(d["conn"], len(d["coords"]), order=2, ncomp=3, host_only=True)
    rows, pairs, ents, verts = special_meshes.block_shapes(pat)
    assert ents.max() == 1 + 9 * 64 and verts.max() == 1 + 3 * 64 and pairs.max() == 64


def test_sell_index_width():
    """The CG iterations read 16-bit column offsets when every column of the sliced-ELL pattern lies
    within 32767 of its row (banded numberings), 32-bit columns otherwise."""
    d = meshgen.poisson_inputs(3, 32, seed=0)
    nv = len(d["coords"])
    assert nv > 32768
    assert tg.Pattern(d["conn"], nv, host_only=True).sell_index_bytes == 2
    perm = np.random.default_rng(3).permutation(nv).astype(np.int32)
    assert tg.Pattern(perm[d["conn"]], nv, host_only=True).sell_index_bytes == 4
    small = meshgen.poisson_inputs(2, 12, seed=0)
    sp = np.random.default_rng(4).permutation(len(small["coords"])).astype(np.int32)
    assert tg.Pattern(sp[small["conn"]], len(small["coords"]), host_only=True).sell_index_bytes == 2


def test_sell_uniform_slices():
    """Slices are padded to one length when that adds at most 1/32 of the entries (the 64^3 structured
    mesh: every slice 15 per row); a mesh with one long row keeps per-slice lengths."""
    d = meshgen.poisson_inputs(3, 64, seed=0)
    pat = tg.Pattern(d["conn"], len(d["coords"]), host_only=True)
    ptr, _, _ = pat.sell()
    assert pat.sell_uniform_len == 15 and np.all(np.diff(ptr) == 64 * 15)
    m = 100  # fan of m triangles around vertex 0: row 0 has m + 1 entries
    ang = np.linspace(0, 2 * np.pi, m, endpoint=False)
    coords = np.concatenate([[[0.0, 0.0]], np.stack([np.cos(ang), np.sin(ang)], 1)])
    conn = np.array([[0, 1 + i, 1 + (i + 1) % m] for i in range(m)], dtype=np.int32)
    pat = tg.Pattern(conn, m + 1, host_only=True)
    ptr, _, _ = pat.sell()
    assert pat.sell_uniform_len == 0 and np.diff(ptr).max() == 64 * (m + 1) and np.diff(ptr).min() < 64 * (m + 1)
    _check_sell(pat)


def _check_sell(pat):
    """Every sliced-ELL entry against the CSR: entry k of row r holds the row's k-th column, padding the
    column min(r, n - 1); with 16-bit offsets, column = min(r, n - 1) + offset for every entry."""
    ptr, cols, off = pat.sell()
    rp, ci = pat.csr()
    n = pat.n_dofs
    nsl = (n + 63) // 64
    assert len(ptr) == nsl + 1 and ptr[0] == 0 and np.all(np.diff(ptr) % 64 == 0) and np.all(np.diff(ptr) > 0)
    for s in range(nsl):
        L = (ptr[s + 1] - ptr[s]) // 64
        rows = np.arange(64 * s, 64 * s + 64)
        lens = np.where(rows < n, rp[np.minimum(rows, n - 1) + 1] - rp[np.minimum(rows, n - 1)], 0)
        assert L == max(1, lens.max())
        for k in range(L):
            got = cols[ptr[s] + 64 * k: ptr[s] + 64 * k + 64]
            want = np.where(k < lens, ci[np.minimum(rp[np.minimum(rows, n - 1)] + k, len(ci) - 1)],
                            np.minimum(rows, n - 1))
            np.testing.assert_array_equal(got, want)
    if off is not None:
        slice_of = np.repeat(np.arange(nsl), np.diff(ptr))
        base = np.minimum(64 * slice_of + np.arange(ptr[-1]) % 64, n - 1)
        np.testing.assert_array_equal(base + off.astype(np.int64), cols)


@pytest.mark.parametrize("renumber", [False, True])
def test_sell_pattern_against_csr(renumber):
    """The sliced-ELL copy of the pattern the CG iterations read (32-bit columns after a random renumbering
    of a 35,937-vertex mesh, 16-bit offsets otherwise) reproduces the CSR entry by entry."""
    d = meshgen.poisson_inputs(3, 32 if renumber else 9, seed=0)
    nv = len(d["coords"])
    conn = np.random.default_rng(5).permutation(nv).astype(np.int32)[d["conn"]] if renumber else d["conn"]
    pat = tg.Pattern(conn, nv, host_only=True)
    assert pat.sell_index_bytes == (4 if renumber else 2)
    _check_sell(pat)


def test_sell_pattern_p2():
    d = meshgen.elasticity_inputs(3, seed=0)
    _check_sell(tg.Pattern(d["conn"], len(d["coords"]), order=2, ncomp=3, host_only=True))
