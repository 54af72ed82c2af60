"""GPU Dirichlet elimination, SpMV and Jacobi-PCG against the oracle's condensed system.

Solver outputs carry the solver tolerance: the true residual of the GPU
solution on the ORACLE's condensed system (Sec. B.1.3, eq. linres) must be
<= rtol (times a small factor for the assembly difference), and RelErr
(eq. relerr) against scipy's direct solve of that system is reported and
bounded by the condition-number estimate.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
tg = pytest.importorskip("paper_2602_05052_amd")


def _setup(dim, n, seed=0, dtype=torch.float64):
    d = meshgen.poisson_inputs(dim, n, seed=seed)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    coords = torch.from_numpy(d["coords"]).cuda()
    vals, rhs = tg.assemble(pat, tg.LAPLACE, coords, torch.from_numpy(d["a"]).to(dtype).cuda(),
                            torch.from_numpy(d["f"]).to(dtype).cuda())
    return d, pat, vals, rhs


def test_dirichlet_elimination_exact():
    d, pat, vals, rhs = _setup(3, 6)
    A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
    before = vals.cpu().numpy().copy()
    tg.apply_dirichlet(pat, vals, rhs)
    after = vals.cpu().numpy()
    rp, ci = pat.csr()
    bnd = np.zeros(pat.n_dofs, bool)
    bnd[pat.constrained_dofs()] = True
    row = np.repeat(np.arange(pat.n_dofs), np.diff(rp))
    expect = np.where(bnd[row] | bnd[ci], np.where(row == ci, 1.0, 0.0), before)
    expect = np.where(bnd[row] & (row == ci), 1.0, expect)
    assert np.array_equal(after, expect)
    r = rhs.cpu().numpy()
    assert np.all(r[bnd] == 0.0)
    np.testing.assert_array_equal(np.sort(pat.constrained_dofs()), meshgen.boundary_vertices(d["coords"]))


@pytest.mark.parametrize("dim,n", [(2, 24), (3, 10)])
def test_pcg_fp64_matches_condensed_direct_solve(dim, n):
    d, pat, vals, rhs = _setup(dim, n)
    tg.apply_dirichlet(pat, vals, rhs)
    x, iters, relres = tg.pcg(pat, vals, rhs, rtol=1e-10, max_iter=10000, check_every=5)
    x = x.cpu().numpy()
    A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
    bnd = meshgen.boundary_vertices(d["coords"])
    assert relres <= 1e-10
    assert np.all(x[bnd] == 0.0)
    assert oracle.relres_lin(A, x, bnd) <= 2e-10
    u = oracle.condensed_solve(A, bnd)
    err = oracle.relerr(x, u)
    print(f"dim={dim} n={n} iters={iters} relres={relres:.3e} relerr={err:.3e}")
    assert err <= 1e-6


def test_pcg_32bit_and_16bit_columns_agree():
    """A random renumbering of a 35,937-vertex mesh puts columns more than 32767 from their rows, so the
    CG iterations read 32-bit columns; the banded original numbering uses 16-bit offsets.  Both solves
    reach the tolerance and agree after undoing the permutation."""
    d = meshgen.poisson_inputs(3, 32, seed=0)
    nv = len(d["coords"])
    perm = np.random.default_rng(3).permutation(nv).astype(np.int32)
    coords_p = np.empty_like(d["coords"])
    coords_p[perm] = d["coords"]
    xs = []
    for conn, coords, width in ((d["conn"], d["coords"], 2), (perm[d["conn"]], coords_p, 4)):
        pat = tg.Pattern(conn, nv)
        assert pat.sell_index_bytes == width
        vals, rhs = tg.assemble(pat, tg.LAPLACE, torch.from_numpy(coords).cuda(), torch.from_numpy(d["a"]).cuda(),
                                torch.from_numpy(d["f"]).cuda())
        tg.apply_dirichlet(pat, vals, rhs)
        x, iters, relres = tg.pcg(pat, vals, rhs, rtol=1e-10, max_iter=10000)
        assert relres <= 1e-10
        xs.append(x.cpu().numpy())
    x16, x32 = xs[0], xs[1][perm]
    assert np.linalg.norm(x32 - x16) <= 1e-8 * np.linalg.norm(x16)


def test_pcg_with_per_slice_lengths():
    """A pattern whose sliced-ELL slices keep lengths of their own (one row of 65 entries among rows of
    about 7): the CG iterations read the slice offsets; the solve still meets the tolerance on the
    oracle's condensed system and matches its direct solve."""
    import special_meshes
    d = special_meshes.polar_disk(64, 12, seed=4)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    assert pat.sell_uniform_len == 0
    vals, rhs = tg.assemble(pat, tg.LAPLACE, torch.from_numpy(d["coords"]).cuda(), torch.from_numpy(d["a"]).cuda(),
                            torch.from_numpy(d["f"]).cuda())
    tg.apply_dirichlet(pat, vals, rhs)
    x, iters, relres = tg.pcg(pat, vals, rhs, rtol=1e-10, max_iter=10000)
    x = x.cpu().numpy()
    A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
    bnd = np.sort(pat.constrained_dofs())
    assert len(bnd) == 64 and relres <= 1e-10  # the outer ring
    assert oracle.relres_lin(A, x, bnd) <= 2e-10
    assert oracle.relerr(x, oracle.condensed_solve(A, bnd)) <= 1e-6


def test_pcg_fp32():
    d, pat, vals, rhs = _setup(3, 12, dtype=torch.float32)
    tg.apply_dirichlet(pat, vals, rhs)
    x, iters, relres = tg.pcg(pat, vals, rhs, rtol=1e-6, max_iter=5000)
    A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
    bnd = meshgen.boundary_vertices(d["coords"])
    assert relres <= 1e-6  # the true residual: restarts from x (residual replacement) until it holds
    assert oracle.relres_lin(A, x.double().cpu().numpy(), bnd) <= 2e-5


def test_pcg_bitwise_reproducible_and_iteration_count_exact():
    d, pat, vals, rhs = _setup(3, 9)
    tg.apply_dirichlet(pat, vals, rhs)
    x1, it1, r1 = tg.pcg(pat, vals, rhs, rtol=1e-9, check_every=1)
    x2, it2, r2 = tg.pcg(pat, vals, rhs, rtol=1e-9, check_every=7)
    assert it1 == it2 and torch.equal(x1, x2) and r1 == r2


def test_pcg_noconv_reported():
    d, pat, vals, rhs = _setup(3, 8)
    tg.apply_dirichlet(pat, vals, rhs)
    with pytest.raises(tg.TGError, match="NOCONV"):
        tg.pcg(pat, vals, rhs, rtol=1e-12, max_iter=3)
    x, it, rr = tg.pcg(pat, vals, rhs, rtol=1e-12, max_iter=3, raise_on_noconv=False)
    assert it == 3 and rr > 1e-12


def test_pcg_zero_rhs():
    d, pat, vals, rhs = _setup(2, 6)
    tg.apply_dirichlet(pat, vals, rhs)
    x, it, rr = tg.pcg(pat, vals, torch.zeros_like(rhs), rtol=1e-8)
    assert it == 0 and rr == 0.0 and torch.count_nonzero(x) == 0


def test_linear_patch_with_nonzero_dirichlet_data():
    """Constant a, f = 0, g = a linear function on the boundary: the discrete solution is that function."""
    d = meshgen.poisson_inputs(3, 7, seed=4)
    E = len(d["conn"])
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    coords = torch.from_numpy(d["coords"]).cuda()
    vals, rhs = tg.assemble(pat, tg.LAPLACE, coords, torch.full((E,), 2.0, dtype=torch.float64, device="cuda"),
                            torch.zeros(E, dtype=torch.float64, device="cuda"))
    u = d["coords"] @ np.array([1.0, -2.0, 0.5]) + 0.25
    g = torch.from_numpy(u).cuda()
    tg.apply_dirichlet(pat, vals, rhs, g)
    x, it, rr = tg.pcg(pat, vals, rhs, rtol=1e-12)
    np.testing.assert_allclose(x.cpu().numpy(), u, atol=1e-9)


def test_spmv_matches_scipy():
    d, pat, vals, rhs = _setup(3, 8)
    rp, ci = pat.csr()
    K = sp.csr_matrix((vals.cpu().numpy(), ci, rp), shape=(pat.n_dofs, pat.n_dofs))
    xv = np.random.default_rng(0).standard_normal(pat.n_dofs)
    y = tg.spmv(pat, vals, torch.from_numpy(xv).cuda()).cpu().numpy()
    np.testing.assert_allclose(y, K @ xv, rtol=1e-13, atol=1e-13 * np.abs(K @ xv).max())


def test_full_64cube_solve_to_1e8():
    """The benchmark system: 64^3 Kuhn mesh, Dirichlet on all faces, Jacobi-PCG to 1e-8."""
    d, pat, vals, rhs = _setup(3, 64)
    tg.apply_dirichlet(pat, vals, rhs)
    x, iters, relres = tg.pcg(pat, vals, rhs, rtol=1e-8, check_every=20)
    print(f"64^3 PCG iters={iters} relres={relres:.3e}", flush=True)
    assert relres <= 1e-8
    A = oracle.assemble_p1(d["coords"], d["conn"], d["a"], d["f"])
    bnd = meshgen.boundary_vertices(d["coords"])
    assert oracle.relres_lin(A, x.cpu().numpy(), bnd) <= 1.05e-8


def test_pcg_nonfinite_rhs_reported():
    _, pat, vals, rhs = _setup(2, 8)
    tg.apply_dirichlet(pat, vals, rhs)
    rhs[5] = float("nan")
    with pytest.raises(tg.TGError, match="TG_E_NONFINITE"):
        tg.pcg(pat, vals, rhs, rtol=1e-8, max_iter=200)
