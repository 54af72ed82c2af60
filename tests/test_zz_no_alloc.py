"""The allocation-free adjoint entry point (tg_adjoint_p1_noalloc) against tg_adjoint_p1, through the C ABI.

Both run the same kernels; the allocation-free one stages the element gradients in the library's fixed
device array instead of the pattern's scratch, so its outputs must equal tg_adjoint_p1's bit for bit: on
two calls in a row (the second on a smaller mesh, with the array holding the first call's contents), for
FP64 and FP32 and every form.  It must never grow a pattern's scratch, and it rejects a mesh beyond its
fixed size before launching anything.
"""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
tg = pytest.importorskip("paper_2602_05052_amd")


def _call(fn, pat, form, dtype, coords, coef, lam, u, w, nbatch):
    E, nv = pat.n_elements, pat.n_vertices
    dlogc = torch.full((E,), float("nan"), dtype=torch.float64, device="cuda")
    dx = torch.full((nv, pat.dim), float("nan"), dtype=torch.float64, device="cuda")
    status = tg.new_status()
    st = fn(pat.handle, form, tg.F64 if dtype == torch.float64 else tg.F32, nbatch, coords.data_ptr(),
            coef.data_ptr() if coef is not None else None, lam.data_ptr(), u.data_ptr(),
            w.data_ptr() if w is not None else None, pat.n_dofs, -1.0, dlogc.data_ptr(), dx.data_ptr(),
            status.data_ptr(), None)
    torch.cuda.synchronize()
    assert st == tg.TG_OK, tg._lib.tg_last_error().decode()
    assert tg.check_status(status) is None
    return dlogc, dx


def _inputs(dim, n, nbatch, dtype, seed):
    d = meshgen.poisson_inputs(dim, n, seed=seed)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    rng = np.random.default_rng(seed)
    nv = len(d["coords"])
    mk = lambda: torch.from_numpy(rng.standard_normal((nbatch, nv))).to(dtype).cuda()
    return (pat, torch.from_numpy(d["coords"]).cuda(), torch.from_numpy(1e-3 * d["a"]).to(dtype).cuda(),
            mk(), mk(), mk())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("form", [tg.LAPLACE, tg.MASS, tg.MASS_LAPLACE])
def test_noalloc_adjoint_equals_adjoint_on_two_calls(form, dtype):
    print(f"noalloc adjoint form={form} dtype={dtype}", flush=True)
    for dim, n, nbatch, seed in ((2, 48, 3, 1), (2, 20, 2, 2), (3, 9, 2, 3)):  # the second call is smaller
        pat, coords, coef, lam, u, w = _inputs(dim, n, nbatch, dtype, seed)
        c = None if form == tg.MASS else coef
        ww = w if form != tg.LAPLACE else None
        got = _call(tg._lib.tg_adjoint_p1_noalloc, pat, form, dtype, coords, c, lam, u, ww, nbatch)
        assert pat.scratch_bytes() == 0  # nothing was allocated for this pattern
        ref = _call(tg._lib.tg_adjoint_p1, pat, form, dtype, coords, c, lam, u, ww, nbatch)
        assert pat.scratch_bytes() > 0
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
        assert torch.isfinite(got[1]).all()


def test_noalloc_adjoint_rejects_meshes_beyond_its_array():
    d = meshgen.poisson_inputs(3, 40, seed=0)  # 384,000 tets: 4,608,000 staged doubles > 2^22
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    coords = torch.from_numpy(d["coords"]).cuda()
    v = torch.zeros(pat.n_dofs, dtype=torch.float64, device="cuda")
    coef = torch.ones(pat.n_elements, dtype=torch.float64, device="cuda")
    dlogc = torch.zeros(pat.n_elements, dtype=torch.float64, device="cuda")
    st = tg._lib.tg_adjoint_p1_noalloc(pat.handle, tg.LAPLACE, tg.F64, 1, coords.data_ptr(), coef.data_ptr(),
                                       v.data_ptr(), v.data_ptr(), None, pat.n_dofs, 1.0, dlogc.data_ptr(), None,
                                       None, None)
    assert st == tg.TG_E_ARG and "exceeds its fixed staging array" in tg._lib.tg_last_error().decode()
    assert pat.scratch_bytes() == 0
