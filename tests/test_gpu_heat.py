"""GPU parity of the adjoint kernels and the differentiable heat rollout (through the C ABI).

Bars:
  * tg_adjoint_p1 for given (lam, u, w): normwise max|x - x*| / max|x*| <= 1e-12 against the
    FP64 oracle, also for FP32 inputs (the kernel computes in FP64; the oracle is fed the same
    FP32-rounded inputs);
  * the rollout and its gradients carry the solver tolerance: states within 1e-8 and gradients
    within 1e-6 (normwise) of the oracle's direct solves at PCG rtol 1e-12;
  * end to end, central differences (h = 1e-6, PCG rtol 1e-13) of L = ||u^N - target||^2 on 20
    random elements and 20 interior coordinates;
  * FP32 compute: gradients within 2e-3 of the FP64 oracle (FP32 matrices and Krylov vectors; the
    bound is derived in the design notes from the FP32 solve accuracy).
"""
import numpy as np
import pytest

import meshgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
tg = pytest.importorskip("paper_2602_05052_amd")
from paper_2602_05052_amd.heat import heat_solve  # noqa: E402


def _rel(x, ref):
    x, ref = np.asarray(x, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _cuda(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


# ---------------------------------------------------------------- tg_adjoint_p1

@pytest.mark.parametrize("dim,n", [(2, 1), (2, 13), (3, 1), (3, 6)])
@pytest.mark.parametrize("form", ["LAPLACE", "MASS", "MASS_LAPLACE"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nbatch", [1, 3])
def test_adjoint_kernel_parity(dim, n, form, dtype, nbatch):
    print(f"adjoint parity dim={dim} n={n} form={form} dtype={dtype} nbatch={nbatch}", flush=True)
    d = meshgen.poisson_inputs(dim, n, seed=7)
    coords, conn = d["coords"], d["conn"]
    nv, E = len(coords), len(conn)
    rng = np.random.default_rng(11)
    lam, u, w = (rng.standard_normal((nbatch, nv)) for _ in range(3))
    c = d["a"]
    # the kernel sees dtype-rounded inputs; feed the oracle exactly those
    rnd = (lambda x: x.astype(np.float32).astype(np.float64)) if dtype == torch.float32 else (lambda x: x)
    lam, u, w, c = rnd(lam), rnd(u), rnd(w), rnd(c)
    fm = getattr(tg, form)
    pat = tg.Pattern(conn, nv)
    dl, dx = tg.adjoint_p1(pat, fm, _cuda(coords), _cuda(c, dtype) if fm != tg.MASS else None,
                           _cuda(lam if nbatch > 1 else lam[0], dtype), _cuda(u if nbatch > 1 else u[0], dtype),
                           _cuda(w if nbatch > 1 else w[0], dtype), scale=-0.5)
    dl, dx = dl.cpu().numpy(), dx.cpu().numpy()
    ref_l, ref_x = np.zeros(E), np.zeros((nv, dim))
    for m in range(nbatch):
        # oracle: mass=True means A holds M; for TG_MASS the stiffness part is dropped with c = 0
        cm = c if fm != tg.MASS else np.zeros(E)
        l1, x1 = oracle.p1_adjoint(coords, conn, cm, lam[m], u[m], w[m], mass=(fm != tg.LAPLACE))
        ref_l += l1
        ref_x += x1
    ref_l *= -0.5
    ref_x *= -0.5
    if fm == tg.MASS:
        assert np.all(dl == 0.0)
    else:
        assert _rel(dl, ref_l) <= 1e-12
    assert _rel(dx, ref_x) <= 1e-12


def test_adjoint_kernel_w_none_and_bitwise_repeat():
    d = meshgen.poisson_inputs(3, 8, seed=2)
    coords, conn = d["coords"], d["conn"]
    nv = len(coords)
    rng = np.random.default_rng(3)
    lam, u = rng.standard_normal(nv), rng.standard_normal(nv)
    pat = tg.Pattern(conn, nv)
    args = (pat, tg.MASS_LAPLACE, _cuda(coords), _cuda(d["a"]), _cuda(lam), _cuda(u))
    dl1, dx1 = tg.adjoint_p1(*args)
    dl2, dx2 = tg.adjoint_p1(*args, w=torch.zeros(nv, dtype=torch.float64, device="cuda"))
    dl3, dx3 = tg.adjoint_p1(*args)
    assert torch.equal(dl1, dl2) and torch.equal(dx1, dx2)
    assert torch.equal(dl1, dl3) and torch.equal(dx1, dx3)
    ref_l, ref_x = oracle.p1_adjoint(coords, conn, d["a"], lam, u, None, mass=True)
    assert _rel(dl1.cpu().numpy(), ref_l) <= 1e-12 and _rel(dx1.cpu().numpy(), ref_x) <= 1e-12
    # only one output asked for
    dl4, dx4 = tg.adjoint_p1(*args, dcoords=None)
    assert dx4 is None and torch.equal(dl4, dl1)
    dl5, dx5 = tg.adjoint_p1(*args, dlogc=None)
    assert dl5 is None and torch.equal(dx5, dx1)


def test_adjoint_kernel_argument_errors():
    d = meshgen.poisson_inputs(2, 3, seed=0)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    x = _cuda(d["coords"])
    v = torch.zeros(len(d["coords"]), dtype=torch.float64, device="cuda")
    a = _cuda(d["a"])
    lib = tg._lib
    h = pat.handle
    s = torch.cuda.current_stream().cuda_stream
    n = pat.n_dofs
    out = torch.empty(pat.n_elements, dtype=torch.float64, device="cuda")
    P = lambda t: t.data_ptr()  # noqa: E731
    assert lib.tg_adjoint_p1(h, tg.LAPLACE, tg.F64, 1, P(x), P(a), P(v), P(v), None, n - 1, 1.0, P(out), None,
                             None, s) == tg.TG_E_ARG  # stride < n_dofs
    assert lib.tg_adjoint_p1(h, tg.LAPLACE, tg.F64, 0, P(x), P(a), P(v), P(v), None, n, 1.0, P(out), None,
                             None, s) == tg.TG_E_ARG  # nbatch 0
    assert lib.tg_adjoint_p1(h, tg.LAPLACE, tg.F64, 1, P(x), P(a), P(v), P(v), None, n, 1.0, None, None,
                             None, s) == tg.TG_E_ARG  # no output
    assert lib.tg_adjoint_p1(h, tg.LAPLACE, tg.F64, 1, P(x), None, P(v), P(v), None, n, 1.0, P(out), None,
                             None, s) == tg.TG_E_ARG  # no coefficient
    assert lib.tg_adjoint_p1(h, tg.ELASTICITY, tg.F64, 1, P(x), P(a), P(v), P(v), None, n, 1.0, P(out), None,
                             None, s) == tg.TG_E_ARG  # form
    e = meshgen.elasticity_inputs(1, seed=0)
    p2 = tg.Pattern(e["conn"], len(e["coords"]), dim=3, order=2, ncomp=3)
    assert lib.tg_adjoint_p1(p2.handle, tg.LAPLACE, tg.F64, 1, P(x), P(a), P(v), P(v), None, p2.n_dofs, 1.0,
                             P(out), None, None, s) == tg.TG_E_ARG  # not P1 scalar
    assert lib.tg_heat_rollout(p2.handle, tg.F64, P(x), P(a), 1e-3, 1, P(v), P(v), 1e-8, 10, 1, None, None,
                               None, s) == tg.TG_E_ARG


# ---------------------------------------------------------------- heat rollout (256 x 256, 20 steps)

DT, NSTEPS = 1e-3, 20


def _heat_case(n, seed=0):
    d = meshgen.heat_inputs(n, seed=seed)
    coords = d["coords"]
    u0 = np.sin(np.pi * coords[:, 0]) * np.sin(np.pi * coords[:, 1])
    bnd = meshgen.boundary_vertices(coords)
    return d, u0, bnd


@pytest.fixture(scope="module")
def heat256():
    d, u0, bnd = _heat_case(256)
    target_log_a = meshgen.heat_inputs(256, seed=1)["log_a"]
    U = oracle.heat_rollout(d["coords"], d["conn"], d["log_a"], u0, DT, NSTEPS, bnd)
    Ut = oracle.heat_rollout(d["coords"], d["conn"], target_log_a, u0, DT, NSTEPS, bnd)
    g = 2.0 * (U[-1] - Ut[-1])
    grads = oracle.heat_adjoint(d["coords"], d["conn"], d["log_a"], U, DT, g, bnd)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    return {"d": d, "u0": u0, "bnd": bnd, "U": U, "target": Ut[-1], "g": g, "grads": grads, "pat": pat}


def test_heat_rollout_parity_256(heat256):
    h = heat256
    print("heat rollout 256^2 FP64", flush=True)
    states, iters, relres = tg.heat_rollout(h["pat"], _cuda(h["d"]["coords"]), _cuda(h["d"]["log_a"]),
                                            _cuda(h["u0"]), DT, NSTEPS, rtol=1e-12)
    S = states.cpu().numpy()
    assert relres <= 1e-10 and iters > 0
    assert np.array_equal(S[0], h["u0"])
    assert np.all(S[1:, h["bnd"]] == 0.0)
    for k in range(1, NSTEPS + 1):
        assert _rel(S[k], h["U"][k]) <= 1e-8, k


def test_heat_gradient_parity_256(heat256):
    h = heat256
    print("heat adjoint 256^2 FP64", flush=True)
    coords, log_a = _cuda(h["d"]["coords"]), _cuda(h["d"]["log_a"])
    states, _, _ = tg.heat_rollout(h["pat"], coords, log_a, _cuda(h["u0"]), DT, NSTEPS, rtol=1e-12)
    g = 2.0 * (states[-1] - _cuda(h["target"]))
    dla, dx, du0, iters, relres = tg.heat_adjoint(h["pat"], coords, log_a, states, g, DT, rtol=1e-12)
    rla, rx, ru0 = h["grads"]
    assert relres <= 1e-10
    assert _rel(dla.cpu().numpy(), rla) <= 1e-6
    assert _rel(dx.cpu().numpy(), rx) <= 1e-6
    assert _rel(du0.cpu().numpy(), ru0) <= 1e-6
    # bitwise reproducible
    dla2, dx2, du02, iters2, _ = tg.heat_adjoint(h["pat"], coords, log_a, states, g, DT, rtol=1e-12)
    assert iters2 == iters and torch.equal(dla, dla2) and torch.equal(dx, dx2) and torch.equal(du0, du02)


def test_heat_gradient_fp32_256(heat256):
    h = heat256
    print("heat adjoint 256^2 FP32", flush=True)
    coords, log_a = _cuda(h["d"]["coords"]), _cuda(h["d"]["log_a"])
    states, _, _ = tg.heat_rollout(h["pat"], coords, log_a, _cuda(h["u0"], torch.float32), DT, NSTEPS, rtol=1e-6)
    assert _rel(states[-1].double().cpu().numpy(), h["U"][-1]) <= 1e-4
    g = 2.0 * (states[-1] - _cuda(h["target"], torch.float32))
    dla, dx, du0, _, _ = tg.heat_adjoint(h["pat"], coords, log_a, states, g, DT, rtol=1e-6)
    rla, rx, ru0 = h["grads"]
    errs = (_rel(dla.cpu().numpy(), rla), _rel(dx.cpu().numpy(), rx), _rel(du0.double().cpu().numpy(), ru0))
    print("fp32 gradient errors", errs, flush=True)
    assert max(errs) <= 2e-3, errs


def test_autograd_function_matches_adjoint_bitwise(heat256):
    h = heat256
    coords = _cuda(h["d"]["coords"]).requires_grad_(True)
    log_a = _cuda(h["d"]["log_a"]).requires_grad_(True)
    u0 = _cuda(h["u0"]).requires_grad_(True)
    target = _cuda(h["target"])
    uN = heat_solve(h["pat"], coords, log_a, u0, DT, NSTEPS, rtol=1e-12)
    loss = ((uN - target) ** 2).sum()
    loss.backward()
    states, _, _ = tg.heat_rollout(h["pat"], coords.detach(), log_a.detach(), u0.detach(), DT, NSTEPS, rtol=1e-12)
    assert torch.equal(uN.detach(), states[-1])
    g = 2.0 * (states[-1] - target)
    dla, dx, du0, _, _ = tg.heat_adjoint(h["pat"], coords.detach(), log_a.detach(), states, g, DT, rtol=1e-12)
    assert torch.equal(log_a.grad, dla) and torch.equal(coords.grad, dx) and torch.equal(u0.grad, du0)
    # only log_a needs a gradient
    la2 = log_a.detach().clone().requires_grad_(True)
    ((heat_solve(h["pat"], coords.detach(), la2, u0.detach(), DT, NSTEPS, rtol=1e-12) - target) ** 2).sum().backward()
    assert torch.equal(la2.grad, dla)


# ---------------------------------------------------------------- end-to-end finite differences

def test_heat_gradient_central_differences():
    """Central differences (h = 1e-6, PCG rtol 1e-13) of the GPU loss on 20 random elements and
    20 interior coordinates (16 x 16 mesh, 20 steps, dt = 1e-3)."""
    d, u0, bnd = _heat_case(16)
    target_log_a = meshgen.heat_inputs(16, seed=1)["log_a"]
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    rt = 1e-13
    coords, log_a, u0t = _cuda(d["coords"]), _cuda(d["log_a"]), _cuda(u0)
    target = tg.heat_rollout(pat, coords, _cuda(target_log_a), u0t, DT, NSTEPS, rtol=rt)[0][-1]

    def loss(c, la):
        uN = tg.heat_rollout(pat, c, la, u0t, DT, NSTEPS, rtol=rt)[0][-1]
        return float(((uN - target) ** 2).sum())

    states = tg.heat_rollout(pat, coords, log_a, u0t, DT, NSTEPS, rtol=rt)[0]
    dla, dx, _, _, _ = tg.heat_adjoint(pat, coords, log_a, states, 2.0 * (states[-1] - target), DT, rtol=rt)
    dla, dx = dla.cpu().numpy(), dx.cpu().numpy()
    rng = np.random.default_rng(0)
    h = 1e-6
    for e in rng.choice(len(d["conn"]), size=20, replace=False):
        p, m = log_a.clone(), log_a.clone()
        p[e] += h
        m[e] -= h
        fd = (loss(coords, p) - loss(coords, m)) / (2 * h)
        assert abs(dla[e] - fd) <= 1e-4 * np.abs(dla).max() + 1e-3 * abs(fd), (e, dla[e], fd)
    interior = np.setdiff1d(np.arange(len(d["coords"])), bnd)
    for v in rng.choice(interior, size=20, replace=False):
        i = int(rng.integers(2))
        p, m = coords.clone(), coords.clone()
        p[v, i] += h
        m[v, i] -= h
        fd = (loss(p, log_a) - loss(m, log_a)) / (2 * h)
        assert abs(dx[v, i] - fd) <= 1e-4 * np.abs(dx).max() + 1e-3 * abs(fd), (v, i, dx[v, i], fd)


def test_heat_chain_through_initial_state():
    """u0 = sin(pi x) sin(pi y) built with torch from the coordinates: the coordinate gradient then
    also flows through u0 (torch's autograd composes with the hand-written node)."""
    d, _, bnd = _heat_case(12)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    log_a = _cuda(d["log_a"])
    target = torch.zeros(len(d["coords"]), dtype=torch.float64, device="cuda")

    def loss(c):
        u0 = torch.sin(np.pi * c[:, 0]) * torch.sin(np.pi * c[:, 1])
        return ((heat_solve(pat, c, log_a, u0, DT, 5, rtol=1e-13) - target) ** 2).sum()

    coords = _cuda(d["coords"]).requires_grad_(True)
    loss(coords).backward()
    gx = coords.grad.cpu().numpy()
    interior = np.setdiff1d(np.arange(len(d["coords"])), bnd)
    h = 1e-6
    for v in interior[[0, 5, 11, 17]]:
        for i in range(2):
            p, m = coords.detach().clone(), coords.detach().clone()
            p[v, i] += h
            m[v, i] -= h
            fd = float((loss(p) - loss(m)) / (2 * h))
            assert abs(gx[v, i] - fd) <= 1e-4 * np.abs(gx).max() + 1e-3 * abs(fd), (v, i, gx[v, i], fd)


# ---------------------------------------------------------------- edge cases

def test_heat_zero_steps_and_zero_state():
    d, u0, bnd = _heat_case(4)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    coords, log_a = _cuda(d["coords"]), _cuda(d["log_a"])
    u0t = _cuda(u0)
    states, iters, _ = tg.heat_rollout(pat, coords, log_a, u0t, DT, 0)
    assert states.shape[0] == 1 and torch.equal(states[0], u0t) and iters == 0
    g = torch.randn(pat.n_dofs, dtype=torch.float64, device="cuda")
    dla, dx, du0, _, _ = tg.heat_adjoint(pat, coords, log_a, states, g, DT)
    assert torch.equal(du0, g) and torch.all(dla == 0) and torch.all(dx == 0)
    # zero initial state: every state and every gradient is zero
    z = torch.zeros_like(u0t)
    states, _, _ = tg.heat_rollout(pat, coords, log_a, z, DT, 3)
    assert torch.all(states == 0)
    dla, dx, du0, _, _ = tg.heat_adjoint(pat, coords, log_a, states, torch.zeros_like(z), DT)
    assert torch.all(dla == 0) and torch.all(dx == 0) and torch.all(du0 == 0)


def test_heat_argument_errors():
    d, u0, _ = _heat_case(4)
    pat = tg.Pattern(d["conn"], len(d["coords"]))
    coords, log_a, u0t = _cuda(d["coords"]), _cuda(d["log_a"]), _cuda(u0)
    with pytest.raises(tg.TGError, match="dt > 0"):
        tg.heat_rollout(pat, coords, log_a, u0t, 0.0, 2)
    with pytest.raises(tg.TGError, match="rtol"):
        tg.heat_rollout(pat, coords, log_a, u0t, DT, 2, rtol=0.0)
    with pytest.raises(ValueError):
        tg.heat_rollout(pat, coords, log_a, u0t[:-1], DT, 2)
