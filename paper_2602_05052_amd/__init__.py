"""Python binding of libtg: batched Galerkin assembly on MI355X (gfx950).

A thin ctypes layer over the C ABI in include/tg.h: argument checks and
marshalling only.  Every step of the assembly and the solve runs in the HIP
kernels of libtg.so; PyTorch provides device memory and streams.  If the
library has not been built this module raises ImportError (there is no CPU
fallback).

    import paper_2602_05052_amd as tg
    pat = tg.Pattern(conn, n_vertices, dim=3)                  # once per mesh
    K, F = tg.assemble(pat, tg.LAPLACE, coords, a, f)          # per call, on the GPU
    tg.apply_dirichlet(pat, K, F)
    x, iters, relres = tg.pcg(pat, K, F, rtol=1e-8)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libtg.so")

if not os.path.exists(_LIB_PATH):
    raise ImportError(
        f"{_LIB_PATH} is missing: build it with `python paper_2602_05052_amd/build.py` "
        "(or __graft_entry__.build()); there is no CPU fallback")

_lib = ctypes.CDLL(_LIB_PATH)

# ---------------------------------------------------------------- C declarations

TG_OK, TG_E_ARG, TG_E_DEGENERATE, TG_E_NONFINITE, TG_E_NOMEM, TG_E_HIP, TG_E_NOCONV, TG_E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32 = 0, 1
LAPLACE, MASS, ELASTICITY, MASS_LAPLACE = 0, 1, 2, 3
BOUNDARY_ALL = -1
STATUS_CLEAN = 2 ** 31 - 1
PATTERN_HOST_ONLY = 1

_STATUS_NAMES = {0: "TG_OK", -1: "TG_E_ARG", -2: "TG_E_DEGENERATE", -3: "TG_E_NONFINITE", -4: "TG_E_NOMEM",
                 -5: "TG_E_HIP", -6: "TG_E_NOCONV", -7: "TG_E_STATE"}


class _Info(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("order", ctypes.c_int32), ("ncomp", ctypes.c_int32),
                ("nodes_per_element", ctypes.c_int32),
                ("n_vertices", ctypes.c_int64), ("n_elements", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("n_dofs", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_constrained", ctypes.c_int64),
                ("n_blocks", ctypes.c_int64),
                ("d_row_ptr", ctypes.c_void_p), ("d_col_idx", ctypes.c_void_p), ("device_bytes", ctypes.c_size_t)]


_vp, _i32p, _i64, _i32 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, ctypes.c_int32
_SIGS = {
    "tg_last_error": (ctypes.c_char_p, []),
    "tg_version": (ctypes.c_char_p, []),
    "tg_pattern_create": (ctypes.c_int, [_i32, _i32, _i32, _i64, _i64, _i32p, _i32p, _i64, ctypes.c_uint32,
                                         ctypes.POINTER(_vp)]),
    "tg_pattern_query": (ctypes.c_int, [_vp, ctypes.POINTER(_Info)]),
    "tg_pattern_copy_csr": (ctypes.c_int, [_vp, _i32p, _i32p]),
    "tg_pattern_copy_constrained": (ctypes.c_int, [_vp, _i32p]),
    "tg_pattern_copy_element_nodes": (ctypes.c_int, [_vp, _i32p]),
    "tg_pattern_copy_routing": (ctypes.c_int, [_vp, _i32p, _i32p, _i32p, _i32p, _i32p,
                                               ctypes.POINTER(ctypes.c_uint16)]),
    "tg_pattern_destroy": (None, [_vp]),
    "tg_assemble": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tg_assemble_batched": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                           _vp]),
    "tg_apply_dirichlet": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "tg_spmv": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "tg_pcg": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, ctypes.c_double, _i32, _i32, _i32p,
                              ctypes.POINTER(ctypes.c_double), _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


class TGError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _check(st: int):
    if st != TG_OK:
        raise TGError(st, _lib.tg_last_error().decode())


def version() -> str:
    return _lib.tg_version().decode()


def library_path() -> str:
    return _LIB_PATH


# ---------------------------------------------------------------- torch helpers

def _torch():
    import torch
    return torch


def _dtype_code(dtype) -> int:
    torch = _torch()
    if dtype in (torch.float64, "f64", "float64", F64):
        return F64
    if dtype in (torch.float32, "f32", "float32", F32):
        return F32
    raise ValueError(f"unsupported dtype {dtype}")


def _torch_dtype(code: int):
    torch = _torch()
    return torch.float64 if code == F64 else torch.float32


def _stream_handle(stream) -> int | None:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev(t, dtype, shape, name):
    """Check a device tensor: CUDA (HIP), contiguous, dtype, number of elements."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != int(np.prod(shape)):
        raise ValueError(f"{name} must have {int(np.prod(shape))} elements ({shape}), got {t.numel()}")
    return t.data_ptr()


# ---------------------------------------------------------------- Pattern

class Pattern:
    """CSR pattern and routing of one mesh topology (built once, Sec. 2 Stage II).

    conn        : [E, dim+1] int vertex ids per simplex (host array or tensor).
    n_vertices  : number of vertices (default: conn.max() + 1).
    order/ncomp : (1, 1) P1 scalar; (2, 3) P2 elasticity (dim 3).
    dirichlet   : "boundary" (every vertex on the topological boundary), None,
                  or an array of constrained vertex ids.
    host_only   : build host arrays only (no GPU needed).
    """

    def __init__(self, conn, n_vertices: int | None = None, dim: int | None = None, order: int = 1,
                 ncomp: int = 1, dirichlet="boundary", host_only: bool = False):
        conn = np.ascontiguousarray(np.asarray(conn.cpu() if hasattr(conn, "cpu") else conn), dtype=np.int32)
        if conn.ndim != 2:
            raise ValueError("conn must be [E, dim+1]")
        dim = conn.shape[1] - 1 if dim is None else dim
        if conn.shape[1] != dim + 1:
            raise ValueError("conn must have dim+1 columns")
        nv = int(conn.max()) + 1 if n_vertices is None else int(n_vertices)
        if isinstance(dirichlet, str):
            if dirichlet != "boundary":
                raise ValueError("dirichlet must be 'boundary', None or an array")
            dptr, nd, darr = None, BOUNDARY_ALL, None
        elif dirichlet is None:
            dptr, nd, darr = None, 0, None
        else:
            darr = np.ascontiguousarray(np.asarray(dirichlet), dtype=np.int32)
            dptr, nd = darr.ctypes.data_as(_i32p), darr.size
        h = _vp()
        _check(_lib.tg_pattern_create(dim, order, ncomp, nv, conn.shape[0], conn.ctypes.data_as(_i32p), dptr, nd,
                                      PATTERN_HOST_ONLY if host_only else 0, ctypes.byref(h)))
        self._h = h
        info = _Info()
        _check(_lib.tg_pattern_query(h, ctypes.byref(info)))
        self.dim, self.order, self.ncomp = info.dim, info.order, info.ncomp
        self.k = info.nodes_per_element
        self.n_vertices, self.n_elements = info.n_vertices, info.n_elements
        self.n_nodes, self.n_dofs, self.nnz = info.n_nodes, info.n_dofs, info.nnz
        self.n_constrained, self.n_blocks = info.n_constrained, info.n_blocks
        self.device_bytes = info.device_bytes
        self.host_only = host_only

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.tg_pattern_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def csr(self):
        """(row_ptr [n_dofs+1], col_idx [nnz]) as host int32 numpy arrays."""
        rp = np.zeros(self.n_dofs + 1, dtype=np.int32)
        ci = np.zeros(max(self.nnz, 1), dtype=np.int32)
        _check(_lib.tg_pattern_copy_csr(self._h, rp.ctypes.data_as(_i32p), ci.ctypes.data_as(_i32p)))
        return rp, ci[: self.nnz]

    def constrained_dofs(self):
        out = np.zeros(max(self.n_constrained, 1), dtype=np.int32)
        _check(_lib.tg_pattern_copy_constrained(self._h, out.ctypes.data_as(_i32p)))
        return out[: self.n_constrained]

    def element_nodes(self):
        out = np.zeros((self.n_elements, self.k), dtype=np.int32)
        _check(_lib.tg_pattern_copy_element_nodes(self._h, out.ctypes.data_as(_i32p)))
        return out

    def routing(self):
        """The routing tables of Sec. 2 Stage II as host numpy arrays (see tg_pattern_copy_routing)."""
        N, P = self.n_nodes, self.n_elements * self.k
        Z = self.nnz // (self.ncomp * self.ncomp)
        out = dict(inc_ptr=np.zeros(N + 1, np.int32), inc=np.zeros(P, np.int32),
                   blk_row=np.zeros(self.n_blocks + 1, np.int32), node_rp=np.zeros(N + 1, np.int32),
                   seg_ptr=np.zeros(Z + 1, np.int32), slot=np.zeros(P * self.k, np.uint16))
        _check(_lib.tg_pattern_copy_routing(
            self._h, *(out[k].ctypes.data_as(_i32p) for k in ("inc_ptr", "inc", "blk_row", "node_rp", "seg_ptr")),
            out["slot"].ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))))
        return out

    def row_ptr_device(self):
        torch = _torch()
        rp, ci = self.csr()
        return torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()


# ---------------------------------------------------------------- operations

def assemble(pattern: Pattern, form: int, coords, coef=None, load=None, dtype=None, values=None, rhs=None,
             status=None, stream=None):
    """Assemble CSR values [nnz] and right-hand side [n_dofs] on the GPU (one fused kernel).

    coords : [n_vertices, dim] float64 device tensor.
    coef   : LAPLACE [E]; ELASTICITY [2, E] (lambda, mu); MASS None.
    load   : LAPLACE [E]; ELASTICITY [E, 3]; None for no right-hand side.
    dtype  : torch.float64 or torch.float32 (the type of coef, load and outputs).
    values, rhs : optional preallocated outputs; status : optional int32 device
    word holding STATUS_CLEAN (see tg_assemble).  Returns (values, rhs-or-None).
    """
    torch = _torch()
    if dtype is None:
        dtype = coef.dtype if coef is not None else torch.float64
    code = _dtype_code(dtype)
    tdt = _torch_dtype(code)
    E = pattern.n_elements
    cp = _dev(coords, torch.float64, (pattern.n_vertices, pattern.dim), "coords")
    if form in (LAPLACE, MASS_LAPLACE):
        coef_p = _dev(coef, tdt, (E,), "coef")
        load_p = _dev(load, tdt, (E,), "load") if load is not None else None
    elif form == ELASTICITY:
        coef_p = _dev(coef, tdt, (2, E), "coef")
        load_p = _dev(load, tdt, (E, 3), "load") if load is not None else None
    elif form == MASS:
        coef_p, load_p = None, None
    else:
        raise ValueError("form must be LAPLACE, MASS or ELASTICITY")
    dev = coords.device
    if values is None:
        values = torch.empty(pattern.nnz, dtype=tdt, device=dev)
    vp = _dev(values, tdt, (pattern.nnz,), "values")
    want_rhs = load_p is not None
    if want_rhs and rhs is None:
        rhs = torch.empty(pattern.n_dofs, dtype=tdt, device=dev)
    rp = _dev(rhs, tdt, (pattern.n_dofs,), "rhs") if (want_rhs and rhs is not None) else None
    sp = _dev(status, torch.int32, (1,), "status") if status is not None else None
    _check(_lib.tg_assemble(pattern.handle, form, code, cp, coef_p, load_p, vp, rp, sp, _stream_handle(stream)))
    return values, (rhs if want_rhs else None)


def assemble_batched(pattern: Pattern, form: int, coords, coef, load=None, values=None, rhs=None, status=None,
                     stream=None):
    """Assemble B coefficient sets in one launch (tg_assemble_batched).

    coef, load: [B, E] tensors of one dtype (load may be None).  Returns
    (values [B, nnz], rhs [B, n_dofs] or None); member b equals assemble() of
    coef[b], load[b] bitwise.
    """
    torch = _torch()
    if form not in (LAPLACE, MASS_LAPLACE):
        raise ValueError("batched assembly supports LAPLACE and MASS_LAPLACE")
    code = _dtype_code(coef.dtype)
    tdt = _torch_dtype(code)
    if coef.dim() != 2:
        raise ValueError("coef must be [B, E]")
    B = coef.shape[0]
    E = pattern.n_elements
    cp = _dev(coords, torch.float64, (pattern.n_vertices, pattern.dim), "coords")
    coef_p = _dev(coef, tdt, (B, E), "coef")
    load_p = _dev(load, tdt, (B, E), "load") if load is not None else None
    if values is None:
        values = torch.empty(B, pattern.nnz, dtype=tdt, device=coords.device)
    vp = _dev(values, tdt, (B, pattern.nnz), "values")
    if load_p is not None and rhs is None:
        rhs = torch.empty(B, pattern.n_dofs, dtype=tdt, device=coords.device)
    rp = _dev(rhs, tdt, (B, pattern.n_dofs), "rhs") if load_p is not None else None
    sp = _dev(status, torch.int32, (1,), "status") if status is not None else None
    _check(_lib.tg_assemble_batched(pattern.handle, form, code, B, cp, coef_p, load_p, vp, rp, sp,
                                    _stream_handle(stream)))
    return values, (rhs if load_p is not None else None)


def new_status(device="cuda"):
    """A device status word initialised to STATUS_CLEAN."""
    torch = _torch()
    return torch.full((1,), STATUS_CLEAN, dtype=torch.int32, device=device)


def check_status(status) -> int | None:
    """Index of the first bad element recorded in `status`, or None (synchronises)."""
    v = int(status.item())
    return None if v == STATUS_CLEAN else v


def apply_dirichlet(pattern: Pattern, values, rhs=None, g=None, stream=None):
    """Symmetric elimination of the pattern's constrained DoFs, in place (tg_apply_dirichlet)."""
    torch = _torch()
    code = _dtype_code(values.dtype)
    vp = _dev(values, values.dtype, (pattern.nnz,), "values")
    rp = _dev(rhs, values.dtype, (pattern.n_dofs,), "rhs") if rhs is not None else None
    gp = _dev(g, values.dtype, (pattern.n_dofs,), "g") if g is not None else None
    _check(_lib.tg_apply_dirichlet(pattern.handle, code, vp, rp, gp, _stream_handle(stream)))
    return values, rhs


def spmv(pattern: Pattern, values, x, y=None, stream=None):
    """y = K x on the GPU."""
    torch = _torch()
    code = _dtype_code(values.dtype)
    if y is None:
        y = torch.empty(pattern.n_dofs, dtype=values.dtype, device=values.device)
    _check(_lib.tg_spmv(pattern.handle, code, _dev(values, values.dtype, (pattern.nnz,), "values"),
                        _dev(x, values.dtype, (pattern.n_dofs,), "x"), _dev(y, values.dtype, (pattern.n_dofs,), "y"),
                        _stream_handle(stream)))
    return y


def pcg(pattern: Pattern, values, rhs, rtol: float = 1e-8, max_iter: int = 10000, check_every: int = 10, x=None,
        stream=None, raise_on_noconv: bool = True):
    """Jacobi-PCG from x0 = 0 (tg_pcg).  Returns (x, iterations, true relative residual)."""
    torch = _torch()
    code = _dtype_code(values.dtype)
    if x is None:
        x = torch.empty(pattern.n_dofs, dtype=values.dtype, device=values.device)
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    st = _lib.tg_pcg(pattern.handle, code, _dev(values, values.dtype, (pattern.nnz,), "values"),
                     _dev(rhs, values.dtype, (pattern.n_dofs,), "rhs"), _dev(x, values.dtype, (pattern.n_dofs,), "x"),
                     float(rtol), int(max_iter), int(check_every), ctypes.byref(it), ctypes.byref(rr),
                     _stream_handle(stream))
    if st != TG_OK and not (st == TG_E_NOCONV and not raise_on_noconv):
        _check(st)
    return x, it.value, rr.value
