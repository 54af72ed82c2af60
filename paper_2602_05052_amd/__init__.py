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
import sys

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
TG_E_ACCURACY = -8
F64, F32 = 0, 1
LAPLACE, MASS, ELASTICITY, MASS_LAPLACE = 0, 1, 2, 3
BOUNDARY_ALL = -1
STATUS_CLEAN = 2 ** 31 - 1
PATTERN_HOST_ONLY = 1

_STATUS_NAMES = {0: "TG_OK", -1: "TG_E_ARG", -2: "TG_E_DEGENERATE", -3: "TG_E_NONFINITE", -4: "TG_E_NOMEM",
                 -5: "TG_E_HIP", -6: "TG_E_NOCONV", -7: "TG_E_STATE", -8: "TG_E_ACCURACY"}


class _Info(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("order", ctypes.c_int32), ("ncomp", ctypes.c_int32),
                ("nodes_per_element", ctypes.c_int32),
                ("n_vertices", ctypes.c_int64), ("n_elements", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("n_dofs", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_constrained", ctypes.c_int64),
                ("n_blocks", ctypes.c_int64),
                ("d_row_ptr", ctypes.c_void_p), ("d_col_idx", ctypes.c_void_p), ("device_bytes", ctypes.c_size_t),
                ("n_slot", ctypes.c_int64), ("scratch_bytes", ctypes.c_size_t),
                ("sell_index_bytes", ctypes.c_int64), ("sell_uniform_len", ctypes.c_int64)]


class ServerResult(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_int64), ("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("relres", ctypes.c_double), ("bad_element", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_done", ctypes.c_double)]


class _ServerInfo(ctypes.Structure):
    _fields_ = [("n_queued", ctypes.c_int64), ("n_active", ctypes.c_int64), ("n_slots", ctypes.c_int64),
                ("n_groups", ctypes.c_int64), ("n_results", ctypes.c_int64), ("hbm_used", ctypes.c_size_t),
                ("hbm_budget", ctypes.c_size_t), ("n_patterns", ctypes.c_int64),
                ("n_pattern_builds", ctypes.c_int64), ("n_pattern_evictions", ctypes.c_int64),
                ("pattern_build_s", ctypes.c_double)]


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
    "tg_pattern_copy_block_vertices": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), _i32p, _i32p,
                                                      ctypes.POINTER(ctypes.c_uint32)]),
    "tg_pattern_copy_sell": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), _i32p, _i32p,
                                            ctypes.POINTER(ctypes.c_int16)]),
    "tg_pattern_copy_compact_routing": (ctypes.c_int, [_vp, _i32p, ctypes.POINTER(ctypes.c_uint16),
                                                       ctypes.POINTER(ctypes.c_uint8)]),
    "tg_pattern_destroy": (None, [_vp]),
    "tg_assemble": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tg_assemble_batched": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                           _vp]),
    "tg_apply_dirichlet": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "tg_spmv": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "tg_pcg": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, ctypes.c_double, _i32, _i32, _i32p,
                              ctypes.POINTER(ctypes.c_double), _vp]),
    "tg_adjoint_p1": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _i32, _vp, _vp, _vp, _vp, _vp, _i64,
                                     ctypes.c_double, _vp, _vp, _vp, _vp]),
    "tg_adjoint_p1_noalloc": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _i32, _vp, _vp, _vp, _vp, _vp, _i64,
                                             ctypes.c_double, _vp, _vp, _vp, _vp]),
    "tg_heat_rollout": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_double, _i32, _vp, _vp,
                                       ctypes.c_double, _i32, _i32, ctypes.POINTER(_i64),
                                       ctypes.POINTER(ctypes.c_double), _vp, _vp]),
    "tg_heat_adjoint": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_double, _i32, _vp, _vp, _vp, _vp,
                                       _vp, ctypes.c_double, _i32, _i32, ctypes.POINTER(_i64),
                                       ctypes.POINTER(ctypes.c_double), _vp, _vp]),
    "tg_server_create": (ctypes.c_int, [ctypes.c_size_t, _i32, _i32, _vp, ctypes.POINTER(_vp)]),
    "tg_server_submit": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _vp,
                                        ctypes.c_double, _i32, ctypes.POINTER(_i64)]),
    "tg_server_step": (ctypes.c_int, [_vp, _i32p, _i32p]),
    "tg_server_submit_mesh": (ctypes.c_int, [_vp, _i32, _i64, _i64, _vp, ctypes.c_uint64, ctypes.c_int,
                                             ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_double, _i32,
                                             ctypes.POINTER(_i64)]),
    "tg_server_poll": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ServerResult), _i32p]),
    "tg_server_query": (ctypes.c_int, [_vp, ctypes.POINTER(_ServerInfo)]),
    "tg_server_slot_bytes": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    "tg_server_destroy": (None, [_vp]),
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
        self.n_slot = info.n_slot
        self.sell_index_bytes = info.sell_index_bytes
        self.sell_uniform_len = info.sell_uniform_len
        self.host_only = host_only

    def scratch_bytes(self) -> int:
        """Bytes of the pattern's scratch (grown by tg_adjoint_p1 / tg_heat_*; 0 until first used)."""
        info = _Info()
        _check(_lib.tg_pattern_query(self._h, ctypes.byref(info)))
        return int(info.scratch_bytes)

    def __del__(self, _destroy=_lib.tg_pattern_destroy, _finalizing=sys.is_finalizing):
        h = getattr(self, "_h", None)
        if h is not None and h.value and not _finalizing():  # at exit the process releases everything
            _destroy(h)
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
                   seg_ptr=np.zeros(Z + 1, np.int32), slot=np.zeros(max(1, self.n_slot), np.uint16))
        _check(_lib.tg_pattern_copy_routing(
            self._h, *(out[k].ctypes.data_as(_i32p) for k in ("inc_ptr", "inc", "blk_row", "node_rp", "seg_ptr")),
            out["slot"].ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))))
        return out

    def sell(self):
        """(sell_ptr, cols, offsets) of the CG iterations' sliced-ELL pattern; offsets is None when the
        kernels read 32-bit columns (see tg_pattern_copy_sell)."""
        ne = ctypes.c_int64(0)
        _check(_lib.tg_pattern_copy_sell(self._h, ctypes.byref(ne), None, None, None))
        ptr = np.zeros((self.n_dofs + 63) // 64 + 1, np.int32)
        cols = np.zeros(max(1, ne.value), np.int32)
        off = np.zeros(max(1, ne.value), np.int16) if self.sell_index_bytes == 2 else None
        _check(_lib.tg_pattern_copy_sell(self._h, ctypes.byref(ne), ptr.ctypes.data_as(_i32p),
                                         cols.ctypes.data_as(_i32p),
                                         None if off is None else off.ctypes.data_as(ctypes.POINTER(ctypes.c_int16))))
        return ptr, cols[:ne.value], None if off is None else off[:ne.value]

    def compact_routing(self):
        """(ent16 [Z], slot8) of the P1 kernel's one-byte routing, or None when the pattern uses the wide form
        (see tg_pattern_copy_compact_routing)."""
        flag = ctypes.c_int32(0)
        _check(_lib.tg_pattern_copy_compact_routing(self._h, ctypes.byref(flag), None, None))
        if not flag.value:
            return None
        Z = self.nnz // (self.ncomp * self.ncomp)
        ent = np.zeros(max(1, Z), np.uint16)
        s8 = np.zeros(max(4, (self.n_elements * self.k * (self.k - 1) + 3) // 4 * 4), np.uint8)
        _check(_lib.tg_pattern_copy_compact_routing(self._h, ctypes.byref(flag),
                                                    ent.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                                    s8.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return ent[:Z], s8

    def block_vertices(self):
        """(blk_vptr [B+1], blk_vert, pair_lv [P]) of the kernels' per-block coordinate staging."""
        nvert = ctypes.c_int64(0)
        _check(_lib.tg_pattern_copy_block_vertices(self._h, ctypes.byref(nvert), None, None, None))
        vptr = np.zeros(self.n_blocks + 1, dtype=np.int32)
        vert = np.zeros(max(1, nvert.value), dtype=np.int32)
        lv = np.zeros(max(1, self.n_elements * self.k), dtype=np.uint32)
        _check(_lib.tg_pattern_copy_block_vertices(
            self._h, None, vptr.ctypes.data_as(_i32p), vert.ctypes.data_as(_i32p),
            lv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
        return vptr, vert[:nvert.value], lv[:self.n_elements * self.k]

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
    """Symmetric elimination of the pattern's constrained DoFs, in place (tg_apply_dirichlet).

    With values=None (and g=None) only rhs is touched: its constrained entries are set to 0.
    """
    ref = values if values is not None else rhs
    code = _dtype_code(ref.dtype)
    vp = _dev(values, ref.dtype, (pattern.nnz,), "values") if values is not None else None
    rp = _dev(rhs, ref.dtype, (pattern.n_dofs,), "rhs") if rhs is not None else None
    gp = _dev(g, ref.dtype, (pattern.n_dofs,), "g") if g is not None else None
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
        stream=None, raise_on_noconv: bool = True, return_status: bool = False):
    """Jacobi-PCG from x0 = 0 (tg_pcg).  Returns (x, iterations, true relative residual).  With
    raise_on_noconv=False, TG_E_NOCONV and TG_E_ACCURACY (rtol below the dtype's attainable true residual)
    return the last iterate instead of raising; return_status adds the status as a fourth value."""
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
    if st != TG_OK and not (st in (TG_E_NOCONV, TG_E_ACCURACY) and not raise_on_noconv):
        _check(st)
    return (x, it.value, rr.value, st) if return_status else (x, it.value, rr.value)


def adjoint_p1(pattern: Pattern, form: int, coords, coef, lam, u, w=None, scale: float = 1.0, dlogc=True,
               dcoords=True, status=None, stream=None):
    """Derivatives of Phi = scale * sum_m lam_m^T (A u_m - M w_m) (tg_adjoint_p1).

    lam, u, w : [n_dofs] or [B, n_dofs] tensors of one dtype (w may be None); coef [E] of that dtype
    (None for MASS).  dlogc / dcoords: True to allocate, a preallocated FP64 tensor, or None/False to
    skip.  Returns (dlogc [E] or None, dcoords [n_vertices, dim] or None), both FP64.
    """
    torch = _torch()
    code = _dtype_code(lam.dtype)
    tdt = _torch_dtype(code)
    n = pattern.n_dofs
    B = 1 if lam.dim() == 1 else lam.shape[0]
    shape = (n,) if lam.dim() == 1 else (B, n)
    cp = _dev(coords, torch.float64, (pattern.n_vertices, pattern.dim), "coords")
    coef_p = _dev(coef, tdt, (pattern.n_elements,), "coef") if form != MASS else None
    lp = _dev(lam, tdt, shape, "lam")
    up = _dev(u, tdt, shape, "u")
    wp = _dev(w, tdt, shape, "w") if w is not None else None
    dev = coords.device
    if dlogc is True:
        dlogc = torch.empty(pattern.n_elements, dtype=torch.float64, device=dev)
    if dcoords is True:
        dcoords = torch.empty(pattern.n_vertices, pattern.dim, dtype=torch.float64, device=dev)
    dlp = _dev(dlogc, torch.float64, (pattern.n_elements,), "dlogc") if dlogc is not None and dlogc is not False else None
    dxp = (_dev(dcoords, torch.float64, (pattern.n_vertices, pattern.dim), "dcoords")
           if dcoords is not None and dcoords is not False else None)
    sp = _dev(status, torch.int32, (1,), "status") if status is not None else None
    _check(_lib.tg_adjoint_p1(pattern.handle, form, code, B, cp, coef_p, lp, up, wp, n, float(scale), dlp, dxp, sp,
                              _stream_handle(stream)))
    return (dlogc if dlp is not None else None), (dcoords if dxp is not None else None)


def heat_rollout(pattern: Pattern, coords, log_a, u0, dt: float, nsteps: int, rtol: float = 1e-10,
                 max_iter: int = 10000, check_every: int = 10, states=None, status=None, stream=None):
    """Implicit-Euler rollout (tg_heat_rollout).  u0 [n_dofs] of the compute dtype; returns
    (states [nsteps+1, n_dofs], total PCG iterations, worst true relative residual)."""
    torch = _torch()
    code = _dtype_code(u0.dtype)
    n = pattern.n_dofs
    cp = _dev(coords, torch.float64, (pattern.n_vertices, pattern.dim), "coords")
    ap = _dev(log_a, torch.float64, (pattern.n_elements,), "log_a")
    up = _dev(u0, u0.dtype, (n,), "u0")
    if states is None:
        states = torch.empty(nsteps + 1, n, dtype=u0.dtype, device=u0.device)
    xp = _dev(states, u0.dtype, (nsteps + 1, n), "states")
    sp = _dev(status, torch.int32, (1,), "status") if status is not None else None
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    _check(_lib.tg_heat_rollout(pattern.handle, code, cp, ap, float(dt), int(nsteps), up, xp, float(rtol),
                                int(max_iter), int(check_every), ctypes.byref(it), ctypes.byref(rr), sp,
                                _stream_handle(stream)))
    return states, it.value, rr.value


def heat_adjoint(pattern: Pattern, coords, log_a, states, g, dt: float, rtol: float = 1e-10, max_iter: int = 10000,
                 check_every: int = 10, want=(True, True, True), status=None, stream=None):
    """Discrete adjoint of heat_rollout for dL/du^N = g (tg_heat_adjoint).  Returns
    (dL/dlog_a [E] FP64, dL/dcoords [n_vertices, dim] FP64, dL/du0 [n_dofs] of the dtype, iters, relres);
    outputs not asked for in `want` come back as None."""
    torch = _torch()
    code = _dtype_code(states.dtype)
    n = pattern.n_dofs
    nsteps = states.shape[0] - 1
    dev = coords.device
    cp = _dev(coords, torch.float64, (pattern.n_vertices, pattern.dim), "coords")
    ap = _dev(log_a, torch.float64, (pattern.n_elements,), "log_a")
    xp = _dev(states, states.dtype, (nsteps + 1, n), "states")
    gp = _dev(g, states.dtype, (n,), "g")
    dla = torch.empty(pattern.n_elements, dtype=torch.float64, device=dev) if want[0] else None
    dx = torch.empty(pattern.n_vertices, pattern.dim, dtype=torch.float64, device=dev) if want[1] else None
    du0 = torch.empty(n, dtype=states.dtype, device=dev) if want[2] else None
    sp = _dev(status, torch.int32, (1,), "status") if status is not None else None
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    _check(_lib.tg_heat_adjoint(pattern.handle, code, cp, ap, float(dt), int(nsteps), xp, gp,
                                dla.data_ptr() if dla is not None else None,
                                dx.data_ptr() if dx is not None else None,
                                du0.data_ptr() if du0 is not None else None, float(rtol), int(max_iter),
                                int(check_every), ctypes.byref(it), ctypes.byref(rr), sp, _stream_handle(stream)))
    return dla, dx, du0, it.value, rr.value


def server_slot_bytes(pattern: Pattern, dtype="f64") -> int:
    """Device bytes of one server slot for systems on `pattern` in `dtype` (the unit of the HBM budget)."""
    out = ctypes.c_size_t()
    _check(_lib.tg_server_slot_bytes(pattern.handle, _dtype_code(dtype), ctypes.byref(out)))
    return int(out.value)


class Server:
    """Continuous-batching request server (tg_server_*): assemble + Dirichlet + PCG requests, grouped by
    (pattern, dtype) into batched CG launches; requests join and leave between iterations.

        srv = Server(hbm_budget=8 << 30, max_slots=16, check_every=10)
        rid = srv.submit(pat, LAPLACE, coords, a, f, x=x)   # x receives the solution
        while srv.pending(): srv.step()
        for r in srv.poll(): ...                           # dicts: request_id, status, iters, relres, ...

    Every tensor handed to submit() is kept referenced until its result is polled.
    """

    def __init__(self, hbm_budget: int = 8 << 30, max_slots: int = 16, check_every: int = 10, stream=None):
        self._h = _vp()
        self._stream = stream
        _check(_lib.tg_server_create(int(hbm_budget), int(max_slots), int(check_every), _stream_handle(stream),
                                     ctypes.byref(self._h)))
        self._keep = {}

    def __del__(self, _destroy=_lib.tg_server_destroy, _finalizing=sys.is_finalizing):
        h = getattr(self, "_h", None)
        if h is not None and h.value and not _finalizing():  # at exit the process releases everything
            _destroy(h)
            self._h = None

    def submit(self, pattern: Pattern, form: int, coords, coef, load, x=None, g=None, rtol: float = 1e-8,
               max_iter: int = 10000, dtype=None) -> int:
        torch = _torch()
        if dtype is None:
            dtype = coef.dtype
        code = _dtype_code(dtype)
        tdt = _torch_dtype(code)
        E = pattern.n_elements
        cp = _dev(coords, torch.float64, (pattern.n_vertices, pattern.dim), "coords")
        if form == ELASTICITY:
            coef_p = _dev(coef, tdt, (2, E), "coef")
            load_p = _dev(load, tdt, (E, 3), "load")
        else:
            coef_p = _dev(coef, tdt, (E,), "coef")
            load_p = _dev(load, tdt, (E,), "load")
        if x is None:
            x = torch.empty(pattern.n_dofs, dtype=tdt, device=coords.device)
        xp = _dev(x, tdt, (pattern.n_dofs,), "x")
        gp = _dev(g, tdt, (pattern.n_dofs,), "g") if g is not None else None
        rid = ctypes.c_int64(0)
        _check(_lib.tg_server_submit(self._h, pattern.handle, form, code, cp, coef_p, load_p, gp, xp, float(rtol),
                                     int(max_iter), ctypes.byref(rid)))
        self._keep[rid.value] = (pattern, coords, coef, load, g, x)
        return rid.value

    def submit_mesh(self, conn, n_vertices: int, form: int, coords, coef, load, topology_key: int, x=None,
                    rtol: float = 1e-8, max_iter: int = 10000, dtype=None) -> int:
        """Queue a request on a mesh given by its connectivity (host int32 [E][dim+1]); the server builds and
        caches its CSR pattern (Dirichlet on the whole boundary) under `topology_key` (equal keys must mean
        equal connectivity)."""
        import numpy as np
        torch = _torch()
        if dtype is None:
            dtype = coef.dtype
        code = _dtype_code(dtype)
        tdt = _torch_dtype(code)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        E, dim = conn.shape[0], conn.shape[1] - 1
        p2 = form == ELASTICITY
        cp = _dev(coords, torch.float64, (int(n_vertices), dim), "coords")
        if p2:
            coef_p = _dev(coef, tdt, (2, E), "coef")
            load_p = _dev(load, tdt, (E, 3), "load")
        else:
            coef_p = _dev(coef, tdt, (E,), "coef")
            load_p = _dev(load, tdt, (E,), "load")
        if x is None:
            if p2:
                raise ValueError("pass x (the P2 DoF count depends on the edges)")
            x = torch.empty(int(n_vertices), dtype=tdt, device=coords.device)
        xp = _dev(x, tdt, (x.numel(),), "x")
        rid = ctypes.c_int64(0)
        _check(_lib.tg_server_submit_mesh(self._h, dim, int(n_vertices), E, conn.ctypes.data_as(_vp), int(topology_key),
                                          form, code, cp, coef_p, load_p, xp, float(rtol), int(max_iter),
                                          ctypes.byref(rid)))
        self._keep[rid.value] = (conn, coords, coef, load, None, x)
        return rid.value

    def solution(self, request_id: int):
        return self._keep[request_id][5]

    def step(self):
        """One scheduling round; returns (systems in flight, queued requests)."""
        a, q = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(_lib.tg_server_step(self._h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def info(self) -> dict:
        i = _ServerInfo()
        _check(_lib.tg_server_query(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _ServerInfo._fields_}

    def pending(self) -> bool:
        i = self.info()
        return i["n_queued"] + i["n_active"] > 0

    def poll(self, max_results: int = 1024, release: bool = True):
        """Finished requests as dicts (the solution tensor under "x")."""
        buf = (ServerResult * max_results)()
        n = ctypes.c_int32(0)
        _check(_lib.tg_server_poll(self._h, max_results, buf, ctypes.byref(n)))
        out = []
        for r in buf[:n.value]:
            d = {f: getattr(r, f) for f, _ in ServerResult._fields_ if f != "pad"}
            keep = self._keep.pop(r.request_id) if release else self._keep[r.request_id]
            d["x"] = keep[5]
            out.append(d)
        return out

    def drain(self, max_steps: int = 1_000_000):
        """Step until nothing is queued or in flight; returns every result (RuntimeError after max_steps
        scheduling rounds)."""
        res = []
        steps = 0
        while self.pending():
            if steps >= max_steps:
                raise RuntimeError(f"server still busy after {max_steps} rounds: {self.info()}")
            self.step()
            steps += 1
            res += self.poll()
        return res + self.poll()
