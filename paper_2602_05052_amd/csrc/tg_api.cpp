// C ABI of libtg (declared in include/tg.h): argument checks, device upload
// of the pattern, and dispatch to the kernels.  Nothing here throws across
// the ABI: every entry point catches and converts to a tg_status.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "tg_internal.h"

namespace {

thread_local std::string g_last_error;

tg_status fail(tg_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

tg_status ok() {
    g_last_error.clear();
    return TG_OK;
}

template <typename V>
hipError_t upload(const std::vector<V> &h, V **d, size_t &bytes) {
    const size_t n = h.size() ? h.size() : 1;
    hipError_t e = hipMalloc((void **)d, n * sizeof(V));
    if (e != hipSuccess) return e;
    bytes += n * sizeof(V);
    if (h.empty()) return hipSuccess;
    return hipMemcpy(*d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice);
}

void free_device(tg::DevicePattern &d) {
    void *ptrs[] = {d.conn,    d.inc_ptr, d.inc,      d.blk_row,     d.blk_desc, d.node_rp, d.node_ci, d.node_vp, d.seg_ptr,
                    d.blk_vert, d.pair_lv,
                    d.slot,    d.ent16,   d.slot8,    d.row_ptr,     d.col_idx, d.diag_pos, d.constrained,
                    d.work,    d.partials, d.state, d.dir_rows,  d.pcg_slot, d.pcg_list, d.sell_ptr,
                    d.sell_col, d.sell_off, d.sell_vals};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (d.ws) (void)hipFree(d.ws);
    if (d.host_state) (void)hipHostFree(d.host_state);
    for (hipEvent_t ev : d.poll_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (d.host_pcg_slot) (void)hipHostFree(d.host_pcg_slot);
    d = tg::DevicePattern{};
}

// The host arrays a pattern uploads (host field, device field), one list for
// the upload and for the byte count the request server plans with.
#define TG_PATTERN_ARRAYS(X)                                                                                   \
    X(conn, conn) X(inc_ptr, inc_ptr) X(inc, inc) X(blk_row, blk_row) X(blk_desc, blk_desc) X(blk_vert, blk_vert) \
    X(pair_lv, pair_lv) X(node_rp, node_rp) X(node_ci, node_ci) X(node_vp, node_vp) X(seg_ptr, seg_ptr) X(slot, slot) X(ent16, ent16) \
    X(slot8, slot8) X(row_ptr, row_ptr) X(col_idx, col_idx) X(diag_pos, diag_pos) X(constrained, constrained)    \
    X(dirichlet_rows, dir_rows) X(sell_ptr, sell_ptr) X(sell_col, sell_col) X(sell_off, sell_off)

template <typename V>
size_t array_bytes(const std::vector<V> &h) {
    return (h.size() ? h.size() : 1) * sizeof(V);
}

// Device bytes of the PCG workspace of a pattern: Krylov vectors, the sliced-ELL
// copy of the values, partials, state, the solo slot and its list.
size_t workspace_bytes(const tg::HostPattern &h) {
    using namespace tg;
    const int64_t sell_nnz = h.sell_ptr.empty() ? 0 : (int64_t)h.sell_ptr.back();
    return (size_t)kPcgWorkVectors * h.n_dofs * sizeof(double) + (size_t)std::max<int64_t>(1, sell_nnz) * sizeof(double) +
           (size_t)kNumPartials * kMaxGrid * sizeof(double) + sizeof(PcgState) + sizeof(PcgSlot) + sizeof(int32_t);
}

tg_status create_device(tg_pattern &pt) {
    using namespace tg;
    const HostPattern &h = pt.host;
    DevicePattern &d = pt.dev;
    size_t bytes = 0;
    hipError_t e = hipGetDevice(&pt.device);
#define TG_UP(vec, field) \
    if (e == hipSuccess) e = upload(h.vec, &d.field, bytes);
    TG_PATTERN_ARRAYS(TG_UP)
#undef TG_UP
    d.n_dir_rows = (int64_t)h.dirichlet_rows.size();
    d.n_slices = h.sell_ptr.empty() ? 0 : (int64_t)h.sell_ptr.size() - 1;
    d.sell_nnz = h.sell_ptr.empty() ? 0 : (int64_t)h.sell_ptr.back();
    d.sell16 = !h.sell_off.empty();
    d.sell_len = h.sell_len;
    if (e == hipSuccess) {
        const size_t sb = (size_t)std::max<int64_t>(1, d.sell_nnz) * sizeof(double);
        e = hipMalloc((void **)&d.sell_vals, sb);
        bytes += sb;
    }
    if (e == hipSuccess) {
        const size_t wb = (size_t)kPcgWorkVectors * h.n_dofs * sizeof(double);
        e = hipMalloc((void **)&d.work, wb);
        bytes += wb;
    }
    if (e == hipSuccess) {
        const size_t pb = (size_t)kNumPartials * kMaxGrid * sizeof(double);
        e = hipMalloc((void **)&d.partials, pb);
        bytes += pb;
    }
    if (e == hipSuccess) {
        e = hipMalloc((void **)&d.state, sizeof(PcgState));
        bytes += sizeof(PcgState);
    }
    if (e == hipSuccess) e = hipHostMalloc((void **)&d.host_state, 2 * sizeof(PcgState), hipHostMallocDefault);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&d.poll_ev[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void **)&d.host_pcg_slot, sizeof(PcgSlot), hipHostMallocDefault);
    if (e == hipSuccess) {
        e = hipMalloc((void **)&d.pcg_slot, sizeof(PcgSlot));
        bytes += sizeof(PcgSlot);
    }
    if (e == hipSuccess) {
        e = hipMalloc((void **)&d.pcg_list, sizeof(int32_t));
        bytes += sizeof(int32_t);
    }
    if (e == hipSuccess) {
        const int32_t zero = 0;
        e = hipMemcpy(d.pcg_list, &zero, sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        const tg_status st = (e == hipErrorOutOfMemory) ? TG_E_NOMEM : TG_E_HIP;
        const std::string msg = std::string("device setup of the pattern failed: ") + hipGetErrorString(e);
        free_device(d);
        return fail(st, msg);
    }
    d.bytes = bytes;  // == device_bytes(h): the arrays above plus workspace_bytes(h)
    // lanes per row in the SpMV: about a quarter of the mean row length (two
    // entries per lane, more rows in flight per wave), power of two in [4, 32]
    const double mean_row = h.n_dofs ? (double)h.nnz / (double)h.n_dofs : 1.0;
    int g = 4;
    while (g < 32 && g < mean_row / 4) g *= 2;
    d.spmv_group = g;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, pt.device) == hipSuccess && prop.multiProcessorCount > 0)
        d.n_cu = prop.multiProcessorCount;
    return TG_OK;
}

bool valid_dtype(tg_dtype t) { return t == TG_F64 || t == TG_F32; }

}  // namespace

namespace tg {

size_t device_bytes(const HostPattern &h) {
    size_t bytes = 0;
#define TG_SUM(vec, field) bytes += array_bytes(h.vec);
    TG_PATTERN_ARRAYS(TG_SUM)
#undef TG_SUM
    return bytes + workspace_bytes(h);
}

tg_status upload_pattern(tg_pattern *p) {
    if (!p || !p->host_only) return api_fail(TG_E_STATE, "pattern is already on the device");
    const tg_status st = create_device(*p);
    if (st == TG_OK) p->host_only = false;
    return st;
}

}  // namespace tg

namespace {

tg_status check_device_pattern(const tg_pattern *p) {
    if (!p) return fail(TG_E_ARG, "pattern is NULL");
    if (p->host_only) return fail(TG_E_STATE, "pattern was created with TG_PATTERN_HOST_ONLY");
    return TG_OK;
}

}  // namespace

extern "C" {

const char *tg_last_error(void) { return g_last_error.c_str(); }

const char *tg_version(void) { return "libtg 0.1.0 (gfx950)"; }

tg_status tg_pattern_create(int32_t dim, int32_t order, int32_t ncomp, int64_t n_vertices, int64_t n_elements,
                            const int32_t *conn, const int32_t *dirichlet_vertices, int64_t n_dirichlet,
                            uint32_t flags, tg_pattern **out) {
    if (!out) return fail(TG_E_ARG, "out is NULL");
    *out = nullptr;
    if (flags & ~TG_PATTERN_HOST_ONLY) return fail(TG_E_ARG, "unknown flags");
    try {
        tg_pattern *pt = new tg_pattern();
        std::string msg;
        tg_status st = tg::build_host_pattern(dim, order, ncomp, n_vertices, n_elements, conn, dirichlet_vertices,
                                              n_dirichlet, pt->host, msg);
        if (st != TG_OK) {
            delete pt;
            return fail(st, msg);
        }
        pt->host_only = (flags & TG_PATTERN_HOST_ONLY) != 0;
        if (!pt->host_only) {
            st = create_device(*pt);
            if (st != TG_OK) {
                delete pt;
                return st;
            }
        }
        *out = pt;
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(TG_E_NOMEM, "host allocation failed");
    } catch (const std::exception &ex) {
        return fail(TG_E_ARG, ex.what());
    }
}

tg_status tg_pattern_query(const tg_pattern *p, tg_pattern_info *info) {
    if (!p || !info) return fail(TG_E_ARG, "NULL argument");
    const tg::HostPattern &h = p->host;
    info->dim = h.dim;
    info->order = h.order;
    info->ncomp = h.ncomp;
    info->nodes_per_element = h.k;
    info->n_vertices = h.nv;
    info->n_elements = h.E;
    info->n_nodes = h.n_nodes;
    info->n_dofs = h.n_dofs;
    info->nnz = h.nnz;
    info->n_constrained = (int64_t)h.constrained_list.size();
    info->n_blocks = h.n_blocks();
    info->d_row_ptr = p->dev.row_ptr;
    info->d_col_idx = p->dev.col_idx;
    info->device_bytes = p->host_only ? tg::device_bytes(h) : p->dev.bytes;
    info->scratch_bytes = p->host_only ? 0 : p->dev.ws_bytes;
    info->n_slot = (int64_t)h.slot.size();
    info->sell_index_bytes = h.sell_off.empty() ? 4 : 2;
    info->sell_uniform_len = h.sell_len;
    return ok();
}

tg_status tg_pattern_copy_csr(const tg_pattern *p, int32_t *h_row_ptr, int32_t *h_col_idx) {
    if (!p) return fail(TG_E_ARG, "pattern is NULL");
    if (h_row_ptr) std::memcpy(h_row_ptr, p->host.row_ptr.data(), sizeof(int32_t) * p->host.row_ptr.size());
    if (h_col_idx) std::memcpy(h_col_idx, p->host.col_idx.data(), sizeof(int32_t) * p->host.col_idx.size());
    return ok();
}

tg_status tg_pattern_copy_constrained(const tg_pattern *p, int32_t *h_dofs) {
    if (!p || !h_dofs) return fail(TG_E_ARG, "NULL argument");
    std::memcpy(h_dofs, p->host.constrained_list.data(), sizeof(int32_t) * p->host.constrained_list.size());
    return ok();
}

tg_status tg_pattern_copy_element_nodes(const tg_pattern *p, int32_t *h_nodes) {
    if (!p || !h_nodes) return fail(TG_E_ARG, "NULL argument");
    std::memcpy(h_nodes, p->host.elem_nodes.data(), sizeof(int32_t) * p->host.elem_nodes.size());
    return ok();
}

tg_status tg_pattern_copy_routing(const tg_pattern *p, int32_t *h_inc_ptr, int32_t *h_inc, int32_t *h_blk_row,
                                  int32_t *h_node_rp, int32_t *h_seg_ptr, uint16_t *h_slot) {
    if (!p) return fail(TG_E_ARG, "pattern is NULL");
    const tg::HostPattern &h = p->host;
    auto cp = [](auto *dst, const auto &v) {
        if (dst) std::memcpy(dst, v.data(), sizeof(v[0]) * v.size());
    };
    cp(h_inc_ptr, h.inc_ptr);
    cp(h_inc, h.inc);
    cp(h_blk_row, h.blk_row);
    cp(h_node_rp, h.node_rp);
    cp(h_seg_ptr, h.seg_ptr);
    cp(h_slot, h.slot);
    return ok();
}

tg_status tg_pattern_copy_sell(const tg_pattern *p, int64_t *n_entries, int32_t *h_sell_ptr, int32_t *h_cols,
                               int16_t *h_offsets) {
    if (!p) return fail(TG_E_ARG, "pattern is NULL");
    const tg::HostPattern &h = p->host;
    const int64_t ne = h.sell_ptr.empty() ? 0 : (int64_t)h.sell_ptr.back();
    if (n_entries) *n_entries = ne;
    if (h_sell_ptr) std::memcpy(h_sell_ptr, h.sell_ptr.data(), sizeof(int32_t) * h.sell_ptr.size());
    if (h_cols) {
        if (h.sell_off.empty()) {
            std::memcpy(h_cols, h.sell_col.data(), sizeof(int32_t) * h.sell_col.size());
        } else {
            const int64_t nsl = (int64_t)h.sell_ptr.size() - 1;
            for (int64_t s = 0; s < nsl; ++s)
                for (int64_t q = h.sell_ptr[s]; q < h.sell_ptr[s + 1]; ++q)
                    h_cols[q] = (int32_t)(std::min<int64_t>(s * tg::kSellRows + q % tg::kSellRows, h.n_dofs - 1) +
                                          h.sell_off[q]);
        }
    }
    if (h_offsets && !h.sell_off.empty()) std::memcpy(h_offsets, h.sell_off.data(), sizeof(int16_t) * ne);
    return ok();
}

tg_status tg_pattern_copy_compact_routing(const tg_pattern *p, int32_t *compact, uint16_t *h_ent16,
                                          uint8_t *h_slot8) {
    if (!p) return fail(TG_E_ARG, "pattern is NULL");
    const tg::HostPattern &h = p->host;
    if (h.order != 1) return fail(TG_E_ARG, "the compact routing exists for P1 patterns only");
    if (compact) *compact = h.compact ? 1 : 0;
    if (h.compact) {
        if (h_ent16) std::memcpy(h_ent16, h.ent16.data(), h.ent16.size() * sizeof(uint16_t));
        if (h_slot8) std::memcpy(h_slot8, h.slot8.data(), h.slot8.size());
    }
    return ok();
}

tg_status tg_pattern_copy_block_vertices(const tg_pattern *p, int64_t *n_vert, int32_t *h_blk_vptr,
                                         int32_t *h_blk_vert, uint32_t *h_pair_lv) {
    if (!p) return fail(TG_E_ARG, "pattern is NULL");
    const tg::HostPattern &h = p->host;
    if (n_vert) *n_vert = (int64_t)h.blk_vert.size();
    if (h_blk_vptr) {
        const int64_t nb = h.n_blocks();
        for (int64_t b = 0; b < nb; ++b) h_blk_vptr[b] = h.blk_desc[b * tg::kBlkDesc + 6];
        h_blk_vptr[nb] = (int32_t)h.blk_vert.size();
    }
    if (h_blk_vert) std::memcpy(h_blk_vert, h.blk_vert.data(), sizeof(int32_t) * h.blk_vert.size());
    if (h_pair_lv) std::memcpy(h_pair_lv, h.pair_lv.data(), sizeof(uint32_t) * h.pair_lv.size());
    return ok();
}

void tg_pattern_destroy(tg_pattern *p) {
    if (!p) return;
    if (!p->host_only) free_device(p->dev);
    delete p;
}

}  // extern "C"

namespace tg {

tg_status api_fail(tg_status st, const std::string &msg) { return fail(st, msg); }
tg_status api_ok() { return ok(); }
tg_status api_check_pattern(const tg_pattern *p) { return check_device_pattern(p); }

tg_status validate_assemble(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch, const double *d_coords,
                            const void *d_coef, const void *d_values) {
    tg_status st = check_device_pattern(p);
    if (st != TG_OK) return st;
    if (!valid_dtype(dtype)) return fail(TG_E_ARG, "invalid dtype");
    if (!d_coords || !d_values) return fail(TG_E_ARG, "d_coords and d_values are required");
    if (nbatch < 1) return fail(TG_E_ARG, "nbatch must be >= 1");
    const tg::HostPattern &h = p->host;
    const bool scalar_p1 = (h.order == 1 && h.ncomp == 1);
    // the kernels address every array with 32-bit byte offsets
    const uint64_t elt = dtype == TG_F64 ? 8 : 4, lim = (uint64_t)1 << 32, nb = (uint64_t)nbatch;
    if (nb * h.nnz * elt >= lim || (uint64_t)h.nv * h.dim * 8 >= lim || nb * h.E * 5 * elt >= lim ||
        nb * h.n_dofs * elt >= lim || (uint64_t)h.E * h.k * h.k * 2 >= lim)
        return fail(TG_E_ARG, "an array of this call exceeds 4 GiB, beyond the kernels' 32-bit offsets");
    if (form == TG_LAPLACE || form == TG_MASS || form == TG_MASS_LAPLACE) {
        if (!scalar_p1) return fail(TG_E_ARG, "LAPLACE, MASS and MASS_LAPLACE need a P1 scalar pattern (order 1, ncomp 1)");
        if (form != TG_MASS && !d_coef) return fail(TG_E_ARG, "this form needs d_coef");
        if (form == TG_MASS && nbatch != 1) return fail(TG_E_ARG, "MASS has no coefficients to batch");
    } else if (form == TG_ELASTICITY) {
        if (h.order != 2 || h.ncomp != 3) return fail(TG_E_ARG, "ELASTICITY needs a P2 vector pattern (3, 2, 3)");
        if (!d_coef) return fail(TG_E_ARG, "ELASTICITY needs d_coef (lambda, mu)");
        if (nbatch != 1) return fail(TG_E_ARG, "batched ELASTICITY is not supported");
    } else {
        return fail(TG_E_ARG, "invalid form");
    }
    return TG_OK;
}

hipError_t launch_assemble(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch, const double *d_coords,
                           const void *d_coef, const void *d_load, void *d_values, void *d_rhs, int32_t *d_status,
                           hipStream_t s) {
    if (form == TG_ELASTICITY)
        return tg::launch_assemble_p2(*p, dtype, d_coords, d_coef, d_load, d_values, d_rhs, d_status, s);
    return tg::launch_assemble_p1(*p, form, dtype, nbatch, d_coords, d_coef, form == TG_MASS ? nullptr : d_load,
                                  d_values, d_rhs, d_status, s);
}

}  // namespace tg

namespace {

tg_status assemble_impl(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch, const double *d_coords,
                        const void *d_coef, const void *d_load, void *d_values, void *d_rhs, int32_t *d_status,
                        void *stream) {
    const tg_status st = tg::validate_assemble(p, form, dtype, nbatch, d_coords, d_coef, d_values);
    if (st != TG_OK) return st;
    const hipError_t e = tg::launch_assemble(p, form, dtype, nbatch, d_coords, d_coef, d_load, d_values, d_rhs,
                                             d_status, (hipStream_t)stream);
    if (e != hipSuccess) return fail(TG_E_HIP, std::string("assembly launch failed: ") + hipGetErrorString(e));
    return ok();
}

}  // namespace

extern "C" {

tg_status tg_assemble(const tg_pattern *p, tg_form form, tg_dtype dtype, const double *d_coords, const void *d_coef,
                      const void *d_load, void *d_values, void *d_rhs, int32_t *d_status, void *stream) {
    return assemble_impl(p, form, dtype, 1, d_coords, d_coef, d_load, d_values, d_rhs, d_status, stream);
}

tg_status tg_assemble_batched(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch,
                              const double *d_coords, const void *d_coef, const void *d_load, void *d_values,
                              void *d_rhs, int32_t *d_status, void *stream) {
    if (form != TG_LAPLACE && form != TG_MASS_LAPLACE)
        return fail(TG_E_ARG, "tg_assemble_batched supports LAPLACE and MASS_LAPLACE");
    return assemble_impl(p, form, dtype, nbatch, d_coords, d_coef, d_load, d_values, d_rhs, d_status, stream);
}

tg_status tg_apply_dirichlet(const tg_pattern *p, tg_dtype dtype, void *d_values, void *d_rhs, const void *d_g,
                             void *stream) {
    tg_status st = check_device_pattern(p);
    if (st != TG_OK) return st;
    if (!valid_dtype(dtype)) return fail(TG_E_ARG, "invalid dtype");
    if (!d_values && (d_g || !d_rhs)) return fail(TG_E_ARG, "d_values is required unless only d_rhs is given");
    const hipError_t e = tg::launch_dirichlet(*p, dtype, d_values, d_rhs, d_g, (hipStream_t)stream);
    if (e != hipSuccess) return fail(TG_E_HIP, std::string("dirichlet launch failed: ") + hipGetErrorString(e));
    return ok();
}

tg_status tg_spmv(const tg_pattern *p, tg_dtype dtype, const void *d_values, const void *d_x, void *d_y,
                  void *stream) {
    tg_status st = check_device_pattern(p);
    if (st != TG_OK) return st;
    if (!valid_dtype(dtype)) return fail(TG_E_ARG, "invalid dtype");
    if (!d_values || !d_x || !d_y) return fail(TG_E_ARG, "NULL device array");
    const hipError_t e = tg::launch_spmv(*p, dtype, d_values, d_x, d_y, (hipStream_t)stream);
    if (e != hipSuccess) return fail(TG_E_HIP, std::string("spmv launch failed: ") + hipGetErrorString(e));
    return ok();
}

tg_status tg_pcg(const tg_pattern *p, tg_dtype dtype, const void *d_values, const void *d_rhs, void *d_x, double rtol,
                 int32_t max_iter, int32_t check_every, int32_t *iters, double *relres, void *stream) {
    tg_status st = check_device_pattern(p);
    if (st != TG_OK) return st;
    if (!valid_dtype(dtype)) return fail(TG_E_ARG, "invalid dtype");
    if (!d_values || !d_rhs || !d_x) return fail(TG_E_ARG, "NULL device array");
    if (!(rtol > 0.0) || max_iter < 1 || check_every < 1) return fail(TG_E_ARG, "need rtol > 0, max_iter >= 1, check_every >= 1");
    std::string msg;
    st = tg::run_pcg(*p, dtype, d_values, d_rhs, d_x, rtol, max_iter, check_every, iters, relres,
                     (hipStream_t)stream, msg);
    if (st != TG_OK) return fail(st, msg);
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------------- adjoint and heat rollout

namespace {

bool p1_scalar(const tg_pattern *p) { return p->host.order == 1 && p->host.ncomp == 1; }

// Argument checks shared by tg_adjoint_p1 and tg_adjoint_p1_noalloc.
tg_status check_adjoint(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch, const double *d_coords,
                        const void *d_coef, const void *d_lam, const void *d_u, int64_t stride, const double *d_dlogc,
                        const double *d_dcoords) {
    tg_status st = check_device_pattern(p);
    if (st != TG_OK) return st;
    if (!valid_dtype(dtype)) return fail(TG_E_ARG, "invalid dtype");
    if (!p1_scalar(p)) return fail(TG_E_ARG, "tg_adjoint_p1 needs a P1 scalar pattern (order 1, ncomp 1)");
    if (form != TG_LAPLACE && form != TG_MASS && form != TG_MASS_LAPLACE) return fail(TG_E_ARG, "invalid form");
    if (!d_coords || !d_lam || !d_u) return fail(TG_E_ARG, "d_coords, d_lam and d_u are required");
    if (form != TG_MASS && !d_coef) return fail(TG_E_ARG, "this form needs d_coef");
    if (!d_dlogc && !d_dcoords) return fail(TG_E_ARG, "nothing to compute: d_dlogc and d_dcoords are NULL");
    const tg::HostPattern &h = p->host;
    if (nbatch < 1) return fail(TG_E_ARG, "nbatch must be >= 1");
    if (stride < h.n_dofs) return fail(TG_E_ARG, "stride must be >= n_dofs");
    const uint64_t elt = dtype == TG_F64 ? 8 : 4, lim = (uint64_t)1 << 32;
    if (((uint64_t)(nbatch - 1) * stride + h.n_dofs) * elt >= lim || (uint64_t)h.E * h.k * h.dim * 8 >= lim ||
        (uint64_t)h.nv * h.dim * 8 >= lim)
        return fail(TG_E_ARG, "an array of this call exceeds 4 GiB, beyond the kernels' 32-bit offsets");
    return TG_OK;
}

// Grows the pattern's scratch to at least `bytes` (previous contents are lost).
tg_status ensure_workspace(const tg_pattern *p, size_t bytes) {
    tg::DevicePattern &d = const_cast<tg_pattern *>(p)->dev;
    if (d.ws_bytes >= bytes) return TG_OK;
    if (d.ws) (void)hipFree(d.ws);
    d.ws = nullptr;
    d.ws_bytes = 0;
    const hipError_t e = hipMalloc(&d.ws, bytes);
    if (e != hipSuccess) {
        d.ws = nullptr;
        return fail(e == hipErrorOutOfMemory ? TG_E_NOMEM : TG_E_HIP,
                    std::string("workspace allocation failed: ") + hipGetErrorString(e));
    }
    d.ws_bytes = bytes;
    return TG_OK;
}

// Consecutive 256-byte aligned pieces of one allocation.
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    }
};

tg_status check_heat(const tg_pattern *p, tg_dtype dtype, const double *d_coords, const double *d_log_a, double dt,
                     int32_t nsteps, double rtol, int32_t max_iter, int32_t check_every) {
    tg_status st = check_device_pattern(p);
    if (st != TG_OK) return st;
    if (!valid_dtype(dtype)) return fail(TG_E_ARG, "invalid dtype");
    if (!p1_scalar(p)) return fail(TG_E_ARG, "the heat rollout needs a P1 scalar pattern (order 1, ncomp 1)");
    if (!d_coords || !d_log_a) return fail(TG_E_ARG, "d_coords and d_log_a are required");
    if (!(dt > 0.0) || nsteps < 0) return fail(TG_E_ARG, "need dt > 0 and nsteps >= 0");
    if (!(rtol > 0.0) || max_iter < 1 || check_every < 1)
        return fail(TG_E_ARG, "need rtol > 0, max_iter >= 1, check_every >= 1");
    const tg::HostPattern &h = p->host;
    const uint64_t elt = dtype == TG_F64 ? 8 : 4, lim = (uint64_t)1 << 32;
    if ((uint64_t)(nsteps + 1) * h.n_dofs * elt >= lim || (uint64_t)h.nnz * elt >= lim ||
        (uint64_t)h.E * h.k * h.dim * 8 >= lim || (uint64_t)h.nv * h.dim * 8 >= lim)
        return fail(TG_E_ARG, "an array of this call exceeds 4 GiB, beyond the kernels' 32-bit offsets");
    return TG_OK;
}

// Coefficient c = dt exp(log_a), then M and A = M + K(c) with Dirichlet rows/columns in A.
hipError_t heat_matrices(const tg_pattern *p, tg_dtype dtype, const double *coords, const double *log_a, double dt,
                         void *coef, void *vals_m, void *vals_a, int32_t *status, hipStream_t s) {
    hipError_t e = tg::launch_scaled_exp(dtype, p->host.E, dt, log_a, coef, s);
    if (e == hipSuccess)
        e = tg::launch_assemble_p1(*p, TG_MASS, dtype, 1, coords, nullptr, nullptr, vals_m, nullptr, status, s);
    if (e == hipSuccess)
        e = tg::launch_assemble_p1(*p, TG_MASS_LAPLACE, dtype, 1, coords, coef, nullptr, vals_a, nullptr, status,
                                   s);
    if (e == hipSuccess) e = tg::launch_dirichlet(*p, dtype, vals_a, nullptr, nullptr, s);
    return e;
}

// One implicit solve A x = rhs on the free DoFs (rhs is zeroed on the constrained ones first).
// x0: the initial guess (the neighbouring step's solution), or NULL for x0 = 0.
tg_status heat_solve(const tg_pattern *p, tg_dtype dtype, const void *vals_a, void *rhs, void *x, const void *x0,
                     double rtol, int32_t max_iter, int32_t check_every, int64_t &iters, double &worst,
                     hipStream_t s) {
    const size_t bytes = (size_t)p->host.n_dofs * (dtype == TG_F64 ? 8 : 4);
    hipError_t e = tg::launch_dirichlet(*p, dtype, nullptr, rhs, nullptr, s);
    if (e == hipSuccess && x0) e = hipMemcpyAsync(x, x0, bytes, hipMemcpyDeviceToDevice, s);
    // constrained entries of the guess set to their value 0, so that they stay exactly 0
    if (e == hipSuccess && x0) e = tg::launch_dirichlet(*p, dtype, nullptr, x, nullptr, s);
    if (e != hipSuccess) return fail(TG_E_HIP, std::string("heat solve setup failed: ") + hipGetErrorString(e));
    int32_t it = 0;
    double rr = 0.0;
    std::string msg;
    const tg_status st =
        tg::run_pcg(*p, dtype, vals_a, rhs, x, rtol, max_iter, check_every, &it, &rr, s, msg, x0 != nullptr,
                    /*strict=*/false);
    iters += it;
    if (rr > worst) worst = rr;
    if (st != TG_OK) return fail(st, msg);
    return TG_OK;
}

}  // namespace

extern "C" {

tg_status tg_adjoint_p1(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch, const double *d_coords,
                        const void *d_coef, const void *d_lam, const void *d_u, const void *d_w, int64_t stride,
                        double scale, double *d_dlogc, double *d_dcoords, int32_t *d_status, void *stream) {
    tg_status st = check_adjoint(p, form, dtype, nbatch, d_coords, d_coef, d_lam, d_u, stride, d_dlogc, d_dcoords);
    if (st != TG_OK) return st;
    const tg::HostPattern &h = p->host;
    st = ensure_workspace(p, std::max<size_t>(256, (size_t)h.E * h.k * h.dim * sizeof(double)));
    if (st != TG_OK) return st;
    const hipError_t e =
        tg::launch_adjoint_p1(*p, form, dtype, nbatch, d_coords, d_coef, d_lam, d_u, d_w, stride, scale, d_dlogc,
                              d_dcoords, (double *)p->dev.ws, d_status, (hipStream_t)stream);
    if (e != hipSuccess) return fail(TG_E_HIP, std::string("adjoint launch failed: ") + hipGetErrorString(e));
    return ok();
}

tg_status tg_adjoint_p1_noalloc(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch,
                                const double *d_coords, const void *d_coef, const void *d_lam, const void *d_u,
                                const void *d_w, int64_t stride, double scale, double *d_dlogc, double *d_dcoords,
                                int32_t *d_status, void *stream) {
    tg_status st = check_adjoint(p, form, dtype, nbatch, d_coords, d_coef, d_lam, d_u, stride, d_dlogc, d_dcoords);
    if (st != TG_OK) return st;
    const tg::HostPattern &h = p->host;
    const uint64_t need = (uint64_t)h.E * h.k * h.dim;
    if (need > tg::kNoAllocStageDoubles)
        return fail(TG_E_ARG, "tg_adjoint_p1_noalloc: n_elements * (dim + 1) * dim = " + std::to_string(need) +
                                  " doubles exceeds its fixed staging array of " +
                                  std::to_string(tg::kNoAllocStageDoubles) + " (use tg_adjoint_p1)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return fail(TG_E_STATE, "tg_adjoint_p1_noalloc: the current device is not the pattern's device");
    double *stage = nullptr;
    hipError_t e = tg::noalloc_stage(&stage);
    if (e != hipSuccess)
        return fail(TG_E_HIP, std::string("tg_adjoint_p1_noalloc: staging array address: ") + hipGetErrorString(e));
    e = tg::launch_adjoint_p1(*p, form, dtype, nbatch, d_coords, d_coef, d_lam, d_u, d_w, stride, scale, d_dlogc,
                              d_dcoords, stage, d_status, (hipStream_t)stream);
    if (e != hipSuccess) return fail(TG_E_HIP, std::string("adjoint launch failed: ") + hipGetErrorString(e));
    return ok();
}

tg_status tg_heat_rollout(const tg_pattern *p, tg_dtype dtype, const double *d_coords, const double *d_log_a,
                          double dt, int32_t nsteps, const void *d_u0, void *d_states, double rtol, int32_t max_iter,
                          int32_t check_every, int64_t *iters, double *relres, int32_t *d_status, void *stream) {
    tg_status st = check_heat(p, dtype, d_coords, d_log_a, dt, nsteps, rtol, max_iter, check_every);
    if (st != TG_OK) return st;
    if (!d_u0 || !d_states) return fail(TG_E_ARG, "d_u0 and d_states are required");
    const tg::HostPattern &h = p->host;
    const size_t elt = dtype == TG_F64 ? 8 : 4, n = (size_t)h.n_dofs;
    Carve cv;
    const size_t o_coef = cv.take(h.E * elt), o_m = cv.take(h.nnz * elt), o_a = cv.take(h.nnz * elt),
                 o_rhs = cv.take(n * elt);
    st = ensure_workspace(p, cv.off);
    if (st != TG_OK) return st;
    char *ws = (char *)p->dev.ws;
    const hipStream_t s = (hipStream_t)stream;
    char *states = (char *)d_states;
    hipError_t e = hipMemcpyAsync(states, d_u0, n * elt, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && nsteps > 0)
        e = heat_matrices(p, dtype, d_coords, d_log_a, dt, ws + o_coef, ws + o_m, ws + o_a, d_status, s);
    if (e != hipSuccess) return fail(TG_E_HIP, std::string("heat setup failed: ") + hipGetErrorString(e));
    int64_t it = 0;
    double worst = 0.0;
    for (int32_t k = 0; k < nsteps; ++k) {
        e = tg::launch_spmv(*p, dtype, ws + o_m, states + (size_t)k * n * elt, ws + o_rhs, s);
        if (e != hipSuccess) return fail(TG_E_HIP, std::string("spmv launch failed: ") + hipGetErrorString(e));
        // u^k starts the solve for u^{k+1}
        st = heat_solve(p, dtype, ws + o_a, ws + o_rhs, states + (size_t)(k + 1) * n * elt,
                        states + (size_t)k * n * elt, rtol, max_iter, check_every, it, worst, s);
        if (st != TG_OK) break;
    }
    if (iters) *iters = it;
    if (relres) *relres = worst;
    return st == TG_OK ? ok() : st;
}

tg_status tg_heat_adjoint(const tg_pattern *p, tg_dtype dtype, const double *d_coords, const double *d_log_a,
                          double dt, int32_t nsteps, const void *d_states, const void *d_g, double *d_dlog_a,
                          double *d_dcoords, void *d_du0, double rtol, int32_t max_iter, int32_t check_every,
                          int64_t *iters, double *relres, int32_t *d_status, void *stream) {
    tg_status st = check_heat(p, dtype, d_coords, d_log_a, dt, nsteps, rtol, max_iter, check_every);
    if (st != TG_OK) return st;
    if (!d_states || !d_g) return fail(TG_E_ARG, "d_states and d_g are required");
    if (!d_dlog_a && !d_dcoords && !d_du0) return fail(TG_E_ARG, "no output requested");
    const tg::HostPattern &h = p->host;
    const size_t elt = dtype == TG_F64 ? 8 : 4, n = (size_t)h.n_dofs;
    const hipStream_t s = (hipStream_t)stream;
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    if (nsteps == 0) {  // u^N = u^0: the gradient is g itself
        hipError_t e = hipSuccess;
        if (d_dlog_a && h.E) e = hipMemsetAsync(d_dlog_a, 0, h.E * sizeof(double), s);
        if (e == hipSuccess && d_dcoords && h.nv) e = hipMemsetAsync(d_dcoords, 0, h.nv * h.dim * sizeof(double), s);
        if (e == hipSuccess && d_du0) e = hipMemcpyAsync(d_du0, d_g, n * elt, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(TG_E_HIP, std::string("copy failed: ") + hipGetErrorString(e));
        return ok();
    }
    Carve cv;
    const size_t o_coef = cv.take(h.E * elt), o_m = cv.take(h.nnz * elt), o_a = cv.take(h.nnz * elt),
                 o_rhs = cv.take(n * elt), o_lam = cv.take((size_t)nsteps * n * elt),
                 o_scr = cv.take((size_t)h.E * h.k * h.dim * sizeof(double));
    st = ensure_workspace(p, cv.off);
    if (st != TG_OK) return st;
    char *ws = (char *)p->dev.ws;
    char *lam = ws + o_lam;  // lam[k] holds lambda^{k+1}
    hipError_t e = heat_matrices(p, dtype, d_coords, d_log_a, dt, ws + o_coef, ws + o_m, ws + o_a, d_status, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + o_rhs, d_g, n * elt, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return fail(TG_E_HIP, std::string("heat setup failed: ") + hipGetErrorString(e));
    int64_t it = 0;
    double worst = 0.0;
    // A lambda^N = g;  A lambda^k = M lambda^{k+1}  (A and M symmetric)
    st = heat_solve(p, dtype, ws + o_a, ws + o_rhs, lam + (size_t)(nsteps - 1) * n * elt, nullptr, rtol, max_iter,
                    check_every, it, worst, s);
    for (int32_t k = nsteps - 1; st == TG_OK && k >= 1; --k) {
        e = tg::launch_spmv(*p, dtype, ws + o_m, lam + (size_t)k * n * elt, ws + o_rhs, s);
        if (e != hipSuccess) {
            st = fail(TG_E_HIP, std::string("spmv launch failed: ") + hipGetErrorString(e));
            break;
        }
        // lambda^{k+1} starts the solve for lambda^k
        st = heat_solve(p, dtype, ws + o_a, ws + o_rhs, lam + (size_t)(k - 1) * n * elt, lam + (size_t)k * n * elt,
                        rtol, max_iter, check_every, it, worst, s);
    }
    if (iters) *iters = it;
    if (relres) *relres = worst;
    if (st != TG_OK) return st;
    // dL/dtheta = -sum_k dPhi_k/dtheta with Phi_k = lambda^k^T (A u^k - M u^{k-1})
    if (d_dlog_a || d_dcoords) {
        e = tg::launch_adjoint_p1(*p, TG_MASS_LAPLACE, dtype, nsteps, d_coords, ws + o_coef, lam,
                                  (const char *)d_states + n * elt, d_states, (int64_t)n, -1.0, d_dlog_a, d_dcoords,
                                  (double *)(ws + o_scr), d_status, s);
        if (e != hipSuccess) return fail(TG_E_HIP, std::string("adjoint launch failed: ") + hipGetErrorString(e));
    }
    if (d_du0) {  // dL/du^0 = M lambda^1
        e = tg::launch_spmv(*p, dtype, ws + o_m, lam, d_du0, s);
        if (e != hipSuccess) return fail(TG_E_HIP, std::string("spmv launch failed: ") + hipGetErrorString(e));
    }
    return ok();
}

}  // extern "C"
