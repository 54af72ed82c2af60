// C ABI of libtg (declared in include/tg.h): argument checks, device upload
// of the pattern, and dispatch to the kernels.  Nothing here throws across
// the ABI: every entry point catches and converts to a tg_status.
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
    void *ptrs[] = {d.conn,    d.inc_ptr, d.inc,      d.blk_row,     d.blk_desc, d.node_rp, d.node_ci, d.seg_ptr,
                    d.slot,    d.row_ptr, d.col_idx,  d.diag_pos,    d.constrained,
                    d.work,    d.partials, d.state, d.dir_rows};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (d.host_state) (void)hipHostFree(d.host_state);
    d = tg::DevicePattern{};
}

tg_status create_device(tg_pattern &pt) {
    using namespace tg;
    const HostPattern &h = pt.host;
    DevicePattern &d = pt.dev;
    size_t bytes = 0;
    hipError_t e = hipGetDevice(&pt.device);
#define TG_UP(vec, field) \
    if (e == hipSuccess) e = upload(h.vec, &d.field, bytes)
    TG_UP(conn, conn);
    TG_UP(inc_ptr, inc_ptr);
    TG_UP(inc, inc);
    TG_UP(blk_row, blk_row);
    TG_UP(blk_desc, blk_desc);
    TG_UP(node_rp, node_rp);
    TG_UP(node_ci, node_ci);
    TG_UP(seg_ptr, seg_ptr);
    TG_UP(slot, slot);
    TG_UP(row_ptr, row_ptr);
    TG_UP(col_idx, col_idx);
    TG_UP(diag_pos, diag_pos);
    TG_UP(constrained, constrained);
    TG_UP(dirichlet_rows, dir_rows);
#undef TG_UP
    d.n_dir_rows = (int64_t)h.dirichlet_rows.size();
    if (e == hipSuccess) {
        const size_t wb = 6 * (size_t)h.n_dofs * sizeof(double);
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
    if (e == hipSuccess) e = hipHostMalloc((void **)&d.host_state, sizeof(PcgState), hipHostMallocDefault);
    if (e != hipSuccess) {
        const tg_status st = (e == hipErrorOutOfMemory) ? TG_E_NOMEM : TG_E_HIP;
        const std::string msg = std::string("device setup of the pattern failed: ") + hipGetErrorString(e);
        free_device(d);
        return fail(st, msg);
    }
    d.bytes = bytes;
    // lanes per row in the SpMV: about half the mean row length, power of two in [4, 32]
    const double mean_row = h.n_dofs ? (double)h.nnz / (double)h.n_dofs : 1.0;
    int g = 4;
    while (g < 32 && g < mean_row / 2) g *= 2;
    d.spmv_group = g;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, pt.device) == hipSuccess && prop.multiProcessorCount > 0)
        d.n_cu = prop.multiProcessorCount;
    return TG_OK;
}

bool valid_dtype(tg_dtype t) { return t == TG_F64 || t == TG_F32; }

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
    info->device_bytes = p->dev.bytes;
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

void tg_pattern_destroy(tg_pattern *p) {
    if (!p) return;
    if (!p->host_only) free_device(p->dev);
    delete p;
}

static tg_status assemble_impl(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch,
                               const double *d_coords, const void *d_coef, const void *d_load, void *d_values,
                               void *d_rhs, int32_t *d_status, void *stream) {
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
    hipError_t e;
    if (form == TG_LAPLACE || form == TG_MASS || form == TG_MASS_LAPLACE) {
        if (!scalar_p1) return fail(TG_E_ARG, "LAPLACE, MASS and MASS_LAPLACE need a P1 scalar pattern (order 1, ncomp 1)");
        if (form != TG_MASS && !d_coef) return fail(TG_E_ARG, "this form needs d_coef");
        if (form == TG_MASS && nbatch != 1) return fail(TG_E_ARG, "MASS has no coefficients to batch");
        e = tg::launch_assemble_p1(*p, form, dtype, nbatch, d_coords, d_coef, form == TG_MASS ? nullptr : d_load,
                                   d_values, d_rhs, d_status, (hipStream_t)stream);
    } else if (form == TG_ELASTICITY) {
        if (h.order != 2 || h.ncomp != 3) return fail(TG_E_ARG, "ELASTICITY needs a P2 vector pattern (3, 2, 3)");
        if (!d_coef) return fail(TG_E_ARG, "ELASTICITY needs d_coef (lambda, mu)");
        if (nbatch != 1) return fail(TG_E_ARG, "batched ELASTICITY is not supported");
        e = tg::launch_assemble_p2(*p, dtype, d_coords, d_coef, d_load, d_values, d_rhs, d_status,
                                   (hipStream_t)stream);
    } else {
        return fail(TG_E_ARG, "invalid form");
    }
    if (e != hipSuccess) return fail(TG_E_HIP, std::string("assembly launch failed: ") + hipGetErrorString(e));
    return ok();
}

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
    if (!d_values) return fail(TG_E_ARG, "d_values is required");
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
