// Internal declarations of libtg (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "tg.h"

namespace tg {

// Row-block capacities of the fused Map+Reduce kernels, in (node, element)
// pairs.  A block is a run of consecutive node rows whose pairs all fit in
// LDS; the greedy partition fills a block up to the target and a single row
// may use up to the capacity.
constexpr int kP1Threads = 256;
constexpr int kP1BlockTarget = 256;
constexpr int kP1BlockCap = 512;
constexpr int kP1BlockVerts = 256;  // distinct vertices of a block (8-bit local ids)
constexpr int kP2Threads = 192;  // three waves: one per set of column nodes
// P2: one lane per pair in each wave, so at most 64 pairs; the target keeps an
// FP64 block's LDS (about 0.55 KB per pair) within a fifth of the CU's 160 KB,
// as many blocks as the FP64 kernel's registers allow (measured at 32^3: 48
// pairs FP64 as fast as 52, FP32 5% faster; 56 slower in both).
constexpr int kP2BlockTarget = 48;
constexpr int kP2BlockCap = 64;
constexpr int kBlkDesc = 12;  // ints per row-block descriptor
constexpr int kSellRows = 64;  // rows per slice of the sliced-ELL pattern: one per lane of a wave
// Largest pair count of a row for the compact P1 routing: its one-byte
// row-relative slot codes (pair offset * k + b) stay below 256.
constexpr int compact_row_pairs(int k) { return 256 / k; }

// Host-side topology of one mesh: numbering, node-level CSR and the routing
// of element slots to CSR entries.
struct HostPattern {
    int dim = 0, order = 0, ncomp = 0, k = 0;  // k = nodes per element
    int64_t nv = 0, E = 0, n_nodes = 0, n_dofs = 0;
    int64_t nnz_nodes = 0;  // node-level entries (node pairs sharing an element)
    int64_t nnz = 0;        // scalar entries = ncomp^2 * nnz_nodes

    std::vector<int32_t> conn;        // [E][dim+1] vertex ids (as given)
    std::vector<int32_t> elem_nodes;  // [E][k] global node ids
    std::vector<int32_t> node_rp;     // [n_nodes+1] node-level CSR rows
    std::vector<int32_t> node_ci;     // [nnz_nodes] node-level CSR columns (sorted)
    // P2: node_vp[i] = vertex-node columns in rows 0 .. i-1 (a row's vertex-node
    // columns come first: vertices are numbered before edges).  Empty for P1.
    std::vector<int32_t> node_vp;     // [n_nodes+1]
    // S_vec routing: pairs (node i, element e, local node a) grouped by node,
    // ascending e inside a node.  pair code = e * k + a.
    std::vector<int32_t> inc_ptr;  // [n_nodes+1]
    std::vector<int32_t> inc;      // [n_pairs]
    // Row blocks for the fused kernels.
    std::vector<int32_t> blk_row;   // [n_blocks+1]
    // [n_blocks][kBlkDesc]: r0, r1, q0, q1, v0, v1, w0, w1, s0, s1, c0, c1 (rows, pairs,
    // node entries, vertices, routing slots; P2: node_vp[r0], node_vp[r1], else 0)
    std::vector<int32_t> blk_desc;
    // The distinct vertices of each block's elements (ascending), and per pair
    // the block-local ids of its element's vertices, one byte each in local
    // vertex order (P2: in the pair's frame) (the Map reads coordinates from a
    // per-block LDS copy).
    std::vector<int32_t> blk_vert;  // [sum of block vertex counts]
    std::vector<uint32_t> pair_lv;  // [n_pairs]
    // S_mat routing: node-level entry p sums slots slot[seg_ptr[p] .. seg_ptr[p+1]),
    // ascending element order; slot = b * (pairs of the block) + (pair - first pair of the block),
    // b the column's local node (P2: in the pair's frame, tg_pattern.cpp p2_frame_order).
    // Diagonal entries have empty segments (the kernels sum them from the row's pairs).
    // P1: the diagonal entry of a row has an empty segment; its value is the sum over
    // the row's pairs (S_vec order) of the element's diagonal entry K_e[a][a].
    std::vector<int32_t> seg_ptr;  // [nnz_nodes+1]
    std::vector<uint16_t> slot;    // [seg_ptr[nnz_nodes]] rounded up to a multiple of 4
    // Compact form of the same P1 routing (used by the kernel when every row has at
    // most compact_row_pairs(k) pairs and every block at most 255 rows): the slots of
    // row i are slot8[inc_ptr[i] (k-1) ...], one byte each, coded (pair - inc_ptr[i]) k + b;
    // entry z of row i (block-local row r) is ent16[z] = r << 8 | (seg_ptr[z] - inc_ptr[i] (k-1)).
    bool compact = false;
    std::vector<uint16_t> ent16;  // [nnz_nodes]
    std::vector<uint8_t> slot8;   // [n_pairs (k-1)] rounded up to a multiple of 4
    // Scalar CSR (DoF = ncomp * node + c).
    std::vector<int32_t> row_ptr;   // [n_dofs+1]
    std::vector<int32_t> col_idx;   // [nnz]
    std::vector<int32_t> diag_pos;  // [n_dofs]
    // Sliced-ELL copy of the scalar pattern (the CG iterations' SpMV): slices of
    // kSellRows consecutive rows, entry k of row r at sell_ptr[r / kSellRows] +
    // kSellRows k + r % kSellRows; padding entries name the row itself (rows past
    // the last DoF: the last DoF), value 0.  When every column lies within 32767
    // of its row's clamped index min(r, n_dofs - 1), the columns are kept as
    // 16-bit offsets from it (sell_off) and sell_col is empty.
    std::vector<int32_t> sell_ptr;  // [n_slices+1]
    std::vector<int32_t> sell_col;  // [sell_ptr[n_slices]] or empty
    std::vector<int16_t> sell_off;  // [sell_ptr[n_slices]] or empty
    // > 0 when every slice is padded to this many entries per row (sell_ptr[s] =
    // 64 s sell_len): the CG iteration then locates a slice without reading sell_ptr
    int32_t sell_len = 0;
    // Dirichlet.
    std::vector<uint8_t> constrained;  // [n_dofs] 0/1
    std::vector<int32_t> constrained_list;
    std::vector<int32_t> dirichlet_rows;  // rows touched by the elimination, ascending

    // Largest row block, for sizing the kernels' LDS.
    int32_t max_block_pairs = 0;
    int32_t max_block_entries = 0;  // node-level CSR entries
    int32_t max_block_verts = 0;    // distinct vertices
    int32_t max_block_rows = 0;

    int64_t n_pairs() const { return (int64_t)inc.size(); }
    int64_t n_blocks() const { return (int64_t)blk_row.size() - 1; }
};

// Builds everything above; returns TG_OK or an error with *msg set.
tg_status build_host_pattern(int dim, int order, int ncomp, int64_t nv, int64_t E, const int32_t *conn,
                             const int32_t *dirichlet, int64_t n_dirichlet, HostPattern &hp, std::string &msg);

// PCG device state (one per system).
struct PcgState {
    double bb;        // b.b
    double rr;        // true residual r.r after the final check
    double tol2;      // rtol^2 * b.b
    int32_t done;     // 1 once the stop test held
    int32_t iters;    // iteration at which it held
    double alpha[2];  // step length of iteration i, kept at [i & 1] for iteration i + 1
    double gamma[2];  // r.u of iteration i, kept at [i & 1]
};

// One CG system in flight.  The solo solver (tg_pcg) uses one; the request
// server one per slot.  Lives in device memory; the kernels of a batched
// launch read slots[list[blockIdx.y]] (the solo iteration kernel takes it by
// value).
struct PcgSlot {
    const void *values;  // T[nnz], Dirichlet applied
    const void *sell;    // T[sell_nnz]: the same values in the sliced-ELL layout (the iterations' SpMV)
    const void *b;       // T[n]
    void *x;             // T[n], the iterate (output)
    void *work;          // T[kPcgWorkVectors n]: records {u, w/K_ii, s/K_ii} x 2 (by parity), p, 1/K_ii
    double *partials;    // [kNumPartials][kMaxGrid]
    PcgState *state;
    double rtol2;
    int32_t start;       // launch step of this system's iteration 0 (iteration = step - start)
    int32_t max_iter;    // no update past this iteration (the stop test still runs there)
    int32_t warm = 0;    // 1: x holds the initial guess and the stop test is relative to ||b||
};

constexpr int kVecThreads = 1024;  // threads per block of the PCG setup and residual kernels
constexpr int kMaxGrid = 2048;       // partial sums per kind: the CG iteration kernel's block cap
constexpr int kSetupMaxGrid = 1024;  // blocks of the PCG setup and residual kernels (grid-stride beyond)
// Threads per block of the CG iteration kernel: 4 slices in FP64, whose 1000+
// blocks on a 64^3 mesh then spread more evenly over the 256 CUs, 8 in FP32,
// where the wider block measured faster.
template <typename T>
constexpr int iter_threads() {
    return sizeof(T) == 8 ? 256 : 512;
}
constexpr int kFillThreads = 512;  // threads per block of the sliced-ELL fill: 8 slices
// Per-block partial sums of the PCG kernels, kMaxGrid doubles each: r.u, w.u and r.r
// of an iterate at kGam/kDel/kRr + 3 (iteration & 1), and the true residual at kResid.
constexpr int kGam = 0, kDel = 1, kRr = 2, kResid = 6, kNumPartials = 7;
// Krylov workspace of one system, in vectors of n values of the dtype: two
// records of 3 values per row (by iteration parity), p and the Jacobi factor.
constexpr int kPcgWorkVectors = 8;

struct DevicePattern {
    int32_t *conn = nullptr;      // [E][dim+1]
    int32_t *inc_ptr = nullptr;   // [n_nodes+1]
    int32_t *inc = nullptr;       // [n_pairs]
    int32_t *blk_row = nullptr;   // [n_blocks+1]
    int32_t *blk_desc = nullptr;  // [n_blocks][kBlkDesc]
    int32_t *blk_vert = nullptr;  // block vertex lists
    uint32_t *pair_lv = nullptr;  // [n_pairs] packed block-local vertex ids
    int32_t *node_rp = nullptr;   // [n_nodes+1]
    int32_t *node_ci = nullptr;   // [nnz_nodes]
    int32_t *node_vp = nullptr;   // [n_nodes+1] (P2)
    int32_t *seg_ptr = nullptr;   // [nnz_nodes+1]
    uint16_t *slot = nullptr;     // [n_pairs*k]
    uint16_t *ent16 = nullptr;    // compact P1 routing (HostPattern::compact)
    uint8_t *slot8 = nullptr;
    int32_t *row_ptr = nullptr;   // [n_dofs+1]
    int32_t *col_idx = nullptr;   // [nnz]
    int32_t *diag_pos = nullptr;  // [n_dofs]
    uint8_t *constrained = nullptr;  // [n_dofs]
    int32_t *sell_ptr = nullptr;     // [n_slices+1] sliced-ELL pattern (HostPattern::sell_ptr)
    int32_t *sell_col = nullptr;     // [sell_nnz] 32-bit columns, or
    int16_t *sell_off = nullptr;     // [sell_nnz] 16-bit offsets from the row (sell16)
    bool sell16 = false;
    int sell_len = 0;                // HostPattern::sell_len
    int64_t n_slices = 0, sell_nnz = 0;
    double *sell_vals = nullptr;     // the solo solver's sliced-ELL copy of the values (sell_nnz, used as T)
    // PCG workspace: kPcgWorkVectors vectors of n_dofs doubles (used as T), partials, state.
    double *work = nullptr;
    double *partials = nullptr;  // [kNumPartials][kMaxGrid]
    int32_t *dir_rows = nullptr; // rows that are constrained or have a constrained column
    int64_t n_dir_rows = 0;
    PcgState *state = nullptr;
    PcgState *host_state = nullptr;  // pinned mirrors [2] (the solver polls one while the other fills)
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    PcgSlot *pcg_slot = nullptr;       // the solo solver's slot (device) ...
    PcgSlot *host_pcg_slot = nullptr;  // ... and its pinned staging copy
    int32_t *pcg_list = nullptr;       // device {0}
    size_t bytes = 0;
    // Scratch for the adjoint and the heat rollout, grown on demand (ensure_workspace).
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int spmv_group = 4;  // lanes per CSR row in the SpMV
    int n_cu = 1;        // compute units of the pattern's device (persistent grids)
};

}  // namespace tg

struct tg_pattern {
    tg::HostPattern host;
    tg::DevicePattern dev;
    bool host_only = false;
    int device = -1;
};

// Kernel launchers (tg_assemble.hip, tg_solve.hip).  They return hipError_t.
namespace tg {
hipError_t launch_assemble_p1(const tg_pattern &p, tg_form form, tg_dtype dtype, int nbatch, const double *coords,
                              const void *coef, const void *load, void *values, void *rhs, int32_t *status,
                              hipStream_t s);
hipError_t launch_assemble_p2(const tg_pattern &p, tg_dtype dtype, const double *coords, const void *coef,
                              const void *load, void *values, void *rhs, int32_t *status, hipStream_t s);
hipError_t launch_dirichlet(const tg_pattern &p, tg_dtype dtype, void *values, void *rhs, const void *g,
                            hipStream_t s);
hipError_t launch_spmv(const tg_pattern &p, tg_dtype dtype, const void *values, const void *x, void *y,
                       hipStream_t s);
// The sliced-ELL copy of CSR values (both of dtype) for the CG iterations.
hipError_t launch_sell_fill(const tg_pattern &p, tg_dtype dtype, const void *values, void *sell, hipStream_t s);
// Adjoint of P1 assembly (tg_adjoint.hip): dlogc [E] (may be NULL) and dcoords [nv][dim]
// (may be NULL) of scale * sum_m lam_m^T (A u_m - M w_m); stage holds E*(dim+1)*dim doubles.
hipError_t launch_adjoint_p1(const tg_pattern &p, tg_form form, tg_dtype dtype, int nbatch, const double *coords,
                             const void *coef, const void *lam, const void *u, const void *w, int64_t stride,
                             double scale, double *dlogc, double *dcoords, double *stage, int32_t *status,
                             hipStream_t s);
// The allocation-free adjoint entry point's staging array: kNoAllocStageDoubles
// doubles per GPU (32 MiB), its address on the current device.
constexpr size_t kNoAllocStageDoubles = size_t(1) << 22;
constexpr int kNoAllocMaxDevices = 64;
hipError_t noalloc_stage(double **out);
// y[i] = dt * exp(x[i]) in dtype (FP64 input).
hipError_t launch_scaled_exp(tg_dtype dtype, int64_t n, double dt, const double *x, void *y, hipStream_t s);
// Batched PCG over the slots listed in `list` (device int32[count]); every slot
// holds a system on pattern p in dtype.  One launch per iteration (tg_solve.hip).
hipError_t launch_pcg_init(const tg_pattern &p, tg_dtype dtype, const PcgSlot *slots, const int32_t *list, int count,
                           hipStream_t s);
// Warm start of the listed slots from their x (which holds the initial guess):
// r = b - K x, p = s = 0, w = K u, and the stop test relative to ||b||.
hipError_t launch_pcg_warm_init(const tg_pattern &p, tg_dtype dtype, const PcgSlot *slots, const int32_t *list,
                                int count, hipStream_t s);
// With solo (a host copy of the one slot of a solo solve), the iteration kernel
// takes the slot by value and slots/list are not read.
hipError_t launch_pcg_step(const tg_pattern &p, tg_dtype dtype, const PcgSlot *slots, const int32_t *list, int count,
                           int step, hipStream_t s, const PcgSlot *solo = nullptr);
// Per-block partials of ||b - K x||^2 into each listed slot's RR partials; returns the block count.
hipError_t launch_pcg_residual(const tg_pattern &p, tg_dtype dtype, const PcgSlot *slots, const int32_t *list,
                               int count, int *n_partials, hipStream_t s);
// Device bytes a host-only pattern takes once uploaded (arrays and PCG
// workspace, as tg_pattern_create allocates them), and its upload (the
// request server builds patterns on the host first and uploads them when
// they fit its budget).
size_t device_bytes(const HostPattern &h);
tg_status upload_pattern(tg_pattern *p);
// ABI helpers shared by the entry-point files (tg_api.cpp): the thread's last
// error message, pattern and argument checks, and the assembly dispatch.
tg_status api_fail(tg_status st, const std::string &msg);
tg_status api_ok();
tg_status api_check_pattern(const tg_pattern *p);
tg_status validate_assemble(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch, const double *d_coords,
                            const void *d_coef, const void *d_values);
hipError_t launch_assemble(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch, const double *d_coords,
                           const void *d_coef, const void *d_load, void *d_values, void *d_rhs, int32_t *d_status,
                           hipStream_t s);
// How a CG run ends.  A run stops on the recursive residual (||r_k|| <= rtol
// ||b||); then the true relative residual ||b - K x|| / ||b|| is checked.  Above
// rtol, the run is restarted from its x (residual replacement) while iterations
// remain, at most kPcgRestarts times, and only while each restart at least
// halves the true residual: when it does not, rtol is below what the dtype
// can reach (in FP32 the rounding of x alone leaves a relative residual of
// about 1e-7 to 1e-5 on Poisson and heat systems) and the run ends with
// kAccuracy.  The solo solver and the request server take the same decisions.
constexpr int kPcgRestarts = 4;
enum class RunEnd { kOk, kRestart, kNoConv, kAccuracy, kNonFinite };
RunEnd run_end(bool done, double relres, double prev_relres, double rtol, bool nonfinite, int run, int total,
               int max_iter);
bool state_finite(const PcgState &st);  // every scalar of the state is finite
// Runs the whole PCG; returns TG_OK / TG_E_NOCONV / TG_E_ACCURACY / TG_E_NONFINITE / TG_E_HIP with *msg
// on failure.  warm: x holds the initial guess (else x0 = 0); the stop test is ||r|| <= rtol ||b|| either
// way.  strict: check the true residual and restart as run_end says; otherwise one run, stopped on the
// recursive residual (relres still reports the true one).
tg_status run_pcg(const tg_pattern &p, tg_dtype dtype, const void *values, const void *rhs, void *x, double rtol,
                  int32_t max_iter, int32_t check_every, int32_t *iters, double *relres, hipStream_t s,
                  std::string &msg, bool warm = false, bool strict = true);
}  // namespace tg
