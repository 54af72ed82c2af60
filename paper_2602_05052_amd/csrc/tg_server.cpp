// Request server: continuous batching of assemble + Dirichlet + PCG requests
// with iteration-level scheduling.
//
// The paper generates data in batches (SM B.1.4, efficient batch data
// generation); a stream of independent solves is served here the way LLM
// servers batch token generation.  Requests are grouped by (pattern, dtype).
// Each group owns slots: per-slot device buffers (values, rhs, Krylov
// workspace, partial sums, state) that live as long as the server.  Between
// CG iterations the scheduler retires finished systems and admits queued
// requests into the freed slots (their assembly, Dirichlet elimination and CG
// initialisation run then); every iteration is one launch over all active
// slots of a group (blockIdx.y = slot).
// The per-slot reductions never mix: a slot's scalars come from its own
// partials in the same fixed order as a solo tg_pcg on the same kernels, so a
// request's solution is bitwise the same whether it ran alone or in a mix.
//
// Admission: a request enters when its group has a free slot, or when one more
// slot fits in the server's HBM budget and under the per-group slot limit.
//
// Each group runs on a stream of its own (default priority), forked from the
// caller's stream at the start of a scheduling round and joined back before
// the round's synchronisation, so the launches of groups on different patterns
// (often small, latency-bound systems) overlap on the GPU.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <memory>
#include <vector>

#include "tg_internal.h"

namespace {

using tg::PcgSlot;
using tg::PcgState;

struct Request {
    int64_t id;
    const tg_pattern *p;
    tg_form form;
    tg_dtype dtype;
    const double *coords;
    const void *coef, *load, *g;
    void *x;
    double rtol;
    int32_t max_iter;
    double t_submit;
};

struct SlotMem {
    void *values = nullptr, *sell = nullptr, *b = nullptr, *work = nullptr;
    double *partials = nullptr;
};

struct Group {
    const tg_pattern *p = nullptr;
    tg_dtype dtype = TG_F64;
    int max_slots = 0;
    std::vector<SlotMem> mem;      // allocated slots
    std::vector<int> busy;         // 1 while a request occupies the slot
    std::vector<Request> req;      // request per slot
    std::vector<int> active;       // slot ids in the batch, admission order
    // device tables (max_slots entries) and their pinned staging copies
    PcgSlot *d_slots = nullptr, *h_slots = nullptr;
    PcgState *d_states = nullptr, *h_states = nullptr;
    int32_t *d_status = nullptr, *h_status = nullptr;
    int32_t *d_lists = nullptr, *h_lists = nullptr;  // [active | fresh | finished], max_slots each
    int step = 0;
    size_t slot_bytes = 0;
    hipStream_t stream = nullptr;  // the group's own stream
    hipEvent_t joined = nullptr;   // recorded on it at the end of a round
    // retirement in flight between the launch and the finish phase of a round
    std::vector<int> fin, keep;
    std::vector<double> parts;
    int n_parts = 0;
};

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct tg_server {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr;  // recorded on `stream` at the start of a round
    size_t budget = 0, used = 0;
    int max_slots = 1;
    int check_every = 1;
    int64_t next_id = 1;
    double t0 = 0.0;
    std::deque<Request> queue;
    std::vector<std::unique_ptr<Group>> groups;
    std::deque<tg_server_result> done;
};

namespace {

const size_t kPartialBytes = (size_t)tg::kNumPartials * tg::kMaxGrid * sizeof(double);

size_t slot_bytes(const tg_pattern *p, tg_dtype dtype) {
    const size_t elt = dtype == TG_F64 ? 8 : 4, n = (size_t)p->host.n_dofs;
    return ((size_t)p->host.nnz + (size_t)p->dev.sell_nnz + (1 + tg::kPcgWorkVectors) * n) * elt + kPartialBytes;
}

void free_group(Group &g) {
    for (SlotMem &m : g.mem) {
        (void)hipFree(m.values);
        (void)hipFree(m.sell);
        (void)hipFree(m.b);
        (void)hipFree(m.work);
        (void)hipFree(m.partials);
    }
    (void)hipFree(g.d_slots);
    (void)hipFree(g.d_states);
    (void)hipFree(g.d_status);
    (void)hipFree(g.d_lists);
    (void)hipHostFree(g.h_slots);
    (void)hipHostFree(g.h_states);
    (void)hipHostFree(g.h_status);
    (void)hipHostFree(g.h_lists);
    if (g.joined) (void)hipEventDestroy(g.joined);
    if (g.stream) (void)hipStreamDestroy(g.stream);
}

tg_status hip_fail(hipError_t e, const char *what) {
    return tg::api_fail(e == hipErrorOutOfMemory ? TG_E_NOMEM : TG_E_HIP,
                        std::string(what) + ": " + hipGetErrorString(e));
}

Group *find_group(tg_server *srv, const tg_pattern *p, tg_dtype dtype) {
    for (auto &g : srv->groups)
        if (g->p == p && g->dtype == dtype) return g.get();
    return nullptr;
}

tg_status make_group(tg_server *srv, const tg_pattern *p, tg_dtype dtype, Group **out) {
    auto g = std::make_unique<Group>();
    g->p = p;
    g->dtype = dtype;
    g->max_slots = srv->max_slots;
    const size_t S = (size_t)srv->max_slots;
    g->slot_bytes = slot_bytes(p, dtype);
    const size_t table = S * (sizeof(PcgSlot) + sizeof(PcgState) + 4 * sizeof(int32_t));
    hipError_t e = hipMalloc((void **)&g->d_slots, S * sizeof(PcgSlot));
    if (e == hipSuccess) e = hipMalloc((void **)&g->d_states, S * sizeof(PcgState));
    if (e == hipSuccess) e = hipMalloc((void **)&g->d_status, S * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&g->d_lists, 3 * S * sizeof(int32_t));
    if (e == hipSuccess) e = hipHostMalloc((void **)&g->h_slots, S * sizeof(PcgSlot), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&g->h_states, S * sizeof(PcgState), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&g->h_status, S * sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&g->h_lists, 3 * S * sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->joined, hipEventDisableTiming);
    if (e != hipSuccess) {
        free_group(*g);
        return hip_fail(e, "server group allocation failed");
    }
    srv->used += table;
    *out = g.get();
    srv->groups.push_back(std::move(g));
    return TG_OK;
}

// A free slot of g, allocating one within the budget; -1 if none.
int take_slot(tg_server *srv, Group &g, tg_status &st) {
    st = TG_OK;
    for (size_t i = 0; i < g.mem.size(); ++i)
        if (!g.busy[i]) return (int)i;
    if ((int)g.mem.size() >= g.max_slots || srv->used + g.slot_bytes > srv->budget) return -1;
    const size_t elt = g.dtype == TG_F64 ? 8 : 4, n = (size_t)g.p->host.n_dofs;
    SlotMem m;
    hipError_t e = hipMalloc(&m.values, std::max<size_t>(1, g.p->host.nnz) * elt);
    if (e == hipSuccess) e = hipMalloc(&m.sell, std::max<size_t>(1, (size_t)g.p->dev.sell_nnz) * elt);
    if (e == hipSuccess) e = hipMalloc(&m.b, std::max<size_t>(1, n) * elt);
    if (e == hipSuccess) e = hipMalloc(&m.work, std::max<size_t>(1, tg::kPcgWorkVectors * n) * elt);
    if (e == hipSuccess) e = hipMalloc((void **)&m.partials, kPartialBytes);
    if (e != hipSuccess) {
        (void)hipFree(m.values);
        (void)hipFree(m.sell);
        (void)hipFree(m.b);
        (void)hipFree(m.work);
        (void)hipFree(m.partials);
        st = hip_fail(e, "server slot allocation failed");
        return -1;
    }
    srv->used += g.slot_bytes;
    g.mem.push_back(m);
    g.busy.push_back(0);
    g.req.emplace_back();
    return (int)g.mem.size() - 1;
}

void finish(tg_server *srv, const Request &r, tg_status status, int32_t iters, double relres, int32_t bad) {
    tg_server_result res;
    res.request_id = r.id;
    res.status = status;
    res.iters = iters;
    res.relres = relres;
    res.bad_element = bad;
    res.t_submit = r.t_submit - srv->t0;
    res.t_done = now_s() - srv->t0;
    srv->done.push_back(res);
}

// Admit queued requests of group g into free slots; returns the fresh slot ids.
tg_status admit(tg_server *srv, Group &g, std::vector<int> &fresh) {
    tg_status st = TG_OK;
    for (auto it = srv->queue.begin(); it != srv->queue.end();) {
        if (it->p != g.p || it->dtype != g.dtype) {
            ++it;
            continue;
        }
        const int s = take_slot(srv, g, st);
        if (st != TG_OK) return st;
        if (s < 0) {
            if (g.active.empty() && fresh.empty() && g.mem.empty()) {  // can never run: budget too small
                finish(srv, *it, TG_E_NOMEM, 0, 0.0, -1);
                it = srv->queue.erase(it);
                continue;
            }
            break;  // FIFO within the group: wait for a slot
        }
        g.busy[s] = 1;
        g.req[s] = *it;
        const SlotMem &m = g.mem[s];
        g.h_slots[s] = PcgSlot{m.values, m.sell, m.b, it->x, m.work, m.partials, g.d_states + s, it->rtol * it->rtol,
                               g.step, it->max_iter};
        g.h_states[s] = PcgState{};  // all zero: not done, no iterations
        g.h_status[s] = TG_STATUS_CLEAN;
        fresh.push_back(s);
        it = srv->queue.erase(it);
    }
    if (fresh.empty()) return TG_OK;
    const hipStream_t str = g.stream;
    const int S = g.max_slots;
    for (int s : fresh) g.active.push_back(s);
    for (size_t i = 0; i < g.active.size(); ++i) g.h_lists[i] = g.active[i];
    for (size_t i = 0; i < fresh.size(); ++i) g.h_lists[S + i] = fresh[i];
    // Only the fresh slots' entries are written: the other slots' device state is live.
    hipError_t e = hipSuccess;
    for (int s : fresh) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(g.d_slots + s, g.h_slots + s, sizeof(PcgSlot), hipMemcpyHostToDevice, str);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g.d_states + s, g.h_states + s, sizeof(PcgState), hipMemcpyHostToDevice, str);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g.d_status + s, g.h_status + s, sizeof(int32_t), hipMemcpyHostToDevice, str);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(g.d_lists, g.h_lists, 2 * S * sizeof(int32_t), hipMemcpyHostToDevice, str);
    for (int s : fresh) {
        if (e != hipSuccess) break;
        const Request &r = g.req[s];
        const SlotMem &m = g.mem[s];
        e = tg::launch_assemble(r.p, r.form, r.dtype, 1, r.coords, r.coef, r.load, m.values, m.b, g.d_status + s, str);
        if (e == hipSuccess) e = tg::launch_dirichlet(*r.p, r.dtype, m.values, m.b, r.g, str);
        if (e == hipSuccess) e = tg::launch_sell_fill(*r.p, r.dtype, m.values, m.sell, str);
    }
    if (e == hipSuccess) e = tg::launch_pcg_init(*g.p, g.dtype, g.d_slots, g.d_lists + S, (int)fresh.size(), str);
    if (e != hipSuccess) return hip_fail(e, "server admission failed");
    return TG_OK;
}

// Retirement, phase 1 (states already copied to the host and synchronised):
// pick the finished systems of g and enqueue their true-residual partials and
// the new active list on the group's stream.
tg_status retire_launch(Group &g) {
    const int S = g.max_slots;
    g.fin.clear();
    g.keep.clear();
    g.n_parts = 0;
    for (int s : g.active) {
        const PcgState &st = g.h_states[s];
        const int it = g.step - g.h_slots[s].start;
        if (st.done || it > g.h_slots[s].max_iter) g.fin.push_back(s);
        else g.keep.push_back(s);
    }
    if (g.fin.empty()) return TG_OK;
    const hipStream_t str = g.stream;
    // The pinned lists are rewritten here only after a synchronisation, and the
    // copies below complete before the round's finish phase.
    for (size_t i = 0; i < g.keep.size(); ++i) g.h_lists[i] = g.keep[i];
    for (size_t i = 0; i < g.fin.size(); ++i) g.h_lists[2 * S + i] = g.fin[i];
    int ns = 0;
    hipError_t e = hipMemcpyAsync(g.d_lists + 2 * S, g.h_lists + 2 * S, g.fin.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, str);
    if (e == hipSuccess)
        e = tg::launch_pcg_residual(*g.p, g.dtype, g.d_slots, g.d_lists + 2 * S, (int)g.fin.size(), &ns, str);
    g.n_parts = ns;
    g.parts.assign(g.fin.size() * (size_t)std::max(ns, 1), 0.0);
    for (size_t i = 0; i < g.fin.size() && e == hipSuccess; ++i)
        e = hipMemcpyAsync(g.parts.data() + i * ns, g.mem[g.fin[i]].partials + (size_t)tg::kResid * tg::kMaxGrid,
                           ns * sizeof(double), hipMemcpyDeviceToHost, str);
    if (e == hipSuccess && !g.keep.empty())
        e = hipMemcpyAsync(g.d_lists, g.h_lists, g.keep.size() * sizeof(int32_t), hipMemcpyHostToDevice, str);
    if (e != hipSuccess) return hip_fail(e, "server retirement failed");
    return TG_OK;
}

// Retirement, phase 2 (the group's stream synchronised): results of the finished systems.
void retire_finish(tg_server *srv, Group &g) {
    if (g.fin.empty()) return;
    const int ns = g.n_parts;
    for (size_t i = 0; i < g.fin.size(); ++i) {
        const int s = g.fin[i];
        const PcgState &st = g.h_states[s];
        double rr = 0.0;
        for (int k = 0; k < ns; ++k) rr += g.parts[i * ns + k];
        const double relres = st.bb > 0.0 ? std::sqrt(rr / st.bb) : std::sqrt(rr);
        tg_status status = st.done ? TG_OK : TG_E_NOCONV;
        int32_t bad = -1;
        if (g.h_status[s] != TG_STATUS_CLEAN) {
            status = TG_E_DEGENERATE;
            bad = g.h_status[s];
        }
        finish(srv, g.req[s], status, st.done ? st.iters : g.h_slots[s].max_iter, relres, bad);
        g.busy[s] = 0;
    }
    g.active = g.keep;
    g.fin.clear();
}

}  // namespace

extern "C" {

tg_status tg_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t check_every, void *stream,
                           tg_server **out) {
    if (!out) return tg::api_fail(TG_E_ARG, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 65535 || check_every < 1)
        return tg::api_fail(TG_E_ARG, "need 1 <= max_slots <= 65535 and check_every >= 1");
    tg_server *srv = new (std::nothrow) tg_server;
    if (!srv) return tg::api_fail(TG_E_NOMEM, "out of host memory");
    srv->stream = (hipStream_t)stream;
    if (hipEventCreateWithFlags(&srv->fork, hipEventDisableTiming) != hipSuccess) {
        delete srv;
        return tg::api_fail(TG_E_HIP, "server event creation failed");
    }
    srv->budget = hbm_budget_bytes;
    srv->max_slots = max_slots;
    srv->check_every = check_every;
    srv->t0 = now_s();
    *out = srv;
    return tg::api_ok();
}

tg_status tg_server_submit(tg_server *srv, const tg_pattern *p, tg_form form, tg_dtype dtype, const double *d_coords,
                           const void *d_coef, const void *d_load, const void *d_g, void *d_x, double rtol,
                           int32_t max_iter, int64_t *request_id) {
    if (!srv) return tg::api_fail(TG_E_ARG, "server is NULL");
    if (!d_x) return tg::api_fail(TG_E_ARG, "d_x is required");
    // d_values is checked as non-NULL: the slot provides it
    tg_status st = tg::validate_assemble(p, form, dtype, 1, d_coords, d_coef, (const void *)d_x);
    if (st != TG_OK) return st;
    if (form == TG_MASS) return tg::api_fail(TG_E_ARG, "MASS has no right-hand side to solve for");
    if (!d_load) return tg::api_fail(TG_E_ARG, "d_load is required (the right-hand side)");
    if (!(rtol > 0.0) || max_iter < 1) return tg::api_fail(TG_E_ARG, "need rtol > 0 and max_iter >= 1");
    if ((uint64_t)max_iter + 2 * (uint64_t)srv->check_every >= (uint64_t)1 << 30)
        return tg::api_fail(TG_E_ARG, "max_iter too large");
    Request r{srv->next_id++, p, form, dtype, d_coords, d_coef, d_load, d_g, d_x, rtol, max_iter, now_s()};
    srv->queue.push_back(r);
    if (request_id) *request_id = r.id;
    return tg::api_ok();
}

tg_status tg_server_step(tg_server *srv, int32_t *n_active, int32_t *n_queued) {
    if (!srv) return tg::api_fail(TG_E_ARG, "server is NULL");
    const hipStream_t str = srv->stream;
    // groups for queued requests
    for (const Request &r : srv->queue) {
        if (!find_group(srv, r.p, r.dtype)) {
            Group *g = nullptr;
            const tg_status st = make_group(srv, r.p, r.dtype, &g);
            if (st != TG_OK) return st;
        }
    }
    // fork: every group's stream starts after the work already on the caller's stream
    hipError_t e = hipEventRecord(srv->fork, str);
    if (e != hipSuccess) return hip_fail(e, "server fork failed");
    bool any = false;
    for (auto &gp : srv->groups) {
        Group &g = *gp;
        bool waits = false;
        for (const Request &r : srv->queue) waits = waits || (r.p == g.p && r.dtype == g.dtype);
        if (g.active.empty() && !waits) continue;
        e = hipStreamWaitEvent(g.stream, srv->fork, 0);
        if (e != hipSuccess) return hip_fail(e, "server fork failed");
        std::vector<int> fresh;
        tg_status st = admit(srv, g, fresh);
        if (st != TG_OK) return st;
        if (g.active.empty()) continue;
        any = true;
        for (int k = 0; k < srv->check_every; ++k) {
            e = tg::launch_pcg_step(*g.p, g.dtype, g.d_slots, g.d_lists, (int)g.active.size(), g.step, g.stream);
            if (e != hipSuccess) return hip_fail(e, "server iteration launch failed");
            ++g.step;
        }
        e = hipMemcpyAsync(g.h_states, g.d_states, g.mem.size() * sizeof(PcgState), hipMemcpyDeviceToHost,
                           g.stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g.h_status, g.d_status, g.mem.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                               g.stream);
        if (e == hipSuccess) e = hipEventRecord(g.joined, g.stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(str, g.joined, 0);  // join
        if (e != hipSuccess) return hip_fail(e, "server state copy failed");
    }
    if (any) {
        e = hipStreamSynchronize(str);
        if (e != hipSuccess) return hip_fail(e, "server synchronisation failed");
        bool retiring = false;
        for (auto &gp : srv->groups) {
            if (gp->active.empty()) continue;
            const tg_status st = retire_launch(*gp);
            if (st != TG_OK) return st;
            if (!gp->fin.empty()) {
                retiring = true;
                e = hipEventRecord(gp->joined, gp->stream);
                if (e == hipSuccess) e = hipStreamWaitEvent(str, gp->joined, 0);
                if (e != hipSuccess) return hip_fail(e, "server retirement failed");
            }
        }
        if (retiring) {
            e = hipStreamSynchronize(str);
            if (e != hipSuccess) return hip_fail(e, "server retirement failed");
            for (auto &gp : srv->groups) retire_finish(srv, *gp);
        }
    }
    int32_t act = 0;
    for (auto &gp : srv->groups) act += (int32_t)gp->active.size();
    if (n_active) *n_active = act;
    if (n_queued) *n_queued = (int32_t)srv->queue.size();
    return tg::api_ok();
}

tg_status tg_server_poll(tg_server *srv, int32_t max_results, tg_server_result *out, int32_t *n_out) {
    if (!srv || !n_out || (max_results > 0 && !out)) return tg::api_fail(TG_E_ARG, "NULL argument");
    int32_t k = 0;
    while (k < max_results && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    *n_out = k;
    return tg::api_ok();
}

tg_status tg_server_slot_bytes(const tg_pattern *p, tg_dtype dtype, size_t *bytes) {
    if (!p || !bytes) return tg::api_fail(TG_E_ARG, "NULL pattern or output");
    if (p->host_only) return tg::api_fail(TG_E_STATE, "pattern was created with TG_PATTERN_HOST_ONLY");
    if (dtype != TG_F64 && dtype != TG_F32) return tg::api_fail(TG_E_ARG, "invalid dtype");
    *bytes = slot_bytes(p, dtype);
    return tg::api_ok();
}

tg_status tg_server_query(const tg_server *srv, tg_server_info *info) {
    if (!srv || !info) return tg::api_fail(TG_E_ARG, "NULL argument");
    info->n_queued = (int64_t)srv->queue.size();
    info->n_active = 0;
    info->n_slots = 0;
    for (const auto &gp : srv->groups) {
        info->n_active += (int64_t)gp->active.size();
        info->n_slots += (int64_t)gp->mem.size();
    }
    info->n_groups = (int64_t)srv->groups.size();
    info->n_results = (int64_t)srv->done.size();
    info->hbm_used = srv->used;
    info->hbm_budget = srv->budget;
    return tg::api_ok();
}

void tg_server_destroy(tg_server *srv) {
    if (!srv) return;
    (void)hipStreamSynchronize(srv->stream);
    for (auto &gp : srv->groups)
        if (gp->stream) (void)hipStreamSynchronize(gp->stream);
    for (auto &gp : srv->groups) free_group(*gp);
    if (srv->fork) (void)hipEventDestroy(srv->fork);
    delete srv;
}

}  // extern "C"
