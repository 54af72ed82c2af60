// Request server: continuous batching of assemble + Dirichlet + PCG requests
// with iteration-level scheduling.
//
// The paper generates data in batches (SM B.1.4, efficient batch data
// generation); a stream of independent solves is served here the way LLM
// servers batch token generation.  Requests are grouped by (pattern, dtype).
// Each group owns slots: per-slot device buffers (values, rhs, Krylov
// workspace, partial sums, state).  Between CG iterations the scheduler
// retires finished systems and admits queued requests into the freed slots
// (their assembly, Dirichlet elimination and CG initialisation run then);
// every iteration is one launch over all active slots of a group
// (blockIdx.y = slot).  The per-slot reductions never mix: a slot's scalars
// come from its own partials in the same fixed order as a solo tg_pcg on the
// same kernels, and a slot takes the solo solver's decisions (residual
// replacement included), so a request's solution is bitwise the same whether
// it ran alone or in a mix.
//
// Memory: everything the server allocates is counted against its HBM budget:
// group tables, slots, and the CSR patterns it builds for requests submitted
// by connectivity (tg_server_submit_mesh; a cache keyed by the caller's
// topology key).  When a request needs memory that the budget does not have,
// the server frees what no request is using, least recently used first: idle
// slots of other groups, then groups without slots, then cached patterns that
// no running request needs (a queued request's pattern only when that request
// is younger than the one memory is made for; it is rebuilt when its turn
// comes).  A request fails with TG_E_NOMEM only when one slot of it (with its
// group's tables and, for a cached topology, its pattern) exceeds the whole
// budget; otherwise it waits until memory frees.  A missing pattern is built
// on the host first and uploaded once its device bytes fit.
//
// Scheduling: queued requests are admitted oldest first across groups, and
// strictly in order once one of them has to wait for memory, so the oldest
// request always makes progress.  Each
// group runs on a stream of its own (default priority), forked from the
// caller's stream at the start of a scheduling round and joined back before
// the round's synchronisation, so the launches of groups on different patterns
// (often small, latency-bound systems) overlap on the GPU.  Patterns of new
// topologies are built on host worker threads while rounds run on the GPU;
// requests whose patterns are resident go ahead meanwhile.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <future>
#include <memory>
#include <thread>
#include <vector>

#include "tg_internal.h"

namespace {

using tg::PcgSlot;
using tg::PcgState;

struct Request {
    int64_t id;
    const tg_pattern *p;  // NULL for a mesh request whose pattern is not resident yet
    // a mesh request's topology (caller-owned connectivity)
    bool mesh;
    int32_t dim;
    int64_t nv, E;
    const int32_t *conn;
    uint64_t key;
    tg_form form;
    tg_dtype dtype;
    const double *coords;
    const void *coef, *load, *g;
    void *x;
    double rtol;
    int32_t max_iter;
    double t_submit;
    int32_t iters_done;  // iterations of earlier CG runs (residual replacement)
    int32_t run;         // CG runs started before the current one
    bool checked;        // validated against its pattern
    double prev_relres;  // the previous run's true residual
};

struct SlotMem {
    void *values = nullptr, *sell = nullptr, *b = nullptr, *work = nullptr;
    double *partials = nullptr;
    uint64_t last_used = 0;
    bool allocated() const { return values != nullptr; }
};

struct Group {
    const tg_pattern *p = nullptr;
    tg_dtype dtype = TG_F64;
    int max_slots = 0;
    std::vector<SlotMem> mem;      // slot buffers; freed ones stay as empty entries
    std::vector<int> busy;         // 1 while a request occupies the slot
    std::vector<Request> req;      // request per slot
    std::vector<int> active;       // slot ids in the batch, admission order
    // device tables (max_slots entries) and their pinned staging copies
    PcgSlot *d_slots = nullptr, *h_slots = nullptr;
    PcgState *d_states = nullptr, *h_states = nullptr;
    int32_t *d_status = nullptr, *h_status = nullptr;
    int32_t *d_lists = nullptr, *h_lists = nullptr;  // [active | fresh | finished], max_slots each
    int step = 0;
    size_t slot_bytes = 0, table_bytes = 0;
    uint64_t last_used = 0;
    hipStream_t stream = nullptr;  // the group's own stream
    hipEvent_t joined = nullptr;   // recorded on it at the end of a round
    // retirement in flight between the launch and the finish phase of a round
    std::vector<int> fin, keep;
    std::vector<double> parts;
    int n_parts = 0;
    int n_allocated() const {
        int k = 0;
        for (const SlotMem &m : mem) k += m.allocated();
        return k;
    }
    bool any_busy() const { return std::find(busy.begin(), busy.end(), 1) != busy.end(); }
};

// A pattern the server built for mesh requests: on the host only while it
// waits for memory (`resident` false), then uploaded.
struct CachedPattern {
    uint64_t key;
    int32_t dim, order;
    int64_t nv, E;
    tg_pattern *p;
    size_t bytes;  // device bytes (counted against the budget while resident)
    uint64_t last_used;
    bool resident;
};

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// A host pattern build in flight on a worker thread (its own copy of the
// connectivity: the caller may release a request's arrays once its result is
// polled, while the build may still run).
struct BuildResult {
    tg_status status;
    tg_pattern *p;
    double seconds;
};
struct PendingBuild {
    uint64_t key;
    int32_t dim, order;
    int64_t nv, E;
    std::vector<int32_t> conn;
    std::future<BuildResult> done;
};

}  // namespace

struct tg_server {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr;  // recorded on `stream` at the start of a round
    size_t budget = 0, used = 0;
    int max_slots = 1;
    int check_every = 1;
    int64_t next_id = 1;
    uint64_t clock = 0;  // scheduling rounds so far (the LRU clock)
    double t0 = 0.0;
    std::deque<Request> queue;
    std::vector<std::unique_ptr<Group>> groups;
    std::vector<CachedPattern> patterns;
    std::vector<std::unique_ptr<PendingBuild>> building;
    int build_threads = 1;
    int64_t mem_blocked = -1;  // the request whose built pattern waits for memory (admission stops there)
    int64_t n_builds = 0, n_evictions = 0;
    double build_s = 0.0;
    std::deque<tg_server_result> done;
};

namespace {

const size_t kPartialBytes = (size_t)tg::kNumPartials * tg::kMaxGrid * sizeof(double);

size_t slot_bytes(const tg_pattern *p, tg_dtype dtype) {
    const size_t elt = dtype == TG_F64 ? 8 : 4, n = (size_t)p->host.n_dofs;
    return ((size_t)p->host.nnz + (size_t)p->dev.sell_nnz + (1 + tg::kPcgWorkVectors) * n) * elt + kPartialBytes;
}

// The same for a pattern still on the host (its sliced-ELL size is known).
size_t slot_bytes_planned(const tg::HostPattern &h, tg_dtype dtype) {
    const size_t elt = dtype == TG_F64 ? 8 : 4, n = (size_t)h.n_dofs;
    const size_t sell = h.sell_ptr.empty() ? 0 : (size_t)h.sell_ptr.back();
    return ((size_t)h.nnz + sell + (1 + tg::kPcgWorkVectors) * n) * elt + kPartialBytes;
}

size_t table_bytes(int max_slots) {
    return (size_t)max_slots * (sizeof(PcgSlot) + sizeof(PcgState) + 4 * sizeof(int32_t));
}

void free_slot(SlotMem &m) {
    (void)hipFree(m.values);
    (void)hipFree(m.sell);
    (void)hipFree(m.b);
    (void)hipFree(m.work);
    (void)hipFree(m.partials);
    m = SlotMem{};
}

void free_group(Group &g) {
    if (g.stream) (void)hipStreamSynchronize(g.stream);
    for (SlotMem &m : g.mem) free_slot(m);
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

CachedPattern *find_cached(tg_server *srv, const Request &r) {
    const int order = r.form == TG_ELASTICITY ? 2 : 1;
    for (CachedPattern &c : srv->patterns)
        if (c.key == r.key && c.dim == r.dim && c.order == order && c.nv == r.nv && c.E == r.E) return &c;
    return nullptr;
}

const CachedPattern *cached_entry(const tg_server *srv, const tg_pattern *p) {
    for (const CachedPattern &c : srv->patterns)
        if (c.p == p) return &c;
    return nullptr;
}

// A running system, or a queued request older than `prio` (a request id),
// needs pattern p.
bool pattern_needed(const tg_server *srv, const tg_pattern *p, int64_t prio) {
    for (const Request &r : srv->queue)
        if (r.p == p && r.id <= prio) return true;
    for (const auto &g : srv->groups)
        if (g->p == p && (!g->active.empty() || g->any_busy())) return true;
    return false;
}

bool group_idle(const tg_server *srv, const Group &g) {
    if (!g.active.empty() || g.any_busy()) return false;
    for (const Request &r : srv->queue)
        if (r.p == g.p && r.dtype == g.dtype) return false;
    return true;
}

void destroy_group_at(tg_server *srv, size_t i) {
    free_group(*srv->groups[i]);
    srv->used -= srv->groups[i]->table_bytes;
    srv->groups.erase(srv->groups.begin() + (std::ptrdiff_t)i);
}

// Frees memory until `need` more bytes fit in the budget, for request `prio`
// (an id): idle slots of groups other than `keep_g` (least recently used
// first), then idle groups without slots, then cached patterns that no running
// system and no queued request older than `prio` needs (other than `keep_p`),
// least recently used first; queued requests of an evicted pattern will have
// it rebuilt.  A slot goes idle only at retirement, after the round's
// synchronisation, so its work has completed.  Returns whether the bytes fit.
bool reclaim(tg_server *srv, size_t need, const Group *keep_g, const tg_pattern *keep_p, int64_t prio) {
    auto fits = [&] { return srv->used + need <= srv->budget; };
    while (!fits()) {
        Group *bg = nullptr;
        int bs = -1;
        for (auto &gp : srv->groups) {
            if (gp.get() == keep_g) continue;
            for (size_t s = 0; s < gp->mem.size(); ++s)
                if (gp->mem[s].allocated() && !gp->busy[s] &&
                    (bs < 0 || gp->mem[s].last_used < bg->mem[bs].last_used)) {
                    bg = gp.get();
                    bs = (int)s;
                }
        }
        if (bs < 0) break;
        free_slot(bg->mem[bs]);
        srv->used -= bg->slot_bytes;
    }
    for (size_t i = 0; i < srv->groups.size() && !fits();) {
        const Group &g = *srv->groups[i];
        if (&g != keep_g && g.n_allocated() == 0 && group_idle(srv, g))
            destroy_group_at(srv, i);
        else
            ++i;
    }
    while (!fits()) {
        int bi = -1;
        for (size_t i = 0; i < srv->patterns.size(); ++i) {
            const CachedPattern &c = srv->patterns[i];
            if (!c.resident || c.p == keep_p || pattern_needed(srv, c.p, prio)) continue;
            bool has_slots = false;
            for (auto &gp : srv->groups) has_slots = has_slots || (gp->p == c.p && gp->n_allocated() > 0);
            if (has_slots) continue;
            if (bi < 0 || c.last_used < srv->patterns[bi].last_used) bi = (int)i;
        }
        if (bi < 0) break;
        tg_pattern *p = srv->patterns[bi].p;
        for (size_t i = 0; i < srv->groups.size();) {  // its groups (idle, without slots) go with it
            if (srv->groups[i]->p == p)
                destroy_group_at(srv, i);
            else
                ++i;
        }
        for (Request &r : srv->queue)
            if (r.p == p) {
                r.p = nullptr;
                r.checked = false;
            }
        srv->used -= srv->patterns[bi].bytes;
        tg_pattern_destroy(p);
        srv->patterns.erase(srv->patterns.begin() + bi);
        ++srv->n_evictions;
    }
    return fits();
}

// The group of (p, dtype), creating it (tables within the budget); *out is
// NULL when the tables do not fit now.
tg_status get_group(tg_server *srv, const tg_pattern *p, tg_dtype dtype, int64_t prio, Group **out) {
    *out = find_group(srv, p, dtype);
    if (*out) return TG_OK;
    const size_t tb = table_bytes(srv->max_slots);
    if (!reclaim(srv, tb, nullptr, p, prio)) return TG_OK;
    auto g = std::make_unique<Group>();
    g->p = p;
    g->dtype = dtype;
    g->max_slots = srv->max_slots;
    g->slot_bytes = slot_bytes(p, dtype);
    g->table_bytes = tb;
    const size_t S = (size_t)srv->max_slots;
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
    srv->used += tb;
    g->last_used = srv->clock;
    *out = g.get();
    srv->groups.push_back(std::move(g));
    return TG_OK;
}

// A free slot of g, allocating one within the budget (reclaiming memory for
// request `prio` first); -1 if none.
int take_slot(tg_server *srv, Group &g, int64_t prio, tg_status &st) {
    st = TG_OK;
    int hole = -1;
    for (size_t i = 0; i < g.mem.size(); ++i) {
        if (g.mem[i].allocated() && !g.busy[i]) return (int)i;
        if (!g.mem[i].allocated() && hole < 0) hole = (int)i;
    }
    if (hole < 0 && (int)g.mem.size() >= g.max_slots) return -1;
    if (!reclaim(srv, g.slot_bytes, &g, g.p, prio)) return -1;
    const size_t elt = g.dtype == TG_F64 ? 8 : 4, n = (size_t)g.p->host.n_dofs;
    SlotMem m;
    hipError_t e = hipMalloc(&m.values, std::max<size_t>(1, g.p->host.nnz) * elt);
    if (e == hipSuccess) e = hipMalloc(&m.sell, std::max<size_t>(1, (size_t)g.p->dev.sell_nnz) * elt);
    if (e == hipSuccess) e = hipMalloc(&m.b, std::max<size_t>(1, n) * elt);
    if (e == hipSuccess) e = hipMalloc(&m.work, std::max<size_t>(1, tg::kPcgWorkVectors * n) * elt);
    if (e == hipSuccess) e = hipMalloc((void **)&m.partials, kPartialBytes);
    if (e != hipSuccess) {
        free_slot(m);
        st = hip_fail(e, "server slot allocation failed");
        return -1;
    }
    srv->used += g.slot_bytes;
    if (hole >= 0) {
        g.mem[hole] = m;
        return hole;
    }
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
    res.pad = 0;
    res.t_submit = r.t_submit - srv->t0;
    res.t_done = now_s() - srv->t0;
    srv->done.push_back(res);
}

// The bytes one request on (p, dtype) needs at least: above the whole budget
// it can never run.
size_t min_bytes(const tg_server *srv, const tg_pattern *p, tg_dtype dtype) {
    const CachedPattern *c = cached_entry(srv, p);
    return slot_bytes(p, dtype) + table_bytes(srv->max_slots) + (c ? c->bytes : 0);
}

// The slot's CG record for a (re)started run of its request.
void set_slot(Group &g, int s, int step) {
    const Request &r = g.req[s];
    const SlotMem &m = g.mem[s];
    g.h_slots[s] = PcgSlot{m.values, m.sell, m.b, r.x, m.work, m.partials, g.d_states + s, r.rtol * r.rtol,
                           step, r.max_iter - r.iters_done, r.run > 0 ? 1 : 0};
    g.h_states[s] = PcgState{};  // all zero: not done, no iterations
}

// Upload the listed slots' records and states (and status words).
hipError_t upload_slots(Group &g, const std::vector<int> &slots, bool status) {
    const hipStream_t str = g.stream;
    hipError_t e = hipSuccess;
    for (int s : slots) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(g.d_slots + s, g.h_slots + s, sizeof(PcgSlot), hipMemcpyHostToDevice, str);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g.d_states + s, g.h_states + s, sizeof(PcgState), hipMemcpyHostToDevice, str);
        if (status && e == hipSuccess)
            e = hipMemcpyAsync(g.d_status + s, g.h_status + s, sizeof(int32_t), hipMemcpyHostToDevice, str);
    }
    return e;
}

using Fresh = std::vector<std::pair<Group *, std::vector<int>>>;

// Admit queued requests into free slots, oldest first across groups; `fresh`
// collects the admitted slots per group.  A request whose pattern is still
// being built is passed over; once a request has to wait for memory or a slot
// (or its built pattern waits for memory) no younger request is admitted in
// this round, so the oldest request always makes progress.
tg_status admit(tg_server *srv, Fresh &fresh) {
    tg_status st = TG_OK;
    for (auto it = srv->queue.begin(); it != srv->queue.end();) {
        if (!it->p) {
            if (it->id == srv->mem_blocked) break;
            ++it;  // its pattern is being built
            continue;
        }
        if (min_bytes(srv, it->p, it->dtype) > srv->budget) {  // can never run
            finish(srv, *it, TG_E_NOMEM, 0, 0.0, -1);
            it = srv->queue.erase(it);
            continue;
        }
        Group *g = nullptr;
        st = get_group(srv, it->p, it->dtype, it->id, &g);
        if (st != TG_OK) return st;
        const int s = g ? take_slot(srv, *g, it->id, st) : -1;
        if (st != TG_OK) return st;
        if (s < 0) break;
        g->busy[s] = 1;
        g->req[s] = *it;
        g->mem[s].last_used = srv->clock;
        g->last_used = srv->clock;
        set_slot(*g, s, g->step);
        g->h_status[s] = TG_STATUS_CLEAN;
        auto f = std::find_if(fresh.begin(), fresh.end(), [&](const auto &x) { return x.first == g; });
        if (f == fresh.end()) {
            fresh.emplace_back(g, std::vector<int>{});
            f = fresh.end() - 1;
        }
        f->second.push_back(s);
        it = srv->queue.erase(it);
    }
    return TG_OK;
}

// Enqueue the admitted requests' assembly, Dirichlet elimination and CG
// initialisation on their group's stream.
tg_status launch_admitted(Group &g, const std::vector<int> &fresh) {
    const hipStream_t str = g.stream;
    const int S = g.max_slots;
    for (int s : fresh) g.active.push_back(s);
    for (size_t i = 0; i < g.active.size(); ++i) g.h_lists[i] = g.active[i];
    for (size_t i = 0; i < fresh.size(); ++i) g.h_lists[S + i] = fresh[i];
    // Only the fresh slots' entries are written: the other slots' device state is live.
    hipError_t e = upload_slots(g, fresh, true);
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
        if (st.done || it > g.h_slots[s].max_iter || !tg::state_finite(st)) g.fin.push_back(s);
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

// Retirement, phase 2 (the group's stream synchronised): results of the
// finished systems, or a restart from x of those whose true residual stayed
// above rtol (the solo solver's residual replacement: tg::run_end decides for
// both).  Restarted slots rejoin the batch after a warm initialisation.
tg_status retire_finish(tg_server *srv, Group &g) {
    if (g.fin.empty()) return TG_OK;
    const int ns = g.n_parts;
    std::vector<int> restart;
    for (size_t i = 0; i < g.fin.size(); ++i) {
        const int s = g.fin[i];
        const PcgState &st = g.h_states[s];
        Request &r = g.req[s];
        double rr = 0.0;
        for (int k = 0; k < ns; ++k) rr += g.parts[i * ns + k];
        const double relres = st.bb > 0.0 ? std::sqrt(rr / st.bb) : std::sqrt(rr);
        const bool done = st.done != 0;
        const int32_t total = r.iters_done + (done ? st.iters : r.max_iter - r.iters_done);
        if (g.h_status[s] != TG_STATUS_CLEAN) {  // a bad element: the system is meaningless
            finish(srv, r, TG_E_DEGENERATE, total, relres, g.h_status[s]);
            g.busy[s] = 0;
            continue;
        }
        const tg::RunEnd end =
            tg::run_end(done, relres, r.prev_relres, r.rtol, !tg::state_finite(st), r.run, total, r.max_iter);
        r.prev_relres = relres;
        if (end == tg::RunEnd::kRestart) {
            r.iters_done = total;
            ++r.run;
            set_slot(g, s, g.step);
            restart.push_back(s);
            continue;
        }
        const tg_status status = end == tg::RunEnd::kOk          ? TG_OK
                                 : end == tg::RunEnd::kNonFinite ? TG_E_NONFINITE
                                 : end == tg::RunEnd::kAccuracy  ? TG_E_ACCURACY
                                                                 : TG_E_NOCONV;
        finish(srv, r, status, total, relres, -1);
        g.busy[s] = 0;
    }
    g.active = g.keep;
    g.fin.clear();
    if (restart.empty()) return TG_OK;
    const int S = g.max_slots;
    for (int s : restart) g.active.push_back(s);
    for (size_t i = 0; i < g.active.size(); ++i) g.h_lists[i] = g.active[i];
    for (size_t i = 0; i < restart.size(); ++i) g.h_lists[S + i] = restart[i];
    hipError_t e = upload_slots(g, restart, false);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g.d_lists, g.h_lists, 2 * S * sizeof(int32_t), hipMemcpyHostToDevice, g.stream);
    if (e == hipSuccess)
        e = tg::launch_pcg_warm_init(*g.p, g.dtype, g.d_slots, g.d_lists + S, (int)restart.size(), g.stream);
    // the pinned staging copies may be rewritten by the next round's admission
    if (e == hipSuccess) e = hipStreamSynchronize(g.stream);
    if (e != hipSuccess) return hip_fail(e, "server restart failed");
    return TG_OK;
}

// Patterns for mesh requests: collects finished host builds, starts builds
// (on worker threads, up to build_threads at once) for queued topologies that
// have no pattern, and uploads built patterns, oldest request first, when
// their device bytes fit the budget (making room for them as for that
// request; the first that does not fit stops the uploads and admission).  A
// topology that tg_pattern_create rejects fails its requests with that status;
// one whose pattern with one slot exceeds the whole budget fails them with
// TG_E_NOMEM.
void progress_patterns(tg_server *srv) {
    auto same_topology = [](const Request &q, uint64_t key, int32_t dim, int32_t order, int64_t nv, int64_t E) {
        return q.mesh && q.key == key && q.dim == dim && (q.form == TG_ELASTICITY ? 2 : 1) == order && q.nv == nv &&
               q.E == E;
    };
    auto fail_topology = [&](tg_status st, uint64_t key, int32_t dim, int32_t order, int64_t nv, int64_t E) {
        for (auto q = srv->queue.begin(); q != srv->queue.end();) {
            if (!q->p && same_topology(*q, key, dim, order, nv, E)) {
                finish(srv, *q, st, 0, 0.0, -1);
                q = srv->queue.erase(q);
            } else {
                ++q;
            }
        }
    };
    // finished builds
    for (size_t i = 0; i < srv->building.size();) {
        PendingBuild &b = *srv->building[i];
        if (b.done.wait_for(std::chrono::seconds(0)) != std::future_status::ready) {
            ++i;
            continue;
        }
        const BuildResult r = b.done.get();
        srv->build_s += r.seconds;
        ++srv->n_builds;
        if (r.status != TG_OK)
            fail_topology(r.status, b.key, b.dim, b.order, b.nv, b.E);
        else
            srv->patterns.push_back(CachedPattern{b.key, b.dim, b.order, b.nv, b.E, r.p, tg::device_bytes(r.p->host),
                                                  srv->clock, false});
        srv->building.erase(srv->building.begin() + (std::ptrdiff_t)i);
    }
    // new builds, oldest request first
    for (const Request &q : srv->queue) {
        if (q.p || !q.mesh || (int)srv->building.size() >= srv->build_threads) continue;
        const int32_t order = q.form == TG_ELASTICITY ? 2 : 1;
        if (find_cached(srv, q)) continue;
        bool in_flight = false;
        for (const auto &b : srv->building) in_flight = in_flight || same_topology(q, b->key, b->dim, b->order, b->nv, b->E);
        if (in_flight) continue;
        auto job = std::make_unique<PendingBuild>();
        *job = PendingBuild{q.key, q.dim, order, q.nv, q.E,
                            std::vector<int32_t>(q.conn, q.conn + q.E * (int64_t)(q.dim + 1)), {}};
        const PendingBuild *jp = job.get();
        job->done = std::async(std::launch::async, [jp]() {
            const double t = now_s();
            tg_pattern *p = nullptr;
            const bool p2 = jp->order == 2;
            const tg_status st = tg_pattern_create(jp->dim, p2 ? 2 : 1, p2 ? 3 : 1, jp->nv, jp->E, jp->conn.data(),
                                                   nullptr, TG_BOUNDARY_ALL, TG_PATTERN_HOST_ONLY, &p);
            return BuildResult{st, st == TG_OK ? p : nullptr, now_s() - t};
        });
        srv->building.push_back(std::move(job));
    }
    // uploads, oldest request first (a topology that fails is dropped from the
    // queue, and the pass starts again)
    auto upload_pass = [&]() -> bool {
        srv->mem_blocked = -1;
        for (Request &r : srv->queue) {
            if (r.p || !r.mesh) continue;
            CachedPattern *c = find_cached(srv, r);
            if (!c) continue;  // still being built
            if (!c->resident) {
                const uint64_t key = c->key;
                const int32_t dim = c->dim, order = c->order;
                const int64_t nv = c->nv, E = c->E;
                tg_pattern *const cp = c->p;
                const size_t one_slot = slot_bytes_planned(cp->host, r.dtype) + table_bytes(srv->max_slots);
                tg_status st = TG_OK;
                if (c->bytes + one_slot > srv->budget) {
                    st = TG_E_NOMEM;  // can never run
                } else {
                    const bool fits = reclaim(srv, c->bytes, nullptr, cp, r.id);  // may erase other cache entries
                    c = &*std::find_if(srv->patterns.begin(), srv->patterns.end(),
                                       [&](const CachedPattern &x) { return x.p == cp; });
                    if (!fits) {
                        srv->mem_blocked = r.id;  // waits for running requests to finish
                        return false;
                    }
                    const double t = now_s();
                    st = tg::upload_pattern(cp);
                    srv->build_s += now_s() - t;
                }
                if (st != TG_OK) {
                    srv->patterns.erase(srv->patterns.begin() + (c - srv->patterns.data()));
                    tg_pattern_destroy(cp);
                    fail_topology(st, key, dim, order, nv, E);
                    return true;
                }
                c->resident = true;
                srv->used += c->bytes;
            }
            c->last_used = srv->clock;
            for (Request &q : srv->queue)
                if (!q.p && q.mesh)
                    if (CachedPattern *e = find_cached(srv, q); e && e->resident) q.p = e->p;
        }
        return false;
    };
    while (upload_pass()) {
    }
}

// Mesh requests are validated against their pattern once it is resident;
// those that fail finish with the error.
void validate_resolved(tg_server *srv) {
    for (auto it = srv->queue.begin(); it != srv->queue.end();) {
        if (it->p && !it->checked) {
            it->checked = true;
            const tg_status st = tg::validate_assemble(it->p, it->form, it->dtype, 1, it->coords, it->coef, it->x);
            if (st != TG_OK) {
                finish(srv, *it, st, 0, 0.0, -1);
                it = srv->queue.erase(it);
                continue;
            }
        }
        ++it;
    }
}

tg_status check_request(tg_server *srv, tg_form form, const void *d_load, void *d_x, double rtol, int32_t max_iter) {
    if (!srv) return tg::api_fail(TG_E_ARG, "server is NULL");
    if (!d_x) return tg::api_fail(TG_E_ARG, "d_x is required");
    if (form == TG_MASS) return tg::api_fail(TG_E_ARG, "MASS has no right-hand side to solve for");
    if (!d_load) return tg::api_fail(TG_E_ARG, "d_load is required (the right-hand side)");
    if (!(rtol > 0.0) || max_iter < 1) return tg::api_fail(TG_E_ARG, "need rtol > 0 and max_iter >= 1");
    if ((uint64_t)max_iter + 2 * (uint64_t)srv->check_every >= (uint64_t)1 << 30)
        return tg::api_fail(TG_E_ARG, "max_iter too large");
    return TG_OK;
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
    srv->build_threads = (int)std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
    srv->t0 = now_s();
    *out = srv;
    return tg::api_ok();
}

tg_status tg_server_submit(tg_server *srv, const tg_pattern *p, tg_form form, tg_dtype dtype, const double *d_coords,
                           const void *d_coef, const void *d_load, const void *d_g, void *d_x, double rtol,
                           int32_t max_iter, int64_t *request_id) {
    tg_status st = check_request(srv, form, d_load, d_x, rtol, max_iter);
    if (st != TG_OK) return st;
    // d_values is checked as non-NULL: the slot provides it
    st = tg::validate_assemble(p, form, dtype, 1, d_coords, d_coef, (const void *)d_x);
    if (st != TG_OK) return st;
    Request r{srv->next_id++, p,     false, 0,     0,        0,   nullptr, 0, form, dtype, d_coords, d_coef,
              d_load,         d_g,   d_x,   rtol,  max_iter, now_s(), 0,   0, true, INFINITY};
    srv->queue.push_back(r);
    if (request_id) *request_id = r.id;
    return tg::api_ok();
}

tg_status tg_server_submit_mesh(tg_server *srv, int32_t dim, int64_t n_vertices, int64_t n_elements,
                                const int32_t *conn, uint64_t topology_key, tg_form form, tg_dtype dtype,
                                const double *d_coords, const void *d_coef, const void *d_load, void *d_x,
                                double rtol, int32_t max_iter, int64_t *request_id) {
    tg_status st = check_request(srv, form, d_load, d_x, rtol, max_iter);
    if (st != TG_OK) return st;
    if (dim != 2 && dim != 3) return tg::api_fail(TG_E_ARG, "dim must be 2 or 3");
    if (form != TG_LAPLACE && form != TG_MASS_LAPLACE && form != TG_ELASTICITY)
        return tg::api_fail(TG_E_ARG, "invalid form");
    if (form == TG_ELASTICITY && dim != 3) return tg::api_fail(TG_E_ARG, "ELASTICITY needs dim 3");
    if (dtype != TG_F64 && dtype != TG_F32) return tg::api_fail(TG_E_ARG, "invalid dtype");
    if (n_vertices <= 0 || n_elements <= 0 || !conn || !d_coords || !d_coef)
        return tg::api_fail(TG_E_ARG, "need n_vertices, n_elements > 0 and conn, d_coords, d_coef");
    Request r{srv->next_id++, nullptr, true,    dim,  n_vertices, n_elements, conn, topology_key, form, dtype,
              d_coords,       d_coef,  d_load,  nullptr, d_x,     rtol,       max_iter, now_s(), 0, 0, false,
              INFINITY};
    if (CachedPattern *c = find_cached(srv, r); c && c->resident) r.p = c->p;
    srv->queue.push_back(r);
    if (request_id) *request_id = r.id;
    return tg::api_ok();
}

tg_status tg_server_step(tg_server *srv, int32_t *n_active, int32_t *n_queued) {
    if (!srv) return tg::api_fail(TG_E_ARG, "server is NULL");
    const hipStream_t str = srv->stream;
    ++srv->clock;
    progress_patterns(srv);
    validate_resolved(srv);
    for (const Request &r : srv->queue)  // the cached patterns queued requests need are in use
        for (CachedPattern &c : srv->patterns)
            if (c.p == r.p) c.last_used = srv->clock;
    // fork: every group's stream starts after the work already on the caller's stream
    hipError_t e = hipEventRecord(srv->fork, str);
    if (e != hipSuccess) return hip_fail(e, "server fork failed");
    Fresh fresh;
    tg_status st = admit(srv, fresh);
    if (st != TG_OK) return st;
    bool any = false;
    for (auto &gp : srv->groups) {
        Group &g = *gp;
        auto f = std::find_if(fresh.begin(), fresh.end(), [&](const auto &x) { return x.first == &g; });
        if (g.active.empty() && f == fresh.end()) continue;
        e = hipStreamWaitEvent(g.stream, srv->fork, 0);
        if (e != hipSuccess) return hip_fail(e, "server fork failed");
        if (f != fresh.end()) {
            st = launch_admitted(g, f->second);
            if (st != TG_OK) return st;
        }
        any = true;
        g.last_used = srv->clock;
        for (CachedPattern &c : srv->patterns)
            if (c.p == g.p) c.last_used = srv->clock;
        for (size_t s = 0; s < g.mem.size(); ++s)
            if (g.busy[s]) g.mem[s].last_used = srv->clock;
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
            st = retire_launch(*gp);
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
            for (auto &gp : srv->groups) {
                st = retire_finish(srv, *gp);
                if (st != TG_OK) return st;
            }
        }
    }
    // nothing ran on the GPU and builds are in flight: wait for the oldest
    // instead of returning at once (callers step until the queue drains)
    if (!any && !srv->building.empty()) srv->building.front()->done.wait();
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
        info->n_slots += (int64_t)gp->n_allocated();
    }
    info->n_groups = (int64_t)srv->groups.size();
    info->n_results = (int64_t)srv->done.size();
    info->hbm_used = srv->used;
    info->hbm_budget = srv->budget;
    info->n_patterns = (int64_t)srv->patterns.size();
    info->n_pattern_builds = srv->n_builds;
    info->n_pattern_evictions = srv->n_evictions;
    info->pattern_build_s = srv->build_s;
    return tg::api_ok();
}

void tg_server_destroy(tg_server *srv) {
    if (!srv) return;
    (void)hipStreamSynchronize(srv->stream);
    for (auto &gp : srv->groups) free_group(*gp);
    for (auto &b : srv->building) {  // wait for the builds in flight
        const BuildResult r = b->done.get();
        if (r.p) tg_pattern_destroy(r.p);
    }
    for (CachedPattern &c : srv->patterns) tg_pattern_destroy(c.p);
    if (srv->fork) (void)hipEventDestroy(srv->fork);
    delete srv;
}

}  // extern "C"
