// Serving: a request loop over resident graphs (host runtime; the searches
// are the single-root and batched engines' kernels).
//
// Requests wait in one queue per graph. Each of `slots` worker threads owns
// a HIP stream and a pinned mailbox; when free it picks the graph whose
// oldest request has the highest response ratio (its wait plus the graph's
// expected service time, over that expected time: short jobs go first,
// long waits are not starved), takes up to max_batch of that graph's
// requests, and answers them either one by one with the direction-optimizing
// single-root search (csbfs_bfs_ws) or all at once with one batched search
// (csbfs_batch_bfs), whichever the measured per-graph costs say is cheaper
// for that many roots. A request's output buffer is written on the slot's
// stream after an event the submitter recorded on its own stream.
//
// Memory: per (slot, graph) one block holds the batched engine, its result
// buffer, the single-root workspace and a parent scratch vector. Blocks are
// admitted under the HBM budget and come from the stream-ordered allocator
// (hipMallocAsync / hipFreeAsync on the slot's stream), so creating or
// evicting one (idle blocks go first, least recently used first) never
// synchronizes the device or stalls the other slots.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "graph.hpp"

using namespace csbfs;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    int32_t *out = nullptr;
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream (null: no output)
    bool done = false;
    csbfs_request_info info{};
};

struct Block {
    void *mem = nullptr;  // one stream-ordered allocation
    csbfs_batch_engine *eng = nullptr;
    int32_t *levels = nullptr;  // [max_batch][n], batched results
    void *ws = nullptr;         // single-root workspace
    int32_t *parent = nullptr;  // [n], single-root parents (not returned)
    int64_t bytes = 0;
    bool busy = false;
    uint64_t last_use = 0;
};

struct GraphState {
    const csbfs_graph *g = nullptr;
    int64_t batch_bytes = 0, levels_bytes = 0, ws_bytes = 0, parent_bytes = 0, need = 0;
    std::deque<int64_t> pending;
    // expected costs (seconds, exponentially weighted): one single-root
    // search, and one batched search (about flat in the number of roots)
    double single_s = 0.0, batch_s = 0.0;
    int single_n = 0, batch_n = 0;
};

constexpr double kEwma = 0.3;
// Until a graph has been measured both ways, batches of at least this many
// roots go to the batched engine.
constexpr int kBatchFirst = 8;

}  // namespace

struct csbfs_server {
    csbfs_server_config cfg{};
    int device = -1;
    std::deque<GraphState> graphs;  // stable addresses while graphs are added
    std::mutex mu;
    std::condition_variable cv_work;
    std::condition_variable cv_done;
    int64_t n_pending = 0;
    std::unordered_map<int64_t, Request> reqs;
    std::vector<hipEvent_t> free_events;
    int64_t next_id = 0;
    int running = 0;   // batches in flight
    int creating = 0;  // blocks being allocated (their bytes already reserved)
    int64_t held = 0;
    uint64_t use_clock = 0;
    std::map<std::pair<int, int>, Block> blocks;  // (slot, graph)
    std::vector<hipStream_t> streams;
    unsigned long long *mailboxes = nullptr;  // pinned [slots][4]: batched counts, single-root mailbox
    std::vector<std::thread> workers;
    bool stop = false;
};

namespace {

csbfs_search_config single_cfg() {
    csbfs_search_config c{};
    c.max_levels = 64;
    return c;
}

// Release a block's engine and queue its memory's release on `st`.
void release_block(Block &b, hipStream_t st) {
    if (b.eng) batch_engine_release(b.eng);
    if (b.mem) (void)hipFreeAsync(b.mem, st);
    b = Block{};
}

void finish(csbfs_server *s, const std::vector<int64_t> &ids, const std::vector<int> &status,
            const std::vector<int32_t> &n_levels, int batch, int slot, double t_start, bool batched = false) {
    const double t = now_s();
    for (size_t k = 0; k < ids.size(); ++k) {
        Request &r = s->reqs[ids[k]];
        r.info.status = status[k];
        r.info.n_levels = n_levels[k];
        r.info.batch_size = batch;
        r.info.slot = slot;
        r.info.batched = batched ? 1 : 0;
        r.info.t_start = t_start;
        r.info.t_done = t;
        r.done = true;
        if (r.ready) {
            s->free_events.push_back(r.ready);
            r.ready = nullptr;
        }
    }
}

void fail_one(csbfs_server *s, GraphState &gs, int rc, int slot) {
    const int64_t id = gs.pending.front();
    gs.pending.pop_front();
    s->n_pending--;
    finish(s, {id}, {rc}, {0}, 1, slot, now_s());
    s->cv_done.notify_all();
}

// The graph to serve next: highest (wait + expected) / expected.
int pick_graph(csbfs_server *s, double now) {
    int best = -1;
    double best_ratio = -1.0;
    for (int g = 0; g < (int)s->graphs.size(); ++g) {
        GraphState &gs = s->graphs[g];
        if (gs.pending.empty()) continue;
        const double wait = now - s->reqs[gs.pending.front()].info.t_submit;
        const int take = (int)std::min<size_t>(gs.pending.size(), (size_t)s->cfg.max_batch);
        double est = gs.batch_n ? gs.batch_s : 0.0;
        if (gs.single_n) est = est > 0.0 ? std::min(est, take * gs.single_s) : take * gs.single_s;
        if (est <= 0.0) est = 1e-3 * ((double)gs.g->n / (double)(1 << 20));  // unmeasured: ~1 ms per 2^20 vertices
        const double ratio = (wait + est) / est;
        if (ratio > best_ratio) {
            best_ratio = ratio;
            best = g;
        }
    }
    return best;
}

// true: answer `take` roots with one batched search
bool use_batched(const GraphState &gs, int take) {
    if (take <= 1) return false;
    if (gs.batch_n && gs.single_n) return gs.batch_s < take * gs.single_s;
    return take >= kBatchFirst;
}

void worker(csbfs_server *s, int slot) {
    (void)hipSetDevice(s->device);
    hipStream_t st = s->streams[slot];
    unsigned long long *mb = s->mailboxes + 4 * slot;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_work.wait(lk, [&] { return s->stop || s->n_pending > 0; });
        if (s->n_pending == 0) {
            if (s->stop) return;
            continue;
        }
        const int g = pick_graph(s, now_s());
        if (g < 0) continue;
        GraphState &gs = s->graphs[g];
        Block &bk = s->blocks[{slot, g}];
        if (!bk.mem) {
            const int64_t need = gs.need;
            // make room: release idle blocks, least recently used first
            bool freed = false;
            while (s->held + need > s->cfg.hbm_budget) {
                Block *lru = nullptr;
                for (auto &kv : s->blocks) {
                    Block &c = kv.second;
                    if (c.mem && !c.busy && (!lru || c.last_use < lru->last_use)) lru = &c;
                }
                if (!lru) break;
                s->held -= lru->bytes;
                release_block(*lru, st);  // stream-ordered: no device-wide wait
                freed = true;
            }
            if (freed) continue;  // the queues may have changed meanwhile
            if (s->held + need > s->cfg.hbm_budget) {
                if (s->running == 0 && s->creating == 0) {
                    fail_one(s, gs, CSBFS_ENOSPACE, slot);  // nothing will free memory
                } else {
                    s->cv_work.wait(lk);  // a running batch will release its block
                }
                continue;
            }
            // reserve, then allocate outside the lock
            s->held += need;
            bk.busy = true;
            s->creating++;
            lk.unlock();
            void *mem = nullptr;
            csbfs_batch_engine *eng = nullptr;
            int rc = CSBFS_OK;
            if (hipMallocAsync(&mem, (size_t)need, st) != hipSuccess) {
                (void)hipGetLastError();
                rc = CSBFS_EHIP;
                mem = nullptr;
            }
            if (rc == CSBFS_OK)
                rc = batch_engine_make(gs.g, s->cfg.max_batch, s->cfg.max_levels, 0, mem, mb, st, &eng);
            lk.lock();
            s->creating--;
            s->cv_work.notify_all();
            Block &b2 = s->blocks[{slot, g}];
            b2.busy = false;
            if (rc != CSBFS_OK) {
                s->held -= need;
                if (mem) (void)hipFreeAsync(mem, st);
                if (!gs.pending.empty()) fail_one(s, gs, rc, slot);
                continue;
            }
            char *at = (char *)mem + gs.batch_bytes;
            b2.mem = mem;
            b2.eng = eng;
            b2.levels = (int32_t *)at;
            b2.ws = at + gs.levels_bytes;
            b2.parent = (int32_t *)((char *)b2.ws + gs.ws_bytes);
            b2.bytes = need;
            continue;  // re-pick with the block in place
        }
        // the oldest waiting requests of this graph, in order
        std::vector<int64_t> ids;
        std::vector<int64_t> roots;
        std::vector<int32_t *> outs;
        std::vector<hipEvent_t> ready;
        while (!gs.pending.empty() && (int)ids.size() < s->cfg.max_batch) {
            const int64_t id = gs.pending.front();
            gs.pending.pop_front();
            s->n_pending--;
            const Request &r = s->reqs[id];
            ids.push_back(id);
            roots.push_back(r.info.root);
            outs.push_back(r.out);
            ready.push_back(r.ready);
        }
        const bool batched = use_batched(gs, (int)ids.size());
        bk.busy = true;
        bk.last_use = ++s->use_clock;
        s->running++;
        Block b = bk;
        const int64_t n = gs.g->n;
        const csbfs_graph *gr = gs.g;
        const int64_t ws_bytes = gs.ws_bytes;
        lk.unlock();

        const double t_start = now_s();
        std::vector<int> status(ids.size(), CSBFS_OK);
        std::vector<int32_t> nls(ids.size(), 0);
        // outputs are written only after the submitters' own work on them
        for (hipEvent_t ev : ready)
            if (ev && hipStreamWaitEvent(st, ev, 0) != hipSuccess) std::fill(status.begin(), status.end(), CSBFS_EHIP);
        if (batched) {
            int32_t nl = 0;
            int rc = status[0] != CSBFS_OK ? status[0]
                                            : csbfs_batch_bfs(b.eng, roots.data(), (int32_t)roots.size(), b.levels,
                                                              nullptr, 0, &nl, st);
            if (rc == CSBFS_OK) {
                for (size_t r = 0; r < outs.size() && rc == CSBFS_OK; ++r)
                    if (outs[r] && hipMemcpyAsync(outs[r], b.levels + (int64_t)r * n, sizeof(int32_t) * n,
                                                  hipMemcpyDeviceToDevice, st) != hipSuccess)
                        rc = CSBFS_EHIP;
                if (rc == CSBFS_OK && hipStreamSynchronize(st) != hipSuccess) rc = CSBFS_EHIP;
            }
            std::fill(status.begin(), status.end(), rc);
            std::fill(nls.begin(), nls.end(), nl);
        } else {
            const csbfs_search_config cfg = single_cfg();
            for (size_t r = 0; r < ids.size(); ++r) {
                if (status[r] != CSBFS_OK) continue;
                int32_t *lv = outs[r] ? outs[r] : b.levels;
                status[r] = csbfs_bfs_ws(gr, roots[r], &cfg, lv, b.parent, nullptr, 0, &nls[r], b.ws,
                                         (size_t)ws_bytes, (uint64_t *)(mb + 2), st);
            }
        }
        const double dt = now_s() - t_start;

        lk.lock();
        if (batched) {
            gs.batch_s = gs.batch_n++ ? (1 - kEwma) * gs.batch_s + kEwma * dt : dt;
        } else {
            const double per = dt / (double)ids.size();
            gs.single_s = gs.single_n++ ? (1 - kEwma) * gs.single_s + kEwma * per : per;
        }
        finish(s, ids, status, nls, (int)ids.size(), slot, t_start, batched);
        Block &b3 = s->blocks[{slot, g}];
        b3.busy = false;
        s->running--;
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

}  // namespace

extern "C" int csbfs_server_create(const csbfs_server_config *cfg, csbfs_server **out) {
    if (!cfg || !out) return fail(CSBFS_EINVAL, "csbfs_server_create: null argument");
    *out = nullptr;
    if (cfg->slots < 1 || cfg->slots > 16 || cfg->max_batch < 1 || cfg->max_batch > 64 || cfg->max_levels < 1 ||
        cfg->max_levels > 65536 || cfg->hbm_budget <= 0 || cfg->reserved != 0)
        return fail(CSBFS_EINVAL, "csbfs_server_create: slots 1..16, max_batch 1..64, max_levels 1..65536, "
                                  "hbm_budget > 0, reserved 0");
    csbfs_server *s = new csbfs_server();
    s->cfg = *cfg;
    hipError_t err = hipGetDevice(&s->device);
    for (int k = 0; k < cfg->slots && err == hipSuccess; ++k) {
        hipStream_t st = nullptr;
        err = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (err == hipSuccess) s->streams.push_back(st);
    }
    if (err == hipSuccess) err = hipHostMalloc((void **)&s->mailboxes, sizeof(unsigned long long) * 4 * cfg->slots);
    if (err != hipSuccess) {
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        if (s->mailboxes) (void)hipHostFree(s->mailboxes);
        delete s;
        return hip_fail(err, "csbfs_server_create", __FILE__, __LINE__);
    }
    for (int k = 0; k < cfg->slots; ++k) s->workers.emplace_back(worker, s, k);
    *out = s;
    return CSBFS_OK;
}

extern "C" int csbfs_server_add_graph(csbfs_server *s, const csbfs_graph *g, int32_t *graph_id) {
    if (!s || !g || !graph_id) return fail(CSBFS_EINVAL, "csbfs_server_add_graph: null argument");
    if (g->device != s->device) return fail(CSBFS_EINVAL, "csbfs_server_add_graph: graph on another device");
    GraphState gs;
    gs.g = g;
    gs.batch_bytes = align_up(csbfs_batch_engine_bytes(g, s->cfg.max_batch, s->cfg.max_levels, 0));
    gs.levels_bytes = align_up((int64_t)sizeof(int32_t) * s->cfg.max_batch * g->n);
    csbfs_sizes sz{};
    const csbfs_search_config cfg = single_cfg();
    if (gs.batch_bytes < 0 || csbfs_layout_query(g->n, g->n_tuples, g->P, &cfg, &sz) != CSBFS_OK)
        return fail(CSBFS_EINVAL, "csbfs_server_add_graph: graph sizes not admissible");
    gs.ws_bytes = align_up(sz.workspace_bytes);
    gs.parent_bytes = align_up((int64_t)sizeof(int32_t) * g->n);
    gs.need = gs.batch_bytes + gs.levels_bytes + gs.ws_bytes + gs.parent_bytes;
    if (gs.need > s->cfg.hbm_budget)
        return fail(CSBFS_ENOSPACE, "csbfs_server_add_graph: one block of this graph exceeds the budget");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(CSBFS_EINVAL, "csbfs_server_add_graph: server stopped");
    s->graphs.push_back(std::move(gs));
    *graph_id = (int32_t)s->graphs.size() - 1;
    return CSBFS_OK;
}

extern "C" int csbfs_server_submit(csbfs_server *s, int32_t graph_id, int64_t root, int32_t *level_out, void *stream,
                                   int64_t *request_id) {
    if (!s || !request_id) return fail(CSBFS_EINVAL, "csbfs_server_submit: null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(CSBFS_EINVAL, "csbfs_server_submit: server stopped");
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size())
        return fail(CSBFS_EINVAL, "csbfs_server_submit: unknown graph");
    if (root < 0 || root >= s->graphs[graph_id].g->n) return fail(CSBFS_ERANGE, "csbfs_server_submit: root outside [0, n)");
    hipEvent_t ev = nullptr;
    if (level_out) {
        if (!s->free_events.empty()) {
            ev = s->free_events.back();
            s->free_events.pop_back();
        } else {
            CSBFS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        }
        const hipError_t e = hipEventRecord(ev, as_stream(stream));
        if (e != hipSuccess) {
            s->free_events.push_back(ev);
            return hip_fail(e, "csbfs_server_submit: hipEventRecord", __FILE__, __LINE__);
        }
    }
    const int64_t id = s->next_id++;
    Request &r = s->reqs[id];
    r.out = level_out;
    r.ready = ev;
    r.info.id = id;
    r.info.root = root;
    r.info.graph_id = graph_id;
    r.info.t_submit = now_s();
    s->graphs[graph_id].pending.push_back(id);
    s->n_pending++;
    *request_id = id;
    s->cv_work.notify_one();
    return CSBFS_OK;
}

extern "C" int csbfs_server_wait(csbfs_server *s, int64_t request_id, csbfs_request_info *info) {
    if (!s || !info) return fail(CSBFS_EINVAL, "csbfs_server_wait: null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return fail(CSBFS_EINVAL, "csbfs_server_wait: unknown or collected request");
    s->cv_done.wait(lk, [&] { return s->reqs[request_id].done; });
    *info = s->reqs[request_id].info;
    s->reqs.erase(request_id);
    return CSBFS_OK;
}

extern "C" int csbfs_server_drain(csbfs_server *s) {
    if (!s) return fail(CSBFS_EINVAL, "csbfs_server_drain: null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->n_pending == 0 && s->running == 0; });
    return CSBFS_OK;
}

extern "C" int64_t csbfs_server_graph_bytes(const csbfs_server *s, int32_t graph_id) {
    if (!s) return -1;
    std::lock_guard<std::mutex> lk(const_cast<csbfs_server *>(s)->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size()) return -1;
    return s->graphs[graph_id].need;
}

extern "C" int64_t csbfs_server_bytes_held(const csbfs_server *s) {
    if (!s) return -1;
    std::lock_guard<std::mutex> lk(const_cast<csbfs_server *>(s)->mu);
    return s->held;
}

extern "C" int csbfs_server_free(csbfs_server *s) {
    if (!s) return CSBFS_OK;
    (void)csbfs_server_drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    for (auto &kv : s->blocks) release_block(kv.second, s->streams[kv.first.first]);
    for (hipStream_t st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t ev : s->free_events) (void)hipEventDestroy(ev);
    if (s->mailboxes) (void)hipHostFree(s->mailboxes);
    delete s;
    return CSBFS_OK;
}
