// Serving: a request loop over resident graphs (host runtime; the searches
// are the batched engine's kernels).
//
// One queue of requests in arrival order. Each of `slots` worker threads
// owns a HIP stream; when free it takes the oldest waiting request and up to
// max_batch - 1 more waiting requests for the same graph, runs one batched
// search on its stream, copies each root's levels to the request's buffer
// and marks the requests done. Batch engines (and a max_batch x n result
// buffer) are kept per (slot, graph) and admitted under the HBM budget:
// idle ones are released, least recently used first, when a new one does
// not fit; a batch that still does not fit waits until a running batch ends.
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
    bool done = false;
    csbfs_request_info info{};
};

struct EngineEntry {
    csbfs_batch_engine *eng = nullptr;
    int32_t *levels = nullptr;  // device [max_batch][n]
    int64_t bytes = 0;
    bool busy = false;
    uint64_t last_use = 0;
};

}  // namespace

struct csbfs_server {
    csbfs_server_config cfg{};
    int device = -1;
    std::vector<const csbfs_graph *> graphs;
    std::vector<int64_t> need;  // per graph: engine + result buffer bytes
    std::mutex mu;
    std::condition_variable cv_work;
    std::condition_variable cv_done;
    std::deque<int64_t> pending;
    std::unordered_map<int64_t, Request> reqs;
    int64_t next_id = 0;
    int running = 0;   // batches in flight
    int creating = 0;  // engines being allocated (their bytes already reserved)
    int64_t held = 0;
    uint64_t use_clock = 0;
    std::map<std::pair<int, int>, EngineEntry> engines;  // (slot, graph)
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    bool stop = false;
};

namespace {

void release_entry(EngineEntry &en) {
    if (en.eng) (void)csbfs_batch_engine_free(en.eng);
    if (en.levels) (void)hipFree(en.levels);
    en.eng = nullptr;
    en.levels = nullptr;
}

void finish(csbfs_server *s, const std::vector<int64_t> &ids, int status, int32_t n_levels, int slot,
            double t_start) {
    const double t = now_s();
    for (int64_t id : ids) {
        Request &r = s->reqs[id];
        r.info.status = status;
        r.info.n_levels = n_levels;
        r.info.batch_size = (int32_t)ids.size();
        r.info.slot = slot;
        r.info.t_start = t_start;
        r.info.t_done = t;
        r.done = true;
    }
}

void worker(csbfs_server *s, int slot) {
    (void)hipSetDevice(s->device);
    hipStream_t st = s->streams[slot];
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
        if (s->pending.empty()) {
            if (s->stop) return;
            continue;
        }
        const int64_t first = s->pending.front();
        const int g = s->reqs[first].info.graph_id;
        EngineEntry &en = s->engines[{slot, g}];
        if (!en.eng) {
            const int64_t need = s->need[g];
            // make room: release idle engines, least recently used first
            std::vector<EngineEntry> victims;
            while (s->held + need > s->cfg.hbm_budget) {
                EngineEntry *lru = nullptr;
                for (auto &kv : s->engines) {
                    EngineEntry &c = kv.second;
                    if (c.eng && !c.busy && (!lru || c.last_use < lru->last_use)) lru = &c;
                }
                if (!lru) break;
                s->held -= lru->bytes;
                victims.push_back(*lru);
                lru->eng = nullptr;
                lru->levels = nullptr;
                lru->bytes = 0;
            }
            if (!victims.empty()) {
                lk.unlock();
                for (auto &v : victims) release_entry(v);
                lk.lock();
                continue;  // the queue may have changed meanwhile
            }
            if (s->held + need > s->cfg.hbm_budget) {
                if (s->running == 0 && s->creating == 0) {
                    // nothing will free memory: this graph cannot be served
                    s->pending.pop_front();
                    finish(s, {first}, CSBFS_ENOSPACE, 0, slot, now_s());
                    s->cv_done.notify_all();
                } else {
                    s->cv_work.wait(lk);  // a running batch will release its slot
                }
                continue;
            }
            // reserve, then allocate outside the lock
            s->held += need;
            en.busy = true;
            s->creating++;
            lk.unlock();
            const csbfs_graph *gr = s->graphs[g];
            csbfs_batch_engine *eng = nullptr;
            int32_t *lv = nullptr;
            int rc = csbfs_batch_engine_create(gr, s->cfg.max_batch, s->cfg.max_levels, 0, &eng);
            if (rc == CSBFS_OK && hipMalloc(&lv, sizeof(int32_t) * s->cfg.max_batch * gr->n) != hipSuccess) {
                rc = CSBFS_EHIP;
                lv = nullptr;
            }
            lk.lock();
            s->creating--;
            s->cv_work.notify_all();
            EngineEntry &e2 = s->engines[{slot, g}];
            e2.busy = false;
            if (rc != CSBFS_OK) {
                s->held -= need;
                if (eng) {
                    lk.unlock();
                    (void)csbfs_batch_engine_free(eng);
                    lk.lock();
                }
                if (!s->pending.empty() && s->pending.front() == first) {
                    s->pending.pop_front();
                    finish(s, {first}, rc, 0, slot, now_s());
                    s->cv_done.notify_all();
                }
                continue;
            }
            e2.eng = eng;
            e2.levels = lv;
            e2.bytes = need;
            continue;  // re-pick with the engine in place
        }
        // the batch: the oldest waiting requests of this graph, in order
        std::vector<int64_t> ids;
        std::vector<int64_t> roots;
        for (auto it = s->pending.begin(); it != s->pending.end() && (int)ids.size() < s->cfg.max_batch;) {
            const Request &r = s->reqs[*it];
            if (r.info.graph_id == g) {
                ids.push_back(*it);
                roots.push_back(r.info.root);
                it = s->pending.erase(it);
            } else {
                ++it;
            }
        }
        en.busy = true;
        en.last_use = ++s->use_clock;
        s->running++;
        std::vector<int32_t *> outs;
        for (int64_t id : ids) outs.push_back(s->reqs[id].out);
        csbfs_batch_engine *eng = en.eng;
        int32_t *lv = en.levels;
        const int64_t n = s->graphs[g]->n;
        lk.unlock();

        const double t_start = now_s();
        int32_t nl = 0;
        int rc = csbfs_batch_bfs(eng, roots.data(), (int32_t)roots.size(), lv, nullptr, 0, &nl, st);
        if (rc == CSBFS_OK) {
            for (size_t r = 0; r < outs.size() && rc == CSBFS_OK; ++r)
                if (outs[r] && hipMemcpyAsync(outs[r], lv + (int64_t)r * n, sizeof(int32_t) * n,
                                              hipMemcpyDeviceToDevice, st) != hipSuccess)
                    rc = CSBFS_EHIP;
            if (rc == CSBFS_OK && hipStreamSynchronize(st) != hipSuccess) rc = CSBFS_EHIP;
        }

        lk.lock();
        finish(s, ids, rc, nl, slot, t_start);
        EngineEntry &e3 = s->engines[{slot, g}];
        e3.busy = false;
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
    if (err != hipSuccess) {
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
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
    const int64_t eb = csbfs_batch_engine_bytes(g, s->cfg.max_batch, s->cfg.max_levels, 0);
    const int64_t need = eb + (int64_t)sizeof(int32_t) * s->cfg.max_batch * g->n;
    if (eb < 0 || need > s->cfg.hbm_budget)
        return fail(CSBFS_ENOSPACE, "csbfs_server_add_graph: one engine of this graph exceeds the budget");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(CSBFS_EINVAL, "csbfs_server_add_graph: server stopped");
    s->graphs.push_back(g);
    s->need.push_back(need);
    *graph_id = (int32_t)s->graphs.size() - 1;
    return CSBFS_OK;
}

extern "C" int csbfs_server_submit(csbfs_server *s, int32_t graph_id, int64_t root, int32_t *level_out,
                                   int64_t *request_id) {
    if (!s || !request_id) return fail(CSBFS_EINVAL, "csbfs_server_submit: null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(CSBFS_EINVAL, "csbfs_server_submit: server stopped");
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size())
        return fail(CSBFS_EINVAL, "csbfs_server_submit: unknown graph");
    if (root < 0 || root >= s->graphs[graph_id]->n) return fail(CSBFS_ERANGE, "csbfs_server_submit: root outside [0, n)");
    const int64_t id = s->next_id++;
    Request &r = s->reqs[id];
    r.out = level_out;
    r.info.id = id;
    r.info.root = root;
    r.info.graph_id = graph_id;
    r.info.t_submit = now_s();
    s->pending.push_back(id);
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
    s->cv_done.wait(lk, [&] { return s->pending.empty() && s->running == 0; });
    return CSBFS_OK;
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
    for (auto &kv : s->engines) release_entry(kv.second);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return CSBFS_OK;
}
