// server.cpp -- request server with memory admission and continuous batching.
//
// Requests (rhg_params) are queued in arrival order.  Worker lanes, each with
// its own context and HIP stream, take work as soon as they are free and the
// estimated memory of the work fits the budget next to what is already in
// flight (a request larger than the whole budget runs alone):
//   - when the oldest waiting request is small (n <= GROUP_N), it and the
//     other small requests waiting behind it (up to GROUP_MAX, within the
//     budget) are generated together in seven launches with no host step
//     in between (small_group_spread): the sort and the scans by one
//     workgroup per request, the keys, table rows and window plan, count and
//     emit of the whole group over the chip; one shared output pool, one
//     host synchronisation for the whole group;
//   - otherwise the oldest request runs through the multi-launch path
//     (the rhg_generate path) on the lane's stream.
// Lanes overlap on the device, so requests that arrive while others run are
// admitted as lanes and memory free up.  A small request that outgrows its
// preallocated scratch is rerun on the multi-launch path.  Every result is
// the same edge list rhg_generate returns for the same parameters.
//
// Device memory of the lanes and of the results comes from a cache owned by
// the server (size classes of 1/8 of a power of two), so that the steady
// state calls neither hipMalloc nor hipFree (which synchronises the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/rhg.h"
#include "rhg_internal.h"
#include "rhg_kernels.h"

using namespace rhgi;
using rhgd::BITMAP_WORDS;
using rhgd::UNIT;
using Clock = std::chrono::steady_clock;

namespace {

constexpr int N_LANES = 4;
constexpr int GROUP_MAX = 128;
// Largest request taken into a group: measured at fixed arrival rates (6000
// and 8000 requests/s) between 24576 and 98304 points with the bucket sort
// per request; larger cutoffs raise the saturation rate, and p99 at 8000
// requests/s was lowest at 65536.
constexpr uint64_t GROUP_N = 65536;
static_assert(GROUP_MAX <= rhgk::SMALL_GROUP_MAX, "a group fits the spread launch");

// ---------------------------------------------------------------------------
// Device memory cache.  Blocks are handed out by size class and come back on
// free; idle blocks are kept up to `limit` bytes.  The cache outlives the
// server while graphs from it are alive (the last free deletes it).
// ---------------------------------------------------------------------------
struct DevCache {
    int device = 0;
    std::mutex mu;
    std::multimap<size_t, void *> idle;
    std::unordered_map<void *, size_t> cls;
    uint64_t idle_bytes = 0, limit = 0, live = 0;
    bool server_gone = false;
};

size_t size_class(size_t b) {
    if (b <= 4096) return 4096;
    int e = 63 - __builtin_clzll((unsigned long long)(b - 1));  // 2^e < b <= 2^(e+1)
    const size_t step = ((size_t)1 << e) >> 3;
    return (b + step - 1) / step * step;
}

void cache_release_idle(DevCache *C, std::vector<void *> &out) {
    for (auto &kv : C->idle) {
        out.push_back(kv.second);
        C->cls.erase(kv.second);
    }
    C->idle.clear();
    C->idle_bytes = 0;
}

void *cache_alloc(size_t bytes, void *user) {
    DevCache *C = static_cast<DevCache *>(user);
    const size_t s = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(C->mu);
        auto it = C->idle.find(s);
        if (it != C->idle.end()) {
            void *p = it->second;
            C->idle.erase(it);
            C->idle_bytes -= s;
            C->live++;
            return p;
        }
    }
    (void)hipSetDevice(C->device);
    void *p = nullptr;
    if (hipMalloc(&p, s) != hipSuccess) {
        (void)hipGetLastError();
        std::vector<void *> drop;  // give idle blocks back and try once more
        {
            std::lock_guard<std::mutex> lk(C->mu);
            cache_release_idle(C, drop);
        }
        for (void *q : drop) (void)hipFree(q);
        p = nullptr;
        if (hipMalloc(&p, s) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> lk(C->mu);
    C->cls[p] = s;
    C->live++;
    return p;
}

void cache_free(void *p, void *user) {
    if (!p) return;
    DevCache *C = static_cast<DevCache *>(user);
    bool keep = false, last = false;
    {
        std::lock_guard<std::mutex> lk(C->mu);
        auto it = C->cls.find(p);
        const size_t s = it == C->cls.end() ? 0 : it->second;
        C->live--;
        if (s && !C->server_gone && C->idle_bytes + s <= C->limit) {
            C->idle.emplace(s, p);
            C->idle_bytes += s;
            keep = true;
        } else if (it != C->cls.end()) {
            C->cls.erase(it);
        }
        last = C->server_gone && C->live == 0;
    }
    if (!keep) {
        (void)hipSetDevice(C->device);
        (void)hipFree(p);
    }
    if (last) delete C;
}

// Marks the server gone; the cache goes with the last live block.
void cache_detach(DevCache *C) {
    std::vector<void *> drop;
    bool last;
    {
        std::lock_guard<std::mutex> lk(C->mu);
        C->server_gone = true;
        cache_release_idle(C, drop);
        last = C->live == 0;
    }
    (void)hipSetDevice(C->device);
    for (void *p : drop) (void)hipFree(p);
    if (last) delete C;
}

// ---------------------------------------------------------------------------

struct SReq {
    uint64_t ticket = 0;
    Request rq;
    uint64_t est_bytes = 0;
    bool small = false;
    double kbar = 0.0;
    Clock::time_point t_submit, t_done;
    bool done = false;
    rhg_status status = RHG_OK;
    Graph *result = nullptr;
};

}  // namespace

struct rhg_server {
    int device = 0;
    uint64_t budget = 0;
    DevCache *cache = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<SReq *> queue;
    std::unordered_map<uint64_t, SReq *> reqs;
    uint64_t next_ticket = 1, in_flight = 0, peak = 0, completed = 0, batched = 0, groups = 0, fallbacks = 0;
    bool stop = false;
    std::vector<std::thread> workers;
};

namespace {

// Estimated device memory of one request: its edge list (n kbar / 2 pairs of
// 8 bytes, with 25% headroom for the average-degree approximation) plus the
// per-point work buffers.
uint64_t estimate_bytes(const Request &rq, double kbar) {
    const double edges = (double)rq.n * std::max(kbar, 1.0) / 2.0;
    return (uint64_t)(edges * 8.0 * 1.25) + rq.n * 256ull + (1ull << 20);
}

// Scratch layout of one small request inside a group buffer.
SmallLayout small_layout(uint64_t n, int B, double kbar, bool fp32) {
    const uint64_t nb = (n + 63) / 64;
    // candidates per query are a small multiple of the degree in the model's
    // range; a request that needs more units reruns on the multi-launch path
    const double est_cand = std::min(0.5 * (double)n * (double)(n + 1), 3.0 * (double)n * kbar + 2.0 * (double)n);
    return small_layout_units(n, B, (uint64_t)(est_cand / UNIT) * 2 + nb + 16, fp32);
}

constexpr size_t ZERO_WORDS = 32 + 2 * GROUP_MAX;  // [pool_used, 31 spare, stats 2 x GROUP_MAX]

struct Lane {
    rhg_server *srv = nullptr;
    hipStream_t stream = nullptr;  // non-blocking: lanes run concurrently with each other and the null stream
    Ctx *ctx = nullptr;
    void *arena = nullptr;  // grow-only scratch of small groups (from the cache)
    uint64_t arena_cap = 0;
    rhgk::SmallDesc *h_desc = nullptr;   // pinned, GROUP_MAX
    rhgk::SmallResult *h_res = nullptr;  // pinned, GROUP_MAX
    rhgk::SmallDesc *d_desc = nullptr;
    rhgk::SmallResult *d_res = nullptr;
    unsigned long long *d_zero = nullptr;  // ZERO_WORDS, cleared before every group
    rhgk::QueryArgs *d_qa = nullptr;       // GROUP_MAX: the requests' query arguments (spread launch)
};

void finish(SReq *r, rhg_status st, Graph *g) {
    r->status = st;
    r->result = g;
    r->t_done = Clock::now();
    r->done = true;
}

// Multi-launch path for one request.
void run_one(Lane &L, SReq *r) {
    Graph *g = nullptr;
    rhg_status st = generate(L.ctx, r->rq, true, &g, nullptr);
    std::lock_guard<std::mutex> lk(L.srv->mu);
    finish(r, st, st == RHG_OK ? g : nullptr);
}

// Returns a shared output pool to the cache when its last graph goes.
struct PoolHolder {
    DevCache *cache;
    void *ptr;
    PoolHolder(DevCache *c, void *p) : cache(c), ptr(p) {}
    PoolHolder(const PoolHolder &) = delete;
    PoolHolder &operator=(const PoolHolder &) = delete;
    ~PoolHolder() { cache_free(ptr, cache); }
};

// One launch for a group of small requests.
void run_group(Lane &L, std::vector<SReq *> &grp) {
    Ctx *c = L.ctx;
    DevCache *C = L.srv->cache;
    (void)hipSetDevice(c->device);
    const int G = (int)grp.size();
    std::vector<Plan> plans(G);
    std::vector<SmallLayout> lay(G);
    std::vector<uint64_t> off(G, 0);
    std::vector<int> slot(G, -1);
    uint64_t total = 0, pool_pairs = 0;
    int q = 0;
    for (int k = 0; k < G; ++k) {
        if (describe(grp[k]->rq, plans[k]) != RHG_OK) continue;
        lay[k] = small_layout(plans[k].n, plans[k].B, grp[k]->kbar, plans[k].fp32);
        off[k] = total;
        total += lay[k].bytes;
        pool_pairs += (uint64_t)(1.5 * (double)plans[k].n * grp[k]->kbar / 2.0) + 4096;
        slot[k] = q++;
    }
    rhg_status err = RHG_OK;
    if (total > L.arena_cap) {
        cache_free(L.arena, C);
        L.arena_cap = 0;
        L.arena = cache_alloc(total + total / 4, C);
        if (!L.arena) err = RHG_ENOMEM;
        else L.arena_cap = total + total / 4;
    }
    std::shared_ptr<PoolHolder> pool;
    if (err == RHG_OK && q) {
        void *p = cache_alloc(pool_pairs * sizeof(int2), C);
        if (!p) err = RHG_ENOMEM;
        else pool = std::make_shared<PoolHolder>(C, p);
    }
    hipStream_t st = c->stream;
    if (err == RHG_OK && q) {
        for (int k = 0; k < G; ++k)
            if (slot[k] >= 0)
            {
                small_fill_desc(L.h_desc[slot[k]], plans[k], grp[k]->rq, lay[k], (char *)L.arena + off[k],
                          L.d_zero + 32 + 2 * slot[k]);
                L.h_desc[slot[k]].qa = L.d_qa + slot[k];
            }
        err = hip_status(hipMemsetAsync(L.d_zero, 0, sizeof(unsigned long long) * ZERO_WORDS, st));
        if (err == RHG_OK)
            err = hip_status(hipMemcpyAsync(L.d_desc, L.h_desc, sizeof(rhgk::SmallDesc) * q, hipMemcpyHostToDevice, st));
        if (err == RHG_OK) {
            (void)hipGetLastError();
            rhgk::small_group_spread(L.d_desc, L.d_res, q, (int2 *)pool->ptr, L.d_zero, pool_pairs, st);
            err = hip_status(hipGetLastError());
        }
        if (err == RHG_OK)
            err = hip_status(hipMemcpyAsync(L.h_res, L.d_res, sizeof(rhgk::SmallResult) * q, hipMemcpyDeviceToHost, st));
        if (err == RHG_OK) err = hip_status(hipStreamSynchronize(st));
    }
    std::vector<Graph *> out(G, nullptr);
    std::vector<rhg_status> stv(G, err);
    std::vector<char> fallback(G, 0);
    for (int k = 0; k < G; ++k) {
        if (slot[k] < 0) {
            stv[k] = RHG_EINVAL;
            continue;
        }
        if (err != RHG_OK) continue;
        const rhgk::SmallResult &Z = L.h_res[slot[k]];
        if (Z.status != 0) {
            fallback[k] = 1;
            continue;
        }
        Graph *g = new (std::nothrow) Graph();
        if (!g) {
            stv[k] = RHG_ENOMEM;
            continue;
        }
        g->device = c->device;
        g->rq = grp[k]->rq;
        g->pl = plans[k];
        g->pl.m = Z.m;
        g->pl.candidates = Z.candidates;
        g->pl.windows = Z.windows;
        g->pl.rechecks = Z.rechecks;
        g->pl.emitted = true;
        g->edges = (int32_t *)((int2 *)pool->ptr + Z.out_off);
        g->edge_owner = pool;
        out[k] = g;
        stv[k] = RHG_OK;
    }
    for (int k = 0; k < G; ++k) {
        if (!fallback[k]) continue;
        Graph *g = nullptr;
        stv[k] = generate(c, grp[k]->rq, true, &g, nullptr);
        out[k] = stv[k] == RHG_OK ? g : nullptr;
    }
    pool.reset();  // the graphs hold the pool now (or nobody does)
    std::lock_guard<std::mutex> lk(L.srv->mu);
    for (int k = 0; k < G; ++k) {
        finish(grp[k], stv[k], out[k]);
        L.srv->fallbacks += fallback[k] ? 1 : 0;
    }
    L.srv->batched += (uint64_t)G;
    L.srv->groups += q ? 1 : 0;
}

void worker(rhg_server *S, Lane *L) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_work.wait(lk, [&] {
            if (S->stop) return true;
            if (S->queue.empty()) return false;
            SReq *h = S->queue.front();
            return S->in_flight == 0 || S->in_flight + h->est_bytes <= S->budget;
        });
        if (S->queue.empty()) {
            if (S->stop) break;
            continue;
        }
        std::vector<SReq *> grp;
        uint64_t bytes = 0;
        SReq *h = S->queue.front();
        if (h->small) {
            // the oldest request and the small requests waiting behind it
            for (auto it = S->queue.begin(); it != S->queue.end() && (int)grp.size() < GROUP_MAX;) {
                SReq *r = *it;
                if (!r->small) {
                    ++it;
                    continue;
                }
                if (!grp.empty() && S->in_flight + bytes + r->est_bytes > S->budget) break;
                grp.push_back(r);
                bytes += r->est_bytes;
                it = S->queue.erase(it);
            }
        } else {
            grp.push_back(h);
            bytes = h->est_bytes;
            S->queue.pop_front();
        }
        S->in_flight += bytes;
        S->peak = std::max(S->peak, S->in_flight);
        lk.unlock();
        if (!grp[0]->small) run_one(*L, grp[0]);
        else run_group(*L, grp);
        lk.lock();
        S->in_flight -= bytes;
        S->completed += grp.size();
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

void lane_release(Lane *L, DevCache *C) {
    if (!L) return;
    (void)hipSetDevice(C->device);
    cache_free(L->arena, C);
    if (L->h_desc) (void)hipHostFree(L->h_desc);
    if (L->h_res) (void)hipHostFree(L->h_res);
    if (L->d_desc) (void)hipFree(L->d_desc);
    if (L->d_res) (void)hipFree(L->d_res);
    if (L->d_zero) (void)hipFree(L->d_zero);
    if (L->d_qa) (void)hipFree(L->d_qa);
    rhg_ctx_destroy(reinterpret_cast<rhg_ctx *>(L->ctx));
    if (L->stream) (void)hipStreamDestroy(L->stream);
    delete L;
}

}  // namespace

extern "C" rhg_status rhg_server_create(int device, uint64_t mem_budget_bytes, rhg_server **out) {
    if (!out || mem_budget_bytes == 0) return RHG_EINVAL;
    rhg_server *S = new (std::nothrow) rhg_server();
    if (!S) return RHG_ENOMEM;
    S->device = device;
    S->budget = mem_budget_bytes;
    S->cache = new (std::nothrow) DevCache();
    if (!S->cache) {
        delete S;
        return RHG_ENOMEM;
    }
    S->cache->device = device;
    S->cache->limit = mem_budget_bytes;
    std::vector<Lane *> lanes;
    rhg_status st = RHG_OK;
    for (int k = 0; k < N_LANES && st == RHG_OK; ++k) {
        Lane *L = new (std::nothrow) Lane();
        if (!L) {
            st = RHG_ENOMEM;
            break;
        }
        L->srv = S;
        lanes.push_back(L);
        if (hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            L->stream = nullptr;
            st = RHG_EDEVICE;
            break;
        }
        rhg_ctx *c = nullptr;
        st = rhg_ctx_create(device, L->stream, &c);
        if (st != RHG_OK) break;
        L->ctx = reinterpret_cast<Ctx *>(c);
        st = rhg_ctx_set_allocator(c, cache_alloc, cache_free, S->cache);
        if (st != RHG_OK) break;
        if (hipHostMalloc((void **)&L->h_desc, sizeof(rhgk::SmallDesc) * GROUP_MAX, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void **)&L->h_res, sizeof(rhgk::SmallResult) * GROUP_MAX, hipHostMallocDefault) !=
                hipSuccess ||
            hipMalloc((void **)&L->d_desc, sizeof(rhgk::SmallDesc) * GROUP_MAX) != hipSuccess ||
            hipMalloc((void **)&L->d_res, sizeof(rhgk::SmallResult) * GROUP_MAX) != hipSuccess ||
            hipMalloc((void **)&L->d_zero, sizeof(unsigned long long) * ZERO_WORDS) != hipSuccess ||
            hipMalloc((void **)&L->d_qa, sizeof(rhgk::QueryArgs) * GROUP_MAX) != hipSuccess) {
            (void)hipGetLastError();
            st = RHG_ENOMEM;
        }
    }
    if (st != RHG_OK) {
        for (Lane *L : lanes) lane_release(L, S->cache);
        cache_detach(S->cache);
        delete S;
        return st;
    }
    for (Lane *L : lanes) S->workers.emplace_back([S, L] {
        worker(S, L);
        lane_release(L, S->cache);
    });
    *out = S;
    return RHG_OK;
}

// Validated request with its sizing degree and admission charge.
static rhg_status admit_params(const rhg_params *params, Request &rq, double &kbar, uint64_t &bytes) {
    rhg_status st = request_from_params(params, rq);
    if (st == RHG_OK) {
        Plan pl;
        st = describe(rq, pl);
    }
    if (st != RHG_OK) return st;
    // average degree used for sizing: the requested one, or the one R implies
    kbar = params->R > 0.0 ? expected_degree(rq.n, rq.alpha, rq.R) : params->kbar;
    if (!std::isfinite(kbar) || kbar < 1.0) kbar = 1.0;
    kbar = std::min(kbar, (double)rq.n);
    bytes = estimate_bytes(rq, kbar);
    return RHG_OK;
}

extern "C" rhg_status rhg_server_estimate_bytes(const rhg_params *params, uint64_t *bytes) {
    if (!params || !bytes) return RHG_EINVAL;
    Request rq;
    double kbar = 0.0;
    uint64_t b = 0;
    rhg_status st = admit_params(params, rq, kbar, b);
    if (st == RHG_OK) *bytes = b;
    return st;
}

extern "C" rhg_status rhg_server_submit(rhg_server *S, const rhg_params *params, uint64_t *ticket) {
    if (!S || !params || !ticket) return RHG_EINVAL;
    SReq *r = new (std::nothrow) SReq();
    if (!r) return RHG_ENOMEM;
    rhg_status st = admit_params(params, r->rq, r->kbar, r->est_bytes);
    if (st != RHG_OK) {
        delete r;
        return st;
    }
    r->small = r->rq.n <= GROUP_N;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
        delete r;
        return RHG_EINVAL;
    }
    r->ticket = S->next_ticket++;
    S->reqs[r->ticket] = r;
    S->queue.push_back(r);
    *ticket = r->ticket;
    S->cv_work.notify_one();
    return RHG_OK;
}

extern "C" rhg_status rhg_server_wait(rhg_server *S, uint64_t ticket, int timeout_ms, rhg_graph **out,
                                      double *latency_ms) {
    if (!S || !out) return RHG_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return RHG_EINVAL;
    SReq *r = it->second;
    if (timeout_ms < 0) {
        S->cv_done.wait(lk, [&] { return r->done; });
    } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return r->done; })) {
        return RHG_EBUSY;
    }
    S->reqs.erase(it);
    lk.unlock();
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    rhg_status st = r->status;
    *out = st == RHG_OK ? reinterpret_cast<rhg_graph *>(r->result) : nullptr;
    delete r;
    return st;
}

extern "C" rhg_status rhg_server_counters(rhg_server *S, rhg_server_stats *out) {
    if (!S || !out) return RHG_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    out->completed = S->completed;
    out->batched = S->batched;
    out->groups = S->groups;
    out->fallbacks = S->fallbacks;
    out->peak_bytes = S->peak;
    out->budget_bytes = S->budget;
    return RHG_OK;
}

extern "C" void rhg_server_destroy(rhg_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    for (auto &t : S->workers) t.join();
    for (auto &kv : S->reqs) {
        if (kv.second->result) graph_release(kv.second->result);
        delete kv.second;
    }
    cache_detach(S->cache);
    delete S;
}
