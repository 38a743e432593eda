// Served form: a request loop on its own host thread with continuous batching.
//
// Graphs are registered once and stay resident. A query (graph id, target set) goes
// through: queued -> admission, when its device bytes fit the free part of the HBM
// budget: Build_SK's first phase on the device (P', frontiers, per-part counts), the
// query's block, the second phase (renumbering, intra-part CSR, cut arcs) -> Dijkstra_SK
// as one resident launch on a side stream -> skeleton assembly -> Brandes_SK +
// Centrality as one resident launch on a side stream -> scores copied to the host.
// Launches of different queries overlap on the device (the side streams), and a
// query's memory returns to the pool as soon as it finishes. With BC_ENGINE_ONLY a
// query's groups go into the shared multi-group engine instead, which iterates over
// all installed groups of all such queries. Each query's arithmetic is the same as
// when it runs alone (its groups hold the same sources in the same order), so its
// result does not depend on what else is in flight.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "engine.h"
#include "graph.h"
#include "skbuild.h"

namespace bcpp {

// First-fit allocator over one device buffer (the HBM budget).
struct Pool {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    std::atomic<size_t> peak{0};  // read by bc_server_stats_get on other threads
    std::map<size_t, size_t> free_;  // offset -> size

    void init(char* b, size_t c) {
        base = b;
        cap = c;
        free_.clear();
        free_[0] = c;
        used = 0;
        peak = 0;
    }
    static size_t round(size_t x) { return (x + 4095) & ~size_t(4095); }
    bool alloc(size_t bytes, size_t* off) {
        bytes = round(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used += bytes;
            if (used > peak.load()) peak = used;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round(std::max<size_t>(bytes, 1));
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Block {
    size_t off = 0, size = 0;
    bool live = false;
};

// Q_RDSK / Q_RES: Dijkstra_SK, or Brandes_SK + Centrality, running as resident
// launches on a side stream (Q_DSK / Q_BSK: the same on the shared engine)
enum { Q_QUEUED = 0, Q_DSK = 1, Q_BSK = 2, Q_DONE = 3, Q_FAILED = 4, Q_RES = 5, Q_RDSK = 6 };

struct Query {
    uint64_t ticket = 0;
    int32_t gid = 0;
    std::vector<int32_t> S;
    uint32_t flags = 0;
    // written by the loop thread, read by bc_query_poll / bc_server_stats_get
    std::atomic<int> state{Q_QUEUED};
    int status = BC_OK;
    std::string err;
    std::vector<double> result;
    std::unique_ptr<SkBuild> build;
    std::unique_ptr<bc_skeleton> sk;
    std::vector<int32_t> slots;
    std::vector<GroupDesc> groups;
    Block tmp, store, bsk;
    Arena a_tmp, a_store, a_bsk;
    // Q_RES: completion event, error word and scores on the device
    hipEvent_t ev = nullptr;
    uint32_t* d_err = nullptr;
    double* d_out = nullptr;
    std::chrono::steady_clock::time_point t_submit, t_done;
};

}  // namespace bcpp

using namespace bcpp;

struct bc_server {
    std::mutex mu;
    std::condition_variable cv;
    std::thread th;
    bool stop = false;
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;
    int32_t max_inflight = 64;
    // registered graphs
    std::vector<std::unique_ptr<bc_graph>> graphs;
    std::vector<std::vector<int32_t>> parts;
    std::vector<int32_t> ks;
    std::vector<std::unique_ptr<DskCache>> caches;
    std::atomic<int64_t> cache_bytes{0}, dsk_cached{0}, dsk_run{0};
    // queries
    uint64_t next_ticket = 1;
    std::deque<uint64_t> incoming;  // submitted, not yet seen by the loop
    std::map<uint64_t, std::unique_ptr<Query>> queries;
    int64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_iters = 0;
    std::vector<double> lat_ms;
    // device side (used by the loop thread only)
    char* d_pool = nullptr;
    Pool pool;
    Arena engine_mem;
    Engine eng;
    int32_t slot_cap = 0;
    int64_t pos_cap = 0, pos_used = 0;
    std::vector<GroupDesc> slot_desc;
    std::vector<uint64_t> slot_owner;  // ticket, 0 = free
    GroupDyn* h_dyn = nullptr;
    int32_t slot_hi = 0;  // slots [slot_hi, slot_cap) have never been used
    int run_error = BC_OK;
    // side streams of the resident launches (round robin), a stream for their result
    // copies, and the event that orders a launch after its skeleton's assembly
    static constexpr int NRS = 4;
    hipStream_t rs[NRS] = {};
    unsigned rnext = 0;
    hipStream_t cs = nullptr;
    hipEvent_t asm_ev = nullptr;

    ~bc_server();
};

namespace bcpp {

static int64_t positions_of(const GroupDesc& G) {
    return std::max<int64_t>((int64_t)G.hi - G.lo, (G.flags & GF_CENT) ? G.tn : 0);
}

static bool alloc_block(bc_server* sv, size_t bytes, Block& b, Arena& a) {
    size_t off = 0;
    if (!sv->pool.alloc(bytes, &off)) return false;
    b.off = off;
    b.size = bytes;
    b.live = true;
    a = Arena::view(sv->pool.base + off, Pool::round(bytes));
    return true;
}

static void free_block(bc_server* sv, Block& b, Arena& a) {
    if (!b.live) return;
    sv->pool.release(b.off, b.size);
    b.live = false;
    a = Arena();
}

static hipStream_t next_side_stream(bc_server* sv) { return sv->rs[sv->rnext++ % bc_server::NRS]; }

static int free_slots(bc_server* sv) {
    int c = 0;
    for (auto o : sv->slot_owner) c += o == 0;
    return c;
}

// Install q->groups into free slots and rebuild the scan-chunk table.
static int install_groups(bc_server* sv, Query* q) {
    q->slots.clear();
    int32_t at = 0;
    for (auto& G : q->groups) {
        while (at < sv->slot_cap && sv->slot_owner[at]) ++at;
        if (at >= sv->slot_cap) return fail(BC_E_NOMEM, "server: no free group slot");
        sv->slot_owner[at] = q->ticket;
        sv->slot_desc[at] = G;
        q->slots.push_back(at);
        sv->pos_used += positions_of(G);
        sv->slot_hi = std::max(sv->slot_hi, at + 1);
        ++at;
    }
    std::vector<int32_t> live;
    for (int32_t i = 0; i < sv->slot_hi; ++i)
        if (sv->slot_owner[i]) live.push_back(i);
    return sv->eng.install_at(q->groups.data(), q->slots.data(), (int32_t)q->groups.size(), sv->slot_desc,
                              live);
}

static void release_slots(bc_server* sv, Query* q) {
    for (int32_t s : q->slots) {
        sv->slot_owner[s] = 0;
        sv->pos_used -= positions_of(sv->slot_desc[s]);
    }
    q->slots.clear();
}

static void drop_event(Query* q) {
    if (q->ev) (void)hipEventDestroy(q->ev);
    q->ev = nullptr;
}

static void fail_query(bc_server* sv, Query* q, int code, const std::string& msg) {
    drop_event(q);
    release_slots(sv, q);
    free_block(sv, q->tmp, q->a_tmp);
    free_block(sv, q->bsk, q->a_bsk);
    free_block(sv, q->store, q->a_store);
    q->sk.reset();
    q->build.reset();
    std::lock_guard<std::mutex> lk(sv->mu);
    q->state = Q_FAILED;
    q->status = code;
    q->err = msg;
    sv->n_failed++;
}

static void finish_query(bc_server* sv, Query* q, std::vector<double>&& res) {
    drop_event(q);
    release_slots(sv, q);
    free_block(sv, q->tmp, q->a_tmp);
    free_block(sv, q->bsk, q->a_bsk);
    free_block(sv, q->store, q->a_store);
    q->sk.reset();
    q->build.reset();
    const auto t = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(sv->mu);
    q->result = std::move(res);
    q->t_done = t;
    q->state = Q_DONE;
    sv->n_completed++;
    sv->lat_ms.push_back(std::chrono::duration<double, std::milli>(t - q->t_submit).count());
}

// Dijkstra_SK finished (or was empty): assemble the skeleton, then start Brandes_SK.
// Returns BC_E_AGAIN when the Brandes_SK memory is not free yet. *started tells
// whether Brandes_SK groups were installed; when it is false after BC_OK the query has
// been completed (and may be gone: the caller must not touch it again).
static int start_bsk(bc_server* sv, Query* q, bool* started) {
    *started = false;
    hipStream_t s = sv->stream;
    if (q->ev) {
        (void)hipEventDestroy(q->ev);
        q->ev = nullptr;
    }
    if (!q->sk) {
        auto sk = std::make_unique<bc_skeleton>();
        BC_TRY(q->build->assemble(q->a_tmp, s, sk.get(), [&](size_t bytes, Arena*& A) -> int {
            if (!alloc_block(sv, bytes, q->store, q->a_store))
                return fail(BC_E_NOMEM, "server: skeleton does not fit the budget");
            A = &q->a_store;
            return BC_OK;
        }));
        q->sk = std::move(sk);
        free_block(sv, q->tmp, q->a_tmp);
    }
    bc_skeleton* sk = q->sk.get();
    const int32_t n = sk->n;
    const int32_t nsrc = (int32_t)sk->h_src.size();
    if (getenv("BCPP_DEBUG"))
        fprintf(stderr, "server: query %llu skeleton n_sk %d n_int %d arcs %lld sources %d\n",
                (unsigned long long)q->ticket, sk->n_sk, sk->n_int, (long long)sk->m_arcs, nsrc);
    if (nsrc < 2 || sk->n_sk == 0) {
        finish_query(sv, q, std::vector<double>(n, 0.0));
        return BC_OK;
    }
    if (!(q->flags & BC_ENGINE_ONLY) && resident_takes(sk->n_sk)) {
        // one LDS-resident launch on a side stream; the loop polls its event. Every
        // host-to-device copy goes on the loop's own stream (idle here), so nothing
        // below waits for a kernel.
        std::vector<GroupDesc> groups = resident_bsk_groups(sk);
        size_t need = resident_launch_bytes(groups.size()) + 2 * (groups.size() * 8 + 256) +
                      (size_t)n * 8 + 256 + 4096;
        for (const GroupDesc& G : groups) need += resident_group_bytes(G);
        // the query holds its skeleton store meanwhile: if both never fit together it
        // can never start, whatever else finishes
        if (need + (q->store.live ? Pool::round(q->store.size) : 0) > sv->pool.cap)
            return fail(BC_E_NOMEM, "server: query needs more than the configured budget");
        if (!alloc_block(sv, need, q->bsk, q->a_bsk)) return BC_E_AGAIN;
        for (GroupDesc& G : groups)
            if (!resident_alloc(q->a_bsk, G)) return fail(BC_E_NOMEM, "server: block too small");
        q->groups = std::move(groups);
        ResidentLaunch L;
        ReducePtrs R;
        BC_TRY(resident_upload(s, q->a_bsk, q->groups, &L));
        BC_TRY(reduce_upload(s, q->a_bsk, q->groups, &R));
        q->d_err = L.d_err;
        q->d_out = q->a_bsk.take<double>(std::max(n, 1));
        if (!q->d_out) return fail(BC_E_NOMEM, "server: block too small");
        BC_HIP(hipEventCreateWithFlags(&q->ev, hipEventDisableTiming));
        hipStream_t r = next_side_stream(sv);
        BC_HIP(hipEventRecord(sv->asm_ev, s));
        BC_HIP(hipStreamWaitEvent(r, sv->asm_ev, 0));
        // once a launch is enqueued, a later failure waits for the side stream before
        // the caller releases the blocks the launch uses
        const double scale = (q->flags & BC_ORDERED) ? 1.0 : 0.5;
        int rc = resident_launch(r, L);
        if (rc == BC_OK)
            rc = reduce_launch(r, R, n, nullptr, nullptr, sk->d_out_idx, sk->d_out_which, scale, q->d_out, false);
        if (rc == BC_OK && hipEventRecord(q->ev, r) != hipSuccess)
            rc = fail(BC_E_DEVICE, "server: event record failed");
        if (rc != BC_OK) {
            (void)hipStreamSynchronize(r);
            return rc;
        }
        q->state = Q_RES;
        *started = true;
        return BC_OK;
    }
    q->groups = bsk_groups(sk, sk->h_src.data(), nsrc, 0, sk->n_sk, 0, sk->n_int);
    const int64_t steps = max_steps_bound(sk->n_sk, LANES, sk->max_dist);
    // group states, then finish_bsk's chunk table, score vector and reduction pointers
    size_t need = 0, chunks = 0;
    int64_t pos = 0;
    for (auto& G : q->groups) {
        need += group_bytes(G, steps) + 512;
        pos += positions_of(G);
        chunks += ((size_t)(G.hi - G.lo) + 255) / 256;
    }
    need += 2 * (chunks * 4 + 256) + (size_t)n * 8 + 256 + 2 * (q->groups.size() * 8 + 256) + 4096;
    if (need > sv->pool.cap || (int32_t)q->groups.size() > sv->slot_cap || pos > sv->pos_cap)
        return fail(BC_E_NOMEM, "server: query needs more than the configured budget");
    if ((int32_t)q->groups.size() > free_slots(sv) || sv->pos_used + pos > sv->pos_cap ||
        !alloc_block(sv, need, q->bsk, q->a_bsk))
        return BC_E_AGAIN;
    for (auto& G : q->groups)
        if (!group_alloc(q->a_bsk, G, steps)) return fail(BC_E_NOMEM, "server: block too small");
    BC_TRY(install_groups(sv, q));
    q->state = Q_BSK;
    *started = true;
    return BC_OK;
}

static int finish_bsk(bc_server* sv, Query* q) {
    hipStream_t s = sv->stream;
    bc_skeleton* sk = q->sk.get();
    const int32_t n = sk->n;
    // per-node sums of the lanes' dependencies, for this query's groups only
    std::vector<int32_t> cg, co;
    for (int32_t j = 0; j < (int32_t)q->slots.size(); ++j) {
        const GroupDesc& G = q->groups[j];
        for (int64_t off = 0; off < (int64_t)G.hi - G.lo; off += 256) {
            cg.push_back(q->slots[j]);
            co.push_back((int32_t)off);
        }
    }
    int32_t* d_cg = q->a_bsk.take<int32_t>(std::max<size_t>(cg.size(), 1));
    int32_t* d_co = q->a_bsk.take<int32_t>(std::max<size_t>(co.size(), 1));
    double* d_out = q->a_bsk.take<double>(std::max(n, 1));
    if (!d_cg || !d_co || !d_out) return fail(BC_E_NOMEM, "server: block too small");
    BC_HIP(hipMemcpyAsync(d_cg, cg.data(), cg.size() * 4, hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(d_co, co.data(), co.size() * 4, hipMemcpyHostToDevice, s));
    BC_TRY(lane_sum(s, sv->eng.d_desc, d_cg, d_co, (int64_t)cg.size()));
    const double scale = (q->flags & BC_ORDERED) ? 1.0 : 0.5;
    BC_TRY(reduce_scores(s, q->a_bsk, q->groups, n, nullptr, nullptr, sk->d_out_idx, sk->d_out_which,
                         scale, d_out, false));
    std::vector<double> res(n);
    BC_HIP(hipMemcpyAsync(res.data(), d_out, (size_t)n * 8, hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    if (getenv("BCPP_DEBUG")) {
        double tot = 0;
        for (double x : res) tot += x;
        std::vector<GroupDyn> dy(q->slots.size());
        for (size_t j = 0; j < q->slots.size(); ++j) dy[j] = sv->h_dyn[q->slots[j]];
        fprintf(stderr, "server: query %llu done, %zu groups, sum %g, nrec0 %d\n",
                (unsigned long long)q->ticket, q->groups.size(), tot, dy.empty() ? -1 : dy[0].nrec);
    }
    finish_query(sv, q, std::move(res));
    return BC_OK;
}

// A resident launch completed: read its error word and scores.
static int finish_res(bc_server* sv, Query* q) {
    const int32_t n = q->sk->n;
    uint32_t err = 0;
    std::vector<double> res(n);
    BC_HIP(hipMemcpyAsync(&err, q->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, sv->cs));
    BC_HIP(hipMemcpyAsync(res.data(), q->d_out, (size_t)n * 8, hipMemcpyDeviceToHost, sv->cs));
    BC_HIP(hipStreamSynchronize(sv->cs));
    if (err & ERR_OVERFLOW) return fail(BC_E_OVERFLOW, "a shortest-path count reached 2^64");
    finish_query(sv, q, std::move(res));
    return BC_OK;
}

static int admit_prepared(bc_server* sv, Query* q);

// Admission: Build_SK's first phase on the device (into the graph's scratch, which the
// next query's build reuses, so a query that cannot be admitted now drops its build and
// redoes it later), then the query's block and the second phase.
static int admit(bc_server* sv, Query* q) {
    const bc_graph* g = nullptr;
    const int32_t* part = nullptr;
    int32_t k = 0;
    {
        // graph objects and partition buffers never move once registered
        std::lock_guard<std::mutex> lk(sv->mu);
        g = sv->graphs[q->gid].get();
        part = sv->parts[q->gid].data();
        k = sv->ks[q->gid];
    }
    q->build = std::make_unique<SkBuild>();
    int rc = q->build->prepare(g, part, k, q->S.data(), (int32_t)q->S.size(), false);
    if (rc == BC_OK) rc = admit_prepared(sv, q);
    if (rc == BC_E_AGAIN) q->build.reset();
    return rc;
}

static int admit_prepared(bc_server* sv, Query* q) {
    SkBuild& b = *q->build;
    q->groups = b.groups;
    bool res = !(q->flags & BC_ENGINE_ONLY);
    for (auto& G : q->groups) res = res && resident_takes((int64_t)G.hi - G.lo);
    if (res) {
        // parts without a target take their Dijkstra_SK lanes from the graph's cache
        std::vector<uint8_t> preset(b.groups.size(), 0);
        const DskCache* C = nullptr;
        const int32_t* part = nullptr;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            C = sv->caches[q->gid].get();
            part = sv->parts[q->gid].data();
        }
        // (BCPP_SERVE_CACHE=0 runs every part's Dijkstra_SK, for comparisons)
        static const bool use_cache = [] {
            const char* e = getenv("BCPP_SERVE_CACHE");
            return !(e && e[0] == '0');
        }();
        if (use_cache && C && C->ok) dsk_preset_from_cache(b, *C, part, preset);
        // Dijkstra_SK as one resident launch on a side stream; parts larger than LDS
        // keep their one-source state in the query's block. A query without
        // Dijkstra_SK groups launches nothing and goes on to Brandes_SK when polled
        // (on the engine it would make the loop step the engine for nothing).
        size_t need = b.temp_bytes() + resident_launch_bytes(q->groups.size()) + 8192;
        for (auto& G : q->groups)
            if ((int64_t)G.hi - G.lo > resident_max_range()) need += (size_t)(G.hi - G.lo) * 12 + 512;
        if (need > sv->pool.cap) return fail(BC_E_NOMEM, "server: query needs more than the configured budget");
        if (!alloc_block(sv, need, q->tmp, q->a_tmp)) return BC_E_AGAIN;
        BC_TRY(b.upload(q->a_tmp, sv->stream));
        for (auto& G : b.groups) {
            if ((int64_t)G.hi - G.lo <= resident_max_range()) continue;
            G.gdist = q->a_tmp.take<uint32_t>((size_t)(G.hi - G.lo));
            G.gsig = q->a_tmp.take<uint64_t>((size_t)(G.hi - G.lo));
            if (!G.gdist || !G.gsig) return fail(BC_E_NOMEM, "server: block too small");
        }
        q->groups.clear();
        for (size_t i = 0; i < b.groups.size(); ++i)
            if (!preset[i]) q->groups.push_back(b.groups[i]);
        sv->dsk_cached += (int64_t)(b.groups.size() - q->groups.size());
        sv->dsk_run += (int64_t)q->groups.size();
        ResidentLaunch L;
        BC_TRY(resident_upload(sv->stream, q->a_tmp, q->groups, &L));
        q->d_err = L.d_err;
        BC_HIP(hipEventCreateWithFlags(&q->ev, hipEventDisableTiming));
        hipStream_t r = next_side_stream(sv);
        BC_HIP(hipEventRecord(sv->asm_ev, sv->stream));
        BC_HIP(hipStreamWaitEvent(r, sv->asm_ev, 0));
        int rc = resident_launch(r, L);
        if (rc == BC_OK && hipEventRecord(q->ev, r) != hipSuccess)
            rc = fail(BC_E_DEVICE, "server: event record failed");
        if (rc != BC_OK) {
            (void)hipStreamSynchronize(r);
            return rc;
        }
        q->state = Q_RDSK;
        return BC_OK;
    }
    const size_t need = b.temp_bytes() + 4096;
    int64_t pos = 0;
    for (auto& G : q->groups) pos += positions_of(G);
    if (need > sv->pool.cap || (int32_t)q->groups.size() > sv->slot_cap || pos > sv->pos_cap)
        return fail(BC_E_NOMEM, "server: query needs more than the configured budget");
    if ((int32_t)q->groups.size() > free_slots(sv) || sv->pos_used + pos > sv->pos_cap ||
        !alloc_block(sv, need, q->tmp, q->a_tmp))
        return BC_E_AGAIN;
    BC_TRY(b.upload(q->a_tmp, sv->stream));
    q->groups = b.groups;  // now with device pointers
    // a query with no Dijkstra_SK work holds no slots: the loop sees it finished
    // at its next step and moves it on to Brandes_SK
    if (!q->groups.empty()) BC_TRY(install_groups(sv, q));
    q->state = Q_DSK;
    return BC_OK;
}


static void server_loop(bc_server* sv) {
    (void)hipSetDevice(sv->device);
    std::vector<Query*> active;     // admitted, not finished
    std::deque<Query*> waiting;     // not yet admitted
    std::vector<Query*> bsk_wait;   // Dijkstra_SK done, Brandes_SK memory not free yet
    std::vector<Query*> res_run;    // resident launches in flight
    std::vector<Query*> res_run_new;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (active.empty() && waiting.empty() && bsk_wait.empty() && sv->incoming.empty() && !sv->stop)
                sv->cv.wait_for(lk, res_run.empty() ? std::chrono::microseconds(20000)
                                                    : std::chrono::microseconds(200));
            if (sv->stop) break;
            while (!sv->incoming.empty()) {
                auto it = sv->queries.find(sv->incoming.front());
                sv->incoming.pop_front();
                if (it != sv->queries.end()) waiting.push_back(it->second.get());
            }
        }
        // finished resident launches
        for (size_t i = 0; i < res_run.size();) {
            Query* q = res_run[i];
            const hipError_t e = hipEventQuery(q->ev);
            if (e == hipErrorNotReady) {
                ++i;
                continue;
            }
            res_run.erase(res_run.begin() + i);
            if (e != hipSuccess) {
                fail_query(sv, q, BC_E_DEVICE, "server: resident launch failed");
                continue;
            }
            if (q->state == Q_RES) {
                const int rc = finish_res(sv, q);
                if (rc != BC_OK) fail_query(sv, q, rc, bc_last_error());
                continue;
            }
            // Dijkstra_SK done: check its overflow flag, then assembly and Brandes_SK
            uint32_t err = 0;
            if (hipMemcpyAsync(&err, q->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, sv->cs) != hipSuccess ||
                hipStreamSynchronize(sv->cs) != hipSuccess) {
                fail_query(sv, q, BC_E_DEVICE, "server: device copy failed");
                continue;
            }
            if (err & ERR_OVERFLOW) {
                fail_query(sv, q, BC_E_OVERFLOW, "a shortest-path count reached 2^64");
                continue;
            }
            bool started = false;
            const int rc = start_bsk(sv, q, &started);
            if (rc == BC_E_AGAIN) {
                bsk_wait.push_back(q);
                continue;
            }
            if (rc != BC_OK)
                fail_query(sv, q, rc, bc_last_error());
            else if (started)
                (q->state == Q_RES ? res_run_new : active).push_back(q);
        }
        res_run.insert(res_run.end(), res_run_new.begin(), res_run_new.end());
        res_run_new.clear();
        // Brandes_SK starts for queries whose skeleton is ready (they go first)
        for (size_t i = 0; i < bsk_wait.size();) {
            Query* q = bsk_wait[i];
            bool started = false;
            int rc = start_bsk(sv, q, &started);
            if (rc == BC_E_AGAIN) {
                ++i;
                continue;
            }
            bsk_wait.erase(bsk_wait.begin() + i);
            if (rc != BC_OK)
                fail_query(sv, q, rc, bc_last_error());
            else if (started)
                (q->state == Q_RES ? res_run : active).push_back(q);
        }
        // admission of new queries, in arrival order, while memory and slots allow
        while (bsk_wait.empty() && !waiting.empty() &&
               (int32_t)(active.size() + res_run.size()) < sv->max_inflight) {
            Query* q = waiting.front();
            int rc = admit(sv, q);
            if (rc == BC_E_AGAIN) break;
            waiting.pop_front();
            if (rc != BC_OK) {
                fail_query(sv, q, rc, bc_last_error());
                continue;
            }
            if (q->state == Q_RDSK)
                res_run.push_back(q);
            else if (q->state == Q_DSK || q->state == Q_BSK)
                active.push_back(q);
        }
        // nothing can make progress: no launch in flight and no engine group installed,
        // so no memory will be freed, and the oldest skeleton waiting for its Brandes_SK
        // memory cannot get it; it fails, and its store goes back to the pool
        if (active.empty() && res_run.empty() && !bsk_wait.empty()) {
            Query* q = bsk_wait.front();
            bsk_wait.erase(bsk_wait.begin());
            fail_query(sv, q, BC_E_NOMEM, "server: Brandes_SK state does not fit the budget");
            continue;
        }
        if (active.empty()) continue;
        // one engine step for every installed group of every admitted query
        if (sv->eng.iterate(2) != BC_OK ||
            hipMemcpyAsync(sv->h_dyn, sv->eng.d_dyn, sizeof(GroupDyn) * std::max(sv->slot_hi, 1),
                           hipMemcpyDeviceToHost, sv->stream) != hipSuccess ||
            hipStreamSynchronize(sv->stream) != hipSuccess) {
            for (Query* q : active) fail_query(sv, q, BC_E_DEVICE, "server: device step failed");
            active.clear();
            continue;
        }
        sv->n_iters += 2;
        // queries that start Brandes_SK below are checked from the next step on: the
        // phase snapshot read above predates their groups
        std::vector<Query*> started_now;
        for (size_t i = 0; i < active.size();) {
            Query* q = active[i];
            bool done = true;
            uint32_t err = 0;
            for (int32_t s : q->slots) {
                done = done && sv->h_dyn[s].phase == PH_DONE;
                err |= sv->h_dyn[s].err;
            }
            if (!done) {
                ++i;
                continue;
            }
            active.erase(active.begin() + i);
            if (err) {
                fail_query(sv, q, (err & ERR_OVERFLOW) ? BC_E_OVERFLOW : BC_E_DEVICE,
                           (err & ERR_OVERFLOW) ? "a shortest-path count reached 2^64" : "engine error");
                continue;
            }
            int rc = BC_OK;
            if (q->state == Q_DSK) {
                release_slots(sv, q);
                bool started = false;
                rc = start_bsk(sv, q, &started);
                if (rc == BC_E_AGAIN) {
                    bsk_wait.push_back(q);
                    continue;
                }
                if (rc == BC_OK && started) (q->state == Q_RES ? res_run : started_now).push_back(q);
            } else {
                rc = finish_bsk(sv, q);
            }
            if (rc != BC_OK) fail_query(sv, q, rc, bc_last_error());
        }
        active.insert(active.end(), started_now.begin(), started_now.end());
    }
    // shut down: let launches in flight end before their memory is released, then fail
    // whatever is left
    for (hipStream_t r : sv->rs)
        if (r) (void)hipStreamSynchronize(r);
    for (Query* q : res_run) fail_query(sv, q, BC_E_DEVICE, "server stopped");
    for (Query* q : active) fail_query(sv, q, BC_E_DEVICE, "server stopped");
    for (Query* q : bsk_wait) fail_query(sv, q, BC_E_DEVICE, "server stopped");
    for (Query* q : waiting) fail_query(sv, q, BC_E_DEVICE, "server stopped");
}

}  // namespace bcpp

bc_server::~bc_server() {
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv.notify_all();
    if (th.joinable()) th.join();
    if (stream) (void)hipStreamSynchronize(stream);
    for (hipStream_t r : rs)
        if (r) (void)hipStreamSynchronize(r);
    engine_mem.release();
    if (d_pool) (void)hipFree(d_pool);
    if (h_dyn) (void)hipHostFree(h_dyn);
    if (eng.h_ctr) (void)hipHostFree(eng.h_ctr);
    graphs.clear();
    for (hipStream_t r : rs)
        if (r) (void)hipStreamDestroy(r);
    if (cs) (void)hipStreamDestroy(cs);
    if (asm_ev) (void)hipEventDestroy(asm_ev);
    if (stream) (void)hipStreamDestroy(stream);
}

extern "C" {

int bc_server_create(size_t hbm_budget_bytes, int32_t max_inflight, bc_server** out) {
    if (!out) return fail(BC_E_INVAL, "null output handle");
    *out = nullptr;
    if (hbm_budget_bytes < ((size_t)64 << 20)) return fail(BC_E_INVAL, "budget below 64 MiB");
    if (max_inflight < 1) return fail(BC_E_INVAL, "max_inflight must be >= 1");
    auto sv = std::make_unique<bc_server>();
    sv->budget = hbm_budget_bytes;
    sv->max_inflight = max_inflight;
    BC_HIP(hipGetDevice(&sv->device));
    BC_HIP(hipStreamCreate(&sv->stream));
    for (hipStream_t& r : sv->rs) BC_HIP(hipStreamCreate(&r));
    BC_HIP(hipStreamCreate(&sv->cs));
    BC_HIP(hipEventCreateWithFlags(&sv->asm_ev, hipEventDisableTiming));
    // engine: group slots and scan positions sized from the budget
    sv->slot_cap = 4096;
    sv->pos_cap = (int64_t)std::max<size_t>(hbm_budget_bytes / 512, (size_t)1 << 20);
    BC_TRY(sv->engine_mem.reserve(engine_bytes(sv->slot_cap, sv->pos_cap)));
    BC_TRY(sv->eng.setup(sv->engine_mem, sv->stream, sv->slot_cap, sv->pos_cap));
    // empty slots: phase DONE
    std::vector<GroupDyn> dy(sv->slot_cap);
    std::memset(dy.data(), 0, dy.size() * sizeof(GroupDyn));
    BC_HIP(hipMemcpyAsync(sv->eng.d_dyn, dy.data(), dy.size() * sizeof(GroupDyn), hipMemcpyHostToDevice,
                          sv->stream));
    BC_HIP(hipStreamSynchronize(sv->stream));
    sv->slot_desc.resize(sv->slot_cap);
    sv->slot_owner.assign(sv->slot_cap, 0);
    BC_HIP(hipHostMalloc((void**)&sv->h_dyn, sizeof(GroupDyn) * sv->slot_cap));
    hipError_t e = hipMalloc((void**)&sv->d_pool, hbm_budget_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(BC_E_NOMEM, "server: cannot allocate the HBM budget");
    }
    sv->pool.init(sv->d_pool, hbm_budget_bytes);
    bc_server* raw = sv.get();
    sv->th = std::thread([raw] { server_loop(raw); });
    *out = sv.release();
    return BC_OK;
}

int bc_server_add_graph(bc_server* s, const bc_csr* g, const int32_t* part, int32_t k, int32_t* gid) {
    if (!s || !g || !gid) return fail(BC_E_INVAL, "null argument");
    if (g->n > 0 && !part) return fail(BC_E_INVAL, "null partition");
    if (g->n > 0 && k < 1) return fail(BC_E_INVAL, "k must be >= 1");
    for (int32_t v = 0; v < g->n; ++v)
        if (part[v] < 0 || part[v] >= k) return fail(BC_E_INVAL, "partition label out of range");
    bc_graph* gr = nullptr;
    BC_TRY(graph_create(g, s->stream, &gr));
    std::unique_ptr<bc_graph> keep(gr);
    // Dijkstra_SK of every part without targets, kept for the queries (built before the
    // graph is visible to the loop, so nothing else uses the graph's buffers meanwhile)
    auto cache = std::make_unique<DskCache>();
    if (g->n > 0) BC_TRY(build_dsk_cache(gr, part, k, cache.get()));
    gr->work.release();
    gr->pre.release();
    s->cache_bytes += (int64_t)cache->bytes;
    std::lock_guard<std::mutex> lk(s->mu);
    s->graphs.push_back(std::move(keep));
    s->parts.emplace_back(part, part + g->n);
    s->ks.push_back(k);
    s->caches.push_back(std::move(cache));
    *gid = (int32_t)s->graphs.size() - 1;
    return BC_OK;
}

int bc_query_submit(bc_server* s, int32_t gid, const int32_t* S, int32_t nS, uint32_t flags,
                    uint64_t* ticket) {
    if (!s || !ticket) return fail(BC_E_INVAL, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (gid < 0 || gid >= (int32_t)s->graphs.size()) return fail(BC_E_NOTFOUND, "unknown graph id");
    const int32_t n = s->graphs[gid]->n;
    lk.unlock();
    BC_TRY(validate_targets(n, S, nS));
    lk.lock();
    if (s->stop) return fail(BC_E_INVAL, "server stopped");
    if (s->incoming.size() >= 65536) return fail(BC_E_AGAIN, "queue full");
    auto q = std::make_unique<Query>();
    q->ticket = s->next_ticket++;
    q->gid = gid;
    q->S.assign(S, S + nS);
    q->flags = flags;
    q->t_submit = std::chrono::steady_clock::now();
    *ticket = q->ticket;
    s->incoming.push_back(q->ticket);
    s->queries[q->ticket] = std::move(q);
    s->n_submitted++;
    lk.unlock();
    s->cv.notify_all();
    return BC_OK;
}

int bc_query_poll(bc_server* s, uint64_t ticket, double* bc_out, int32_t* done) {
    if (!s || !done) return fail(BC_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->queries.find(ticket);
    if (it == s->queries.end()) return fail(BC_E_NOTFOUND, "unknown ticket");
    Query* q = it->second.get();
    *done = 0;
    if (q->state == Q_FAILED) {
        const int code = q->status;
        set_error(q->err);
        s->queries.erase(it);
        *done = 1;
        return code;
    }
    if (q->state != Q_DONE) return BC_OK;
    if (bc_out) std::copy(q->result.begin(), q->result.end(), bc_out);
    s->queries.erase(it);
    *done = 1;
    return BC_OK;
}

int bc_server_stats_get(bc_server* s, bc_server_stats* out) {
    if (!s || !out) return fail(BC_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->n_submitted;
    out->completed = s->n_completed;
    out->failed = s->n_failed;
    int64_t inflight = 0, queued = 0;
    for (auto& kv : s->queries) {
        const int st = kv.second->state;
        inflight += (st == Q_DSK || st == Q_BSK || st == Q_RES || st == Q_RDSK);
        queued += st == Q_QUEUED;
    }
    out->queued = queued;
    out->inflight = inflight;
    out->iterations = s->n_iters;
    std::vector<double> l = s->lat_ms;
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
        if (l.empty()) return 0.0;
        size_t i = (size_t)std::min<double>((double)l.size() - 1, std::ceil(p * l.size()) - 1);
        return l[i];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    out->peak_bytes = (int64_t)s->pool.peak;
    out->cache_bytes = s->cache_bytes;
    out->dsk_groups_cached = s->dsk_cached;
    out->dsk_groups_run = s->dsk_run;
    return BC_OK;
}

void bc_server_destroy(bc_server* s) { delete s; }

}  // extern "C"
