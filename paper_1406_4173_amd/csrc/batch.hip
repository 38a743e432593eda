// Batched form: many independent graphs in one device run.
//
// The graphs are laid side by side as one disjoint union (node ids offset per graph).
// Plain Brandes gives each graph its own groups of 64 sources over its own node
// range. Brandes++ builds P' per graph (targets as singleton parts inside that graph's
// label range), so the union's skeleton is the disjoint union of the graphs'
// skeletons and each graph's skeleton nodes and table rows are contiguous id ranges;
// Dijkstra_SK then covers every part of every graph, and Brandes_SK + Centrality every
// graph's groups, each in a single run of launches. Scores of a disjoint union
// restricted to one graph are that graph's own scores (no shortest path joins two
// graphs). Each pass is captured as a HIP graph on its first run and replayed after.
#include <algorithm>
#include <memory>

#include "engine.h"
#include "graph.h"
#include "skbuild.h"

namespace bcpp {
// A batch's plain Brandes as a captured HIP graph. The batch never changes, so its
// groups, their buffers, the launch records and the reduction pointers are built once;
// each run replays the graph, which runs every kernel again (clear the error word, the
// resident launches, the reduction) and copies the scores and the error word to pinned
// host memory. Nothing in the graph is a memset node.
struct PlainPlan {
    bool ready = false;
    Arena mem;
    std::vector<GroupDesc> groups;
    hipStream_t stream = nullptr;  // capture needs a stream of its own
    double* h_out = nullptr;       // pinned
    uint32_t* h_err = nullptr;     // pinned
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    PlainPlan() = default;
    PlainPlan(const PlainPlan&) = delete;
    PlainPlan& operator=(const PlainPlan&) = delete;
    ~PlainPlan() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (h_out) (void)hipHostFree(h_out);
        if (h_err) (void)hipHostFree(h_err);
        mem.release();
        if (stream) (void)hipStreamDestroy(stream);
    }
};
// Brandes++ over the batch as one captured HIP graph. The first run builds the skeleton
// of the union graph on the device in arenas the plan owns (the graph's own arenas are
// swapped out meanwhile), keeps the build and every launch record, and captures the
// device work of a whole run: phase 1 and 2 of Build_SK, the Dijkstra_SK launch, the
// clique and table counts, the skeleton fill, the Brandes_SK + Centrality launch, the
// reduction and the copies out. A replay recomputes all of it; only host bookkeeping
// (sizes, offsets, group lists and launch records, fixed by the batch's graphs,
// partitions and targets) is taken from the first run. Needs every group on the
// resident kernel; otherwise the batch runs eagerly.
struct PpPlan {
    Arena pre, work, run;
    std::unique_ptr<bc_skeleton> sk;
    PartitionKeep part;
    ResidentLaunch L;
    ReducePtrs R;
    uint32_t* d_err = nullptr;
    double* d_out = nullptr;
    hipStream_t stream = nullptr;
    double* h_out = nullptr;    // pinned
    uint32_t* h_err = nullptr;  // pinned
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    PpPlan() = default;
    PpPlan(const PpPlan&) = delete;
    PpPlan& operator=(const PpPlan&) = delete;
    ~PpPlan() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (h_out) (void)hipHostFree(h_out);
        if (h_err) (void)hipHostFree(h_err);
        sk.reset();
        run.release();
        work.release();
        pre.release();
        if (stream) (void)hipStreamDestroy(stream);
    }
};

}  // namespace bcpp

struct bc_batch {
    int32_t ng = 0;
    std::vector<int32_t> n_off;  // [ng+1] node offset of each graph in the union
    std::vector<int32_t> s_off;  // [ng+1] offset of each graph's targets in S_all
    std::vector<int32_t> S_all;  // targets, union ids, graph-major
    std::vector<int32_t> lab;    // P' labels of the union (targets singleton)
    std::vector<int32_t> maxw;   // [ng] each graph's largest weight (1 for unit weights)
    int32_t nlab = 0;
    bc_graph* G = nullptr;       // the union graph
    std::unique_ptr<bcpp::PlainPlan> plan;  // plain Brandes, captured on first use
    std::unique_ptr<bcpp::PpPlan> pp_plan;  // Brandes++, captured on first use
    bool pp_eager = false;                  // Brandes++ cannot be captured (runs eagerly)
    ~bc_batch() {
        plan.reset();
        pp_plan.reset();
        delete G;
    }
};

namespace bcpp {

// Run a list of groups of which some (resident[i]) go to the LDS-resident kernel and
// the rest to the engine; the score pointers end up in groups[i] either way, so the
// list keeps its order (each graph's groups contiguous) for the reduction.
static int run_mixed(Arena& W, hipStream_t s, std::vector<GroupDesc>& groups,
                     const std::vector<uint8_t>& resident, int64_t steps) {
    std::vector<GroupDesc> E;
    std::vector<const GroupDesc*> R;
    for (size_t i = 0; i < groups.size(); ++i) {
        if (!resident[i]) {
            E.push_back(groups[i]);
            continue;
        }
        if (!resident_alloc(W, groups[i])) return fail(BC_E_NOMEM, "batch: workspace too small");
        R.push_back(&groups[i]);
    }
    if (!R.empty()) BC_TRY(run_resident(s, W, R.data(), R.size()));
    if (!E.empty()) BC_TRY(run_groups(W, s, E, steps));
    size_t e = 0;
    for (size_t i = 0; i < groups.size(); ++i)
        if (!resident[i]) groups[i] = E[e++];
    return BC_OK;
}

// Workspace of the groups of run_mixed.
static size_t mixed_bytes(const std::vector<GroupDesc>& groups, const std::vector<uint8_t>& resident,
                          int64_t steps) {
    size_t need = 0, nres = 0, neng = 0;
    int64_t positions = 0;
    for (size_t i = 0; i < groups.size(); ++i) {
        const GroupDesc& D = groups[i];
        if (resident[i]) {
            need += resident_group_bytes(D);
            ++nres;
        } else {
            need += group_bytes(D, steps);
            positions += std::max<int64_t>((int64_t)D.hi - D.lo, (D.flags & GF_CENT) ? D.tn : 0);
            ++neng;
        }
    }
    if (nres) need += resident_launch_bytes(nres);
    if (neng) need += engine_bytes((int32_t)neng, positions);
    return need;
}

static int batch_plain(bc_batch* b, uint32_t flags, double* d_out) {
    bc_graph* G = b->G;
    hipStream_t s = G->stream;
    const int32_t n = G->n;
    std::vector<GroupDesc> groups;
    std::vector<uint8_t> resident;
    groups.reserve(b->S_all.size() + (size_t)b->ng);
    resident.reserve(b->S_all.size() + (size_t)b->ng);
    std::vector<int32_t> g0(n, 0), g1(n, 0), idx(n, -1);
    int64_t steps = 1;
    const bool allow_res = !(flags & BC_ENGINE_ONLY);
    for (int32_t gi = 0; gi < b->ng; ++gi) {
        const int32_t lo = b->n_off[gi], hi = b->n_off[gi + 1];
        const int32_t ns = b->s_off[gi + 1] - b->s_off[gi];
        const int32_t first_group = (int32_t)groups.size();
        if (ns >= 2) {
            const bool res = allow_res && resident_takes(hi - lo);
            const int32_t per = res ? resident_sources_per_group(ns) : LANES;
            if (!res) steps = std::max(steps, max_steps_bound(hi - lo, LANES, (int64_t)(hi - lo) * G->maxw));
            for (int32_t c = 0; c < ns; c += per) {
                GroupDesc D;
                D.lo = lo;
                D.hi = hi;
                D.arc_lo = G->h_row_ptr[lo];
                D.arcs = G->h_row_ptr[hi] - G->h_row_ptr[lo];
                D.ring_len = b->maxw[gi] + 1;
                D.flags = GF_BACKWARD | (G->unit ? GF_UNIT : 0u);
                D.nsrc = std::min(per, ns - c);
                for (int l = 0; l < LANES; ++l)
                    D.src[l] = l < D.nsrc ? b->S_all[b->s_off[gi] + c + l] : -1;
                groups.push_back(D);
                resident.push_back(res ? 1 : 0);
            }
        }
        for (int32_t v = lo; v < hi; ++v) {
            g0[v] = first_group;
            g1[v] = (int32_t)groups.size();
            idx[v] = v - lo;
        }
    }
    Arena& W = G->work;
    const size_t need = mixed_bytes(groups, resident, steps) + (size_t)n * 13 +
                        (size_t)groups.size() * 16 + (1 << 20);
    BC_TRY(W.reserve(need));
    uint8_t* d_flag = W.take<uint8_t>(n);
    int32_t* d_g0 = W.take<int32_t>(n);
    int32_t* d_g1 = W.take<int32_t>(n);
    int32_t* d_idx = W.take<int32_t>(n);
    if (!d_flag || !d_g0 || !d_g1 || !d_idx) return fail(BC_E_NOMEM, "batch: workspace too small");
    std::vector<uint8_t> flag(n, 0);
    for (int32_t v : b->S_all) flag[v] = (uint8_t)NF_TARGET;
    BC_HIP(hipMemcpyAsync(d_flag, flag.data(), n, hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(d_g0, g0.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(d_g1, g1.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(d_idx, idx.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    for (auto& D : groups) {
        D.g.row_ptr = G->d_row_ptr;
        D.g.col = G->d_col;
        D.g.len = G->d_len;
        D.g.nflag = d_flag;
        D.g.twin = G->d_twin;
        D.g.arc = G->d_arc;
    }
    BC_TRY(run_mixed(W, s, groups, resident, steps));
    BC_TRY(reduce_scores(s, W, groups, n, d_g0, d_g1, d_idx, nullptr, 0.5, d_out, false));
    return BC_OK;
}

__global__ void k_clear_word(uint32_t* __restrict__ p) {
    if (threadIdx.x == 0) p[0] = 0u;
}

// Build the plain plan and capture its graph (first plain run of the batch).
static int build_plain_plan(bc_batch* b) {
    bc_graph* G = b->G;
    hipStream_t s0 = G->stream;
    const int32_t n = G->n;
    auto P = std::make_unique<PlainPlan>();
    std::vector<int32_t> g0(n, 0), g1(n, 0), idx(n, -1);
    P->groups.reserve(b->S_all.size() + (size_t)b->ng);
    for (int32_t gi = 0; gi < b->ng; ++gi) {
        const int32_t lo = b->n_off[gi], hi = b->n_off[gi + 1];
        const int32_t ns = b->s_off[gi + 1] - b->s_off[gi];
        const int32_t first_group = (int32_t)P->groups.size();
        if (ns >= 2) {
            const int32_t per = resident_sources_per_group(ns);
            for (int32_t c = 0; c < ns; c += per) {
                GroupDesc D;
                D.lo = lo;
                D.hi = hi;
                D.arc_lo = G->h_row_ptr[lo];
                D.arcs = G->h_row_ptr[hi] - G->h_row_ptr[lo];
                D.flags = GF_BACKWARD;
                D.ring_len = b->maxw[gi] + 1;
                D.nsrc = std::min(per, ns - c);
                for (int l = 0; l < LANES; ++l) D.src[l] = l < D.nsrc ? b->S_all[b->s_off[gi] + c + l] : -1;
                P->groups.push_back(D);
            }
        }
        for (int32_t v = lo; v < hi; ++v) {
            g0[v] = first_group;
            g1[v] = (int32_t)P->groups.size();
            idx[v] = v - lo;
        }
    }
    size_t need = resident_launch_bytes(P->groups.size()) + 2 * (P->groups.size() * 8 + 256) +
                  (size_t)n * 21 + (1 << 20);
    for (const GroupDesc& D : P->groups) need += resident_group_bytes(D);
    BC_TRY(P->mem.reserve(need));
    uint8_t* d_flag = P->mem.take<uint8_t>(std::max(n, 1));
    int32_t* d_g0 = P->mem.take<int32_t>(std::max(n, 1));
    int32_t* d_g1 = P->mem.take<int32_t>(std::max(n, 1));
    int32_t* d_idx = P->mem.take<int32_t>(std::max(n, 1));
    double* d_out = P->mem.take<double>(std::max(n, 1));
    if (!d_flag || !d_g0 || !d_g1 || !d_idx || !d_out) return fail(BC_E_NOMEM, "batch: workspace too small");
    std::vector<uint8_t> flag(n, 0);
    for (int32_t v : b->S_all) flag[v] = (uint8_t)NF_TARGET;
    BC_HIP(hipMemcpyAsync(d_flag, flag.data(), n, hipMemcpyHostToDevice, s0));
    BC_HIP(hipMemcpyAsync(d_g0, g0.data(), (size_t)n * 4, hipMemcpyHostToDevice, s0));
    BC_HIP(hipMemcpyAsync(d_g1, g1.data(), (size_t)n * 4, hipMemcpyHostToDevice, s0));
    BC_HIP(hipMemcpyAsync(d_idx, idx.data(), (size_t)n * 4, hipMemcpyHostToDevice, s0));
    for (GroupDesc& D : P->groups) {
        D.g.row_ptr = G->d_row_ptr;
        D.g.col = G->d_col;
        D.g.len = G->d_len;
        D.g.nflag = d_flag;
        D.g.twin = G->d_twin;
        D.g.arc = G->d_arc;
        if (!resident_alloc(P->mem, D)) return fail(BC_E_NOMEM, "batch: workspace too small");
    }
    ResidentLaunch L;
    ReducePtrs R;
    BC_TRY(resident_upload(s0, P->mem, P->groups, &L));
    BC_TRY(reduce_upload(s0, P->mem, P->groups, &R));
    BC_HIP(hipHostMalloc((void**)&P->h_out, (size_t)std::max(n, 1) * 8));
    BC_HIP(hipHostMalloc((void**)&P->h_err, sizeof(uint32_t)));
    BC_HIP(hipStreamSynchronize(s0));
    BC_HIP(hipStreamCreate(&P->stream));
    // capture; launch timing is off while capturing (its events are not graph nodes)
    hipStream_t s = P->stream;
    const bool prof_on = profiler().on;
    profiler().on = false;
    BC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    int rc = BC_OK;
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, s, L.d_err);
    if (hipGetLastError() != hipSuccess) rc = fail(BC_E_DEVICE, "batch: capture failed");
    if (rc == BC_OK) rc = resident_launch(s, L);
    if (rc == BC_OK) rc = reduce_launch(s, R, n, d_g0, d_g1, d_idx, nullptr, 0.5, d_out, false);
    if (rc == BC_OK && (hipMemcpyAsync(P->h_out, d_out, (size_t)n * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                        hipMemcpyAsync(P->h_err, L.d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess))
        rc = fail(BC_E_DEVICE, "batch: capture of the copies failed");
    const hipError_t ec = hipStreamEndCapture(s, &P->graph);
    profiler().on = prof_on;
    BC_TRY(rc);
    if (ec != hipSuccess) return fail(BC_E_DEVICE, std::string("batch: capture failed: ") + hipGetErrorString(ec));
    BC_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
    P->ready = true;
    b->plan = std::move(P);
    return BC_OK;
}

// Plain Brandes over the batch by replaying its captured graph.
static int batch_plain_graph(bc_batch* b, double scale, double* const* bc_out) {
    if (!b->plan) BC_TRY(build_plain_plan(b));
    PlainPlan& P = *b->plan;
    PhaseTrace tr("batch plain (graph)");
    BC_HIP(hipGraphLaunch(P.exec, P.stream));
    BC_HIP(hipStreamSynchronize(P.stream));
    tr.mark("replay");
    if (*P.h_err & ERR_OVERFLOW) return fail(BC_E_OVERFLOW, "a shortest-path count reached 2^64");
    for (int32_t i = 0; i < b->ng; ++i) {
        if (!bc_out[i]) continue;
        for (int32_t v = b->n_off[i]; v < b->n_off[i + 1]; ++v)
            bc_out[i][v - b->n_off[i]] = P.h_out[v] * scale;
    }
    return BC_OK;
}

// Brandes_SK + Centrality groups of every graph of the batch over the union skeleton,
// and the reduction maps (node -> its graph's groups, its row in them).
struct PpGroups {
    std::vector<GroupDesc> groups;
    std::vector<uint8_t> resident;
    std::vector<int32_t> g0, g1, idx;
    std::vector<uint8_t> which;
    int64_t steps = 1;
};

static int pp_groups(const bc_batch* b, const bc_skeleton* sk, bool allow_res, PpGroups* out) {
    const bc_graph* G = b->G;
    const int32_t n = G->n;
    // per node: skeleton id or table row (the skeleton was assembled on the graph's stream)
    std::vector<int32_t> oi(n);
    std::vector<uint8_t> ow(n);
    if (n) {
        BC_HIP(hipMemcpyAsync(oi.data(), sk->d_out_idx, (size_t)n * 4, hipMemcpyDeviceToHost, G->stream));
        BC_HIP(hipMemcpyAsync(ow.data(), sk->d_out_which, n, hipMemcpyDeviceToHost, G->stream));
        BC_HIP(hipStreamSynchronize(G->stream));
    }
    PpGroups& Q = *out;
    Q.groups.reserve(b->S_all.size() + (size_t)b->ng);
    Q.resident.reserve(b->S_all.size() + (size_t)b->ng);
    Q.g0.assign(n, 0);
    Q.g1.assign(n, 0);
    Q.idx.assign(n, -1);
    Q.which.assign(n, 0);
    for (int32_t gi = 0; gi < b->ng; ++gi) {
        const int32_t lo = b->n_off[gi], hi = b->n_off[gi + 1];
        int32_t sk_lo = INT32_MAX, sk_hi = -1, t_lo = INT32_MAX, t_hi = -1;
        for (int32_t v = lo; v < hi; ++v) {
            if (oi[v] < 0) continue;
            if (ow[v] == 0) {
                sk_lo = std::min(sk_lo, oi[v]);
                sk_hi = std::max(sk_hi, oi[v] + 1);
            } else {
                t_lo = std::min(t_lo, oi[v]);
                t_hi = std::max(t_hi, oi[v] + 1);
            }
        }
        std::vector<int32_t> src;
        for (int32_t j = b->s_off[gi]; j < b->s_off[gi + 1]; ++j) {
            const int32_t v = b->S_all[j];
            if (oi[v] >= 0 && ow[v] == 0) src.push_back(oi[v]);
        }
        const int32_t first_group = (int32_t)Q.groups.size();
        if (src.size() >= 2 && sk_hi > sk_lo) {
            const int32_t N = sk_hi - sk_lo;
            const int32_t tn = t_hi > t_lo ? t_hi - t_lo : 0;
            const bool res = allow_res && resident_takes(N);
            const size_t per = res ? (size_t)resident_sources_per_group((int64_t)src.size()) : LANES;
            if (!res) Q.steps = std::max(Q.steps, max_steps_bound(N, LANES, (int64_t)(hi - lo) * G->maxw));
            for (size_t c = 0; c < src.size(); c += per) {
                GroupDesc D;
                D.g.row_ptr = sk->d_row_ptr;
                D.g.col = sk->d_col;
                D.g.len = sk->d_len;
                D.g.mult = sk_mult(sk);
                D.g.nflag = sk->d_nflag;
                D.g.twin = sk->d_twin;
                D.g.arc = sk->d_arc;
                D.lo = sk_lo;
                D.hi = sk_hi;
                D.arc_lo = sk->h_row_ptr[sk_lo];
                D.arcs = sk->h_row_ptr[sk_hi] - sk->h_row_ptr[sk_lo];
                D.ring_len = sk->max_len + 1;
                D.flags = GF_BACKWARD | (tn ? GF_CENT : 0u);
                D.trow = sk->d_trow;
                D.tcol = sk->d_tcol;
                D.tlen = sk->d_tlen;
                D.tsig = sk->d_tsig;
                D.t_lo = tn ? t_lo : 0;
                D.tn = tn;
                D.nsrc = (int32_t)std::min<size_t>(per, src.size() - c);
                for (int l = 0; l < LANES; ++l) D.src[l] = l < D.nsrc ? src[c + l] : -1;
                Q.groups.push_back(D);
                Q.resident.push_back(res ? 1 : 0);
            }
        }
        for (int32_t v = lo; v < hi; ++v) {
            Q.g0[v] = first_group;
            Q.g1[v] = (int32_t)Q.groups.size();
            if (oi[v] >= 0 && Q.g1[v] > Q.g0[v]) {
                Q.idx[v] = ow[v] == 0 ? oi[v] - sk_lo : oi[v] - t_lo;
                Q.which[v] = ow[v];
            }
        }
    }
    return BC_OK;
}

static int batch_pp(bc_batch* b, uint32_t flags, double* d_out) {
    bc_graph* G = b->G;
    hipStream_t s = G->stream;
    const int32_t n = G->n;
    PhaseTrace tr("batch Brandes++");
    bc_skeleton* skp = nullptr;
    BC_TRY(partition_impl(G, b->lab.data(), b->nlab, b->S_all.data(), (int32_t)b->S_all.size(), &skp,
                          true));
    tr.mark("partition");
    std::unique_ptr<bc_skeleton> sk(skp);
    PpGroups Q;
    BC_TRY(pp_groups(b, sk.get(), !(flags & BC_ENGINE_ONLY), &Q));
    Arena& W = G->work;
    const size_t need = mixed_bytes(Q.groups, Q.resident, Q.steps) + (size_t)n * 13 +
                        (size_t)Q.groups.size() * 16 + (1 << 20);
    BC_TRY(W.reserve(need));
    int32_t* d_g0 = W.take<int32_t>(n);
    int32_t* d_g1 = W.take<int32_t>(n);
    int32_t* d_idx = W.take<int32_t>(n);
    uint8_t* d_which = W.take<uint8_t>(n);
    if (!d_g0 || !d_g1 || !d_idx || !d_which) return fail(BC_E_NOMEM, "batch: workspace too small");
    BC_HIP(hipMemcpyAsync(d_g0, Q.g0.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(d_g1, Q.g1.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(d_idx, Q.idx.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(d_which, Q.which.data(), n, hipMemcpyHostToDevice, s));
    tr.mark("groups");
    BC_TRY(run_mixed(W, s, Q.groups, Q.resident, Q.steps));
    tr.mark("Brandes_SK");
    BC_TRY(reduce_scores(s, W, Q.groups, n, d_g0, d_g1, d_idx, d_which, 0.5, d_out, false));
    tr.mark("reduce");
    return BC_OK;
}

__global__ void k_or_words(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, uint32_t* __restrict__ out) {
    if (threadIdx.x == 0) out[0] = a[0] | b[0];
}

// Builds b->pp_plan, or leaves it empty (and returns BC_OK) when some group would not
// run on the resident kernel.
static int build_pp_plan(bc_batch* b) {
    bc_graph* G = b->G;
    hipStream_t s0 = G->stream;
    const int32_t n = G->n;
    auto P = std::make_unique<PpPlan>();
    std::swap(G->pre, P->pre);
    std::swap(G->work, P->work);
    bc_skeleton* skp = nullptr;
    const int rc0 = partition_impl(G, b->lab.data(), b->nlab, b->S_all.data(), (int32_t)b->S_all.size(), &skp,
                                   true, &P->part);
    std::swap(G->pre, P->pre);
    std::swap(G->work, P->work);
    P->sk.reset(skp);
    BC_TRY(rc0);
    if (!P->part.resident && !P->part.b.groups.empty()) return BC_OK;
    PpGroups Q;
    BC_TRY(pp_groups(b, P->sk.get(), true, &Q));
    for (uint8_t r : Q.resident)
        if (!r) return BC_OK;
    size_t need = resident_launch_bytes(Q.groups.size()) + 2 * (Q.groups.size() * 8 + 256) + (size_t)n * 21 +
                  (1 << 20);
    for (const GroupDesc& D : Q.groups) need += resident_group_bytes(D);
    BC_TRY(P->run.reserve(need));
    int32_t* d_g0 = P->run.take<int32_t>(std::max(n, 1));
    int32_t* d_g1 = P->run.take<int32_t>(std::max(n, 1));
    int32_t* d_idx = P->run.take<int32_t>(std::max(n, 1));
    uint8_t* d_which = P->run.take<uint8_t>(std::max(n, 1));
    P->d_out = P->run.take<double>(std::max(n, 1));
    P->d_err = P->run.take<uint32_t>(1);
    if (!d_g0 || !d_g1 || !d_idx || !d_which || !P->d_out || !P->d_err)
        return fail(BC_E_NOMEM, "batch: workspace too small");
    BC_HIP(hipMemcpyAsync(d_g0, Q.g0.data(), (size_t)n * 4, hipMemcpyHostToDevice, s0));
    BC_HIP(hipMemcpyAsync(d_g1, Q.g1.data(), (size_t)n * 4, hipMemcpyHostToDevice, s0));
    BC_HIP(hipMemcpyAsync(d_idx, Q.idx.data(), (size_t)n * 4, hipMemcpyHostToDevice, s0));
    BC_HIP(hipMemcpyAsync(d_which, Q.which.data(), n, hipMemcpyHostToDevice, s0));
    for (GroupDesc& D : Q.groups)
        if (!resident_alloc(P->run, D)) return fail(BC_E_NOMEM, "batch: workspace too small");
    BC_TRY(resident_upload(s0, P->run, Q.groups, &P->L));
    BC_TRY(reduce_upload(s0, P->run, Q.groups, &P->R));
    BC_HIP(hipHostMalloc((void**)&P->h_out, (size_t)std::max(n, 1) * 8));
    BC_HIP(hipHostMalloc((void**)&P->h_err, sizeof(uint32_t)));
    BC_HIP(hipStreamSynchronize(s0));
    BC_HIP(hipStreamCreate(&P->stream));
    hipStream_t s = P->stream;
    const SkBuild& B = P->part.b;
    const bool prof_on = profiler().on;
    profiler().on = false;
    BC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, s, P->d_err);
    int rc = B.issue_phase1(s);
    if (rc == BC_OK) rc = B.issue_phase2(s);
    if (rc == BC_OK && P->part.resident) {
        hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, s, P->part.L.d_err);
        rc = resident_launch(s, P->part.L);
    }
    if (rc == BC_OK) rc = B.issue_count(s);
    if (rc == BC_OK) rc = B.issue_fill(s, P->sk.get());
    if (rc == BC_OK && !Q.groups.empty()) {
        hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, s, P->L.d_err);
        rc = resident_launch(s, P->L);
    }
    if (rc == BC_OK) rc = reduce_launch(s, P->R, n, d_g0, d_g1, d_idx, d_which, 0.5, P->d_out, false);
    if (rc == BC_OK) {
        // the error words of the two launches (a missing launch reads the cleared word)
        uint32_t* e1 = P->part.resident ? P->part.L.d_err : P->d_err;
        uint32_t* e2 = Q.groups.empty() ? P->d_err : P->L.d_err;
        hipLaunchKernelGGL(k_or_words, dim3(1), dim3(64), 0, s, e1, e2, P->d_err);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(P->h_out, P->d_out, (size_t)n * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(P->h_err, P->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
            rc = fail(BC_E_DEVICE, "batch: capture of the copies failed");
    }
    const hipError_t ec = hipStreamEndCapture(s, &P->graph);
    profiler().on = prof_on;
    BC_TRY(rc);
    if (ec != hipSuccess) return fail(BC_E_DEVICE, std::string("batch: capture failed: ") + hipGetErrorString(ec));
    // a memset node would be replayed wrongly on this platform: the build clears with
    // fill kernels, and a library that recorded one makes the plan unusable
    size_t nn = 0;
    BC_HIP(hipGraphGetNodes(P->graph, nullptr, &nn));
    std::vector<hipGraphNode_t> nodes(nn);
    BC_HIP(hipGraphGetNodes(P->graph, nodes.data(), &nn));
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType t;
        BC_HIP(hipGraphNodeGetType(nd, &t));
        if (t == hipGraphNodeTypeMemset) return fail(BC_E_DEVICE, "batch: captured Brandes++ holds a memset");
    }
    BC_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
    b->pp_plan = std::move(P);
    return BC_OK;
}

// Brandes++ over the batch by replaying its captured graph (built on first use).
// Returns BC_E_NOTFOUND when the batch cannot be captured (the caller runs it eagerly).
static int batch_pp_graph(bc_batch* b, double scale, double* const* bc_out) {
    if (!b->pp_plan) {
        if (b->pp_eager) return BC_E_NOTFOUND;
        BC_TRY(build_pp_plan(b));
        if (!b->pp_plan) {
            b->pp_eager = true;
            return BC_E_NOTFOUND;
        }
    }
    PpPlan& P = *b->pp_plan;
    PhaseTrace tr("batch Brandes++ (graph)");
    BC_HIP(hipGraphLaunch(P.exec, P.stream));
    BC_HIP(hipStreamSynchronize(P.stream));
    tr.mark("replay");
    if (*P.h_err & ERR_OVERFLOW) return fail(BC_E_OVERFLOW, "a shortest-path count reached 2^64");
    for (int32_t i = 0; i < b->ng; ++i) {
        if (!bc_out[i]) continue;
        for (int32_t v = b->n_off[i]; v < b->n_off[i + 1]; ++v)
            bc_out[i][v - b->n_off[i]] = P.h_out[v] * scale;
    }
    return BC_OK;
}

}  // namespace bcpp

using namespace bcpp;

extern "C" {

int bc_batch_create(int32_t ngraphs, const bc_csr* graphs, const int32_t* const* parts,
                    const int32_t* ks, const int32_t* const* S, const int32_t* nS, void* hip_stream,
                    bc_batch** out) {
    if (!out) return fail(BC_E_INVAL, "null output handle");
    *out = nullptr;
    if (ngraphs < 1 || !graphs || !parts || !ks || !S || !nS) return fail(BC_E_INVAL, "bad batch arguments");
    auto b = std::make_unique<bc_batch>();
    b->ng = ngraphs;
    b->n_off.assign(ngraphs + 1, 0);
    b->s_off.assign(ngraphs + 1, 0);
    int64_t ntot = 0, atot = 0;
    int32_t maxw = 1;
    bool any_w = false, all_w = true;
    for (int32_t i = 0; i < ngraphs; ++i) {
        int32_t mw = 1;
        BC_TRY(validate_csr(&graphs[i], &mw));
        maxw = std::max(maxw, mw);
        b->maxw.push_back(mw);
        ntot += graphs[i].n;
        atot += graphs[i].nnz;
        if (graphs[i].w) any_w = true; else all_w = false;
        if (ntot >= INT32_MAX) return fail(BC_E_INVAL, "batch too large");
        b->n_off[i + 1] = (int32_t)ntot;
        if (ks[i] < 1 && graphs[i].n > 0) return fail(BC_E_INVAL, "k must be >= 1");
        for (int32_t v = 0; v < graphs[i].n; ++v)
            if (parts[i][v] < 0 || parts[i][v] >= ks[i]) return fail(BC_E_INVAL, "partition label out of range");
        BC_TRY(validate_targets(graphs[i].n, S[i], nS[i]));
        b->s_off[i + 1] = b->s_off[i] + nS[i];
    }
    (void)all_w;
    // union CSR (weights materialised when any graph is weighted)
    std::vector<int64_t> rp(ntot + 1, 0);
    std::vector<int32_t> col;
    std::vector<int32_t> w;
    col.reserve(atot);
    if (any_w) w.reserve(atot);
    b->lab.assign(ntot, 0);
    int64_t lab_off = 0;
    for (int32_t i = 0; i < ngraphs; ++i) {
        const bc_csr& g = graphs[i];
        const int32_t off = b->n_off[i];
        for (int32_t v = 0; v < g.n; ++v) {
            for (int64_t e = g.row_ptr[v]; e < g.row_ptr[v + 1]; ++e) {
                col.push_back(g.col[e] + off);
                if (any_w) w.push_back(g.w ? g.w[e] : 1);
            }
            rp[off + v + 1] = (int64_t)col.size();
            b->lab[off + v] = (int32_t)(lab_off + parts[i][v]);
        }
        for (int32_t j = 0; j < nS[i]; ++j) {
            const int32_t v = S[i][j];
            b->S_all.push_back(v + off);
            b->lab[off + v] = (int32_t)(lab_off + ks[i] + j);
        }
        lab_off += (int64_t)ks[i] + nS[i];
        if (lab_off >= INT32_MAX) return fail(BC_E_INVAL, "batch too large");
    }
    b->nlab = (int32_t)std::max<int64_t>(lab_off, 1);
    bc_csr u{(int32_t)ntot, (int64_t)col.size(), rp.data(), col.data(), any_w ? w.data() : nullptr};
    BC_TRY(graph_create(&u, (hipStream_t)hip_stream, &b->G));
    *out = b.release();
    return BC_OK;
}

int bc_batch_run(bc_batch* b, uint32_t flags, double* const* bc_out) {
    if (!b || !bc_out) return fail(BC_E_INVAL, "null batch or outputs");
    bc_graph* G = b->G;
    const int32_t n = G->n;
    if (n == 0) return BC_OK;
    if (!(flags & (BC_BATCH_PP | BC_ENGINE_ONLY | BC_NO_GRAPH))) {
        bool res = true;
        for (int32_t i = 0; i < b->ng; ++i) res = res && resident_takes(b->n_off[i + 1] - b->n_off[i]);
        if (res) return batch_plain_graph(b, (flags & BC_ORDERED) ? 2.0 : 1.0, bc_out);
    }
    if ((flags & BC_BATCH_PP) && !(flags & (BC_ENGINE_ONLY | BC_NO_GRAPH))) {
        const int rc = batch_pp_graph(b, (flags & BC_ORDERED) ? 2.0 : 1.0, bc_out);
        if (rc != BC_E_NOTFOUND) return rc;
    }
    BC_TRY(G->out.reserve((size_t)n * 8 + 256));
    double* d_out = G->out.take<double>(n);
    PhaseTrace tr("batch run");
    BC_TRY((flags & BC_BATCH_PP) ? batch_pp(b, flags, d_out) : batch_plain(b, flags, d_out));
    tr.mark("traversal");
    std::vector<double> all(n);
    BC_HIP(hipMemcpyAsync(all.data(), d_out, (size_t)n * 8, hipMemcpyDeviceToHost, G->stream));
    BC_HIP(hipStreamSynchronize(G->stream));
    const double scale = (flags & BC_ORDERED) ? 2.0 : 1.0;
    for (int32_t i = 0; i < b->ng; ++i) {
        if (!bc_out[i]) continue;
        for (int32_t v = b->n_off[i]; v < b->n_off[i + 1]; ++v) bc_out[i][v - b->n_off[i]] = all[v] * scale;
    }
    tr.mark("copy out");
    return BC_OK;
}

void bc_batch_destroy(bc_batch* b) { delete b; }

}  // extern "C"
