// Brandes++All (Sec. 6, Alg. 3): betweenness over all pairs of nodes from the
// skeleton. For every ordered pair of parts (P_i, P_j), including i = j, the skeleton
// is built with the nodes of P_i and P_j as singleton parts; Brandes_SK then runs from
// the sources S_sc = P_i with the destination indicator I[v in S_dest], S_dest = P_j
// (eq. multibrandes), followed by Centrality (eq. localcentrality); the per-pair
// scores C_ij add up to C over every ordered pair of distinct nodes, since P covers V.
// The Dijkstra_SK results of P's parts are computed once and shared by the k^2 builds,
// and the passes' Brandes_SK groups run together in as few launches as memory allows.
#include <algorithm>
#include <memory>
#include <vector>

#include "engine.h"
#include "graph.h"
#include "skbuild.h"

namespace bcpp {

// One pass (P_i, P_j) waiting for its Brandes_SK launch: its skeleton G_SK^{ij}, its
// groups and the destination flags.
struct PairPass {
    std::unique_ptr<bc_skeleton> sk;
    std::vector<GroupDesc> groups;
    std::vector<uint8_t> dest;
};

// Brandes_SK + Centrality of the pending passes as one resident launch, then each
// pass's scores added into out in pass order (the order of the pairs (i, j)).
static int run_pending(bc_graph* g, Arena& B, std::vector<PairPass>& passes, double scale, double* out_dev) {
    if (passes.empty()) return BC_OK;
    hipStream_t s = g->stream;
    size_t need = 65536, ng = 0;
    for (const PairPass& P : passes) {
        need += P.dest.size() + 256 + 2 * (P.groups.size() * 8 + 256);
        for (const GroupDesc& G : P.groups) need += resident_group_bytes(G);
        ng += P.groups.size();
    }
    need += resident_launch_bytes(ng);
    BC_TRY(B.reserve(need));
    std::vector<const GroupDesc*> all;
    all.reserve(ng);
    for (PairPass& P : passes) {
        uint8_t* d_dest = B.take<uint8_t>(P.dest.size());
        if (!d_dest) return fail(BC_E_NOMEM, "Brandes++All: workspace too small");
        BC_HIP(hipMemcpyAsync(d_dest, P.dest.data(), P.dest.size(), hipMemcpyHostToDevice, s));
        for (GroupDesc& G : P.groups) {
            G.g.nflag = d_dest;
            if (!resident_alloc(B, G)) return fail(BC_E_NOMEM, "Brandes++All: workspace too small");
            all.push_back(&G);
        }
    }
    BC_TRY(run_resident(s, B, all.data(), all.size()));
    for (PairPass& P : passes) {
        ReducePtrs R;
        BC_TRY(reduce_upload(s, B, P.groups, &R));
        BC_TRY(reduce_launch(s, R, g->n, nullptr, nullptr, P.sk->d_out_idx, P.sk->d_out_which, scale, out_dev,
                             true));
    }
    BC_HIP(hipStreamSynchronize(s));
    passes.clear();
    return BC_OK;
}

static int pp_all_run(bc_graph* g, const int32_t* part, int32_t k, uint32_t flags, double* out_dev) {
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    if (n == 0) return BC_OK;
    if (!part) return fail(BC_E_INVAL, "null partition");
    if (k < 1) return fail(BC_E_INVAL, "k must be >= 1");
    std::vector<std::vector<int32_t>> members(k);
    for (int32_t v = 0; v < n; ++v) {
        if (part[v] < 0 || part[v] >= k)
            return fail(BC_E_INVAL, "partition label out of range at node " + std::to_string(v));
        members[part[v]].push_back(v);
    }
    const double scale = (flags & BC_ORDERED) ? 1.0 : 0.5;
    BC_TRY(zero_device(s, out_dev, (size_t)n * 8));
    // Build_SK once for P (Alg. 3): the Dijkstra_SK results of every part. A pass takes
    // them for every part other than P_i and P_j (whose nodes are all singletons there,
    // with no Dijkstra_SK of their own), so its build only assembles G_SK^{ij}.
    // (BCPP_PPALL_REUSE=0 runs every pass's Dijkstra_SK, for comparisons.)
    const char* env = getenv("BCPP_PPALL_REUSE");
    DskCache base;
    if (!(env && env[0] == '0')) BC_TRY(build_dsk_cache(g, part, k, &base));
    // passes wait for one shared launch until their state would pass this many bytes
    // (BCPP_PPALL_PENDING_MB sets it, for tests of the launches' boundaries)
    size_t pending_cap = std::min<size_t>(state_budget() / 4, (size_t)1 << 30);
    if (const char* e = getenv("BCPP_PPALL_PENDING_MB")) pending_cap = (size_t)atoll(e) << 20;
    std::vector<PairPass> passes;
    Arena B;
    size_t pending = 0;
    std::vector<int32_t> S, src;
    for (int32_t i = 0; i < k; ++i) {
        if (members[i].empty()) continue;
        for (int32_t j = 0; j < k; ++j) {
            if (members[j].empty()) continue;
            // targets: S_sc = P_i first, then S_dest = P_j (the same nodes when i = j)
            S = members[i];
            if (j != i) S.insert(S.end(), members[j].begin(), members[j].end());
            if (S.size() < 2) continue;
            bc_skeleton* raw = nullptr;
            BC_TRY(partition_impl(g, part, k, S.data(), (int32_t)S.size(), &raw, false, nullptr,
                                  base.ok ? &base : nullptr));
            PairPass P;
            P.sk.reset(raw);
            const bc_skeleton* sk = P.sk.get();
            const size_t ni = members[i].size();
            src.clear();
            for (size_t t = 0; t < ni; ++t)
                if (sk->h_target_sk[t] >= 0) src.push_back(sk->h_target_sk[t]);
            if (src.empty() || sk->n_sk == 0) continue;
            P.dest.assign((size_t)sk->n_sk, 0);
            for (size_t t = (j == i ? 0 : ni); t < S.size(); ++t)
                if (sk->h_target_sk[t] >= 0) P.dest[sk->h_target_sk[t]] = (uint8_t)NF_TARGET;
            P.groups = resident_bsk_groups(sk, src, nullptr);
            size_t bytes = (size_t)sk->stats.device_bytes + P.dest.size();
            for (const GroupDesc& G : P.groups) bytes += resident_group_bytes(G);
            if (!passes.empty() && pending + bytes > pending_cap) {
                BC_TRY(run_pending(g, B, passes, scale, out_dev));
                pending = 0;
            }
            pending += bytes;
            passes.push_back(std::move(P));
        }
    }
    BC_TRY(run_pending(g, B, passes, scale, out_dev));
    BC_HIP(hipStreamSynchronize(s));
    return BC_OK;
}

}  // namespace bcpp

using namespace bcpp;

extern "C" {

int bc_brandes_pp_all(const bc_graph* gc, const int32_t* part, int32_t k, uint32_t flags, double* bc_out) {
    if (!gc || !bc_out) return fail(BC_E_INVAL, "null graph or output");
    if (flags & ~(uint32_t)BC_ORDERED) return fail(BC_E_INVAL, "only BC_ORDERED is accepted here");
    bc_graph* g = const_cast<bc_graph*>(gc);
    if (g->n == 0) return BC_OK;
    if (!resident_takes(g->n)) return fail(BC_E_INVAL, "Brandes++All runs on the resident kernel, which is switched off");
    BC_TRY(g->out.reserve((size_t)g->n * 8 + 256));
    double* d_out = g->out.take<double>(g->n);
    BC_TRY(pp_all_run(g, part, k, flags, d_out));
    BC_HIP(hipMemcpyAsync(bc_out, d_out, (size_t)g->n * 8, hipMemcpyDeviceToHost, g->stream));
    BC_HIP(hipStreamSynchronize(g->stream));
    return BC_OK;
}

}  // extern "C"
