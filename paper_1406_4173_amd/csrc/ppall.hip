// Brandes++All (Sec. 6, Alg. 3): betweenness over all pairs of nodes from the
// skeleton. For every ordered pair of parts (P_i, P_j), including i = j, the skeleton
// is built with the nodes of P_i and P_j as singleton parts; Brandes_SK then runs from
// the sources S_sc = P_i with the destination indicator I[v in S_dest], S_dest = P_j
// (eq. multibrandes), followed by Centrality (eq. localcentrality); the per-pair
// scores C_ij add up to C over every ordered pair of distinct nodes, since P covers V.
#include <algorithm>
#include <memory>
#include <vector>

#include "engine.h"
#include "graph.h"
#include "skbuild.h"

namespace bcpp {

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
    std::vector<int32_t> S, src;
    std::vector<uint8_t> dest;
    for (int32_t i = 0; i < k; ++i) {
        if (members[i].empty()) continue;
        for (int32_t j = 0; j < k; ++j) {
            if (members[j].empty()) continue;
            // targets: S_sc = P_i first, then S_dest = P_j (the same nodes when i = j)
            S = members[i];
            if (j != i) S.insert(S.end(), members[j].begin(), members[j].end());
            if (S.size() < 2) continue;
            bc_skeleton* raw = nullptr;
            BC_TRY(partition_impl(g, part, k, S.data(), (int32_t)S.size(), &raw, false));
            std::unique_ptr<bc_skeleton> sk(raw);
            const size_t ni = members[i].size();
            src.clear();
            for (size_t t = 0; t < ni; ++t)
                if (sk->h_target_sk[t] >= 0) src.push_back(sk->h_target_sk[t]);
            if (src.empty() || sk->n_sk == 0) continue;
            dest.assign((size_t)sk->n_sk, 0);
            for (size_t t = (j == i ? 0 : ni); t < S.size(); ++t)
                if (sk->h_target_sk[t] >= 0) dest[sk->h_target_sk[t]] = (uint8_t)NF_TARGET;
            std::vector<GroupDesc> groups = resident_bsk_groups(sk.get(), src, nullptr);
            size_t need = resident_launch_bytes(groups.size()) + 2 * (groups.size() * 8 + 256) + 65536 +
                          (size_t)sk->n_sk + 256;
            for (const GroupDesc& G : groups) need += resident_group_bytes(G);
            BC_TRY(g->work.reserve(need));
            uint8_t* d_dest = g->work.take<uint8_t>((size_t)sk->n_sk);
            if (!d_dest) return fail(BC_E_NOMEM, "Brandes++All: workspace too small");
            BC_HIP(hipMemcpyAsync(d_dest, dest.data(), dest.size(), hipMemcpyHostToDevice, s));
            for (GroupDesc& G : groups) {
                G.g.nflag = d_dest;
                if (!resident_alloc(g->work, G)) return fail(BC_E_NOMEM, "Brandes++All: workspace too small");
            }
            BC_TRY(run_resident(s, g->work, groups));
            BC_TRY(reduce_scores(s, g->work, groups, n, nullptr, nullptr, sk->d_out_idx, sk->d_out_which, scale,
                                 out_dev, true));
        }
    }
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
