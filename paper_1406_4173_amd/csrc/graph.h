// Graph and skeleton handles shared by the library's translation units.
#pragma once

#include <vector>

#include "engine.h"

struct bc_graph {
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t maxw = 1;
    bool unit = true;
    hipStream_t stream = nullptr;
    // host copy of the CSR (the partition step reads it)
    std::vector<int64_t> h_row_ptr;
    std::vector<int32_t> h_col;
    std::vector<int32_t> h_w;
    // device copy
    int64_t* d_row_ptr = nullptr;
    int32_t* d_col = nullptr;
    uint32_t* d_len = nullptr;  // null for unit weights
    int64_t* d_twin = nullptr;  // reverse arc of each arc
    bcpp::ArcRec* d_arc = nullptr;    // packed arc records (EGraph::arc), or null
    bcpp::Arena store;  // graph arrays
    bcpp::Arena work;   // per-call workspace
    bcpp::Arena out;    // staging for host-pointer outputs
    bcpp::Arena pre;    // scratch of the skeleton build's first phase (one build at a time)
};

struct bc_skeleton {
    const bc_graph* graph = nullptr;
    int32_t n = 0;           // nodes of G
    int32_t n_sk = 0;        // skeleton nodes
    int32_t n_int = 0;       // interior nodes with table entries
    int64_t m_arcs = 0;      // skeleton arcs
    int64_t t_nnz = 0;       // table entries
    int64_t max_dist = 0;    // bound on skeleton distances
    int32_t max_len = 1;     // longest skeleton arc
    bc_sk_stats stats{};
    // skeleton targets in skeleton ids (the sources of Brandes_SK), in target order
    std::vector<int32_t> h_src;
    // skeleton id of every target, in target order (-1: an isolated target)
    std::vector<int32_t> h_target_sk;
    // device arrays (all in `store`)
    int64_t* d_row_ptr = nullptr;  // [n_sk+1]
    int32_t* d_col = nullptr;      // [m_arcs]
    uint32_t* d_len = nullptr;     // [m_arcs]
    uint64_t* d_mult = nullptr;    // [m_arcs]
    int64_t* d_twin = nullptr;     // [m_arcs] reverse arc
    bcpp::ArcRec* d_arc = nullptr;       // [m_arcs] packed arc records (EGraph::arc), or null
    bcpp::ArcRec* d_arc_store = nullptr;  // their storage (filled by every build or replay)
    std::vector<int64_t> h_row_ptr;  // host copy of d_row_ptr
    uint8_t* d_nflag = nullptr;    // [n_sk] NF_TARGET
    int64_t* d_trow = nullptr;     // [n_int+1]
    int32_t* d_tcol = nullptr;     // [t_nnz] skeleton ids
    uint32_t* d_tlen = nullptr;    // [t_nnz]
    uint64_t* d_tsig = nullptr;    // [t_nnz]
    int32_t* d_nodes = nullptr;    // [n_sk] original ids
    int32_t* d_tnode = nullptr;    // [n_int] original ids
    int32_t* d_out_idx = nullptr;  // [n] per original node: skeleton id, interior row, or -1
    uint8_t* d_out_which = nullptr;  // [n] 0 = skeleton id, 1 = interior row
    bcpp::Arena store;
};

namespace bcpp {
// Multiplicities of a skeleton's arcs, or nullptr (all 1) when it has no clique arcs:
// then every arc is a cut arc <w, 1> and the traversals skip the multiplications.
inline const uint64_t* sk_mult(const bc_skeleton* sk) {
    return sk->stats.clique_arcs == 0 ? nullptr : sk->d_mult;
}
int graph_create(const bc_csr* csr, hipStream_t stream, bc_graph** out);
struct PartitionKeep;
struct DskCache;
// Build_SK on g's stream. With keep, the build and the Dijkstra_SK launch stay in
// *keep for a later replay of the device work (see SkBuild). With cache (built over the
// same graph and partition), the parts that hold no target take their Dijkstra_SK
// results from it instead of running their groups.
int partition_impl(const bc_graph* g, const int32_t* part, int32_t k, const int32_t* S, int32_t nS,
                   bc_skeleton** out, bool given_singletons, PartitionKeep* keep = nullptr,
                   const DskCache* cache = nullptr);
int validate_csr(const bc_csr* g, int32_t* maxw_out);
int validate_targets(int32_t n, const int32_t* S, int32_t nS);
int64_t max_steps_bound(int64_t range, int32_t lanes, int64_t max_dist);
size_t state_budget();
}  // namespace bcpp
