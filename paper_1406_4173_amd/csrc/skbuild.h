// Build_SK in stages, so that a caller can run the Dijkstra_SK groups on an engine of
// its own (the serving loop shares one engine among queries).
#pragma once

#include <functional>
#include <vector>

#include "engine.h"
#include "graph.h"

namespace bcpp {

// Per Dijkstra_SK group: which slice of its part's frontier it searches from.
struct DskInfo {
    int32_t nf;       // |F_p|
    int32_t fl0;      // local index of the group's lane 0 source
    int32_t nsrc;     // sources in this group
    int32_t sk_base;  // skeleton id of the part's first frontier node
};

struct SkBuild {
    const bc_graph* g = nullptr;
    int32_t n = 0;
    int64_t nlab = 0;
    bool weighted = false;
    std::vector<int32_t> S;         // targets (original ids)
    std::vector<int32_t> lab;       // P' labels
    std::vector<uint8_t> fr, is_t;  // frontier and target flags
    std::vector<int64_t> psize, pnf, poff, fbase;
    std::vector<int32_t> nid, old;  // renumbering (parts contiguous, frontier first)
    int32_t nsk = 0;
    std::vector<int64_t> irp;  // intra-part CSR, renumbered
    std::vector<int32_t> icol;
    std::vector<uint32_t> iw;
    std::vector<int64_t> rptr;  // cut arcs by skeleton id, rows sorted
    std::vector<int32_t> rcol;
    std::vector<uint32_t> rw;
    int64_t nR = 0;
    std::vector<GroupDesc> groups;  // Dijkstra_SK groups
    std::vector<DskInfo> info;
    std::vector<int32_t> int_local, int_g0, int_ng, int_node;  // interior table rows
    std::vector<int32_t> out_idx;
    std::vector<uint8_t> out_which;
    int32_t nint = 0;
    int64_t largest = 0, kprime = 0, clique_pairs = 0, table_pairs = 0;
    // device temporaries (set by upload)
    int64_t* d_irp = nullptr;
    int32_t* d_icol = nullptr;
    uint32_t* d_iw = nullptr;
    uint8_t* d_blk = nullptr;
    int64_t* d_rptr = nullptr;
    int32_t* d_rcol = nullptr;
    uint32_t* d_rw = nullptr;
    int32_t* d_rdeg = nullptr;
    int32_t* d_cdeg = nullptr;
    DskInfo* d_info = nullptr;
    int32_t *d_il = nullptr, *d_ig0 = nullptr, *d_ing = nullptr, *d_tdeg = nullptr;
    uint32_t* d_maxlen = nullptr;
    GroupDesc* d_desc = nullptr;

    // Host part: P', frontiers, renumbering, intra-part CSR, cut arcs, groups.
    int prepare(const bc_graph* g, const int32_t* part, int32_t k, const int32_t* S, int32_t nS,
                bool given_singletons);
    // Device bytes of upload(): temporaries plus the Dijkstra_SK group states.
    size_t temp_bytes() const;
    // Upper bound of the skeleton's own device bytes (all clique pairs and table
    // entries kept).
    size_t skeleton_bytes_bound() const;
    // Copy the temporaries to the device and carve the group states out of W.
    int upload(Arena& W, hipStream_t s);
    // After the Dijkstra_SK groups have run: count, size and fill the skeleton.
    // get_store(bytes, arena) must hand back an arena with at least `bytes` free.
    int assemble(Arena& W, hipStream_t s, bc_skeleton* sk,
                 const std::function<int(size_t, Arena*&)>& get_store);
};

// Brandes_SK groups (with the fused Centrality pass) over a skeleton, sources
// src[0..nsrc) in skeleton ids, restricted to skeleton ids [lo, hi) and table rows
// [t_lo, t_lo + tn).
std::vector<GroupDesc> bsk_groups(const bc_skeleton* sk, const int32_t* src, int32_t nsrc,
                                  int32_t lo, int32_t hi, int32_t t_lo, int32_t tn);
// Brandes_SK + Centrality groups of the whole skeleton for the LDS-resident kernel
// (resident_sources_per_group sources each, in target order); buffers not yet carved.
std::vector<GroupDesc> resident_bsk_groups(const bc_skeleton* sk);

}  // namespace bcpp
