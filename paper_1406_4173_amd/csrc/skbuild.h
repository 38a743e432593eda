// Build_SK on the device, in stages, so that a caller can run the Dijkstra_SK groups
// where it likes (the serving loop runs them as launches of their own).
//
//   prepare  validation on the host, then phase 1 on the graph's stream in the
//            graph's scratch arena: P' labels and target flags, frontier flags, and per
//            part of P' its size, frontier count and intra-part arc count, copied back;
//            on the host from those: part offsets, Dijkstra_SK groups, interior row
//            bases and the exact device bytes of phase 2.
//   upload   phase 2 into the caller's arena: renumbering (a stable radix sort on
//            (part, not frontier)), intra-part CSR and cut-arc rows (count, scan,
//            fill), blocked flags, interior rows, output maps, group states. After it
//            nothing refers to the scratch arena, so the next prepare may reuse it.
//   assemble after the Dijkstra_SK groups: skeleton rows, clique arcs, tables.
//
// The device work of each stage is also available on its own (issue_*): the same
// kernels and copies on the same buffers, with no host synchronisation. Given the same
// graph, partition and targets, the host values that the stages read back are the same
// every time, so a caller that keeps the SkBuild, its arenas and the skeleton can
// enqueue (or capture into a HIP graph) the whole build again without the host. Every
// buffer that a kernel accumulates into is cleared by a fill kernel inside the stage.
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
    int32_t n = 0, nS = 0;
    int64_t nlab = 0;
    int32_t k_in = 0;    // k of the given partition
    bool given = false;  // targets already carry singleton labels
    bool weighted = false;
    std::vector<int32_t> S;  // targets (original ids)
    // per part of P' (host copies of phase 1, and their prefix sums)
    std::vector<int32_t> psize, pnf;
    std::vector<uint64_t> parc;                 // intra-part arcs
    std::vector<int64_t> poff, fbase, aoff;     // node, skeleton-id and arc offsets
    std::vector<int32_t> p_g0, p_ng, ibase;     // groups and interior rows of each part
    int32_t nsk = 0, nint = 0;
    int64_t n_intra = 0, nR = 0;
    std::vector<GroupDesc> groups;  // Dijkstra_SK groups
    std::vector<DskInfo> info;
    int64_t largest = 0, kprime = 0, clique_pairs = 0, table_pairs = 0;
    size_t scan_bytes = 0;  // scratch of the device scans (exclusive_scan)
    int32_t ntiles = 1;    // tiles of the renumbering sort
    // phase 1 (graph scratch arena)
    int32_t* p_part = nullptr;
    int32_t* p_lab = nullptr;
    uint8_t* p_ist = nullptr;
    uint8_t* p_fr = nullptr;
    int32_t* p_S = nullptr;
    int32_t* p_psize = nullptr;
    int32_t* p_pnf = nullptr;
    unsigned long long* p_parc = nullptr;
    unsigned long long* p_cross = nullptr;
    // phase 2 (caller's arena)
    uint32_t *d_keys = nullptr, *d_keys2 = nullptr;  // renumbering sort
    int32_t* d_vals = nullptr;
    int32_t *d_hist = nullptr, *d_hoff = nullptr;
    int64_t *d_icnt = nullptr, *d_rcnt = nullptr;    // row counts before the scans
    int64_t *d_poff = nullptr, *d_fbase = nullptr;   // per part (copies of the host values)
    int32_t *d_ppnf = nullptr, *d_pg0 = nullptr, *d_png = nullptr, *d_ibase = nullptr;
    void* d_scan = nullptr;
    int32_t* d_old = nullptr;  // renumbered position -> original node
    int32_t* d_nid = nullptr;  // original node -> renumbered position
    int64_t* d_irp = nullptr;  // intra-part CSR, renumbered
    int32_t* d_icol = nullptr;
    uint32_t* d_iw = nullptr;
    uint8_t* d_blk = nullptr;
    int32_t* d_rdeg = nullptr;  // cut arcs per skeleton node
    int64_t* d_rptr = nullptr;  // cut arcs by skeleton id, rows sorted
    int32_t* d_rcol = nullptr;
    uint32_t* d_rw = nullptr;
    int32_t* d_cdeg = nullptr;
    DskInfo* d_info = nullptr;
    int32_t *d_il = nullptr, *d_ig0 = nullptr, *d_ing = nullptr, *d_tdeg = nullptr, *d_inode = nullptr;
    int32_t* d_out_idx = nullptr;
    uint8_t* d_out_which = nullptr;
    int32_t* d_nodes = nullptr;  // skeleton id -> original node
    uint8_t* d_sflag = nullptr;  // skeleton id -> NF_TARGET
    int32_t* d_srcsk = nullptr;  // target -> skeleton id, or -1 (isolated target)
    uint32_t* d_maxlen = nullptr;
    uint32_t* d_rmax = nullptr;
    uint32_t* d_bigm = nullptr;  // a multiplicity beyond 32 bits (packed arc records unused)
    GroupDesc* d_desc = nullptr;
    // row lengths (with a trailing zero) and their exclusive scans: the skeleton's
    // and the interior table's row offsets, copied into the skeleton by the fill
    int64_t *d_slen = nullptr, *d_srow = nullptr, *d_tlen = nullptr, *d_trow = nullptr;

    int prepare(const bc_graph* g, const int32_t* part, int32_t k, const int32_t* S, int32_t nS,
                bool given_singletons);
    // Device bytes of upload(): phase 2 arrays plus the Dijkstra_SK group states. A group
    // whose output lanes (dist, sigma) are set before upload() keeps them: it gets no
    // state, and the caller does not run it.
    size_t temp_bytes() const;
    int upload(Arena& W, hipStream_t s);
    // After the Dijkstra_SK groups have run: count, size and fill the skeleton.
    // get_store(bytes, arena) must hand back an arena with at least `bytes` free.
    int assemble(Arena& W, hipStream_t s, bc_skeleton* sk,
                 const std::function<int(size_t, Arena*&)>& get_store);

    // Device work only, on stream s: phase 1; phase 2 (sort, CSR, rows, maps); the
    // clique and table counts with the row offsets they give; the skeleton fill
    // into sk's arrays.
    int issue_phase1(hipStream_t s) const;
    int issue_phase2(hipStream_t s) const;
    int issue_count(hipStream_t s) const;
    int issue_fill(hipStream_t s, const bc_skeleton* sk) const;
};

// What partition_impl leaves behind for a caller that replays the build: the build
// itself and, when the Dijkstra_SK groups ran on the resident kernel, their launch.
struct PartitionKeep {
    SkBuild b;
    bool resident = false;
    ResidentLaunch L;
};

// Dijkstra_SK results of a graph's parts, kept from one build without targets. A part
// that holds no target of a later build over the same partition has the same nodes,
// induced subgraph and frontier in that build's P' (a node next to a target of another
// part is a frontier already), and its nodes keep their order in the renumbering, so
// its Dijkstra_SK groups would write exactly these lanes: the later build takes them
// instead of running the groups (Sec. 5: parts are independent).
struct DskCache {
    bool ok = false;
    std::vector<int32_t> first, count, nf;  // per part: cached groups [first, first+count), |F_p|
    std::vector<uint32_t*> dist;            // per cached group: its output lanes
    std::vector<uint64_t*> sig;
    Arena store;
    size_t bytes = 0;
};

// Build_SK's Dijkstra_SK of every part of g under part (no targets) into *c, on g's
// stream, in g's work arena. Leaves c->ok false when a group would not take the
// resident kernel.
int build_dsk_cache(bc_graph* g, const int32_t* part, int32_t k, DskCache* c);

// After b.prepare and before b.upload: point the output lanes of b's Dijkstra_SK groups
// at c's for every part of the given partition that holds none of b's targets and has
// the cached group count and frontier size; preset[i] = 1 for each such group i.
// Returns the number of groups preset.
int32_t dsk_preset_from_cache(SkBuild& b, const DskCache& c, const int32_t* part,
                              std::vector<uint8_t>& preset);

// Brandes_SK groups (with the fused Centrality pass) over a skeleton, sources
// src[0..nsrc) in skeleton ids, restricted to skeleton ids [lo, hi) and table rows
// [t_lo, t_lo + tn).
std::vector<GroupDesc> bsk_groups(const bc_skeleton* sk, const int32_t* src, int32_t nsrc,
                                  int32_t lo, int32_t hi, int32_t t_lo, int32_t tn);
// Brandes_SK + Centrality groups of the whole skeleton for the LDS-resident kernel
// (resident_sources_per_group sources each, in target order); buffers not yet carved.
std::vector<GroupDesc> resident_bsk_groups(const bc_skeleton* sk);
// The same for the sources src (skeleton ids) with the target flags nflag ([n_sk]
// NF_TARGET bits: the nodes whose paths count as destinations).
std::vector<GroupDesc> resident_bsk_groups(const bc_skeleton* sk, const std::vector<int32_t>& src,
                                           const uint8_t* nflag);

}  // namespace bcpp
