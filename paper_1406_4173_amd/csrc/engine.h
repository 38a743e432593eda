// The multi-group Brandes engine: shortest-path counting and dependency accumulation
// for many groups of up to 64 sources at once, each group over its own node range
// of a CSR graph.
//
// One group = one wave64 row per node: lane b of the row holds the state of source
// src[b] at that node (distance, path count, dependency coefficient). The search is
// distance-synchronous: a group's step D settles exactly the (node, source) pairs at
// distance D, pulls their path counts from tight parents (Sec. 3, eq. parentsall, or
// eq. multiparents with multiplicities), then relaxes their out-arcs. The backward
// sweep replays the recorded steps in reverse and pulls dependencies from tight
// children (eq. brandes, or eq. multibrandes). Every group advances one step per
// engine iteration, so groups of different graphs, sizes and phases share launches.
#pragma once

#include <functional>

#include "common.h"

namespace bcpp {

enum : uint32_t { NF_TARGET = 1u, NF_BLOCKED = 2u };

enum : uint32_t {
    GF_RESTRICT = 1u,  // Dijkstra_SK: blocked (frontier) parents add no paths, except the source
    GF_BACKWARD = 2u,  // run the dependency sweep after the forward search
    GF_CENT = 4u,      // then the interior-node Centrality pass over the tables
    GF_UNIT = 8u,      // every arc has length 1 (plain stores replace atomics)
    GF_EXPORT = 16u,   // resident backward groups: also write d and sigma after the forward
    // resident GF_CENT groups: the interior rows are swept after the launch by a kernel
    // of their own, for all of the group's sources at once, from d and sigma (odist,
    // osig) and the backward's coefficients (ocoef) of every node per source; set by
    // resident_alloc for the groups that qualify (resident_interior_split)
    GF_ISPLIT = 32u,
};

enum : int32_t { PH_DONE = 0, PH_FWD = 1, PH_BWD = 2, PH_CENT = 3 };

enum : uint32_t { ERR_OVERFLOW = 1u, ERR_HIST = 2u, ERR_REC = 4u, ERR_TWIN = 8u };

// An arc's head, length, reverse arc and multiplicity in one 16-byte record.
struct __align__(16) ArcRec {
    uint32_t head, len, twin, mult;
};

struct EGraph {
    const int64_t* row_ptr = nullptr;  // [nodes+1]
    const int32_t* col = nullptr;      // [arcs]
    const uint32_t* len = nullptr;     // [arcs] >= 1; nullptr = all 1
    const uint64_t* mult = nullptr;    // [arcs]; nullptr = all 1
    const uint8_t* nflag = nullptr;    // [nodes] NF_* bits; nullptr = none
    const int64_t* twin = nullptr;     // [arcs] index of the reverse arc (backward groups)
    // [arcs] the same four per arc in one 16-byte record (head, length, reverse arc,
    // multiplicity, each uint32), or nullptr; device-memory groups read it, so that an
    // arc's reverse arc and multiplicity come in the line that holds its head
    const ArcRec* arc = nullptr;
};

struct GroupDesc {
    EGraph g;
    int32_t lo = 0, hi = 0;  // node range [lo, hi) of g this group searches
    uint32_t flags = 0;
    int32_t nsrc = 0;
    int64_t arc_lo = 0;         // row_ptr[lo]: first arc of the range
    int64_t arcs = 0;           // row_ptr[hi] - row_ptr[lo]
    uint32_t* dist = nullptr;   // [(hi-lo)*64] settled distance, INF while unsettled
    uint64_t* sigma = nullptr;  // [(hi-lo)*64] path count
    double* coef = nullptr;     // [(hi-lo)*64] (I[v in S] + delta(s|v)) / sigma(s,v)
    double* delta = nullptr;    // [(hi-lo)*64] delta(s|v)
    uint32_t* nd = nullptr;     // [hi-lo] smallest pending distance over unsettled lanes
    uint64_t* done = nullptr;   // [hi-lo] lanes settled at the node
    // offers: ring[node][D mod ring_len] = lanes offered distance D by a settled
    // neighbour (ring_len = longest arc + 1, so pending offers never share a slot;
    // 0 = not known: the engine refuses such a group, the resident kernel scans)
    uint64_t* ring = nullptr;
    int32_t ring_len = 0;
    double* cacc = nullptr;     // [hi-lo] this group's share of the scores
    uint64_t* tmask = nullptr;  // [arcs] per arc u->x: lanes in which u is a tight parent of x
    int32_t* hist = nullptr;    // settled nodes in step order (backward only)
    uint64_t* hmask = nullptr;  // and the lanes each settled
    int64_t hist_cap = 0;
    uint32_t* rec_d = nullptr;  // per recorded step: distance, history offset, count
    int64_t* rec_off = nullptr;
    int32_t* rec_cnt = nullptr;
    int32_t rec_cap = 0;
    // Centrality tables (GF_CENT): interior row i has entries trow[i]..trow[i+1] of
    // (tcol = node of g in this group's range, tlen = d(f,v), tsig = sigma(f,v)).
    const int64_t* trow = nullptr;
    const int32_t* tcol = nullptr;
    const uint32_t* tlen = nullptr;
    const uint64_t* tsig = nullptr;
    int32_t t_lo = 0;        // first table row of this group; rows [t_lo, t_lo + tn)
    int32_t tn = 0;
    double* cint = nullptr;  // [tn] this group's share of the interior scores
    // resident groups too large for LDS: the one-source state in device memory
    uint32_t* gdist = nullptr;  // [hi-lo]
    uint64_t* gsig = nullptr;   // [hi-lo]
    uint32_t* gtb = nullptr;    // [ceil(arcs/32)] their backward's tight-arc bitmap
    // resident backward groups: the forward's per-wave queue record and step distances
    int32_t* rlist = nullptr;
    uint32_t* steps = nullptr;  // [hi-lo+1]
    // GF_EXPORT: d and sigma of every node of the range after each source's forward
    // sweep, source-major: row b (the group's b-th source) is odist[b * (hi-lo) ..]
    uint32_t* odist = nullptr;
    uint64_t* osig = nullptr;
    // GF_ISPLIT: (I[v in S] + delta(s|v)) / sigma(s,v) of every node after each source's
    // backward sweep (fp64 bits), laid out as odist
    uint64_t* ocoef = nullptr;
    // GF_ISPLIT: the same three node-major, [hi-lo][lanes] each (lanes: a power of two
    // >= nsrc), for the interior sweep; see interior_rows_bytes for the layout
    unsigned char* xsave = nullptr;
    int32_t src[LANES];      // source node ids of g, -1 = unused lane
};

// A unit of work in a list: a node of a group and the lanes it handles this step
// (for centrality items, v is the table row).
struct NodeItem {
    int32_t g;
    int32_t v;
    unsigned long long mask;
};

struct GroupDyn {
    uint32_t D;
    int32_t phase;
    int32_t nrec;
    int32_t rec_i;
    int64_t hist_len;
    int64_t rec_start;
    uint32_t nextmin;
    uint32_t err;
};

// Device memory needed by a group shaped like G (range, arcs, nsrc, flags, tn,
// ring_len), with room for max_steps recorded steps.
size_t group_bytes(const GroupDesc& G, int64_t max_steps);

// Carve a group's buffers from the arena. Returns false if it does not fit.
bool group_alloc(Arena& a, GroupDesc& G, int64_t max_steps);

// An engine instance: slots for groups, the scan-chunk table and the work lists.
struct Engine {
    hipStream_t stream = nullptr;
    int32_t cap = 0;           // group slots
    GroupDesc* d_desc = nullptr;
    GroupDyn* d_dyn = nullptr;
    int32_t* d_chunk_g = nullptr;
    int32_t* d_chunk_off = nullptr;
    int64_t nchunks = 0;
    int64_t chunk_cap = 0;
    NodeItem* d_wl = nullptr;  // 3 lists: forward, backward, centrality
    int64_t wl_cap = 0;
    uint32_t* d_ctr = nullptr; // [0..2] list counts, [3] active groups
    uint32_t* h_ctr = nullptr; // pinned mirror
    int blocks = 0;            // persistent grid of the work kernels
    bool profile_bytes = false;

    // Allocate the engine's own buffers in `a` for up to `slots` groups covering at
    // most `positions` scan positions (sum over groups of max(range, tn)).
    int setup(Arena& a, hipStream_t s, int32_t slots, int64_t positions);
    // Install groups into slots [first, first + n) and initialise their state.
    int install(const GroupDesc* groups, int32_t first, int32_t n);
    // Install groups[j] into slot slots[j] (any free slots), initialise their state and
    // make the slots in `live` the engine's working set. One synchronisation.
    int install_at(const GroupDesc* groups, const int32_t* slots, int32_t n,
                   const std::vector<GroupDesc>& host_desc, const std::vector<int32_t>& live);
    GroupDesc* d_stage = nullptr;  // staging for install_at
    int32_t* d_stage_slot = nullptr;
    // Rebuild the scan-chunk table from host descriptors of slots [0, nslots).
    int set_chunks(const std::vector<GroupDesc>& host_desc, const std::vector<int32_t>& live);
    // Issue `iters` engine iterations (no host synchronisation).
    int iterate(int iters);
    // Sum each backward group's per-lane dependencies into its node scores.
    int finish_scores();
    // Run until every installed group is done; then read back per-group errors.
    int run_to_completion(int32_t nslots, std::vector<GroupDyn>* dyn_out = nullptr);
};

// Run the given groups to completion on a fresh engine (synchronous helper).
int run_groups(Arena& a, hipStream_t s, std::vector<GroupDesc>& groups, int64_t max_steps);
// Per-node sums of the lanes' dependencies for the backward groups named by the chunk
// table (chunks of 256 positions, as built by Engine::set_chunks).
int lane_sum(hipStream_t s, const GroupDesc* d_desc, const int32_t* d_chunk_g,
             const int32_t* d_chunk_off, int64_t nchunks);
// Same, for groups whose state has already been carved out (group_alloc).
int run_groups_prealloc(Arena& a, hipStream_t s, std::vector<GroupDesc>& groups);

// Sum per-group partial scores into out[v] for v in [0, n), in group order:
//   out[v] (+)= scale * sum_{g in [g0[v], g1[v])} part[g][idx[v]]
// where part[g] is cacc (which[v] == 0) or cint (which[v] == 1) of group g. A null
// g0/g1 means all groups, a null idx means idx[v] = v, idx[v] < 0 gives 0.
int reduce_scores(hipStream_t s, Arena& a, const std::vector<GroupDesc>& groups,
                  int32_t n, const int32_t* d_g0, const int32_t* d_g1,
                  const int32_t* d_idx, const uint8_t* d_which, double scale,
                  double* out_dev, bool accumulate);
// The same in two parts (no synchronisation): reduce_upload copies the groups' score
// pointers to the device (on s), reduce_launch only enqueues the reduction.
struct ReducePtrs {
    const double** pc = nullptr;
    const double** pi = nullptr;
    int32_t ngroups = 0;
};
int reduce_upload(hipStream_t s, Arena& a, const std::vector<GroupDesc>& groups, ReducePtrs* R);
int reduce_launch(hipStream_t s, const ReducePtrs& R, int32_t n, const int32_t* d_g0, const int32_t* d_g1,
                  const int32_t* d_idx, const uint8_t* d_which, double scale, double* out_dev,
                  bool accumulate);

}  // namespace bcpp

namespace bcpp {
// Zero `bytes` bytes of device memory at p on stream s with a fill kernel.
int zero_device(hipStream_t s, void* p, size_t bytes);
// Exclusive prefix sum out[i] = in[0] + .. + in[i-1] of n items (T = int32_t or
// int64_t; in == out allowed), with scan_scratch_bytes(n) bytes of scratch.
size_t scan_scratch_bytes(int64_t n);
template <class T>
int exclusive_scan(hipStream_t s, const T* in, T* out, int64_t n, void* scratch);
// Device bytes an Engine needs for `slots` groups over `positions` scan positions.
size_t engine_bytes(int32_t slots, int64_t positions);

// ---- LDS-resident kernel (resident.hip) ----
// One workgroup per group runs the group's sources one after another with the state
// of one source (distance and path count of every node of the range) in LDS. Used
// for groups whose node range fits; fills cacc (and cint for GF_CENT groups). For
// resident groups, dist and sigma point at [tn] interior scratch instead of per-lane
// state, and no other engine buffer is used.
// Largest node range that fits in LDS (0: kernel unavailable or switched off).
int64_t resident_max_range();
// Whether the resident kernel takes a group over `range` nodes: in LDS when it fits,
// else with the state in device memory. Environment BCPP_RESIDENT=lds keeps larger
// ranges on the engine, BCPP_RESIDENT=0 every range.
bool resident_takes(int64_t range);
// Sources per resident group for a source set of nsrc (a function of nsrc only, so a
// graph is split the same way alone and inside a batch).
int32_t resident_sources_per_group(int64_t nsrc);
// Sources per Dijkstra_SK group for a part whose nodes plus arcs are part_work: 64, or
// with a tuned work budget per group, budget / part_work within [8, 64]. A function of
// the part alone, so a part is split the same way in every build that holds it.
int32_t dsk_sources_per_group(int64_t part_work);
size_t resident_group_bytes(const GroupDesc& G);
// Whether a Brandes_SK group with tables sweeps its interior rows in the kernel of its
// own (GF_ISPLIT): at most 64 sources, at least 4 or at least 8192 table rows, and its
// saved rows within a fixed size; a function of the group alone. Environment
// BCPP_ISPLIT=0 keeps every group's rows in the resident kernel.
bool resident_interior_split(const GroupDesc& G);
bool resident_alloc(Arena& a, GroupDesc& G);
// Workspace run_resident takes from the arena for `ngroups` groups.
size_t resident_launch_bytes(size_t ngroups);
// Run the groups to completion (synchronises); BC_E_OVERFLOW if a count reached 2^64.
int run_resident(hipStream_t s, Arena& a, const std::vector<GroupDesc>& groups);
int run_resident(hipStream_t s, Arena& a, const GroupDesc* const* groups, size_t n);
// The same in two parts for callers that must not block: resident_upload copies
// compact launch records (host to device, on s) and clears the error word;
// resident_launch only enqueues kernels, so it can go on a stream with work still
// pending. After the launch completes, *d_err has ERR_OVERFLOW set if a count reached
// 2^64. Classes 0-2 hold the state in LDS (256, 512, 1024 threads), class 3 in device
// memory, class 4 its distances as one byte per node in LDS and its counts in device
// memory (ranges beyond LDS whose arcs are at most 63 long).
struct RGroup;
struct RCtx;
struct IGroup;
struct ResidentLaunch {
    RGroup* d_rg[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int32_t count[5] = {0, 0, 0, 0, 0};
    size_t lds[5] = {0, 0, 0, 0, 0};
    const RCtx* d_ctx = nullptr;
    const int32_t* d_src = nullptr;
    uint32_t* d_err = nullptr;
    // GF_ISPLIT groups: their interior-row sweep, launched after the groups' kernels
    const IGroup* d_ig = nullptr;
    int32_t n_ig = 0;
    int32_t n_ig_wide = 0;   // the first n_ig_wide share entry loads across a row's threads
    int64_t ig_blocks = 0;   // k_interior blocks of those
    int64_t ig_nblocks = 0;  // and of the rest
    int64_t ig_tblocks = 0;  // blocks of the transpose before them
    // each grid's blocks per group when every group owns the same number, else 0
    int64_t ig_wstride = 0, ig_nstride = 0, ig_tstride = 0;
    // profiler kind of the launches: BC_K_DIJKSTRA_SK when every group is forward-only
    int kind = BC_K_RESIDENT;
};
int resident_upload(hipStream_t s, Arena& a, const std::vector<GroupDesc>& groups, ResidentLaunch* L);
int resident_upload(hipStream_t s, Arena& a, const GroupDesc* const* groups, size_t n, ResidentLaunch* L);
int resident_launch(hipStream_t s, const ResidentLaunch& L);
// Distances and path counts from resident groups run with GF_EXPORT, copied out
// source-major over a range of n nodes (-1 and 0 where a node is unreachable).
// Group j holds the sources [j * spg, j * spg + nsrc_j) of the call. make(g0, g1)
// gives the descriptors of groups [g0, g1); bind(W, groups), once the workspace is
// reserved (bind_bytes of it for bind), takes what they share from W and completes them.
int run_exported(hipStream_t s, Arena& W, int32_t n, int32_t nsrc, int32_t spg,
                 const std::function<std::vector<GroupDesc>(int32_t, int32_t)>& make,
                 const std::function<int(Arena&, std::vector<GroupDesc>&)>& bind, size_t bind_bytes,
                 int64_t* d, uint64_t* sigma);
}  // namespace bcpp
