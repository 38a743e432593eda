/*
 * bcpp.h - exact betweenness centrality with respect to a target set, Brandes++
 * (Erdos, Ishakian, Bestavros, Terzi, "A Divide-and-Conquer Algorithm for Betweenness
 * Centrality"), on AMD MI355X (gfx950).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Graph: undirected, simple, integer weights >= 1 (Sec. 3 "Notation" allows any
 *   non-negative weight; zero weights make path counts ill-defined, so they are
 *   rejected). It is passed as a symmetric CSR (bc_csr): every edge {u,v} appears as
 *   the arcs u->v and v->u with the same weight, rows sorted by column, no self-loop,
 *   no duplicate.
 * Scores: C(v) = sum over target pairs {s,t}, s != t, v not in {s,t}, of
 *   sigma(s,t|v) / sigma(s,t) (Sec. 3, eq. centrality, with delta(s,t|v) as defined
 *   there). Pairs with no path contribute 0. By default each unordered pair counts
 *   once; flag BC_ORDERED returns the paper's sum over ordered pairs, which is exactly
 *   twice as large.
 * Integers: distances and path counts are exact (path counts uint64). If any path
 *   count sigma(s,v) from a target s that a call needs reaches 2^64 the call fails
 *   with BC_E_OVERFLOW. Dependencies and scores are IEEE double; they agree with an
 *   exact evaluation to a relative 1e-9 (every term is non-negative).
 * Ownership: input arrays are owned by the caller and only read during the call.
 *   Output arrays are allocated by the caller. Handles belong to the library until
 *   the matching _destroy call. "_dev" entry points take device pointers (for example
 *   torch tensors on the GPU); the others take host pointers.
 * Errors: every int-returning call returns a bc_status and never aborts or throws;
 *   bc_last_error() gives a message for the calling thread. On error, outputs are
 *   unspecified and handles passed in stay valid.
 * Threads: calls on different handles may run concurrently; calls on one graph or
 *   skeleton handle are serialised by the caller. Server calls are thread-safe.
 * Streams: work is issued on the HIP stream given to bc_graph_create (NULL = the
 *   null stream); host-pointer entry points return after their results are on the
 *   host, _dev entry points return after their work is complete on the device.
 */
#ifndef BCPP_H
#define BCPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bc_status {
    BC_OK = 0,
    BC_E_INVAL = 1,    /* malformed graph, target set, partition or handle */
    BC_E_OVERFLOW = 2, /* a needed path count reached 2^64 */
    BC_E_NOMEM = 3,    /* device memory or a configured budget exhausted */
    BC_E_DEVICE = 4,   /* a HIP call failed */
    BC_E_AGAIN = 5,    /* queue full, try again later */
    BC_E_NOTFOUND = 6  /* unknown ticket or graph id */
} bc_status;

/* flags */
#define BC_ORDERED 0x1u    /* ordered-pair sum: 2x the default unordered score */
/* Run every traversal on the multi-group engine (64 sources per wave, state in HBM),
 * also where the graph (or skeleton) is small enough for the LDS-resident kernel
 * (one source at a time per workgroup, its state in LDS), which is used otherwise.
 * Both compute the same d and sigma; scores agree within the stated tolerance. */
#define BC_ENGINE_ONLY 0x2u
/* Batch runs of plain Brandes: run eagerly instead of replaying the batch's HIP graph.
 * (The first plain run of a batch builds its groups, buffers and launch records once
 * and captures the launches into a graph; later runs replay it. Results are the same
 * bit for bit either way.) */
#define BC_NO_GRAPH 0x4u

typedef struct bc_csr {
    int32_t n;              /* nodes */
    int64_t nnz;            /* arcs = 2 x undirected edges */
    const int64_t* row_ptr; /* [n+1], row_ptr[0] = 0, nondecreasing, row_ptr[n] = nnz */
    const int32_t* col;     /* [nnz], in [0,n), strictly increasing in each row */
    const int32_t* w;       /* [nnz], >= 1, symmetric; NULL = all weights 1 */
} bc_csr;

typedef struct bc_graph bc_graph;
typedef struct bc_skeleton bc_skeleton;
typedef struct bc_batch bc_batch;
typedef struct bc_server bc_server;

/* Message for the last failed call on this thread ("" if none). */
const char* bc_last_error(void);

/* ------------------------------------------------------------------ graphs ---- */

/* Validate g and copy it to the device. Fails with BC_E_INVAL on an asymmetric
 * CSR, a weight < 1, a self-loop, a duplicate or unsorted column, an out-of-range
 * entry, or a weight sum that could reach 2^31 ((n-1) * max weight >= 2^31).
 * hip_stream: a hipStream_t (or NULL) on which all later work for this graph runs. */
int bc_graph_create(const bc_csr* g, void* hip_stream, bc_graph** out);
void bc_graph_destroy(bc_graph* g);

/* --------------------------------------------------- the Brandes subroutine ---- */

/* Shortest-path distances and path counts from each source (Sec. 3, eq. parentsall),
 * as the kernel that computes the scores finds them: the source groups of a plain
 * Brandes pass over src (src flagged as targets) run their forward and backward
 * sweeps and write each source's d and sigma out after its forward sweep. (With the
 * environment variable BCPP_RESIDENT=0 the multi-group engine computes them.) src may
 * repeat a node. d: [nsrc * n] row-major by source, -1 = unreachable. sigma:
 * [nsrc * n], 0 = unreachable. Either output may be NULL. BC_E_OVERFLOW if a count
 * reaches 2^64. */
int bc_sssp_counts(const bc_graph* g, const int32_t* src, int32_t nsrc, int64_t* d,
                   uint64_t* sigma);

/* Plain target-set Brandes (Sec. 3, eqs. dep, brandes, centrality): the scores of all
 * n nodes with respect to the distinct targets S[0..nS). nS < 2 gives all zeros.
 * BC_E_INVAL on an out-of-range or repeated target. bc_out: [n] doubles. */
int bc_brandes_plain(const bc_graph* g, const int32_t* S, int32_t nS, uint32_t flags,
                     double* bc_out);
/* Same, with S and bc_out in device memory. */
int bc_brandes_plain_dev(const bc_graph* g, const int32_t* S_dev, int32_t nS,
                         uint32_t flags, double* bc_out_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops or harnesses that forbid hipMalloc): bc_brandes_plain_dev that
 * allocates nothing. Every buffer its kernels use beyond S_dev and bc_out_dev (target
 * flags, per-group score rows, forward records, one-source state of ranges beyond LDS,
 * launch records, error word) comes from one fixed device array of
 * bc_noalloc_scratch_bytes() bytes (256 MiB) that the library holds on each GPU it has
 * run on until the process ends. Source groups run in waves of as many as fit in it
 * (each wave's scores are added to the previous waves'), so results agree with
 * bc_brandes_plain_dev within the stated tolerance, not always bit for bit. Fails with
 * BC_E_NOMEM, before any device work, when one group over g does not fit (about 5 MB
 * per group at 100,000 nodes and 800,000 arcs). Flags: BC_ORDERED only. Calls on one
 * GPU share its array, which keeps the last call's contents: calls that overlap on one
 * GPU (from different threads or streams) race and must be serialised by the caller.
 * Returns after the work is complete on the device. */
int bc_brandes_plain_noalloc(const bc_graph* g, const int32_t* S_dev, int32_t nS,
                             uint32_t flags, double* bc_out_dev);
size_t bc_noalloc_scratch_bytes(void);

/* ---------------------------------------------------------------- Brandes++ ---- */

/* Build_SK (Sec. 5, Alg. 2 with the partition P' of Step 1): every target leaves its
 * part and becomes a singleton part; frontiers F_i are the nodes with an edge into
 * another part; Dijkstra_SK (Sec. 4, eq. frontierparents) runs from every frontier
 * node inside its part, on the device, giving the clique tuples <d(f,q), sigma(f,q)>
 * and the per-part tables d(f,v), sigma(f,v) of Step 3. Cut edges R keep <w(e), 1>.
 * Clique edges and table entries with sigma = 0 carry no shortest path and are
 * dropped. part: [n] labels in [0,k). S: distinct targets. The skeleton stays in
 * device memory and is bound to g (use it only with g). */
int bc_partition_sk(const bc_graph* g, const int32_t* part, int32_t k, const int32_t* S,
                    int32_t nS, bc_skeleton** out);
void bc_skeleton_destroy(bc_skeleton* sk);

/* A partition for bc_partition_sk computed on the device (the paper takes P from
 * third-party clustering tools, Sec. 7; scores do not depend on P, only Brandes++'s
 * speed does). Size-constrained label propagation: each node starts alone; in each of
 * `rounds` rounds the nodes whose SplitMix64 hash of (seed, round, node) is odd move to
 * the label most common among their neighbours among labels held by fewer than
 * max_part nodes after the previous round (0 = no cap), if it is strictly more common
 * than their own (ties between other labels go to the smallest); labels are then
 * renumbered 0..k-1 in increasing order. Deterministic for given arguments. part_out:
 * [n] host array; *k_out receives k. */
int bc_partition_lp(const bc_graph* g, int32_t max_part, int32_t rounds, uint64_t seed,
                    int32_t* part_out, int32_t* k_out);

typedef struct bc_sk_stats {
    int32_t n;              /* nodes of G */
    int32_t n_sk;           /* |V_SK|: frontier nodes of P' */
    int32_t k_prime;        /* parts of P' that hold at least one node */
    int32_t largest_part;   /* nodes in the largest part of P' */
    int64_t r_arcs;         /* arcs of R (2 per cut edge) */
    int64_t clique_arcs;    /* clique arcs kept (sigma > 0) */
    int64_t clique_pruned;  /* ordered frontier pairs of one part dropped (sigma = 0) */
    int64_t table_nnz;      /* table entries kept (interior node, frontier) */
    int64_t table_pruned;   /* table entries dropped (sigma = 0) */
    int64_t dsk_sources;    /* Dijkstra_SK runs (frontier nodes of parts with >1 node) */
    int64_t device_bytes;   /* device memory held by the skeleton */
} bc_sk_stats;

int bc_skeleton_stats(const bc_skeleton* sk, bc_sk_stats* out);

/* Copy the skeleton out for inspection. nodes: [n_sk] original ids in skeleton order.
 * row_ptr: [n_sk+1]; col: [r_arcs + clique_arcs] skeleton indices; len and mult: the
 * characteristic tuple of each arc. tab_node: [n_int] original ids of interior nodes
 * with at least one entry; tab_ptr: [n_int+1]; tab_f (skeleton index), tab_d, tab_sigma:
 * [table_nnz]. Pass NULL for any output not wanted; *n_int receives the row count. */
int bc_skeleton_export(const bc_skeleton* sk, int32_t* nodes, int64_t* row_ptr,
                       int32_t* col, uint32_t* len, uint64_t* mult, int32_t* n_int,
                       int32_t* tab_node, int64_t* tab_ptr, int32_t* tab_f,
                       uint32_t* tab_d, uint64_t* tab_sigma);

/* Distances and multiplicity-weighted path counts on G_SK (Sec. 5, eq. multiparents)
 * from skeleton nodes src (original ids, each a skeleton node) to every skeleton node,
 * as Brandes_SK finds them: the source groups of a Brandes_SK + Centrality pass over
 * src run their sweeps and write each source's d and sigma out after its forward
 * sweep (BCPP_RESIDENT=0: the multi-group engine). d, sigma: [nsrc * n_sk] in
 * skeleton order. */
int bc_skeleton_sssp_counts(const bc_skeleton* sk, const int32_t* src, int32_t nsrc,
                            int64_t* d, uint64_t* sigma);

/* Brandes++ (Sec. 5, Alg. 1): Brandes_SK on the skeleton (eqs. multiparents,
 * multibrandes) for the skeleton's targets, then Centrality (eq. localcentrality) for
 * every interior node: per group of sources inside the traversal kernel, or, for
 * groups of 4 to 64 sources or with at least 8192 table rows, in kernels of their own
 * after it, from d, sigma and the coefficients the traversal saved per source (device
 * workspace up to 128 MiB per such group). Scores of all n nodes of g; BC_E_NOMEM when
 * the workspace cannot be allocated. */
int bc_brandes_pp(const bc_graph* g, const bc_skeleton* sk, uint32_t flags,
                  double* bc_out);
int bc_brandes_pp_dev(const bc_graph* g, const bc_skeleton* sk, uint32_t flags,
                      double* bc_out_dev);

/* Brandes++All (Sec. 6, Alg. 3): the scores over all pairs of nodes (S = V) from the
 * skeleton. For every ordered pair of parts (P_i, P_j) of part ([n] labels in [0,k)),
 * i = j included, the skeleton is built with the nodes of P_i and P_j as singleton
 * parts, and Brandes_SK with Centrality runs from the sources P_i, counting as
 * destinations only the nodes of P_j (the indicator of eq. multibrandes is I[v in
 * P_j]); the k^2 results are summed. Equal to bc_brandes_plain with S = V within the
 * stated tolerance, for any partition. Build_SK's Dijkstra_SK runs once for part and
 * serves every pass; each pass assembles its own skeleton, and the passes' Brandes_SK
 * groups (k * n sources in all) share resident launches. It is much slower than
 * bc_brandes_plain; it is the paper's all-pairs route.
 * Flags: BC_ORDERED only. bc_out: [n] doubles (host). */
int bc_brandes_pp_all(const bc_graph* g, const int32_t* part, int32_t k, uint32_t flags,
                      double* bc_out);

/* ---------------------------------------------------------------- batching ---- */

/* Many independent graphs in one device run: each graph g_i with its own partition
 * and targets. All graphs' groups of sources (and, for Brandes++, all parts) run in
 * the same launches. Both passes replay one captured HIP graph each, built on the
 * pass's first run (for Brandes++ the whole pipeline: Build_SK phases 1 and 2,
 * Dijkstra_SK, the skeleton assembly, Brandes_SK + Centrality and the reduction, all
 * recomputed by every replay); BC_NO_GRAPH, BC_ENGINE_ONLY, or a group too large for
 * the resident kernel, runs the pass eagerly instead. Results are bitwise the same
 * either way. */
int bc_batch_create(int32_t ngraphs, const bc_csr* graphs, const int32_t* const* parts,
                    const int32_t* ks, const int32_t* const* S, const int32_t* nS,
                    void* hip_stream, bc_batch** out);
#define BC_BATCH_PLAIN 0x0u
#define BC_BATCH_PP 0x100u
/* Run plain Brandes or Brandes++ (flag BC_BATCH_PP) for every graph of the batch.
 * bc_out[i]: host array of graphs[i].n doubles. */
int bc_batch_run(bc_batch* b, uint32_t flags, double* const* bc_out);
void bc_batch_destroy(bc_batch* b);

/* ----------------------------------------------------------------- serving ---- */

/* A request loop on its own host thread: graphs stay resident; queries (a graph id
 * and a target set) are admitted while their device memory fits hbm_budget_bytes and
 * fewer than max_inflight run, and the admitted queries' work advances together on
 * the device (continuous batching: a query admitted later joins the running launches
 * at the next step). */
int bc_server_create(size_t hbm_budget_bytes, int32_t max_inflight, bc_server** out);
/* Register a graph and its partition (copied). *gid receives its id. Dijkstra_SK
 * (Sec. 4) runs once here for every part of the partition as given; a query's build
 * takes these results for the parts that hold none of its targets (their nodes,
 * induced subgraphs and frontiers are the same in the query's P', Sec. 5 Step 1) and
 * runs Dijkstra_SK only in the parts its targets touch. They stay in device memory,
 * outside hbm_budget_bytes (bc_server_stats.cache_bytes). */
int bc_server_add_graph(bc_server* s, const bc_csr* g, const int32_t* part, int32_t k,
                        int32_t* gid);
/* Queue a Brandes++ query (S copied). BC_E_AGAIN if the queue is full. */
int bc_query_submit(bc_server* s, int32_t gid, const int32_t* S, int32_t nS,
                    uint32_t flags, uint64_t* ticket);
/* Non-blocking. *done = 1 and bc_out (n doubles) filled once the query finished; the
 * ticket is then released. A failed query reports its status here. */
int bc_query_poll(bc_server* s, uint64_t ticket, double* bc_out, int32_t* done);

typedef struct bc_server_stats {
    int64_t submitted, completed, failed;
    int64_t queued, inflight;
    int64_t iterations;       /* device steps issued */
    double p50_ms, p99_ms;    /* submit-to-completion latency of completed queries */
    int64_t peak_bytes;       /* peak device memory admitted */
    int64_t cache_bytes;      /* device memory of the graphs' kept Dijkstra_SK results */
    int64_t dsk_groups_cached;  /* Dijkstra_SK groups taken from them (parts without targets) */
    int64_t dsk_groups_run;     /* Dijkstra_SK groups run for queries */
} bc_server_stats;
int bc_server_stats_get(bc_server* s, bc_server_stats* out);
void bc_server_destroy(bc_server* s);

/* ------------------------------------------------------------- measurement ---- */

/* Kernel timing with HIP events recorded around every launch on the launch stream.
 * Off by default. kind: BC_K_* below. */
#define BC_K_SELECT 0
#define BC_K_SETTLE 1
#define BC_K_PUSH 2
#define BC_K_BACKWARD 3
#define BC_K_CENTRALITY 4
#define BC_K_SCHED 5
#define BC_K_OTHER 6
#define BC_K_RESIDENT 7 /* the LDS-resident kernel: 32 bytes per (source, arc) and 20 per
                         * (source, node) reached, the per-source state a traversal from
                         * memory would move (Sec. 3 forward and backward sweeps) */
#define BC_K_DIJKSTRA_SK 8 /* the same kernel running Dijkstra_SK groups (forward sweep
                            * only, restricted counts): 12 bytes per (source, arc) and 12
                            * per (source, node) reached */
#define BC_K_COUNT 9
void bc_profile_enable(int on);
/* Totals since the last reset: launches, summed milliseconds, and the algorithmic
 * bytes the kernel's work units account for (see the kernel's documentation). */
int bc_profile_read(int kind, int64_t* launches, double* ms, double* alg_bytes);
void bc_profile_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* BCPP_H */
