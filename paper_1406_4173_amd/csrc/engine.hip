// Kernels and host driver of the multi-group Brandes engine (see engine.h).
//
// Layout. A group's per-source state is row-major [node - lo][64]: lane b of a node's
// row belongs to source src[b]. Distances are uint32 (INF = all ones, not settled),
// path counts uint64 with overflow checks, dependencies double.
//
// Distance-synchronous search. A group at step D settles exactly the (node, source)
// pairs at distance D. Settled nodes offer D + len to their neighbours: the offered
// lanes are or-ed into the neighbour's ring slot (D + len) mod ring_len and its pending
// distance nd is lowered. Since every arc is at least 1 long, every lane offered D
// and still open when step D comes has final distance D.
//
// One engine iteration = select -> settle -> push -> backward -> centrality -> sched:
//   select  (thread per node) forward groups: the nodes with nd = D take their ring
//           slot D as the lanes to settle, record them, and move nd to the next
//           offered distance; backward groups replay one recorded step; centrality
//           groups list their table rows. Output: node items (group, node, lane mask).
//   settle  (one lane per settling (node, source) pair; a wave expands up to 16 node
//           items into 64 pairs) pulls sigma from the tight parents (eq. parentsall /
//           eq. multiparents; restricted to non-frontier parents for Dijkstra_SK, eq.
//           frontierparents) and marks each tight parent arc for the backward sweep.
//   push    (wave per node item, lanes over its arcs) makes the offers.
//   backward(one lane per pair) delta(s|v) = sigma(s,v) * sum over tight children x of
//           mult(v,x) * coef(s,x), coef(s,v) = (I[v in S] + delta(s|v)) / sigma(s,v)
//           (eq. brandes / eq. multibrandes).
//   centrality (wave per interior row, lanes = sources) eq. localcentrality.
//   sched   (thread per group) records the step and moves the group on.
// After the last iteration the per-lane dependencies are summed per node (sources'
// own lanes are never written, so they add nothing).
#include "engine.h"

#include <algorithm>

namespace bcpp {

constexpr int WG = 256;  // threads per workgroup
constexpr int WAVES_PER_WG = WG / 64;
constexpr int ITEMS_PER_WAVE = 16;  // node items a wave expands into lanes at once
constexpr int UNR = 8;              // arcs whose loads a lane issues together

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (unsigned long long)__shfl_xor((long long)v, o, 64);
    return v;
}

__device__ __forceinline__ int popc_below(unsigned long long mask, int lane) {
    return __popcll(mask & ((1ull << lane) - 1ull));
}

// index of the k-th (0-based) set bit of m; m has more than k set bits
__device__ __forceinline__ int nth_bit(unsigned long long m, int k) {
    for (int t = 0; t < k; ++t) m &= m - 1ull;
    return __ffsll((long long)m) - 1;
}

// ------------------------------------------------------------------ init -------

// Fill the state of the groups listed in the chunk table (4 positions x 64 lanes per
// pass of a workgroup). A source node starts with its lane offered distance 0 and one
// path, so the group's first step settles exactly the sources.
__global__ void __launch_bounds__(WG) k_init(const GroupDesc* __restrict__ desc,
                                             const int32_t* __restrict__ chunk_g,
                                             const int32_t* __restrict__ chunk_off,
                                             int64_t nchunks) {
    const int64_t c = blockIdx.x;
    if (c >= nchunks) return;
    const int g = chunk_g[c];
    const GroupDesc& G = desc[g];
    const int64_t range = (int64_t)G.hi - G.lo;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int32_t mysrc = G.src[lane];
    const int64_t base = chunk_off[c];
    for (int p = wv; p < WG; p += WAVES_PER_WG) {
        const int64_t i = base + p;
        if (i < range) {
            const int32_t v = G.lo + (int32_t)i;
            const bool is_src = (mysrc == v);
            G.dist[i * 64 + lane] = is_src ? 0u : INF32;
            G.sigma[i * 64 + lane] = is_src ? 1ull : 0ull;
            if (G.coef) G.coef[i * 64 + lane] = 0.0;
            if (G.delta) G.delta[i * 64 + lane] = 0.0;
            const unsigned long long any = __ballot(is_src);
            for (int r = lane; r < G.ring_len; r += 64) G.ring[i * G.ring_len + r] = r == 0 ? any : 0ull;
            if (lane == 0) {
                G.nd[i] = any ? 0u : INF32;
                G.done[i] = 0ull;
                if (G.cacc) G.cacc[i] = 0.0;
            }
        }
        if ((G.flags & GF_CENT) && i < G.tn && lane == 0) G.cint[i] = 0.0;
    }
    // tight-parent masks: the chunk's share of the group's arcs
    if (G.tmask && base < range) {
        const int64_t chunks = (range + WG - 1) / WG;
        const int64_t k = base / WG;
        const int64_t a0 = G.arcs * k / chunks, a1 = G.arcs * (k + 1) / chunks;
        for (int64_t e = a0 + threadIdx.x; e < a1; e += WG) G.tmask[e] = 0ull;
    }
}

// Copy staged group descriptors into their slots and reset the slots' dynamic state.
__global__ void k_scatter_groups(const GroupDesc* __restrict__ stage, const int32_t* __restrict__ slots,
                                 int32_t n, GroupDesc* __restrict__ desc, GroupDyn* __restrict__ dyn) {
    const int j = blockIdx.x;
    if (j >= n) return;
    const int32_t s = slots[j];
    const uint32_t* src = (const uint32_t*)(stage + j);
    uint32_t* dst = (uint32_t*)(desc + s);
    for (int k = threadIdx.x; k < (int)(sizeof(GroupDesc) / 4); k += blockDim.x) dst[k] = src[k];
    if (threadIdx.x == 0) {
        GroupDyn d;
        d.D = 0;
        d.phase = PH_FWD;
        d.nrec = 0;
        d.rec_i = 0;
        d.hist_len = 0;
        d.rec_start = 0;
        d.nextmin = INF32;
        d.err = 0;
        dyn[s] = d;
    }
}

// ---------------------------------------------------------------- select -------

// Append node items for the lanes with sel set to list `list` (wave-level compaction).
__device__ __forceinline__ void emit_items(NodeItem* __restrict__ wl, int64_t wl_cap,
                                           uint32_t* __restrict__ ctr, int list, bool sel,
                                           NodeItem item) {
    const int lane = threadIdx.x & 63;
    const unsigned long long mask = __ballot(sel);
    if (mask == 0) return;
    uint32_t wbase = 0;
    if (lane == 0) wbase = atomicAdd(&ctr[list], (uint32_t)__popcll(mask));
    wbase = (uint32_t)__shfl((int)wbase, 0, 64);
    if (sel) wl[(int64_t)list * wl_cap + (int64_t)wbase + popc_below(mask, lane)] = item;
}

__global__ void __launch_bounds__(WG) k_select(const GroupDesc* __restrict__ desc,
                                               GroupDyn* __restrict__ dyn,
                                               const int32_t* __restrict__ chunk_g,
                                               const int32_t* __restrict__ chunk_off,
                                               int64_t nchunks, NodeItem* __restrict__ wl,
                                               int64_t wl_cap, uint32_t* __restrict__ ctr) {
    const int64_t c = blockIdx.x;
    if (c >= nchunks) return;
    const int g = chunk_g[c];
    const int32_t phase = dyn[g].phase;
    if (phase == PH_DONE) return;
    const GroupDesc& G = desc[g];
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)chunk_off[c] + threadIdx.x;
    if (phase == PH_BWD) {
        const int r = dyn[g].rec_i;
        const int64_t off = G.rec_off[r];
        const int32_t cnt = G.rec_cnt[r];
        const bool sel = i < cnt;
        NodeItem it;
        it.g = g;
        it.v = sel ? G.hist[off + i] : 0;
        it.mask = sel ? G.hmask[off + i] : 0ull;
        emit_items(wl, wl_cap, ctr, 1, sel, it);
        return;
    }
    if (phase == PH_CENT) {
        NodeItem it;
        it.g = g;
        it.v = G.t_lo + (int32_t)i;
        it.mask = 0ull;
        emit_items(wl, wl_cap, ctr, 2, i < G.tn, it);
        return;
    }
    // PH_FWD
    const int64_t range = (int64_t)G.hi - G.lo;
    const uint32_t D = dyn[g].D;
    const uint32_t pend = (i < range) ? G.nd[i] : INF32;
    const bool sel = (pend == D);
    unsigned long long cand = 0ull;
    uint32_t next = INF32;
    if (sel) {
        const int R = G.ring_len;
        uint64_t* ring = G.ring + i * R;
        const int slot = (int)(D % (uint32_t)R);
        const unsigned long long done0 = G.done[i];
        cand = ring[slot] & ~done0;
        ring[slot] = 0ull;
        const unsigned long long done1 = done0 | cand;
        G.done[i] = done1;
        // next offered distance: scan the ring in blocks of 8 slots, loads issued together
        for (int j0 = 1; j0 < R && next == INF32; j0 += 8) {
            unsigned long long w[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int j = j0 + k;
                w[k] = j < R ? ring[(slot + j) % R] : 0ull;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (next == INF32 && (w[k] & ~done1)) next = D + (uint32_t)(j0 + k);
        }
        G.nd[i] = next;
    }
    const uint32_t other = wave_min_u32(sel ? next : pend);
    if (lane == 0 && other != INF32) atomicMin(&dyn[g].nextmin, other);
    const bool emit = sel && cand != 0ull;
    const unsigned long long mask = __ballot(emit);
    if (mask == 0) return;
    const int cnt = __popcll(mask);
    const int rank = popc_below(mask, lane);
    uint32_t wbase = 0;
    unsigned long long hbase = 0;
    if (lane == 0) {
        wbase = atomicAdd(&ctr[0], (uint32_t)cnt);
        if (G.flags & GF_BACKWARD)
            hbase = atomicAdd((unsigned long long*)&dyn[g].hist_len, (unsigned long long)cnt);
    }
    wbase = (uint32_t)__shfl((int)wbase, 0, 64);
    hbase = (unsigned long long)__shfl((long long)hbase, 0, 64);
    if (emit) {
        NodeItem it;
        it.g = g;
        it.v = G.lo + (int32_t)i;
        it.mask = cand;
        wl[(int64_t)wbase + rank] = it;
        if (G.flags & GF_BACKWARD) {
            if ((int64_t)(hbase + rank) < G.hist_cap) {
                G.hist[hbase + rank] = it.v;
                G.hmask[hbase + rank] = cand;
            } else {
                atomicOr(&dyn[g].err, ERR_HIST);
            }
        }
    }
}

// -------------------------------------------------------- pair expansion -------

// A wave takes ITEMS_PER_WAVE consecutive node items and spreads their (node, lane)
// pairs over its 64 lanes, 64 pairs per round; body(pair) runs once per lane and
// round (pair.valid false on lanes past the last pair). All lanes stay converged.
struct PairCursor {
    int32_t g, v, b;
    bool valid;
};

template <class Body>
__device__ __forceinline__ void for_pairs(const NodeItem* __restrict__ list, uint32_t count,
                                          Body&& body) {
    const int lane = threadIdx.x & 63;
    const int64_t W = (int64_t)gridDim.x * WAVES_PER_WG;
    for (int64_t chunk = (int64_t)blockIdx.x * WAVES_PER_WG + (threadIdx.x >> 6);
         chunk * ITEMS_PER_WAVE < (int64_t)count; chunk += W) {
        const int64_t idx = chunk * ITEMS_PER_WAVE + lane;
        const bool have = lane < ITEMS_PER_WAVE && idx < (int64_t)count;
        int32_t ig = 0, iv = 0;
        unsigned long long im = 0ull;
        if (have) {
            const NodeItem it = list[idx];
            ig = it.g;
            iv = it.v;
            im = it.mask;
        }
        const int pc = __popcll(im);
        int incl = pc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        const int total = __shfl(incl, 63, 64);
        const int excl = incl - pc;
        const int lo32 = (int)(uint32_t)im, hi32 = (int)(uint32_t)(im >> 32);
        for (int r = 0; r < total; r += 64) {
            const int p = r + lane;
            int j = 0;
#pragma unroll
            for (int k = 0; k < ITEMS_PER_WAVE; ++k) j += (__shfl(incl, k, 64) <= p) ? 1 : 0;
            const int jj = min(j, ITEMS_PER_WAVE - 1);
            PairCursor P;
            P.g = __shfl(ig, jj, 64);
            P.v = __shfl(iv, jj, 64);
            const unsigned long long m =
                ((unsigned long long)(uint32_t)__shfl(hi32, jj, 64) << 32) |
                (unsigned long long)(uint32_t)__shfl(lo32, jj, 64);
            const int ex = __shfl(excl, jj, 64);
            P.valid = p < total;
            P.b = P.valid ? nth_bit(m, p - ex) : 0;
            body(P);
        }
    }
}

// ---------------------------------------------------------------- settle -------

__global__ void __launch_bounds__(WG) k_settle(const GroupDesc* __restrict__ desc,
                                               GroupDyn* __restrict__ dyn,
                                               const NodeItem* __restrict__ wl,
                                               const uint32_t* __restrict__ ctr,
                                               unsigned long long* __restrict__ prof) {
    const uint32_t count = ctr[0];
    unsigned long long bytes = 0;
    for_pairs(wl, count, [&](const PairCursor& P) {
        if (!P.valid) return;
        const GroupDesc& G = desc[P.g];
        const int32_t b = P.b;
        const int32_t v = P.v;
        if (G.src[b] == v) return;  // a source's own lane: distance 0, one path (preset)
        const uint32_t D = dyn[P.g].D;
        const int64_t row = (int64_t)(v - G.lo);
        const bool restrict_parents = (G.flags & GF_RESTRICT) != 0;
        const int32_t mysrc = G.src[b];
        const int64_t e0 = G.g.row_ptr[v], e1 = G.g.row_ptr[v + 1];
        uint64_t sum = 0;
        bool ovf = false;
        int tight = 0;
        for (int64_t e = e0; e < e1; e += UNR) {
            int32_t u[UNR];
            uint32_t L[UNR], du[UNR];
#pragma unroll
            for (int k = 0; k < UNR; ++k) {
                const bool in = e + k < e1;
                u[k] = in ? G.g.col[e + k] : G.lo;
                L[k] = in ? (G.g.len ? G.g.len[e + k] : 1u) : INF32;
            }
#pragma unroll
            for (int k = 0; k < UNR; ++k)
                du[k] = (L[k] <= D) ? G.dist[(int64_t)(u[k] - G.lo) * 64 + b] : INF32;
#pragma unroll
            for (int k = 0; k < UNR; ++k) {
                if (du[k] == INF32 || du[k] + L[k] != D) continue;
                ++tight;
                const bool ok = !restrict_parents || u[k] == mysrc || !G.g.nflag ||
                                !(G.g.nflag[u[k]] & NF_BLOCKED);
                if (ok) {
                    uint64_t x = G.sigma[(int64_t)(u[k] - G.lo) * 64 + b];
                    if (G.g.mult && x) {
                        const uint64_t m = G.g.mult[e + k];
                        if (__umul64hi(x, m) != 0) ovf = true;
                        x *= m;
                    }
                    const uint64_t r = sum + x;
                    if (r < sum) ovf = true;
                    sum = r;
                }
                if (G.tmask) {
                    const int64_t t = G.g.twin[e + k] - G.arc_lo;
                    if (t >= 0 && t < G.arcs)
                        atomicOr((unsigned long long*)&G.tmask[t], 1ull << b);
                    else
                        atomicOr(&dyn[P.g].err, ERR_TWIN);
                }
            }
        }
        G.dist[row * 64 + b] = D;
        G.sigma[row * 64 + b] = sum;
        if (ovf) atomicOr(&dyn[P.g].err, ERR_OVERFLOW);
        if (prof) {
            // algorithmic bytes: one distance per arc, a count per tight parent, the
            // distance and count written
            const unsigned long long deg = (unsigned long long)(e1 - e0);
            bytes += 4ull * deg + 8ull * (unsigned)tight + 12ull;
        }
    });
    if (prof) {
        bytes = wave_sum_u64(bytes);
        if ((threadIdx.x & 63) == 0 && bytes) atomicAdd(&prof[BC_K_SETTLE], bytes);
    }
}

// ------------------------------------------------------------------ push -------

// A node whose lanes settled at D offers D + len to each neighbour: the lanes still
// open there are or-ed into the neighbour's ring slot for that distance and its
// pending distance is lowered to it. A wave takes ITEMS_PER_WAVE node items and
// spreads all their arcs over its lanes, 64 arcs per round.
__global__ void __launch_bounds__(WG) k_push(const GroupDesc* __restrict__ desc,
                                             GroupDyn* __restrict__ dyn,
                                             const NodeItem* __restrict__ wl,
                                             const uint32_t* __restrict__ ctr,
                                             unsigned long long* __restrict__ prof) {
    const int lane = threadIdx.x & 63;
    const int64_t W = (int64_t)gridDim.x * WAVES_PER_WG;
    const uint32_t count = ctr[0];
    unsigned long long bytes = 0;
    for (int64_t chunk = (int64_t)blockIdx.x * WAVES_PER_WG + (threadIdx.x >> 6);
         chunk * ITEMS_PER_WAVE < (int64_t)count; chunk += W) {
        const int64_t idx = chunk * ITEMS_PER_WAVE + lane;
        const bool have = lane < ITEMS_PER_WAVE && idx < (int64_t)count;
        int32_t ig = 0;
        unsigned long long im = 0ull;
        int64_t ie0 = 0;
        int deg = 0;
        if (have) {
            const NodeItem it = wl[idx];
            ig = it.g;
            im = it.mask;
            const GroupDesc& G = desc[ig];
            ie0 = G.g.row_ptr[it.v];
            deg = (int)(G.g.row_ptr[it.v + 1] - ie0);
        }
        int incl = deg;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        const int total = __shfl(incl, 63, 64);
        const int excl = incl - deg;
        const int lo32 = (int)(uint32_t)im, hi32 = (int)(uint32_t)(im >> 32);
        const int e0lo = (int)(uint32_t)ie0, e0hi = (int)(uint32_t)((uint64_t)ie0 >> 32);
        for (int r = 0; r < total; r += 64) {
            const int p = r + lane;
            int j = 0;
#pragma unroll
            for (int k = 0; k < ITEMS_PER_WAVE; ++k) j += (__shfl(incl, k, 64) <= p) ? 1 : 0;
            const int jj = min(j, ITEMS_PER_WAVE - 1);
            const int g = __shfl(ig, jj, 64);
            const unsigned long long amask =
                ((unsigned long long)(uint32_t)__shfl(hi32, jj, 64) << 32) |
                (unsigned long long)(uint32_t)__shfl(lo32, jj, 64);
            const int64_t e0 = (int64_t)(((uint64_t)(uint32_t)__shfl(e0hi, jj, 64) << 32) |
                                         (uint64_t)(uint32_t)__shfl(e0lo, jj, 64));
            const int ex = __shfl(excl, jj, 64);
            if (p >= total) continue;
            const GroupDesc& G = desc[g];
            const uint32_t D = dyn[g].D;
            const int64_t e = e0 + (p - ex);
            const int64_t ur = (int64_t)(G.g.col[e] - G.lo);
            const uint32_t nv = D + (G.g.len ? G.g.len[e] : 1u);
            const int R = G.ring_len;
            unsigned long long* slot = (unsigned long long*)&G.ring[ur * R + nv % (uint32_t)R];
            // the three reads do not depend on each other: issue them together
            const unsigned long long dn = G.done[ur];
            const unsigned long long cur = *slot;
            const uint32_t ndu = G.nd[ur];
            const unsigned long long open = amask & ~dn;
            if (open) {
                if (open & ~cur) atomicOr(slot, open);
                if (ndu > nv) {
                    if (G.flags & GF_UNIT)
                        G.nd[ur] = nv;  // every writer of this step stores D + 1
                    else
                        atomicMin(&G.nd[ur], nv);
                    atomicMin(&dyn[g].nextmin, nv);
                }
            }
            if (prof) bytes += 4ull + (G.g.len ? 4ull : 0ull) + 8ull + 8ull;
        }
    }
    if (prof) {
        bytes = wave_sum_u64(bytes);
        if (lane == 0 && bytes) atomicAdd(&prof[BC_K_PUSH], bytes);
    }
}

// -------------------------------------------------------------- backward -------

__global__ void __launch_bounds__(WG) k_backward(const GroupDesc* __restrict__ desc,
                                                 GroupDyn* __restrict__ dyn,
                                                 const NodeItem* __restrict__ wl,
                                                 int64_t wl_cap,
                                                 const uint32_t* __restrict__ ctr,
                                                 unsigned long long* __restrict__ prof) {
    (void)dyn;
    const uint32_t count = ctr[1];
    unsigned long long bytes = 0;
    for_pairs(wl + wl_cap, count, [&](const PairCursor& P) {
        if (!P.valid) return;
        const GroupDesc& G = desc[P.g];
        const int32_t b = P.b;
        const int32_t v = P.v;
        if (G.src[b] == v) return;
        const int64_t row = (int64_t)(v - G.lo);
        const int64_t e0 = G.g.row_ptr[v], e1 = G.g.row_ptr[v + 1];
        double acc = 0.0;
        int kids = 0;
        for (int64_t e = e0; e < e1; e += UNR) {
            bool tk[UNR];
            int32_t u[UNR];
#pragma unroll
            for (int k = 0; k < UNR; ++k) {
                const bool in = e + k < e1;
                tk[k] = in && ((G.tmask[e + k - G.arc_lo] >> b) & 1ull);
                u[k] = in ? G.g.col[e + k] : G.lo;
            }
            double c[UNR];
#pragma unroll
            for (int k = 0; k < UNR; ++k) c[k] = tk[k] ? G.coef[(int64_t)(u[k] - G.lo) * 64 + b] : 0.0;
#pragma unroll
            for (int k = 0; k < UNR; ++k) {
                if (!tk[k]) continue;
                acc += G.g.mult ? (double)G.g.mult[e + k] * c[k] : c[k];
                ++kids;
            }
        }
        const double sg = (double)G.sigma[row * 64 + b];
        const double dl = sg * acc;
        const double ind = (G.g.nflag && (G.g.nflag[v] & NF_TARGET)) ? 1.0 : 0.0;
        G.coef[row * 64 + b] = (ind + dl) / sg;
        G.delta[row * 64 + b] = dl;
        if (prof) {
            const unsigned long long deg = (unsigned long long)(e1 - e0);
            bytes += 8ull * deg + 8ull * (unsigned)kids + 8ull + 16ull;
        }
    });
    if (prof) {
        bytes = wave_sum_u64(bytes);
        if ((threadIdx.x & 63) == 0 && bytes) atomicAdd(&prof[BC_K_BACKWARD], bytes);
    }
}

// ------------------------------------------------------------ centrality -------

// Interior node i of a part (Sec. 5, Step 3): with the tables d(f,v), sigma(f,v) over
// the part's frontier f and the group's skeleton state d(s,f), sigma(s,f), coef(s,f):
//   d(s,v)     = min_f d(s,f) + d(f,v)
//   sigma(s,v) = sum over f with d(s,f) + d(f,v) = d(s,v) of sigma(s,f) sigma(f,v)
//   delta(s|v) = sigma(s,v) * sum over f with d(s,v) + d(v,f) = d(s,f) of
//                sigma(v,f) * coef(s,f)                       (eq. localcentrality)
__global__ void __launch_bounds__(WG) k_centrality(const GroupDesc* __restrict__ desc,
                                                   GroupDyn* __restrict__ dyn,
                                                   const NodeItem* __restrict__ wl,
                                                   int64_t wl_cap,
                                                   const uint32_t* __restrict__ ctr,
                                                   unsigned long long* __restrict__ prof) {
    const int lane = threadIdx.x & 63;
    const int64_t W = (int64_t)gridDim.x * WAVES_PER_WG;
    const uint32_t count = ctr[2];
    const NodeItem* list = wl + 2 * wl_cap;
    unsigned long long bytes = 0;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_WG + (threadIdx.x >> 6); it < count;
         it += W) {
        const NodeItem item = list[it];
        const int g = item.g;
        const int32_t i = item.v;
        const GroupDesc& G = desc[g];
        const int64_t e0 = G.trow[i], e1 = G.trow[i + 1];
        uint32_t dv = INF32;
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t fr = (int64_t)(G.tcol[e] - G.lo);
            const uint32_t tf = G.dist[fr * 64 + lane];
            if (tf != INF32) dv = min(dv, tf + G.tlen[e]);
        }
        double delta = 0.0;
        bool ovf = false;
        if (dv != INF32) {
            uint64_t sv = 0;
            double acc = 0.0;
            for (int64_t e = e0; e < e1; ++e) {
                const int64_t fr = (int64_t)(G.tcol[e] - G.lo);
                const uint32_t tf = G.dist[fr * 64 + lane];
                if (tf == INF32) continue;
                const uint32_t L = G.tlen[e];
                if (tf + L == dv) {
                    const uint64_t a = G.sigma[fr * 64 + lane];
                    const uint64_t bb = G.tsig[e];
                    if (__umul64hi(a, bb) != 0) ovf = true;
                    const uint64_t p = a * bb;
                    const uint64_t r = sv + p;
                    if (r < sv) ovf = true;
                    sv = r;
                } else if (tf == dv + L) {
                    acc += (double)G.tsig[e] * G.coef[fr * 64 + lane];
                }
            }
            delta = (double)sv * acc;
        }
        if (__ballot(ovf) && lane == 0) atomicOr(&dyn[g].err, ERR_OVERFLOW);
        const double tot = wave_sum_f64(delta);
        if (lane == 0) G.cint[i - G.t_lo] += tot;
        if (prof) {
            // per (source, entry): d(s,f) twice, sigma(s,f) or coef(s,f) once; per
            // entry the table row once
            const unsigned long long ent = (unsigned long long)(e1 - e0);
            bytes += 64ull * ent * (4ull + 4ull + 8ull) + ent * (4ull + 4ull + 8ull) + 16ull;
        }
    }
    if (prof && lane == 0 && bytes) atomicAdd(&prof[BC_K_CENTRALITY], bytes);
}

// ----------------------------------------------------------------- sched -------

__global__ void k_sched(const GroupDesc* __restrict__ desc, GroupDyn* __restrict__ dyn,
                        int32_t nslots, uint32_t* __restrict__ ctr) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) {
        ctr[0] = 0;
        ctr[1] = 0;
        ctr[2] = 0;
    }
    if (g >= nslots) return;
    GroupDyn d = dyn[g];
    if (d.phase == PH_DONE) return;
    const GroupDesc& G = desc[g];
    int32_t phase = d.phase;
    if (phase == PH_FWD) {
        if (G.flags & GF_BACKWARD) {
            const int64_t cnt = d.hist_len - d.rec_start;
            if (cnt > 0) {
                if (d.nrec < G.rec_cap) {
                    G.rec_d[d.nrec] = d.D;
                    G.rec_off[d.nrec] = d.rec_start;
                    G.rec_cnt[d.nrec] = (int32_t)cnt;
                    d.nrec++;
                } else {
                    d.err |= ERR_REC;
                }
            }
            d.rec_start = d.hist_len;
        }
        const uint32_t nm = d.nextmin;
        d.nextmin = INF32;
        if (nm == INF32 || d.err) {
            if ((G.flags & GF_BACKWARD) && d.nrec > 1 && !d.err) {
                phase = PH_BWD;
                d.rec_i = d.nrec - 1;
                d.D = G.rec_d[d.rec_i];
            } else {
                phase = PH_DONE;
            }
        } else {
            d.D = nm;
        }
    } else if (phase == PH_BWD) {
        d.rec_i -= 1;
        if (d.rec_i < 1) {  // record 0 holds only the sources (distance 0)
            phase = (G.flags & GF_CENT) ? PH_CENT : PH_DONE;
        } else {
            d.D = G.rec_d[d.rec_i];
        }
    } else {  // PH_CENT
        phase = PH_DONE;
    }
    d.phase = phase;
    dyn[g] = d;
    if (phase == PH_DONE) atomicSub(&ctr[3], 1u);
}

// ------------------------------------------------------------- lane sum -------

// Each node's score share of a backward group: the sum over its lanes of delta(s|v),
// in a fixed order (a wave reduction), written once.
__global__ void __launch_bounds__(WG) k_lane_sum(const GroupDesc* __restrict__ desc,
                                                 const int32_t* __restrict__ chunk_g,
                                                 const int32_t* __restrict__ chunk_off,
                                                 int64_t nchunks) {
    const int64_t c = blockIdx.x;
    if (c >= nchunks) return;
    const GroupDesc& G = desc[chunk_g[c]];
    if (!(G.flags & GF_BACKWARD)) return;
    const int64_t range = (int64_t)G.hi - G.lo;
    const int lane = threadIdx.x & 63;
    for (int p = threadIdx.x >> 6; p < WG; p += WAVES_PER_WG) {
        const int64_t i = chunk_off[c] + p;
        if (i >= range) break;
        const double s = wave_sum_f64(G.delta[i * 64 + lane]);
        if (lane == 0) G.cacc[i] = s;
    }
}

// ---------------------------------------------------------------- reduce -------

__global__ void k_reduce(const double* const* __restrict__ cacc,
                         const double* const* __restrict__ cint, int32_t n,
                         const int32_t* __restrict__ g0, const int32_t* __restrict__ g1,
                         const int32_t* __restrict__ idx, const uint8_t* __restrict__ which,
                         int32_t ga, int32_t gb, double scale, int accumulate,
                         double* __restrict__ out) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t i = idx ? idx[v] : v;
    double s = 0.0;
    if (i >= 0) {
        const double* const* parts = (which && which[v]) ? cint : cacc;
        const int32_t a = g0 ? g0[v] : ga;
        const int32_t b = g1 ? g1[v] : gb;
        // eight groups' loads in flight at a time, added in group order (the same sum,
        // bit for bit, as one group after another)
        int32_t g = a;
        for (; g + 8 <= b; g += 8) {
            double x[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = parts[g + j][i];
#pragma unroll
            for (int j = 0; j < 8; ++j) s += x[j];
        }
        for (; g < b; ++g) s += parts[g][i];
    }
    s *= scale;
    out[v] = accumulate ? out[v] + s : s;
}

// ==================================================================== host ======

size_t group_bytes(const GroupDesc& G, int64_t max_steps) {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int64_t range = (int64_t)G.hi - G.lo;
    size_t b = 0;
    b += al(range * 64 * 4);                   // dist
    b += al(range * 64 * 8);                   // sigma
    b += al(range * 4);                        // nd
    b += al(range * 8);                        // done
    b += al(range * (int64_t)G.ring_len * 8);  // offer ring
    if (G.flags & GF_BACKWARD) {
        b += al(range * 64 * 8);                     // coef
        b += al(range * 64 * 8);                     // delta
        b += al(range * 8);                          // cacc
        b += al(std::max<int64_t>(G.arcs, 1) * 8);  // tight-parent masks
        const int64_t hc = range * (int64_t)std::max(G.nsrc, 1);
        b += al(hc * 4) + al(hc * 8);                // history: node, lanes
        b += al(max_steps * 4) + al(max_steps * 8) + al(max_steps * 4);
    }
    if (G.flags & GF_CENT) b += al((size_t)std::max(G.tn, 1) * 8);
    return b;
}

bool group_alloc(Arena& a, GroupDesc& G, int64_t max_steps) {
    const int64_t range = (int64_t)G.hi - G.lo;
    if (G.ring_len < 2) return false;
    G.dist = a.take<uint32_t>(range * 64);
    G.sigma = a.take<uint64_t>(range * 64);
    G.nd = a.take<uint32_t>(range);
    G.done = a.take<uint64_t>(range);
    G.ring = a.take<uint64_t>(range * (int64_t)G.ring_len);
    if (!G.dist || !G.sigma || !G.nd || !G.done || !G.ring) return false;
    if (G.flags & GF_BACKWARD) {
        if (!G.g.twin) return false;
        G.coef = a.take<double>(range * 64);
        G.delta = a.take<double>(range * 64);
        G.cacc = a.take<double>(range);
        G.tmask = a.take<uint64_t>(std::max<int64_t>(G.arcs, 1));
        G.hist_cap = range * (int64_t)std::max(G.nsrc, 1);
        G.hist = a.take<int32_t>(G.hist_cap);
        G.hmask = a.take<uint64_t>(G.hist_cap);
        G.rec_cap = (int32_t)std::min<int64_t>(max_steps, INT32_MAX);
        G.rec_d = a.take<uint32_t>(G.rec_cap);
        G.rec_off = a.take<int64_t>(G.rec_cap);
        G.rec_cnt = a.take<int32_t>(G.rec_cap);
        if (!G.coef || !G.delta || !G.cacc || !G.tmask || !G.hist || !G.hmask || !G.rec_d ||
            !G.rec_off || !G.rec_cnt)
            return false;
    }
    if (G.flags & GF_CENT) {
        G.cint = a.take<double>(std::max(G.tn, 1));
        if (!G.cint) return false;
    }
    return true;
}

size_t engine_bytes(int32_t slots, int64_t positions) {
    const int64_t chunks = (positions + WG - 1) / WG + slots;
    return (size_t)slots * (2 * sizeof(GroupDesc) + sizeof(GroupDyn) + 1024) + (size_t)chunks * 8 +
           (size_t)chunks * WG * 3 * sizeof(NodeItem) + 8192;
}

int Engine::setup(Arena& a, hipStream_t s, int32_t slots, int64_t positions) {
    stream = s;
    cap = slots;
    chunk_cap = (positions + WG - 1) / WG + slots;
    wl_cap = chunk_cap * WG;
    d_desc = a.take<GroupDesc>(slots);
    d_dyn = a.take<GroupDyn>(slots);
    d_chunk_g = a.take<int32_t>(chunk_cap);
    d_chunk_off = a.take<int32_t>(chunk_cap);
    d_wl = a.take<NodeItem>(3 * wl_cap);
    d_ctr = a.take<uint32_t>(8);
    d_stage = a.take<GroupDesc>(slots);
    d_stage_slot = a.take<int32_t>(slots);
    if (!d_desc || !d_dyn || !d_chunk_g || !d_chunk_off || !d_wl || !d_ctr || !d_stage || !d_stage_slot)
        return fail(BC_E_NOMEM, "engine: workspace too small");
    if (!h_ctr) BC_HIP(hipHostMalloc((void**)&h_ctr, 8 * sizeof(uint32_t)));
    BC_HIP(hipMemsetAsync(d_ctr, 0, 8 * sizeof(uint32_t), stream));
    int dev = 0, cus = 0;
    BC_HIP(hipGetDevice(&dev));
    BC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    blocks = std::max(1, cus) * 8;
    profile_bytes = profiler().on;
    return BC_OK;
}

int Engine::set_chunks(const std::vector<GroupDesc>& host_desc, const std::vector<int32_t>& live) {
    std::vector<int32_t> cg, co;
    for (int32_t g : live) {
        const GroupDesc& G = host_desc[g];
        int64_t pos = std::max<int64_t>((int64_t)G.hi - G.lo, (G.flags & GF_CENT) ? G.tn : 0);
        for (int64_t off = 0; off < pos; off += WG) {
            cg.push_back(g);
            co.push_back((int32_t)off);
        }
    }
    if ((int64_t)cg.size() > chunk_cap) return fail(BC_E_NOMEM, "engine: too many scan chunks");
    nchunks = (int64_t)cg.size();
    if (nchunks) {
        BC_HIP(hipMemcpyAsync(d_chunk_g, cg.data(), cg.size() * 4, hipMemcpyHostToDevice, stream));
        BC_HIP(hipMemcpyAsync(d_chunk_off, co.data(), co.size() * 4, hipMemcpyHostToDevice, stream));
        // keep the host vectors alive until the copies are done
        BC_HIP(hipStreamSynchronize(stream));
    }
    return BC_OK;
}

int Engine::install(const GroupDesc* groups, int32_t first, int32_t n) {
    if (n <= 0) return BC_OK;
    std::vector<GroupDyn> dy(n);
    for (int32_t j = 0; j < n; ++j) {
        GroupDyn& d = dy[j];
        d.D = 0;
        d.phase = PH_FWD;
        d.nrec = 0;
        d.rec_i = 0;
        d.hist_len = 0;
        d.rec_start = 0;
        d.nextmin = INF32;
        d.err = 0;
    }
    BC_HIP(hipMemcpyAsync(d_desc + first, groups, sizeof(GroupDesc) * n, hipMemcpyHostToDevice, stream));
    BC_HIP(hipMemcpyAsync(d_dyn + first, dy.data(), sizeof(GroupDyn) * n, hipMemcpyHostToDevice, stream));
    // chunk table of the new groups only, for the state fill
    std::vector<int32_t> cg, co;
    for (int32_t j = 0; j < n; ++j) {
        const GroupDesc& G = groups[j];
        int64_t pos = std::max<int64_t>((int64_t)G.hi - G.lo, (G.flags & GF_CENT) ? G.tn : 0);
        for (int64_t off = 0; off < pos; off += WG) {
            cg.push_back(first + j);
            co.push_back((int32_t)off);
        }
    }
    if ((int64_t)cg.size() > chunk_cap) return fail(BC_E_NOMEM, "engine: too many init chunks");
    if (!cg.empty()) {
        BC_HIP(hipMemcpyAsync(d_chunk_g, cg.data(), cg.size() * 4, hipMemcpyHostToDevice, stream));
        BC_HIP(hipMemcpyAsync(d_chunk_off, co.data(), co.size() * 4, hipMemcpyHostToDevice, stream));
        {
            KTimer kt(BC_K_OTHER, stream);
            hipLaunchKernelGGL(k_init, dim3((unsigned)cg.size()), dim3(WG), 0, stream, d_desc,
                               d_chunk_g, d_chunk_off, (int64_t)cg.size());
        }
        BC_HIP(hipGetLastError());
        BC_HIP(hipStreamSynchronize(stream));
    }
    // active += n (host-side read-modify-write: the engine is idle here)
    BC_HIP(hipMemcpyAsync(h_ctr, d_ctr, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    BC_HIP(hipStreamSynchronize(stream));
    h_ctr[3] += (uint32_t)n;
    BC_HIP(hipMemcpyAsync(d_ctr + 3, h_ctr + 3, sizeof(uint32_t), hipMemcpyHostToDevice, stream));
    BC_HIP(hipStreamSynchronize(stream));
    return BC_OK;
}

int Engine::install_at(const GroupDesc* groups, const int32_t* slots, int32_t n,
                       const std::vector<GroupDesc>& host_desc, const std::vector<int32_t>& live) {
    if (n > 0) {
        if (n > cap) return fail(BC_E_NOMEM, "engine: too many groups to install");
        BC_HIP(hipMemcpyAsync(d_stage, groups, sizeof(GroupDesc) * n, hipMemcpyHostToDevice, stream));
        BC_HIP(hipMemcpyAsync(d_stage_slot, slots, sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL(k_scatter_groups, dim3(n), dim3(128), 0, stream, d_stage, d_stage_slot, n,
                           d_desc, d_dyn);
        BC_HIP(hipGetLastError());
        std::vector<int32_t> cg, co;
        for (int32_t j = 0; j < n; ++j) {
            const GroupDesc& G = groups[j];
            int64_t pos = std::max<int64_t>((int64_t)G.hi - G.lo, (G.flags & GF_CENT) ? G.tn : 0);
            for (int64_t off = 0; off < pos; off += WG) {
                cg.push_back(slots[j]);
                co.push_back((int32_t)off);
            }
        }
        if ((int64_t)cg.size() > chunk_cap) return fail(BC_E_NOMEM, "engine: too many init chunks");
        if (!cg.empty()) {
            BC_HIP(hipMemcpyAsync(d_chunk_g, cg.data(), cg.size() * 4, hipMemcpyHostToDevice, stream));
            BC_HIP(hipMemcpyAsync(d_chunk_off, co.data(), co.size() * 4, hipMemcpyHostToDevice, stream));
            KTimer kt(BC_K_OTHER, stream);
            hipLaunchKernelGGL(k_init, dim3((unsigned)cg.size()), dim3(WG), 0, stream, d_desc, d_chunk_g,
                               d_chunk_off, (int64_t)cg.size());
        }
        BC_HIP(hipGetLastError());
        BC_HIP(hipStreamSynchronize(stream));  // the staged host arrays are reused after this
    }
    return set_chunks(host_desc, live);
}

int Engine::iterate(int iters) {
    unsigned long long* prof = profile_bytes ? profiler().d_bytes : nullptr;
    const unsigned sel_blocks = (unsigned)std::max<int64_t>(nchunks, 1);
    for (int k = 0; k < iters; ++k) {
        {
            KTimer kt(BC_K_SELECT, stream);
            hipLaunchKernelGGL(k_select, dim3(sel_blocks), dim3(WG), 0, stream, d_desc, d_dyn,
                               d_chunk_g, d_chunk_off, nchunks, d_wl, wl_cap, d_ctr);
        }
        {
            KTimer kt(BC_K_SETTLE, stream);
            hipLaunchKernelGGL(k_settle, dim3(blocks), dim3(WG), 0, stream, d_desc, d_dyn, d_wl,
                               d_ctr, prof);
        }
        {
            KTimer kt(BC_K_PUSH, stream);
            hipLaunchKernelGGL(k_push, dim3(blocks), dim3(WG), 0, stream, d_desc, d_dyn, d_wl,
                               d_ctr, prof);
        }
        {
            KTimer kt(BC_K_BACKWARD, stream);
            hipLaunchKernelGGL(k_backward, dim3(blocks), dim3(WG), 0, stream, d_desc, d_dyn,
                               d_wl, wl_cap, d_ctr, prof);
        }
        {
            KTimer kt(BC_K_CENTRALITY, stream);
            hipLaunchKernelGGL(k_centrality, dim3(blocks), dim3(WG), 0, stream, d_desc, d_dyn,
                               d_wl, wl_cap, d_ctr, prof);
        }
        {
            KTimer kt(BC_K_SCHED, stream);
            hipLaunchKernelGGL(k_sched, dim3((cap + 255) / 256), dim3(256), 0, stream, d_desc,
                               d_dyn, cap, d_ctr);
        }
    }
    BC_HIP(hipGetLastError());
    return BC_OK;
}

int Engine::finish_scores() {
    if (!nchunks) return BC_OK;
    {
        KTimer kt(BC_K_OTHER, stream);
        hipLaunchKernelGGL(k_lane_sum, dim3((unsigned)nchunks), dim3(WG), 0, stream, d_desc,
                           d_chunk_g, d_chunk_off, nchunks);
    }
    BC_HIP(hipGetLastError());
    return BC_OK;
}

int lane_sum(hipStream_t s, const GroupDesc* d_desc, const int32_t* d_chunk_g,
             const int32_t* d_chunk_off, int64_t nchunks) {
    if (!nchunks) return BC_OK;
    {
        KTimer kt(BC_K_OTHER, s);
        hipLaunchKernelGGL(k_lane_sum, dim3((unsigned)nchunks), dim3(WG), 0, s, d_desc, d_chunk_g,
                           d_chunk_off, nchunks);
    }
    BC_HIP(hipGetLastError());
    return BC_OK;
}

int Engine::run_to_completion(int32_t nslots, std::vector<GroupDyn>* dyn_out) {
    // Every group finishes within 2 * (steps + 1) + 1 iterations; steps per group are
    // bounded by its record capacity, so the loop below always terminates.
    int batch = 4;
    for (int64_t total = 0;; total += batch) {
        BC_TRY(iterate(batch));
        BC_HIP(hipMemcpyAsync(h_ctr + 4, d_ctr + 3, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
        BC_HIP(hipStreamSynchronize(stream));
        if (h_ctr[4] == 0) break;
        if (total > (int64_t)1 << 40) return fail(BC_E_DEVICE, "engine: no progress");
        batch = std::min(batch * 2, 32);
    }
    BC_TRY(finish_scores());
    std::vector<GroupDyn> dy(nslots);
    BC_HIP(hipMemcpyAsync(dy.data(), d_dyn, sizeof(GroupDyn) * nslots, hipMemcpyDeviceToHost, stream));
    BC_HIP(hipStreamSynchronize(stream));
    uint32_t err = 0;
    for (auto& d : dy) err |= d.err;
    if (dyn_out) *dyn_out = dy;
    if (err & ERR_OVERFLOW) return fail(BC_E_OVERFLOW, "a shortest-path count reached 2^64");
    if (err & (ERR_HIST | ERR_REC)) return fail(BC_E_DEVICE, "engine: history capacity exceeded");
    if (err & ERR_TWIN) return fail(BC_E_DEVICE, "engine: graph arc without a reverse arc");
    return BC_OK;
}

int run_groups(Arena& a, hipStream_t s, std::vector<GroupDesc>& groups, int64_t max_steps) {
    if (groups.empty()) return BC_OK;
    for (auto& G : groups)
        if (!group_alloc(a, G, max_steps)) return fail(BC_E_NOMEM, "engine: group state does not fit");
    return run_groups_prealloc(a, s, groups);
}

int run_groups_prealloc(Arena& a, hipStream_t s, std::vector<GroupDesc>& groups) {
    if (groups.empty()) return BC_OK;
    int64_t positions = 0;
    for (auto& G : groups)
        positions += std::max<int64_t>((int64_t)G.hi - G.lo, (G.flags & GF_CENT) ? G.tn : 0);
    Engine E;
    int rc = E.setup(a, s, (int32_t)groups.size(), positions);
    if (rc == BC_OK) rc = E.install(groups.data(), 0, (int32_t)groups.size());
    std::vector<int32_t> live(groups.size());
    for (size_t i = 0; i < live.size(); ++i) live[i] = (int32_t)i;
    if (rc == BC_OK) rc = E.set_chunks(groups, live);
    if (rc == BC_OK) rc = E.run_to_completion((int32_t)groups.size());
    if (E.h_ctr) (void)hipHostFree(E.h_ctr);
    return rc;
}

int reduce_upload(hipStream_t s, Arena& a, const std::vector<GroupDesc>& groups, ReducePtrs* R) {
    const size_t ng = std::max<size_t>(groups.size(), 1);
    std::vector<const double*> pc(ng, nullptr), pi(ng, nullptr);
    for (size_t g = 0; g < groups.size(); ++g) {
        pc[g] = groups[g].cacc;
        pi[g] = groups[g].cint;
    }
    R->pc = a.take<const double*>(ng);
    R->pi = a.take<const double*>(ng);
    R->ngroups = (int32_t)groups.size();
    if (!R->pc || !R->pi) return fail(BC_E_NOMEM, "reduce: workspace too small");
    BC_HIP(hipMemcpyAsync(R->pc, pc.data(), ng * sizeof(void*), hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(R->pi, pi.data(), ng * sizeof(void*), hipMemcpyHostToDevice, s));
    return BC_OK;
}

int reduce_launch(hipStream_t s, const ReducePtrs& R, int32_t n, const int32_t* d_g0, const int32_t* d_g1,
                  const int32_t* d_idx, const uint8_t* d_which, double scale, double* out_dev,
                  bool accumulate) {
    if (n <= 0) return BC_OK;
    {
        KTimer kt(BC_K_OTHER, s);
        hipLaunchKernelGGL(k_reduce, dim3((n + 255) / 256), dim3(256), 0, s, R.pc, R.pi, n, d_g0, d_g1,
                           d_idx, d_which, 0, R.ngroups, scale, accumulate ? 1 : 0, out_dev);
    }
    BC_HIP(hipGetLastError());
    return BC_OK;
}

int reduce_scores(hipStream_t s, Arena& a, const std::vector<GroupDesc>& groups, int32_t n,
                  const int32_t* d_g0, const int32_t* d_g1, const int32_t* d_idx,
                  const uint8_t* d_which, double scale, double* out_dev, bool accumulate) {
    if (n <= 0) return BC_OK;
    ReducePtrs R;
    BC_TRY(reduce_upload(s, a, groups, &R));
    BC_TRY(reduce_launch(s, R, n, d_g0, d_g1, d_idx, d_which, scale, out_dev, accumulate));
    BC_HIP(hipStreamSynchronize(s));
    return BC_OK;
}

}  // namespace bcpp
