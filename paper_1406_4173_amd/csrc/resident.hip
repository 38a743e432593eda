// LDS-resident Brandes: one workgroup per group of sources, the group's sources one
// after another, with the distance and path count of every node of the group's range
// held in LDS (12 bytes per node: up to about 13,000 nodes in gfx950's 160 KB).
//
// For one source s the workgroup runs (Sec. 3 and Sec. 5, Step 2):
//   forward   distance-synchronous steps D = 0, then the next pending distance: every
//             node with tentative distance D is settled, pulls sigma(s,v) from its
//             tight parents (eq. parentsall, or eq. multiparents with multiplicities)
//             and lowers its neighbours' tentative distances with LDS atomics. Arc
//             lengths are at least 1, so a node whose tentative distance equals the
//             current step's D is final, and its parents were settled (and their counts
//             written) in earlier steps, behind a barrier. Each tight parent arc found
//             marks its reverse arc in a bitmap: the arcs to each node's children.
//   interior  (skeleton groups with tables, Sec. 5, Step 3) d(s,v) and sigma(s,v) of
//             every interior row from the frontier state.
//   backward  the same steps in decreasing distance: delta(s|v) = sigma(s,v) * sum over
//             tight children x of m(v,x) * coef(s,x), coef(s,v) = (I[v in S] + delta(s|v))
//             / sigma(s,v) (eq. brandes / eq. multibrandes). coef replaces sigma in LDS.
//             Only the arcs marked in the bitmap are read.
//   interior  delta(s|v) of the interior rows (eq. localcentrality).
// A group's node scores (cacc) and interior scores (cint) are owned by its workgroup
// and accumulated in source order, so results do not depend on what else runs.
// Dijkstra_SK groups (Sec. 4) run the forward sweep only, with path counts restricted
// to non-frontier parents or the source (eq. frontierparents), and write d(f,v) and
// sigma(f,v) of every node of the part to the group's [node][64] output lanes.
//
// The graph's CSR is read from global memory; it is small enough to stay in L2 for the
// graphs this kernel takes, so the only HBM traffic is the first touch of the CSR and
// the per-group score rows.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>

#include "engine.h"
#include "tuned.h"

namespace bcpp {

namespace {

__device__ __forceinline__ uint32_t wmin_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

// Inclusive wave scans with DPP (GFX9 family: row shifts inside 16-lane rows and row
// broadcasts; VALU only, no LDS round trip): shifts by 1, 2, 4 and 8 inside each row,
// then lane 15's value into row 1 and lane 47's into row 3, then lane 31's into rows 2
// and 3. A lane whose source lies outside its row, or whose row is masked off, takes
// the identity.
constexpr int DPP_ROW_SHR = 0x110, DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;

__device__ __forceinline__ int wscan_add(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR | 1, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR | 2, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR | 4, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR | 8, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_BCAST15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_BCAST31, 0xc, 0xf, false);
    return x;
}

// The same for max over values >= -1 (identity -1).
__device__ __forceinline__ int wscan_max(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, DPP_ROW_SHR | 1, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, DPP_ROW_SHR | 2, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, DPP_ROW_SHR | 4, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, DPP_ROW_SHR | 8, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, DPP_BCAST15, 0xa, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, DPP_BCAST31, 0xc, 0xf, false));
    return x;
}

// fp64 value of the lane O places lower in the same 16-lane row (0 where there is none).
template <int O>
__device__ __forceinline__ double dpp_row_shr(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, DPP_ROW_SHR | O, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), DPP_ROW_SHR | O, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
}

// Segmented inclusive sum over the wave: lane l adds the values of lanes seg .. l (its
// segment starts at lane seg <= l; segments are contiguous). Inside each 16-lane row
// by DPP shifts of 1, 2, 4 and 8; then, row by row, a lane whose segment began in an
// earlier row adds the final value of the previous row's last lane. The order of the
// additions depends only on the segments, so the sums are reproducible.
__device__ __forceinline__ double wseg_sum(double c, int seg) {
    const int lane = threadIdx.x & 63;
    const int lim = max(seg, lane & ~15);
    double t;
    t = dpp_row_shr<1>(c);
    if (lane - 1 >= lim) c += t;
    t = dpp_row_shr<2>(c);
    if (lane - 2 >= lim) c += t;
    t = dpp_row_shr<4>(c);
    if (lane - 4 >= lim) c += t;
    t = dpp_row_shr<8>(c);
    if (lane - 8 >= lim) c += t;
#pragma unroll
    for (int rr = 1; rr < 4; ++rr) {
        const double carry = readlane_f64(c, 16 * rr - 1);
        if ((lane >> 4) == rr && seg < 16 * rr) c += carry;
    }
    return c;
}

// The same segmented inclusive scan for the minimum of uint32 values.
__device__ __forceinline__ uint32_t wseg_min_u32(uint32_t c, int seg) {
    const int lane = threadIdx.x & 63;
    const int lim = max(seg, lane & ~15);
    uint32_t t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)c, DPP_ROW_SHR | 1, 0xf, 0xf, false);
    if (lane - 1 >= lim) c = min(c, t);
    t = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)c, DPP_ROW_SHR | 2, 0xf, 0xf, false);
    if (lane - 2 >= lim) c = min(c, t);
    t = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)c, DPP_ROW_SHR | 4, 0xf, 0xf, false);
    if (lane - 4 >= lim) c = min(c, t);
    t = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)c, DPP_ROW_SHR | 8, 0xf, 0xf, false);
    if (lane - 8 >= lim) c = min(c, t);
#pragma unroll
    for (int rr = 1; rr < 4; ++rr) {
        const uint32_t carry = (uint32_t)__builtin_amdgcn_readlane((int)c, 16 * rr - 1);
        if ((lane >> 4) == rr && seg < 16 * rr) c = min(c, carry);
    }
    return c;
}

// uint64 value of the lane O places lower in the same 16-lane row (0 where there is none).
template <int O>
__device__ __forceinline__ uint64_t dpp_row_shr_u64(uint64_t x) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, DPP_ROW_SHR | O, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), DPP_ROW_SHR | O, 0xf, 0xf, false);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// The same segmented inclusive scan for sums of uint64 values; *ovf is set where an
// addition wraps (all terms are counts, so any wrap means the total reaches 2^64).
__device__ __forceinline__ uint64_t wseg_sum_u64(uint64_t c, int seg, bool* ovf) {
    const int lane = threadIdx.x & 63;
    const int lim = max(seg, lane & ~15);
    uint64_t t;
    t = dpp_row_shr_u64<1>(c);
    if (lane - 1 >= lim) { *ovf |= c + t < c; c += t; }
    t = dpp_row_shr_u64<2>(c);
    if (lane - 2 >= lim) { *ovf |= c + t < c; c += t; }
    t = dpp_row_shr_u64<4>(c);
    if (lane - 4 >= lim) { *ovf |= c + t < c; c += t; }
    t = dpp_row_shr_u64<8>(c);
    if (lane - 8 >= lim) { *ovf |= c + t < c; c += t; }
#pragma unroll
    for (int rr = 1; rr < 4; ++rr) {
        const uint64_t carry = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(c >> 32), 16 * rr - 1) << 32) |
                               (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)c, 16 * rr - 1);
        if ((lane >> 4) == rr && seg < 16 * rr) { *ovf |= c + carry < c; c += carry; }
    }
    return c;
}

__device__ __forceinline__ unsigned long long wsum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (unsigned long long)__shfl_xor((long long)v, o, 64);
    return v;
}

// Position (0..31) of the j-th (from 0) set bit of x; x has more than j set bits.
__device__ __forceinline__ int nth_set_bit(uint32_t x, int j) {
    int pos = 0;
#pragma unroll
    for (int h = 16; h > 0; h >>= 1) {
        const int cl = __popc(x & ((1u << h) - 1u));
        if (j >= cl) {
            j -= cl;
            x >>= h;
            pos += h;
        }
    }
    return pos;
}

// Set bits in positions [a, a + n) of a bitmap whose word w is ld(w).
template <class LD>
__device__ __forceinline__ int bits_in(LD&& ld, int a, int n) {
    if (n <= 0) return 0;
    const int w0 = a >> 5, w1 = (a + n - 1) >> 5;
    const uint32_t m0 = ~0u << (a & 31), m1 = ~0u >> (31 - ((a + n - 1) & 31));
    if (w0 == w1) return __popc(ld(w0) & m0 & m1);
    int c = __popc(ld(w0) & m0) + __popc(ld(w1) & m1);
    for (int w = w0 + 1; w < w1; ++w) c += __popc(ld(w));
    return c;
}

// Position of the j-th (from 0) set bit at or after position a; the caller knows that
// many bits are set there.
template <class LD>
__device__ __forceinline__ int select_bit(LD&& ld, int a, int j) {
    int w = a >> 5;
    uint32_t x = ld(w) & (~0u << (a & 31));
    int c = __popc(x);
    while (j >= c) {
        j -= c;
        x = ld(++w);
        c = __popc(x);
    }
    return (w << 5) + nth_set_bit(x, j);
}

// Visit the nodes v of [0, n) for which sel(v) holds. Wave w owns the BLK-node blocks b
// with b % (T / 64) == w and scans 64 of its nodes per pass (64 / BLK blocks), in
// increasing order; it appends the selected ones to its own LDS
// queue wq (128 entries) and hands every full queue of 64, and the last partial one,
// to body(v, valid) with all lanes converged. A step that settles few nodes thus costs
// one round of neighbour loads per wave instead of one per scan pass. sel is
// evaluated for SCAN passes (loads in flight together) before their nodes are handed on, so it must not depend
// on what body does to other nodes in the same step. The queue is private to the
// wave, whose LDS accesses complete in order.
constexpr int WQ = 128;
// Arrays of a wave's forward record: queued nodes, step numbers, step ends, and, with
// the state in device memory, each queued node's first arc (two halves) and degree, so
// that the backward reads a node's arcs without an L2 trip through the row pointers.
// (For LDS-state groups, mostly small, the extra stores cost more than they save.)
__host__ __device__ constexpr int rec_arrays(bool global_state) { return global_state ? 6 : 3; }
template <int T, int SCAN, int BLK, class Sel, class Body>
__device__ __forceinline__ void for_selected(int32_t n, int32_t* wq, Sel&& sel, Body&& body) {
    constexpr int NW = T / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // pass q of wave w reads blocks w + NW * (q * 64 / BLK + j), j = lane / BLK
    const int32_t off = NW * BLK * (lane / BLK) + lane % BLK;
    int cnt = 0;
    for (int32_t base0 = wave * BLK; base0 < n; base0 += SCAN * T) {
        unsigned long long ms[SCAN];
        bool hit[SCAN];
#pragma unroll
        for (int p = 0; p < SCAN; ++p) {
            const int32_t v = base0 + p * T + off;
            hit[p] = v < n && sel(v);
            ms[p] = __ballot(hit[p]);
        }
#pragma unroll
        for (int p = 0; p < SCAN; ++p) {
            const unsigned long long m = ms[p];
            if (m == 0ull) continue;
            const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (hit[p]) wq[cnt + rank] = base0 + p * T + off;
            cnt += __popcll(m);
            if (cnt >= 64) {
                body(wq[lane], true);
                const int rest = cnt - 64;
                const int32_t t = lane < rest ? wq[64 + lane] : 0;
                if (lane < rest) wq[lane] = t;
                cnt = rest;
            }
        }
    }
    if (cnt > 0) body(lane < cnt ? wq[lane] : 0, lane < cnt);
}

// Visit the nodes whose bits are set in row (W words of a bucket bitmap) and for which
// keep(v) holds, clearing the row. Word i holds nodes 32i .. 32i+31; wave w takes the
// words of the 64-node blocks b with b % NW == w, 32 blocks (64 words, one per lane) per
// pass, and queues the kept nodes in increasing order. Those are the queues, and the
// body calls, that for_selected builds from the same selection, so a step may use
// either one without changing any result. A pass places its set bits in order with a
// scan of the per-lane bit counts; output slot P then finds its word by a binary search
// over the lanes and its bit by a search over the word's bit counts, so no lane loops
// over the bits of a dense word while the others wait.
template <int T, class Keep, class Body>
__device__ __forceinline__ void for_bucket(uint32_t* __restrict__ row, int32_t W, int32_t* wq,
                                           Keep&& keep, Body&& body) {
    constexpr int NW = T / 64;
    const int lane = threadIdx.x & 63;
    const int32_t nblk = (W + 1) >> 1;
    int cnt = 0;
    for (int32_t b0 = threadIdx.x >> 6; b0 < nblk; b0 += NW * 32) {
        const int32_t i = 2 * (b0 + NW * (lane >> 1)) + (lane & 1);
        uint32_t bits = 0u;
        if (i < W) {
            bits = row[i];
            if (bits) row[i] = 0u;
        }
        const unsigned long long any = __ballot(bits != 0u);
        if (any == 0ull) continue;
        const int pc = __popc(bits);
        int incl = pc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        const int excl = incl - pc;
        const int total = __shfl(incl, 63, 64);
        for (int q = 0; q < total; q += 64) {
            const int P = q + lane;
            // the last lane whose first slot is at or before P holds slot P
            int l = 0;
#pragma unroll
            for (int st = 32; st > 0; st >>= 1)
                if (__shfl(excl, l + st, 64) <= P) l += st;
            uint32_t w = (uint32_t)__shfl((int)bits, l, 64);
            int r = P - __shfl(excl, l, 64), pos = 0;
#pragma unroll
            for (int h = 16; h > 0; h >>= 1) {
                const int c = __popc(w & ((1u << h) - 1u));
                if (r >= c) {
                    r -= c;
                    w >>= h;
                    pos += h;
                }
            }
            const int32_t v = (2 * (b0 + NW * (l >> 1)) + (l & 1)) * 32 + pos;
            const bool hit = P < total && keep(v);
            const unsigned long long m = __ballot(hit);
            if (m == 0ull) continue;
            const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (hit) wq[cnt + rank] = v;
            cnt += __popcll(m);
            if (cnt >= 64) {
                body(wq[lane], true);
                const int rest = cnt - 64;
                const int32_t t = lane < rest ? wq[64 + lane] : 0;
                if (lane < rest) wq[lane] = t;
                cnt = rest;
            }
        }
    }
    if (cnt > 0) body(lane < cnt ? wq[lane] : 0, lane < cnt);
}

// Arc expansion of a queue: lane i holds queued node q (valid) whose arcs are
// [rp[lo+q], rp[lo+q+1]) (the calling lane's slot holds the arcs [e0, e0 + deg), deg = 0
// for an empty slot). Round r covers the queue's arcs r .. r+63, in node order, one per
// lane: owner = queue slot of the arc's node, e = the arc, ok = false past the last arc;
// incl/excl are each lane's own inclusive/exclusive arc offsets (its slot's range
// [excl, incl)).
// The owner of arc p is the last slot with arcs whose range starts at or before p:
// each slot with arcs starting in the round writes its index at that position of the
// 64-entry LDS scratch own (position 0 holds the previous round's last owner), and a
// max-scan over the lanes fills the gaps. own is free between rounds. It is the first
// half of the wave's queue, which the caller has read into q already: own must not be
// declared restrict, or that read may be moved past the writes here.
struct QueueRounds {
    int32_t* own;
    int deg, incl, excl, total, e0lo, e0hi, carry;
    __device__ __forceinline__ QueueRounds(int64_t e0, int deg_, int32_t* own_) : own(own_), deg(deg_) {
        incl = wscan_add(deg);
        total = __builtin_amdgcn_readlane(incl, 63);
        excl = incl - deg;
        e0lo = (int)(uint32_t)(uint64_t)e0;
        e0hi = (int)(uint32_t)((uint64_t)e0 >> 32);
        carry = -1;
    }
    // This lane's owner slot, arc and validity in round rk (all lanes converged; rounds
    // asked for in increasing order, each once; ok = false for every lane past the end)
    __device__ __forceinline__ void round(int rk, int& o_, int64_t& e_, bool& ok_) {
        const int lane = threadIdx.x & 63;
        o_ = 0;
        e_ = 0;
        ok_ = false;
        if (rk >= total) return;
        __builtin_amdgcn_wave_barrier();  // the previous round's reads first
        own[lane] = -1;
        if (deg > 0 && excl >= rk && excl < rk + 64) own[excl - rk] = lane;
        __builtin_amdgcn_wave_barrier();  // other lanes' writes before the read
        int o = own[lane];
        if (lane == 0) o = max(o, carry);
        const int i = wscan_max(o);
        carry = __builtin_amdgcn_readlane(i, 63);
        const int p = rk + lane;
        const int ex = __shfl(excl, i, 64);
        const uint64_t base = ((uint64_t)(uint32_t)__shfl(e0hi, i, 64) << 32) | (uint32_t)__shfl(e0lo, i, 64);
        o_ = i;
        e_ = (int64_t)base + (p - ex);
        ok_ = p < total;
    }
};

// One round at a time: f(owner, e, ok, incl, excl, r). All lanes stay converged, so f
// may use cross-lane operations before it branches on ok.
template <class F>
__device__ __forceinline__ void for_queue_arcs(int64_t e0, int deg, int32_t* own, F&& f) {
    QueueRounds Q(e0, deg, own);
    for (int r = 0; r < Q.total; r += 64) {
        int i;
        int64_t e;
        bool ok;
        Q.round(r, i, e, ok);
        f(i, e, ok, Q.incl, Q.excl, r);
    }
}

// K rounds handed over at once: f(owner[K], e[K], ok[K]) gets the queue's arcs r ..
// r + 64K - 1, arc r + 64k + lane in slot k, so that it can issue the loads of K arcs
// per lane before it waits for any of them.
template <int K, class F>
__device__ __forceinline__ void for_queue_arcs_k(int64_t e0, int deg, int32_t* own, F&& f) {
    QueueRounds Q(e0, deg, own);
    for (int r = 0; r < Q.total; r += 64 * K) {
        int ow[K];
        int64_t ee[K];
        bool ok[K];
#pragma unroll
        for (int k = 0; k < K; ++k) Q.round(r + 64 * k, ow[k], ee[k], ok[k]);
        f(ow, ee, ok);
    }
}

// Three stages per round, pipelined one round deep: x = load(e, ok) issues the round's
// first loads; y = issue(owner, e, ok, incl, excl, r, x) uses them and issues the loads
// that depend on them; then the next round's owners are found and its load() issued,
// and only then finish(owner, e, ok, incl, excl, r, x, y) waits for the dependent loads. Rounds run in order (finish of
// round r before issue of round r + 64), so what finish leaves behind (a row's running
// minimum, its sums) is seen by the next round exactly as in for_queue_arcs.
template <class LD, class IS, class FN>
__device__ __forceinline__ void for_queue_arcs_pipe(int64_t e0, int deg, int32_t* own, LD&& load, IS&& issue,
                                                    FN&& finish) {
    QueueRounds Q(e0, deg, own);
    if (Q.total == 0) return;
    int ow;
    int64_t e;
    bool ok;
    Q.round(0, ow, e, ok);
    auto x = load(e, ok);
    for (int r = 0; r < Q.total; r += 64) {
        const auto y = issue(ow, e, ok, Q.incl, Q.excl, r, x);
        int ow2;
        int64_t e2;
        bool ok2;
        Q.round(r + 64, ow2, e2, ok2);
        const auto x2 = load(e2, ok2);
        finish(ow, e, ok, Q.incl, Q.excl, r, x, y);
        ow = ow2;
        e = e2;
        ok = ok2;
        x = x2;
    }
}

// One table entry (frontier f, d(f,v)) of an interior row, and what the interior
// sweeps carry from a round's tests to its sums.
struct IEnt {
    int32_t f;
    uint32_t L;
};
struct IMin {
    uint32_t sm;  // segmented minimum up to this lane
    int seg;
    bool on;      // the entry attains the row's minimum so far
    uint64_t a, t;  // sigma(s,f), sigma(f,v)
};
struct IDel {
    int seg;
    bool on;      // v lies on a shortest path from s to f
    uint64_t t, cf;  // sigma(f,v), coef(s,f) (its bits)
};

}  // namespace

// Compact launch records: a group (node range, its sources in a shared array, its
// score rows) and the graph it runs on, stored once for all groups over that graph.
struct RCtx {
    EGraph g;
    const int64_t* trow;
    const int32_t* tcol;
    const uint32_t* tlen;
    const uint64_t* tsig;
};
struct RGroup {
    int32_t ctx, lo, hi, nsrc;
    int32_t t_lo, tn;
    uint32_t flags;
    int32_t lg;     // bucket bitmaps: log2 of the bucket count (>= longest arc + 1); -1 = scan
    int32_t dense;  // a bucket step with more bits than this scans the range instead
    int32_t tw;     // words of the tight-arc bitmap (0 = none): in LDS after the state, or gtb
    int64_t src_off;
    double* cacc;
    double* cint;
    uint32_t* idist;  // [tn] interior d(s,v) of the current source
    uint64_t* isig;   // [tn] interior sigma(s,v) of the current source
    uint32_t* gdist;  // [hi-lo] one-source state in device memory (ranges beyond LDS)
    uint64_t* gsig;
    uint32_t* gtb;    // [tw] their tight-arc bitmap (state in device memory only)
    int32_t* rlist;   // backward groups: per-wave record of the forward's queues
    uint32_t* steps;  // backward groups: distance of each forward step
    uint32_t* odist;  // GF_EXPORT: [nsrc][hi-lo] d(s,v) after each source's forward sweep
    uint64_t* osig;   //            [nsrc][hi-lo] sigma(s,v)
    uint64_t* ocoef;  // GF_ISPLIT: [nsrc][hi-lo] coef(s,v) after each source's backward
};

// A saved value of one (node, source) for k_interior: d(s,v) and a 64-bit word,
// sigma(s,v) or coef(s,v); 16 bytes, so that a row's threads read one line per node.
struct IRec {
    uint32_t d, pad;
    uint64_t x;
};

// One GF_ISPLIT group for k_interior: its table rows, the rows its resident kernel saved
// for each source, its interior scores, and its first block in the launch.
struct IGroup {
    int32_t lo, n, t_lo, tn;
    int32_t nsrc, lanes;  // lanes per table row: a power of two >= nsrc, at most 64
    int64_t blk0;         // first k_interior block
    int64_t tblk0;        // first block of the transpose
    const int64_t* trow;
    const int32_t* tcol;
    const uint32_t* tlen;
    const uint64_t* tsig;
    const uint32_t* odist;  // [nsrc][n], as the resident kernel saved them
    const uint64_t* osig;
    const uint64_t* ocoef;
    IRec* xa;  // [n][lanes], node-major: {d, sigma} for the first sweep
    IRec* xb;  //                         {d, coef} for the second
    double* cint;  // [tn]
};

namespace {

// Device-memory arrays are used through global-address-space pointers. The launch
// records hold generic pointers, whose accesses compile to flat instructions, and a
// wait for a flat load's data also waits for every LDS operation in flight (and the
// reverse), which serialises the arc rounds' L2 loads with their LDS atomics.
#define GAS __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GAS T* gas(T* p) {
    return (GAS T*)p;
}

// One packed arc record (the four 32-bit fields are adjacent and 16-byte aligned).
__device__ __forceinline__ ArcRec load_arc(const GAS ArcRec* p, int64_t e) {
    const GAS uint32_t* q = (const GAS uint32_t*)(p + e);
    return ArcRec{q[0], q[1], q[2], q[3]};
}


template <int T, bool GLOBAL, bool BYTE>
__global__ void __launch_bounds__(T) k_resident(const RGroup* __restrict__ rgs,
                                                const RCtx* __restrict__ ctxs,
                                                const int32_t* __restrict__ srcs,
                                                uint32_t* __restrict__ err,
                                                unsigned long long* __restrict__ prof) {
    // prof: null, or this launch's counter of algorithmic bytes
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ uint32_t fwd_next[3];  // rotating: step k writes [k%3], clears [(k+1)%3]
    __shared__ uint32_t ovf_flag;
    __shared__ int32_t wqueue[T / 64][WQ];
    // device-memory groups: per wave, the path counts of its queue's nodes being summed
    __shared__ unsigned long long wsig[GLOBAL ? T / 64 : 1][64];

    const RGroup& R = rgs[blockIdx.x];
    const RCtx& C = ctxs[R.ctx];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    int32_t* wq = wqueue[tid >> 6];  // also the arc rounds' owner scratch: not restrict
    const int32_t lo = R.lo;
    const int32_t n = R.hi - R.lo;
    // One source's state: in LDS, or (GLOBAL) in device memory, changed through L2
    // atomics and read past the CU's L1 (agent-scope atomic loads), always through
    // global-address-space pointers
    uint32_t* __restrict__ dist = reinterpret_cast<uint32_t*>(lds);
    uint64_t* __restrict__ sig = reinterpret_cast<uint64_t*>(lds + (((size_t)n * 4 + 15) & ~(size_t)15));
    GAS uint32_t* __restrict__ gdist = gas(R.gdist);
    GAS uint64_t* __restrict__ gsig = gas(R.gsig);
    // BYTE (ranges beyond LDS with arcs of at most 63): the distance state is one byte
    // per node in LDS: 0xFF unreached; 0x00..0x7F pending, the tentative distance mod
    // 128; 0x80 | (d mod 127) settled. Pending distances lie within the longest arc
    // above the step's D, and a settled neighbour of a node at distance D lies within
    // the arc's length of D on either side, so these residues decide every comparison
    // the sweeps make exactly. A node's exact distance goes to gdist when it settles
    // (read only for settled nodes); path counts stay in gsig as with GLOBAL.
    uint8_t* __restrict__ db = lds;
    uint32_t* db32 = reinterpret_cast<uint32_t*>(lds);
    auto settled_b = [](uint32_t b) { return b >= 0x80u && b != 0xFFu; };
    // (x - L) mod 127 and (x + L) mod 127 for a residue x < 127 and 0 <= L <= 126
    auto sub127 = [](uint32_t x, uint32_t L) { return x >= L ? x - L : x + 127u - L; };
    auto add127 = [](uint32_t x, uint32_t L) { return x + L >= 127u ? x + L - 127u : x + L; };
    auto D_ = [&](int32_t i) -> uint32_t {
        if constexpr (BYTE)
            return settled_b(db[i]) ? __hip_atomic_load(gdist + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                    : INF32;
        else if constexpr (GLOBAL)
            return __hip_atomic_load(gdist + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            return dist[i];
    };
    auto S_ = [&](int32_t i) -> uint64_t {
        if constexpr (GLOBAL)
            return __hip_atomic_load(gsig + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            return sig[i];
    };
    auto setD = [&](int32_t i, uint32_t v) {
        if constexpr (GLOBAL)
            gdist[i] = v;
        else
            dist[i] = v;
    };
    auto setS = [&](int32_t i, uint64_t v) {
        if constexpr (GLOBAL)
            gsig[i] = v;
        else
            sig[i] = v;
    };
    auto minD = [&](int32_t i, uint32_t v) -> uint32_t {
        if constexpr (GLOBAL)
            return __hip_atomic_fetch_min(gdist + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            return atomicMin(&dist[i], v);
    };
    auto addS = [&](int32_t i, uint64_t v) -> uint64_t {
        if constexpr (GLOBAL)
            return __hip_atomic_fetch_add(gsig + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            return atomicAdd((unsigned long long*)&sig[i], (unsigned long long)v);
    };
    // device-memory arrays, read and written as global memory (see gas)
    const GAS int64_t* __restrict__ rp = gas(C.g.row_ptr);
    const GAS int32_t* __restrict__ col = gas(C.g.col);
    const GAS uint32_t* __restrict__ len = gas(C.g.len);
    const GAS uint64_t* __restrict__ mult = gas(C.g.mult);
    // packed arc records (device-memory groups): head, length, reverse arc and
    // multiplicity of an arc in one 16-byte load
    const GAS ArcRec* __restrict__ arcp = GLOBAL ? gas(C.g.arc) : nullptr;
    const GAS uint8_t* __restrict__ nflag = gas(C.g.nflag);
    const GAS int64_t* __restrict__ trow = gas(C.trow);
    const GAS int32_t* __restrict__ tcol = gas(C.tcol);
    const GAS uint32_t* __restrict__ tlen = gas(C.tlen);
    const GAS uint64_t* __restrict__ tsig = gas(C.tsig);
    const bool cent = (R.flags & GF_CENT) != 0 && R.tn > 0;
    // the interior rows are left to k_interior: this kernel saves d, sigma and coef of
    // every node per source instead
    const bool isplit = cent && (R.flags & GF_ISPLIT) != 0;
    GAS double* __restrict__ cacc = gas(R.cacc);
    GAS double* __restrict__ cint = gas(R.cint);
    GAS uint32_t* __restrict__ steps = gas(R.steps);
    // interior scratch of the current source: d(s,v) and sigma(s,v) per table row
    GAS uint32_t* __restrict__ idist = gas(R.idist);
    GAS uint64_t* __restrict__ isig = gas(R.isig);

    // Dijkstra_SK groups (no GF_BACKWARD): forward only, restricted path counts, and
    // d and sigma of every node written out per source lane
    const bool bwd = (R.flags & GF_BACKWARD) != 0;
    // Node ownership blocks of the scan: a step's nodes cluster (communities are runs of
    // ids), and the step lasts as long as its busiest wave, so LDS-state groups deal
    // 16-node blocks round the waves. Device-memory state keeps 64-node blocks (those of
    // the bucket visit; with the byte state, a wave's 64 consecutive nodes share the lines
    // of their arc records and counts, which outweighs the finer balance: pareto_100k's
    // plain pass 28.6 ms with 16-node blocks, 26.6 ms with 64; whole per-wave slices
    // lose the balance, 43 ms against 40 for Brandes_SK).
    constexpr int OWN_BLK = GLOBAL ? 64 : 16;
    const bool restrict_ = (R.flags & GF_RESTRICT) != 0;
    // Bucket bitmaps (state in device memory and R.lg >= 0), in LDS: bucket d mod 2^lg
    // holds one bit per node offered distance d (the pending distances D+1 .. D+longest
    // arc never share a bucket), and a counter of bits set per bucket and per parity of
    // d >> lg. A sparse step reads and clears its bucket instead of reading every node's
    // distance from L2; the next step is the nearest distance whose counter is non-zero.
    // Offers made during a step go to other buckets, and to the other counter copy of
    // the bucket being retired, so no write races the retiring. (With the state in LDS a
    // scan step costs a few LDS reads per thread, less than the bitmaps' atomics and the
    // occupancy their LDS would take.)
    const bool bucket = GLOBAL && !BYTE && R.lg >= 0;
    const int lg = bucket ? R.lg : 0;
    const uint32_t RM = bucket ? (1u << lg) - 1u : 0u;
    const int32_t W = (n + 31) >> 5;
    uint32_t* __restrict__ bm = reinterpret_cast<uint32_t*>(lds);  // [RM+1][W]
    uint32_t* __restrict__ bc = bm + (size_t)(RM + 1) * W;         // [RM+1][2]
    auto cidx = [&](uint32_t d) { return ((d & RM) << 1) | ((d >> lg) & 1u); };
    // Tight-arc bitmap (backward groups whose graph has reverse-arc indices): one bit per
    // arc of the range, in LDS after the state, or in device memory (R.gtb) with the
    // state. For every tight parent arc x -> v that the forward finds, it sets the bit of
    // the reverse arc v -> x (same length and multiplicity), so the backward expands only
    // v's arcs to its children, in arc order: exactly the arcs whose test
    // dx == dv + len would pass, without reading the others.
    const GAS int64_t* __restrict__ twin = gas(C.g.twin);
    uint32_t* __restrict__ tb = reinterpret_cast<uint32_t*>(lds + (((size_t)n * 4 + 15) & ~(size_t)15) + (size_t)n * 8);
    GAS uint32_t* __restrict__ gtb = gas(R.gtb);
    int64_t abase = 0;
    uint32_t tbits = 0;  // arcs of the range
    bool tight = false;
    if (bwd && R.tw > 0 && twin && (!GLOBAL || R.gtb)) {
        abase = rp[lo];
        const int64_t na = rp[R.hi] - abase;
        tight = na > 0 && na < ((int64_t)1 << 31) - 64 && ((na + 31) >> 5) <= (int64_t)R.tw;
        tbits = tight ? (uint32_t)na : 0u;
    }
    auto tb_ld = [&](int w) -> uint32_t {
        if constexpr (GLOBAL)
            return __hip_atomic_load(gtb + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            return tb[w];
    };
    // this wave's record region (backward groups): nodes, then step numbers, then ends;
    // a wave queues only nodes of its own blocks (at most 64 * ceil(n / T) of them)
    const int32_t wcap = 64 * ((n + T - 1) / T);
    // (and with GLOBAL each queued node's first arc, split in halves, and its degree)
    constexpr bool REC_ARCS = GLOBAL;
    GAS int32_t* __restrict__ rnodes = bwd ? gas(R.rlist) + (int64_t)(tid >> 6) * rec_arrays(GLOBAL) * wcap : nullptr;
    GAS int32_t* __restrict__ rsegk = bwd ? rnodes + wcap : nullptr;
    GAS int32_t* __restrict__ rsege = bwd ? rnodes + 2 * wcap : nullptr;
    GAS int32_t* __restrict__ re0lo = bwd && REC_ARCS ? rnodes + 3 * wcap : nullptr;
    GAS int32_t* __restrict__ re0hi = bwd && REC_ARCS ? rnodes + 4 * wcap : nullptr;
    GAS int32_t* __restrict__ rdeg = bwd && REC_ARCS ? rnodes + 5 * wcap : nullptr;
    if (bwd)
        for (int32_t v = tid; v < n; v += T) cacc[v] = 0.0;
    if (cent)
        for (int32_t i = tid; i < R.tn; i += T) cint[i] = 0.0;
    unsigned long long bytes = 0;
    if (tid == 0) ovf_flag = 0u;  // ordered before any use by the barrier below

    for (int b = 0; b < R.nsrc; ++b) {
        const int32_t s = srcs[R.src_off + b] - lo;
        if constexpr (BYTE) {
            // every node unreached but s, pending at distance 0
            for (int32_t i = tid; i < ((n + 3) >> 2); i += T)
                db32[i] = (i == (s >> 2)) ? ~(0xFFu << ((s & 3) * 8)) : 0xFFFFFFFFu;
            // counts are stored as nodes settle and read only for settled nodes
            if (tid == 0) setS(s, 1ull);
        } else {
            for (int32_t v = tid; v < n; v += T) {
                setD(v, (v == s) ? 0u : INF32);
                setS(v, (v == s) ? 1ull : 0ull);
            }
        }
        if (tight)
            for (int32_t i = tid; i < R.tw; i += T) {
                if constexpr (GLOBAL)
                    gtb[i] = 0u;
                else
                    tb[i] = 0u;
            }
        if (tid == 0) fwd_next[0] = fwd_next[1] = fwd_next[2] = INF32;
        if (bucket) {
            const int32_t tot = (int32_t)(RM + 1) * W;
            for (int32_t i = tid; i < tot; i += T) bm[i] = (i == (s >> 5)) ? (1u << (s & 31)) : 0u;
            for (int32_t i = tid; i < 2 * (int32_t)(RM + 1); i += T) bc[i] = (i == 0) ? 1u : 0u;
        }
        __syncthreads();

        // ------------------------------------------------------------ forward ----
        // Backward groups record, per wave, the nodes each step queued (in queue order)
        // and a (step, end) entry for every step in which the wave queued any; the
        // backward sweep replays these in reverse instead of scanning again. A wave
        // only ever queues nodes of its own scan passes, so its region holds at most
        // 64 * ceil(n / T) nodes and as many entries.
        uint32_t D = 0;
        bool ovf = false;
        // A bucket step can find only stale bits; it queues nothing and does not count
        // as a step, so the record holds at most one step per distinct final distance.
        int32_t wcur = 0, wseg = 0, wstep0 = 0, nsteps = 0;
        for (int it = 0, k = 0;; ++it) {
            uint32_t mn = INF32;
            const uint32_t d127 = D % 127u;
            if (bwd && tid == 0) steps[k] = D;
            auto fbody =
                [&](int32_t q, bool valid) {
                    if (prof && valid) bytes += 12ull;
                    int64_t e0 = 0;
                    int deg = 0;
                    if (valid) {
                        e0 = rp[lo + q];
                        deg = (int)(rp[lo + q + 1] - e0);
                    }
                    if (bwd) {
                        if (valid) {
                            rnodes[wcur + lane] = q;
                            if constexpr (REC_ARCS) {
                                re0lo[wcur + lane] = (int32_t)(uint32_t)(uint64_t)e0;
                                re0hi[wcur + lane] = (int32_t)(uint32_t)((uint64_t)e0 >> 32);
                                rdeg[wcur + lane] = deg;
                            }
                        }
                        wcur += (int32_t)__popcll(__ballot(valid));
                    }
                    // device-memory counts: each node's count is the sum over its own arcs
                    // (pull), so the wave sums its lanes' terms per node (segmented sums,
                    // carried across rounds in the node's lane) and stores it once
                    // (per wave: slot i of wsig sums the terms of queue slot i's node)
                    if constexpr (GLOBAL) wsig[tid >> 6][lane] = 0ull;
                    auto arc = [&](int owner, int64_t e, bool ok, int incl, int excl, int r, int32_t ucol, uint32_t L,
                                   uint32_t tw, uint32_t mu) {
                        const int32_t v = __shfl(q, owner, 64);
                        uint64_t xs = 0;
                        if (ok) {
                            if (prof) bytes += 12ull;
                            const int32_t u = ucol - lo;
                            // (device-memory groups read the reverse arc only for tight arcs)
                            const int64_t te = tight && !GLOBAL ? twin[e] : 0;
                            // one read of u's distance serves both tests below: if another
                            // lane lowers it meanwhile, the offer test passes at worst for an
                            // offer that then changes nothing
                            uint32_t du = 0, uw = 0;
                            bool parent = false;
                            if constexpr (BYTE) {
                                // u settled at D - L: a settled neighbour lies in [D - L, D],
                                // L + 1 <= 64 values with distinct residues mod 127
                                uw = db32[u >> 2];
                                const uint32_t bu = (uw >> ((u & 3) * 8)) & 0xFFu;
                                parent = L <= D && settled_b(bu) && (bu & 0x7Fu) == sub127(d127, L);
                            } else {
                                du = D_(u);
                                parent = du != INF32 && du + L == D;
                            }
                            // u is a parent of v if it settled at D - L in an earlier step (eq.
                            // parentsall / eq. multiparents); the count adds in with an atomic,
                            // exact for integers, and a wrap of any addition is an overflow
                            if (v != s && L <= D) {
                                // Dijkstra_SK (eq. frontierparents): a frontier parent other
                                // than the source is tight but adds no paths
                                if (parent &&
                                    !(restrict_ && u != s && nflag && (nflag[lo + u] & NF_BLOCKED))) {
                                    if (tight) {
                                        const uint64_t t =
                                            (uint64_t)((GLOBAL ? (arcp ? (int64_t)tw : twin[e]) : te) - abase);
                                        if (t < tbits) {
                                            if constexpr (GLOBAL)
                                                __hip_atomic_fetch_or(gtb + (t >> 5), 1u << (t & 31),
                                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                            else
                                                atomicOr(&tb[t >> 5], 1u << (t & 31));
                                        }
                                    }
                                    uint64_t x = S_(u);
                                    if (mult) {
                                        const uint64_t m = arcp ? (uint64_t)mu : mult[e];
                                        if (__umul64hi(x, m) != 0) ovf = true;
                                        x *= m;
                                    }
                                    if constexpr (GLOBAL) {
                                        xs = x;
                                    } else if (x) {
                                        const uint64_t old = addS(v, x);
                                        if (old + x < old) ovf = true;
                                    }
                                }
                            }
                            // offers: all above D, so they never meet the parent test above
                            const uint32_t nv = D + L;
                            if constexpr (BYTE) {
                                // lower u's byte to nv's residue unless u is settled or already
                                // pending at most L above D (offsets of pending bytes from D
                                // are at most the longest arc); a compare-and-swap on the word
                                // holding it, retried while other bytes of the word change
                                const int sh = (u & 3) * 8;
                                for (;;) {
                                    const uint32_t bu = (uw >> sh) & 0xFFu;
                                    if (settled_b(bu) || (bu != 0xFFu && ((bu - D) & 127u) <= L)) break;
                                    const uint32_t nw = (uw & ~(0xFFu << sh)) | ((nv & 127u) << sh);
                                    const uint32_t prev = atomicCAS(&db32[u >> 2], uw, nw);
                                    if (prev == uw) {
                                        mn = min(mn, nv);
                                        break;
                                    }
                                    uw = prev;
                                }
                            } else if (nv < du) {
                                if (bucket) {
                                    // a bit per successful offer (a failed one leaves none)
                                    const uint32_t old = minD(u, nv);
                                    if (nv < old) {
                                        const uint32_t bit = 1u << (u & 31);
                                        const uint32_t ow = atomicOr(&bm[(size_t)(nv & RM) * W + (u >> 5)], bit);
                                        if (!(ow & bit)) atomicAdd(&bc[cidx(nv)], 1u);
                                    }
                                } else {
                                    // the smallest offer to a node always lands, so the least
                                    // offer made is the least new tentative distance, and no
                                    // offer has to wait for the atomic's old value
                                    minD(u, nv);
                                    mn = min(mn, nv);
                                }
                            }
                        }
                        if constexpr (GLOBAL) {
                            if (xs) {
                                const unsigned long long o = atomicAdd(&wsig[tid >> 6][owner], (unsigned long long)xs);
                                if (o + xs < o) ovf = true;
                            }
                        }
                    };
                    // byte state with packed records: two arcs per lane in flight, each
                    // stage (byte tests, count loads, offers, sums) over both before the
                    // next, so that a lane waits once per stage; and the next two arcs'
                    // records are loaded behind the count loads of the current two, so
                    // that their wait overlaps the offers and sums
                    bool done = false;
                    if constexpr (BYTE) {
                        if (arcp) {
                            done = true;
                            QueueRounds Q(e0, deg, wq);
                            int ow[2];
                            int64_t ee[2];
                            bool ok[2];
                            ArcRec a[2];
#pragma unroll
                            for (int j = 0; j < 2; ++j) Q.round(64 * j, ow[j], ee[j], ok[j]);
#pragma unroll
                            for (int j = 0; j < 2; ++j)
                                a[j] = ok[j] ? load_arc(arcp, ee[j]) : ArcRec{(uint32_t)lo, 1u, 0u, 1u};
                            for (int r = 0; r < Q.total; r += 128) {
                                int32_t u[2];
                                uint32_t uw[2];
                                bool par[2];
                                uint64_t x[2];
#pragma unroll
                                for (int j = 0; j < 2; ++j) {
                                    const int32_t v = __shfl(q, ow[j], 64);
                                    u[j] = (int32_t)a[j].head - lo;
                                    uw[j] = 0u;
                                    par[j] = false;
                                    if (ok[j]) {
                                        if (prof) bytes += 12ull;
                                        const uint32_t L = a[j].len;
                                        uw[j] = db32[u[j] >> 2];
                                        const uint32_t bu = (uw[j] >> ((u[j] & 3) * 8)) & 0xFFu;
                                        // u settled at D - L (eq. parentsall / eq. multiparents);
                                        // Dijkstra_SK: a frontier parent other than the source
                                        // adds no paths (eq. frontierparents)
                                        par[j] = v != s && L <= D && settled_b(bu) && (bu & 0x7Fu) == sub127(d127, L) &&
                                                 !(restrict_ && u[j] != s && nflag && (nflag[lo + u[j]] & NF_BLOCKED));
                                    }
                                }
#pragma unroll
                                for (int j = 0; j < 2; ++j) {
                                    x[j] = 0ull;
                                    if (par[j]) {
                                        if (tight) {
                                            const uint64_t t = (uint64_t)((int64_t)a[j].twin - abase);
                                            if (t < tbits)
                                                __hip_atomic_fetch_or(gtb + (t >> 5), 1u << (t & 31), __ATOMIC_RELAXED,
                                                                      __HIP_MEMORY_SCOPE_AGENT);
                                        }
                                        x[j] = S_(u[j]);
                                    }
                                }
                                // the next two arcs: owners, then record loads
                                int ow2[2];
                                int64_t ee2[2];
                                bool ok2[2];
                                ArcRec a2[2];
#pragma unroll
                                for (int j = 0; j < 2; ++j) Q.round(r + 128 + 64 * j, ow2[j], ee2[j], ok2[j]);
#pragma unroll
                                for (int j = 0; j < 2; ++j)
                                    a2[j] = ok2[j] ? load_arc(arcp, ee2[j]) : ArcRec{(uint32_t)lo, 1u, 0u, 1u};
                                // offers (all above D): lower u's byte to D + L's residue unless
                                // u is settled or already pending at most L above D
#pragma unroll
                                for (int j = 0; j < 2; ++j) {
                                    if (!ok[j]) continue;
                                    const uint32_t L = a[j].len, nv = D + L;
                                    const int sh = (u[j] & 3) * 8;
                                    uint32_t w = uw[j];
                                    for (;;) {
                                        const uint32_t bu = (w >> sh) & 0xFFu;
                                        if (settled_b(bu) || (bu != 0xFFu && ((bu - D) & 127u) <= L)) break;
                                        const uint32_t nw = (w & ~(0xFFu << sh)) | ((nv & 127u) << sh);
                                        const uint32_t prev = atomicCAS(&db32[u[j] >> 2], w, nw);
                                        if (prev == w) {
                                            mn = min(mn, nv);
                                            break;
                                        }
                                        w = prev;
                                    }
                                }
#pragma unroll
                                for (int j = 0; j < 2; ++j) {
                                    if (!par[j]) continue;
                                    uint64_t xx = x[j];
                                    if (mult) {
                                        const uint64_t m = a[j].mult;
                                        if (__umul64hi(xx, m) != 0) ovf = true;
                                        xx *= m;
                                    }
                                    if (xx) {
                                        const unsigned long long o =
                                            atomicAdd(&wsig[tid >> 6][ow[j]], (unsigned long long)xx);
                                        if (o + xx < o) ovf = true;
                                    }
                                }
#pragma unroll
                                for (int j = 0; j < 2; ++j) {
                                    ow[j] = ow2[j];
                                    ee[j] = ee2[j];
                                    ok[j] = ok2[j];
                                    a[j] = a2[j];
                                }
                            }
                        }
                    }
                    if constexpr (!GLOBAL && T <= 512) {
                        // LDS state on a small skeleton with clique arcs: the same staging,
                        // two arcs per lane, from the packed records (a parent's
                        // multiplicity then comes with its head instead of from a load of
                        // its own). (The 1024-thread class keeps one arc per lane: there
                        // the staging measured slower.)
                        const GAS ArcRec* __restrict__ arcl = mult ? gas(C.g.arc) : nullptr;
                        if (arcl) {
                            done = true;
                            for_queue_arcs_k<2>(e0, deg, wq, [&](const int* ow, const int64_t* ee, const bool* ok) {
                                ArcRec a[2];
                                int32_t u[2], vv[2];
                                uint32_t du[2];
                                bool par[2];
#pragma unroll
                                for (int j = 0; j < 2; ++j)
                                    a[j] = ok[j] ? load_arc(arcl, ee[j]) : ArcRec{(uint32_t)lo, 1u, 0u, 1u};
#pragma unroll
                                for (int j = 0; j < 2; ++j) {
                                    const int32_t v = __shfl(q, ow[j], 64);
                                    vv[j] = v;
                                    u[j] = (int32_t)a[j].head - lo;
                                    du[j] = INF32;
                                    par[j] = false;
                                    if (ok[j]) {
                                        if (prof) bytes += 12ull;
                                        const uint32_t L = a[j].len;
                                        du[j] = dist[u[j]];
                                        par[j] = v != s && L <= D && du[j] != INF32 && du[j] + L == D &&
                                                 !(restrict_ && u[j] != s && nflag && (nflag[lo + u[j]] & NF_BLOCKED));
                                    }
                                }
#pragma unroll
                                for (int j = 0; j < 2; ++j) {
                                    if (!par[j]) continue;
                                    if (tight) {
                                        const uint64_t t = (uint64_t)((int64_t)a[j].twin - abase);
                                        if (t < tbits) atomicOr(&tb[t >> 5], 1u << (t & 31));
                                    }
                                    uint64_t x = sig[u[j]];
                                    if (mult) {
                                        const uint64_t m = a[j].mult;
                                        if (__umul64hi(x, m) != 0) ovf = true;
                                        x *= m;
                                    }
                                    if (x) {
                                        const uint64_t old = addS(vv[j], x);
                                        if (old + x < old) ovf = true;
                                    }
                                }
#pragma unroll
                                for (int j = 0; j < 2; ++j) {
                                    const uint32_t nv = D + a[j].len;
                                    if (ok[j] && nv < du[j]) {
                                        minD(u[j], nv);
                                        mn = min(mn, nv);
                                    }
                                }
                            });
                        }
                    }
                    if (!done)
                    for_queue_arcs(e0, deg, wq, [&](int owner, int64_t e, bool ok, int incl, int excl, int r) {
                        int32_t c = 0;
                        uint32_t L = 1u, tw = 0u, mu = 1u;
                        if (ok) {
                            if (arcp) {
                                const ArcRec a = load_arc(arcp, e);
                                c = (int32_t)a.head;
                                L = a.len;
                                tw = a.twin;
                                mu = a.mult;
                            } else {
                                c = col[e];
                                L = len ? len[e] : 1u;
                            }
                        }
                        arc(owner, e, ok, incl, excl, r, c, L, tw, mu);
                    });
                    if constexpr (GLOBAL) {
                        // (the wave's own LDS atomics complete in order before this read)
                        if (valid && q != s) setS(q, (uint64_t)wsig[tid >> 6][lane]);
                    }
                };
            if (bucket) {
                // both visits queue the same nodes in the same order, so the choice (made
                // on a count that stale bits inflate by a racy amount) changes no result
                uint32_t* row = bm + (size_t)(D & RM) * W;
                if (bc[cidx(D)] > (uint32_t)R.dense) {
                    for_selected<T, GLOBAL ? 8 : 2, OWN_BLK>(n, wq, [&](int32_t v) { return D_(v) == D; }, fbody);
                    for (int32_t i = tid; i < W; i += T) row[i] = 0u;
                } else {
                    for_bucket<T>(row, W, wq, [&](int32_t v) { return D_(v) == D; }, fbody);
                }
            } else if constexpr (BYTE) {
                // pending at D: settle (its byte and its exact distance) as it is selected;
                // within the step nothing else writes a node pending at D, and a node
                // settled at D passes no parent test of the step (arcs are 1..126 long)
                const uint32_t dres = D & 127u, sres = 0x80u | (D % 127u);
                for_selected<T, 4, OWN_BLK>(
                    n, wq,
                    [&](int32_t v) {
                        const uint32_t b = db[v];
                        if (b == dres) {
                            db[v] = (uint8_t)sres;
                            gdist[v] = D;
                            return true;
                        }
                        if (b < 0x80u) mn = min(mn, D + ((b - D) & 127u));
                        return false;
                    },
                    fbody);
            } else {
                for_selected<T, GLOBAL ? 8 : 2, OWN_BLK>(
                    n, wq,
                    [&](int32_t v) {
                        const uint32_t dv = D_(v);
                        if (dv == D) return true;
                        if (dv > D && dv != INF32) mn = min(mn, dv);
                        return false;
                    },
                    fbody);
            }
            const bool mine = bwd && wcur != wstep0;
            if (mine) {
                if (lane == 0) {
                    rsegk[wseg] = k;
                    rsege[wseg] = wcur;
                }
                ++wseg;
                wstep0 = wcur;
            }
            if (bucket) {
                // fwd_next[it % 3] != INF32: some wave queued a node in this step
                if (mine && lane == 0) fwd_next[it % 3] = 0u;
                if (tid == 0) fwd_next[(it + 1) % 3] = INF32;
                __syncthreads();
                if (!bwd || fwd_next[it % 3] != INF32) nsteps = ++k;
                if (tid == 0) bc[cidx(D)] = 0u;
                uint32_t nx = INF32;
                for (uint32_t j = 1; j <= RM; ++j)
                    if (bc[cidx(D + j)]) {
                        nx = D + j;
                        break;
                    }
                if (nx == INF32) break;
                D = nx;
                continue;
            }
            nsteps = ++k;
            mn = wmin_u32(mn);
            if (lane == 0 && mn != INF32) atomicMin(&fwd_next[it % 3], mn);
            if (tid == 0) fwd_next[(it + 1) % 3] = INF32;
            __syncthreads();
            const uint32_t nx = fwd_next[it % 3];
            if (nx == INF32) break;
            D = nx;
        }
        if (ovf) ovf_flag = 1u;
        if (bwd && ((R.flags & GF_EXPORT) || isplit)) {
            // (the last step ended with a barrier: every count is final; the barrier
            // after the interior rows orders these reads before the backward's writes)
            GAS uint32_t* __restrict__ od = gas(R.odist) + (int64_t)b * n;
            GAS uint64_t* __restrict__ os = gas(R.osig) + (int64_t)b * n;
            // eight nodes per thread at a time, their loads issued before any is used
            // (four: 0.2 ms more of pareto_100k's launch)
            constexpr int XU = 8;
            for (int32_t v0 = tid; v0 < n; v0 += XU * T) {
                uint32_t dv[XU];
                uint64_t sv[XU];
#pragma unroll
                for (int u = 0; u < XU; ++u) dv[u] = v0 + u * T < n ? D_(v0 + u * T) : INF32;
#pragma unroll
                for (int u = 0; u < XU; ++u) sv[u] = dv[u] != INF32 ? S_(v0 + u * T) : 0ull;
#pragma unroll
                for (int u = 0; u < XU; ++u)
                    if (v0 + u * T < n) {
                        od[v0 + u * T] = dv[u];
                        os[v0 + u * T] = sv[u];
                    }
            }
        }
        if (!bwd) {
            // (the last step ended with a barrier: every count is final)
            for (int32_t v = tid; v < n; v += T) {
                const uint32_t dv = D_(v);
                idist[(int64_t)v * 64 + b] = dv;
                isig[(int64_t)v * 64 + b] = dv == INF32 ? 0ull : S_(v);
            }
            __syncthreads();
            continue;
        }

        // ------------------------------------------- interior rows: d and sigma ----
        // Each wave takes 64 table rows at a time and spreads their entries over its lanes
        // (as the sweeps spread a queue's arcs): first the row minimum of d(s,f) + d(f,v)
        // by segmented minima, then the sum of sigma(s,f) * sigma(f,v) over the entries
        // that attain it by segmented sums (eq. localcentrality's tight frontiers).
        if (cent && !isplit) {
            for (int32_t r0 = (tid >> 6) * 64; r0 < R.tn; r0 += T) {
                const int32_t i = r0 + lane;
                const bool valid = i < R.tn;
                int64_t e0 = 0;
                int deg = 0;
                if (valid) {
                    e0 = trow[R.t_lo + i];
                    deg = (int)(trow[R.t_lo + i + 1] - e0);
                    if (prof) bytes += 32ull * (unsigned long long)deg;
                }
                // BYTE: one exact distance per row, its first entry's frontier f0; the
                // frontiers of one row are all reachable or none (each has a path to v
                // inside the part), and d(s,f) is within d(f,v) of d(s,v), so
                // d(s,f) - d(s,f0) follows from the residues when d(f,v) + d(f0,v) <= 63
                uint32_t adist = INF32, ares = 0u, alen = 0u;
                if constexpr (BYTE) {
                    if (valid && deg > 0) {
                        const int32_t f0 = tcol[e0] - lo;
                        alen = tlen[e0];
                        const uint32_t b0 = db[f0];
                        if (settled_b(b0)) {
                            adist = D_(f0);
                            ares = b0 & 0x7Fu;
                        }
                    }
                }
                // One sweep over the row's entries: per round, the segmented minimum of
                // the values, and the sum of sigma(s,f) * sigma(f,v) over the entries that
                // attain the smaller of that minimum and the row's minimum so far; the row
                // keeps the sum of its smallest value (a smaller round minimum restarts it)
                uint32_t rmin = INF32;
                uint64_t rsum = 0;
                bool rovf = false;
                for_queue_arcs_pipe(
                    e0, deg, wq,
                    [&](int64_t e, bool ok) {
                        IEnt x{0, 0u};
                        if (ok) {
                            x.f = tcol[e] - lo;
                            x.L = tlen[e];
                        }
                        return x;
                    },
                    [&](int owner, int64_t e, bool ok, int incl, int excl, int r, const IEnt& x) {
                        IMin y;
                        y.seg = max(__shfl(excl, owner, 64) - r, 0);
                        uint32_t val = INF32;
                        if constexpr (BYTE) {
                            const uint32_t ad = (uint32_t)__shfl((int)adist, owner, 64);
                            const uint32_t ar = (uint32_t)__shfl((int)ares, owner, 64);
                            const uint32_t al = (uint32_t)__shfl((int)alen, owner, 64);
                            if (ok && ad != INF32) {
                                uint32_t tf;
                                if (x.L + al <= 63u) {
                                    int dl = (int)(db[x.f] & 0x7Fu) - (int)ar;
                                    if (dl > 63) dl -= 127;
                                    if (dl < -63) dl += 127;
                                    tf = (uint32_t)((int)ad + dl);
                                } else {
                                    tf = D_(x.f);
                                }
                                val = tf + x.L;
                            }
                        } else if (ok) {
                            const uint32_t tf = D_(x.f);
                            if (tf != INF32) val = tf + x.L;
                        }
                        y.sm = wseg_min_u32(val, y.seg);
                        // the round minimum of this lane's row sits at the row's last lane here
                        const int last = min(__shfl(incl, owner, 64) - r, 64) - 1;
                        const uint32_t m =
                            min((uint32_t)__shfl((int)y.sm, last, 64), (uint32_t)__shfl((int)rmin, owner, 64));
                        y.on = val != INF32 && val == m;
                        y.a = y.on ? S_(x.f) : 0ull;
                        y.t = y.on ? tsig[e] : 0ull;
                        return y;
                    },
                    [&](int owner, int64_t e, bool ok, int incl, int excl, int r, const IEnt& x, const IMin& y) {
                        uint64_t c = 0;
                        bool lo2 = false;
                        if (y.on) {
                            if (__umul64hi(y.a, y.t) != 0) lo2 = true;
                            c = y.a * y.t;
                        }
                        c = wseg_sum_u64(c, y.seg, &lo2);
                        const unsigned long long ovm = __ballot(lo2);
                        const int ab = max(excl - r, 0), bb = min(incl - r, 64);
                        const uint32_t pmin = (uint32_t)__shfl((int)y.sm, max(bb - 1, 0), 64);
                        const uint64_t part = (uint64_t)__shfl((long long)c, max(bb - 1, 0), 64);
                        if (bb > ab && pmin != INF32) {
                            const int w = bb - ab;
                            const bool povf = ((ovm >> ab) & (w >= 64 ? ~0ull : ((1ull << w) - 1ull))) != 0ull;
                            if (pmin < rmin) {
                                rmin = pmin;
                                rsum = part;
                                rovf = povf;
                            } else if (pmin == rmin) {
                                rovf = rovf || povf || rsum + part < rsum;
                                rsum += part;
                            }
                        }
                    });
                bool o2 = rovf;
                if (valid) {
                    idist[i] = rmin;
                    isig[i] = rsum;
                }
                if (o2) ovf_flag = 1u;
            }
        }
        __syncthreads();

        // ----------------------------------------------------------- backward ----
        // steps in reverse (step 0 is the source alone); each wave replays the queues it
        // recorded for the step, so a node meets the same lanes as in the forward sweep
        int32_t seg = wseg - 1;
        for (int k = nsteps - 1; k >= 1; --k) {
            D = steps[k];
            const uint32_t d127 = D % 127u;
            auto body = [&](int32_t q, int64_t e0, int deg, bool valid) {
                    double prev = 0.0, ind = 0.0, acc = 0.0;
                    if (prof && valid) bytes += 8ull;
                    if (valid) {
                        prev = cacc[q];
                        ind = (nflag && (nflag[lo + q] & NF_TARGET)) ? 1.0 : 0.0;
                    }
                    if (tight) {
                        // only the arcs to v's children: their bits, in arc order. A node
                        // whose arcs span at most two bitmap words keeps those words (its
                        // own bits only) in registers, and the lanes that take its arcs
                        // read them with shuffles; a wider node's lanes read the bitmap.
                        const int a = valid ? (int)(e0 - abase) : 0;
                        const int dg = valid ? deg : 0;
                        const int sh = a & 31;
                        const bool narrow = sh + dg <= 64;
                        uint32_t x0 = 0u, x1 = 0u;
                        int td = 0;
                        if (dg > 0) {
                            if (narrow) {
                                x0 = tb_ld(a >> 5) & (~0u << sh);
                                if (sh + dg < 32)
                                    x0 &= ~0u >> (32 - (sh + dg));
                                else if (sh + dg > 32)
                                    x1 = tb_ld((a >> 5) + 1) & (~0u >> (64 - (sh + dg)));
                                td = __popc(x0) + __popc(x1);
                            } else {
                                td = bits_in(tb_ld, a, dg);
                            }
                        }
                        if (prof && valid) bytes += 20ull * (unsigned long long)deg;
                        const int an = narrow ? a : ~a;  // start bit, negative for a wide node
                        for_queue_arcs(0, td, wq, [&](int owner, int64_t j, bool ok, int incl, int excl, int r) {
                            const int seg = max(__shfl(excl, owner, 64) - r, 0);
                            const int ao = __shfl(an, owner, 64);
                            const uint32_t y0 = (uint32_t)__shfl((int)x0, owner, 64);
                            const uint32_t y1 = (uint32_t)__shfl((int)x1, owner, 64);
                            double c = 0.0;
                            if (ok) {
                                int pos;
                                if (ao >= 0) {
                                    const int c0 = __popc(y0);
                                    pos = (int)j < c0 ? ((ao >> 5) << 5) + nth_set_bit(y0, (int)j)
                                                      : (((ao >> 5) + 1) << 5) + nth_set_bit(y1, (int)j - c0);
                                } else {
                                    pos = select_bit(tb_ld, ~ao, (int)j);
                                }
                                const int64_t e = abase + pos;
                                if (arcp) {
                                    const ArcRec a = load_arc(arcp, e);
                                    c = __longlong_as_double((long long)S_((int32_t)a.head - lo));
                                    if (mult) c *= (double)a.mult;
                                } else {
                                    c = __longlong_as_double((long long)S_(col[e] - lo));
                                    if (mult) c *= (double)mult[e];
                                }
                            }
                            c = wseg_sum(c, seg);
                            const int ab = max(excl - r, 0), b = min(incl - r, 64);
                            const double part = __shfl(c, max(b - 1, 0), 64);
                            if (b > ab) acc += part;
                        });
                    } else
                    for_queue_arcs(e0, deg, wq, [&](int owner, int64_t e, bool ok, int incl, int excl, int r) {
                        // segment of this lane's arc: lanes from its node's first arc in
                        // this round
                        const int seg = max(__shfl(excl, owner, 64) - r, 0);
                        double c = 0.0;
                        if (ok) {
                            if (prof) bytes += 20ull;
                            ArcRec a;
                            if (arcp)
                                a = load_arc(arcp, e);
                            else
                                a = ArcRec{(uint32_t)col[e], len ? len[e] : 1u, 0u, 1u};
                            const int32_t x = (int32_t)a.head - lo;
                            const uint32_t L = a.len;
                            bool child;
                            if constexpr (BYTE) {
                                // a settled neighbour of a node at D lies in [D - L, D + L],
                                // at most 127 values: residues mod 127 are distinct
                                const uint32_t bx = db[x];
                                child = settled_b(bx) && (bx & 0x7Fu) == add127(d127, L);
                            } else {
                                const uint32_t dx = D_(x);
                                child = dx != INF32 && dx == D + L;
                            }
                            if (child) {
                                c = __longlong_as_double((long long)S_(x));
                                if (mult) c *= arcp ? (double)a.mult : (double)mult[e];
                            }
                        }
                        // per-node sums of the round: segmented inclusive scan
                        c = wseg_sum(c, seg);
                        // each slot takes the sum at the last lane of its arcs in the round
                        const int a = max(excl - r, 0), b = min(incl - r, 64);
                        const double part = __shfl(c, max(b - 1, 0), 64);
                        if (b > a) acc += part;
                    });
                    if (valid) {
                        const double sv = (double)S_(q);
                        const double dl = sv * acc;
                        cacc[q] = prev + dl;
                        setS(q, (uint64_t)__double_as_longlong((ind + dl) / sv));
                    }
                };
            if (seg >= 0 && rsegk[seg] == k) {
                const int32_t beg = seg > 0 ? rsege[seg - 1] : 0, end = rsege[seg];
                for (int32_t c = beg; c < end; c += 64) {
                    const bool valid = c + lane < end;
                    int32_t q = 0, d = 0;
                    int64_t e0 = 0;
                    if (valid) {
                        q = rnodes[c + lane];
                        if constexpr (REC_ARCS) {
                            e0 = (int64_t)(((uint64_t)(uint32_t)re0hi[c + lane] << 32) | (uint32_t)re0lo[c + lane]);
                            d = rdeg[c + lane];
                        } else {
                            e0 = rp[lo + q];
                            d = (int)(rp[lo + q + 1] - e0);
                        }
                    }
                    body(q, e0, d, valid);
                }
                --seg;
            }
            __syncthreads();
        }

        // --------------------------------------------- interior rows: delta ----
        // the same spread: sum of sigma(f,v) * coef(s,f) over the frontiers f for which v
        // lies on a shortest path from s to f, times sigma(s,v) (eq. localcentrality)
        if (isplit) {
            // (the backward's last step ended with a barrier: every coefficient is final)
            GAS uint64_t* __restrict__ oc = gas(R.ocoef) + (int64_t)b * n;
            constexpr int XU = 8;
            for (int32_t v0 = tid; v0 < n; v0 += XU * T) {
                uint64_t cv[XU];
#pragma unroll
                for (int u = 0; u < XU; ++u) cv[u] = v0 + u * T < n ? S_(v0 + u * T) : 0ull;
#pragma unroll
                for (int u = 0; u < XU; ++u)
                    if (v0 + u * T < n) oc[v0 + u * T] = cv[u];
            }
        } else if (cent) {
            for (int32_t r0 = (tid >> 6) * 64; r0 < R.tn; r0 += T) {
                const int32_t i = r0 + lane;
                const bool valid = i < R.tn;
                uint32_t dv = INF32;
                int64_t e0 = 0;
                int deg = 0;
                if (valid) {
                    dv = idist[i];
                    e0 = trow[R.t_lo + i];
                    deg = dv == INF32 ? 0 : (int)(trow[R.t_lo + i + 1] - e0);
                }
                double acc = 0.0;
                for_queue_arcs_pipe(
                    e0, deg, wq,
                    [&](int64_t e, bool ok) {
                        IEnt x{0, 0u};
                        if (ok) {
                            x.f = tcol[e] - lo;
                            x.L = tlen[e];
                        }
                        return x;
                    },
                    [&](int owner, int64_t e, bool ok, int incl, int excl, int r, const IEnt& x) {
                        IDel y;
                        y.seg = max(__shfl(excl, owner, 64) - r, 0);
                        const uint32_t m = (uint32_t)__shfl((int)dv, owner, 64);
                        y.on = false;
                        if (ok) {
                            if constexpr (BYTE) {
                                // d(s,f) lies in [d(s,v) - L, d(s,v) + L]: residues decide
                                // when 2L + 1 <= 127, the exact distance otherwise
                                if (x.L <= 63) {
                                    const uint32_t bf = db[x.f];
                                    y.on = settled_b(bf) && (bf & 0x7Fu) == add127(m % 127u, x.L);
                                } else {
                                    y.on = D_(x.f) == m + x.L;
                                }
                            } else {
                                const uint32_t tf = D_(x.f);
                                y.on = tf != INF32 && tf == m + x.L;
                            }
                        }
                        y.t = y.on ? tsig[e] : 0ull;
                        y.cf = y.on ? S_(x.f) : 0ull;
                        return y;
                    },
                    [&](int owner, int64_t e, bool ok, int incl, int excl, int r, const IEnt& x, const IDel& y) {
                        double c = y.on ? (double)y.t * __longlong_as_double((long long)y.cf) : 0.0;
                        c = wseg_sum(c, y.seg);
                        const int ab = max(excl - r, 0), bb = min(incl - r, 64);
                        const double part = __shfl(c, max(bb - 1, 0), 64);
                        if (bb > ab) acc += part;
                    });
                if (valid && dv != INF32) cint[i] += (double)isig[i] * acc;
            }
        }
        __syncthreads();
    }
    if (ovf_flag && tid == 0) atomicOr(err, ERR_OVERFLOW);
    if (prof) {
        bytes = wsum_u64(bytes);
        if (lane == 0 && bytes) atomicAdd(prof, bytes);
    }
}

constexpr int IT = 256;  // threads of a k_interior block
constexpr int IU = 4;    // entries a thread has in flight

// The group of logical block lb of an interior launch, and the block's index within it:
// with a stride, every group owns `stride` consecutive blocks (those past its rows or
// nodes find nothing to do); without, groups own their blocks from blk0 (or tblk0 for
// the transpose) on, found by a binary search.
__device__ __forceinline__ void block_group(const IGroup* __restrict__ igs, int32_t nig, int64_t lb,
                                            int64_t stride, bool transpose, int32_t* g, int64_t* local) {
    if (stride > 0) {
        *g = (int32_t)(lb / stride);
        *local = lb - (int64_t)*g * stride;
        return;
    }
    int32_t glo = 0, ghi = nig - 1;
    while (glo < ghi) {
        const int32_t mid = (glo + ghi + 1) >> 1;
        if ((transpose ? igs[mid].tblk0 : igs[mid].blk0) <= lb)
            glo = mid;
        else
            ghi = mid - 1;
    }
    *g = glo;
    *local = lb - (transpose ? igs[glo].tblk0 : igs[glo].blk0);
}

// The saved rows of GF_ISPLIT groups, source-major as the resident kernel writes them
// (one source at a time, in full lines), node-major for k_interior: a block takes
// IT / lanes consecutive nodes of one group, thread j of a node its j-th source; reads
// run along nodes per source and writes along the block.
__global__ void __launch_bounds__(IT) k_itranspose(const IGroup* __restrict__ igs, int32_t nig, int64_t nblk,
                                                    int64_t stride) {
    const int64_t lb = blockIdx.x;
    int32_t glo;
    int64_t local;
    block_group(igs, nig, lb, stride, true, &glo, &local);
    const IGroup& G = igs[glo];
    const int P = G.lanes;
    const int t = threadIdx.x;
    const int j = t & (P - 1);
    const int64_t v = local * (IT / P) + t / P;
    if (v >= G.n || j >= G.nsrc) return;
    const int64_t i = (int64_t)j * G.n + v, o = v * P + j;
    const uint32_t d = gas(G.odist)[i];
    GAS IRec* a = gas(G.xa) + o;
    GAS IRec* c = gas(G.xb) + o;
    a->d = d;
    a->pad = 0u;
    a->x = gas(G.osig)[i];
    c->d = d;
    c->pad = 0u;
    c->x = gas(G.ocoef)[i];
}

// Interior rows of GF_ISPLIT groups (Sec. 5, Step 3, eq. localcentrality), after the
// groups' resident kernel. A block takes IT / lanes consecutive table rows of one group;
// a row takes `lanes` consecutive threads, thread j for the group's j-th source. Each
// thread sweeps its row's entries (f, d(f,v), sigma(f,v)) twice, in entry order: first
// for d(s,v), the least d(s,f) + d(f,v), and sigma(s,v), the sum of sigma(s,f) *
// sigma(f,v) over the f that attain it; then for the sum of sigma(f,v) * coef(s,f) over
// the f for which v lies on a shortest path from s to f (d(s,f) = d(s,v) + d(f,v)),
// which times sigma(s,v) is delta(s|v). The row's score is the sum of these over the
// group's sources, in source order, as the resident kernel would add them. A row's
// threads share its entry loads and read the saved values node-major (k_itranspose
// lays them out so), one line per node for all of them; each thread loads IU entries
// and then their saved values before it uses any, so that its loads overlap.
template <bool SHARE>
__global__ void __launch_bounds__(IT) k_interior(const IGroup* __restrict__ igs, int32_t nig, int64_t nblk,
                                                  int64_t stride, uint32_t* __restrict__ err) {
    // Blocks go to the 8 XCDs in turn by index; consecutive logical blocks (rows of one
    // group, reading the same saved rows) are kept on one XCD and so in one L2.
    const int64_t b = blockIdx.x;
    const int64_t per = nblk / 8, rem = nblk % 8, x = b % 8;
    const int64_t lb = (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + b / 8;
    int32_t glo;
    int64_t local;
    block_group(igs, nig, lb, stride, false, &glo, &local);
    const IGroup& G = igs[glo];
    const int P = G.lanes;
    const int t = threadIdx.x;
    const int j = t & (P - 1);
    const int32_t row = (int32_t)(local * (IT / P) + t / P);
    const bool act = row < G.tn && j < G.nsrc;
    const GAS int64_t* __restrict__ trow = gas(G.trow);
    const GAS int32_t* __restrict__ tcol = gas(G.tcol);
    const GAS uint32_t* __restrict__ tlen = gas(G.tlen);
    const GAS uint64_t* __restrict__ tsig = gas(G.tsig);
    uint32_t dmin = INF32;
    uint64_t ssum = 0;
    bool ovf = false;
    double acc = 0.0;
    const int base = (t & 63) & ~(P - 1);  // the row's first lane in the wave
    if (row < G.tn) {
        const int64_t e0 = trow[G.t_lo + row], e1 = trow[G.t_lo + row + 1];
        // this source's saved records, indexed by the graph's node id f: the record of
        // node f of the range sits at (f - lo) * P + j, so the bases are shifted by
        // lo * P records (in integer arithmetic: they may point before the arrays, and
        // only base + f * P is dereferenced), which saves a subtraction per record
        const uintptr_t sh = (uintptr_t)((int64_t)j - (int64_t)G.lo * P) * sizeof(IRec);
        const GAS IRec* __restrict__ xa = (const GAS IRec*)((uintptr_t)G.xa + sh);
        const GAS IRec* __restrict__ xb = (const GAS IRec*)((uintptr_t)G.xb + sh);
        // The row's entries in chunks of P: thread j loads entry j of the chunk, and the
        // row's threads pass them round with shuffles (every thread of the row runs the
        // same trip counts); then each thread loads its source's records for up to IU of
        // them before it uses any.
        for (int sweep = 0; sweep < 2; ++sweep) {
            if (sweep == 1 && __ballot(dmin != INF32 && act) == 0ull) break;
            const GAS IRec* __restrict__ xr = sweep == 0 ? xa : xb;
            // (SHARE: rows of at least IU threads; narrower rows' threads load IU entries
            // each themselves)
            const int CH = SHARE ? P : IU;
            for (int64_t c0 = e0; c0 < e1; c0 += CH) {
                const int64_t q = c0 + j;
                int32_t fj = 0;
                uint32_t Lj = 0u;
                uint64_t mj = 0ull;
                if (SHARE && q < e1) {
                    fj = tcol[q];
                    Lj = tlen[q];
                    mj = tsig[q];
                }
                const int cnt = (int)min<int64_t>(CH, e1 - c0);
                for (int u0 = 0; u0 < cnt; u0 += IU) {
                    int32_t f[IU];
                    uint32_t L[IU];
                    uint64_t m[IU];
                    IRec r[IU];
#pragma unroll
                    for (int k = 0; k < IU; ++k) {
                        if constexpr (SHARE) {
                            const int sl = base + min(u0 + k, cnt - 1);
                            f[k] = __shfl(fj, sl, 64);
                            L[k] = (uint32_t)__shfl((int)Lj, sl, 64);
                            m[k] = (uint64_t)__shfl((long long)mj, sl, 64);
                        } else {
                            const int64_t qk = c0 + min(u0 + k, cnt - 1);
                            f[k] = tcol[qk];
                            L[k] = tlen[qk];
                            m[k] = tsig[qk];
                        }
                    }
#pragma unroll
                    for (int k = 0; k < IU; ++k)
                        if (act) {
                            // one 16-byte load per record
                            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
                            const u32x4 w =
                                *reinterpret_cast<const GAS u32x4*>(xr + (int64_t)f[k] * P);
                            r[k].d = w.x;
                            r[k].x = ((uint64_t)w.w << 32) | w.z;
                        }
                    if (!act) continue;
#pragma unroll
                    for (int k = 0; k < IU; ++k) {
                        if (u0 + k >= cnt || r[k].d == INF32) continue;
                        if (sweep == 0) {
                            const uint32_t val = r[k].d + L[k];
                            if (val > dmin) continue;
                            const bool o = __umul64hi(r[k].x, m[k]) != 0ull;
                            const uint64_t pr = r[k].x * m[k];
                            if (val < dmin) {
                                dmin = val;
                                ssum = pr;
                                ovf = o;
                            } else {
                                ovf = ovf || o || ssum + pr < ssum;
                                ssum += pr;
                            }
                        } else if (dmin != INF32 && r[k].d == dmin + L[k]) {
                            acc += (double)m[k] * __longlong_as_double((long long)r[k].x);
                        }
                    }
                }
            }
        }
        if (act && dmin != INF32 && ovf) atomicOr(err, ERR_OVERFLOW);
    }
    const double c = (act && dmin != INF32) ? (double)ssum * acc : 0.0;
    // the row's sum over its sources, in source order (every lane of the wave takes part)
    double sum = 0.0;
    for (int jj = 0; jj < G.nsrc; ++jj) sum += __shfl(c, base + jj, 64);
    if (j == 0 && row < G.tn) gas(G.cint)[row] = sum;
}

// With the profiler on: the algorithmic bytes of the interior sweeps, 32 per (source,
// table entry), one thread per group (a count per wave of k_interior would make one
// device-wide atomic per wave).
__global__ void k_interior_bytes(const IGroup* __restrict__ igs, int32_t nig, unsigned long long* __restrict__ prof) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nig) return;
    const IGroup& G = igs[g];
    const int64_t ents = G.trow[G.t_lo + G.tn] - G.trow[G.t_lo];
    atomicAdd(prof, 32ull * (unsigned long long)G.nsrc * (unsigned long long)ents);
}

size_t lds_bytes(int64_t range) { return (((size_t)range * 4 + 15) & ~(size_t)15) + (size_t)range * 8; }
// LDS of the one-byte distance state (BYTE)
size_t byte_lds_bytes(int64_t range) { return ((size_t)range + 15) & ~(size_t)15; }
// The one-byte distance state for ranges beyond LDS: arcs at most 63 long (ring_len is
// the longest arc + 1) and one byte per node within LDS; BCPP_BYTE=0 switches it off.
bool byte_state_on() {
    const char* e = getenv("BCPP_BYTE");
    return !(e && strcmp(e, "0") == 0);
}

// Bucket bitmaps of a group: log2 of the bucket count for arcs up to ring_len - 1 long
// (at most 64 buckets), or -1 when the longest arc is unknown or too long.
int bucket_lg(int32_t ring_len) {
    if (ring_len < 2 || ring_len > 64) return -1;
    int lg = 0;
    while ((1 << lg) < ring_len) ++lg;
    return lg;
}
size_t bucket_bytes(int64_t range, int lg) {
    const size_t R2 = (size_t)1 << lg;
    return (R2 * (size_t)((range + 31) / 32) + 2 * R2) * 4;
}

struct ResidentLimits {
    bool init = false;
    size_t lds = 0;     // usable dynamic LDS per workgroup, state in LDS (classes 0-2)
    size_t lds_dev = 0;  // the same for the device-memory classes (3, 4: more static LDS)
};

ResidentLimits& limits() {
    static ResidentLimits L;
    return L;
}

int query_limits() {
    ResidentLimits& L = limits();
    if (L.init) return BC_OK;
    int dev = 0, v = 0;
    BC_HIP(hipGetDevice(&dev));
    BC_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // each instance: the device's LDS less its own static LDS (wave queues and step
    // variables, and for device-memory groups the per-wave count sums)
    const void* fns[5] = {(const void*)k_resident<1024, false, false>, (const void*)k_resident<512, false, false>,
                          (const void*)k_resident<256, false, false>, (const void*)k_resident<1024, true, false>,
                          (const void*)k_resident<1024, true, true>};
    size_t use[5];
    for (int i = 0; i < 5; ++i) {
        hipFuncAttributes fa;
        BC_HIP(hipFuncGetAttributes(&fa, fns[i]));
        const size_t stat = (size_t)fa.sharedSizeBytes + 256;
        use[i] = (size_t)v > stat ? (size_t)v - stat : 0;
        if (use[i] > 65536 &&
            hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)use[i]) != hipSuccess) {
            (void)hipGetLastError();
            use[i] = 65536 > stat ? 65536 - stat : 0;
        }
    }
    L.lds_dev = std::min(use[3], use[4]);
    const size_t usable = std::min({use[0], use[1], use[2]});
    L.lds = usable;
    L.init = true;
    return BC_OK;
}

// Launch shapes: the tuned table, or for a tuning sweep the environment overrides
// BCPP_TUNE_SMALL, BCPP_TUNE_MID (range thresholds of the 256- and 512-thread classes)
// and BCPP_TUNE_SPG_DIV (sources per group = ceil(|S| / div)).
int64_t tune_value(const char* name, int64_t dflt) {
    const char* e = getenv(name);
    if (!e || !*e) return dflt;
    const long long v = atoll(e);
    return v >= 0 ? (int64_t)v : dflt;
}
// The backward's tight-arc bitmap; BCPP_TIGHT=0 switches it off (every arc is tested).
// A range takes it with at least TIGHT_MIN_DEG arcs per node: on sparser ranges (the
// skeletons of graphs with small communities, 3 to 5 arcs per node) few arcs are
// skipped, and the forward's reverse-arc loads and marks cost more than that saves.
constexpr int64_t TIGHT_MIN_DEG = 6;
bool tight_arcs_on() {
    static const bool on = [] {
        const char* e = getenv("BCPP_TIGHT");
        return !(e && strcmp(e, "0") == 0);
    }();
    return on;
}
bool tight_pays(int64_t range, int64_t arcs) { return arcs > 0 && arcs >= TIGHT_MIN_DEG * range; }
struct SizeClasses {
    int64_t small = tune_value("BCPP_TUNE_SMALL", tuned_small_range);
    int64_t mid = tune_value("BCPP_TUNE_MID", tuned_mid_range);
    int64_t dense_shift = std::min<int64_t>(63, tune_value("BCPP_TUNE_DENSE_SHIFT", tuned_dense_shift));
    // Dijkstra_SK groups: each runs up to 64 sources of one part one after another, and
    // the launch lasts as long as its longest group, so larger parts take wider
    // workgroups sooner than scoring groups do
    int64_t dsk_small = tune_value("BCPP_TUNE_DSK_SMALL", tuned_dsk_small_range);
    int64_t dsk_mid = tune_value("BCPP_TUNE_DSK_MID", tuned_dsk_mid_range);
    int of(int64_t range, bool dsk) const {
        const int64_t a = dsk ? dsk_small : small, b = dsk ? dsk_mid : mid;
        return range <= a ? 0 : range <= b ? 1 : 2;
    }
};

}  // namespace

int64_t resident_max_range() {
    if (const char* e = getenv("BCPP_RESIDENT")) {
        if (strcmp(e, "0") == 0) return 0;
    }
    if (query_limits() != BC_OK) return 0;
    const size_t cap = limits().lds;
    int64_t n = (int64_t)(cap / 12);
    while (n > 0 && lds_bytes(n) > cap) --n;
    return n;
}

int32_t dsk_sources_per_group(int64_t part_work) {
    const int64_t budget = tune_value("BCPP_TUNE_DSK_WORK", tuned_dsk_group_work);
    if (budget <= 0 || part_work <= 0) return LANES;
    return (int32_t)std::min<int64_t>(LANES, std::max<int64_t>(8, budget / part_work));
}

int32_t resident_sources_per_group(int64_t nsrc) {
    const int64_t div = std::max<int64_t>(1, tune_value("BCPP_TUNE_SPG_DIV", tuned_spg_div));
    return (int32_t)std::min<int64_t>(LANES, std::max<int64_t>(1, (nsrc + div - 1) / div));
}

// Ints of a backward group's forward record: rec_arrays * T * ceil(range / T) for any
// T <= 1024 (the state is in device memory exactly when the range exceeds LDS).
size_t record_ints(int64_t range) {
    return (size_t)rec_arrays(range > resident_max_range()) * ((size_t)range + 1024) + 64;
}

bool resident_takes(int64_t range) {
    const char* e = getenv("BCPP_RESIDENT");
    if (e && strcmp(e, "0") == 0) return false;
    if (e && strcmp(e, "lds") == 0) return range <= resident_max_range();
    return query_limits() == BC_OK;
}

// A backward group whose state is in device memory keeps its tight-arc bitmap there.
static bool device_tight_bitmap(const GroupDesc& G) {
    return tight_arcs_on() && (G.flags & GF_BACKWARD) && tight_pays((int64_t)G.hi - G.lo, G.arcs) &&
           G.arcs < ((int64_t)1 << 31) - 64;
}

// Lanes of a table row in k_interior: a power of two >= nsrc.
static int32_t interior_lanes(int32_t nsrc) {
    int32_t P = 1;
    while (P < nsrc) P <<= 1;
    return P;
}
// The node-major saved records of a split group: {d, sigma} [range][P], then {d, coef}
// [range][P], each array starting on 256 bytes.
static size_t xsave_bytes(int64_t range, int32_t P) {
    const size_t c = (size_t)range * (size_t)P;
    return ((c * sizeof(IRec) + 255) & ~(size_t)255) * 2;
}

size_t resident_group_bytes(const GroupDesc& G) {
    const int64_t range = (int64_t)G.hi - G.lo;
    size_t b = ((size_t)range * 8 + 255) & ~(size_t)255;
    if (range > resident_max_range()) {
        b += (((size_t)range * 4 + 255) & ~(size_t)255) + (((size_t)range * 8 + 255) & ~(size_t)255);
        if (device_tight_bitmap(G)) b += ((size_t)((G.arcs + 31) / 32) * 4 + 255) & ~(size_t)255;
    }
    if ((G.flags & GF_CENT) && G.tn > 0)
        b += (((size_t)G.tn * 8 + 255) & ~(size_t)255) * 2 + (((size_t)G.tn * 4 + 255) & ~(size_t)255);
    if (G.flags & GF_BACKWARD)
        b += ((record_ints(range) * 4 + 255) & ~(size_t)255) + (((size_t)(range + 1) * 4 + 255) & ~(size_t)255);
    if (resident_interior_split(G)) {
        const size_t rows = (size_t)G.nsrc * (size_t)range;
        b += ((rows * 4 + 255) & ~(size_t)255) + ((rows * 8 + 255) & ~(size_t)255) * 2 +
             xsave_bytes(range, interior_lanes(G.nsrc));
    }
    return b + 256;
}

bool resident_interior_split(const GroupDesc& G) {
    const char* e = getenv("BCPP_ISPLIT");
    if (e && e[0] == '0') return false;
    if (!(G.flags & GF_CENT) || !(G.flags & GF_BACKWARD) || (G.flags & GF_RESTRICT) || G.tn <= 0) return false;
    // 4 sources or more, or many rows: a sweep per source then fills a whole launch
    // (BCPP_ISPLIT_MIN and BCPP_ISPLIT_ROWS set the two bounds, for the tuning sweeps)
    int32_t lo = 4;
    int64_t rows = 8192;
    if (const char* m = getenv("BCPP_ISPLIT_MIN")) lo = std::max(1, atoi(m));
    if (const char* r = getenv("BCPP_ISPLIT_ROWS")) rows = std::max<int64_t>(1, atoll(r));
    if (G.nsrc > 64 || (G.nsrc < lo && G.tn < rows)) return false;
    // saved rows: d (4 bytes), sigma and coef (8 each) per source and node, source-major,
    // and two 16-byte records per lane and node, node-major: at most 128 MiB
    return ((size_t)G.nsrc * 20 + (size_t)interior_lanes(G.nsrc) * 32) * (size_t)((int64_t)G.hi - G.lo) <=
           ((size_t)128 << 20);
}

bool resident_alloc(Arena& a, GroupDesc& G) {
    const int64_t range = (int64_t)G.hi - G.lo;
    G.cacc = a.take<double>((size_t)std::max<int64_t>(range, 1));
    if (!G.cacc) return false;
    if (range > resident_max_range()) {
        G.gdist = a.take<uint32_t>((size_t)range);
        G.gsig = a.take<uint64_t>((size_t)range);
        if (!G.gdist || !G.gsig) return false;
        if (device_tight_bitmap(G)) {
            G.gtb = a.take<uint32_t>((size_t)((G.arcs + 31) / 32));
            if (!G.gtb) return false;
        }
    }
    if (G.flags & GF_BACKWARD) {
        G.rlist = a.take<int32_t>(record_ints(range));
        G.steps = a.take<uint32_t>((size_t)range + 1);
        if (!G.rlist || !G.steps) return false;
    }
    if ((G.flags & GF_CENT) && G.tn > 0) {
        G.cint = a.take<double>((size_t)G.tn);
        G.dist = a.take<uint32_t>((size_t)G.tn);
        G.sigma = a.take<uint64_t>((size_t)G.tn);
        if (!G.cint || !G.dist || !G.sigma) return false;
    }
    // the saved rows of a split group (a GF_EXPORT caller's own d and sigma rows serve)
    G.flags &= ~(uint32_t)GF_ISPLIT;
    G.ocoef = nullptr;
    G.xsave = nullptr;
    if (!(G.flags & GF_EXPORT)) G.odist = nullptr, G.osig = nullptr;
    if (resident_interior_split(G)) {
        const size_t rows = (size_t)G.nsrc * (size_t)range;
        if (!(G.flags & GF_EXPORT)) {
            G.odist = a.take<uint32_t>(rows);
            G.osig = a.take<uint64_t>(rows);
        }
        G.ocoef = a.take<uint64_t>(rows);
        G.xsave = a.take<unsigned char>(xsave_bytes(range, interior_lanes(G.nsrc)));
        if (!G.odist || !G.osig || !G.ocoef || !G.xsave) return false;
        G.flags |= GF_ISPLIT;
    }
    return true;
}

size_t resident_launch_bytes(size_t ngroups) {
    // records, contexts and sources of up to five uploads, each rounded to 256 B
    return ngroups * (sizeof(RGroup) + sizeof(RCtx) + LANES * 4 + sizeof(IGroup)) + 9 * 256 + 512;
}

int resident_upload(hipStream_t s, Arena& a, const GroupDesc* const* groups, size_t ng, ResidentLaunch* L) {
    *L = ResidentLaunch();
    BC_TRY(query_limits());
    // one launch per size class; class 3 keeps its state in device memory, class 4 its
    // distance state as one byte per node in LDS and its path counts in device memory
    std::vector<RGroup> cls[5];
    std::vector<RCtx> ctx;
    std::vector<int32_t> src;
    std::vector<IGroup> ig, ig_narrow;  // rows of >= IU threads, and narrower
    int64_t ig_blocks = 0, ig_nblocks = 0, ig_tblocks = 0;
    std::map<std::pair<const void*, const void*>, int32_t> ctx_of;
    const SizeClasses sc;
    bool all_forward = ng > 0;
    for (size_t i = 0; i < ng; ++i) all_forward = all_forward && !(groups[i]->flags & GF_BACKWARD);
    L->kind = all_forward ? BC_K_DIJKSTRA_SK : BC_K_RESIDENT;
    for (size_t i = 0; i < ng; ++i) {
        const GroupDesc& G = *groups[i];
        const int64_t range = (int64_t)G.hi - G.lo;
        const size_t state = lds_bytes(range);
        const int lg0 = bucket_lg(G.ring_len);
        const size_t bb = lg0 >= 0 ? bucket_bytes(range, lg0) : 0;
        int c, lg = -1;
        int32_t tw = 0;
        size_t need;
        if (state > limits().lds) {
            if (!G.gdist || !G.gsig) return fail(BC_E_INVAL, "resident: no state buffers for a large range");
            if (G.gtb && G.g.twin && (G.flags & GF_BACKWARD) && G.arcs > 0) tw = (int32_t)((G.arcs + 31) / 32);
            if (byte_state_on() && G.ring_len >= 2 && G.ring_len <= 64 && byte_lds_bytes(range) <= limits().lds_dev) {
                c = 4;
                need = byte_lds_bytes(range);
            } else {
                c = 3;
                lg = (lg0 >= 0 && bb <= limits().lds_dev) ? lg0 : -1;
                need = lg >= 0 ? bb : 0;
            }
        } else {
            c = sc.of(range, !(G.flags & GF_BACKWARD));
            need = state;
            // the tight-arc bitmap, where it fits beside the state
            if (tight_arcs_on() && (G.flags & GF_BACKWARD) && G.g.twin && tight_pays(range, G.arcs)) {
                const int64_t words = (G.arcs + 31) / 32;
                if (state + (size_t)words * 4 <= limits().lds) {
                    tw = (int32_t)words;
                    need = state + (size_t)words * 4;
                }
            }
        }
        L->lds[c] = std::max(L->lds[c], need);
        const auto key = std::make_pair((const void*)G.g.row_ptr, (const void*)G.trow);
        auto it = ctx_of.find(key);
        if (it == ctx_of.end()) {
            it = ctx_of.emplace(key, (int32_t)ctx.size()).first;
            ctx.push_back(RCtx{G.g, G.trow, G.tcol, G.tlen, G.tsig});
        }
        RGroup r{};
        r.lg = lg;
        r.dense = (int32_t)(range >> sc.dense_shift);
        r.tw = tw;
        r.ctx = it->second;
        r.lo = G.lo;
        r.hi = G.hi;
        r.nsrc = G.nsrc;
        r.t_lo = G.t_lo;
        r.tn = G.tn;
        r.flags = G.flags;
        r.src_off = (int64_t)src.size();
        src.insert(src.end(), G.src, G.src + G.nsrc);
        r.cacc = G.cacc;
        r.cint = G.cint;
        r.idist = G.dist;
        r.isig = G.sigma;
        r.gdist = G.gdist;
        r.gsig = G.gsig;
        r.gtb = tw > 0 && c >= 3 ? G.gtb : nullptr;
        r.rlist = G.rlist;
        r.steps = G.steps;
        r.odist = G.odist;
        r.osig = G.osig;
        r.ocoef = G.ocoef;
        if ((G.flags & GF_EXPORT) && (!G.odist || !G.osig || !(G.flags & GF_BACKWARD)))
            return fail(BC_E_INVAL, "resident: export needs a backward group and output rows");
        if (G.flags & GF_ISPLIT) {
            if (!G.odist || !G.osig || !G.ocoef || !G.xsave || !G.cint || !(G.flags & GF_CENT) || G.tn <= 0 ||
                G.nsrc < 1 || G.nsrc > 64)
                return fail(BC_E_INVAL, "resident: split interior rows need saved rows and scores");
            IGroup q{};
            q.lo = G.lo;
            q.n = (int32_t)range;
            q.t_lo = G.t_lo;
            q.tn = G.tn;
            q.nsrc = G.nsrc;
            q.lanes = interior_lanes(G.nsrc);
            int64_t& nb = q.lanes >= IU ? ig_blocks : ig_nblocks;
            q.blk0 = nb;
            const size_t c = (size_t)range * (size_t)q.lanes;
            q.xa = reinterpret_cast<IRec*>(G.xsave);
            q.xb = reinterpret_cast<IRec*>(G.xsave + ((c * sizeof(IRec) + 255) & ~(size_t)255));
            q.trow = G.trow;
            q.tcol = G.tcol;
            q.tlen = G.tlen;
            q.tsig = G.tsig;
            q.odist = G.odist;
            q.osig = G.osig;
            q.ocoef = G.ocoef;
            q.cint = G.cint;
            nb += ((int64_t)G.tn + IT / q.lanes - 1) / (IT / q.lanes);
            (q.lanes >= IU ? ig : ig_narrow).push_back(q);
        }
        if ((G.flags & GF_BACKWARD) && (!G.rlist || !G.steps))
            return fail(BC_E_INVAL, "resident: no record buffers for a backward group");
        cls[c].push_back(r);
    }
    // largest groups first in each class: workgroups start in index order, so the
    // longest ones do not start last (each group's work is independent of its slot)
    for (auto& cv : cls)
        std::stable_sort(cv.begin(), cv.end(), [](const RGroup& x, const RGroup& y) {
            return (int64_t)x.nsrc * ((int64_t)x.hi - x.lo + x.tn) > (int64_t)y.nsrc * ((int64_t)y.hi - y.lo + y.tn);
        });
    L->d_err = a.take<uint32_t>(1);
    RCtx* d_ctx = a.take<RCtx>(std::max<size_t>(ctx.size(), 1));
    int32_t* d_src = a.take<int32_t>(std::max<size_t>(src.size(), 1));
    if (!L->d_err || !d_ctx || !d_src) return fail(BC_E_NOMEM, "resident: workspace too small");
    BC_TRY(zero_device(s, L->d_err, sizeof(uint32_t)));
    if (!ctx.empty()) BC_HIP(hipMemcpyAsync(d_ctx, ctx.data(), ctx.size() * sizeof(RCtx), hipMemcpyHostToDevice, s));
    if (!src.empty()) BC_HIP(hipMemcpyAsync(d_src, src.data(), src.size() * 4, hipMemcpyHostToDevice, s));
    L->d_ctx = d_ctx;
    L->d_src = d_src;
    for (int c = 0; c < 5; ++c) {
        L->count[c] = (int32_t)cls[c].size();
        if (cls[c].empty()) continue;
        L->d_rg[c] = a.take<RGroup>(cls[c].size());
        if (!L->d_rg[c]) return fail(BC_E_NOMEM, "resident: workspace too small");
        BC_HIP(hipMemcpyAsync(L->d_rg[c], cls[c].data(), cls[c].size() * sizeof(RGroup), hipMemcpyHostToDevice,
                              s));
    }
    if (!ig.empty() || !ig_narrow.empty()) {
        // one array, the narrow rows' groups last; the transpose's blocks over all of them
        const int32_t nwide = (int32_t)ig.size();
        ig.insert(ig.end(), ig_narrow.begin(), ig_narrow.end());
        for (IGroup& q : ig) {
            q.tblk0 = ig_tblocks;
            ig_tblocks += ((int64_t)q.n + IT / q.lanes - 1) / (IT / q.lanes);
        }
        if (ig_blocks >= ((int64_t)1 << 31) || ig_nblocks >= ((int64_t)1 << 31) || ig_tblocks >= ((int64_t)1 << 31))
            return fail(BC_E_INVAL, "resident: too many interior rows");
        // Each instance's grid: with a stride (every group owns as many blocks as the
        // largest needs) when that at most doubles the blocks, so that a block finds its
        // group by a division; else the blocks the groups need, found by a search.
        auto shape = [&](int32_t g0, int32_t g1, bool transpose, int64_t need, int64_t* grid, int64_t* stride) {
            int64_t mx = 0;
            for (int32_t g = g0; g < g1; ++g) {
                const IGroup& q = ig[g];
                const int64_t units = transpose ? (int64_t)q.n : (int64_t)q.tn;
                mx = std::max(mx, (units + IT / q.lanes - 1) / (IT / q.lanes));
            }
            const int64_t full = mx * (int64_t)(g1 - g0);
            *stride = (g1 > g0 && full <= 2 * need && full < ((int64_t)1 << 31)) ? mx : 0;
            *grid = *stride ? full : need;
        };
        shape(0, nwide, false, ig_blocks, &ig_blocks, &L->ig_wstride);
        shape(nwide, (int32_t)ig.size(), false, ig_nblocks, &ig_nblocks, &L->ig_nstride);
        shape(0, (int32_t)ig.size(), true, ig_tblocks, &ig_tblocks, &L->ig_tstride);
        IGroup* d_ig = a.take<IGroup>(ig.size());
        if (!d_ig) return fail(BC_E_NOMEM, "resident: workspace too small");
        BC_HIP(hipMemcpyAsync(d_ig, ig.data(), ig.size() * sizeof(IGroup), hipMemcpyHostToDevice, s));
        L->d_ig = d_ig;
        L->n_ig = (int32_t)ig.size();
        L->n_ig_wide = nwide;
        L->ig_blocks = ig_blocks;
        L->ig_nblocks = ig_nblocks;
        L->ig_tblocks = ig_tblocks;
    }
    return BC_OK;
}

int resident_upload(hipStream_t s, Arena& a, const std::vector<GroupDesc>& groups, ResidentLaunch* L) {
    std::vector<const GroupDesc*> ptr(groups.size());
    for (size_t i = 0; i < groups.size(); ++i) ptr[i] = &groups[i];
    return resident_upload(s, a, ptr.data(), ptr.size(), L);
}

static void launch_class(int c, hipStream_t s, const ResidentLaunch& L, unsigned long long* prof) {
    const dim3 grid((unsigned)L.count[c]);
    if (c == 4)
        hipLaunchKernelGGL((k_resident<1024, true, true>), grid, dim3(1024), L.lds[c], s, L.d_rg[c], L.d_ctx,
                           L.d_src, L.d_err, prof);
    else if (c == 3)
        hipLaunchKernelGGL((k_resident<1024, true, false>), grid, dim3(1024), L.lds[c], s, L.d_rg[c], L.d_ctx,
                           L.d_src, L.d_err, prof);
    else if (c == 2)
        hipLaunchKernelGGL((k_resident<1024, false, false>), grid, dim3(1024), L.lds[c], s, L.d_rg[c], L.d_ctx,
                           L.d_src, L.d_err, prof);
    else if (c == 1)
        hipLaunchKernelGGL((k_resident<512, false, false>), grid, dim3(512), L.lds[c], s, L.d_rg[c], L.d_ctx,
                           L.d_src, L.d_err, prof);
    else
        hipLaunchKernelGGL((k_resident<256, false, false>), grid, dim3(256), L.lds[c], s, L.d_rg[c], L.d_ctx,
                           L.d_src, L.d_err, prof);
}

// Streams and events on which the classes of a launch issued to stream s run side by
// side: one set per issuing stream, made on first use (default priority) and kept.
struct SideSet {
    hipStream_t st[5] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[5] = {};
};

static int side_set(hipStream_t s, SideSet** out) {
    static std::mutex mu;
    static std::map<std::pair<int, hipStream_t>, SideSet> sets;
    int dev = 0;
    BC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = sets.find({dev, s});
    if (it == sets.end()) {
        SideSet z;
        for (int c = 0; c < 5; ++c) {
            BC_HIP(hipStreamCreateWithFlags(&z.st[c], hipStreamNonBlocking));
            BC_HIP(hipEventCreateWithFlags(&z.join[c], hipEventDisableTiming));
        }
        BC_HIP(hipEventCreateWithFlags(&z.fork, hipEventDisableTiming));
        it = sets.emplace(std::make_pair(dev, s), z).first;
    }
    *out = &it->second;
    return BC_OK;
}

// The interior rows of the launch's GF_ISPLIT groups, after their resident kernels.
static int launch_interior(hipStream_t s, const ResidentLaunch& L) {
    if (L.n_ig == 0) return BC_OK;
    unsigned long long* prof =
        profiler().on && profiler().d_bytes ? profiler().d_bytes + BC_K_CENTRALITY : nullptr;
    KTimer kt(BC_K_CENTRALITY, s);
    hipLaunchKernelGGL(k_itranspose, dim3((unsigned)L.ig_tblocks), dim3(IT), 0, s, L.d_ig, L.n_ig, L.ig_tblocks,
                       L.ig_tstride);
    if (L.n_ig_wide > 0)
        hipLaunchKernelGGL(k_interior<true>, dim3((unsigned)L.ig_blocks), dim3(IT), 0, s, L.d_ig, L.n_ig_wide,
                           L.ig_blocks, L.ig_wstride, L.d_err);
    if (L.n_ig > L.n_ig_wide)
        hipLaunchKernelGGL(k_interior<false>, dim3((unsigned)L.ig_nblocks), dim3(IT), 0, s, L.d_ig + L.n_ig_wide,
                           L.n_ig - L.n_ig_wide, L.ig_nblocks, L.ig_nstride, L.d_err);
    if (prof) hipLaunchKernelGGL(k_interior_bytes, dim3((unsigned)((L.n_ig + 255) / 256)), dim3(256), 0, s, L.d_ig, L.n_ig, prof);
    BC_HIP(hipGetLastError());
    return BC_OK;
}

static int launch_classes(hipStream_t s, const ResidentLaunch& L);

int resident_launch(hipStream_t s, const ResidentLaunch& L) {
    BC_TRY(launch_classes(s, L));
    return launch_interior(s, L);
}

static int launch_classes(hipStream_t s, const ResidentLaunch& L) {
    unsigned long long* prof = profiler().on && profiler().d_bytes ? profiler().d_bytes + L.kind : nullptr;
    int ncls = 0;
    for (int c = 0; c < 5; ++c) ncls += L.count[c] > 0;
    if (ncls == 0) return BC_OK;
    KTimer kt(L.kind, s);
    if (ncls == 1) {
        for (int c = 0; c < 5; ++c)
            if (L.count[c]) launch_class(c, s, L, prof);
        BC_HIP(hipGetLastError());
        return BC_OK;
    }
    // several classes: each on a side stream, all after the work already on s, and s
    // waits for all of them (under capture these become parallel branches of the graph)
    SideSet* ss = nullptr;
    BC_TRY(side_set(s, &ss));
    BC_HIP(hipEventRecord(ss->fork, s));
    for (int c = 4; c >= 0; --c) {
        if (!L.count[c]) continue;
        BC_HIP(hipStreamWaitEvent(ss->st[c], ss->fork, 0));
        launch_class(c, ss->st[c], L, prof);
        BC_HIP(hipEventRecord(ss->join[c], ss->st[c]));
        BC_HIP(hipStreamWaitEvent(s, ss->join[c], 0));
    }
    BC_HIP(hipGetLastError());
    return BC_OK;
}

int run_resident(hipStream_t s, Arena& a, const GroupDesc* const* groups, size_t ng) {
    if (ng == 0) return BC_OK;
    ResidentLaunch L;
    BC_TRY(resident_upload(s, a, groups, ng, &L));
    BC_TRY(resident_launch(s, L));
    uint32_t herr = 0;
    BC_HIP(hipMemcpyAsync(&herr, L.d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    if (herr & ERR_OVERFLOW) return fail(BC_E_OVERFLOW, "a shortest-path count reached 2^64");
    return BC_OK;
}

int run_resident(hipStream_t s, Arena& a, const std::vector<GroupDesc>& groups) {
    std::vector<const GroupDesc*> ptr(groups.size());
    for (size_t i = 0; i < groups.size(); ++i) ptr[i] = &groups[i];
    return run_resident(s, a, ptr.data(), ptr.size());
}

}  // namespace bcpp
