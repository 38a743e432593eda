// Kernels and host driver of the multi-group Brandes engine (see engine.h).
//
// Layout. A group's state is row-major [node - lo][64]: the 64 lanes of a wave read
// one node's row for all 64 sources in one coalesced access, and every CSR arc the
// wave walks serves all 64 sources at once. Distances are uint32 (INF = all ones),
// path counts uint64 with overflow checks, dependency coefficients double.
//
// One engine iteration = select -> settle -> push -> backward -> centrality -> sched:
//   select  (grid over scan chunks) builds this iteration's work lists: forward groups
//           take the nodes whose pending distance nd equals the group's step D,
//           backward groups replay one recorded step, centrality groups list their
//           table rows;
//   settle  (persistent, wave per item) fixes sigma(s,v) of the lanes settled at D by
//           summing sigma(s,u) * mult(u,v) over tight parents u (eq. parentsall /
//           eq. multiparents; with GF_RESTRICT only non-frontier parents or the source
//           count, eq. frontierparents) and recomputes nd(v);
//   push    (persistent) relaxes the out-arcs of the settled lanes: tent(s,x) =
//           min(tent, D + len), nd(x) likewise;
//   backward(persistent) for the lanes at distance D:
//           delta = sigma(s,v) * sum over tight children x of mult * coef(s,x),
//           coef(s,v) = (I[v in S] + delta) / sigma(s,v) (eq. brandes / multibrandes),
//           and adds the lanes' delta (sources excluded) to the group's scores;
//   centrality (persistent) evaluates eq. localcentrality for interior nodes from the
//           skeleton state of the group's sources;
//   sched   (thread per group) records the step and moves the group to its next step
//           or phase.
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <thread>

namespace bcpp {

constexpr int WG = 256;           // threads per workgroup
constexpr int WAVES_PER_WG = WG / 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

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
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long t = (unsigned long long)__shfl_xor((long long)v, o, 64);
        v += t;
    }
    return v;
}

__device__ __forceinline__ int popc_below(unsigned long long mask, int lane) {
    return __popcll(mask & ((1ull << lane) - 1ull));
}

// ------------------------------------------------------------------ init -------

// Fill the state of the groups listed in `slots` (chunked like select, 4 positions x
// 64 lanes per pass of a workgroup). Sources start at distance 0 with one path.
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
        int64_t i = base + p;
        if (i < range) {
            const int32_t v = G.lo + (int32_t)i;
            const bool is_src = (mysrc == v);
            G.tent[i * 64 + lane] = is_src ? 0u : INF32;
            G.sigma[i * 64 + lane] = is_src ? 1ull : 0ull;
            if (G.coef) G.coef[i * 64 + lane] = 0.0;
            unsigned long long any = __ballot(is_src);
            if (lane == 0) {
                G.nd[i] = any ? 0u : INF32;
                if (G.cacc) G.cacc[i] = 0.0;
            }
        }
        if ((G.flags & GF_CENT) && i < G.tn && lane == 0) G.cint[i] = 0.0;
    }
}

// ---------------------------------------------------------------- select -------

// Append (g, y) for the lanes with sel set to work list `list` (wave-level compaction).
__device__ __forceinline__ void emit_items(int2* __restrict__ wl, int64_t wl_cap,
                                           uint32_t* __restrict__ ctr, int list, int g, bool sel,
                                           int32_t y) {
    const int lane = threadIdx.x & 63;
    const unsigned long long mask = __ballot(sel);
    if (mask == 0) return;
    const int cnt = __popcll(mask);
    uint32_t wbase = 0;
    if (lane == 0) wbase = atomicAdd(&ctr[list], (uint32_t)cnt);
    wbase = (uint32_t)__shfl((int)wbase, 0, 64);
    if (sel) wl[(int64_t)list * wl_cap + wbase + popc_below(mask, lane)] = make_int2(g, y);
}

__global__ void __launch_bounds__(WG) k_select(const GroupDesc* __restrict__ desc,
                                               GroupDyn* __restrict__ dyn,
                                               const int32_t* __restrict__ chunk_g,
                                               const int32_t* __restrict__ chunk_off,
                                               int64_t nchunks, int2* __restrict__ wl,
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
        const int32_t y = sel ? G.hist[off + i] : 0;
        emit_items(wl, wl_cap, ctr, 1, g, sel, y);
        return;
    }
    if (phase == PH_CENT) {
        emit_items(wl, wl_cap, ctr, 2, g, i < G.tn, G.t_lo + (int32_t)i);
        return;
    }
    // PH_FWD: the nodes whose smallest pending distance is the group's step D
    const int64_t range = (int64_t)G.hi - G.lo;
    const uint32_t D = dyn[g].D;
    const uint32_t pend = (i < range) ? G.nd[i] : INF32;
    const bool sel = (pend == D);
    const uint32_t other = wave_min_u32(sel ? INF32 : pend);
    if (lane == 0 && other != INF32) atomicMin(&dyn[g].nextmin, other);
    const int32_t y = G.lo + (int32_t)i;
    const unsigned long long mask = __ballot(sel);
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
    if (sel) {
        wl[wbase + rank] = make_int2(g, y);
        if (G.flags & GF_BACKWARD) {
            if ((int64_t)(hbase + rank) < G.hist_cap)
                G.hist[hbase + rank] = y;
            else
                atomicOr(&dyn[g].err, ERR_HIST);
        }
    }
}

// ---------------------------------------------------------------- settle -------

__global__ void __launch_bounds__(WG) k_settle(const GroupDesc* __restrict__ desc,
                                               GroupDyn* __restrict__ dyn,
                                               const int2* __restrict__ wl,
                                               const uint32_t* __restrict__ ctr,
                                               unsigned long long* __restrict__ prof) {
    const int lane = threadIdx.x & 63;
    const int64_t W = (int64_t)gridDim.x * WAVES_PER_WG;
    const uint32_t count = ctr[0];
    unsigned long long bytes = 0;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_WG + (threadIdx.x >> 6); it < count;
         it += W) {
        const int2 item = wl[it];
        const int g = item.x;
        const int32_t v = item.y;
        const GroupDesc& G = desc[g];
        const uint32_t D = dyn[g].D;
        const int64_t row = (int64_t)(v - G.lo);
        const uint32_t t = G.tent[row * 64 + lane];
        const int32_t mysrc = G.src[lane];
        const bool act = (t == D) && (mysrc != v);
        const bool restrict_parents = (G.flags & GF_RESTRICT) != 0;
        const int64_t e0 = G.g.row_ptr[v], e1 = G.g.row_ptr[v + 1];
        uint64_t sum = 0;
        bool ovf = false;
        int tight = 0;
        if (act) {
            for (int64_t e = e0; e < e1; ++e) {
                const int32_t u = G.g.col[e];
                const uint32_t L = G.g.len ? G.g.len[e] : 1u;
                if (L > D) continue;
                const int64_t ur = (int64_t)(u - G.lo);
                const uint32_t tu = G.tent[ur * 64 + lane];
                if (tu != D - L) continue;
                if (restrict_parents && u != mysrc && G.g.nflag &&
                    (G.g.nflag[u] & NF_BLOCKED))
                    continue;
                uint64_t s = G.sigma[ur * 64 + lane];
                if (G.g.mult) {
                    const uint64_t m = G.g.mult[e];
                    if (__umul64hi(s, m) != 0) ovf = true;
                    s *= m;
                }
                const uint64_t r = sum + s;
                if (r < sum) ovf = true;
                sum = r;
                ++tight;
            }
            G.sigma[row * 64 + lane] = sum;
        }
        if (__ballot(ovf) && lane == 0) atomicOr(&dyn[g].err, ERR_OVERFLOW);
        const uint32_t pend = wave_min_u32(t > D ? t : INF32);
        if (lane == 0) {
            G.nd[row] = pend;
            if (pend != INF32) atomicMin(&dyn[g].nextmin, pend);
        }
        if (prof) {
            // algorithmic bytes: per settled lane, one distance per arc, a count per
            // tight parent, the count written; per item the CSR row once
            const unsigned long long deg = (unsigned long long)(e1 - e0);
            unsigned long long mine = act ? (4ull * deg + 8ull * (unsigned)tight + 8ull) : 0ull;
            mine = wave_sum_u64(mine);
            bytes += mine + 16ull + deg * (4ull + (G.g.len ? 4ull : 0ull) +
                                           (G.g.mult ? 8ull : 0ull));
        }
    }
    if (prof && lane == 0 && bytes) atomicAdd(&prof[BC_K_SETTLE], bytes);
}

// ------------------------------------------------------------------ push -------

__global__ void __launch_bounds__(WG) k_push(const GroupDesc* __restrict__ desc,
                                             GroupDyn* __restrict__ dyn,
                                             const int2* __restrict__ wl,
                                             const uint32_t* __restrict__ ctr,
                                             unsigned long long* __restrict__ prof) {
    const int lane = threadIdx.x & 63;
    const int64_t W = (int64_t)gridDim.x * WAVES_PER_WG;
    const uint32_t count = ctr[0];
    unsigned long long bytes = 0;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_WG + (threadIdx.x >> 6); it < count;
         it += W) {
        const int2 item = wl[it];
        const int g = item.x;
        const int32_t v = item.y;
        const GroupDesc& G = desc[g];
        const uint32_t D = dyn[g].D;
        const int64_t row = (int64_t)(v - G.lo);
        const bool act = G.tent[row * 64 + lane] == D;
        const bool unit = (G.flags & GF_UNIT) != 0;
        const int64_t e0 = G.g.row_ptr[v], e1 = G.g.row_ptr[v + 1];
        uint32_t best = INF32;
        for (int64_t e = e0; e < e1; ++e) {
            const int32_t u = G.g.col[e];
            const uint32_t L = G.g.len ? G.g.len[e] : 1u;
            const uint32_t nv = D + L;
            const int64_t ur = (int64_t)(u - G.lo);
            bool improved = false;
            if (act) {
                uint32_t* p = &G.tent[ur * 64 + lane];
                const uint32_t cur = *p;
                if (cur > nv) {
                    if (unit) {
                        *p = nv;  // every writer of this step stores the same D + 1
                        improved = true;
                    } else {
                        improved = atomicMin(p, nv) > nv;
                    }
                }
            }
            if (__ballot(improved)) {
                if (lane == 0) {
                    if (unit) {
                        if (G.nd[ur] > nv) G.nd[ur] = nv;
                    } else {
                        atomicMin(&G.nd[ur], nv);
                    }
                }
                best = min(best, nv);
            }
        }
        if (lane == 0 && best != INF32) atomicMin(&dyn[g].nextmin, best);
        if (prof) {
            const unsigned long long deg = (unsigned long long)(e1 - e0);
            unsigned long long mine = act ? 4ull * deg : 0ull;
            mine = wave_sum_u64(mine);
            bytes += mine + 16ull + deg * (4ull + (G.g.len ? 4ull : 0ull));
        }
    }
    if (prof && lane == 0 && bytes) atomicAdd(&prof[BC_K_PUSH], bytes);
}

// -------------------------------------------------------------- backward -------

__global__ void __launch_bounds__(WG) k_backward(const GroupDesc* __restrict__ desc,
                                                 GroupDyn* __restrict__ dyn,
                                                 const int2* __restrict__ wl,
                                                 int64_t wl_cap,
                                                 const uint32_t* __restrict__ ctr,
                                                 unsigned long long* __restrict__ prof) {
    const int lane = threadIdx.x & 63;
    const int64_t W = (int64_t)gridDim.x * WAVES_PER_WG;
    const uint32_t count = ctr[1];
    const int2* list = wl + wl_cap;
    unsigned long long bytes = 0;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_WG + (threadIdx.x >> 6); it < count;
         it += W) {
        const int2 item = list[it];
        const int g = item.x;
        const int32_t v = item.y;
        const GroupDesc& G = desc[g];
        const uint32_t D = dyn[g].D;
        const int64_t row = (int64_t)(v - G.lo);
        const uint32_t t = G.tent[row * 64 + lane];
        const bool act = (t == D) && (G.src[lane] != v);
        const int64_t e0 = G.g.row_ptr[v], e1 = G.g.row_ptr[v + 1];
        double delta = 0.0;
        int kids = 0;
        if (act) {
            double acc = 0.0;
            for (int64_t e = e0; e < e1; ++e) {
                const int32_t u = G.g.col[e];
                const uint32_t L = G.g.len ? G.g.len[e] : 1u;
                const int64_t ur = (int64_t)(u - G.lo);
                const uint32_t tu = G.tent[ur * 64 + lane];
                if (tu != D + L) continue;
                const double c = G.coef[ur * 64 + lane];
                acc += G.g.mult ? (double)G.g.mult[e] * c : c;
                ++kids;
            }
            const double sg = (double)G.sigma[row * 64 + lane];
            delta = sg * acc;
            const double ind = (G.g.nflag && (G.g.nflag[v] & NF_TARGET)) ? 1.0 : 0.0;
            G.coef[row * 64 + lane] = (ind + delta) / sg;
        }
        const double tot = wave_sum_f64(delta);
        if (lane == 0 && G.cacc) G.cacc[row] += tot;
        if (prof) {
            const unsigned long long deg = (unsigned long long)(e1 - e0);
            unsigned long long mine =
                act ? (4ull * deg + 8ull * (unsigned)kids + 8ull + 8ull) : 0ull;
            mine = wave_sum_u64(mine);
            bytes += mine + 16ull + 8ull +
                     deg * (4ull + (G.g.len ? 4ull : 0ull) + (G.g.mult ? 8ull : 0ull));
        }
    }
    if (prof && lane == 0 && bytes) atomicAdd(&prof[BC_K_BACKWARD], bytes);
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
                                                   const int2* __restrict__ wl,
                                                   int64_t wl_cap,
                                                   const uint32_t* __restrict__ ctr,
                                                   unsigned long long* __restrict__ prof) {
    const int lane = threadIdx.x & 63;
    const int64_t W = (int64_t)gridDim.x * WAVES_PER_WG;
    const uint32_t count = ctr[2];
    const int2* list = wl + 2 * wl_cap;
    unsigned long long bytes = 0;
    for (int64_t it = (int64_t)blockIdx.x * WAVES_PER_WG + (threadIdx.x >> 6); it < count;
         it += W) {
        const int2 item = list[it];
        const int g = item.x;
        const int32_t i = item.y;
        const GroupDesc& G = desc[g];
        const int64_t e0 = G.trow[i], e1 = G.trow[i + 1];
        uint32_t dv = INF32;
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t fr = (int64_t)(G.tcol[e] - G.lo);
            const uint32_t tf = G.tent[fr * 64 + lane];
            if (tf != INF32) dv = min(dv, tf + G.tlen[e]);
        }
        double delta = 0.0;
        bool ovf = false;
        if (dv != INF32) {
            uint64_t sv = 0;
            double acc = 0.0;
            for (int64_t e = e0; e < e1; ++e) {
                const int64_t fr = (int64_t)(G.tcol[e] - G.lo);
                const uint32_t tf = G.tent[fr * 64 + lane];
                if (tf == INF32) continue;
                const uint32_t L = G.tlen[e];
                if (tf + L == dv) {
                    const uint64_t a = G.sigma[fr * 64 + lane];
                    const uint64_t b = G.tsig[e];
                    if (__umul64hi(a, b) != 0) ovf = true;
                    const uint64_t p = a * b;
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
        for (int32_t g = a; g < b; ++g) s += parts[g][i];
    }
    s *= scale;
    out[v] = accumulate ? out[v] + s : s;
}

// ==================================================================== host ======

size_t group_bytes(int64_t range, int32_t nsrc, uint32_t flags, int64_t max_steps, int32_t tn) {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    size_t b = 0;
    b += al(range * 64 * 4);  // tent
    b += al(range * 64 * 8);  // sigma
    b += al(range * 4);       // nd
    if (flags & GF_BACKWARD) {
        b += al(range * 64 * 8);  // coef
        b += al(range * 8);       // cacc
        b += al(range * (int64_t)std::max(nsrc, 1) * 4);  // history
        b += al(max_steps * 4) + al(max_steps * 8) + al(max_steps * 4);
    }
    if (flags & GF_CENT) b += al((size_t)tn * 8);
    return b;
}

bool group_alloc(Arena& a, GroupDesc& G, int64_t max_steps) {
    const int64_t range = (int64_t)G.hi - G.lo;
    G.tent = a.take<uint32_t>(range * 64);
    G.sigma = a.take<uint64_t>(range * 64);
    G.nd = a.take<uint32_t>(range);
    if (!G.tent || !G.sigma || !G.nd) return false;
    if (G.flags & GF_BACKWARD) {
        G.coef = a.take<double>(range * 64);
        G.cacc = a.take<double>(range);
        G.hist_cap = range * (int64_t)std::max(G.nsrc, 1);
        G.hist = a.take<int32_t>(G.hist_cap);
        G.rec_cap = (int32_t)std::min<int64_t>(max_steps, INT32_MAX);
        G.rec_d = a.take<uint32_t>(G.rec_cap);
        G.rec_off = a.take<int64_t>(G.rec_cap);
        G.rec_cnt = a.take<int32_t>(G.rec_cap);
        if (!G.coef || !G.cacc || !G.hist || !G.rec_d || !G.rec_off || !G.rec_cnt)
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
    return (size_t)slots * (sizeof(GroupDesc) + sizeof(GroupDyn) + 512) + (size_t)chunks * 8 +
           (size_t)chunks * WG * 3 * sizeof(int2) + 8192;
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
    d_wl = a.take<int2>(3 * wl_cap);
    d_ctr = a.take<uint32_t>(8);
    if (!d_desc || !d_dyn || !d_chunk_g || !d_chunk_off || !d_wl || !d_ctr)
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
    uint32_t add = (uint32_t)n;
    // active += n (host-side read-modify-write: the engine is idle here)
    BC_HIP(hipMemcpyAsync(h_ctr, d_ctr, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    BC_HIP(hipStreamSynchronize(stream));
    h_ctr[3] += add;
    BC_HIP(hipMemcpyAsync(d_ctr + 3, h_ctr + 3, sizeof(uint32_t), hipMemcpyHostToDevice, stream));
    BC_HIP(hipStreamSynchronize(stream));
    return BC_OK;
}

int Engine::iterate(int iters) {
    const bool dbg = getenv("BCPP_DEBUG") != nullptr;
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
        if (dbg) {
            GroupDyn d0;
            BC_HIP(hipMemcpy(&d0, d_dyn, sizeof(d0), hipMemcpyDeviceToHost));
            fprintf(stderr, "iter: g0 phase %d D %u nrec %d rec_i %d\n", d0.phase, d0.D, d0.nrec, d0.rec_i);
        }
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
    std::vector<GroupDyn> dy(nslots);
    BC_HIP(hipMemcpyAsync(dy.data(), d_dyn, sizeof(GroupDyn) * nslots, hipMemcpyDeviceToHost, stream));
    BC_HIP(hipStreamSynchronize(stream));
    uint32_t err = 0;
    for (auto& d : dy) err |= d.err;
    if (getenv("BCPP_DEBUG")) {
        fprintf(stderr, "engine: %d slots done\n", nslots);
        for (int32_t g = 0; g < nslots && g < 8; ++g)
            fprintf(stderr, "  group %d: phase %d D %u nrec %d rec_i %d hist %lld err %u\n", g,
                    dy[g].phase, dy[g].D, dy[g].nrec, dy[g].rec_i, (long long)dy[g].hist_len,
                    dy[g].err);
    }
    if (dyn_out) *dyn_out = dy;
    if (err & ERR_OVERFLOW) return fail(BC_E_OVERFLOW, "a shortest-path count reached 2^64");
    if (err & (ERR_HIST | ERR_REC)) return fail(BC_E_DEVICE, "engine: history capacity exceeded");
    return BC_OK;
}

int run_groups(Arena& a, hipStream_t s, std::vector<GroupDesc>& groups, int64_t max_steps) {
    if (groups.empty()) return BC_OK;
    int64_t positions = 0;
    for (auto& G : groups) {
        if (!group_alloc(a, G, max_steps)) return fail(BC_E_NOMEM, "engine: group state does not fit");
        positions += std::max<int64_t>((int64_t)G.hi - G.lo, (G.flags & GF_CENT) ? G.tn : 0);
    }
    Engine E;
    BC_TRY(E.setup(a, s, (int32_t)groups.size(), positions));
    BC_TRY(E.install(groups.data(), 0, (int32_t)groups.size()));
    std::vector<int32_t> live(groups.size());
    for (size_t i = 0; i < live.size(); ++i) live[i] = (int32_t)i;
    BC_TRY(E.set_chunks(groups, live));
    int rc = E.run_to_completion((int32_t)groups.size());
    if (E.h_ctr) (void)hipHostFree(E.h_ctr);
    return rc;
}

int reduce_scores(hipStream_t s, Arena& a, const std::vector<GroupDesc>& groups, int32_t n,
                  const int32_t* d_g0, const int32_t* d_g1, const int32_t* d_idx,
                  const uint8_t* d_which, double scale, double* out_dev, bool accumulate) {
    if (n <= 0) return BC_OK;
    const size_t ng = std::max<size_t>(groups.size(), 1);
    std::vector<const double*> pc(ng, nullptr), pi(ng, nullptr);
    for (size_t g = 0; g < groups.size(); ++g) {
        pc[g] = groups[g].cacc;
        pi[g] = groups[g].cint;
    }
    const double** d_pc = a.take<const double*>(ng);
    const double** d_pi = a.take<const double*>(ng);
    if (!d_pc || !d_pi) return fail(BC_E_NOMEM, "reduce: workspace too small");
    BC_HIP(hipMemcpyAsync(d_pc, pc.data(), ng * sizeof(void*), hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(d_pi, pi.data(), ng * sizeof(void*), hipMemcpyHostToDevice, s));
    {
        KTimer kt(BC_K_OTHER, s);
        hipLaunchKernelGGL(k_reduce, dim3((n + 255) / 256), dim3(256), 0, s, d_pc, d_pi, n, d_g0,
                           d_g1, d_idx, d_which, 0, (int32_t)groups.size(), scale,
                           accumulate ? 1 : 0, out_dev);
    }
    BC_HIP(hipGetLastError());
    BC_HIP(hipStreamSynchronize(s));
    return BC_OK;
}

}  // namespace bcpp
