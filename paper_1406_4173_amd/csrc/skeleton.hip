// Brandes++ (Sec. 5, Alg. 1): Build_SK with the target-singleton partition P',
// Dijkstra_SK over every part on the device, skeleton assembly, Brandes_SK with the
// fused Centrality pass, and the skeleton inspection entry points.
//
// Node order. The nodes of G are renumbered so that every part of P' is contiguous and
// its frontier nodes come first (each class in increasing original id). The skeleton
// node ids are then the frontier nodes in that order, so the frontier of part p is the
// id range [fbase[p], fbase[p] + |F_p|) and a frontier's local index inside its part's
// node range is its offset in that range.
#include <algorithm>
#include <memory>
#include <numeric>


#include "engine.h"
#include "graph.h"
#include "skbuild.h"

namespace bcpp {

// -------------------------------------------------------------- assembly -------

// Clique arcs out of each source f: one per frontier q != f of its part with
// sigma(f,q) > 0 (zero-multiplicity pairs carry no shortest path and are dropped).
// One workgroup of 256 threads per Dijkstra_SK group, whose states are rows
// [frontier j][64 source lanes]: the four waves split the rows, each lane counting for
// its source, and the per-wave counts are summed in LDS.
__global__ void __launch_bounds__(256) k_clique_count(const GroupDesc* __restrict__ desc,
                                                      const DskInfo* __restrict__ info, int32_t ngroups,
                                                      int32_t* __restrict__ cdeg) {
    __shared__ int32_t part[4][64];
    const int g = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const DskInfo I = info[g];
    const uint64_t* __restrict__ sig = desc[g].sigma;
    const int32_t own = I.fl0 + lane;
    int32_t cnt = 0;
    if (lane < I.nsrc)
        for (int32_t j = wave; j < I.nf; j += 4) cnt += (j != own && sig[(int64_t)j * 64 + lane] != 0) ? 1 : 0;
    part[wave][lane] = cnt;
    __syncthreads();
    if (wave == 0 && lane < I.nsrc) cdeg[I.sk_base + own] = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
}

// The arcs themselves, in increasing frontier order after the row's cut arcs. The
// workgroup stages 64 rows of sigma and d at a time in LDS (rows padded to 65 entries
// so that reading one source's column is free of bank conflicts); then each wave takes
// one source's column at a time, keeps the non-zero entries with a ballot and writes
// them to that source's row with consecutive lanes at consecutive positions.
__global__ void __launch_bounds__(256) k_clique_fill(const GroupDesc* __restrict__ desc,
                                                     const DskInfo* __restrict__ info, int32_t ngroups,
                                                     const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ rdeg, int32_t* __restrict__ col,
                                                     uint32_t* __restrict__ len, uint64_t* __restrict__ mult,
                                                     uint32_t* __restrict__ maxlen) {
    __shared__ uint64_t ts[64][65];
    __shared__ uint32_t td[64][65];
    __shared__ int64_t pos[64];
    __shared__ uint32_t bmax;
    const int g = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const DskInfo I = info[g];
    const GroupDesc& G = desc[g];
    if (wave == 0 && lane < I.nsrc) {
        const int32_t f = I.sk_base + I.fl0 + lane;
        pos[lane] = row_ptr[f] + rdeg[f];
    }
    if (threadIdx.x == 0) bmax = 0u;
    uint32_t mx = 0;
    for (int32_t j0 = 0; j0 < I.nf; j0 += 64) {
        __syncthreads();  // pos and bmax set; the previous tile fully read
        for (int r = wave; r < 64; r += 4) {
            const int32_t j = j0 + r;
            uint64_t sv = 0;
            uint32_t dv = 0;
            if (j < I.nf && lane < I.nsrc) {
                sv = G.sigma[(int64_t)j * 64 + lane];
                dv = G.dist[(int64_t)j * 64 + lane];
            }
            ts[r][lane] = sv;
            td[r][lane] = dv;
        }
        __syncthreads();
        for (int32_t src = wave; src < I.nsrc; src += 4) {
            const int32_t j = j0 + lane;
            const uint64_t sv = ts[lane][src];
            const bool keep = j < I.nf && j != I.fl0 + src && sv != 0;
            const unsigned long long m = __ballot(keep);
            if (keep) {
                const int64_t at = pos[src] + __popcll(m & ((1ull << lane) - 1ull));
                const uint32_t d = td[lane][src];
                col[at] = I.sk_base + j;
                len[at] = d;
                mult[at] = sv;
                mx = max(mx, d);
            }
            if (lane == 0) pos[src] += __popcll(m);
        }
    }
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    if (lane == 0 && mx) atomicMax(&bmax, mx);
    __syncthreads();
    if (threadIdx.x == 0 && bmax) atomicMax(maxlen, bmax);
}

// Row lengths of the skeleton (cut arcs, then clique arcs) and of the interior
// table, each with a trailing zero so that an exclusive scan ends on the total.
__global__ void k_row_lengths(int32_t nsk, int32_t nint, const int32_t* __restrict__ rdeg,
                              const int32_t* __restrict__ cdeg, const int32_t* __restrict__ tdeg,
                              int64_t* __restrict__ slen, int64_t* __restrict__ tlen) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= nsk) slen[i] = i < nsk ? (int64_t)rdeg[i] + cdeg[i] : 0;
    if (i <= nint) tlen[i] = (i < nint && tdeg) ? (int64_t)tdeg[i] : 0;
}

// Cut arcs R with tuple <w(e), 1>, placed first in each skeleton row.
__global__ void k_fill_r(int32_t nsk, const int64_t* __restrict__ rptr, const int32_t* __restrict__ rcol,
                         const uint32_t* __restrict__ rw, const int64_t* __restrict__ row_ptr,
                         int32_t* __restrict__ col, uint32_t* __restrict__ len,
                         uint64_t* __restrict__ mult) {
    const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nsk) return;
    int64_t pos = row_ptr[f];
    for (int64_t e = rptr[f]; e < rptr[f + 1]; ++e, ++pos) {
        col[pos] = rcol[e];
        len[pos] = rw[e];
        mult[pos] = 1;
    }
}

// Reverse arc of every skeleton arc. A row is [cut arcs][clique arcs], each segment
// sorted by skeleton id, so the twin of f->q is found by bisection in q's segments.
__global__ void k_sk_twin(int32_t nsk, const int64_t* __restrict__ row_ptr,
                          const int32_t* __restrict__ rdeg, const int32_t* __restrict__ col,
                          int64_t* __restrict__ twin) {
    const int32_t f = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (f >= nsk) return;
    for (int64_t e = row_ptr[f] + lane; e < row_ptr[f + 1]; e += 64) {
        const int32_t q = col[e];
        int64_t lo = row_ptr[q], mid_end = row_ptr[q] + rdeg[q], hi = row_ptr[q + 1];
        int64_t found = -1;
        for (int seg = 0; seg < 2 && found < 0; ++seg) {
            int64_t a = seg ? mid_end : lo, b = seg ? hi : mid_end;
            while (a < b) {
                const int64_t m = (a + b) >> 1;
                if (col[m] < f) a = m + 1; else b = m;
            }
            if (a < (seg ? hi : mid_end) && col[a] == f) found = a;
        }
        twin[e] = found;
    }
}

// Packed arc records {head, length, reverse arc, multiplicity} of the skeleton's m
// arcs; *big is set if a multiplicity does not fit 32 bits (then the records are not
// used).
__global__ void k_pack_arcs(int64_t m, const int32_t* __restrict__ col, const uint32_t* __restrict__ len,
                            const int64_t* __restrict__ twin, const uint64_t* __restrict__ mult,
                            ArcRec* __restrict__ arc, uint32_t* __restrict__ big) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint64_t mu = mult[e];
    if (mu > 0xFFFFFFFFull) atomicOr(big, 1u);
    arc[e] = ArcRec{(uint32_t)col[e], len[e], (uint32_t)twin[e], (uint32_t)mu};
}

// Table rows of interior nodes: entries (f, d(f,v), sigma(f,v)) over the part's
// frontier f with sigma > 0, in frontier order. Wave per interior row.
__global__ void k_table(const GroupDesc* __restrict__ desc, const DskInfo* __restrict__ info,
                        int32_t nint, const int32_t* __restrict__ int_local,
                        const int32_t* __restrict__ int_g0, const int32_t* __restrict__ int_ng,
                        int32_t* __restrict__ tdeg, const int64_t* __restrict__ trow,
                        int32_t* __restrict__ tcol, uint32_t* __restrict__ tlen,
                        uint64_t* __restrict__ tsig) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= nint) return;
    const int64_t local = int_local[i];
    const int32_t g0 = int_g0[i], ng = int_ng[i];
    int64_t pos = trow ? trow[i] : 0;
    int32_t cnt = 0;
    for (int32_t c = 0; c < ng; ++c) {
        const int32_t g = g0 + c;
        const DskInfo I = info[g];
        const GroupDesc& G = desc[g];
        uint64_t s = 0;
        uint32_t d = 0;
        if (lane < I.nsrc) {
            s = G.sigma[local * 64 + lane];
            d = G.dist[local * 64 + lane];
        }
        const bool keep = s != 0;
        const unsigned long long m = __ballot(keep);
        if (trow && keep) {
            const int64_t at = pos + cnt + __popcll(m & ((1ull << lane) - 1ull));
            tcol[at] = I.sk_base + I.fl0 + lane;
            tlen[at] = d;
            tsig[at] = s;
        }
        cnt += __popcll(m);
    }
    if (!trow && lane == 0) tdeg[i] = cnt;
}

// ------------------------------------------------------------ partition_sk -----

// Phase 1: P' labels (targets become singleton parts k + i, Sec. 5 "Target nodes in
// the skeleton"), target flags, frontier flags (a neighbour in another part, Sec. 4),
// and per part of P' its size, frontier count and intra-part arc count.
__global__ void k_p1_labels(int32_t n, const int32_t* __restrict__ part, int32_t* __restrict__ lab,
                            uint8_t* __restrict__ ist) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    lab[v] = part[v];
    ist[v] = 0;
}

__global__ void k_p1_targets(int32_t nS, const int32_t* __restrict__ S, int32_t k, int given,
                             int32_t* __restrict__ lab, uint8_t* __restrict__ ist) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nS) return;
    if (!given) lab[S[i]] = k + i;
    ist[S[i]] = 1;
}

__global__ void k_p1_frontier(int32_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                              const int32_t* __restrict__ lab, uint8_t* __restrict__ fr,
                              int32_t* __restrict__ psize, int32_t* __restrict__ pnf,
                              unsigned long long* __restrict__ parc, unsigned long long* __restrict__ ncross) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long cross = 0;
    if (v < n) {
        const int32_t p = lab[v];
        unsigned long long intra = 0;
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            if (lab[col[e]] == p)
                ++intra;
            else
                ++cross;
        }
        fr[v] = cross ? 1 : 0;
        atomicAdd(&psize[p], 1);
        if (cross) atomicAdd(&pnf[p], 1);
        if (intra) atomicAdd(&parc[p], intra);
    }
    for (int o = 32; o > 0; o >>= 1) cross += (unsigned long long)__shfl_xor((long long)cross, o, 64);
    if ((threadIdx.x & 63) == 0 && cross) atomicAdd(ncross, cross);
}

// Phase 2: renumbering key (part, then frontier before interior; ties keep node order
// in the stable sort) and the inverse map. Labels are below 2^31, so keys fit 32 bits.
__global__ void k_p2_keys(int32_t n, const int32_t* __restrict__ lab, const uint8_t* __restrict__ fr,
                          uint32_t* __restrict__ key, int32_t* __restrict__ val) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    key[v] = (uint32_t)lab[v] * 2u + (fr[v] ? 0u : 1u);
    val[v] = (int32_t)v;
}

// Stable LSD radix sort of (key, value) pairs, 8 key bits per pass, in tiles of
// RS_TILE consecutive items (one workgroup of 256 threads, RS_TILE / 256 rounds of 256
// consecutive items). k_rs_hist counts each tile's digits into hist[digit * ntiles +
// tile]; an exclusive scan of hist gives every (digit, tile) its first output slot;
// k_rs_scatter then places the tile's items in order. Within a round, lanes of one
// wave with equal digits are found with one ballot per digit bit and ranked by lane;
// per-wave counts in LDS order the waves, and a running count per digit orders the
// rounds, so equal keys keep their input order. It uses no library scratch that must
// be cleared beforehand, so a captured graph can replay it.
constexpr int RS_TILE = 1024;

__global__ void k_rs_hist(int32_t n, const uint32_t* __restrict__ key, int shift, int32_t ntiles,
                          int32_t* __restrict__ hist) {
    __shared__ int32_t c[256];
    c[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_TILE / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        if (i < n) atomicAdd(&c[(key[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = c[threadIdx.x];
}

__global__ void k_rs_scatter(int32_t n, const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin,
                             uint32_t* __restrict__ kout, int32_t* __restrict__ vout, int shift,
                             int32_t ntiles, const int32_t* __restrict__ off) {
    __shared__ int32_t run[256];    // next output slot of each digit
    __shared__ int32_t wc[4][256];  // this round: per wave, items of each digit, then slots
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    run[tid] = off[(int64_t)tid * ntiles + blockIdx.x];
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_TILE / 256; ++r) {
#pragma unroll
        for (int w = 0; w < 4; ++w) wc[w][tid] = 0;
        __syncthreads();
        const int64_t i = base + r * 256 + tid;
        const bool ok = i < n;
        const uint32_t k = ok ? kin[i] : 0u;
        const uint32_t d = (k >> shift) & 255u;
        unsigned long long m = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const unsigned long long bb = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const int rank = __popcll(m & below);
        if (ok && (m >> lane) == 1ull) wc[wave][d] = rank + 1;  // last lane of its digit
        __syncthreads();
        int32_t acc = run[tid];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int32_t c = wc[w][tid];
            wc[w][tid] = acc;
            acc += c;
        }
        run[tid] = acc;
        __syncthreads();
        if (ok) {
            const int32_t pos = wc[wave][d] + rank;
            kout[pos] = k;
            vout[pos] = vin[i];
        }
        __syncthreads();
    }
}

// Zero fill of nw 32-bit words (in place of a memset, which a replayed graph must not hold).
__global__ void k_zero_words(uint32_t* __restrict__ p, int64_t nw) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_p2_nid(int32_t n, const int32_t* __restrict__ old, int32_t* __restrict__ nid) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) nid[old[r]] = (int32_t)r;
}

// skeleton id of frontier node v: the part's first skeleton id plus v's offset in the
// part's node range (frontier nodes come first)
__device__ __forceinline__ int32_t skid_of(int32_t v, const int32_t* lab, const int32_t* nid,
                                           const int64_t* poff, const int64_t* fbase) {
    const int32_t p = lab[v];
    return (int32_t)(fbase[p] + (nid[v] - poff[p]));
}

// Per renumbered row: intra-part arcs, and for frontier rows the cut arcs.
__global__ void k_p2_count(int32_t n, const int32_t* __restrict__ old, const int64_t* __restrict__ rp,
                           const int32_t* __restrict__ col, const int32_t* __restrict__ lab,
                           const uint8_t* __restrict__ fr, const int64_t* __restrict__ poff,
                           const int64_t* __restrict__ fbase, int64_t* __restrict__ icnt,
                           int64_t* __restrict__ rcnt, int32_t* __restrict__ rdeg) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t v = old[r];
    const int32_t p = lab[v];
    int64_t ci = 0, cr = 0;
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
        if (lab[col[e]] == p)
            ++ci;
        else
            ++cr;
    }
    icnt[r] = ci;
    if (fr[v]) {
        const int64_t f = fbase[p] + (r - poff[p]);
        rcnt[f] = cr;
        rdeg[f] = (int32_t)cr;
    }
}

// Fill the rows counted above. Intra arcs keep the original row's order; cut arcs are
// inserted sorted by skeleton id (reverse arcs are found by bisection). Largest
// cut-arc length into *rmax.
__global__ void k_p2_fill(int32_t n, const int32_t* __restrict__ old, const int32_t* __restrict__ nid,
                          const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const uint32_t* __restrict__ w, const int32_t* __restrict__ lab,
                          const uint8_t* __restrict__ fr, const int64_t* __restrict__ poff,
                          const int64_t* __restrict__ fbase, const int64_t* __restrict__ irp,
                          const int64_t* __restrict__ rptr, int32_t* __restrict__ icol,
                          uint32_t* __restrict__ iw, int32_t* __restrict__ rcol, uint32_t* __restrict__ rw,
                          uint32_t* __restrict__ rmax) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t v = old[r];
    const int32_t p = lab[v];
    int64_t o = irp[r];
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
        const int32_t u = col[e];
        if (lab[u] != p) continue;
        icol[o] = nid[u];
        if (iw) iw[o] = w ? w[e] : 1u;
        ++o;
    }
    if (!fr[v]) return;
    const int64_t f = fbase[p] + (r - poff[p]);
    const int64_t a = rptr[f];
    int64_t b = a;
    uint32_t mx = 0;
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
        const int32_t u = col[e];
        if (lab[u] == p) continue;
        const int32_t q = skid_of(u, lab, nid, poff, fbase);
        const uint32_t L = w ? w[e] : 1u;
        int64_t j = b;
        while (j > a && rcol[j - 1] > q) {
            rcol[j] = rcol[j - 1];
            rw[j] = rw[j - 1];
            --j;
        }
        rcol[j] = q;
        rw[j] = L;
        ++b;
        mx = max(mx, L);
    }
    if (mx) atomicMax(rmax, mx);
}

// Per renumbered row: blocked flag (frontier nodes, eq. frontierparents), output map
// (skeleton id, interior table row or none), skeleton node lists, interior rows.
__global__ void k_p2_rows(int32_t n, const int32_t* __restrict__ old, const int32_t* __restrict__ lab,
                          const uint8_t* __restrict__ fr, const uint8_t* __restrict__ ist,
                          const int64_t* __restrict__ poff, const int64_t* __restrict__ fbase,
                          const int32_t* __restrict__ pnf, const int32_t* __restrict__ pg0,
                          const int32_t* __restrict__ png, const int32_t* __restrict__ ibase,
                          uint8_t* __restrict__ blk, int32_t* __restrict__ il, int32_t* __restrict__ ig0,
                          int32_t* __restrict__ ing, int32_t* __restrict__ inode, int32_t* __restrict__ out_idx,
                          uint8_t* __restrict__ out_which, int32_t* __restrict__ nodes,
                          uint8_t* __restrict__ sflag) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t v = old[r];
    const int32_t p = lab[v];
    const int64_t loc = r - poff[p];
    blk[r] = fr[v] ? (uint8_t)NF_BLOCKED : 0;
    if (fr[v]) {
        const int64_t f = fbase[p] + loc;
        out_idx[v] = (int32_t)f;
        out_which[v] = 0;
        nodes[f] = v;
        sflag[f] = ist[v] ? (uint8_t)NF_TARGET : 0;
    } else if (png[p] > 0) {
        const int64_t i = ibase[p] + (loc - pnf[p]);
        il[i] = (int32_t)loc;
        ig0[i] = pg0[p];
        ing[i] = png[p];
        inode[i] = v;
        out_idx[v] = (int32_t)i;
        out_which[v] = 1;
    } else {
        out_idx[v] = -1;
        out_which[v] = 0;
    }
}

__global__ void k_p2_src(int32_t nS, const int32_t* __restrict__ S, const uint8_t* __restrict__ fr,
                         const int32_t* __restrict__ lab, const int32_t* __restrict__ nid,
                         const int64_t* __restrict__ poff, const int64_t* __restrict__ fbase,
                         int32_t* __restrict__ srcsk) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nS) return;
    const int32_t v = S[i];
    srcsk[i] = fr[v] ? skid_of(v, lab, nid, poff, fbase) : -1;
}

static unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>((n + 255) / 256, 1); }

static int key_bits(int64_t nlab) {
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) < 2 * nlab + 2) ++b;
    return b;
}

static void zero_bytes(hipStream_t s, void* p, size_t bytes) {
    const int64_t nw = (int64_t)(bytes / 4);
    if (nw <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((nw + 255) / 256, 1024);
    hipLaunchKernelGGL(k_zero_words, dim3(grid), dim3(256), 0, s, (uint32_t*)p, nw);
}

int SkBuild::issue_phase1(hipStream_t s) const {
    if (n <= 0) return BC_OK;
    KTimer kt(BC_K_OTHER, s);
    zero_bytes(s, p_psize, (size_t)nlab * 4);
    zero_bytes(s, p_pnf, (size_t)nlab * 4);
    zero_bytes(s, p_parc, (size_t)nlab * 8);
    zero_bytes(s, p_cross, 8);
    hipLaunchKernelGGL(k_p1_labels, dim3(blocks_for(n)), dim3(256), 0, s, n, p_part, p_lab, p_ist);
    if (nS)
        hipLaunchKernelGGL(k_p1_targets, dim3(blocks_for(nS)), dim3(256), 0, s, nS, p_S, k_in, given ? 1 : 0,
                           p_lab, p_ist);
    hipLaunchKernelGGL(k_p1_frontier, dim3(blocks_for(n)), dim3(256), 0, s, n, g->d_row_ptr, g->d_col, p_lab,
                       p_fr, p_psize, p_pnf, p_parc, p_cross);
    BC_HIP(hipGetLastError());
    return BC_OK;
}

int SkBuild::prepare(const bc_graph* gr, const int32_t* part, int32_t k, const int32_t* Sx, int32_t nSx,
                     bool given_singletons) {
    PhaseTrace tr("prepare");
    g = gr;
    n = g->n;
    nS = nSx;
    if (n > 0 && !part) return fail(BC_E_INVAL, "null partition");
    if (n > 0 && k < 1) return fail(BC_E_INVAL, "k must be >= 1");
    for (int32_t v = 0; v < n; ++v)
        if (part[v] < 0 || part[v] >= k)
            return fail(BC_E_INVAL, "partition label out of range at node " + std::to_string(v));
    BC_TRY(validate_targets(n, Sx, nS));
    S.assign(Sx, Sx + nS);
    k_in = k;
    given = given_singletons;
    weighted = g->d_len != nullptr;
    nlab = (int64_t)k + (given_singletons ? 0 : nS);
    if (nlab >= INT32_MAX) return fail(BC_E_INVAL, "too many parts");
    hipStream_t s = g->stream;
    tr.mark("validate");

    // ---- phase 1 on the device
    psize.assign(nlab, 0);
    pnf.assign(nlab, 0);
    parc.assign(nlab, 0);
    uint64_t cross = 0;
    if (n > 0) {
        bc_graph* gm = const_cast<bc_graph*>(g);
        Arena& P = gm->pre;
        const size_t need = (size_t)n * 4 * 2 + (size_t)n * 2 + (size_t)nS * 4 + (size_t)nlab * 16 + 16 * 256;
        BC_TRY(P.reserve(need));
        p_part = P.take<int32_t>(n);
        p_lab = P.take<int32_t>(n);
        p_ist = P.take<uint8_t>(n);
        p_fr = P.take<uint8_t>(n);
        p_S = P.take<int32_t>(std::max(nS, 1));
        p_psize = P.take<int32_t>(nlab);
        p_pnf = P.take<int32_t>(nlab);
        p_parc = P.take<unsigned long long>(nlab);
        p_cross = P.take<unsigned long long>(1);
        if (!p_cross) return fail(BC_E_NOMEM, "partition: scratch too small");
        BC_HIP(hipMemcpyAsync(p_part, part, (size_t)n * 4, hipMemcpyHostToDevice, s));
        if (nS) BC_HIP(hipMemcpyAsync(p_S, S.data(), (size_t)nS * 4, hipMemcpyHostToDevice, s));
        BC_TRY(issue_phase1(s));
        BC_HIP(hipMemcpyAsync(psize.data(), p_psize, (size_t)nlab * 4, hipMemcpyDeviceToHost, s));
        BC_HIP(hipMemcpyAsync(pnf.data(), p_pnf, (size_t)nlab * 4, hipMemcpyDeviceToHost, s));
        BC_HIP(hipMemcpyAsync(parc.data(), p_parc, (size_t)nlab * 8, hipMemcpyDeviceToHost, s));
        BC_HIP(hipMemcpyAsync(&cross, p_cross, 8, hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
    }
    tr.mark("phase 1 (device)");

    // ---- per part on the host: offsets, Dijkstra_SK groups, interior rows
    poff.assign(nlab + 1, 0);
    fbase.assign(nlab + 1, 0);
    aoff.assign(nlab + 1, 0);
    for (int64_t p = 0; p < nlab; ++p) {
        poff[p + 1] = poff[p] + psize[p];
        fbase[p + 1] = fbase[p] + pnf[p];
        aoff[p + 1] = aoff[p] + (int64_t)parc[p];
    }
    nsk = (int32_t)fbase[nlab];
    n_intra = aoff[nlab];
    nR = (int64_t)cross;
    groups.clear();
    info.clear();
    p_g0.assign(nlab, 0);
    p_ng.assign(nlab, 0);
    ibase.assign(nlab, 0);
    largest = kprime = clique_pairs = table_pairs = 0;
    int64_t rows = 0;
    for (int64_t p = 0; p < nlab; ++p) {
        if (psize[p] > 0) kprime++;
        largest = std::max<int64_t>(largest, psize[p]);
        if (psize[p] < 2 || pnf[p] == 0) continue;
        clique_pairs += (int64_t)pnf[p] * (pnf[p] - 1);
        table_pairs += (int64_t)pnf[p] * (psize[p] - pnf[p]);
        p_g0[p] = (int32_t)groups.size();
        // sources per group: fewer for larger parts (a launch lasts as long as its
        // longest group), the same for a part in every build
        const int64_t spg = dsk_sources_per_group(psize[p] + (int64_t)parc[p]);
        for (int64_t c = 0; c < pnf[p]; c += spg) {
            GroupDesc G;
            G.lo = (int32_t)poff[p];
            G.hi = (int32_t)(poff[p] + psize[p]);
            G.arc_lo = aoff[p];
            G.arcs = (int64_t)parc[p];
            G.flags = GF_RESTRICT | (weighted ? 0u : GF_UNIT);
            G.ring_len = g->maxw + 1;
            G.nsrc = (int32_t)std::min<int64_t>(spg, pnf[p] - c);
            for (int b = 0; b < LANES; ++b) G.src[b] = b < G.nsrc ? (int32_t)(poff[p] + c + b) : -1;
            groups.push_back(G);
            info.push_back({pnf[p], (int32_t)c, G.nsrc, (int32_t)fbase[p]});
        }
        p_ng[p] = (int32_t)groups.size() - p_g0[p];
        ibase[p] = (int32_t)rows;
        rows += psize[p] - pnf[p];
    }
    if (rows >= INT32_MAX) return fail(BC_E_INVAL, "too many interior nodes");
    nint = (int32_t)rows;
    // scratch of the device scans (CSR offsets, and the radix sort's digit offsets)
    ntiles = (int32_t)std::max<int64_t>((n + RS_TILE - 1) / RS_TILE, 1);
    scan_bytes = scan_scratch_bytes(std::max<int64_t>({(int64_t)ntiles * 256, (int64_t)n + 1, (int64_t)nsk + 1,
                                                      (int64_t)nint + 1}));
    tr.mark("groups, interior rows");
    return BC_OK;
}

size_t SkBuild::temp_bytes() const {
    const size_t ng = groups.size();
    size_t need = 0;
    for (const auto& G : groups)
        if (!(G.dist && G.sigma)) need += group_bytes(G, 0);
    const size_t N = (size_t)std::max(n, 1), K = (size_t)std::max(nsk, 1), I = (size_t)std::max(nint, 1);
    need += N * (8 + 8 + 4 + 4 + 4 + 8 + 8 + 1 + 4 + 1) + 16 +  // keys, vals, old, nid, counts, irp, blk, out
            (size_t)n_intra * (weighted ? 8 : 4) + (size_t)nR * 8 + K * (8 + 4 + 8 + 4 + 4 + 1) + 16 +
            ng * (sizeof(DskInfo) + sizeof(GroupDesc)) + I * 20 + (size_t)std::max(nS, 1) * 4 +
            (size_t)(nlab + 1) * (8 * 2 + 4 * 4) + (size_t)ntiles * 256 * 4 * 2 + scan_bytes +
            (K + 1) * 16 + (I + 1) * 16 + 56 * 256;
    return need;
}

int SkBuild::issue_phase2(hipStream_t s) const {
    KTimer kt(BC_K_OTHER, s);
    if (nsk) zero_bytes(s, d_cdeg, (size_t)nsk * 4);
    zero_bytes(s, d_maxlen, 4);
    zero_bytes(s, d_rmax, 4);
    zero_bytes(s, d_icnt + n, 8);
    zero_bytes(s, d_rcnt + nsk, 8);
    if (n > 0) {
        // renumbering: sort (key, node) pairs; the pass count decides which value
        // buffer the first pass reads so that the last one writes d_old
        const int bits = key_bits(nlab), passes = (bits + 7) / 8;
        uint32_t* kb[2] = {d_keys, d_keys2};
        int32_t* vb[2] = {passes % 2 ? d_vals : d_old, passes % 2 ? d_old : d_vals};
        hipLaunchKernelGGL(k_p2_keys, dim3(blocks_for(n)), dim3(256), 0, s, n, p_lab, p_fr, kb[0], vb[0]);
        for (int ps = 0; ps < passes; ++ps) {
            const int i = ps & 1;
            hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(256), 0, s, n, kb[i], 8 * ps, ntiles, d_hist);
            BC_TRY(exclusive_scan<int32_t>(s, d_hist, d_hoff, (int64_t)ntiles * 256, d_scan));
            hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(256), 0, s, n, kb[i], vb[i], kb[i ^ 1], vb[i ^ 1],
                               8 * ps, ntiles, d_hoff);
        }
        hipLaunchKernelGGL(k_p2_nid, dim3(blocks_for(n)), dim3(256), 0, s, n, d_old, d_nid);
        hipLaunchKernelGGL(k_p2_count, dim3(blocks_for(n)), dim3(256), 0, s, n, d_old, g->d_row_ptr, g->d_col,
                           p_lab, p_fr, d_poff, d_fbase, d_icnt, d_rcnt, d_rdeg);
        BC_TRY(exclusive_scan<int64_t>(s, d_icnt, d_irp, (int64_t)n + 1, d_scan));
        BC_TRY(exclusive_scan<int64_t>(s, d_rcnt, d_rptr, (int64_t)nsk + 1, d_scan));
        hipLaunchKernelGGL(k_p2_fill, dim3(blocks_for(n)), dim3(256), 0, s, n, d_old, d_nid, g->d_row_ptr,
                           g->d_col, g->d_len, p_lab, p_fr, d_poff, d_fbase, d_irp, d_rptr, d_icol, d_iw,
                           d_rcol, d_rw, d_rmax);
        hipLaunchKernelGGL(k_p2_rows, dim3(blocks_for(n)), dim3(256), 0, s, n, d_old, p_lab, p_fr, p_ist, d_poff,
                           d_fbase, d_ppnf, d_pg0, d_png, d_ibase, d_blk, d_il, d_ig0, d_ing, d_inode, d_out_idx,
                           d_out_which, d_nodes, d_sflag);
        if (nS)
            hipLaunchKernelGGL(k_p2_src, dim3(blocks_for(nS)), dim3(256), 0, s, nS, p_S, p_fr, p_lab, d_nid,
                               d_poff, d_fbase, d_srcsk);
    }
    BC_HIP(hipGetLastError());
    return BC_OK;
}

int SkBuild::upload(Arena& W, hipStream_t s) {
    PhaseTrace tr("upload");
    const int32_t ng = (int32_t)groups.size();
    const int64_t NL = std::max<int64_t>(nlab, 1);
    d_keys = W.take<uint32_t>(std::max(n, 1));
    d_keys2 = W.take<uint32_t>(std::max(n, 1));
    d_vals = W.take<int32_t>(std::max(n, 1));
    d_old = W.take<int32_t>(std::max(n, 1));
    d_nid = W.take<int32_t>(std::max(n, 1));
    d_icnt = W.take<int64_t>(n + 1);
    d_irp = W.take<int64_t>(n + 1);
    d_icol = W.take<int32_t>(std::max<int64_t>(n_intra, 1));
    d_iw = weighted ? W.take<uint32_t>(std::max<int64_t>(n_intra, 1)) : nullptr;
    d_blk = W.take<uint8_t>(std::max(n, 1));
    d_rcnt = W.take<int64_t>(nsk + 1);
    d_rdeg = W.take<int32_t>(std::max(nsk, 1));
    d_rptr = W.take<int64_t>(nsk + 1);
    d_rcol = W.take<int32_t>(std::max<int64_t>(nR, 1));
    d_rw = W.take<uint32_t>(std::max<int64_t>(nR, 1));
    d_cdeg = W.take<int32_t>(std::max(nsk, 1));
    d_info = W.take<DskInfo>(std::max(ng, 1));
    d_il = W.take<int32_t>(std::max(nint, 1));
    d_ig0 = W.take<int32_t>(std::max(nint, 1));
    d_ing = W.take<int32_t>(std::max(nint, 1));
    d_tdeg = W.take<int32_t>(std::max(nint, 1));
    d_inode = W.take<int32_t>(std::max(nint, 1));
    d_out_idx = W.take<int32_t>(std::max(n, 1));
    d_out_which = W.take<uint8_t>(std::max(n, 1));
    d_nodes = W.take<int32_t>(std::max(nsk, 1));
    d_sflag = W.take<uint8_t>(std::max(nsk, 1));
    d_srcsk = W.take<int32_t>(std::max(nS, 1));
    d_poff = W.take<int64_t>(NL + 1);
    d_fbase = W.take<int64_t>(NL + 1);
    d_ppnf = W.take<int32_t>(NL);
    d_pg0 = W.take<int32_t>(NL);
    d_png = W.take<int32_t>(NL);
    d_ibase = W.take<int32_t>(NL);
    d_maxlen = W.take<uint32_t>(1);
    d_rmax = W.take<uint32_t>(1);
    d_bigm = W.take<uint32_t>(1);
    d_hist = W.take<int32_t>((size_t)ntiles * 256);
    d_hoff = W.take<int32_t>((size_t)ntiles * 256);
    d_scan = W.take<unsigned char>(std::max<size_t>(scan_bytes, 1));
    d_desc = W.take<GroupDesc>(std::max(ng, 1));
    d_slen = W.take<int64_t>(nsk + 1);
    d_srow = W.take<int64_t>(nsk + 1);
    d_tlen = W.take<int64_t>(nint + 1);
    d_trow = W.take<int64_t>(nint + 1);
    if (!d_slen || !d_srow || !d_tlen || !d_trow || !d_bigm) return fail(BC_E_NOMEM, "partition: workspace too small");
    if (!d_keys || !d_keys2 || !d_vals || !d_old || !d_nid || !d_icnt || !d_irp || !d_icol || (weighted && !d_iw) ||
        !d_blk || !d_rcnt || !d_rdeg || !d_rptr || !d_rcol || !d_rw || !d_cdeg || !d_info || !d_il || !d_ig0 ||
        !d_ing || !d_tdeg || !d_inode || !d_out_idx || !d_out_which || !d_nodes || !d_sflag || !d_srcsk ||
        !d_poff || !d_fbase || !d_ppnf || !d_pg0 || !d_png || !d_ibase || !d_maxlen || !d_rmax || !d_hist ||
        !d_hoff || !d_scan || !d_desc)
        return fail(BC_E_NOMEM, "partition: workspace too small");
    auto h2d = [&](void* d, const void* h, size_t b) -> int {
        if (b) BC_HIP(hipMemcpyAsync(d, h, b, hipMemcpyHostToDevice, s));
        return BC_OK;
    };
    BC_TRY(h2d(d_poff, poff.data(), (size_t)(nlab + 1) * 8));
    BC_TRY(h2d(d_fbase, fbase.data(), (size_t)(nlab + 1) * 8));
    BC_TRY(h2d(d_ppnf, pnf.data(), (size_t)nlab * 4));
    BC_TRY(h2d(d_pg0, p_g0.data(), (size_t)nlab * 4));
    BC_TRY(h2d(d_png, p_ng.data(), (size_t)nlab * 4));
    BC_TRY(h2d(d_ibase, ibase.data(), (size_t)nlab * 4));
    BC_TRY(h2d(d_info, info.data(), (size_t)ng * sizeof(DskInfo)));
    BC_TRY(issue_phase2(s));
    for (auto& G : groups) {
        G.g.row_ptr = d_irp;
        G.g.col = d_icol;
        G.g.len = d_iw;
        G.g.nflag = d_blk;
        // a group whose output lanes a caller has already set (results kept from an
        // earlier build of the same part) takes no state here and is not run
        if (G.dist && G.sigma) continue;
        if (!group_alloc(W, G, 0)) return fail(BC_E_NOMEM, "partition: group state does not fit");
    }
    BC_TRY(h2d(d_desc, groups.data(), (size_t)ng * sizeof(GroupDesc)));
    // host arrays above are staged by the runtime; after this only a replay of the
    // device work reads the graph's scratch arena again
    BC_HIP(hipStreamSynchronize(s));
    tr.mark("phase 2 (device)");
    return BC_OK;
}

int SkBuild::issue_count(hipStream_t s) const {
    const int32_t ng = (int32_t)groups.size();
    KTimer kt(BC_K_OTHER, s);
    if (ng > 0) {
        hipLaunchKernelGGL(k_clique_count, dim3(ng), dim3(256), 0, s, d_desc, d_info, ng, d_cdeg);
        if (nint)
            hipLaunchKernelGGL(k_table, dim3((nint + 3) / 4), dim3(256), 0, s, d_desc, d_info, nint, d_il,
                               d_ig0, d_ing, d_tdeg, nullptr, nullptr, nullptr, nullptr);
    }
    // without Dijkstra_SK groups no table row has an entry
    hipLaunchKernelGGL(k_row_lengths, dim3(std::max(nsk, nint) / 256 + 1), dim3(256), 0, s, nsk, nint, d_rdeg,
                       d_cdeg, ng > 0 ? d_tdeg : nullptr, d_slen, d_tlen);
    BC_HIP(hipGetLastError());
    if (n > 0) {
        BC_TRY(exclusive_scan<int64_t>(s, d_slen, d_srow, (int64_t)nsk + 1, d_scan));
        BC_TRY(exclusive_scan<int64_t>(s, d_tlen, d_trow, (int64_t)nint + 1, d_scan));
    } else {
        zero_bytes(s, d_srow, 8);
        zero_bytes(s, d_trow, 8);
    }
    BC_HIP(hipGetLastError());
    return BC_OK;
}

int SkBuild::issue_fill(hipStream_t s, const bc_skeleton* sk) const {
    const int32_t ng = (int32_t)groups.size();
    auto d2d = [&](void* d, const void* h, size_t b) -> int {
        if (b) BC_HIP(hipMemcpyAsync(d, h, b, hipMemcpyDeviceToDevice, s));
        return BC_OK;
    };
    BC_TRY(d2d(sk->d_row_ptr, d_srow, (size_t)(nsk + 1) * 8));
    BC_TRY(d2d(sk->d_trow, d_trow, (size_t)(nint + 1) * 8));
    BC_TRY(d2d(sk->d_nflag, d_sflag, nsk));
    BC_TRY(d2d(sk->d_nodes, d_nodes, (size_t)nsk * 4));
    BC_TRY(d2d(sk->d_tnode, d_inode, (size_t)nint * 4));
    BC_TRY(d2d(sk->d_out_idx, d_out_idx, (size_t)n * 4));
    BC_TRY(d2d(sk->d_out_which, d_out_which, n));
    {
        KTimer kt(BC_K_OTHER, s);
        if (nsk)
            hipLaunchKernelGGL(k_fill_r, dim3((nsk + 255) / 256), dim3(256), 0, s, nsk, d_rptr, d_rcol, d_rw,
                               sk->d_row_ptr, sk->d_col, sk->d_len, sk->d_mult);
        if (ng) {
            hipLaunchKernelGGL(k_clique_fill, dim3(ng), dim3(256), 0, s, d_desc, d_info, ng,
                               sk->d_row_ptr, d_rdeg, sk->d_col, sk->d_len, sk->d_mult, d_maxlen);
            if (nint)
                hipLaunchKernelGGL(k_table, dim3((nint + 3) / 4), dim3(256), 0, s, d_desc, d_info, nint, d_il,
                                   d_ig0, d_ing, nullptr, sk->d_trow, sk->d_tcol, sk->d_tlen, sk->d_tsig);
        }
        if (nsk)
            hipLaunchKernelGGL(k_sk_twin, dim3((nsk + 3) / 4), dim3(256), 0, s, nsk, sk->d_row_ptr, d_rdeg,
                               sk->d_col, sk->d_twin);
        const int64_t m = sk->h_row_ptr.empty() ? 0 : sk->h_row_ptr.back();
        zero_bytes(s, d_bigm, 4);
        if (m > 0 && sk->d_arc_store)
            hipLaunchKernelGGL(k_pack_arcs, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, m, sk->d_col,
                               sk->d_len, sk->d_twin, sk->d_mult, sk->d_arc_store, d_bigm);
    }
    BC_HIP(hipGetLastError());
    return BC_OK;
}

int SkBuild::assemble(Arena& W, hipStream_t s, bc_skeleton* sk,
                      const std::function<int(size_t, Arena*&)>& get_store) {
    (void)W;
    BC_TRY(issue_count(s));
    // read back the skeleton's row offsets (the host keeps them for group ranges)
    // and the table's total; both were scanned on the device
    sk->h_row_ptr.assign(nsk + 1, 0);
    int64_t T = 0;
    BC_HIP(hipMemcpyAsync(sk->h_row_ptr.data(), d_srow, (size_t)(nsk + 1) * 8, hipMemcpyDeviceToHost, s));
    BC_HIP(hipMemcpyAsync(&T, d_trow + nint, 8, hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    const int64_t M = sk->h_row_ptr[nsk];
    // every skeleton row holds its cut arcs (nR in all) and then its clique arcs
    const int64_t ncl = M - nR;

    // ---- the skeleton's own store
    const size_t sbytes = (size_t)(nsk + 1) * 8 + (size_t)M * (4 + 4 + 8 + 8) + (size_t)nsk +
                          (size_t)(nint + 1) * 8 + (size_t)T * (4 + 4 + 8) + (size_t)nsk * 4 +
                          (size_t)nint * 4 + (size_t)n * 5 + (size_t)M * 16 + 34 * 256;
    Arena* Ap = nullptr;
    BC_TRY(get_store(sbytes, Ap));
    Arena& A = *Ap;
    sk->d_row_ptr = A.take<int64_t>(nsk + 1);
    sk->d_col = A.take<int32_t>(std::max<int64_t>(M, 1));
    sk->d_len = A.take<uint32_t>(std::max<int64_t>(M, 1));
    sk->d_mult = A.take<uint64_t>(std::max<int64_t>(M, 1));
    sk->d_twin = A.take<int64_t>(std::max<int64_t>(M, 1));
    sk->d_nflag = A.take<uint8_t>(std::max(nsk, 1));
    sk->d_trow = A.take<int64_t>(nint + 1);
    sk->d_tcol = A.take<int32_t>(std::max<int64_t>(T, 1));
    sk->d_tlen = A.take<uint32_t>(std::max<int64_t>(T, 1));
    sk->d_tsig = A.take<uint64_t>(std::max<int64_t>(T, 1));
    sk->d_nodes = A.take<int32_t>(std::max(nsk, 1));
    sk->d_tnode = A.take<int32_t>(std::max(nint, 1));
    sk->d_out_idx = A.take<int32_t>(std::max(n, 1));
    sk->d_out_which = A.take<uint8_t>(std::max(n, 1));
    sk->d_arc_store = M < ((int64_t)1 << 31) ? A.take<ArcRec>((size_t)std::max<int64_t>(M, 1)) : nullptr;
    if (!sk->d_out_which) return fail(BC_E_NOMEM, "skeleton store too small");
    BC_TRY(issue_fill(s, sk));
    uint32_t clique_max = 0, rmax = 0, bigm = 0;
    std::vector<int32_t> srcsk(nS);
    BC_HIP(hipMemcpyAsync(&bigm, d_bigm, 4, hipMemcpyDeviceToHost, s));
    BC_HIP(hipMemcpyAsync(&clique_max, d_maxlen, 4, hipMemcpyDeviceToHost, s));
    BC_HIP(hipMemcpyAsync(&rmax, d_rmax, 4, hipMemcpyDeviceToHost, s));
    if (nS) BC_HIP(hipMemcpyAsync(srcsk.data(), d_srcsk, (size_t)nS * 4, hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));

    sk->graph = g;
    sk->n = n;
    sk->d_arc = bigm ? nullptr : sk->d_arc_store;
    sk->max_len = (int32_t)std::max<uint32_t>({1u, rmax, clique_max});
    // Brandes_SK sources: targets that have a neighbour (isolated targets reach nobody)
    sk->h_target_sk = srcsk;
    sk->h_src.clear();
    for (int32_t f : srcsk)
        if (f >= 0) sk->h_src.push_back(f);
    sk->n_sk = nsk;
    sk->n_int = nint;
    sk->m_arcs = M;
    sk->t_nnz = T;
    sk->max_dist = (int64_t)std::max(n - 1, 0) * g->maxw;
    bc_sk_stats& st = sk->stats;
    st.n = n;
    st.n_sk = nsk;
    st.k_prime = (int32_t)kprime;
    st.largest_part = (int32_t)largest;
    st.r_arcs = nR;
    st.clique_arcs = ncl;
    st.clique_pruned = clique_pairs - ncl;
    st.table_nnz = T;
    st.table_pruned = table_pairs - T;
    int64_t dsk = 0;
    for (auto& I : info) dsk += I.nsrc;
    st.dsk_sources = dsk;
    st.device_bytes = (int64_t)sbytes;
    return BC_OK;
}

// The skeleton when every node is a target, listed in id order: every part of P' is a
// singleton, so every node with a neighbour is a frontier node, every arc a cut arc
// <w, 1>, there are no clique arcs and no tables, and the renumbering (parts of P' in
// label order, target i labelled k + i) keeps id order, only dropping the isolated
// nodes, which are not frontier nodes (Sec. 5 with S = V: G_SK is G less its isolated
// nodes). This is exactly what the general build assembles. Without isolated nodes it
// reads G's arrays instead of copying them; with some, the arcs keep their positions
// (isolated nodes have none) and only their heads are renumbered.
__global__ void k_identity_nodes(int32_t n, int32_t nsk, const int32_t* __restrict__ remap,
                                 int32_t* __restrict__ nodes, int32_t* __restrict__ out_idx,
                                 uint8_t* __restrict__ out_which, uint8_t* __restrict__ nflag) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) {
        const int32_t f = remap ? remap[v] : v;
        out_idx[v] = f;
        out_which[v] = 0;
        if (f >= 0) nodes[f] = v;
    }
    if (v < nsk) nflag[v] = (uint8_t)NF_TARGET;
}

// Per arc: the all-ones multiplicity, and (with isolated nodes dropped) the renumbered
// head, the length (1 for unit weights), the reverse arc and the packed record.
__global__ void k_identity_arcs(int64_t m, const int32_t* __restrict__ remap, const int32_t* __restrict__ col,
                                const uint32_t* __restrict__ len, const int64_t* __restrict__ twin,
                                int32_t* __restrict__ col_out, uint32_t* __restrict__ len_out,
                                int64_t* __restrict__ twin_out, ArcRec* __restrict__ arc_out,
                                uint64_t* __restrict__ mult) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    mult[e] = 1ull;
    const uint32_t L = len ? len[e] : 1u;
    if (len_out) len_out[e] = L;
    if (col_out) {
        const int32_t c = remap[col[e]];
        col_out[e] = c;
        twin_out[e] = twin[e];
        if (arc_out) arc_out[e] = ArcRec{(uint32_t)c, L, (uint32_t)twin[e], 1u};
    }
}

static bool identity_skeleton_applies(const bc_graph* g, const int32_t* S, int32_t nS, bool given_singletons) {
    // (BCPP_SK_IDENTITY=0 takes the general build, for comparisons)
    const char* e = getenv("BCPP_SK_IDENTITY");
    if ((e && e[0] == '0') || given_singletons || g->n < 1 || nS != g->n || !S) return false;
    for (int32_t i = 0; i < nS; ++i)
        if (S[i] != i) return false;
    return true;
}

static int identity_skeleton(const bc_graph* g, const int32_t* part, int32_t k, bc_skeleton** out) {
    const int32_t n = g->n;
    if (!part) return fail(BC_E_INVAL, "null partition");
    if (k < 1) return fail(BC_E_INVAL, "k must be >= 1");
    for (int32_t v = 0; v < n; ++v)
        if (part[v] < 0 || part[v] >= k)
            return fail(BC_E_INVAL, "partition label out of range at node " + std::to_string(v));
    const int64_t m = g->nnz;
    // skeleton ids: the nodes with a neighbour, in id order
    std::vector<int32_t> remap(n);
    std::vector<int64_t> rp;
    int32_t nsk = 0;
    for (int32_t v = 0; v < n; ++v) remap[v] = g->h_row_ptr[v + 1] > g->h_row_ptr[v] ? nsk++ : -1;
    const bool copy = nsk < n;
    if (copy) {
        rp.reserve((size_t)nsk + 1);
        for (int32_t v = 0; v < n; ++v)
            if (remap[v] >= 0) rp.push_back(g->h_row_ptr[v]);
        rp.push_back(m);
    }
    auto sk = std::make_unique<bc_skeleton>();
    const bool arcs_out = copy && g->d_arc;
    const size_t bytes = (size_t)n * (4 + 4 + 1 + 1) + (size_t)m * 8 +
                         (copy ? (size_t)n * 4 + (size_t)(nsk + 1) * 8 + (size_t)m * (4 + 4 + 8) : 0) +
                         (!copy && !g->d_len ? (size_t)m * 4 : 0) + (arcs_out ? (size_t)m * 16 : 0) + 16 * 256;
    BC_TRY(sk->store.reserve(bytes));
    Arena& A = sk->store;
    const size_t M = (size_t)std::max<int64_t>(m, 1);
    sk->d_nodes = A.take<int32_t>(std::max(nsk, 1));
    sk->d_out_idx = A.take<int32_t>(n);
    sk->d_out_which = A.take<uint8_t>(n);
    sk->d_nflag = A.take<uint8_t>(std::max(nsk, 1));
    sk->d_mult = A.take<uint64_t>(M);
    sk->d_trow = A.take<int64_t>(1);
    int32_t* d_remap = copy ? A.take<int32_t>(n) : nullptr;
    if (copy) {
        sk->d_row_ptr = A.take<int64_t>((size_t)nsk + 1);
        sk->d_col = A.take<int32_t>(M);
        sk->d_len = A.take<uint32_t>(M);
        sk->d_twin = A.take<int64_t>(M);
        sk->d_arc = arcs_out ? A.take<ArcRec>(M) : nullptr;
        sk->d_arc_store = sk->d_arc;
    } else {
        sk->d_row_ptr = g->d_row_ptr;
        sk->d_col = g->d_col;
        sk->d_len = g->d_len ? g->d_len : A.take<uint32_t>(M);
        sk->d_twin = g->d_twin;
        sk->d_arc = g->d_arc;
    }
    if (!sk->d_trow || !sk->d_len || (copy && (!sk->d_twin || (arcs_out && !sk->d_arc))))
        return fail(BC_E_NOMEM, "skeleton store too small");
    hipStream_t s = g->stream;
    if (copy) {
        BC_HIP(hipMemcpyAsync(d_remap, remap.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
        BC_HIP(hipMemcpyAsync(sk->d_row_ptr, rp.data(), rp.size() * 8, hipMemcpyHostToDevice, s));
    }
    hipLaunchKernelGGL(k_identity_nodes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, nsk, d_remap,
                       sk->d_nodes, sk->d_out_idx, sk->d_out_which, sk->d_nflag);
    if (m > 0)
        hipLaunchKernelGGL(k_identity_arcs, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, m, d_remap,
                           g->d_col, g->d_len, g->d_twin, copy ? sk->d_col : nullptr,
                           (copy || !g->d_len) ? sk->d_len : nullptr, copy ? sk->d_twin : nullptr,
                           arcs_out ? sk->d_arc : nullptr, sk->d_mult);
    zero_bytes(s, sk->d_trow, 8);
    BC_HIP(hipGetLastError());
    sk->graph = g;
    sk->n = n;
    sk->n_sk = nsk;
    sk->n_int = 0;
    sk->m_arcs = m;
    sk->t_nnz = 0;
    sk->max_len = std::max<int32_t>(1, m > 0 ? g->maxw : 1);
    sk->max_dist = (int64_t)std::max(n - 1, 0) * g->maxw;
    sk->h_row_ptr = copy ? rp : g->h_row_ptr;
    sk->h_target_sk = remap;
    sk->h_src.clear();
    for (int32_t f : remap)
        if (f >= 0) sk->h_src.push_back(f);
    bc_sk_stats& st = sk->stats;
    st.n = n;
    st.n_sk = nsk;
    st.k_prime = n;
    st.largest_part = 1;
    st.r_arcs = m;
    st.device_bytes = (int64_t)bytes;
    BC_HIP(hipStreamSynchronize(s));
    *out = sk.release();
    return BC_OK;
}

int build_dsk_cache(bc_graph* g, const int32_t* part, int32_t k, DskCache* c) {
    hipStream_t s = g->stream;
    SkBuild b;
    BC_TRY(b.prepare(g, part, k, nullptr, 0, false));
    for (auto& G : b.groups)
        if (!resident_takes((int64_t)G.hi - G.lo)) return BC_OK;
    size_t need = b.temp_bytes() + resident_launch_bytes(b.groups.size()) + 8192;
    size_t bytes = 0;
    for (auto& G : b.groups) {
        const size_t r = (size_t)(G.hi - G.lo);
        if ((int64_t)r > resident_max_range()) need += r * 12 + 512;
        bytes += ((r * 64 * 4 + 255) & ~(size_t)255) + ((r * 64 * 8 + 255) & ~(size_t)255);
    }
    Arena W;
    BC_TRY(W.reserve(need));
    BC_TRY(b.upload(W, s));
    for (auto& G : b.groups) {
        if ((int64_t)G.hi - G.lo <= resident_max_range()) continue;
        G.gdist = W.take<uint32_t>((size_t)(G.hi - G.lo));
        G.gsig = W.take<uint64_t>((size_t)(G.hi - G.lo));
        if (!G.gdist || !G.gsig) return fail(BC_E_NOMEM, "Dijkstra_SK cache: workspace too small");
    }
    BC_TRY(run_resident(s, W, b.groups));
    BC_TRY(c->store.reserve(bytes + 4096));
    for (auto& G : b.groups) {
        const size_t lanes = (size_t)(G.hi - G.lo) * 64;
        uint32_t* d = c->store.take<uint32_t>(lanes);
        uint64_t* q = c->store.take<uint64_t>(lanes);
        if (!d || !q) return fail(BC_E_NOMEM, "Dijkstra_SK cache: store too small");
        BC_HIP(hipMemcpyAsync(d, G.dist, lanes * 4, hipMemcpyDeviceToDevice, s));
        BC_HIP(hipMemcpyAsync(q, G.sigma, lanes * 8, hipMemcpyDeviceToDevice, s));
        c->dist.push_back(d);
        c->sig.push_back(q);
    }
    BC_HIP(hipStreamSynchronize(s));
    c->first.assign(b.p_g0.begin(), b.p_g0.begin() + k);
    c->count.assign(b.p_ng.begin(), b.p_ng.begin() + k);
    c->nf.assign(b.pnf.begin(), b.pnf.begin() + k);
    c->bytes = c->store.cap;
    c->ok = true;
    return BC_OK;
}

int32_t dsk_preset_from_cache(SkBuild& b, const DskCache& c, const int32_t* part, std::vector<uint8_t>& preset) {
    preset.assign(b.groups.size(), 0);
    if (!c.ok || (int32_t)c.count.size() != b.k_in) return 0;
    std::vector<uint8_t> has_t(b.k_in, 0);
    for (int32_t t : b.S) has_t[part[t]] = 1;
    int32_t got = 0;
    for (int32_t p = 0; p < b.k_in; ++p) {
        if (has_t[p] || b.p_ng[p] == 0 || c.count[p] != b.p_ng[p] || c.nf[p] != b.pnf[p]) continue;
        for (int32_t j = 0; j < b.p_ng[p]; ++j) {
            GroupDesc& G = b.groups[b.p_g0[p] + j];
            G.dist = c.dist[c.first[p] + j];
            G.sigma = c.sig[c.first[p] + j];
            preset[b.p_g0[p] + j] = 1;
            ++got;
        }
    }
    return got;
}

int partition_impl(const bc_graph* g, const int32_t* part, int32_t k, const int32_t* S, int32_t nS,
                   bc_skeleton** out, bool given_singletons, PartitionKeep* keep, const DskCache* cache) {
    if (!keep && identity_skeleton_applies(g, S, nS, given_singletons)) return identity_skeleton(g, part, k, out);
    PhaseTrace tr("partition");
    SkBuild local;
    SkBuild& b = keep ? keep->b : local;
    BC_TRY(b.prepare(g, part, k, S, nS, given_singletons));
    tr.mark("prepare (host)");
    bc_graph* gm = const_cast<bc_graph*>(g);
    Arena& W = gm->work;
    hipStream_t s = g->stream;
    // parts without a target take their Dijkstra_SK lanes from the cache (only on the
    // resident kernel, whose lanes the cache holds, and never for a kept build)
    std::vector<uint8_t> preset(b.groups.size(), 0);
    int32_t npreset = 0;
    if (cache && cache->ok && !keep && !given_singletons) {
        bool all_res = true;
        for (auto& G : b.groups) all_res = all_res && resident_takes((int64_t)G.hi - G.lo);
        if (all_res) npreset = dsk_preset_from_cache(b, *cache, part, preset);
    }
    int64_t positions = 0;
    for (auto& G : b.groups) positions += (int64_t)G.hi - G.lo;
    // Dijkstra_SK groups run on the resident kernel (parts larger than LDS keep their
    // one-source state in device memory), or on the engine when it is switched off
    bool res = !b.groups.empty();
    size_t extra = 0;
    for (size_t i = 0; i < b.groups.size(); ++i) {
        const GroupDesc& G = b.groups[i];
        res = res && resident_takes((int64_t)G.hi - G.lo);
        if (!preset[i] && (int64_t)G.hi - G.lo > resident_max_range()) extra += (size_t)(G.hi - G.lo) * 12 + 512;
    }
    extra += resident_launch_bytes(b.groups.size());
    BC_TRY(W.reserve(b.temp_bytes() + std::max(extra, engine_bytes(std::max<int32_t>((int32_t)b.groups.size(), 1),
                                                                   positions))));
    BC_TRY(b.upload(W, s));
    tr.mark("upload");
    if (res && npreset > 0) {
        std::vector<GroupDesc> todo;
        for (size_t i = 0; i < b.groups.size(); ++i) {
            if (preset[i]) continue;
            GroupDesc G = b.groups[i];
            if ((int64_t)G.hi - G.lo > resident_max_range()) {
                G.gdist = W.take<uint32_t>((size_t)(G.hi - G.lo));
                G.gsig = W.take<uint64_t>((size_t)(G.hi - G.lo));
                if (!G.gdist || !G.gsig) return fail(BC_E_NOMEM, "partition: workspace too small");
            }
            todo.push_back(G);
        }
        if (!todo.empty()) BC_TRY(run_resident(s, W, todo));
    } else if (res) {
        for (auto& G : b.groups) {
            if ((int64_t)G.hi - G.lo <= resident_max_range()) continue;
            G.gdist = W.take<uint32_t>((size_t)(G.hi - G.lo));
            G.gsig = W.take<uint64_t>((size_t)(G.hi - G.lo));
            if (!G.gdist || !G.gsig) return fail(BC_E_NOMEM, "partition: workspace too small");
        }
        if (keep) {
            keep->resident = true;
            BC_TRY(resident_upload(s, W, b.groups, &keep->L));
            BC_TRY(resident_launch(s, keep->L));
            uint32_t herr = 0;
            BC_HIP(hipMemcpyAsync(&herr, keep->L.d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            BC_HIP(hipStreamSynchronize(s));
            if (herr & ERR_OVERFLOW) return fail(BC_E_OVERFLOW, "a shortest-path count reached 2^64");
        } else {
            BC_TRY(run_resident(s, W, b.groups));
        }
    } else if (!b.groups.empty()) {
        BC_TRY(run_groups_prealloc(W, s, b.groups));
    }
    tr.mark("Dijkstra_SK");
    auto sk = std::make_unique<bc_skeleton>();
    BC_TRY(b.assemble(W, s, sk.get(), [&](size_t bytes, Arena*& A) -> int {
        BC_TRY(sk->store.reserve(bytes));
        A = &sk->store;
        return BC_OK;
    }));
    tr.mark("assemble");
    *out = sk.release();
    return BC_OK;
}

std::vector<GroupDesc> bsk_groups(const bc_skeleton* sk, const int32_t* src, int32_t nsrc, int32_t lo,
                                  int32_t hi, int32_t t_lo, int32_t tn) {
    std::vector<GroupDesc> groups;
    for (int32_t c = 0; c < nsrc; c += LANES) {
        GroupDesc D;
        D.g.row_ptr = sk->d_row_ptr;
        D.g.col = sk->d_col;
        D.g.len = sk->d_len;
        D.g.mult = sk_mult(sk);
        D.g.nflag = sk->d_nflag;
        D.g.twin = sk->d_twin;
        D.g.arc = sk->d_arc;
        D.lo = lo;
        D.hi = hi;
        D.arc_lo = sk->h_row_ptr[lo];
        D.arcs = sk->h_row_ptr[hi] - sk->h_row_ptr[lo];
        D.ring_len = sk->max_len + 1;
        D.flags = GF_BACKWARD | (tn ? GF_CENT : 0u);
        D.trow = sk->d_trow;
        D.tcol = sk->d_tcol;
        D.tlen = sk->d_tlen;
        D.tsig = sk->d_tsig;
        D.t_lo = tn ? t_lo : 0;
        D.tn = tn;
        D.nsrc = std::min(LANES, nsrc - c);
        for (int l = 0; l < LANES; ++l) D.src[l] = l < D.nsrc ? src[c + l] : -1;
        groups.push_back(D);
    }
    return groups;
}

// --------------------------------------------------------------- Brandes++ -----

std::vector<GroupDesc> resident_bsk_groups(const bc_skeleton* sk) {
    return resident_bsk_groups(sk, sk->h_src, sk->d_nflag);
}

std::vector<GroupDesc> resident_bsk_groups(const bc_skeleton* sk, const std::vector<int32_t>& src,
                                           const uint8_t* nflag) {
    const int32_t nsrc = (int32_t)src.size();
    const int32_t spg = resident_sources_per_group(nsrc);
    const int32_t ngroups = (nsrc + spg - 1) / spg;
    std::vector<GroupDesc> groups(ngroups);
    for (int32_t j = 0; j < ngroups; ++j) {
        GroupDesc& G = groups[j];
        G.g.row_ptr = sk->d_row_ptr;
        G.g.col = sk->d_col;
        G.g.len = sk->d_len;
        G.g.mult = sk_mult(sk);
        G.g.nflag = nflag;
        G.g.twin = sk->d_twin;
        G.g.arc = sk->d_arc;
        G.lo = 0;
        G.hi = sk->n_sk;
        G.arc_lo = 0;
        G.arcs = sk->m_arcs;
        G.ring_len = sk->max_len + 1;
        G.flags = GF_BACKWARD | (sk->n_int ? GF_CENT : 0u);
        G.trow = sk->d_trow;
        G.tcol = sk->d_tcol;
        G.tlen = sk->d_tlen;
        G.tsig = sk->d_tsig;
        G.t_lo = 0;
        G.tn = sk->n_int;
        const int32_t first = j * spg;
        G.nsrc = std::min(spg, nsrc - first);
        for (int b = 0; b < LANES; ++b) G.src[b] = b < G.nsrc ? src[first + b] : -1;
    }
    return groups;
}

// Brandes_SK and Centrality with the LDS-resident kernel: the skeleton fits in LDS.
static int pp_resident(bc_graph* g, const bc_skeleton* sk, double scale, double* out_dev) {
    hipStream_t s = g->stream;
    std::vector<GroupDesc> groups = resident_bsk_groups(sk);
    size_t need = resident_launch_bytes(groups.size()) + 2 * (groups.size() * 8 + 256) + 65536;
    for (const GroupDesc& G : groups) need += resident_group_bytes(G);
    BC_TRY(g->work.reserve(need));
    g->work.used = 0;
    for (GroupDesc& G : groups)
        if (!resident_alloc(g->work, G)) return fail(BC_E_NOMEM, "Brandes++: workspace too small");
    BC_TRY(run_resident(s, g->work, groups));
    return reduce_scores(s, g->work, groups, g->n, nullptr, nullptr, sk->d_out_idx, sk->d_out_which,
                         scale, out_dev, false);
}

int pp_run(const bc_graph* gc, const bc_skeleton* sk, uint32_t flags, double* out_dev) {
    bc_graph* g = const_cast<bc_graph*>(gc);
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    const double scale = (flags & BC_ORDERED) ? 1.0 : 0.5;
    if (n == 0) return BC_OK;
    const int32_t nsrc = (int32_t)sk->h_src.size();
    if (nsrc < 2 || sk->n_sk == 0) {
        BC_HIP(hipMemsetAsync(out_dev, 0, (size_t)n * 8, s));
        BC_HIP(hipStreamSynchronize(s));
        return BC_OK;
    }
    const int32_t N = sk->n_sk;
    if (!(flags & BC_ENGINE_ONLY) && resident_takes(N)) return pp_resident(g, sk, scale, out_dev);
    const int64_t steps = max_steps_bound(N, LANES, sk->max_dist);
    const int32_t ngroups = (nsrc + LANES - 1) / LANES;
    const uint32_t gflags = GF_BACKWARD | (sk->n_int ? GF_CENT : 0u);
    GroupDesc shape;
    shape.hi = N;
    shape.arcs = sk->m_arcs;
    shape.nsrc = LANES;
    shape.flags = gflags;
    shape.tn = sk->n_int;
    shape.ring_len = sk->max_len + 1;
    const size_t per_group = group_bytes(shape, steps);
    int32_t wave_groups = (int32_t)std::max<size_t>(1, state_budget() / std::max<size_t>(per_group, 1));
    if (const char* e = getenv("BCPP_MAX_GROUPS")) wave_groups = std::max(1, atoi(e));
    wave_groups = std::min(wave_groups, ngroups);
    const int64_t positions = (int64_t)std::max(N, sk->n_int) * wave_groups;
    const size_t need = per_group * wave_groups + engine_bytes(wave_groups, positions) + 65536 +
                        (size_t)wave_groups * 16;
    BC_TRY(g->work.reserve(need));
    for (int32_t g0 = 0; g0 < ngroups; g0 += wave_groups) {
        g->work.used = 0;
        const int32_t gn = std::min(wave_groups, ngroups - g0);
        std::vector<GroupDesc> groups(gn);
        for (int32_t j = 0; j < gn; ++j) {
            GroupDesc& G = groups[j];
            G.g.row_ptr = sk->d_row_ptr;
            G.g.col = sk->d_col;
            G.g.len = sk->d_len;
            G.g.mult = sk_mult(sk);
            G.g.nflag = sk->d_nflag;
            G.g.twin = sk->d_twin;
            G.g.arc = sk->d_arc;
            G.lo = 0;
            G.hi = N;
            G.arc_lo = 0;
            G.arcs = sk->m_arcs;
            G.ring_len = sk->max_len + 1;
            G.flags = gflags;
            G.trow = sk->d_trow;
            G.tcol = sk->d_tcol;
            G.tlen = sk->d_tlen;
            G.tsig = sk->d_tsig;
            G.tn = sk->n_int;
            const int32_t first = (g0 + j) * LANES;
            G.nsrc = std::min(LANES, nsrc - first);
            for (int b = 0; b < LANES; ++b) G.src[b] = b < G.nsrc ? sk->h_src[first + b] : -1;
        }
        BC_TRY(run_groups(g->work, s, groups, steps));
        BC_TRY(reduce_scores(s, g->work, groups, n, nullptr, nullptr, sk->d_out_idx, sk->d_out_which,
                             scale, out_dev, g0 > 0));
    }
    return BC_OK;
}

int sk_sssp_run(const bc_skeleton* sk, const int32_t* src, int32_t nsrc, int64_t* d, uint64_t* sigma) {
    bc_graph* g = const_cast<bc_graph*>(sk->graph);
    hipStream_t s = g->stream;
    const int32_t N = sk->n_sk;
    if (nsrc < 0 || (nsrc > 0 && !src)) return fail(BC_E_INVAL, "bad source list");
    // original id -> skeleton id
    std::vector<int32_t> nodes(N), idx(g->n, -1);
    if (N) BC_HIP(hipMemcpyAsync(nodes.data(), sk->d_nodes, (size_t)N * 4, hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    for (int32_t f = 0; f < N; ++f) idx[nodes[f]] = f;
    std::vector<int32_t> ssrc(nsrc);
    for (int32_t i = 0; i < nsrc; ++i) {
        if (src[i] < 0 || src[i] >= g->n || idx[src[i]] < 0)
            return fail(BC_E_INVAL, "source is not a skeleton node");
        ssrc[i] = idx[src[i]];
    }
    if (nsrc == 0 || N == 0) return BC_OK;
    if (resident_takes(N)) {
        // the groups of a Brandes_SK pass over these sources (with the Centrality pass
        // when the skeleton has tables), exporting each source's forward state
        const int32_t spg = resident_sources_per_group(nsrc);
        auto make = [&](int32_t g0, int32_t g1) {
            std::vector<GroupDesc> groups(g1 - g0);
            for (int32_t j = g0; j < g1; ++j) {
                GroupDesc& G = groups[j - g0];
                G.g.row_ptr = sk->d_row_ptr;
                G.g.col = sk->d_col;
                G.g.len = sk->d_len;
                G.g.mult = sk_mult(sk);
                G.g.nflag = sk->d_nflag;
                G.g.twin = sk->d_twin;
                G.g.arc = sk->d_arc;
                G.lo = 0;
                G.hi = N;
                G.arc_lo = 0;
                G.arcs = sk->m_arcs;
                G.ring_len = sk->max_len + 1;
                G.flags = GF_BACKWARD | (sk->n_int ? GF_CENT : 0u);
                G.trow = sk->d_trow;
                G.tcol = sk->d_tcol;
                G.tlen = sk->d_tlen;
                G.tsig = sk->d_tsig;
                G.t_lo = 0;
                G.tn = sk->n_int;
                const int32_t first = j * spg;
                G.nsrc = std::min(spg, nsrc - first);
                for (int b = 0; b < LANES; ++b) G.src[b] = b < G.nsrc ? ssrc[first + b] : -1;
            }
            return groups;
        };
        auto bind = [](Arena&, std::vector<GroupDesc>&) -> int { return BC_OK; };
        return run_exported(s, g->work, N, nsrc, spg, make, bind, 0, d, sigma);
    }
    const int64_t steps = max_steps_bound(N, LANES, sk->max_dist);
    std::vector<uint32_t> ht((size_t)N * LANES);
    std::vector<uint64_t> hs((size_t)N * LANES);
    for (int32_t g0 = 0; g0 * LANES < nsrc; ++g0) {
        std::vector<GroupDesc> groups(1);
        GroupDesc& G = groups[0];
        G.hi = N;
        G.arcs = sk->m_arcs;
        G.nsrc = LANES;
        G.ring_len = sk->max_len + 1;
        BC_TRY(g->work.reserve(group_bytes(G, steps) + engine_bytes(1, N) + 65536));
        G.g.row_ptr = sk->d_row_ptr;
        G.g.col = sk->d_col;
        G.g.len = sk->d_len;
        G.g.mult = sk_mult(sk);
        G.lo = 0;
        G.hi = N;
        const int32_t first = g0 * LANES;
        G.nsrc = std::min(LANES, nsrc - first);
        for (int b = 0; b < LANES; ++b) G.src[b] = b < G.nsrc ? ssrc[first + b] : -1;
        BC_TRY(run_groups(g->work, s, groups, steps));
        BC_HIP(hipMemcpyAsync(ht.data(), G.dist, ht.size() * 4, hipMemcpyDeviceToHost, s));
        BC_HIP(hipMemcpyAsync(hs.data(), G.sigma, hs.size() * 8, hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        for (int b = 0; b < G.nsrc; ++b) {
            const int64_t r = first + b;
            for (int32_t v = 0; v < N; ++v) {
                const uint32_t t = ht[(size_t)v * LANES + b];
                if (d) d[r * N + v] = (t == INF32) ? -1 : (int64_t)t;
                if (sigma) sigma[r * N + v] = (t == INF32) ? 0 : hs[(size_t)v * LANES + b];
            }
        }
    }
    return BC_OK;
}

}  // namespace bcpp

using namespace bcpp;

extern "C" {

int bc_partition_sk(const bc_graph* g, const int32_t* part, int32_t k, const int32_t* S, int32_t nS,
                    bc_skeleton** out) {
    if (!g || !out) return fail(BC_E_INVAL, "null graph or output handle");
    *out = nullptr;
    return partition_impl(g, part, k, S, nS, out, false);
}

void bc_skeleton_destroy(bc_skeleton* sk) { delete sk; }

int bc_skeleton_stats(const bc_skeleton* sk, bc_sk_stats* out) {
    if (!sk || !out) return fail(BC_E_INVAL, "null skeleton or output");
    *out = sk->stats;
    return BC_OK;
}

int bc_skeleton_export(const bc_skeleton* sk, int32_t* nodes, int64_t* row_ptr, int32_t* col,
                       uint32_t* len, uint64_t* mult, int32_t* n_int, int32_t* tab_node,
                       int64_t* tab_ptr, int32_t* tab_f, uint32_t* tab_d, uint64_t* tab_sigma) {
    if (!sk) return fail(BC_E_INVAL, "null skeleton");
    hipStream_t s = sk->graph->stream;
    auto d2h = [&](void* h, const void* d, size_t b) -> int {
        if (h && b) BC_HIP(hipMemcpyAsync(h, d, b, hipMemcpyDeviceToHost, s));
        return BC_OK;
    };
    BC_TRY(d2h(nodes, sk->d_nodes, (size_t)sk->n_sk * 4));
    BC_TRY(d2h(row_ptr, sk->d_row_ptr, (size_t)(sk->n_sk + 1) * 8));
    BC_TRY(d2h(col, sk->d_col, (size_t)sk->m_arcs * 4));
    BC_TRY(d2h(len, sk->d_len, (size_t)sk->m_arcs * 4));
    BC_TRY(d2h(mult, sk->d_mult, (size_t)sk->m_arcs * 8));
    BC_TRY(d2h(tab_node, sk->d_tnode, (size_t)sk->n_int * 4));
    BC_TRY(d2h(tab_ptr, sk->d_trow, (size_t)(sk->n_int + 1) * 8));
    BC_TRY(d2h(tab_f, sk->d_tcol, (size_t)sk->t_nnz * 4));
    BC_TRY(d2h(tab_d, sk->d_tlen, (size_t)sk->t_nnz * 4));
    BC_TRY(d2h(tab_sigma, sk->d_tsig, (size_t)sk->t_nnz * 8));
    BC_HIP(hipStreamSynchronize(s));
    if (n_int) *n_int = sk->n_int;
    return BC_OK;
}

int bc_skeleton_sssp_counts(const bc_skeleton* sk, const int32_t* src, int32_t nsrc, int64_t* d,
                            uint64_t* sigma) {
    if (!sk) return fail(BC_E_INVAL, "null skeleton");
    return sk_sssp_run(sk, src, nsrc, d, sigma);
}

int bc_brandes_pp(const bc_graph* gc, const bc_skeleton* sk, uint32_t flags, double* bc_out) {
    if (!gc || !sk || !bc_out) return fail(BC_E_INVAL, "null graph, skeleton or output");
    if (sk->graph != gc) return fail(BC_E_INVAL, "skeleton was built for another graph");
    bc_graph* g = const_cast<bc_graph*>(gc);
    if (g->n == 0) return BC_OK;
    BC_TRY(g->out.reserve((size_t)g->n * 8 + 256));
    double* d_out = g->out.take<double>(g->n);
    BC_TRY(pp_run(g, sk, flags, d_out));
    BC_HIP(hipMemcpyAsync(bc_out, d_out, (size_t)g->n * 8, hipMemcpyDeviceToHost, g->stream));
    BC_HIP(hipStreamSynchronize(g->stream));
    return BC_OK;
}

int bc_brandes_pp_dev(const bc_graph* gc, const bc_skeleton* sk, uint32_t flags, double* bc_out_dev) {
    if (!gc || !sk || !bc_out_dev) return fail(BC_E_INVAL, "null graph, skeleton or output");
    if (sk->graph != gc) return fail(BC_E_INVAL, "skeleton was built for another graph");
    return pp_run(gc, sk, flags, bc_out_dev);
}

}  // extern "C"
