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
// Thread = (group, lane); the lanes of a wave read one state row together.
__global__ void k_clique_count(const GroupDesc* __restrict__ desc, const DskInfo* __restrict__ info,
                               int32_t ngroups, int32_t* __restrict__ cdeg) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= ngroups) return;
    const DskInfo I = info[g];
    if (lane >= I.nsrc) return;
    const uint64_t* sig = desc[g].sigma;
    const int32_t own = I.fl0 + lane;
    int32_t cnt = 0;
    for (int32_t j = 0; j < I.nf; ++j)
        cnt += (j != own && sig[(int64_t)j * 64 + lane] != 0) ? 1 : 0;
    cdeg[I.sk_base + own] = cnt;
}

__global__ void k_clique_fill(const GroupDesc* __restrict__ desc, const DskInfo* __restrict__ info,
                              int32_t ngroups, const int64_t* __restrict__ row_ptr,
                              const int32_t* __restrict__ rdeg, int32_t* __restrict__ col,
                              uint32_t* __restrict__ len, uint64_t* __restrict__ mult,
                              uint32_t* __restrict__ maxlen) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= ngroups) return;
    const DskInfo I = info[g];
    if (lane >= I.nsrc) return;
    const GroupDesc& G = desc[g];
    const int32_t own = I.fl0 + lane;
    const int32_t f = I.sk_base + own;
    int64_t pos = row_ptr[f] + rdeg[f];
    uint32_t mx = 0;
    for (int32_t j = 0; j < I.nf; ++j) {
        const uint64_t s = G.sigma[(int64_t)j * 64 + lane];
        if (j == own || s == 0) continue;
        const uint32_t d = G.dist[(int64_t)j * 64 + lane];
        col[pos] = I.sk_base + j;
        len[pos] = d;
        mult[pos] = s;
        mx = max(mx, d);
        ++pos;
    }
    if (mx) atomicMax(maxlen, mx);
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

int SkBuild::prepare(const bc_graph* gr, const int32_t* part, int32_t k, const int32_t* Sx,
                     int32_t nS, bool given_singletons) {
    PhaseTrace tr("prepare");
    g = gr;
    n = g->n;
    if (n > 0 && !part) return fail(BC_E_INVAL, "null partition");
    if (n > 0 && k < 1) return fail(BC_E_INVAL, "k must be >= 1");
    for (int32_t v = 0; v < n; ++v)
        if (part[v] < 0 || part[v] >= k)
            return fail(BC_E_INVAL, "partition label out of range at node " + std::to_string(v));
    BC_TRY(validate_targets(n, Sx, nS));
    S.assign(Sx, Sx + nS);
    const int64_t* rp = g->h_row_ptr.data();
    const int32_t* cl = g->h_col.data();
    const int32_t* wt = g->h_w.empty() ? nullptr : g->h_w.data();
    weighted = wt != nullptr;

    // ---- P' (Step 1, "Target nodes in the skeleton") and frontiers (Sec. 4)
    nlab = (int64_t)k + (given_singletons ? 0 : nS);
    lab.assign(part, part + n);
    is_t.assign(n, 0);
    for (int32_t i = 0; i < nS; ++i) {
        if (!given_singletons) lab[S[i]] = k + i;
        is_t[S[i]] = 1;
    }
    fr.assign(n, 0);
    parallel_for(n, 16384, [&](int64_t a, int64_t b) {
        for (int64_t v = a; v < b; ++v)
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
                if (lab[cl[e]] != lab[v]) {
                    fr[v] = 1;
                    break;
                }
    });
    tr.mark("validate, P', frontiers");
    // ---- renumbering: parts contiguous, frontier first
    psize.assign(nlab + 1, 0);
    pnf.assign(nlab, 0);
    for (int32_t v = 0; v < n; ++v) {
        psize[lab[v]]++;
        pnf[lab[v]] += fr[v];
    }
    poff.assign(nlab + 1, 0);
    fbase.assign(nlab + 1, 0);
    for (int64_t p = 0; p < nlab; ++p) {
        poff[p + 1] = poff[p] + psize[p];
        fbase[p + 1] = fbase[p] + pnf[p];
    }
    std::vector<int64_t> fcur(nlab), icur(nlab);
    for (int64_t p = 0; p < nlab; ++p) {
        fcur[p] = poff[p];
        icur[p] = poff[p] + pnf[p];
    }
    nid.assign(n, 0);
    old.assign(n, 0);
    for (int32_t v = 0; v < n; ++v) {
        const int32_t p = lab[v];
        const int64_t r = fr[v] ? fcur[p]++ : icur[p]++;
        nid[v] = (int32_t)r;
        old[r] = v;
    }
    nsk = (int32_t)fbase[nlab];
    auto skid = [&](int32_t v) -> int32_t { return (int32_t)(fbase[lab[v]] + (nid[v] - poff[lab[v]])); };

    tr.mark("renumbering");
    // ---- intra-part CSR (renumbered) and the cut arcs R by skeleton id: count per
    // renumbered row, prefix sums, then fill (rows in parallel)
    irp.assign(n + 1, 0);
    rptr.assign(nsk + 1, 0);
    parallel_for(n, 8192, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) {
            const int32_t v = old[r];
            int64_t ci = 0, cr = 0;
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e) (lab[cl[e]] == lab[v] ? ci : cr)++;
            irp[r + 1] = ci;
            if (fr[v]) rptr[skid(v) + 1] = cr;
        }
    });
    for (int32_t r = 0; r < n; ++r) irp[r + 1] += irp[r];
    for (int32_t f = 0; f < nsk; ++f) rptr[f + 1] += rptr[f];
    icol.resize((size_t)irp[n]);
    iw.resize(wt ? (size_t)irp[n] : 0);
    rcol.resize((size_t)rptr[nsk]);
    rw.resize((size_t)rptr[nsk]);
    parallel_for(n, 8192, [&](int64_t a, int64_t b) {
        std::vector<std::pair<int32_t, uint32_t>> tmp;
        for (int64_t r = a; r < b; ++r) {
            const int32_t v = old[r];
            int64_t oi = irp[r];
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
                const int32_t u = cl[e];
                if (lab[u] == lab[v]) {
                    icol[oi] = nid[u];
                    if (wt) iw[oi] = (uint32_t)wt[e];
                    ++oi;
                }
            }
            if (!fr[v]) continue;
            // cut arcs of a frontier row, sorted by skeleton id (reverse arcs are found
            // by bisection)
            tmp.clear();
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
                const int32_t u = cl[e];
                if (lab[u] != lab[v]) tmp.push_back({skid(u), wt ? (uint32_t)wt[e] : 1u});
            }
            std::sort(tmp.begin(), tmp.end());
            int64_t o = rptr[skid(v)];
            for (auto& t : tmp) {
                rcol[o] = t.first;
                rw[o] = t.second;
                ++o;
            }
        }
    });
    nR = (int64_t)rcol.size();

    tr.mark("intra CSR, R arcs");
    // ---- Dijkstra_SK groups: every part with >= 2 nodes and a frontier
    groups.clear();
    info.clear();
    std::vector<int32_t> p_g0(nlab, 0), p_ng(nlab, 0);
    largest = kprime = clique_pairs = table_pairs = 0;
    for (int64_t p = 0; p < nlab; ++p) {
        if (psize[p] > 0) kprime++;
        largest = std::max(largest, psize[p]);
        if (psize[p] < 2 || pnf[p] == 0) continue;
        clique_pairs += pnf[p] * (pnf[p] - 1);
        table_pairs += pnf[p] * (psize[p] - pnf[p]);
        p_g0[p] = (int32_t)groups.size();
        for (int64_t c = 0; c < pnf[p]; c += LANES) {
            GroupDesc G;
            G.lo = (int32_t)poff[p];
            G.hi = (int32_t)(poff[p] + psize[p]);
            G.arcs = irp[G.hi] - irp[G.lo];
            G.flags = GF_RESTRICT | (wt ? 0u : GF_UNIT);
            G.ring_len = g->maxw + 1;
            G.nsrc = (int32_t)std::min<int64_t>(LANES, pnf[p] - c);
            for (int b = 0; b < LANES; ++b) G.src[b] = b < G.nsrc ? (int32_t)(poff[p] + c + b) : -1;
            groups.push_back(G);
            info.push_back({(int32_t)pnf[p], (int32_t)c, G.nsrc, (int32_t)fbase[p]});
        }
        p_ng[p] = (int32_t)groups.size() - p_g0[p];
    }
    // interior rows: non-frontier nodes of parts with groups, in renumbered order
    int_local.clear();
    int_g0.clear();
    int_ng.clear();
    int_node.clear();
    out_idx.assign(n, -1);
    out_which.assign(n, 0);
    for (int64_t p = 0; p < nlab; ++p) {
        if (p_ng[p] == 0) continue;
        for (int64_t r = poff[p] + pnf[p]; r < poff[p + 1]; ++r) {
            out_idx[old[r]] = (int32_t)int_local.size();
            out_which[old[r]] = 1;
            int_local.push_back((int32_t)(r - poff[p]));
            int_g0.push_back(p_g0[p]);
            int_ng.push_back(p_ng[p]);
            int_node.push_back(old[r]);
        }
    }
    for (int32_t v = 0; v < n; ++v)
        if (fr[v]) out_idx[v] = skid(v);
    nint = (int32_t)int_local.size();
    tr.mark("groups, interior rows");
    return BC_OK;
}

size_t SkBuild::temp_bytes() const {
    const int32_t ng = (int32_t)groups.size();
    size_t need = 0;
    for (const auto& G : groups) need += group_bytes(G, 0);
    need += (size_t)(n + 1) * 8 + icol.size() * 4 + iw.size() * 4 + (size_t)n +
            (size_t)(nsk + 1) * 8 * 2 + (size_t)nR * 8 + (size_t)nsk * 8 + (size_t)ng * sizeof(DskInfo) +
            (size_t)ng * sizeof(GroupDesc) + (size_t)nint * 16 + 64 * 256;
    return need;
}

size_t SkBuild::skeleton_bytes_bound() const {
    const int64_t M = nR + clique_pairs, T = table_pairs;
    return (size_t)(nsk + 1) * 8 + (size_t)M * (4 + 4 + 8 + 8) + (size_t)nsk + (size_t)(nint + 1) * 8 +
           (size_t)T * (4 + 4 + 8) + (size_t)nsk * 4 + (size_t)nint * 4 + (size_t)n * 5 + 32 * 256;
}

int SkBuild::upload(Arena& W, hipStream_t s) {
    const int32_t ng = (int32_t)groups.size();
    d_irp = W.take<int64_t>(n + 1);
    d_icol = W.take<int32_t>(std::max<size_t>(icol.size(), 1));
    d_iw = weighted ? W.take<uint32_t>(std::max<size_t>(iw.size(), 1)) : nullptr;
    d_blk = W.take<uint8_t>(std::max(n, 1));
    d_rptr = W.take<int64_t>(nsk + 1);
    d_rcol = W.take<int32_t>(std::max<int64_t>(nR, 1));
    d_rw = W.take<uint32_t>(std::max<int64_t>(nR, 1));
    d_rdeg = W.take<int32_t>(std::max(nsk, 1));
    d_cdeg = W.take<int32_t>(std::max(nsk, 1));
    d_info = W.take<DskInfo>(std::max(ng, 1));
    d_il = W.take<int32_t>(std::max(nint, 1));
    d_ig0 = W.take<int32_t>(std::max(nint, 1));
    d_ing = W.take<int32_t>(std::max(nint, 1));
    d_tdeg = W.take<int32_t>(std::max(nint, 1));
    d_maxlen = W.take<uint32_t>(1);
    d_desc = W.take<GroupDesc>(std::max(ng, 1));
    if (!d_irp || !d_icol || !d_blk || !d_rptr || !d_rcol || !d_rw || !d_rdeg || !d_cdeg || !d_info ||
        !d_il || !d_ig0 || !d_ing || !d_tdeg || !d_maxlen || !d_desc || (weighted && !d_iw))
        return fail(BC_E_NOMEM, "partition: workspace too small");
    for (auto& G : groups) {
        G.g.row_ptr = d_irp;
        G.g.col = d_icol;
        G.g.len = d_iw;
        G.g.nflag = d_blk;
        if (!group_alloc(W, G, 0)) return fail(BC_E_NOMEM, "partition: group state does not fit");
    }
    std::vector<uint8_t> blk(n);
    for (int32_t r = 0; r < n; ++r) blk[r] = fr[old[r]] ? (uint8_t)NF_BLOCKED : 0;
    std::vector<int32_t> rdeg(nsk);
    for (int32_t f = 0; f < nsk; ++f) rdeg[f] = (int32_t)(rptr[f + 1] - rptr[f]);
    auto h2d = [&](void* d, const void* h, size_t b) -> int {
        if (b) BC_HIP(hipMemcpyAsync(d, h, b, hipMemcpyHostToDevice, s));
        return BC_OK;
    };
    BC_TRY(h2d(d_irp, irp.data(), (size_t)(n + 1) * 8));
    BC_TRY(h2d(d_icol, icol.data(), icol.size() * 4));
    if (weighted) BC_TRY(h2d(d_iw, iw.data(), iw.size() * 4));
    BC_TRY(h2d(d_blk, blk.data(), n));
    BC_TRY(h2d(d_rptr, rptr.data(), (size_t)(nsk + 1) * 8));
    BC_TRY(h2d(d_rcol, rcol.data(), (size_t)nR * 4));
    BC_TRY(h2d(d_rw, rw.data(), (size_t)nR * 4));
    BC_TRY(h2d(d_rdeg, rdeg.data(), (size_t)nsk * 4));
    BC_TRY(h2d(d_info, info.data(), (size_t)ng * sizeof(DskInfo)));
    BC_TRY(h2d(d_il, int_local.data(), (size_t)nint * 4));
    BC_TRY(h2d(d_ig0, int_g0.data(), (size_t)nint * 4));
    BC_TRY(h2d(d_ing, int_ng.data(), (size_t)nint * 4));
    BC_TRY(h2d(d_desc, groups.data(), (size_t)ng * sizeof(GroupDesc)));
    if (nsk) BC_HIP(hipMemsetAsync(d_cdeg, 0, (size_t)nsk * 4, s));
    BC_HIP(hipMemsetAsync(d_maxlen, 0, 4, s));
    // the host copies above are staged by the runtime; wait so the caller may reuse them
    BC_HIP(hipStreamSynchronize(s));
    return BC_OK;
}

int SkBuild::assemble(Arena& W, hipStream_t s, bc_skeleton* sk,
                      const std::function<int(size_t, Arena*&)>& get_store) {
    (void)W;
    const int32_t ng = (int32_t)groups.size();
    if (ng > 0) {
        KTimer kt(BC_K_OTHER, s);
        hipLaunchKernelGGL(k_clique_count, dim3((ng + 3) / 4), dim3(256), 0, s, d_desc, d_info, ng, d_cdeg);
        if (nint)
            hipLaunchKernelGGL(k_table, dim3((nint + 3) / 4), dim3(256), 0, s, d_desc, d_info, nint, d_il,
                               d_ig0, d_ing, d_tdeg, nullptr, nullptr, nullptr, nullptr);
    }
    BC_HIP(hipGetLastError());
    std::vector<int32_t> cdeg(nsk, 0), tdeg(nint, 0);
    if (nsk) BC_HIP(hipMemcpyAsync(cdeg.data(), d_cdeg, (size_t)nsk * 4, hipMemcpyDeviceToHost, s));
    if (nint && ng) BC_HIP(hipMemcpyAsync(tdeg.data(), d_tdeg, (size_t)nint * 4, hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> srow(nsk + 1, 0), trow(nint + 1, 0);
    int64_t ncl = 0;
    for (int32_t f = 0; f < nsk; ++f) {
        srow[f + 1] = srow[f] + (rptr[f + 1] - rptr[f]) + cdeg[f];
        ncl += cdeg[f];
    }
    for (int32_t i = 0; i < nint; ++i) trow[i + 1] = trow[i] + tdeg[i];
    const int64_t M = srow[nsk], T = trow[nint];

    // ---- the skeleton's own store
    const size_t sbytes = (size_t)(nsk + 1) * 8 + (size_t)M * (4 + 4 + 8 + 8) + (size_t)nsk +
                          (size_t)(nint + 1) * 8 + (size_t)T * (4 + 4 + 8) + (size_t)nsk * 4 +
                          (size_t)nint * 4 + (size_t)n * 5 + 32 * 256;
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
    if (!sk->d_out_which) return fail(BC_E_NOMEM, "skeleton store too small");
    auto skid = [&](int32_t v) -> int32_t { return (int32_t)(fbase[lab[v]] + (nid[v] - poff[lab[v]])); };
    std::vector<uint8_t> sflag(nsk, 0);
    std::vector<int32_t> nodes(nsk);
    for (int32_t r = 0; r < n; ++r) {
        const int32_t v = old[r];
        if (!fr[v]) continue;
        const int32_t f = skid(v);
        nodes[f] = v;
        if (is_t[v]) sflag[f] = (uint8_t)NF_TARGET;
    }
    auto h2d = [&](void* d, const void* h, size_t b) -> int {
        if (b) BC_HIP(hipMemcpyAsync(d, h, b, hipMemcpyHostToDevice, s));
        return BC_OK;
    };
    BC_TRY(h2d(sk->d_row_ptr, srow.data(), (size_t)(nsk + 1) * 8));
    BC_TRY(h2d(sk->d_trow, trow.data(), (size_t)(nint + 1) * 8));
    BC_TRY(h2d(sk->d_nflag, sflag.data(), nsk));
    BC_TRY(h2d(sk->d_nodes, nodes.data(), (size_t)nsk * 4));
    BC_TRY(h2d(sk->d_tnode, int_node.data(), (size_t)nint * 4));
    BC_TRY(h2d(sk->d_out_idx, out_idx.data(), (size_t)n * 4));
    BC_TRY(h2d(sk->d_out_which, out_which.data(), n));
    {
        KTimer kt(BC_K_OTHER, s);
        if (nsk)
            hipLaunchKernelGGL(k_fill_r, dim3((nsk + 255) / 256), dim3(256), 0, s, nsk, d_rptr, d_rcol, d_rw,
                               sk->d_row_ptr, sk->d_col, sk->d_len, sk->d_mult);
        if (ng) {
            hipLaunchKernelGGL(k_clique_fill, dim3((ng + 3) / 4), dim3(256), 0, s, d_desc, d_info, ng,
                               sk->d_row_ptr, d_rdeg, sk->d_col, sk->d_len, sk->d_mult, d_maxlen);
            if (nint)
                hipLaunchKernelGGL(k_table, dim3((nint + 3) / 4), dim3(256), 0, s, d_desc, d_info, nint, d_il,
                                   d_ig0, d_ing, nullptr, sk->d_trow, sk->d_tcol, sk->d_tlen, sk->d_tsig);
        }
        if (nsk)
            hipLaunchKernelGGL(k_sk_twin, dim3((nsk + 3) / 4), dim3(256), 0, s, nsk, sk->d_row_ptr, d_rdeg,
                               sk->d_col, sk->d_twin);
    }
    BC_HIP(hipGetLastError());
    uint32_t clique_max = 0;
    BC_HIP(hipMemcpyAsync(&clique_max, d_maxlen, 4, hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    uint32_t rmax = 1;
    for (uint32_t x : rw) rmax = std::max(rmax, x);

    sk->graph = g;
    sk->n = n;
    sk->max_len = (int32_t)std::max(rmax, clique_max);
    // Brandes_SK sources: targets that have a neighbour (isolated targets reach nobody)
    sk->h_src.clear();
    for (int32_t v : S)
        if (fr[v]) sk->h_src.push_back(skid(v));
    sk->h_row_ptr = srow;
    sk->h_out_idx = out_idx;
    sk->h_out_which = out_which;
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

int partition_impl(const bc_graph* g, const int32_t* part, int32_t k, const int32_t* S, int32_t nS,
                   bc_skeleton** out, bool given_singletons) {
    PhaseTrace tr("partition");
    SkBuild b;
    BC_TRY(b.prepare(g, part, k, S, nS, given_singletons));
    tr.mark("prepare (host)");
    bc_graph* gm = const_cast<bc_graph*>(g);
    Arena& W = gm->work;
    hipStream_t s = g->stream;
    int64_t positions = 0;
    for (auto& G : b.groups) positions += (int64_t)G.hi - G.lo;
    // Dijkstra_SK groups run on the resident kernel (parts larger than LDS keep their
    // one-source state in device memory), or on the engine when it is switched off
    bool res = !b.groups.empty();
    size_t extra = 0;
    for (auto& G : b.groups) {
        res = res && resident_takes((int64_t)G.hi - G.lo);
        if ((int64_t)G.hi - G.lo > resident_max_range()) extra += (size_t)(G.hi - G.lo) * 12 + 512;
    }
    extra += resident_launch_bytes(b.groups.size());
    BC_TRY(W.reserve(b.temp_bytes() + std::max(extra, engine_bytes(std::max<int32_t>((int32_t)b.groups.size(), 1),
                                                                   positions))));
    BC_TRY(b.upload(W, s));
    tr.mark("upload");
    if (res) {
        for (auto& G : b.groups) {
            if ((int64_t)G.hi - G.lo <= resident_max_range()) continue;
            G.gdist = W.take<uint32_t>((size_t)(G.hi - G.lo));
            G.gsig = W.take<uint64_t>((size_t)(G.hi - G.lo));
            if (!G.gdist || !G.gsig) return fail(BC_E_NOMEM, "partition: workspace too small");
        }
        BC_TRY(run_resident(s, W, b.groups));
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
    const int32_t nsrc = (int32_t)sk->h_src.size();
    const int32_t spg = resident_sources_per_group(nsrc);
    const int32_t ngroups = (nsrc + spg - 1) / spg;
    std::vector<GroupDesc> groups(ngroups);
    for (int32_t j = 0; j < ngroups; ++j) {
        GroupDesc& G = groups[j];
        G.g.row_ptr = sk->d_row_ptr;
        G.g.col = sk->d_col;
        G.g.len = sk->d_len;
        G.g.mult = sk_mult(sk);
        G.g.nflag = sk->d_nflag;
        G.lo = 0;
        G.hi = sk->n_sk;
        G.flags = GF_BACKWARD | (sk->n_int ? GF_CENT : 0u);
        G.trow = sk->d_trow;
        G.tcol = sk->d_tcol;
        G.tlen = sk->d_tlen;
        G.tsig = sk->d_tsig;
        G.t_lo = 0;
        G.tn = sk->n_int;
        const int32_t first = j * spg;
        G.nsrc = std::min(spg, nsrc - first);
        for (int b = 0; b < LANES; ++b) G.src[b] = b < G.nsrc ? sk->h_src[first + b] : -1;
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
