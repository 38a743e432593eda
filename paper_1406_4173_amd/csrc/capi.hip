// C-ABI entry points: errors, graph handles and validation, plain target-set Brandes,
// path counts, and the measurement hooks.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>

#include "engine.h"
#include "graph.h"

namespace bcpp {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// ------------------------------------------------------------------ arena ------

int Arena::reserve(size_t bytes) {
    bytes = (bytes + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
    if (limit && bytes > limit) return fail(BC_E_NOMEM, "workspace exceeds the configured budget");
    if (bytes <= cap) {
        used = 0;
        return BC_OK;
    }
    if (!owning) return fail(BC_E_NOMEM, "workspace view too small");
    release();
    hipError_t e = hipMalloc((void**)&base, bytes);
    if (e != hipSuccess) {
        base = nullptr;
        (void)hipGetLastError();
        return fail(BC_E_NOMEM, "hipMalloc of " + std::to_string(bytes >> 20) + " MiB failed");
    }
    cap = bytes;
    used = 0;
    return BC_OK;
}

void Arena::release() {
    if (base && owning) (void)hipFree(base);
    base = nullptr;
    cap = used = 0;
}

// -------------------------------------------------------------- profiler -------

Profiler& profiler() {
    static Profiler p;
    return p;
}

hipEvent_t Profiler::get_event() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void Profiler::begin(int kind, hipStream_t s, hipEvent_t* a) {
    (void)kind;
    *a = get_event();
    if (*a) (void)hipEventRecord(*a, s);
}

void Profiler::end(int kind, hipStream_t s, hipEvent_t a) {
    hipEvent_t b = get_event();
    if (!b) return;
    (void)hipEventRecord(b, s);
    pending.push_back({kind, a, b});
    if (pending.size() > 4096) collect();
}

void Profiler::collect() {
    for (auto& p : pending) {
        float ms_ = 0.f;
        (void)hipEventSynchronize(p.b);
        if (hipEventElapsedTime(&ms_, p.a, p.b) == hipSuccess) {
            launches[p.kind] += 1;
            ms[p.kind] += ms_;
        }
        pool.push_back(p.a);
        pool.push_back(p.b);
    }
    pending.clear();
}

// ----------------------------------------------------------- small kernels -----

__global__ void k_mark_targets(const int32_t* __restrict__ S, int32_t nS,
                               uint8_t* __restrict__ flag) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nS) flag[S[i]] = (uint8_t)NF_TARGET;
}

// Zero bytes [p, p + bytes): 16-byte stores where the address is aligned, bytes at the
// ends. (A fill kernel rather than a memset, so that a captured graph may hold it.)
__global__ void k_zero_bytes(unsigned char* __restrict__ p, int64_t head, int64_t nvec, int64_t bytes) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride)
        reinterpret_cast<uint4*>(p + head)[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes; i += stride)
        if (i < head || i >= head + nvec * 16) p[i] = 0;
}

int zero_device(hipStream_t s, void* p, size_t bytes) {
    if (!bytes) return BC_OK;
    unsigned char* c = (unsigned char*)p;
    const int64_t head = std::min<int64_t>((int64_t)bytes, (int64_t)((16 - ((uintptr_t)c & 15)) & 15));
    const int64_t nvec = ((int64_t)bytes - head) / 16;
    const int64_t work = std::max<int64_t>(nvec, std::min<int64_t>((int64_t)bytes, 4096));
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 1024));
    hipLaunchKernelGGL(k_zero_bytes, dim3(grid), dim3(256), 0, s, c, head, nvec, (int64_t)bytes);
    BC_HIP(hipGetLastError());
    return BC_OK;
}

// ------------------------------------------------------------- validation ------

int validate_csr(const bc_csr* g, int32_t* maxw_out) {
    if (!g) return fail(BC_E_INVAL, "null graph");
    if (g->n < 0 || g->nnz < 0) return fail(BC_E_INVAL, "negative size");
    if (g->n > 0 && !g->row_ptr) return fail(BC_E_INVAL, "null row_ptr");
    if (g->nnz > 0 && !g->col) return fail(BC_E_INVAL, "null col");
    const int32_t n = g->n;
    if (n == 0) {
        if (g->nnz != 0) return fail(BC_E_INVAL, "arcs in an empty graph");
        *maxw_out = 1;
        return BC_OK;
    }
    if (g->row_ptr[0] != 0 || g->row_ptr[n] != g->nnz)
        return fail(BC_E_INVAL, "row_ptr must start at 0 and end at nnz");
    int32_t maxw = 1;
    for (int32_t u = 0; u < n; ++u) {
        const int64_t a = g->row_ptr[u], b = g->row_ptr[u + 1];
        if (b < a) return fail(BC_E_INVAL, "row_ptr decreases at row " + std::to_string(u));
        for (int64_t e = a; e < b; ++e) {
            const int32_t v = g->col[e];
            if (v < 0 || v >= n) return fail(BC_E_INVAL, "column out of range at arc " + std::to_string(e));
            if (v == u) return fail(BC_E_INVAL, "self-loop at node " + std::to_string(u));
            if (e > a && g->col[e - 1] >= v)
                return fail(BC_E_INVAL, "row " + std::to_string(u) + " unsorted or has a duplicate");
            if (g->w) {
                if (g->w[e] < 1) return fail(BC_E_INVAL, "weight < 1 at arc " + std::to_string(e));
                maxw = std::max(maxw, g->w[e]);
            }
        }
    }
    // symmetry: every arc u->v has a twin v->u of the same weight
    for (int32_t u = 0; u < n; ++u) {
        for (int64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
            const int32_t v = g->col[e];
            const int32_t* b0 = g->col + g->row_ptr[v];
            const int32_t* b1 = g->col + g->row_ptr[v + 1];
            const int32_t* f = std::lower_bound(b0, b1, u);
            if (f == b1 || *f != u)
                return fail(BC_E_INVAL, "asymmetric: arc " + std::to_string(u) + "->" +
                                            std::to_string(v) + " has no twin");
            if (g->w && g->w[f - g->col] != g->w[e])
                return fail(BC_E_INVAL, "asymmetric weight on edge " + std::to_string(u) + "-" +
                                            std::to_string(v));
        }
    }
    if ((int64_t)(n - 1) * (int64_t)maxw >= ((int64_t)1 << 31))
        return fail(BC_E_INVAL, "(n-1) * max weight must stay below 2^31");
    *maxw_out = maxw;
    return BC_OK;
}

int validate_targets(int32_t n, const int32_t* S, int32_t nS) {
    if (nS < 0) return fail(BC_E_INVAL, "negative target count");
    if (nS > 0 && !S) return fail(BC_E_INVAL, "null target array");
    std::vector<uint8_t> seen(std::max(n, 1), 0);
    for (int32_t i = 0; i < nS; ++i) {
        const int32_t s = S[i];
        if (s < 0 || s >= n) return fail(BC_E_INVAL, "target " + std::to_string(s) + " out of range");
        if (seen[s]) return fail(BC_E_INVAL, "target " + std::to_string(s) + " repeated");
        seen[s] = 1;
    }
    return BC_OK;
}

int64_t max_steps_bound(int64_t range, int32_t lanes, int64_t max_dist) {
    // distinct distances settled by one group: at most one per (node, lane) and at
    // most the number of distance values 0..max_dist
    return std::min<int64_t>(range * std::max(lanes, 1), max_dist + 1) + 1;
}

size_t state_budget() {
    static size_t b = 0;
    if (!b) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = (size_t)8 << 30;
        b = std::min<size_t>(fr / 2, (size_t)48 << 30);
        if (const char* e = getenv("BCPP_STATE_BUDGET_MB")) b = (size_t)atoll(e) << 20;
    }
    return b;
}

// ---------------------------------------------------------- graph handles ------

int graph_create(const bc_csr* csr, hipStream_t stream, bc_graph** out) {
    int32_t maxw = 1;
    BC_TRY(validate_csr(csr, &maxw));
    auto* g = new bc_graph();
    g->n = csr->n;
    g->nnz = csr->nnz;
    g->maxw = maxw;
    g->unit = (csr->w == nullptr);
    g->stream = stream;
    g->h_row_ptr.assign(csr->row_ptr, csr->row_ptr + (csr->n + 1));
    if (csr->nnz) g->h_col.assign(csr->col, csr->col + csr->nnz);
    if (csr->w && csr->nnz) g->h_w.assign(csr->w, csr->w + csr->nnz);
    auto cleanup = [&](int rc) {
        delete g;
        return rc;
    };
    // reverse-arc index of every arc (rows are sorted, so a binary search finds it)
    std::vector<int64_t> twin(g->nnz);
    for (int32_t u = 0; u < g->n; ++u)
        for (int64_t e = csr->row_ptr[u]; e < csr->row_ptr[u + 1]; ++e) {
            const int32_t v = csr->col[e];
            const int32_t* b0 = csr->col + csr->row_ptr[v];
            const int32_t* b1 = csr->col + csr->row_ptr[v + 1];
            twin[e] = std::lower_bound(b0, b1, u) - csr->col;
        }
    // packed arc records: {head, length, reverse arc, multiplicity 1}
    const bool pack = g->nnz > 0 && g->nnz < ((int64_t)1 << 31);
    std::vector<ArcRec> arcs(pack ? (size_t)g->nnz : 0);
    for (int64_t e = 0; pack && e < g->nnz; ++e)
        arcs[(size_t)e] = ArcRec{(uint32_t)csr->col[e], csr->w ? (uint32_t)csr->w[e] : 1u, (uint32_t)twin[e], 1u};
    size_t bytes = (size_t)(g->n + 1) * 8 + (size_t)g->nnz * (4 * (g->unit ? 1 : 2) + 8 + (pack ? 16 : 0)) + 4096;
    int rc = g->store.reserve(bytes);
    if (rc) return cleanup(rc);
    g->d_row_ptr = g->store.take<int64_t>(g->n + 1);
    g->d_col = g->store.take<int32_t>(std::max<int64_t>(g->nnz, 1));
    if (!g->unit) g->d_len = g->store.take<uint32_t>(std::max<int64_t>(g->nnz, 1));
    g->d_twin = g->store.take<int64_t>(std::max<int64_t>(g->nnz, 1));
    if (pack) g->d_arc = g->store.take<ArcRec>((size_t)g->nnz);
    if (hipMemcpyAsync(g->d_row_ptr, csr->row_ptr, (size_t)(g->n + 1) * 8, hipMemcpyHostToDevice, stream) ||
        (g->nnz && hipMemcpyAsync(g->d_col, csr->col, (size_t)g->nnz * 4, hipMemcpyHostToDevice, stream)) ||
        (!g->unit && g->nnz &&
         hipMemcpyAsync(g->d_len, csr->w, (size_t)g->nnz * 4, hipMemcpyHostToDevice, stream)) ||
        (g->nnz && hipMemcpyAsync(g->d_twin, twin.data(), (size_t)g->nnz * 8, hipMemcpyHostToDevice, stream)) ||
        (pack && hipMemcpyAsync(g->d_arc, arcs.data(), (size_t)g->nnz * 16, hipMemcpyHostToDevice, stream)) ||
        hipStreamSynchronize(stream)) {
        return cleanup(fail(BC_E_DEVICE, "graph upload failed"));
    }
    *out = g;
    return BC_OK;
}

// ------------------------------------------------------------ plain Brandes ----

// Plain target-set Brandes with the resident kernel: groups of
// resident_sources_per_group(nS) of the host-validated targets S (host copy) over the
// whole graph; S_dev (device copy or null) marks the targets. Scores go to out_dev.
// With grow, W is sized to run every group at once. Without, W keeps its capacity and
// the groups run in waves of as many as fit; each wave's scores are added to the
// previous waves' (the same groups and sources, so the same d, sigma and per-group
// dependencies; the sum of the group rows only regroups). Nothing here clears memory
// with a memset: fill kernels do.
int plain_resident(bc_graph* g, Arena& W, bool grow, const int32_t* S, int32_t nS, const int32_t* S_dev,
                   double scale, double* out_dev) {
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    const int32_t spg = resident_sources_per_group(nS);
    const int32_t ngroups = (nS + spg - 1) / spg;
    std::vector<GroupDesc> groups(ngroups);
    size_t per_group = 0;
    for (int32_t j = 0; j < ngroups; ++j) {
        GroupDesc& G = groups[j];
        G.lo = 0;
        G.hi = n;
        G.arc_lo = 0;
        G.arcs = g->nnz;
        G.flags = GF_BACKWARD;
        G.ring_len = g->maxw + 1;
        const int32_t first = j * spg;
        G.nsrc = std::min(spg, nS - first);
        for (int b = 0; b < LANES; ++b) G.src[b] = b < G.nsrc ? S[first + b] : -1;
        per_group = std::max(per_group, resident_group_bytes(G) + resident_launch_bytes(1) + 2 * 8);
    }
    // shared by all waves: target flags and (host targets) their device copy
    const size_t fixed = ((size_t)n + 255) / 256 * 256 + ((size_t)nS * 4 + 255) / 256 * 256 + 8 * 256 + 65536;
    if (grow) {
        BC_TRY(W.reserve(fixed + (size_t)ngroups * per_group));
    } else {
        W.reset();
        if (fixed + per_group > W.cap)
            return fail(BC_E_NOMEM, "plain: one source group over " + std::to_string(n) + " nodes needs " +
                                        std::to_string(fixed + per_group) + " bytes of workspace, more than the " +
                                        std::to_string(W.cap) + " available");
    }
    uint8_t* d_flag = W.take<uint8_t>(n);
    const int32_t* d_S = S_dev;
    if (!d_S) {
        int32_t* t = W.take<int32_t>(nS);
        if (!t) return fail(BC_E_NOMEM, "plain: workspace too small");
        BC_HIP(hipMemcpyAsync(t, S, (size_t)nS * 4, hipMemcpyHostToDevice, s));
        d_S = t;
    }
    if (!d_flag) return fail(BC_E_NOMEM, "plain: workspace too small");
    BC_TRY(zero_device(s, d_flag, (size_t)n));
    hipLaunchKernelGGL(k_mark_targets, dim3((nS + 255) / 256), dim3(256), 0, s, d_S, nS, d_flag);
    BC_HIP(hipGetLastError());
    for (GroupDesc& G : groups) {
        G.g.row_ptr = g->d_row_ptr;
        G.g.col = g->d_col;
        G.g.len = g->d_len;
        G.g.nflag = d_flag;
        G.g.twin = g->d_twin;
        G.g.arc = g->d_arc;
    }
    const size_t mark = W.used;
    const int32_t per_wave =
        (int32_t)std::max<size_t>(1, std::min<size_t>(ngroups, (W.cap - std::min(W.cap, mark + 65536)) / per_group));
    for (int32_t g0 = 0; g0 < ngroups; g0 += per_wave) {
        W.used = mark;
        std::vector<GroupDesc> wave(groups.begin() + g0, groups.begin() + std::min(ngroups, g0 + per_wave));
        for (GroupDesc& G : wave)
            if (!resident_alloc(W, G)) return fail(BC_E_NOMEM, "plain: workspace too small");
        BC_TRY(run_resident(s, W, wave));
        BC_TRY(reduce_scores(s, W, wave, n, nullptr, nullptr, nullptr, nullptr, scale, out_dev, g0 > 0));
    }
    return BC_OK;
}

int plain_run(bc_graph* g, const int32_t* S, int32_t nS, const int32_t* S_dev, uint32_t flags,
              double* out_dev) {
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    const double scale = (flags & BC_ORDERED) ? 1.0 : 0.5;
    if (n == 0) return BC_OK;
    if (nS < 2) {
        BC_TRY(zero_device(s, out_dev, (size_t)n * 8));
        BC_HIP(hipStreamSynchronize(s));
        return BC_OK;
    }
    if (!(flags & BC_ENGINE_ONLY) && resident_takes(n))
        return plain_resident(g, g->work, true, S, nS, S_dev, scale, out_dev);
    const int64_t max_dist = (int64_t)(n - 1) * g->maxw;
    const int64_t steps = max_steps_bound(n, LANES, max_dist);
    const int32_t ngroups = (nS + LANES - 1) / LANES;
    GroupDesc shape;
    shape.lo = 0;
    shape.hi = n;
    shape.arcs = g->nnz;
    shape.nsrc = LANES;
    shape.flags = GF_BACKWARD;
    shape.ring_len = g->maxw + 1;
    const size_t per_group = group_bytes(shape, steps);
    int32_t wave_groups = (int32_t)std::max<size_t>(1, state_budget() / std::max<size_t>(per_group, 1));
    if (const char* e = getenv("BCPP_MAX_GROUPS")) wave_groups = std::max(1, atoi(e));
    wave_groups = std::min(wave_groups, ngroups);
    const size_t need = per_group * wave_groups + engine_bytes(wave_groups, (int64_t)n * wave_groups) +
                        (size_t)n + (size_t)nS * 4 + 65536 + (size_t)wave_groups * 16;
    BC_TRY(g->work.reserve(need));
    uint8_t* d_flag = g->work.take<uint8_t>(n);
    const int32_t* d_S = S_dev;
    if (!d_S) {
        int32_t* t = g->work.take<int32_t>(nS);
        BC_HIP(hipMemcpyAsync(t, S, (size_t)nS * 4, hipMemcpyHostToDevice, s));
        d_S = t;
    }
    BC_HIP(hipMemsetAsync(d_flag, 0, n, s));
    hipLaunchKernelGGL(k_mark_targets, dim3((nS + 255) / 256), dim3(256), 0, s, d_S, nS, d_flag);
    BC_HIP(hipGetLastError());
    const size_t mark = g->work.used;
    for (int32_t g0 = 0; g0 < ngroups; g0 += wave_groups) {
        g->work.used = mark;
        const int32_t gn = std::min(wave_groups, ngroups - g0);
        std::vector<GroupDesc> groups(gn);
        for (int32_t j = 0; j < gn; ++j) {
            GroupDesc& G = groups[j];
            G.g.row_ptr = g->d_row_ptr;
            G.g.col = g->d_col;
            G.g.len = g->d_len;
            G.g.nflag = d_flag;
            G.g.twin = g->d_twin;
            G.g.arc = g->d_arc;
            G.lo = 0;
            G.hi = n;
            G.arc_lo = 0;
            G.arcs = g->nnz;
            G.ring_len = g->maxw + 1;
            G.flags = GF_BACKWARD | (g->unit ? GF_UNIT : 0u);
            const int32_t first = (g0 + j) * LANES;
            G.nsrc = std::min(LANES, nS - first);
            for (int b = 0; b < LANES; ++b) G.src[b] = b < G.nsrc ? S[first + b] : -1;
        }
        BC_TRY(run_groups(g->work, s, groups, steps));
        BC_TRY(reduce_scores(s, g->work, groups, n, nullptr, nullptr, nullptr, nullptr, scale,
                             out_dev, g0 > 0));
    }
    return BC_OK;
}

// Run resident groups whose forward state is exported (GF_EXPORT) and copy d and sigma
// out, source-major over a range of n nodes, as the count entry points report them.
// Group j holds the call's sources [j * spg, j * spg + nsrc_j). The groups run in chunks
// whose output rows fit about 1 GiB. make(g0, g1) gives the descriptors of groups
// [g0, g1) without buffers; bind(W, groups), after the workspace is reserved, takes what
// the chunk's groups share from W and fills in their graph pointers.
int run_exported(hipStream_t s, Arena& W, int32_t n, int32_t nsrc, int32_t spg,
                 const std::function<std::vector<GroupDesc>(int32_t, int32_t)>& make,
                 const std::function<int(Arena&, std::vector<GroupDesc>&)>& bind, size_t bind_bytes,
                 int64_t* d, uint64_t* sigma) {
    const int32_t ngroups = (nsrc + spg - 1) / spg;
    const int64_t row_bytes = (int64_t)n * 12;
    const int32_t per_chunk = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>(ngroups, ((int64_t)1 << 30) / std::max<int64_t>(row_bytes * spg, 1)));
    std::vector<uint32_t> hd;
    std::vector<uint64_t> hs;
    for (int32_t g0 = 0; g0 < ngroups; g0 += per_chunk) {
        const int32_t g1 = std::min(ngroups, g0 + per_chunk);
        std::vector<GroupDesc> groups = make(g0, g1);
        int64_t rows = 0;
        size_t need = resident_launch_bytes(groups.size()) + bind_bytes + 4 * 65536;
        for (const GroupDesc& G : groups) {
            need += resident_group_bytes(G) + 2 * 256;
            rows += G.nsrc;
        }
        need += (size_t)rows * (size_t)row_bytes + 512;
        BC_TRY(W.reserve(need));
        BC_TRY(bind(W, groups));
        uint32_t* od = W.take<uint32_t>((size_t)std::max<int64_t>(rows * n, 1));
        uint64_t* os = W.take<uint64_t>((size_t)std::max<int64_t>(rows * n, 1));
        if (!od || !os) return fail(BC_E_NOMEM, "counts: workspace too small");
        int64_t r = 0;
        for (GroupDesc& G : groups) {
            G.flags |= GF_EXPORT;
            G.odist = od + r * n;
            G.osig = os + r * n;
            r += G.nsrc;
            if (!resident_alloc(W, G)) return fail(BC_E_NOMEM, "counts: workspace too small");
        }
        BC_TRY(run_resident(s, W, groups));
        hd.resize((size_t)(rows * n));
        hs.resize((size_t)(rows * n));
        if (rows * n) {
            BC_HIP(hipMemcpyAsync(hd.data(), od, hd.size() * 4, hipMemcpyDeviceToHost, s));
            BC_HIP(hipMemcpyAsync(hs.data(), os, hs.size() * 8, hipMemcpyDeviceToHost, s));
            BC_HIP(hipStreamSynchronize(s));
        }
        const int64_t first = (int64_t)g0 * spg * n;
        for (int64_t i = 0; i < rows * n; ++i) {
            const uint32_t t = hd[(size_t)i];
            if (d) d[first + i] = (t == INF32) ? -1 : (int64_t)t;
            if (sigma) sigma[first + i] = (t == INF32) ? 0 : hs[(size_t)i];
        }
    }
    return BC_OK;
}

// Path counts of G from the kernel that produces every score: the groups of a plain
// Brandes pass over the same sources (resident_sources_per_group each, the sources
// flagged as targets, forward and backward sweeps), which also export each source's
// forward state.
static int sssp_resident(bc_graph* g, const int32_t* src, int32_t nsrc, int64_t* d, uint64_t* sigma) {
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    const int32_t spg = resident_sources_per_group(nsrc);
    auto make = [&](int32_t g0, int32_t g1) {
        std::vector<GroupDesc> groups(g1 - g0);
        for (int32_t j = g0; j < g1; ++j) {
            GroupDesc& G = groups[j - g0];
            G.lo = 0;
            G.hi = n;
            G.arc_lo = 0;
            G.arcs = g->nnz;
            G.flags = GF_BACKWARD;
            G.ring_len = g->maxw + 1;
            const int32_t first = j * spg;
            G.nsrc = std::min(spg, nsrc - first);
            for (int b = 0; b < LANES; ++b) G.src[b] = b < G.nsrc ? src[first + b] : -1;
        }
        return groups;
    };
    auto bind = [&](Arena& W, std::vector<GroupDesc>& groups) -> int {
        uint8_t* d_flag = W.take<uint8_t>(n);
        int32_t* t = W.take<int32_t>(nsrc);
        if (!d_flag || !t) return fail(BC_E_NOMEM, "counts: workspace too small");
        BC_HIP(hipMemcpyAsync(t, src, (size_t)nsrc * 4, hipMemcpyHostToDevice, s));
        BC_HIP(hipMemsetAsync(d_flag, 0, n, s));
        hipLaunchKernelGGL(k_mark_targets, dim3((nsrc + 255) / 256), dim3(256), 0, s, t, nsrc, d_flag);
        BC_HIP(hipGetLastError());
        for (GroupDesc& G : groups) {
            G.g.row_ptr = g->d_row_ptr;
            G.g.col = g->d_col;
            G.g.len = g->d_len;
            G.g.nflag = d_flag;
            G.g.twin = g->d_twin;
            G.g.arc = g->d_arc;
        }
        return BC_OK;
    };
    return run_exported(s, g->work, n, nsrc, spg, make, bind, (size_t)n + (size_t)nsrc * 4 + 512, d, sigma);
}

int sssp_run(const bc_graph* gc, const int32_t* src, int32_t nsrc, int64_t* d, uint64_t* sigma) {
    bc_graph* g = const_cast<bc_graph*>(gc);
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    if (nsrc < 0 || (nsrc > 0 && !src)) return fail(BC_E_INVAL, "bad source list");
    for (int32_t i = 0; i < nsrc; ++i)
        if (src[i] < 0 || src[i] >= n) return fail(BC_E_INVAL, "source out of range");
    if (nsrc == 0 || n == 0) return BC_OK;
    if (resident_takes(n)) return sssp_resident(g, src, nsrc, d, sigma);
    const int64_t steps = max_steps_bound(n, LANES, (int64_t)(n - 1) * g->maxw);
    const int32_t ngroups = (nsrc + LANES - 1) / LANES;
    std::vector<uint32_t> ht((size_t)n * LANES);
    std::vector<uint64_t> hs((size_t)n * LANES);
    for (int32_t g0 = 0; g0 < ngroups; ++g0) {
        std::vector<GroupDesc> groups(1);
        GroupDesc& G = groups[0];
        G.hi = n;
        G.arcs = g->nnz;
        G.nsrc = LANES;
        G.ring_len = g->maxw + 1;
        const size_t need = group_bytes(G, steps) + engine_bytes(1, n) + 65536;
        BC_TRY(g->work.reserve(need));
        G.g.row_ptr = g->d_row_ptr;
        G.g.col = g->d_col;
        G.g.len = g->d_len;
        G.lo = 0;
        G.hi = n;
        G.flags = g->unit ? GF_UNIT : 0u;
        const int32_t first = g0 * LANES;
        G.nsrc = std::min(LANES, nsrc - first);
        for (int b = 0; b < LANES; ++b) G.src[b] = b < G.nsrc ? src[first + b] : -1;
        BC_TRY(run_groups(g->work, s, groups, steps));
        BC_HIP(hipMemcpyAsync(ht.data(), G.dist, ht.size() * 4, hipMemcpyDeviceToHost, s));
        BC_HIP(hipMemcpyAsync(hs.data(), G.sigma, hs.size() * 8, hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        for (int b = 0; b < G.nsrc; ++b) {
            const int64_t r = first + b;
            for (int32_t v = 0; v < n; ++v) {
                const uint32_t t = ht[(size_t)v * LANES + b];
                if (d) d[r * n + v] = (t == INF32) ? -1 : (int64_t)t;
                if (sigma) sigma[r * n + v] = (t == INF32) ? 0 : hs[(size_t)v * LANES + b];
            }
        }
    }
    return BC_OK;
}

}  // namespace bcpp

using namespace bcpp;

// ==================================================================== C ABI =====

extern "C" {

const char* bc_last_error(void) { return g_last_error.c_str(); }

int bc_graph_create(const bc_csr* g, void* hip_stream, bc_graph** out) {
    if (!out) return fail(BC_E_INVAL, "null output handle");
    *out = nullptr;
    return graph_create(g, (hipStream_t)hip_stream, out);
}

void bc_graph_destroy(bc_graph* g) { delete g; }

int bc_sssp_counts(const bc_graph* g, const int32_t* src, int32_t nsrc, int64_t* d,
                   uint64_t* sigma) {
    if (!g) return fail(BC_E_INVAL, "null graph");
    return sssp_run(g, src, nsrc, d, sigma);
}

int bc_brandes_plain(const bc_graph* gc, const int32_t* S, int32_t nS, uint32_t flags,
                     double* bc_out) {
    if (!gc || !bc_out) return fail(BC_E_INVAL, "null graph or output");
    bc_graph* g = const_cast<bc_graph*>(gc);
    BC_TRY(validate_targets(g->n, S, nS));
    if (g->n == 0) return BC_OK;
    double* d_out = nullptr;
    BC_TRY(g->out.reserve((size_t)g->n * 8 + 256));
    d_out = g->out.take<double>(g->n);
    BC_TRY(plain_run(g, S, nS, nullptr, flags, d_out));
    BC_HIP(hipMemcpyAsync(bc_out, d_out, (size_t)g->n * 8, hipMemcpyDeviceToHost, g->stream));
    BC_HIP(hipStreamSynchronize(g->stream));
    return BC_OK;
}

int bc_brandes_plain_dev(const bc_graph* gc, const int32_t* S_dev, int32_t nS, uint32_t flags,
                         double* bc_out_dev) {
    if (!gc || !bc_out_dev) return fail(BC_E_INVAL, "null graph or output");
    bc_graph* g = const_cast<bc_graph*>(gc);
    if (nS < 0 || (nS > 0 && !S_dev)) return fail(BC_E_INVAL, "bad target array");
    std::vector<int32_t> hS(nS);
    if (nS) {
        BC_HIP(hipMemcpyAsync(hS.data(), S_dev, (size_t)nS * 4, hipMemcpyDeviceToHost, g->stream));
        BC_HIP(hipStreamSynchronize(g->stream));
    }
    BC_TRY(validate_targets(g->n, hS.data(), nS));
    return plain_run(g, hS.data(), nS, S_dev, flags, bc_out_dev);
}

void bc_profile_enable(int on) {
    Profiler& p = profiler();
    p.on = on != 0;
    // events are created here, outside any timed region, not on first use
    while (p.on && p.pool.size() + p.pending.size() * 2 < 8192) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) break;
        p.pool.push_back(e);
    }
    if (p.on && !p.d_bytes) {
        if (hipMalloc((void**)&p.d_bytes, BC_K_COUNT * sizeof(unsigned long long)) == hipSuccess)
            (void)hipMemset(p.d_bytes, 0, BC_K_COUNT * sizeof(unsigned long long));
        else
            p.d_bytes = nullptr;
    }
}

void bc_profile_reset(void) {
    Profiler& p = profiler();
    p.collect();
    for (int k = 0; k < BC_K_COUNT; ++k) {
        p.launches[k] = 0;
        p.ms[k] = 0.0;
        p.bytes[k] = 0.0;
    }
    if (p.d_bytes) (void)hipMemset(p.d_bytes, 0, BC_K_COUNT * sizeof(unsigned long long));
}

int bc_profile_read(int kind, int64_t* launches, double* ms, double* alg_bytes) {
    if (kind < 0 || kind >= BC_K_COUNT) return fail(BC_E_INVAL, "bad kernel kind");
    Profiler& p = profiler();
    p.collect();
    unsigned long long b[BC_K_COUNT] = {};
    if (p.d_bytes) {
        BC_HIP(hipDeviceSynchronize());
        BC_HIP(hipMemcpy(b, p.d_bytes, sizeof(b), hipMemcpyDeviceToHost));
    }
    if (launches) *launches = p.launches[kind];
    if (ms) *ms = p.ms[kind];
    if (alg_bytes) *alg_bytes = (double)b[kind];
    return BC_OK;
}

}  // extern "C"
