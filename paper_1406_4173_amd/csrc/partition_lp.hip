// A partition of G computed on the device, for Brandes++'s input P (Sec. 5 takes any
// partition; the paper obtains one from third-party clustering tools). Size-constrained
// label propagation: every node starts in its own part; in each round about half the
// nodes, chosen by a counter-based hash, move to the part most common among their
// neighbours, if that part is below the size cap (a node may always stay), preferring
// to stay on a tie and otherwise the smallest label. Part sizes are recounted after
// every round, so each round depends only on the previous one and the result is a
// function of (graph, cap, rounds, seed). Labels are then renumbered 0..k-1 in
// increasing order of the surviving labels. Betweenness does not depend on the
// partition (Sec. 5); only Brandes++'s speed does.
// One thread per node counts its neighbours' labels by pairwise comparison, which is
// quadratic in the node's degree: meant for sparse graphs (mean degree 6 to 12 here);
// a graph with hubs of thousands of arcs would want a per-node wave and a hash.
#include "engine.h"
#include "graph.h"

namespace bcpp {

namespace {

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014): the output function applied to the counter x.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void k_lp_init(int32_t n, int32_t* __restrict__ lab, int32_t* __restrict__ size) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) {
        lab[v] = v;
        size[v] = 1;
    }
}

__global__ void k_lp_round(int32_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const int32_t* __restrict__ lin, int32_t* __restrict__ lout,
                           const int32_t* __restrict__ size, int32_t cap, uint64_t seed, int32_t round) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t cur = lin[v];
    const uint64_t h = splitmix64(seed ^ ((uint64_t)(uint32_t)round << 32) ^ (uint64_t)(uint32_t)v);
    const int64_t e0 = rp[v], e1 = rp[v + 1];
    if (!(h & 1ull) || e0 == e1) {
        lout[v] = cur;
        return;
    }
    int32_t c0 = 0, bestl = -1, bestc = -1;
    for (int64_t e = e0; e < e1; ++e) {
        const int32_t l = lin[col[e]];
        if (l == cur) {
            ++c0;
            continue;
        }
        bool seen = false;
        for (int64_t f = e0; f < e && !seen; ++f) seen = lin[col[f]] == l;
        if (seen || (cap > 0 && size[l] >= cap)) continue;
        int32_t c = 1;
        for (int64_t f = e + 1; f < e1; ++f) c += lin[col[f]] == l;
        if (c > bestc || (c == bestc && l < bestl)) {
            bestc = c;
            bestl = l;
        }
    }
    lout[v] = bestc > c0 ? bestl : cur;
}

__global__ void k_lp_count(int32_t n, const int32_t* __restrict__ lab, int32_t* __restrict__ size) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) atomicAdd(&size[lab[v]], 1);
}

__global__ void k_lp_used(int32_t n, const int32_t* __restrict__ size, int32_t* __restrict__ used) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) used[v] = size[v] > 0 ? 1 : 0;
}

__global__ void k_lp_relabel(int32_t n, const int32_t* __restrict__ lab, const int32_t* __restrict__ id,
                             int32_t* __restrict__ part) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) part[v] = id[lab[v]];
}

}  // namespace

int partition_lp(bc_graph* g, int32_t cap, int32_t rounds, uint64_t seed, int32_t* part_out, int32_t* k_out) {
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    *k_out = 0;
    if (n == 0) return BC_OK;
    Arena& W = g->work;
    BC_TRY(W.reserve((size_t)n * 4 * 6 + scan_scratch_bytes(n + 1) + 8 * 256));
    int32_t* a = W.take<int32_t>(n);
    int32_t* b = W.take<int32_t>(n);
    int32_t* size = W.take<int32_t>(n);
    int32_t* used = W.take<int32_t>((size_t)n + 1);
    int32_t* id = W.take<int32_t>((size_t)n + 1);
    int32_t* part = W.take<int32_t>(n);
    void* scr = W.take<unsigned char>(scan_scratch_bytes(n + 1));
    if (!a || !b || !size || !used || !id || !part || !scr) return fail(BC_E_NOMEM, "partition: workspace too small");
    const dim3 grid((unsigned)((n + 255) / 256)), blk(256);
    hipLaunchKernelGGL(k_lp_init, grid, blk, 0, s, n, a, size);
    for (int32_t r = 0; r < rounds; ++r) {
        hipLaunchKernelGGL(k_lp_round, grid, blk, 0, s, n, g->d_row_ptr, g->d_col, a, b, size, cap, seed, r);
        BC_TRY(zero_device(s, size, (size_t)n * 4));
        hipLaunchKernelGGL(k_lp_count, grid, blk, 0, s, n, b, size);
        std::swap(a, b);
    }
    hipLaunchKernelGGL(k_lp_used, grid, blk, 0, s, n, size, used);
    BC_TRY(zero_device(s, used + n, 4));
    BC_TRY(exclusive_scan<int32_t>(s, used, id, (int64_t)n + 1, scr));
    hipLaunchKernelGGL(k_lp_relabel, grid, blk, 0, s, n, a, id, part);
    BC_HIP(hipGetLastError());
    BC_HIP(hipMemcpyAsync(part_out, part, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    BC_HIP(hipMemcpyAsync(k_out, id + n, 4, hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    return BC_OK;
}

}  // namespace bcpp

using namespace bcpp;

extern "C" {

int bc_partition_lp(const bc_graph* gc, int32_t max_part, int32_t rounds, uint64_t seed, int32_t* part_out,
                    int32_t* k_out) {
    if (!gc || !part_out || !k_out) return fail(BC_E_INVAL, "null graph or output");
    if (max_part < 0 || rounds < 0) return fail(BC_E_INVAL, "negative size cap or round count");
    return partition_lp(const_cast<bc_graph*>(gc), max_part, rounds, seed, part_out, k_out);
}

}  // extern "C"
