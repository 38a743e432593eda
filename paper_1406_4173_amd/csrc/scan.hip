// Exclusive prefix sums on the device: tiles of 1024 items (256 threads, 4 consecutive
// items each) scan locally and record their totals, one workgroup turns the totals into
// tile offsets, and a last pass adds each tile's offset. The scratch is the totals
// array; nothing has to be cleared beforehand, so a captured graph can replay it.
#include "engine.h"

namespace bcpp {

namespace {

constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_T * SCAN_ITEMS;

// Exclusive sum of x over the workgroup's threads (blockDim.x == 256 or 1024), and the
// total through *total.
template <class T>
__device__ __forceinline__ T block_exclusive(T x, T* lds, T* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    T incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < nw; ++w) {
            const T t = lds[w];
            lds[w] = run;
            run += t;
        }
        lds[16] = run;
    }
    __syncthreads();
    const T r = lds[wave] + incl - x;
    *total = lds[16];
    __syncthreads();
    return r;
}

template <class T>
__global__ void __launch_bounds__(SCAN_T) k_scan_tiles(const T* __restrict__ in, T* out, int64_t n, T* __restrict__ tot) {
    __shared__ T lds[17];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T sum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = base + i < n ? in[base + i] : T(0);
        sum += v[i];
    }
    T total;
    T run = block_exclusive(sum, lds, &total);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// One workgroup of 1024 threads: tot[0..ntiles) becomes its own exclusive prefix sum.
template <class T>
__global__ void __launch_bounds__(1024) k_scan_carry(T* __restrict__ tot, int64_t ntiles) {
    __shared__ T lds[17];
    T carry = 0;
    for (int64_t b = 0; b < ntiles; b += 1024) {
        const int64_t i = b + threadIdx.x;
        const T x = i < ntiles ? tot[i] : T(0);
        T total;
        const T r = block_exclusive(x, lds, &total);
        if (i < ntiles) tot[i] = carry + r;
        carry += total;
    }
}

template <class T>
__global__ void k_scan_add(T* __restrict__ out, int64_t n, const T* __restrict__ tot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tot[i / SCAN_TILE];
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
    const int64_t tiles = std::max<int64_t>((n + SCAN_TILE - 1) / SCAN_TILE, 1);
    return (size_t)tiles * 8 + 256;
}

template <class T>
int exclusive_scan(hipStream_t s, const T* in, T* out, int64_t n, void* scratch) {
    if (n <= 0) return BC_OK;
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    T* tot = reinterpret_cast<T*>(scratch);
    hipLaunchKernelGGL((k_scan_tiles<T>), dim3((unsigned)tiles), dim3(SCAN_T), 0, s, in, out, n, tot);
    if (tiles > 1) {
        hipLaunchKernelGGL((k_scan_carry<T>), dim3(1), dim3(1024), 0, s, tot, tiles);
        hipLaunchKernelGGL((k_scan_add<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n,
                           (const T*)tot);
    }
    BC_HIP(hipGetLastError());
    return BC_OK;
}

template int exclusive_scan<int32_t>(hipStream_t, const int32_t*, int32_t*, int64_t, void*);
template int exclusive_scan<int64_t>(hipStream_t, const int64_t*, int64_t*, int64_t, void*);

}  // namespace bcpp
