// Plain target-set Brandes without device allocation, for callers that cannot allocate
// (code under HIP graph capture, serving loops that forbid it): every buffer the
// kernels need beyond the caller's inputs and outputs comes from one fixed array in
// device memory, `scratch`, that the library holds on each GPU it runs on.
#include <mutex>

#include "engine.h"
#include "graph.h"

namespace bcpp {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;

// The array itself. Host code never uses this name as an address (on the host it is a
// stand-in for the device symbol): scratch_ptr() gives the device address.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

int plain_resident(bc_graph* g, Arena& W, bool grow, const int32_t* S, int32_t nS, const int32_t* S_dev,
                   double scale, double* out_dev);
int validate_targets(int32_t n, const int32_t* S, int32_t nS);

// Device address of `scratch` on the current device, looked up once per device with
// that device current.
static int scratch_ptr(void** out) {
    static std::mutex mu;
    static std::vector<void*> ptrs;
    int dev = 0;
    BC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
    if (!ptrs[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(BC_E_DEVICE, std::string("no device address for the scratch array: ") + hipGetErrorString(e));
        }
        ptrs[dev] = p;
    }
    *out = ptrs[dev];
    return BC_OK;
}

}  // namespace bcpp

using namespace bcpp;

extern "C" {

int bc_brandes_plain_noalloc(const bc_graph* gc, const int32_t* S_dev, int32_t nS, uint32_t flags,
                             double* bc_out_dev) {
    if (!gc || !bc_out_dev) return fail(BC_E_INVAL, "null graph or output");
    bc_graph* g = const_cast<bc_graph*>(gc);
    if (nS < 0 || (nS > 0 && !S_dev)) return fail(BC_E_INVAL, "bad target array");
    if (flags & ~(uint32_t)BC_ORDERED) return fail(BC_E_INVAL, "only BC_ORDERED is accepted here");
    const int32_t n = g->n;
    if (n == 0) return BC_OK;
    if (!resident_takes(n)) return fail(BC_E_INVAL, "the resident kernel is switched off");
    std::vector<int32_t> hS(nS);
    if (nS) {
        BC_HIP(hipMemcpyAsync(hS.data(), S_dev, (size_t)nS * 4, hipMemcpyDeviceToHost, g->stream));
        BC_HIP(hipStreamSynchronize(g->stream));
    }
    BC_TRY(validate_targets(n, hS.data(), nS));
    if (nS < 2) {
        BC_TRY(zero_device(g->stream, bc_out_dev, (size_t)n * 8));
        BC_HIP(hipStreamSynchronize(g->stream));
        return BC_OK;
    }
    void* base = nullptr;
    BC_TRY(scratch_ptr(&base));
    Arena W = Arena::view(base, NOALLOC_SCRATCH_BYTES);
    const double scale = (flags & BC_ORDERED) ? 1.0 : 0.5;
    return plain_resident(g, W, false, hS.data(), nS, S_dev, scale, bc_out_dev);
}

size_t bc_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

}  // extern "C"
