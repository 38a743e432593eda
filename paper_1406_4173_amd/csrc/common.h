// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bcpp.h"

namespace bcpp {

constexpr uint32_t INF32 = 0xFFFFFFFFu;
constexpr int LANES = 64;  // sources per group: one per lane of a wave64

// ---------------------------------------------------------------- errors ------

void set_error(const std::string& msg);

struct Status {
    int code = BC_OK;
    bool ok() const { return code == BC_OK; }
};

#define BC_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ::bcpp::set_error(std::string("HIP error in ") + #call + ": " +          \
                              hipGetErrorString(e_));                                \
            return e_ == hipErrorOutOfMemory ? BC_E_NOMEM : BC_E_DEVICE;             \
        }                                                                            \
    } while (0)

#define BC_TRY(expr)                     \
    do {                                 \
        int rc_ = (expr);                \
        if (rc_ != BC_OK) return rc_;    \
    } while (0)

inline int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

// ------------------------------------------------------- device memory arena ---

// A growable device buffer reused across calls on one handle. Allocation is a bump
// pointer in 256-byte steps; reset() frees everything at once. When a request does
// not fit, the arena is re-created larger (only between runs, when nothing in it is
// live).
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    size_t peak = 0;
    // capacity limit (0 = no limit) so that a budget can be enforced
    size_t limit = 0;
    bool owning = true;  // false: a view of memory owned elsewhere (never freed here)

    // A non-owning arena over [base, base + cap).
    static Arena view(void* base, size_t cap) {
        Arena a;
        a.base = (char*)base;
        a.cap = cap;
        a.owning = false;
        return a;
    }
    Arena() = default;
    Arena(const Arena&) = delete;
    Arena& operator=(const Arena&) = delete;
    Arena(Arena&& o) noexcept { *this = std::move(o); }
    Arena& operator=(Arena&& o) noexcept {
        if (this != &o) {
            release();
            base = o.base;
            cap = o.cap;
            used = o.used;
            peak = o.peak;
            limit = o.limit;
            owning = o.owning;
            o.base = nullptr;
            o.cap = o.used = 0;
        }
        return *this;
    }

    int reserve(size_t bytes);  // ensure cap >= bytes (drops contents)
    void reset() { used = 0; }
    template <class T>
    T* take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        if (used + bytes > cap) return nullptr;
        T* p = reinterpret_cast<T*>(base + used);
        used += bytes;
        if (used > peak) peak = used;
        return p;
    }
    void release();
    ~Arena() { release(); }
};

// ------------------------------------------------------------ profiling -------

struct Profiler {
    bool on = false;
    struct Pending {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    int64_t launches[BC_K_COUNT] = {};
    double ms[BC_K_COUNT] = {};
    double bytes[BC_K_COUNT] = {};
    // device counters of algorithmic bytes, one slot per kernel kind
    unsigned long long* d_bytes = nullptr;

    hipEvent_t get_event();
    void begin(int kind, hipStream_t s, hipEvent_t* a);
    void end(int kind, hipStream_t s, hipEvent_t a);
    void collect();  // resolve pending event pairs (synchronises on them)
};

Profiler& profiler();

// Host phase trace (environment BCPP_TRACE=1): wall-clock time of named host phases,
// printed to stderr; off by default and free when off.
struct PhaseTrace {
    bool on;
    const char* what;
    std::chrono::steady_clock::time_point t0;
    explicit PhaseTrace(const char* w) : on(trace_on()), what(w) {
        if (on) t0 = std::chrono::steady_clock::now();
    }
    void mark(const char* phase) {
        if (!on) return;
        const auto t = std::chrono::steady_clock::now();
        fprintf(stderr, "[bcpp] %s: %s %.3f ms\n", what, phase,
                std::chrono::duration<double, std::milli>(t - t0).count());
        t0 = t;
    }
    static bool trace_on() {
        static const int v = [] {
            const char* e = getenv("BCPP_TRACE");
            return e && e[0] == '1';
        }();
        return v != 0;
    }
};

// Run f(begin, end) over [0, n) split into contiguous chunks on up to 16 host threads
// (one chunk per thread, at least `grain` items each); serial when n is small.
template <class F>
void parallel_for(int64_t n, int64_t grain, F&& f) {
    const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
    const int64_t T = std::min<int64_t>({hw, (int64_t)16, (n + grain - 1) / std::max<int64_t>(grain, 1)});
    if (T <= 1) {
        if (n > 0) f((int64_t)0, n);
        return;
    }
    const int64_t chunk = (n + T - 1) / T;
    std::vector<std::thread> th;
    th.reserve((size_t)T);
    for (int64_t t = 0; t < T; ++t) {
        const int64_t a = t * chunk, b = std::min(n, a + chunk);
        if (a >= b) break;
        th.emplace_back([&f, a, b] { f(a, b); });
    }
    for (auto& x : th) x.join();
}

// Scoped launch timer: records events around the launches in its scope when on.
struct KTimer {
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr;
    KTimer(int k, hipStream_t st) : kind(k), s(st) {
        if (profiler().on) profiler().begin(kind, s, &a);
    }
    ~KTimer() {
        if (profiler().on && a) profiler().end(kind, s, a);
    }
};

}  // namespace bcpp
