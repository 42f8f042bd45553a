// ot_common.h -- definitions shared by the translation units of libotfmm:
// error reporting, sub-grid geometry constants, the graded-lexicographic
// multi-index tables and small host helpers. Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ot_fmm.h"

namespace otfmm {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
inline thread_local std::string g_last_error;

inline int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

inline int hip_fail(hipError_t e, const char* what)
{
    return fail(OT_FMM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define OT_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// ---------------------------------------------------------------------------
// Geometry constants
// ---------------------------------------------------------------------------
constexpr int kSub = 8;
constexpr int kSub3 = 512;
constexpr int kHalo = 24;
constexpr int kPlane = kHalo * kHalo;   // 576 cells per halo z-plane
constexpr int kHalo3 = kPlane * kHalo;  // 13824
constexpr int kReach = 9;               // max |d_k| in the stencil
constexpr int kMaxRows = 2 * (2 * kReach + 1) * (2 * kReach + 1);
constexpr double kFar = 1.0e20;         // centre used for missing cells

// ---------------------------------------------------------------------------
// Multi-indices, graded lexicographic with x most significant
// ---------------------------------------------------------------------------
struct Exp3 {
    int a, b, c;
};

__host__ __device__ constexpr int ncomp(int o) { return (o + 1) * (o + 2) * (o + 3) / 6; }

__host__ __device__ constexpr Exp3 exp_of(int g)
{
    int k = 0;
    for (int n = 0; n <= 8; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b) {
                if (k == g) return Exp3{a, b, n - a - b};
                ++k;
            }
    return Exp3{-1, -1, -1};
}

__host__ __device__ constexpr int ord_of(int g)
{
    return exp_of(g).a + exp_of(g).b + exp_of(g).c;
}

__host__ __device__ constexpr int idx_of(int a, int b, int c)
{
    const int n = a + b + c;
    int k = n > 0 ? ncomp(n - 1) : 0;
    for (int ap = n; ap > a; --ap) k += n - ap + 1;
    return k + (n - a) - b;
}

__host__ __device__ constexpr int sum_idx(int g, int h)
{
    return idx_of(exp_of(g).a + exp_of(h).a, exp_of(g).b + exp_of(h).b,
                  exp_of(g).c + exp_of(h).c);
}

__host__ __device__ constexpr double factorial(int n) { return n <= 1 ? 1.0 : n * factorial(n - 1); }

__host__ __device__ constexpr double inv_multi_factorial(int g)
{
    return 1.0 / (factorial(exp_of(g).a) * factorial(exp_of(g).b) * factorial(exp_of(g).c));
}

__host__ __device__ constexpr double parity_sign(int g) { return (ord_of(g) & 1) ? -1.0 : 1.0; }

constexpr bool check_indices()
{
    for (int g = 0; g < 35; ++g)
        if (idx_of(exp_of(g).a, exp_of(g).b, exp_of(g).c) != g) return false;
    return ord_of(19) == 3 && ord_of(20) == 4 && sum_idx(1, 2) == 5 && sum_idx(4, 3) == 12;
}
static_assert(check_indices(), "multi-index tables");

// Device set-up check: the current device is a gfx950 (one check per device).
int ensure_device();

// A double array's natural alignment: the kernels read and write global
// memory one double at a time.
inline bool aligned8(const void* p)
{
    return p && (reinterpret_cast<uintptr_t>(p) & 7u) == 0;
}

// Copies a host table to a new device allocation (ENOMEM / EHIP on failure;
// *dst is then null or must be freed by the caller).
template <class Tp>
int upload(Tp** dst, const std::vector<Tp>& src)
{
    *dst = nullptr;
    if (src.empty()) return OT_FMM_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(Tp));
    if (e != hipSuccess) {
        *dst = nullptr;
        return fail(OT_FMM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    e = hipMemcpy(*dst, src.data(), src.size() * sizeof(Tp), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    return OT_FMM_OK;
}

}  // namespace otfmm
