// ot_host.h -- host-side argument checks shared by the entry points of
// libotfmm. Internal to the library.
#pragma once

#include <cstdint>

namespace otfmm {

// Do the double ranges [a, a + na) and [b, b + nb) share memory?
inline bool overlap(const double* a, int64_t na, const double* b, int64_t nb)
{
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + (uintptr_t)nb * sizeof(double) && b0 < a0 + (uintptr_t)na * sizeof(double);
}

}  // namespace otfmm
