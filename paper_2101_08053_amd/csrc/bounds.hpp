// Index checks of the band-matrix (ELL) stores, for test builds.
//
// Every store into the band layout vals[slot * n_act + row] (and into the
// row-major scratch arrays that hold a row's slots side by side) takes its
// offset from band_index(). In a build with -DIGA_DEBUG_BOUNDS the offset is
// checked: a slot or row outside its range is counted in this module's
// device word g_bounds_hits and replaced by offset 0, so the store stays
// inside the array and the count reports the error
// (iga_debug_bounds_hits sums the words of every module). Release builds
// compute the offset alone, the same expression as without the check.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace iga {

#ifdef IGA_DEBUG_BOUNDS
// Registers a module's reader (api.hip); the readers are summed by iga_debug_bounds_hits.
int bounds_register(unsigned long long (*read)(bool reset));
namespace {
__device__ unsigned long long g_bounds_hits;  // this module's count of out-of-range offsets
unsigned long long bounds_read(bool reset) {
    unsigned long long v = 0;
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_bounds_hits), sizeof v) != hipSuccess) return ~0ull;
    if (reset) {
        const unsigned long long z = 0;
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_bounds_hits), &z, sizeof z) != hipSuccess) return ~0ull;
    }
    return v;
}
const int g_bounds_registered = bounds_register(&bounds_read);
}  // namespace

__device__ __forceinline__ size_t band_index(int64_t slot, int64_t nslot, int64_t row, int64_t nrow) {
    if (slot < 0 || slot >= nslot || row < 0 || row >= nrow) {
        atomicAdd(&g_bounds_hits, 1ull);
        return 0;
    }
    return (size_t)slot * nrow + row;
}
#else
__device__ __forceinline__ size_t band_index(int64_t slot, int64_t, int64_t row, int64_t nrow) {
    return (size_t)slot * nrow + row;
}
#endif

}  // namespace iga
