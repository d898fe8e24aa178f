// Device-wide exclusive prefix sum of int32 counts (used for the compaction
// of active functions, cut and band elements, crossings, arcs and nodes).
// out has n+1 entries; out[n] is the total. Three launches: block scans,
// a single-block scan of the block sums, and the block offsets.
#include "plan.hpp"

namespace iga {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const int* __restrict__ in, int* __restrict__ out,
                                                             int n, int* __restrict__ bsum) {
    __shared__ int sh[kScanThreads / 64 + 1];
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int tsum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < n) ? in[base + j] : 0;
        tsum += v[j];
    }
    int total;
    int ex = block_excl_scan(tsum, sh, total);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) out[base + j] = ex;
        ex += v[j];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024) k_scan_sums(int* __restrict__ bsum, int nb, int* __restrict__ total_out) {
    __shared__ int sh[1024 / 64 + 1];
    int carry = 0;
    for (int base = 0; base < nb; base += 1024) {
        int idx = base + threadIdx.x;
        int v = (idx < nb) ? bsum[idx] : 0;
        int total;
        int ex = block_excl_scan(v, sh, total);
        if (idx < nb) bsum[idx] = ex + carry;
        carry += total;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(int* __restrict__ out, int n, const int* __restrict__ bsum) {
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int add = bsum[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < n) out[base + j] += add;
}

// One workgroup for short arrays: chunks of 4096 with a running carry.
__global__ void __launch_bounds__(1024) k_scan_single(const int* __restrict__ in, int* __restrict__ out, int n) {
    __shared__ int sh[1024 / 64 + 1];
    int carry = 0;
    for (int base = 0; base < n; base += 4096) {
        const int i0 = base + threadIdx.x * 4;
        int v[4], s = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = (i0 + j < n) ? in[i0 + j] : 0;
            s += v[j];
        }
        int total;
        int ex = block_excl_scan(s, sh, total) + carry;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i0 + j < n) out[i0 + j] = ex;
            ex += v[j];
        }
        carry += total;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

// tmp must hold ceil(n / 1024) + 1 ints.
void exclusive_scan(const int* in, int* out, int n, int* tmp, hipStream_t s) {
    if (n <= 16384) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, s, in, out, n);
        return;
    }
    int nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(kScanThreads), 0, s, in, out, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tmp, nb, out + n);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanThreads), 0, s, out, n, tmp);
}

}  // namespace iga
