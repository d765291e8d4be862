// im_sort.hip -- building blocks of the in-place bottom-up merge sort.
//
// The paper notes that the parallel in-place merge can drive a merge sort
// (Sec. 1, related work on in-place merge sorts and the Akl et al. parallel
// sort) but leaves that use aside.  The driver here sorts tiles in LDS, then
// runs passes of the batched in-place merge with doubling run width; this
// file holds the tile sort and the per-pass instance offsets.
#include <limits>
#include "im_common.h"

namespace imerge {

constexpr int kSortThreads = 512;
constexpr int kSortIpt = 16;
constexpr int kSortTile = kSortThreads * kSortIpt;   // 8192 elements

__device__ __forceinline__ int sphys(int x) { return x + (x >> 5); }

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_tilesort(K *__restrict__ data, int64_t n) {
    __shared__ K s[kSortTile + kSortTile / 32 + 1];
    const int tid = threadIdx.x;
    const K kmax = std::numeric_limits<K>::max();
    for (int64_t tile = blockIdx.x; tile * kSortTile < n; tile += gridDim.x) {
        const int64_t t0 = tile * kSortTile;
        int cnt = (int)(n - t0 < kSortTile ? n - t0 : kSortTile);
        K r[kSortIpt];
        // which elements a thread starts with does not matter for a sort:
        // take a coalesced strided set straight from global memory.
#pragma unroll
        for (int u = 0; u < kSortIpt; ++u) {
            int x = tid + u * kSortThreads;
            r[u] = x < cnt ? data[t0 + x] : kmax;
        }
        // odd-even transposition sort of the thread's registers
#pragma unroll
        for (int round = 0; round < kSortIpt; ++round) {
#pragma unroll
            for (int e = round & 1; e + 1 < kSortIpt; e += 2) {
                K a = r[e], b = r[e + 1];
                r[e] = a < b ? a : b;
                r[e + 1] = a < b ? b : a;
            }
        }
        // merge rounds: runs of width w held by consecutive threads
        for (int w = kSortIpt; w < kSortTile; w <<= 1) {
#pragma unroll
            for (int e = 0; e < kSortIpt; ++e) s[sphys(tid * kSortIpt + e)] = r[e];
            __syncthreads();
            const int dabs = tid * kSortIpt;
            const int p0 = dabs & ~(2 * w - 1);   // start of the pair of runs
            const int d = dabs - p0;
            // co-rank of local diagonal d in runs [p0, p0+w) and [p0+w, p0+2w)
            int lo = d > w ? d - w : 0;
            int hi = d < w ? d : w;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (s[sphys(p0 + mid)] <= s[sphys(p0 + w + d - 1 - mid)]) lo = mid + 1;
                else hi = mid;
            }
            int ia = lo, ib = d - lo;
#pragma unroll
            for (int e = 0; e < kSortIpt; ++e) {
                K a = ia < w ? s[sphys(p0 + ia)] : kmax;
                K b = ib < w ? s[sphys(p0 + w + ib)] : kmax;
                bool ta = (ib >= w) || (ia < w && a <= b);
                r[e] = ta ? a : b;
                if (ta) ++ia; else ++ib;
            }
            __syncthreads();
        }
#pragma unroll
        for (int e = 0; e < kSortIpt; ++e) s[sphys(tid * kSortIpt + e)] = r[e];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kSortIpt; ++u) {
            int x = tid + u * kSortThreads;
            if (x < cnt) data[t0 + x] = s[sphys(x)];
        }
        __syncthreads();
    }
}

int sort_tile_elems(int) { return kSortTile; }

hipError_t launch_tilesort(int key, void *data, int64_t n, hipStream_t s) {
    int64_t tiles = (n + kSortTile - 1) / kSortTile;
    int g = (int)(tiles < 8192 ? (tiles < 1 ? 1 : tiles) : 8192);
    switch (key) {
        case kI32:
            hipLaunchKernelGGL(k_tilesort<int32_t>, dim3(g), dim3(kSortThreads), 0, s,
                               (int32_t *)data, n);
            break;
        case kU32:
            hipLaunchKernelGGL(k_tilesort<uint32_t>, dim3(g), dim3(kSortThreads), 0, s,
                               (uint32_t *)data, n);
            break;
        case kI64:
            hipLaunchKernelGGL(k_tilesort<int64_t>, dim3(g), dim3(kSortThreads), 0, s,
                               (int64_t *)data, n);
            break;
        case kU64:
            hipLaunchKernelGGL(k_tilesort<uint64_t>, dim3(g), dim3(kSortThreads), 0, s,
                               (uint64_t *)data, n);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Instances of one bottom-up pass of width w: [2qw, 2qw+w) | [2qw+w, 2qw+2w),
// clipped to n; a trailing run without a partner gets an empty B.
__global__ void k_pass_offsets(int64_t n, int64_t w, int64_t *__restrict__ off, int64_t n_inst) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q > n_inst) return;
    if (q == n_inst) { off[2 * q] = n; return; }
    int64_t a = 2 * q * w;
    int64_t m = a + w < n ? a + w : n;
    off[2 * q] = a;
    off[2 * q + 1] = m;
}

hipError_t launch_pass_offsets(int64_t n, int64_t width, int64_t *d_off, int64_t n_inst,
                               hipStream_t s) {
    int64_t items = n_inst + 1;
    int g = (int)((items + 255) / 256);
    hipLaunchKernelGGL(k_pass_offsets, dim3(g), dim3(256), 0, s, n, width, d_off, n_inst);
    return hipGetLastError();
}

}  // namespace imerge
