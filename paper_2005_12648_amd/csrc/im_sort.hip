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

// Tile geometry: 64 KiB of keys per workgroup (two workgroups fill a CU's
// LDS), 512 threads holding `ipt` keys each.  (Measured on 2^28 int32: this
// tile with one merge chain of ipt steps per thread and one LDS read per
// step sorts 8% faster than 8192-key tiles with two reads per step; several
// shorter chains per thread, each with its own co-rank search, are slower:
// the rounds are bound by the number of LDS accesses, whose data-dependent
// addresses conflict in the banks, more than by their latency.)
template <typename K>
struct SortGeo {
    static constexpr int threads = 512;
    static constexpr int ipt = sizeof(K) == 4 ? 32 : 16;
    static constexpr int tile = threads * ipt;   // 16384 or 8192 keys
    // one pad element per 32 words: the blocked accesses (stride ipt keys)
    // fall in distinct banks
    static constexpr int shift = sizeof(K) == 4 ? 5 : 4;
    static constexpr int lds = tile + (tile >> shift) + 8;
};

template <typename K>
__device__ __forceinline__ int sphys(int x) {
    return x + (x >> SortGeo<K>::shift);
}

// Sort of each tile of the array, in place.  Per tile:
//   1. a coalesced load, IPT keys per thread (which keys a thread starts
//      with does not matter for a sort);
//   2. a bitonic network sorts each thread's keys in registers;
//   3. merge rounds: runs of width w (w = IPT, 2 IPT, ...) held by
//      consecutive threads are merged pairwise through LDS; a thread finds
//      the co-rank of its first output by a search in LDS, then merges its
//      IPT outputs with the next key of each run in registers and the key
//      type's maximum as the end-of-run sentinel (keys only: an output equal
//      to the sentinel has the same value whichever side it is taken from);
//   4. a coalesced store through LDS.
template <typename K>
__global__ __launch_bounds__(512, 4) void k_tilesort(K *__restrict__ data, int64_t n) {
    using SG = SortGeo<K>;
    constexpr int TH = SG::threads, IPT = SG::ipt, TS = SG::tile;
    __shared__ K s[SG::lds];
    const int tid = threadIdx.x;
    const K kmax = std::numeric_limits<K>::max();
    for (int64_t tile = blockIdx.x; tile * TS < n; tile += gridDim.x) {
        const int64_t t0 = tile * TS;
        const int cnt = (int)(n - t0 < TS ? n - t0 : TS);
        K r[IPT];
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            const int x = tid + u * TH;
            r[u] = x < cnt ? data[t0 + x] : kmax;
        }
        // bitonic sorting network on the thread's registers (ascending)
#pragma unroll
        for (int k = 2; k <= IPT; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
                for (int i = 0; i < IPT; ++i) {
                    const int l = i ^ j;
                    if (l > i) {
                        const K x = r[i], y = r[l];
                        const K mn = x < y ? x : y, mx = x < y ? y : x;
                        const bool up = (i & k) == 0;
                        r[i] = up ? mn : mx;
                        r[l] = up ? mx : mn;
                    }
                }
            }
        }
        for (int w = IPT; w < TS; w <<= 1) {
#pragma unroll
            for (int e = 0; e < IPT; ++e) s[sphys<K>(tid * IPT + e)] = r[e];
            __syncthreads();
            const int dabs = tid * IPT;
            const int p0 = dabs & ~(2 * w - 1);   // the pair of runs [p0, p0+w) | [p0+w, p0+2w)
            const int pb = p0 + w;
            const int d = dabs - p0;             // first output diagonal in the pair
            int lo = d > w ? d - w : 0;
            int hi = d < w ? d : w;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s[sphys<K>(p0 + mid)] <= s[sphys<K>(pb + d - 1 - mid)]) lo = mid + 1;
                else hi = mid;
            }
            // ia, ib: next indices in the two runs; a, b: their keys (the
            // sentinel once a run is used up).  ia may run past w, by fewer
            // than IPT steps, which stays inside the pair.
            int ia = lo, ib = d - lo;
            K a = s[sphys<K>(p0 + ia)];
            K b = s[sphys<K>(pb + ib)];
            a = ia < w ? a : kmax;
            b = ib < w ? b : kmax;
#pragma unroll
            for (int e = 0; e < IPT; ++e) {
                const bool ta = a <= b;
                r[e] = ta ? a : b;
                const int na = ia + 1, nb = ib + 1;
                const K v0 = s[sphys<K>(ta ? p0 + na : pb + nb)];
                const K v = (ta ? na < w : nb < w) ? v0 : kmax;
                ia = ta ? na : ia;
                ib = ta ? ib : nb;
                a = ta ? v : a;
                b = ta ? b : v;
            }
            __syncthreads();
        }
#pragma unroll
        for (int e = 0; e < IPT; ++e) s[sphys<K>(tid * IPT + e)] = r[e];
        __syncthreads();
        // (the opaque copy keeps the compiler from hoisting IPT padded
        // addresses out of the tile loop, which spills)
        int xb = tid;
        asm volatile("" : "+v"(xb));
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            const int x = xb + u * TH;
            if (x < cnt) data[t0 + x] = s[sphys<K>(x)];
        }
        __syncthreads();
    }
}

int sort_tile_elems(int key_bytes) {
    return key_bytes == 4 ? SortGeo<int32_t>::tile : SortGeo<int64_t>::tile;
}

template <typename K>
static hipError_t tilesort_t(void *data, int64_t n, hipStream_t s) {
    const int64_t tiles = (n + SortGeo<K>::tile - 1) / SortGeo<K>::tile;
    const int g = (int)(tiles < 16384 ? (tiles < 1 ? 1 : tiles) : 16384);
    hipLaunchKernelGGL(k_tilesort<K>, dim3(g), dim3(SortGeo<K>::threads), 0, s, (K *)data, n);
    return hipGetLastError();
}

hipError_t launch_tilesort(int key, void *data, int64_t n, hipStream_t s) {
    switch (key) {
        case kI32: return tilesort_t<int32_t>(data, n, s);
        case kU32: return tilesort_t<uint32_t>(data, n, s);
        case kI64: return tilesort_t<int64_t>(data, n, s);
        case kU64: return tilesort_t<uint64_t>(data, n, s);
    }
    return hipErrorInvalidValue;
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
