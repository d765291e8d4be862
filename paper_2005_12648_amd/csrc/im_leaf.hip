// im_leaf.hip -- merge of the pairs produced by the division stage.
//
// After the division (Sec. 3; Alg. 3), each leaf is a contiguous pair
// A_p | B_p whose merged output occupies exactly the leaf's own region, so
// leaves are independent (the per-pair merge of Alg. 2/3).  A leaf is cut
// into tiles of `tile` output elements; the co-rank of every tile diagonal
// inside its leaf is known (k_tilerank).  One workgroup merges one tile:
//   1. load its A-slice and B-slice into LDS (coalesced, contiguous);
//   2. every thread finds its own sub-diagonal by a co-rank search in LDS and
//      merges `ipt` outputs into registers (stable: ties take A);
//   3. outputs go back to LDS (padded to avoid bank conflicts);
//   4. leaf barrier: the tile's output window overlaps input slices that
//      other tiles of the same leaf read, so every tile of the leaf first
//      reports "inputs read" on the leaf's arrival counter and waits for all
//      of them;
//   5. coalesced store of the window.
// The grid is persistent and co-resident (cooperative launch); tile t is
// handled by workgroup t mod G in increasing t, and a leaf has at most G
// tiles, so the leaf holding the smallest unfinished tile always has all of
// its tiles running -- the waits cannot deadlock.  The wait is bounded: on
// expiry the workgroup raises an error bit and skips its store.
#include <type_traits>
#include "im_common.h"

namespace imerge {

struct NoValL {};

constexpr unsigned kSpinLimit = 1u << 26;

template <int T>
struct LdsPad { static constexpr int elems = T + T / 32 + 1; };

template <typename K, typename V, int THREADS, int IPT>
__global__ __launch_bounds__(THREADS) void k_leafmerge(K *__restrict__ keys, V *__restrict__ vals,
                                                       Plan pl, Work w) {
    constexpr int T = THREADS * IPT;
    constexpr bool HAS_V = !std::is_same<V, NoValL>::value;
    constexpr int PE = LdsPad<T>::elems;
    static_assert(32 % IPT == 0 && THREADS % 32 == 0, "padding layout");
    extern __shared__ __align__(16) unsigned char smem[];
    K *sk = reinterpret_cast<K *>(smem);
    V *sv = reinterpret_cast<V *>(smem + (size_t)PE * sizeof(K));
    __shared__ int s_ok;

    const int tid = threadIdx.x;
    const int64_t ntiles = (int64_t)w.ctr->tiles;
    for (int64_t t = blockIdx.x; t < ntiles && t < pl.cap_tiles; t += gridDim.x) {
        const int32_t l = w.tile_leaf[t];
        const Leaf lf = w.leaves[l];
        const int64_t local = t - w.tile_start[l];
        const int64_t S = lf.la + lf.lb;
        const int64_t d0 = local * (int64_t)T;
        const int64_t d1 = d0 + T < S ? d0 + T : S;
        const int n = (int)(d1 - d0);
        const int64_t ia0 = w.tile_rank[t];
        const int64_t ia1 = (local + 1 < lf.ntiles) ? w.tile_rank[t + 1] : lf.la;
        // For ascending runs na = ia1 - ia0 already lies in the interval below;
        // the clamp only keeps every access inside the leaf when a caller
        // passes unsorted runs (then the result is an unspecified permutation).
        int64_t na64 = ia1 - ia0;
        const int64_t na_lo = (d1 - lf.lb - ia0) > 0 ? (d1 - lf.lb - ia0) : 0;
        const int64_t na_hi = (lf.la - ia0) < (int64_t)n ? (lf.la - ia0) : (int64_t)n;
        if (na64 < na_lo) na64 = na_lo;
        if (na64 > na_hi) na64 = na_hi;
        const int na = (int)na64;
        const int nb = n - na;
        const int64_t jb0 = d0 - ia0;
        K *A = keys + lf.base;

        // 1. load.  Offsets are taken relative to the leaf start (a leaf is
        // smaller than 2^31 elements), so every address is a uniform base
        // plus one 32-bit lane offset.
        {
            const int a_off = (int)ia0;                       // A-slice start in the leaf
            const int b_off = (int)(lf.la + jb0) - na;        // B-slice start, minus na
            K r[IPT];
#pragma unroll
            for (int u = 0; u < IPT; ++u) {
                int x = tid + u * THREADS;
                if (x < n) r[u] = A[x < na ? a_off + x : b_off + x];
            }
#pragma unroll
            for (int u = 0; u < IPT; ++u) {
                int x = tid + u * THREADS;
                if (x < n) sk[x] = r[u];
            }
            if constexpr (HAS_V) {
                const V *VL = vals + lf.base;
                V q[IPT];
#pragma unroll
                for (int u = 0; u < IPT; ++u) {
                    int x = tid + u * THREADS;
                    if (x < n) q[u] = VL[x < na ? a_off + x : b_off + x];
                }
#pragma unroll
                for (int u = 0; u < IPT; ++u) {
                    int x = tid + u * THREADS;
                    if (x < n) sv[x] = q[u];
                }
            }
        }
        __syncthreads();

        // 2. per-thread merge path inside LDS
        K out[IPT];
        int src[HAS_V ? IPT : 1];
        {
            int d = tid * IPT;
            if (d > n) d = n;
            int lo = d > nb ? d - nb : 0;
            int hi = d < na ? d : na;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (sk[mid] <= sk[na + d - 1 - mid]) lo = mid + 1;
                else hi = mid;
            }
            int ia = lo, ib = d - lo;
            // sk has PE > n entries, so the look-ahead reads below stay inside LDS.
            K a = sk[ia];
            K b = sk[na + ib];
#pragma unroll
            for (int e = 0; e < IPT; ++e) {
                bool ta = (ib >= nb) || (ia < na && a <= b);
                out[e] = ta ? a : b;
                if constexpr (HAS_V) src[e] = ta ? ia : na + ib;
                int nx = ta ? ia + 1 : na + ib + 1;
                if (nx > PE - 1) nx = PE - 1;
                K v = sk[nx];
                if (ta) { ++ia; a = v; } else { ++ib; b = v; }
            }
        }
        V vout[HAS_V ? IPT : 1];
        if constexpr (HAS_V) {
#pragma unroll
            for (int e = 0; e < IPT; ++e) {
                int x = tid * IPT + e;
                int sidx = src[e];
                if (sidx > PE - 1) sidx = PE - 1;
                if (x < n) vout[e] = sv[sidx];
            }
        }
        __syncthreads();

        // 3. outputs back to LDS, padded: logical x -> x + x/32.  IPT divides
        // 32, so phys(tid*IPT + e) = wbase + e with one base per thread.
        {
            const int wbase = tid * IPT + ((tid * IPT) >> 5);
            const int x0 = tid * IPT;
#pragma unroll
            for (int e = 0; e < IPT; ++e) {
                if (x0 + e < n) {
                    sk[wbase + e] = out[e];
                    if constexpr (HAS_V) sv[wbase + e] = vout[e];
                }
            }
        }
        __syncthreads();

        // 4. leaf barrier (only leaves with several tiles)
        // The counter is touched only with relaxed device-scope atomics: the
        // tile's loads have returned (their values are in LDS), and an
        // acquire/release fence at device scope would write back or
        // invalidate the whole L2 of this XCD on every poll.
        if (lf.ntiles > 1) {
            if (tid == 0) {
                __hip_atomic_fetch_add(&w.arrive[l], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                unsigned spins = 0;
                int ok = 1;
                while (__hip_atomic_load(&w.arrive[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                       (unsigned)lf.ntiles) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > kSpinLimit) {
                        atomicOr(&w.ctr->error, kErrBarrierSpin);
                        ok = 0;
                        break;
                    }
                }
                s_ok = ok;
            }
            __syncthreads();
            if (!s_ok) continue;
        }

        // 5. coalesced store of the output window; THREADS is a multiple of
        // 32, so phys(tid + u*THREADS) = rbase + u*(THREADS + THREADS/32).
        {
            K *O = A + d0;
            const int rbase = tid + (tid >> 5);
            constexpr int RSTEP = THREADS + THREADS / 32;
#pragma unroll
            for (int u = 0; u < IPT; ++u) {
                int x = tid + u * THREADS;
                if (x < n) O[x] = sk[rbase + u * RSTEP];
            }
            if constexpr (HAS_V) {
                V *OV = vals + lf.base + d0;
#pragma unroll
                for (int u = 0; u < IPT; ++u) {
                    int x = tid + u * THREADS;
                    if (x < n) OV[x] = sv[rbase + u * RSTEP];
                }
            }
        }
        __syncthreads();
    }
}

// ---- leaf planning: tiles per leaf, exclusive scan, barrier counters ----
constexpr int kPlanThreads = 1024;

__global__ __launch_bounds__(kPlanThreads) void k_plan(Plan pl, Work w) {
    __shared__ long long buf[kPlanThreads];
    __shared__ long long s_run;
    __shared__ unsigned long long s_elems;
    int64_t L = (int64_t)w.ctr->leaves;
    if (L > pl.cap_leaves) L = pl.cap_leaves;
    const int tid = threadIdx.x;
    unsigned long long my_elems = 0;
    if (tid == 0) { s_run = 0; s_elems = 0; }
    __syncthreads();
    for (int64_t base = 0; base < L; base += kPlanThreads) {
        int64_t l = base + tid;
        long long c = 0;
        if (l < L) {
            int64_t S = w.leaves[l].la + w.leaves[l].lb;
            my_elems += (unsigned long long)S;
            c = (S + pl.tile - 1) / pl.tile;
            w.leaves[l].ntiles = (int32_t)c;
            w.arrive[l] = 0u;
        }
        buf[tid] = c;
        __syncthreads();
        // Hillis-Steele inclusive scan
        for (int off = 1; off < kPlanThreads; off <<= 1) {
            long long v = tid >= off ? buf[tid - off] : 0;
            __syncthreads();
            buf[tid] += v;
            __syncthreads();
        }
        long long run = s_run;
        if (l < L) w.tile_start[l] = run + buf[tid] - c;
        __syncthreads();
        if (tid == kPlanThreads - 1) s_run = run + buf[tid];
        __syncthreads();
    }
    if (my_elems) atomicAdd(&s_elems, my_elems);
    __syncthreads();
    if (tid == 0) {
        w.ctr->leaf_elems = s_elems;
        long long tot = s_run;
        if (tot > pl.cap_tiles) {
            atomicOr(&w.ctr->error, kErrCapacity);
            tot = pl.cap_tiles;
        }
        w.ctr->tiles = (unsigned long long)tot;
    }
}

hipError_t launch_plan(const Plan &pl, const Work &w, hipStream_t s) {
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, s, pl, w);
    return hipGetLastError();
}

// ---- geometry and dispatch ------------------------------------------------
template <typename K, typename V, int THREADS, int IPT>
struct LeafCfg {
    static constexpr int T = THREADS * IPT;
    static size_t lds() {
        return (size_t)LdsPad<T>::elems * sizeof(K) +
               (std::is_same<V, NoValL>::value ? 0 : (size_t)LdsPad<T>::elems * sizeof(V));
    }
    static const void *fn() { return (const void *)&k_leafmerge<K, V, THREADS, IPT>; }
};

// (key bytes, payload bytes) -> (threads, items per thread)
static void geom(int ek, int ev, int *th, int *ipt) {
    if (ev == 0) { *th = 512; *ipt = ek == 4 ? 16 : 8; return; }
    if (ek == 4 && ev == 4) { *th = 512; *ipt = 16; return; }
    *th = 512; *ipt = 8;
}

void leaf_geometry(int esize_k, int esize_v, int *threads, int *ipt, size_t *lds_bytes) {
    geom(esize_k, esize_v, threads, ipt);
    int T = *threads * *ipt;
    size_t pe = (size_t)(T + T / 32 + 1);
    *lds_bytes = pe * esize_k + pe * esize_v;
}

#define IM_LEAF_CASES(X)                        \
    X(int32_t, NoValL, 512, 16)                 \
    X(uint32_t, NoValL, 512, 16)                \
    X(int64_t, NoValL, 512, 8)                  \
    X(uint64_t, NoValL, 512, 8)                 \
    X(int32_t, uint32_t, 512, 16)               \
    X(uint32_t, uint32_t, 512, 16)              \
    X(int64_t, uint32_t, 512, 8)                \
    X(uint64_t, uint32_t, 512, 8)               \
    X(int32_t, uint64_t, 512, 8)                \
    X(uint32_t, uint64_t, 512, 8)               \
    X(int64_t, uint64_t, 512, 8)                \
    X(uint64_t, uint64_t, 512, 8)

template <typename K> struct KeyOf;
template <> struct KeyOf<int32_t> { static constexpr int code = kI32; };
template <> struct KeyOf<uint32_t> { static constexpr int code = kU32; };
template <> struct KeyOf<int64_t> { static constexpr int code = kI64; };
template <> struct KeyOf<uint64_t> { static constexpr int code = kU64; };
template <typename V> struct ValSize { static constexpr int v = sizeof(V); };
template <> struct ValSize<NoValL> { static constexpr int v = 0; };

const void *leaf_kernel_ptr(int key, int esize_v) {
#define X(K, V, TH, IPT)                                                     \
    if (KeyOf<K>::code == key && ValSize<V>::v == esize_v)                   \
        return LeafCfg<K, V, TH, IPT>::fn();
    IM_LEAF_CASES(X)
#undef X
    return nullptr;
}

int leaf_grid(int esize_k, int esize_v) {
    int th, ipt;
    size_t lds;
    leaf_geometry(esize_k, esize_v, &th, &ipt, &lds);
    int key = esize_k == 4 ? kI32 : kI64;
    const void *fn = leaf_kernel_ptr(key, esize_v);
    if (!fn) return 0;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, th, lds) != hipSuccess) return 0;
    if (per_cu < 1) return 0;
    return per_cu * cus;
}

hipError_t launch_leafmerge(int key, int esize_v, void *keys, void *vals, const Plan &pl,
                            const Work &w, hipStream_t s) {
    int th, ipt;
    size_t lds;
    int esize_k = (key == kI32 || key == kU32) ? 4 : 8;
    leaf_geometry(esize_k, esize_v, &th, &ipt, &lds);
    const void *fn = leaf_kernel_ptr(key, esize_v);
    if (!fn) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    Plan plc = pl;
    Work wc = w;
    void *args[] = {&keys, &vals, &plc, &wc};
    return hipLaunchCooperativeKernel(fn, dim3(pl.grid_leaf), dim3(th), args, (unsigned)lds, s);
}

}  // namespace imerge
