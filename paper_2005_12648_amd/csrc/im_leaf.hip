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
//   4. wait: the tile's output window overlaps input slices of other tiles
//      of the same leaf.  Every tile publishes "inputs read" in its own flag
//      as soon as its slices are in LDS; before storing, a tile waits for
//      the flags of exactly the tiles that read its window (k_tiledeps
//      computes that range from the co-ranks: A elements only move right,
//      B elements only move left, so the readers form one contiguous range
//      of tiles around the tile itself);
//   5. coalesced store of the window.
// The grid is persistent and co-resident (cooperative launch); processing
// slot s is handled by workgroup s mod G in increasing s.  Within a leaf the
// slots visit the tiles in increasing order when every A element moves right
// by at most (G-2) tiles (the leaf's B-part is within the leaf span, or the
// whole leaf has at most G tiles), else in decreasing order (then its A-part
// is within the span and every B element moves left by at most (G-2) tiles).
// Either way every tile that reads a window lies less than G slots after
// it, so the workgroup holding it has finished all its earlier slots: the
// smallest unfinished slot always makes progress and the waits cannot
// deadlock.  The wait is bounded: on expiry the workgroup raises an error
// bit and skips its store.
#include <type_traits>
#include "im_common.h"

namespace imerge {

struct NoValL {};

constexpr unsigned kSpinLimit = 1u << 26;

template <int T>
struct LdsPad { static constexpr int elems = T + 2; };   // + look-ahead slack

// Geometry of one tile: its leaf, output window [d0, d0+n) inside the leaf,
// and where its A-slice (na elements) and B-slice (n - na) start.
struct TileGeo {
    int64_t base, d0, tbase;
    int n, na, a_off, b_off;
    int32_t leaf, ntiles, local, wlo, whi;
};

// Geometry of the tile processed in slot s (the slot order reverses the
// tiles of a dir-1 leaf).
__device__ __forceinline__ TileGeo tile_geo(const Work &w, int64_t s, int T) {
    TileGeo g;
    const int32_t l = w.tile_leaf[s];
    const Leaf lf = w.leaves[l];
    const int64_t sl = s - w.tile_start[l];
    const int64_t local = lf.dir ? (int64_t)lf.ntiles - 1 - sl : sl;
    const int64_t t = w.tile_start[l] + local;
    const int64_t S = lf.la + lf.lb;
    const int64_t d0 = local * (int64_t)T;
    const int64_t d1 = d0 + T < S ? d0 + T : S;
    const int n = (int)(d1 - d0);
    const int64_t ia0 = w.tile_rank[t];
    const int64_t ia1 = (local + 1 < lf.ntiles) ? w.tile_rank[t + 1] : lf.la;
    // For ascending runs na = ia1 - ia0 already lies in this interval; the
    // clamp only keeps every access inside the leaf when a caller passes
    // unsorted runs (then the result is an unspecified permutation).
    int64_t na64 = ia1 - ia0;
    const int64_t na_lo = (d1 - lf.lb - ia0) > 0 ? (d1 - lf.lb - ia0) : 0;
    const int64_t na_hi = (lf.la - ia0) < (int64_t)n ? (lf.la - ia0) : (int64_t)n;
    if (na64 < na_lo) na64 = na_lo;
    if (na64 > na_hi) na64 = na_hi;
    g.base = lf.base;
    g.d0 = d0;
    g.n = n;
    g.na = (int)na64;
    // Offsets relative to the leaf start (a leaf is far below 2^31
    // elements): every address is a uniform base plus one 32-bit offset.
    g.a_off = (int)ia0;                                   // A-slice start
    g.b_off = (int)(lf.la + (d0 - ia0)) - g.na;           // B-slice start, minus na
    g.leaf = l;
    g.ntiles = lf.ntiles;
    g.tbase = w.tile_start[l];
    g.local = (int32_t)local;
    g.wlo = w.tile_dep[2 * t];
    g.whi = w.tile_dep[2 * t + 1];
    return g;
}

// Copy a tile's A-slice and B-slice (one contiguous logical range [0, n))
// into LDS with LDS-DMA loads (global_load_lds_dword): no registers, every
// load of the tile in flight at once.  The copy runs over 32-bit words: lane
// slot j = tid + u*THREADS moves word j of the LDS image, i.e. word j % D of
// element j / D (D words per element); a wave's 64 slots are contiguous in
// LDS, as the DMA requires (destination = wave base + 4 * lane).  The caller
// waits for completion (vmcnt) before reading.
template <typename E, int THREADS, int IPT>
__device__ __forceinline__ void stage_tile_dma(const E *__restrict__ base_ptr, const TileGeo &g,
                                               E *__restrict__ s) {
    constexpr int D = (int)(sizeof(E) / 4);
    const uint32_t *L = reinterpret_cast<const uint32_t *>(base_ptr + g.base);
    uint32_t *S = reinterpret_cast<uint32_t *>(s);
    int xb = threadIdx.x;
    asm volatile("" : "+v"(xb));
    const int wbase = __builtin_amdgcn_readfirstlane(threadIdx.x & ~63);
    const int nw = g.n * D;
#pragma unroll
    for (int u = 0; u < IPT * D; ++u) {
        const int j = xb + u * THREADS;
        if (j < nw) {
            const int x = j / D;                      // D is 1 or 2: a shift
            const int src = x < g.na ? g.a_off + x : g.b_off + x;
            __builtin_amdgcn_global_load_lds(L + (int64_t)src * D + (j - x * D),
                                             S + wbase + u * THREADS, 4, 0, 0);
        }
    }
}

__device__ __forceinline__ void wait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Pipeline per workgroup (slots t, t+G, t+2G, ...):
//   merge(t) from LDS into registers -> transpose the outputs through LDS
//   (blocked -> striped) -> stage(t+G) into LDS and publish its flag ->
//   wait for the readers of t's window -> coalesced store of t from
//   registers.
// The next tile is staged and flagged before this tile waits, so a tile's
// flag only needs the workgroup's slot two rounds back to be finished: the
// readers (at most G-1 slots ahead, see the leaf span) are always reachable
// with a full round of slack, and waits rarely stall.
template <typename K, typename V, int THREADS, int IPT>
__global__ __launch_bounds__(THREADS, 4) void k_leafmerge(K *__restrict__ keys, V *__restrict__ vals,
                                                          Plan pl, Work w) {
    constexpr int T = THREADS * IPT;
    constexpr bool HAS_V = !std::is_same<V, NoValL>::value;
    constexpr int PE = LdsPad<T>::elems;
    extern __shared__ __align__(16) unsigned char smem[];
    K *sk = reinterpret_cast<K *>(smem);
    V *sv = reinterpret_cast<V *>(smem + (size_t)PE * sizeof(K));

    const int tid = threadIdx.x;
    int64_t ntiles = (int64_t)w.ctr->tiles;
    if (ntiles > pl.cap_tiles) ntiles = pl.cap_tiles;
    int64_t t = blockIdx.x;
    if (t >= ntiles) return;

    TileGeo g = tile_geo(w, t, T);
    stage_tile_dma<K, THREADS, IPT>(keys, g, sk);
    if constexpr (HAS_V) stage_tile_dma<V, THREADS, IPT>(vals, g, sv);
    wait_dma();
    __syncthreads();
    if (g.ntiles > 1 && tid == 0)            // this tile's inputs are read
        __hip_atomic_store(&w.tile_flag[g.tbase + g.local], pl.epoch, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);

    for (;;) {
        // 1. per-thread merge path inside LDS (stable: ties take A)
        const int n = g.n, na = g.na, nb = g.n - g.na;
        K out[IPT];
        V vout[HAS_V ? IPT : 1];
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
            // sk has PE > n entries, so the look-ahead reads stay inside LDS.
            K a = sk[ia];
            K b = sk[na + ib];
#pragma unroll
            for (int e = 0; e < IPT; ++e) {
                bool ta = (ib >= nb) || (ia < na && a <= b);
                out[e] = ta ? a : b;
                int src = ta ? ia : na + ib;
                if constexpr (HAS_V) vout[e] = sv[src > PE - 1 ? PE - 1 : src];
                int nx = src + 1;
                if (nx > PE - 1) nx = PE - 1;
                K v = sk[nx];
                if (ta) { ++ia; a = v; } else { ++ib; b = v; }
            }
        }
        __syncthreads();                     // LDS inputs of this tile are dead

        // 2. blocked -> striped through LDS: thread p holds outputs
        // p*IPT + e; after the round trip it holds tid + u*THREADS, so the
        // final stores are coalesced.  IPT is odd: the blocked writes (stride
        // IPT words) hit distinct banks.
        {
            const int x0 = tid * IPT;
#pragma unroll
            for (int e = 0; e < IPT; ++e) {
                if (x0 + e < n) {
                    sk[x0 + e] = out[e];
                    if constexpr (HAS_V) sv[x0 + e] = vout[e];
                }
            }
            __syncthreads();
            int xb = tid;
            asm volatile("" : "+v"(xb));
#pragma unroll
            for (int u = 0; u < IPT; ++u) {
                const int x = xb + u * THREADS;
                if (x < n) {
                    out[u] = sk[x];
                    if constexpr (HAS_V) vout[u] = sv[x];
                }
            }
            __syncthreads();
        }

        // 3. stage the next tile of this workgroup and publish its flag
        const int64_t tn = t + gridDim.x;
        const bool has_next = tn < ntiles;
        TileGeo gn = g;
        if (has_next) {
            gn = tile_geo(w, tn, T);
            stage_tile_dma<K, THREADS, IPT>(keys, gn, sk);
            if constexpr (HAS_V) stage_tile_dma<V, THREADS, IPT>(vals, gn, sv);
            wait_dma();
        }
        __syncthreads();
        if (has_next && gn.ntiles > 1 && tid == 0)
            __hip_atomic_store(&w.tile_flag[gn.tbase + gn.local], pl.epoch, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);

        // 4. wait until every tile that reads this window has its inputs in
        // LDS.  Flags are touched only with relaxed device-scope atomics: the
        // readers' loads have returned before they publish, and an
        // acquire/release fence at device scope would write back or
        // invalidate this XCD's whole L2 on every poll.
        int ok = 1;
        if (g.ntiles > 1) {
            int bad = 0;
            for (int q = g.wlo + tid; q <= g.whi && !bad; q += THREADS) {
                if (q == g.local) continue;
                const unsigned *f = &w.tile_flag[g.tbase + q];
                unsigned spins = 0;
                while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
                       pl.epoch) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > kSpinLimit) { bad = 1; break; }
                }
            }
            bad = __syncthreads_or(bad);
            if (bad) {
                if (tid == 0) atomicOr(&w.ctr->error, kErrBarrierSpin);
                ok = 0;
            }
        }

        // 5. coalesced store of this tile's window from registers
        if (ok) {
            int xb = tid;
            asm volatile("" : "+v"(xb));
            K *O = keys + g.base + g.d0;
#pragma unroll
            for (int u = 0; u < IPT; ++u) {
                const int x = xb + u * THREADS;
                if (x < n) O[x] = out[u];
            }
            if constexpr (HAS_V) {
                V *OV = vals + g.base + g.d0;
#pragma unroll
                for (int u = 0; u < IPT; ++u) {
                    const int x = xb + u * THREADS;
                    if (x < n) OV[x] = vout[u];
                }
            }
        }
        if (!has_next) break;
        t = tn;
        g = gn;
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

// Readers of each tile's window.  Tile i of a leaf (parts la, lb, size S)
// writes [iT, min((i+1)T, S)).  The A elements there, [iT, min((i+1)T, la)),
// are read by the tiles j whose A-slice [ia(j), ia(j+1)) meets that range;
// A elements only move right, so these are tiles >= i and the last one is
// the last j with ia(j) < min((i+1)T, la).  The B elements there, B indices
// [max(iT, la) - la, min((i+1)T, S) - la), only move left: their readers
// are tiles <= i, the first being the first j with jb(j+1) > max(iT,la)-la,
// where jb(j) = min(jT, S) - ia(j).  dep = [first B reader, last A reader].
__global__ __launch_bounds__(256) void k_tiledeps(Plan pl, Work w) {
    int64_t ntiles = (int64_t)w.ctr->tiles;
    if (ntiles > pl.cap_tiles) ntiles = pl.cap_tiles;
    const int64_t T = pl.tile;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t l = w.tile_leaf[t];
        const Leaf lf = w.leaves[l];
        const int64_t ts = w.tile_start[l];
        const int64_t nt = lf.ntiles;
        const int64_t i = t - ts;
        const int64_t S = lf.la + lf.lb;
        int64_t wlo = i, whi = i;
        if (nt > 1) {
            auto ia = [&](int64_t j) -> int64_t { return j < nt ? w.tile_rank[ts + j] : lf.la; };
            auto jb = [&](int64_t j) -> int64_t {
                int64_t d = j * T < S ? j * T : S;
                return d - ia(j);
            };
            const int64_t pa0 = i * T;
            const int64_t pa1 = (i + 1) * T < lf.la ? (i + 1) * T : lf.la;
            if (pa0 < lf.la) {                       // window holds A elements
                int64_t lo = 0, hi = nt - 1;         // ia(0) = 0 < pa1
                while (lo < hi) {
                    int64_t mid = (lo + hi + 1) >> 1;
                    if (ia(mid) < pa1) lo = mid; else hi = mid - 1;
                }
                if (lo > whi) whi = lo;
            }
            const int64_t e = (i + 1) * T < S ? (i + 1) * T : S;
            if (e > lf.la) {                         // window holds B elements
                const int64_t pb0 = (pa0 > lf.la ? pa0 : lf.la) - lf.la;
                int64_t lo = 0, hi = nt - 1;         // jb(nt) = lb > pb0
                while (lo < hi) {
                    int64_t mid = (lo + hi) >> 1;
                    if (jb(mid + 1) > pb0) hi = mid; else lo = mid + 1;
                }
                if (lo < wlo) wlo = lo;
            }
        }
        w.tile_dep[2 * t] = (int32_t)wlo;
        w.tile_dep[2 * t + 1] = (int32_t)whi;
    }
}

__global__ void k_fill32(unsigned *p, int64_t n, unsigned v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_tiledeps(const Plan &pl, const Work &w, hipStream_t s) {
    int64_t g = (pl.cap_tiles + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_tiledeps, dim3((int)g), dim3(256), 0, s, pl, w);
    return hipGetLastError();
}

hipError_t launch_fill32(unsigned *p, int64_t n, unsigned v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill32, dim3((int)g), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_plan(const Plan &pl, const Work &w, hipStream_t s) {
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, s, pl, w);
    return hipGetLastError();
}

// ---- geometry and dispatch ----------------------------------------------
// (key bytes, payload bytes, config) -> (threads, items per thread).  Items
// per thread are odd, so the blocked LDS accesses are bank-conflict free.
//   config 0: 8 waves per tile, about 70 KB of LDS (two workgroups fill a CU)
//   config 1: 4 waves per tile, same items per thread (half the tile, four
//             workgroups per CU): finer granularity for many small instances
//   config 2: 4 waves per tile, half the items per thread (quarter tile)
// The tiles resident on the chip bound how far a leaf may move elements, so
// the smaller tiles trade shorter pipelines for more division levels on
// large merges; the autotuner measures the trade per workload class.
static int ipt_big(int eb) { return eb <= 4 ? 35 : (eb <= 8 ? 17 : (eb <= 12 ? 11 : 9)); }
static int ipt_small(int eb) { return eb <= 4 ? 17 : (eb <= 8 ? 9 : 5); }

static void geom(int ek, int ev, int cfg, int *th, int *ipt) {
    const int eb = ek + ev;
    *th = cfg == 0 ? 512 : 256;
    *ipt = cfg == 2 ? ipt_small(eb) : ipt_big(eb);
}

void leaf_geometry(int esize_k, int esize_v, int cfg, int *threads, int *ipt, size_t *lds_bytes) {
    geom(esize_k, esize_v, cfg, threads, ipt);
    int T = *threads * *ipt;
    size_t pe = (size_t)(T + 2);
    *lds_bytes = pe * esize_k + pe * esize_v;
}

// One line per (key, payload): the three configurations' (threads, items).
#define IM_LEAF_KV(X, K, V, BIG, SMALL) \
    X(K, V, 0, 512, BIG)                \
    X(K, V, 1, 256, BIG)                \
    X(K, V, 2, 256, SMALL)

#define IM_LEAF_CASES(X)                        \
    IM_LEAF_KV(X, int32_t, NoValL, 35, 17)      \
    IM_LEAF_KV(X, uint32_t, NoValL, 35, 17)     \
    IM_LEAF_KV(X, int64_t, NoValL, 17, 9)       \
    IM_LEAF_KV(X, uint64_t, NoValL, 17, 9)      \
    IM_LEAF_KV(X, int32_t, uint32_t, 17, 9)     \
    IM_LEAF_KV(X, uint32_t, uint32_t, 17, 9)    \
    IM_LEAF_KV(X, int64_t, uint32_t, 11, 5)     \
    IM_LEAF_KV(X, uint64_t, uint32_t, 11, 5)    \
    IM_LEAF_KV(X, int32_t, uint64_t, 11, 5)     \
    IM_LEAF_KV(X, uint32_t, uint64_t, 11, 5)    \
    IM_LEAF_KV(X, int64_t, uint64_t, 9, 5)      \
    IM_LEAF_KV(X, uint64_t, uint64_t, 9, 5)

template <typename K> struct KeyOf;
template <> struct KeyOf<int32_t> { static constexpr int code = kI32; };
template <> struct KeyOf<uint32_t> { static constexpr int code = kU32; };
template <> struct KeyOf<int64_t> { static constexpr int code = kI64; };
template <> struct KeyOf<uint64_t> { static constexpr int code = kU64; };
template <typename V> struct ValSize { static constexpr int v = sizeof(V); };
template <> struct ValSize<NoValL> { static constexpr int v = 0; };

const void *leaf_kernel_ptr(int key, int esize_v, int cfg) {
#define X(K, V, C, TH, IPT)                                                      \
    if (KeyOf<K>::code == key && ValSize<V>::v == esize_v && C == cfg)         \
        return (const void *)&k_leafmerge<K, V, TH, IPT>;
    IM_LEAF_CASES(X)
#undef X
    return nullptr;
}

int leaf_grid(int esize_k, int esize_v, int cfg) {
    int th, ipt;
    size_t lds;
    leaf_geometry(esize_k, esize_v, cfg, &th, &ipt, &lds);
    int key = esize_k == 4 ? kI32 : kI64;
    const void *fn = leaf_kernel_ptr(key, esize_v, cfg);
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
    leaf_geometry(esize_k, esize_v, pl.cfg, &th, &ipt, &lds);
    const void *fn = leaf_kernel_ptr(key, esize_v, pl.cfg);
    if (!fn) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    Plan plc = pl;
    Work wc = w;
    void *args[] = {&keys, &vals, &plc, &wc};
    return hipLaunchCooperativeKernel(fn, dim3(pl.grid_leaf), dim3(th), args, (unsigned)lds, s);
}

}  // namespace imerge
