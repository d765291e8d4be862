// im_leaf.hip -- merge of the pairs produced by the division stage.
//
// After the division (Sec. 3; Alg. 3), each leaf is a contiguous pair
// A_p | B_p whose merged output occupies exactly the leaf's own region, so
// leaves are independent (the per-pair merge of Alg. 2/3).  A leaf is cut
// into tiles of `tile` output elements (for a single instance: the cells of
// `tile` outputs of the whole output that the leaf meets); the co-rank of
// every tile diagonal inside its leaf is known (k_tilerank, or the cell
// co-ranks found before the division moves data).  One workgroup merges one
// tile:
//   1. load its A-slice and B-slice into LDS (coalesced, contiguous);
//   2. every thread finds its own sub-diagonal by a co-rank search in LDS and
//      merges `ipt` outputs into registers (stable: ties take A);
//   3. outputs go back to LDS (padded to avoid bank conflicts);
//   4. wait: the tile's output window overlaps input slices of other tiles
//      of the same leaf.  Every tile publishes "inputs read" in its own flag
//      as soon as its slices are in LDS; before storing, a tile waits for
//      the flags of exactly the tiles that read its window (k_tiledeps
//      computes them from the co-ranks, with the rest of the tile's
//      geometry, into one record per slot: the tiles whose A-slices meet the
//      window's A elements and those whose B-slices meet its B elements,
//      two contiguous ranges of a few tiles each; A elements only move
//      right and B elements only move left, so the first range starts at or
//      after the tile and the second ends at or before it);
//   5. coalesced store of the window.
// The grid is persistent and co-resident (cooperative launch).  Workgroup b
// takes slots b, b+G, ..., b+(depth-1)G and then further slots from a
// device counter, in increasing order, each after the wait of the step
// before the slot is staged.  Within a leaf the slots visit the tiles in
// increasing order when every A element moves right by at most the leaf
// span (the leaf's B-part is within the span, or the whole leaf is within
// the leaf capacity), else in decreasing order (then its A-part is within
// the span and every B element moves left by at most the span).  The
// planner keeps every reader less than depth*G slots after the tile it
// reads.  Deadlock freedom (depth d): suppose every workgroup that still has
// tiles waits, and let s be the smallest slot not yet stored.  A waiting
// workgroup has staged every slot it holds: the one it waits to store, d-2
// merged into further register sets and one staged in LDS, all at or after
// s.  Either every slot has been handed out (and so staged), or each
// workgroup holds d, and the contiguous handed-out range reaches at least
// s+dG.  Either way the readers of s's window, less than dG slots after s,
// have read their inputs, so s is stored.  The wait is bounded: on expiry
// the workgroup raises an error bit and skips its store.
#include <limits>
#include <type_traits>
#include "im_common.h"
#include "im_search.h"

namespace imerge {

struct NoValL {};

constexpr unsigned kSpinLimit = 1u << 26;

// LDS slots of a tile: T inputs, the B sentinel and the reads of the last
// thread's steps past the end (their outputs are discarded).
template <int T, int IPT>
struct LdsPad { static constexpr int elems = T + IPT + 2; };

template <typename K>
__device__ __forceinline__ K key_max() {
    return std::numeric_limits<K>::max();
}

// The slot index is the same in every lane: the geometry is read once per
// wave and kept in scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int32_t uniform32(int32_t v) {
    return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}

// Geometry of the tile processed in slot s (the slot order reverses the
// tiles of a dir-1 leaf): one record, its loads issued together.
__device__ __forceinline__ TileGeo tile_geo(const Work &w, int64_t s) {
    const TileGeo *r = w.tile_geo + uniform64(s);
    TileGeo g;
    g.out0 = uniform64(r->out0);
    g.a0 = uniform64(r->a0);
    g.b0 = uniform64(r->b0);
    g.tbase = uniform64(r->tbase);
    g.n = uniform32(r->n);
    g.na = uniform32(r->na);
    g.ntiles = uniform32(r->ntiles);
    g.local = uniform32(r->local);
    g.alo = uniform32(r->alo);
    g.ahi = uniform32(r->ahi);
    g.blo = uniform32(r->blo);
    g.bhi = uniform32(r->bhi);
    return g;
}

// Raw buffer resources (base, byte size): a buffer access takes a 32-bit
// per-lane offset next to a wave-uniform descriptor, so the tile loops need
// no 64-bit address per element.  Word 3 selects a raw 32-bit buffer
// without swizzling on CDNA.
constexpr int kBufWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, kBufWord3);
}

// Copy a tile's A-slice and B-slice (one contiguous logical range [0, n))
// into LDS with LDS-DMA loads (global_load_lds_dword): no registers, every
// load of the tile in flight at once.  The copy runs over 32-bit words: lane
// slot j = tid + u*THREADS moves word j of the LDS image, i.e. word j % D of
// element j / D (D words per element); a wave's 64 slots are contiguous in
// LDS, as the DMA requires (destination = wave base + 4 * lane).  Words below
// na*D come from the A-slice, the rest from the B-slice.  The caller waits
// for completion (vmcnt) before reading.  (Measured: the buffer-descriptor
// form of the same DMA, buffer_load_dword ... lds, is about 6% slower here.)
template <typename E, int THREADS, int IPT>
__device__ __forceinline__ void stage_tile_dma(const E *__restrict__ base_ptr, const TileGeo &g,
                                               E *__restrict__ s) {
    constexpr int D = (int)(sizeof(E) / 4);
    const uint32_t *A = reinterpret_cast<const uint32_t *>(base_ptr + g.a0);
    const uint32_t *B = reinterpret_cast<const uint32_t *>(base_ptr + g.b0);
    uint32_t *S = reinterpret_cast<uint32_t *>(s);
    int xb = threadIdx.x;
    asm volatile("" : "+v"(xb));
    const int wbase = __builtin_amdgcn_readfirstlane(threadIdx.x & ~63);
    const int naw = g.na * D, nw = g.n * D;
    // A whole tile (every tile of a leaf but its last) loads every slot: one
    // uniform test for the tile instead of an exec mask around each load.
    if (nw == THREADS * IPT * D) {
#pragma unroll
        for (int u = 0; u < IPT * D; ++u) {
            const int j = xb + u * THREADS;
            const uint32_t *src = j < naw ? A + j : B + (j - naw);
            __builtin_amdgcn_global_load_lds(src, S + wbase + u * THREADS, 4, 0, 0);
        }
    } else {
#pragma unroll
        for (int u = 0; u < IPT * D; ++u) {
            const int j = xb + u * THREADS;
            if (j < nw) {
                const uint32_t *src = j < naw ? A + j : B + (j - naw);
                __builtin_amdgcn_global_load_lds(src, S + wbase + u * THREADS, 4, 0, 0);
            }
        }
    }
}

// Cache policy of the merged output's stores: non-temporal (the NT bit of
// the gfx950 cache-policy operand).  Nothing reads a window again in the
// kernel that writes it, and the streaming hint keeps the written lines from
// lingering dirty in the caches, where the next stage's traffic would have
// to push them out.  (Measured on the 2^27 + 2^27 merge: 1.04 against
// 1.07 ms, the leaf stage and the next merge's exchanges both faster;
// non-temporal loads of the tile inputs, or stores in the exchange kernel,
// were slower.)
constexpr int kStoreNT = 2;

// Store one element through a buffer descriptor (byte offset).
template <typename E>
__device__ __forceinline__ void buf_store(E v, __amdgpu_buffer_rsrc_t r, int off) {
    if constexpr (sizeof(E) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, kStoreNT);
    } else {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, kStoreNT);
    }
}

__device__ __forceinline__ void wait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The tile whose bounded wait expired in some thread of the workgroup
// (its tile index; -1 before any).  Every kernel that waits sets it to -1
// before its first barrier.
__shared__ int64_t s_expired;

__device__ __forceinline__ void init_wait_state() {
    if (threadIdx.x == 0) s_expired = -1;
}

// Wait until every tile that reads this window has its inputs on chip.
// Flags are touched only with relaxed device-scope atomics: the readers'
// loads have returned before they publish, and an acquire/release fence at
// device scope would write back or invalidate this XCD's whole L2 on every
// poll.  Returns false if the bounded wait expired: a thread whose wait
// expires writes the tile's index into s_expired, and after the barrier the
// whole workgroup sees it (a plain barrier and one LDS read instead of a
// workgroup reduction).
template <int THREADS>
__device__ __forceinline__ bool wait_window(const TileGeo &g, const Plan &pl, const Work &w) {
    if (g.ntiles <= 1) return true;
    const int na = g.ahi >= g.alo ? g.ahi - g.alo + 1 : 0;
    const int nb = g.bhi >= g.blo ? g.bhi - g.blo + 1 : 0;
    const int64_t tag = g.tbase + g.local;
    for (int x = (int)threadIdx.x; x < na + nb; x += THREADS) {
        const int q = x < na ? g.alo + x : g.blo + (x - na);
        if (q == g.local) continue;
        const unsigned *f = &w.tile_flag[g.tbase + q];
        unsigned spins = 0;
        bool expired = false;
        while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != pl.epoch) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit) { expired = true; break; }
        }
        if (expired) {
            s_expired = tag;
            break;
        }
    }
    __syncthreads();
    const bool bad = s_expired == tag;
    if (bad && threadIdx.x == 0) raise_error(w, kErrBarrierSpin);
    return !bad;
}

// "Inputs read": the tile's loads have returned in every thread.
__device__ __forceinline__ void publish_read(const TileGeo &g, const Plan &pl, const Work &w) {
    if (g.ntiles > 1 && threadIdx.x == 0)
        __hip_atomic_store(&w.tile_flag[g.tbase + g.local], pl.epoch, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Pieces of the leaf-merge pipeline for one workgroup.
// WIDE: 16-byte groups in the transpose and the stores where the element
// allows it (off for the depth-4 pipeline, whose three register sets leave
// no room for the aligned register quads those accesses need).
template <typename K, typename V, int THREADS, int IPT, bool WIDE = true>
struct LeafOps {
    static constexpr int T = THREADS * IPT;
    static constexpr bool HAS_V = !std::is_same<V, NoValL>::value;
    static constexpr int PE = LdsPad<T, IPT>::elems;
    static constexpr int VN = HAS_V ? IPT : 1;
    // 4-byte keys alone leave the merge in 16-byte groups (VQ per thread, VR
    // outputs left over) and are stored 16 bytes at a time
    static constexpr bool VEC = WIDE && sizeof(K) == 4 && !HAS_V && IPT >= 4;
    static constexpr int VQ = IPT / 4;
    static constexpr int VR = IPT % 4;

    // Load the tile's slices into LDS and publish "inputs read".
    static __device__ __forceinline__ void stage(const K *keys, const V *vals, const TileGeo &g,
                                                 K *sk, V *sv, const Plan &pl, const Work &w) {
        stage_tile_dma<K, THREADS, IPT>(keys, g, sk);
        if constexpr (HAS_V) stage_tile_dma<V, THREADS, IPT>(vals, g, sv);
        wait_dma();
        if (threadIdx.x == 0) sk[g.n] = key_max<K>();   // B sentinel
        __syncthreads();
        if (g.ntiles > 1 && threadIdx.x == 0)
            __hip_atomic_store(&w.tile_flag[g.tbase + g.local], pl.epoch, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }

    // Merge the tile held in LDS into registers (stable: ties take A), then
    // transpose through LDS so that thread p holds outputs p + u*THREADS
    // (coalesced stores).  Leaves the LDS free.  `before_last_sync` runs
    // before the closing barrier (the pipeline hands its next slot over
    // there instead of with a barrier of its own).
    template <bool MATERIALISE, typename Pre>
    static __device__ __forceinline__ void merge(const TileGeo &g, K *sk, V *sv, K (&out)[IPT],
                                                 V (&vout)[VN], Pre before_last_sync) {
        const int tid = threadIdx.x;
        const int n = g.n, na = g.na, nb = g.n - g.na;
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
            // qa, qb: the next A and the next B element in LDS.  A sentinel
            // (the key type's maximum) follows B, so an exhausted B never
            // wins (a <= max, and ties take A anyway); an exhausted A is
            // tested by position, but only in a wave where some lane can
            // reach the end of A within its IPT steps (lane 63 starts
            // furthest along A): elsewhere a <= b alone decides.  Steps past
            // the tile end (last thread) read the padding and their outputs
            // are not stored.
            const K *qa = sk + lo;
            const K *qb = sk + (na + (d - lo));
            const K *const qa_end = sk + na;
            K a = *qa;
            K b = *qb;
            const bool a_may_end = __builtin_amdgcn_readlane(lo, 63) + IPT > na;
            // branch-free steps (selects only): no per-step exec masks
            auto step = [&](int e, bool ta) {
                K o = ta ? a : b;
                // With two register sets live (depth 3), materialise the
                // output now: otherwise the select is sunk to its use and
                // both candidates plus the mask stay live, which spills.
                if constexpr (MATERIALISE) asm volatile("" : "+v"(o));
                out[e] = o;
                const K *q = ta ? qa : qb;
                if constexpr (HAS_V) vout[e] = sv[q - sk];
                const K v = q[1];
                qa = ta ? q + 1 : qa;
                qb = ta ? qb : q + 1;
                a = ta ? v : a;
                b = ta ? b : v;
            };
            if (a_may_end) {
#pragma unroll
                for (int e = 0; e < IPT; ++e) step(e, (qa < qa_end) && (a <= b));
            } else {
#pragma unroll
                for (int e = 0; e < IPT; ++e) step(e, a <= b);
            }
        }
        __syncthreads();                     // LDS inputs of this tile are dead
        // blocked -> striped: IPT is odd, so the blocked writes (stride IPT
        // words) hit distinct banks.  No test against n: every position is
        // below THREADS * IPT, inside the tile's LDS, and outputs past n are
        // never stored (no branch per output, which costs registers).
        const int x0 = tid * IPT;
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            sk[x0 + e] = out[e];
            if constexpr (HAS_V) sv[x0 + e] = vout[e];
        }
        __syncthreads();
        int xb = tid;
        asm volatile("" : "+v"(xb));
        if constexpr (VEC) {
            // 16-byte groups: thread p takes outputs 4p + u*4*THREADS .. +3
            // (one 16-byte LDS read each), then the IPT mod 4 outputs left
            // over one by one (striped).  Reads past n stay in the tile's
            // LDS and are never stored.
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int u = 0; u < VQ; ++u) {
                const int x = 4 * xb + u * 4 * THREADS;
                const u32x4 v = *reinterpret_cast<const u32x4 *>(sk + x);
                // take the four words out of the register quad one by one,
                // so that the held outputs need no aligned quads (with three
                // register sets live that would spill)
                uint32_t w0 = v.x, w1 = v.y, w2 = v.z, w3 = v.w;
                asm volatile("" : "+v"(w0), "+v"(w1), "+v"(w2), "+v"(w3));
                out[4 * u] = __builtin_bit_cast(K, w0);
                out[4 * u + 1] = __builtin_bit_cast(K, w1);
                out[4 * u + 2] = __builtin_bit_cast(K, w2);
                out[4 * u + 3] = __builtin_bit_cast(K, w3);
            }
#pragma unroll
            for (int r = 0; r < VR; ++r) out[4 * VQ + r] = sk[VQ * 4 * THREADS + xb + r * THREADS];
        } else {
#pragma unroll
            for (int u = 0; u < IPT; ++u) {
                out[u] = sk[xb + u * THREADS];
                if constexpr (HAS_V) vout[u] = sv[xb + u * THREADS];
            }
        }
        before_last_sync();
        __syncthreads();
    }

    static __device__ __forceinline__ bool wait_readers(const TileGeo &g, const Plan &pl,
                                                        const Work &w) {
        return wait_window<THREADS>(g, pl, w);
    }

    // Coalesced store of the window from registers (16-byte stores where the
    // outputs were taken in 16-byte groups: a wave writes 1 KB per store).
    static __device__ __forceinline__ void store(K *keys, V *vals, const TileGeo &g,
                                                 const K (&out)[IPT], const V (&vout)[VN]) {
        const int n = g.n;
        int xb = threadIdx.x;
        asm volatile("" : "+v"(xb));
        const __amdgpu_buffer_rsrc_t ro = buf_rsrc(keys + g.out0, (int64_t)n * sizeof(K));
        if constexpr (VEC) {
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int u = 0; u < VQ; ++u) {
                const int x = 4 * xb + u * 4 * THREADS;
                if (x + 3 < n) {
                    // (copied into a fresh quad, as at the LDS read)
                    uint32_t w0 = __builtin_bit_cast(uint32_t, out[4 * u]);
                    uint32_t w1 = __builtin_bit_cast(uint32_t, out[4 * u + 1]);
                    uint32_t w2 = __builtin_bit_cast(uint32_t, out[4 * u + 2]);
                    uint32_t w3 = __builtin_bit_cast(uint32_t, out[4 * u + 3]);
                    asm volatile("" : "+v"(w0), "+v"(w1), "+v"(w2), "+v"(w3));
                    u32x4 v;
                    v.x = w0;
                    v.y = w1;
                    v.z = w2;
                    v.w = w3;
                    __builtin_amdgcn_raw_buffer_store_b128(v, ro, x * 4, 0, kStoreNT);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (x + k < n) buf_store<K>(out[4 * u + k], ro, (x + k) * 4);
                }
            }
#pragma unroll
            for (int r = 0; r < VR; ++r) {
                const int x = VQ * 4 * THREADS + xb + r * THREADS;
                if (x < n) buf_store<K>(out[4 * VQ + r], ro, x * 4);
            }
            return;
        }
        // (outputs past n fall outside the descriptors' ranges: dropped)
#pragma unroll
        for (int u = 0; u < IPT; ++u)
            buf_store<K>(out[u], ro, (xb + u * THREADS) * (int)sizeof(K));
        if constexpr (HAS_V) {
            const __amdgpu_buffer_rsrc_t rv =
                buf_rsrc(vals + g.out0, (int64_t)n * sizeof(V));
#pragma unroll
            for (int u = 0; u < IPT; ++u)
                buf_store<V>(vout[u], rv, (xb + u * THREADS) * (int)sizeof(V));
        }
    }
};

// Slots after each workgroup's static ones come from a counter, in
// increasing order, so that a workgroup that runs slower takes fewer tiles
// instead of falling behind the others (with s -> s mod G the slowest
// workgroup sets the pace, and the others wait for its tiles' flags).  A
// workgroup takes a slot only after its wait of the step before the slot is
// staged, so a waiting workgroup has staged every slot it holds; thread 0
// takes it and hands it over through LDS after the next merge, by which
// time the counter's answer has long returned.
__device__ __forceinline__ unsigned long long take_slot(const Work &w) {
    return atomicAdd(&w.ctr->leaf_next, 1ull);
}

// The slot taken last step (thread 0's `pend`, offset by the static slots),
// as a wave-uniform value in every thread.
__device__ __forceinline__ int64_t hand_over(int64_t *s_slot, unsigned long long pend,
                                             int64_t first, int64_t ntiles, bool taken) {
    if (threadIdx.x == 0) s_slot[0] = taken ? first + (int64_t)pend : ntiles;
    __syncthreads();
    return uniform64(s_slot[0]);
}

// Pipeline state of one workgroup: tile g (merged, in registers `cur`),
// at depth 4 tile gm (merged, in a second register set), tile g1 (staged in
// LDS), and whether gm and g1 exist.
struct LeafPipe {
    int64_t ntiles, first;  // tiles; first slot handed out by the counter ((DEPTH-1)*G)
    bool hasm, has1;
    TileGeo g, gm, g1;
};

// One step: merge g1 from LDS into `nxt`, stage the slot taken last step
// into LDS, wait for the readers of g's window, take the next slot, store g
// from `cur`, advance.  Returns false after the workgroup's last tile.
template <typename K, typename V, int THREADS, int IPT>
__device__ __forceinline__ bool leaf_step(K *keys, V *vals, K *sk, V *sv, const Plan &pl,
                                          const Work &w, LeafPipe &p, int64_t *s_slot,
                                          unsigned long long &pend,
                                          K (&cur)[IPT], V (&vcur)[LeafOps<K, V, THREADS, IPT>::VN],
                                          K (&nxt)[IPT], V (&vnxt)[LeafOps<K, V, THREADS, IPT>::VN]) {
    using Ops = LeafOps<K, V, THREADS, IPT>;
    // the slot taken last step (thread 0's `pend`) reaches every thread
    // through LDS at the merge's closing barrier
    int64_t t2 = p.ntiles;
    if (p.has1) {
        Ops::template merge<true>(p.g1, sk, sv, nxt, vnxt, [&] {
            if (threadIdx.x == 0) s_slot[0] = p.first + (int64_t)pend;
        });
        t2 = uniform64(s_slot[0]);
    }
    const bool has2 = p.has1 && t2 < p.ntiles;
    TileGeo g2 = p.g1;
    if (has2) {
        g2 = tile_geo(w, t2);
        Ops::stage(keys, vals, g2, sk, sv, pl, w);
    }
    const bool ready = Ops::wait_readers(p.g, pl, w);
    if (threadIdx.x == 0 && has2) pend = take_slot(w);
    if (ready) Ops::store(keys, vals, p.g, cur, vcur);
    if (!p.has1) return false;
    p.g = p.g1;
    p.has1 = has2;
    p.g1 = g2;
    return true;
}

// Depth-4 step: as leaf_step, with one more merged tile held in a third
// register set (`mid`) between the one stored this step and the one merged
// this step.  The three sets rotate roles from step to step.
template <typename K, typename V, int THREADS, int IPT>
__device__ __forceinline__ bool leaf_step4(K *keys, V *vals, K *sk, V *sv, const Plan &pl,
                                           const Work &w, LeafPipe &p, int64_t *s_slot,
                                           unsigned long long &pend,
                                           K (&cur)[IPT], V (&vcur)[LeafOps<K, V, THREADS, IPT>::VN],
                                           K (&nxt)[IPT], V (&vnxt)[LeafOps<K, V, THREADS, IPT>::VN]) {
    using Ops = LeafOps<K, V, THREADS, IPT, false>;
    int64_t t2 = p.ntiles;
    if (p.has1) {
        Ops::template merge<true>(p.g1, sk, sv, nxt, vnxt, [&] {
            if (threadIdx.x == 0) s_slot[0] = p.first + (int64_t)pend;
        });
        t2 = uniform64(s_slot[0]);
    }
    const bool has2 = p.has1 && t2 < p.ntiles;
    TileGeo g2 = p.g1;
    if (has2) {
        g2 = tile_geo(w, t2);
        Ops::stage(keys, vals, g2, sk, sv, pl, w);
    }
    const bool ready = Ops::wait_readers(p.g, pl, w);
    if (threadIdx.x == 0 && has2) pend = take_slot(w);
    if (ready) Ops::store(keys, vals, p.g, cur, vcur);
    if (!p.hasm) return false;
    p.g = p.gm;
    p.hasm = p.has1;
    p.gm = p.g1;
    p.has1 = has2;
    p.g1 = g2;
    return true;
}

// Pipeline per workgroup (its static slots b, b+G, ..., then slots from the
// counter; the deadlock argument at the top of this file holds because the
// slots handed out are contiguous and every waiting workgroup holds `depth`
// staged slots, so the slots staged when all wait reach depth*G past the
// oldest unstored one).
//   DEPTH 2: merge t from LDS into registers, stage the next slot into LDS
//            and flag it, wait for the readers of t's window, store t.
//            Readers may be up to 2G-1 slots ahead.
//   DEPTH 3: tile t waits and is stored only after the next slot has been
//            merged into a second register set and the one after staged
//            into LDS and flagged: readers may be up to 3G-1 slots ahead
//            (larger leaves, fewer division levels), at the price of a
//            second register set.
//   DEPTH 4: as depth 3 with a third register set holding one more merged
//            tile: readers may be up to 4G-1 slots ahead.
template <typename K, typename V, int THREADS, int IPT, int DEPTH>
__global__ __launch_bounds__(THREADS, 4) void k_leafmerge(K *__restrict__ keys, V *__restrict__ vals,
                                                          Plan pl, Work w) {
    using Ops = LeafOps<K, V, THREADS, IPT, (DEPTH < 4)>;
    static_assert(DEPTH >= 2 && DEPTH <= 4, "pipeline depth");
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t s_slot[1];
    K *sk = reinterpret_cast<K *>(smem);
    V *sv = reinterpret_cast<V *>(smem + (size_t)Ops::PE * sizeof(K));
    init_wait_state();

    LeafPipe p;
    p.ntiles = (int64_t)w.ctr->tiles;
    if (p.ntiles > pl.cap_tiles) p.ntiles = pl.cap_tiles;
    const int64_t t0 = blockIdx.x;
    if (t0 >= p.ntiles) return;
    const int64_t G = gridDim.x;
    unsigned long long pend = 0;   // thread 0: the counter value taken last

    K ra[IPT];
    V va[Ops::VN];
    p.g = tile_geo(w, t0);
    Ops::stage(keys, vals, p.g, sk, sv, pl, w);
    if constexpr (DEPTH == 2) {
        p.first = G;
        bool more = t0 + G < p.ntiles;
        if (threadIdx.x == 0 && more) pend = take_slot(w);
        for (;;) {
            Ops::template merge<false>(p.g, sk, sv, ra, va, [&] {
                if (threadIdx.x == 0) s_slot[0] = more ? p.first + (int64_t)pend : p.ntiles;
            });
            const int64_t tn = uniform64(s_slot[0]);
            const bool has_next = tn < p.ntiles;
            TileGeo gn = p.g;
            if (has_next) {
                gn = tile_geo(w, tn);
                Ops::stage(keys, vals, gn, sk, sv, pl, w);
            }
            const bool ready = Ops::wait_readers(p.g, pl, w);
            if (threadIdx.x == 0 && has_next) pend = take_slot(w);
            if (ready) Ops::store(keys, vals, p.g, ra, va);
            if (!has_next) break;
            more = true;
            p.g = gn;
        }
    } else if constexpr (DEPTH == 4) {
        K rb[IPT], rc[IPT];
        V vb[Ops::VN], vc[Ops::VN];
        // prologue: b and b+G into registers, b+2G into LDS, the next slot taken
        p.first = 3 * G;
        Ops::template merge<true>(p.g, sk, sv, ra, va, [] {});
        p.hasm = t0 + G < p.ntiles;
        p.gm = p.g;
        p.has1 = false;
        p.g1 = p.g;
        if (p.hasm) {
            p.gm = tile_geo(w, t0 + G);
            Ops::stage(keys, vals, p.gm, sk, sv, pl, w);
            Ops::template merge<true>(p.gm, sk, sv, rb, vb, [] {});
            p.has1 = t0 + 2 * G < p.ntiles;
            if (p.has1) {
                p.g1 = tile_geo(w, t0 + 2 * G);
                Ops::stage(keys, vals, p.g1, sk, sv, pl, w);
                if (threadIdx.x == 0) pend = take_slot(w);
            }
        }
        // the three register sets rotate roles: stored, held, merged into
        for (;;) {
            if (!leaf_step4<K, V, THREADS, IPT>(keys, vals, sk, sv, pl, w, p, s_slot, pend, ra, va,
                                                rc, vc))
                break;
            if (!leaf_step4<K, V, THREADS, IPT>(keys, vals, sk, sv, pl, w, p, s_slot, pend, rb, vb,
                                                ra, va))
                break;
            if (!leaf_step4<K, V, THREADS, IPT>(keys, vals, sk, sv, pl, w, p, s_slot, pend, rc, vc,
                                                rb, vb))
                break;
        }
    } else {
        K rb[IPT];
        V vb[Ops::VN];
        // prologue: b into registers, b+G into LDS, the next slot taken
        p.first = 2 * G;
        Ops::template merge<true>(p.g, sk, sv, ra, va, [] {});
        p.has1 = t0 + G < p.ntiles;
        p.g1 = p.g;
        if (p.has1) {
            p.g1 = tile_geo(w, t0 + G);
            Ops::stage(keys, vals, p.g1, sk, sv, pl, w);
            if (threadIdx.x == 0) pend = take_slot(w);
        }
        // the two register sets alternate roles
        for (;;) {
            if (!leaf_step<K, V, THREADS, IPT>(keys, vals, sk, sv, pl, w, p, s_slot, pend, ra, va,
                                               rb, vb))
                break;
            if (!leaf_step<K, V, THREADS, IPT>(keys, vals, sk, sv, pl, w, p, s_slot, pend, rb, vb,
                                               ra, va))
                break;
        }
    }
}

// ---- one-launch merge of a small pair ---------------------------------------
// A single pair of at most a quarter of the resident tiles is merged by ONE
// launch of plain (non-cooperative) workgroups, one tile each, with no
// division and no planning launches.  Each workgroup finds what the planning
// kernels would give it straight from the keys, six searches side by side,
// one wavefront each with 64 probes per dependent round (im_search.h,
// group_search): the co-ranks of its window's two ends,
// and the tiles that read its window -- the output tiles of the window's
// first and last A elements (A[x] lands at x + #{B < A[x]}) and of its first
// and last B elements (B[y] lands at y + #{A <= B[y]}).  Then, as a leaf
// tile: stage in LDS and publish "inputs read", merge, wait for the readers'
// flags, store.  Every workgroup publishes before it waits, so the waits end
// once every workgroup of the grid has started.  The grid is at most a
// quarter of what the device holds at once: with the stream's earlier work
// finished, its workgroups are dispatched together even beside up to three
// other such launches; a wait that gives up raises the error bit and skips
// its store.  Workgroup 0 resets the counters (no other workgroup writes
// them, except the error bit of a wait that gave up, which takes seconds).
template <typename K, typename V, int THREADS, int IPT>
__global__ __launch_bounds__(THREADS, 4) void k_smallmerge(K *__restrict__ keys, V *__restrict__ vals,
                                                           int64_t la, int64_t lb, Plan pl, Work w) {
    using Ops = LeafOps<K, V, THREADS, IPT>;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t s_geo[6];
    K *sk = reinterpret_cast<K *>(smem);
    V *sv = reinterpret_cast<V *>(smem + (size_t)Ops::PE * sizeof(K));
    init_wait_state();
    const int64_t S = la + lb, T = Ops::T;
    const int64_t ntiles = (S + T - 1) / T;
    const int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int64_t d0 = t * T, d1 = d0 + T < S ? d0 + T : S;
    const K *A = keys, *B = keys + la;
    if (t == 0) {
        constexpr int64_t kWords = (int64_t)(sizeof(Counters) / sizeof(unsigned long long));
        for (int64_t q = threadIdx.x; q < kWords; q += THREADS)
            reinterpret_cast<unsigned long long *>(w.ctr)[q] = 0ull;
        __syncthreads();
        if (threadIdx.x == 0) {
            w.ctr->level_nodes[0] = 1;
            w.ctr->levels_used = 1;
            w.ctr->leaves = 1;
            w.ctr->tiles = (unsigned long long)ntiles;
            w.ctr->leaf_elems = (unsigned long long)S;
        }
    }
    // the six searches, one wave each, 64 probes per dependent round
    const int q = threadIdx.x >> 6;
    if (q < 6) {
        uint32_t rounds = 0;
        int64_t r = -1;
        if (q < 2) {
            // co-rank of diagonal d0 (q = 0) or d1 (q = 1)
            const int64_t d = q == 0 ? d0 : d1;
            const int64_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
            r = group_search<64>(lo, hi, [&](int64_t m) { return A[m] <= B[d - 1 - m]; }, rounds);
        } else if (q < 4) {
            // output tile of the window's first / last A element
            const int64_t x0 = d0, x1 = d1 < la ? d1 : la;
            if (x0 < x1) {
                const int64_t x = q == 2 ? x0 : x1 - 1;
                const K v = A[x];
                r = (x + group_search<64>(0, lb, [&](int64_t m) { return B[m] < v; }, rounds)) / T;
            }
        } else {
            // output tile of the window's first / last B element
            const int64_t y0 = (d0 > la ? d0 : la) - la, y1 = d1 - la;
            if (y0 < y1) {
                const int64_t y = q == 4 ? y0 : y1 - 1;
                const K v = B[y];
                r = (y + group_search<64>(0, la, [&](int64_t m) { return A[m] <= v; }, rounds)) / T;
            }
        }
        if ((threadIdx.x & 63) == 0) s_geo[q] = r;
    }
    __syncthreads();
    const int64_t ia0 = uniform64(s_geo[0]), ia1 = uniform64(s_geo[1]);
    TileGeo g;
    const int n = (int)(d1 - d0);
    int64_t na64 = ia1 - ia0;    // clamped as the planning kernel does (only unsorted input needs it)
    const int64_t na_lo = (d1 - lb - ia0) > 0 ? (d1 - lb - ia0) : 0;
    const int64_t na_hi = (la - ia0) < (int64_t)n ? (la - ia0) : (int64_t)n;
    if (na64 < na_lo) na64 = na_lo;
    if (na64 > na_hi) na64 = na_hi;
    g.out0 = d0;
    g.n = n;
    g.na = (int)na64;
    g.a0 = ia0;
    g.b0 = la + (d0 - ia0);
    g.tbase = 0;
    g.ntiles = (int32_t)ntiles;
    g.local = (int32_t)t;
    const int64_t a_lo = uniform64(s_geo[2]), a_hi = uniform64(s_geo[3]);
    const int64_t b_lo = uniform64(s_geo[4]), b_hi = uniform64(s_geo[5]);
    g.alo = a_lo >= 0 ? (int32_t)a_lo : 0;
    g.ahi = a_lo >= 0 ? (int32_t)a_hi : -1;
    g.blo = b_lo >= 0 ? (int32_t)b_lo : 0;
    g.bhi = b_lo >= 0 ? (int32_t)b_hi : -1;
    Ops::stage(keys, vals, g, sk, sv, pl, w);
    K out[IPT];
    V vout[Ops::VN];
    Ops::template merge<false>(g, sk, sv, out, vout, [] {});
    if (Ops::wait_readers(g, pl, w)) Ops::store(keys, vals, g, out, vout);
}

// ---- wide rows --------------------------------------------------------------
// Leaf merge of rows of W bytes ordered by their leading key: the elements of
// the paper's experiments (Sec. 4), a key followed by a payload.  Rows move
// in chunks of CH = 16, 8 or 4 bytes; a thread holds CPT chunks of a tile and
// a workgroup DEPTH tiles in registers, one of the row kinds below:
//   kind  CH  CPT  DEPTH  tile bytes
//    0     4   40    2     80 KiB   (the paper's largest element, a key and
//    1     8   16    2     64 KiB    16384 ints = 65540 bytes, is one row of
//    2    16    7    3     56 KiB    a kind-0 tile)
//    3    16    8    2     64 KiB
// A tile is R output rows with R * W <= 512 * CPT * CH.  Per tile:
//   1. the keys of its A- and B-slices go to LDS (one load per row);
//   2. each thread merges four consecutive outputs (stable, ties take A) and
//      records each output row's input row in LDS;
//   3. the rows are gathered chunk by chunk straight into registers in
//      output order: chunk c of the tile is chunk c of its output window;
//   4. "inputs read" is published once every load has returned;
//   5. after the readers of the window have published, a coalesced store.
// Grid, slot order and reader ranges are those of k_leafmerge (static slots
// b, b+G, ..., then slots from the counter).  At depth 3 the three register
// sets hold the tile waiting to be stored, the next one, and the one read
// before the wait; at depth 2 the first and last.  The read-ahead argument
// above applies, so a leaf may have DEPTH x G tiles.  The host takes the
// widest chunk that divides W and the address, and among the two 16-byte
// kinds the one whose workgroup holds more bytes of whole rows.
// (Measured on 1 GiB of 64-byte rows: a node of 128 MiB is a leaf for kind 2
// and not for kind 3, so kind 3 would need a fourth division level; seven
// chunks per thread beat six by 4-8% in the leaf stage; eight at depth 3
// spilled registers.)
constexpr int kRowThreads = 512;
constexpr int kRowKinds = 4;
__host__ __device__ constexpr int row_ch(int kind) { return kind == 0 ? 4 : (kind == 1 ? 8 : 16); }
__host__ __device__ constexpr int row_cpt(int kind) {
    return kind == 0 ? 40 : (kind == 1 ? 16 : (kind == 2 ? 7 : 8));
}
__host__ __device__ constexpr int row_depth(int kind) { return kind == 2 ? 3 : 2; }
constexpr int kRowMaxRows = 2048;
constexpr int kRowOutsPerThread = kRowMaxRows / kRowThreads;

template <int CH> struct ChunkT;
template <> struct ChunkT<4> { typedef uint32_t type; };
template <> struct ChunkT<8> { typedef uint32_t type __attribute__((ext_vector_type(2))); };
template <> struct ChunkT<16> { typedef uint32_t type __attribute__((ext_vector_type(4))); };

template <int CH>
__device__ __forceinline__ void chunk_store(typename ChunkT<CH>::type v, __amdgpu_buffer_rsrc_t r,
                                            int off) {
    if constexpr (CH == 4) __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, kStoreNT);
    else if constexpr (CH == 8) __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, kStoreNT);
    else __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, kStoreNT);
}

// Row shape of a call: bytes per row, chunks per row, rows per tile, and
// for cpr >= 2 magic = floor(2^32 / cpr) + 1, so that c / cpr equals the
// high word of c * magic for every chunk index c of a tile (c * cpr < 2^32).
struct RowGeo {
    int64_t W;
    uint32_t magic;
    int32_t cpr, R, pad;
};

template <typename K, int KIND>
struct RowOps {
    static constexpr int CH = row_ch(KIND);
    static constexpr int CPT = row_cpt(KIND);
    typedef typename ChunkT<CH>::type C;

    static __device__ __forceinline__ int64_t row_of(const TileGeo &g, int x) {
        return x < g.na ? g.a0 + x : g.b0 + (x - g.na);
    }

    // Keys to LDS, then the byte offset of the source row of every output
    // row of the tile into so.
    static __device__ __forceinline__ void order(const unsigned char *data, const RowGeo &rg,
                                                 const TileGeo &g, K *sk, int64_t *so) {
        const int tid = threadIdx.x;
        const int n = g.n, na = g.na, nb = g.n - g.na;
        for (int x = tid; x < n; x += kRowThreads)
            sk[x] = *reinterpret_cast<const K *>(data + row_of(g, x) * rg.W);
        if (tid == 0) sk[n] = key_max<K>();   // B sentinel: an exhausted B never wins
        __syncthreads();
        const int d = tid * kRowOutsPerThread;
        if (d < n) {
            int lo = d > nb ? d - nb : 0;
            int hi = d < na ? d : na;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sk[mid] <= sk[na + d - 1 - mid]) lo = mid + 1;
                else hi = mid;
            }
            int ia = lo, bi = na + (d - lo);
#pragma unroll
            for (int e = 0; e < kRowOutsPerThread; ++e) {
                if (d + e < n) {
                    const bool ta = ia < na && sk[ia] <= sk[bi];
                    so[d + e] = row_of(g, ta ? ia : bi) * rg.W;
                    ia += ta ? 1 : 0;
                    bi += ta ? 0 : 1;
                }
            }
        }
        __syncthreads();
    }

    // Gather the tile into registers (output order), wait for the loads,
    // publish "inputs read".  The LDS is free again on return.
    static __device__ __forceinline__ void read(const unsigned char *data, const RowGeo &rg,
                                                const TileGeo &g, K *sk, int64_t *so,
                                                C (&r)[CPT], const Plan &pl, const Work &w) {
        order(data, rg, g, sk, so);
        // Branch-free gather: a lane past the tile's last chunk reloads that
        // chunk (its store is dropped by the store descriptor's range), so
        // every load of the tile is in flight at once.  (A tile always has a
        // row; the uniform test only keeps an empty one from reading so[].)
        const int last = g.n * rg.cpr - 1;
        if (last >= 0) {
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const int c = min((int)threadIdx.x + q * kRowThreads, last);
                const int o = rg.cpr == 1 ? c : (int)__umulhi((uint32_t)c, rg.magic);
                const int part = c - o * rg.cpr;
                r[q] = *reinterpret_cast<const C *>(data + so[o] + part * CH);
            }
        }
        wait_dma();
        __syncthreads();
        publish_read(g, pl, w);
    }

    static __device__ __forceinline__ void store(unsigned char *data, const RowGeo &rg,
                                                 const TileGeo &g, const C (&r)[CPT]) {
        const int nch = g.n * rg.cpr;
        const __amdgpu_buffer_rsrc_t ro = buf_rsrc(data + g.out0 * rg.W, (int64_t)nch * CH);
#pragma unroll
        for (int q = 0; q < CPT; ++q)   // (offsets past nch * CH are dropped)
            chunk_store<CH>(r[q], ro, ((int)threadIdx.x + q * kRowThreads) * CH);
    }
};

template <typename K, int KIND>
__device__ __forceinline__ bool row_step(unsigned char *data, const RowGeo &rg, const Plan &pl,
                                         const Work &w, K *sk, int64_t *so, int64_t ntiles,
                                         int64_t &t, TileGeo &g, int64_t *s_slot,
                                         unsigned long long &pend, bool &more,
                                         typename RowOps<K, KIND>::C (&cur)[RowOps<K, KIND>::CPT],
                                         typename RowOps<K, KIND>::C (&nxt)[RowOps<K, KIND>::CPT]) {
    const int64_t tn = hand_over(s_slot, pend, gridDim.x, ntiles, more);
    const bool has = tn < ntiles;
    TileGeo gn = g;
    if (has) {
        gn = tile_geo(w, tn);
        RowOps<K, KIND>::read(data, rg, gn, sk, so, nxt, pl, w);
    }
    const bool ready = wait_window<kRowThreads>(g, pl, w);
    if (threadIdx.x == 0 && has) pend = take_slot(w);
    if (ready) RowOps<K, KIND>::store(data, rg, g, cur);
    if (!has) return false;
    more = true;
    t = tn;
    g = gn;
    return true;
}

// Depth-3 step: read the slot taken last step into `nxt`, wait for the
// readers of the oldest tile's window, take the next slot, store the oldest
// from `cur`; the tile in between stays in the third register set.
template <typename K, int KIND>
__device__ __forceinline__ bool row_step3(unsigned char *data, const RowGeo &rg, const Plan &pl,
                                          const Work &w, K *sk, int64_t *so, int64_t ntiles,
                                          int64_t first, TileGeo &g, TileGeo &gm, bool &has_m,
                                          int64_t *s_slot, unsigned long long &pend, bool &took,
                                          typename RowOps<K, KIND>::C (&cur)[RowOps<K, KIND>::CPT],
                                          typename RowOps<K, KIND>::C (&nxt)[RowOps<K, KIND>::CPT]) {
    const int64_t t2 = hand_over(s_slot, pend, first, ntiles, took);
    const bool has2 = took && t2 < ntiles;
    TileGeo g2 = gm;
    if (has2) {
        g2 = tile_geo(w, t2);
        RowOps<K, KIND>::read(data, rg, g2, sk, so, nxt, pl, w);
    }
    const bool ready = wait_window<kRowThreads>(g, pl, w);
    if (threadIdx.x == 0 && has2) pend = take_slot(w);
    took = has2;
    if (ready) RowOps<K, KIND>::store(data, rg, g, cur);
    if (!has_m) return false;
    g = gm;
    gm = g2;
    has_m = has2;
    return true;
}

template <typename K, int KIND>
__global__ __launch_bounds__(kRowThreads, 4) void k_leafrows(unsigned char *__restrict__ data,
                                                             RowGeo rg, Plan pl, Work w) {
    using Ops = RowOps<K, KIND>;
    __shared__ K sk[kRowMaxRows + 1];
    __shared__ int64_t so[kRowMaxRows];
    int64_t ntiles = (int64_t)w.ctr->tiles;
    if (ntiles > pl.cap_tiles) ntiles = pl.cap_tiles;
    __shared__ int64_t s_slot[1];
    init_wait_state();
    int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    typename Ops::C ra[Ops::CPT], rb[Ops::CPT];
    TileGeo g = tile_geo(w, t);
    Ops::read(data, rg, g, sk, so, ra, pl, w);
    unsigned long long pend = 0;
    if constexpr (row_depth(KIND) == 3) {
        typename Ops::C rc[Ops::CPT];
        const int64_t G = gridDim.x;
        TileGeo gm = g;
        bool has_m = t + G < ntiles, took = false;
        if (has_m) {
            gm = tile_geo(w, t + G);
            Ops::read(data, rg, gm, sk, so, rb, pl, w);
            took = true;
            if (threadIdx.x == 0) pend = take_slot(w);
        }
        // the three register sets rotate roles: stored, held, read into
        for (;;) {
            if (!row_step3<K, KIND>(data, rg, pl, w, sk, so, ntiles, 2 * G, g, gm, has_m, s_slot,
                                  pend, took, ra, rc))
                break;
            if (!row_step3<K, KIND>(data, rg, pl, w, sk, so, ntiles, 2 * G, g, gm, has_m, s_slot,
                                  pend, took, rb, ra))
                break;
            if (!row_step3<K, KIND>(data, rg, pl, w, sk, so, ntiles, 2 * G, g, gm, has_m, s_slot,
                                  pend, took, rc, rb))
                break;
        }
    } else {
        bool more = t + gridDim.x < ntiles;
        if (threadIdx.x == 0 && more) pend = take_slot(w);
        for (;;) {
            if (!row_step<K, KIND>(data, rg, pl, w, sk, so, ntiles, t, g, s_slot, pend, more, ra, rb)) break;
            if (!row_step<K, KIND>(data, rg, pl, w, sk, so, ntiles, t, g, s_slot, pend, more, rb, ra)) break;
        }
    }
}

template <typename K>
static const void *rows_kernel_kind(int kind) {
    switch (kind) {
        case 0: return (const void *)&k_leafrows<K, 0>;
        case 1: return (const void *)&k_leafrows<K, 1>;
        case 2: return (const void *)&k_leafrows<K, 2>;
        case 3: return (const void *)&k_leafrows<K, 3>;
    }
    return nullptr;
}

static const void *rows_kernel(int key, int kind) {
    switch (key) {
        case kI32: return rows_kernel_kind<int32_t>(kind);
        case kU32: return rows_kernel_kind<uint32_t>(kind);
        case kI64: return rows_kernel_kind<int64_t>(kind);
        case kU64: return rows_kernel_kind<uint64_t>(kind);
    }
    return nullptr;
}

int rows_kinds() { return kRowKinds; }
int rows_chunk_bytes(int kind) { return row_ch(kind); }
int rows_depth(int kind) { return row_depth(kind); }

int rows_tile(int64_t row_bytes, int kind) {
    if (kind < 0 || kind >= kRowKinds || row_bytes <= 0) return 0;
    int64_t r = (int64_t)kRowThreads * row_cpt(kind) * row_ch(kind) / row_bytes;
    if (r > kRowMaxRows) r = kRowMaxRows;
    return r < 1 ? 0 : (int)r;
}

int rows_grid(int key, int kind) {
    const void *fn = rows_kernel(key, kind);
    if (!fn) return 0;
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kRowThreads, 0) != hipSuccess)
        return 0;
    return per_cu < 1 ? 0 : per_cu * cus;
}

hipError_t launch_leafrows(int key, int kind, void *data, int64_t row_bytes, const Plan &pl,
                           const Work &w, hipStream_t s) {
    const void *fn = rows_kernel(key, kind);
    const int R = rows_tile(row_bytes, kind);
    if (!fn || R < 1 || pl.tile != R) return hipErrorInvalidValue;
    const int ch = row_ch(kind);
    if (row_bytes % ch != 0) return hipErrorInvalidValue;
    RowGeo rg;
    rg.W = row_bytes;
    rg.cpr = (int32_t)(row_bytes / ch);
    rg.magic = rg.cpr >= 2 ? (uint32_t)((((uint64_t)1 << 32) / (uint64_t)rg.cpr) + 1) : 0u;
    rg.R = R;
    rg.pad = 0;
    Plan plc = pl;
    Work wc = w;
    unsigned char *d = (unsigned char *)data;
    void *args[] = {&d, &rg, &plc, &wc};
    return hipLaunchCooperativeKernel(fn, dim3(pl.grid_leaf), dim3(kRowThreads), args, 0, s);
}

// ---- out-of-place merge (comparator) ---------------------------------------
// The classic merge into a separate buffer: tile t of the output takes
// in[ia_t, ia_{t+1}) and in[la + t*T - ia_t, ...) (co-ranks of the tile
// diagonals), merged in LDS exactly like a leaf tile, and stored to out.
// No flags and no waits: input and output do not overlap.  One workgroup per
// tile.
template <typename K, int THREADS, int IPT>
__global__ __launch_bounds__(THREADS, 4) void k_merge_oop(const K *__restrict__ in,
                                                          K *__restrict__ out, int64_t la,
                                                          int64_t lb,
                                                          const int64_t *__restrict__ rank,
                                                          int64_t ntiles) {
    using Ops = LeafOps<K, NoValL, THREADS, IPT>;
    extern __shared__ __align__(16) unsigned char smem[];
    K *sk = reinterpret_cast<K *>(smem);
    const int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int64_t S = la + lb;
    const int64_t d0 = t * (int64_t)Ops::T;
    const int64_t d1 = d0 + Ops::T < S ? d0 + Ops::T : S;
    const int n = (int)(d1 - d0);
    const int64_t ia0 = uniform64(rank[t]);
    const int64_t ia1 = t + 1 < ntiles ? uniform64(rank[t + 1]) : la;
    // clamp (only matters for unsorted input): keep both slices inside A, B
    int64_t na = ia1 - ia0;
    const int64_t na_lo = (d1 - lb - ia0) > 0 ? (d1 - lb - ia0) : 0;
    const int64_t na_hi = (la - ia0) < (int64_t)n ? (la - ia0) : (int64_t)n;
    if (na < na_lo) na = na_lo;
    if (na > na_hi) na = na_hi;
    TileGeo g;
    g.out0 = d0;
    g.a0 = ia0;
    g.b0 = la + (d0 - ia0);
    g.n = n;
    g.na = (int)na;
    g.tbase = 0;
    g.ntiles = 1;
    g.local = 0;
    g.alo = 0;
    g.ahi = -1;
    g.blo = 0;
    g.bhi = -1;
    stage_tile_dma<K, THREADS, IPT>(in, g, sk);
    wait_dma();
    if (threadIdx.x == 0) sk[g.n] = key_max<K>();   // B sentinel
    __syncthreads();
    K r[IPT];
    NoValL v[1];
    Ops::template merge<false>(g, sk, nullptr, r, v, [] {});
    Ops::store(out, nullptr, g, r, v);
}

__global__ void k_tile_diagonals(int64_t n, int64_t tile, int64_t *d_k) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t * tile < n) d_k[t] = t * tile;
}

int merge_oop_tile(int esize) { return esize == 4 ? 512 * 35 : 512 * 17; }

hipError_t launch_tile_diagonals(int64_t n, int64_t tile, int64_t *d_k, hipStream_t s) {
    const int64_t nt = (n + tile - 1) / tile;
    if (nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_diagonals, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, n,
                       tile, d_k);
    return hipGetLastError();
}

template <typename K, int IPT>
static hipError_t merge_oop_t(const void *in, void *out, int64_t la, int64_t lb,
                              const int64_t *rank, hipStream_t s) {
    constexpr int TH = 512;
    const int64_t T = (int64_t)TH * IPT;
    const int64_t nt = (la + lb + T - 1) / T;
    if (nt <= 0) return hipSuccess;
    const size_t lds = (size_t)LdsPad<TH * IPT, IPT>::elems * sizeof(K);
    const void *fn = (const void *)&k_merge_oop<K, TH, IPT>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_merge_oop<K, TH, IPT>), dim3((unsigned)nt), dim3(TH), lds, s,
                       (const K *)in, (K *)out, la, lb, rank, nt);
    return hipGetLastError();
}

hipError_t launch_merge_oop(int key, const void *in, void *out, int64_t la, int64_t lb,
                            const int64_t *d_rank, hipStream_t s) {
    switch (key) {
        case kI32: return merge_oop_t<int32_t, 35>(in, out, la, lb, d_rank, s);
        case kU32: return merge_oop_t<uint32_t, 35>(in, out, la, lb, d_rank, s);
        case kI64: return merge_oop_t<int64_t, 17>(in, out, la, lb, d_rank, s);
        case kU64: return merge_oop_t<uint64_t, 17>(in, out, la, lb, d_rank, s);
    }
    return hipErrorInvalidValue;
}

// Readers of each tile's window.  Tile i of a leaf (parts la, lb, size S)
// writes [c_i, c_{i+1}): c_i = iT, or with Plan::cells the boundaries of the
// instance's cells of T outputs inside the leaf (c_0 = 0, c_nt = S).  The A
// elements there, [pa0, pa1) = [c_i, min(c_{i+1}, la)), are read by the
// tiles j whose A-slice [ia(j), ia(j+1)) meets that range: from the first j
// with ia(j+1) > pa0 to the last j with ia(j) < pa1.  The B elements there,
// B indices [pb0, pb1) = [max(c_i, la) - la, c_{i+1} - la), are read by the
// tiles whose B-slice [jb(j), jb(j+1)) meets it, jb(j) = c_j - ia(j): from
// the first j with jb(j+1) > pb0 to the last j with jb(j) < pb1.  An empty
// range is stored as [0, -1].  (Every tile between the window and its last
// reader used to be polled as well: hundreds of device-scope flag loads per
// tile on large leaves, against a handful.)  Each tile's whole geometry goes
// into the record of the slot that processes it, so that the pipeline reads
// one record in one round of loads (it used to follow tile -> leaf -> co-rank
// -> readers, three dependent rounds, about a tenth of a pipeline step).
__global__ __launch_bounds__(256) void k_tiledeps(Plan pl, Work w) {
    int64_t ntiles = (int64_t)w.ctr->tiles;
    if (ntiles > pl.cap_tiles) ntiles = pl.cap_tiles;
    int64_t nleaves = (int64_t)w.ctr->leaves;
    if (nleaves > pl.cap_leaves) nleaves = pl.cap_leaves;
    const int64_t T = pl.tile;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t l;
        if (pl.cells) {
            // leaf = last l with tile_start[l] <= t (no tile search ran)
            int64_t lo = 0, hi = nleaves;
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (w.tile_start[mid] <= t) lo = mid; else hi = mid;
            }
            l = lo;
        } else {
            l = w.tile_leaf[t];
        }
        const Leaf lf = w.leaves[l];
        const int64_t ts = w.tile_start[l];
        const int64_t nt = lf.ntiles;
        const int64_t i = t - ts;
        const int64_t S = lf.la + lf.lb;
        // Leaf-local output start of tile j (j = nt: the leaf's end): j*T, or
        // with cells the boundary of the instance's cell m0 + j.
        const int64_t m0 = pl.cells ? lf.k0 / T : 0;
        auto cstart = [&](int64_t j) -> int64_t {
            if (j >= nt) return S;
            if (j == 0) return 0;
            return pl.cells ? (m0 + j) * T - lf.k0 : j * T;
        };
        // Co-rank at tile j's start; a cell co-rank is clamped to the range a
        // co-rank can take there, which only unsorted runs ever leave.
        auto ia = [&](int64_t j) -> int64_t {
            if (j >= nt) return lf.la;
            if (!pl.cells) return w.tile_rank[ts + j];
            if (j == 0) return 0;
            const int64_t d = cstart(j);
            const int64_t v = w.cell_rank[m0 + j] - lf.i0;
            const int64_t vlo = d - lf.lb > 0 ? d - lf.lb : 0;
            const int64_t vhi = d < lf.la ? d : lf.la;
            return v < vlo ? vlo : (v > vhi ? vhi : v);
        };
        auto jb = [&](int64_t j) -> int64_t { return cstart(j) - ia(j); };
        const int64_t d0 = cstart(i);
        const int64_t d1 = cstart(i + 1);
        int64_t alo = 0, ahi = -1, blo = 0, bhi = -1;
        if (nt > 1) {
            const int64_t pa0 = d0;
            const int64_t pa1 = d1 < lf.la ? d1 : lf.la;
            const int64_t e = d1;
            const int64_t pb0 = (pa0 > lf.la ? pa0 : lf.la) - lf.la;
            const int64_t pb1 = e - lf.la;
            const bool has_a = pa0 < lf.la;          // window holds A elements
            const bool has_b = e > lf.la;            // window holds B elements
            // The four bisections over [0, nt - 1] run side by side, so that
            // each round issues its loads together:
            //   0: first j with ia(j + 1) > pa0  (true at nt - 1: ia(nt) = la > pa0)
            //   1: last j with ia(j) < pa1       (true at 0: ia(0) = 0 < pa1)
            //   2: first j with jb(j + 1) > pb0  (true at nt - 1: jb(nt) = lb > pb0)
            //   3: last j with jb(j) < pb1       (true at 0: jb(0) = 0 < pb1)
            // A search whose part is absent starts empty (lo = hi).
            int64_t lo0 = 0, hi0 = has_a ? nt - 1 : 0, lo1 = 0, hi1 = hi0;
            int64_t lo2 = 0, hi2 = has_b ? nt - 1 : 0, lo3 = 0, hi3 = hi2;
            while (lo0 < hi0 || lo1 < hi1 || lo2 < hi2 || lo3 < hi3) {
                const int64_t m0_ = (lo0 + hi0) >> 1, m1 = (lo1 + hi1 + 1) >> 1;
                const int64_t m2 = (lo2 + hi2) >> 1, m3 = (lo3 + hi3 + 1) >> 1;
                // every index is in [0, nt]; ia(nt) needs no load
                const int64_t v0 = ia(m0_ + 1), v1 = ia(m1), v2 = jb(m2 + 1), v3 = jb(m3);
                if (lo0 < hi0) { if (v0 > pa0) hi0 = m0_; else lo0 = m0_ + 1; }
                if (lo1 < hi1) { if (v1 < pa1) lo1 = m1; else hi1 = m1 - 1; }
                if (lo2 < hi2) { if (v2 > pb0) hi2 = m2; else lo2 = m2 + 1; }
                if (lo3 < hi3) { if (v3 < pb1) lo3 = m3; else hi3 = m3 - 1; }
            }
            if (has_a) { alo = lo0; ahi = lo1; }
            if (has_b) { blo = lo2; bhi = lo3; }
        }
        // the record of the slot that processes tile t (a dir-1 leaf takes
        // its tiles in decreasing order)
        const int64_t n = d1 - d0;
        const int64_t ia0 = ia(i);
        const int64_t ia1 = ia(i + 1);
        // For ascending runs na = ia1 - ia0 already lies in this interval; the
        // clamp only keeps every access inside the leaf when a caller passes
        // unsorted runs (then the result is an unspecified permutation).
        int64_t na = ia1 - ia0;
        const int64_t na_lo = (d1 - lf.lb - ia0) > 0 ? (d1 - lf.lb - ia0) : 0;
        const int64_t na_hi = (lf.la - ia0) < n ? (lf.la - ia0) : n;
        if (na < na_lo) na = na_lo;
        if (na > na_hi) na = na_hi;
        TileGeo g;
        g.out0 = lf.base + d0;
        g.a0 = lf.base + ia0;                    // A elements before the window: ia0
        g.b0 = lf.base + lf.la + (d0 - ia0);     // B elements before the window: d0 - ia0
        g.tbase = ts;
        g.n = (int)n;
        g.na = (int)na;
        g.ntiles = (int32_t)nt;
        g.local = (int32_t)i;
        g.alo = (int32_t)alo;
        g.ahi = (int32_t)ahi;
        g.blo = (int32_t)blo;
        g.bhi = (int32_t)bhi;
        w.tile_geo[ts + (lf.dir ? nt - 1 - i : i)] = g;
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


// ---- geometry and dispatch ----------------------------------------------
// (key bytes, payload bytes, config) -> (threads, items per thread, depth).
// Items per thread are odd, so the blocked LDS accesses are bank-conflict
// free.
//   config 0: 8 waves per tile, about 70 KB of LDS (two workgroups fill a
//             CU), pipeline depth 3 -- depth 4 for 4-byte keys, whose three
//             register sets of 33 items still fit the 128 registers a lane
//             has at two workgroups per CU: the largest leaves.  (Measured
//             on the 2^27+2^27 int32 merge: leaves of 2048 tiles of 16896
//             hold the four 2^26-element nodes of the second level, so the
//             third division level and its exchange go: 0.98 -> 0.84 ms.)
//   config 1: as 0 with depth 2 (one register set, smaller leaves)
//   config 2: 4 waves per tile, same items per thread (half the tile, four
//             workgroups per CU), depth 2: finer grain for many instances
//   config 3: 4 waves per tile, half the items per thread, depth 3
// The tiles the chip holds on chip bound how far a leaf may move elements,
// so the variants trade pipeline overlap against division levels; the
// autotuner measures the trade per workload class.
static int ipt_big(int eb) { return eb <= 4 ? 35 : (eb <= 8 ? 17 : (eb <= 12 ? 11 : 9)); }
static int ipt_small(int eb) { return eb <= 4 ? 17 : (eb <= 8 ? 9 : 5); }

static void geom(int ek, int ev, int cfg, int *th, int *ipt, int *depth) {
    const int eb = ek + ev;
    *th = cfg <= 1 ? 512 : 256;
    *ipt = cfg == 3 ? ipt_small(eb) : ipt_big(eb);
    *depth = (cfg == 0 || cfg == 3) ? 3 : 2;
    if (cfg == 0 && eb <= 4) {
        *ipt = 33;
        *depth = 4;
    }
}

void leaf_geometry(int esize_k, int esize_v, int cfg, int *threads, int *ipt, int *depth,
                   size_t *lds_bytes) {
    geom(esize_k, esize_v, cfg, threads, ipt, depth);
    int T = *threads * *ipt;
    size_t pe = (size_t)(T + *ipt + 2);     // LdsPad
    *lds_bytes = pe * esize_k + pe * esize_v;
}

// One line per (key, payload): the configurations' (threads, items, depth),
// config 0 with its own items and depth.
#define IM_LEAF_KV(X, K, V, IPT0, DEPTH0, BIG, SMALL) \
    X(K, V, 0, 512, IPT0, DEPTH0)                     \
    X(K, V, 1, 512, BIG, 2)                           \
    X(K, V, 2, 256, BIG, 2)                           \
    X(K, V, 3, 256, SMALL, 3)

#define IM_LEAF_CASES(X)                              \
    IM_LEAF_KV(X, int32_t, NoValL, 33, 4, 35, 17)     \
    IM_LEAF_KV(X, uint32_t, NoValL, 33, 4, 35, 17)    \
    IM_LEAF_KV(X, int64_t, NoValL, 17, 3, 17, 9)      \
    IM_LEAF_KV(X, uint64_t, NoValL, 17, 3, 17, 9)     \
    IM_LEAF_KV(X, int32_t, uint32_t, 17, 3, 17, 9)    \
    IM_LEAF_KV(X, uint32_t, uint32_t, 17, 3, 17, 9)   \
    IM_LEAF_KV(X, int64_t, uint32_t, 11, 3, 11, 5)    \
    IM_LEAF_KV(X, uint64_t, uint32_t, 11, 3, 11, 5)   \
    IM_LEAF_KV(X, int32_t, uint64_t, 11, 3, 11, 5)    \
    IM_LEAF_KV(X, uint32_t, uint64_t, 11, 3, 11, 5)   \
    IM_LEAF_KV(X, int64_t, uint64_t, 9, 3, 9, 5)      \
    IM_LEAF_KV(X, uint64_t, uint64_t, 9, 3, 9, 5)

template <typename K> struct KeyOf;
template <> struct KeyOf<int32_t> { static constexpr int code = kI32; };
template <> struct KeyOf<uint32_t> { static constexpr int code = kU32; };
template <> struct KeyOf<int64_t> { static constexpr int code = kI64; };
template <> struct KeyOf<uint64_t> { static constexpr int code = kU64; };
template <typename V> struct ValSize { static constexpr int v = sizeof(V); };
template <> struct ValSize<NoValL> { static constexpr int v = 0; };

const void *leaf_kernel_ptr(int key, int esize_v, int cfg) {
#define X(K, V, C, TH, IPT, DEPTH)                                               \
    if (KeyOf<K>::code == key && ValSize<V>::v == esize_v && C == cfg)         \
        return (const void *)&k_leafmerge<K, V, TH, IPT, DEPTH>;
    IM_LEAF_CASES(X)
#undef X
    return nullptr;
}

static const void *small_kernel_ptr(int key, int esize_v) {
#define X(K, V, C, TH, IPT, DEPTH)                                               \
    if constexpr (C == 0) {                                                      \
        if (KeyOf<K>::code == key && ValSize<V>::v == esize_v)                   \
            return (const void *)&k_smallmerge<K, V, TH, IPT>;                   \
    }
    IM_LEAF_CASES(X)
#undef X
    return nullptr;
}

hipError_t launch_smallmerge(int key, int esize_v, void *keys, void *vals, int64_t la, int64_t lb,
                             const Plan &pl, const Work &w, hipStream_t s) {
    int th, ipt, depth;
    size_t lds;
    const int esize_k = (key == kI32 || key == kU32) ? 4 : 8;
    leaf_geometry(esize_k, esize_v, 0, &th, &ipt, &depth, &lds);
    const void *fn = small_kernel_ptr(key, esize_v);
    if (!fn || pl.tile != (int64_t)th * ipt) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int64_t ntiles = (la + lb + pl.tile - 1) / pl.tile;
    Plan plc = pl;
    Work wc = w;
    void *args[] = {&keys, &vals, &la, &lb, &plc, &wc};
    return hipLaunchKernel(fn, dim3((unsigned)ntiles), dim3(th), args, (unsigned)lds, s);
}

int leaf_grid(int esize_k, int esize_v, int cfg) {
    int th, ipt, depth;
    size_t lds;
    leaf_geometry(esize_k, esize_v, cfg, &th, &ipt, &depth, &lds);
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
    int th, ipt, depth;
    size_t lds;
    int esize_k = (key == kI32 || key == kU32) ? 4 : 8;
    leaf_geometry(esize_k, esize_v, pl.cfg, &th, &ipt, &depth, &lds);
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
