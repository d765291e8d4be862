// im_rotate.hip -- partition exchange X|Y -> Y|X (Sec. 3.4), segmented.
//
// All exchanges of one division level run in one launch.  Each exchange is
// cut into work items of kRotChunk element pairs; the items of a level are
// numbered contiguously exchange after exchange (k_split reserves them with
// one packed atomic, so exchange slots are in item order) and a persistent
// grid walks them.
//
// |X| == |Y|: one linear-shifting step is the whole exchange -- swap X with
//   the block that occupies its destination, element pair by element pair.
//   Every element is read once and written once, with contiguous, coalesced
//   access (the property Sec. 3.4 gives linear shifting over circular
//   shifting).
// |X| != |Y|: linear shifting would need a data-dependent number of
//   dependent steps (one per quotient of Euclid's algorithm on the two
//   lengths), each a grid-wide dependency.  The exchange is instead done as
//   reverse(X), reverse(Y) (phase A) then reverse(X|Y) (phase B): two
//   launches, every element read and written twice, always contiguous.
#include <type_traits>
#include "im_common.h"

namespace imerge {

constexpr int kRotThreads = 256;
constexpr int kRotPer = (int)(kRotChunk / kRotThreads);   // pairs per thread

struct NoVal {};

// 16-byte vectors with only element alignment: gfx950 runs global memory in
// unaligned-access mode, so each becomes one dwordx4 access (used by the
// reversals, where they measured faster than element accesses).
template <typename E>
struct __attribute__((aligned(sizeof(E)))) Vec {
    static constexpr int N = 16 / (int)sizeof(E);
    E v[N];
};

// Swap pairs [c0, c1) of (p[a + t], p[b + t]), one element per lane and
// access (64 lanes = one contiguous 256-byte run per wave and region).
// Measured on MI355X, this beats 16-byte vectors here (two independent
// read streams and two write streams at unrelated alignments).
template <typename E>
__device__ __forceinline__ void swap_chunk(E *__restrict__ p, int64_t a, int64_t b, int64_t c0,
                                           int64_t c1) {
    E x[kRotPer], y[kRotPer];
#pragma unroll
    for (int u = 0; u < kRotPer; ++u) {
        int64_t t = c0 + threadIdx.x + (int64_t)u * kRotThreads;
        if (t < c1) { x[u] = p[a + t]; y[u] = p[b + t]; }
    }
#pragma unroll
    for (int u = 0; u < kRotPer; ++u) {
        int64_t t = c0 + threadIdx.x + (int64_t)u * kRotThreads;
        if (t < c1) { p[a + t] = y[u]; p[b + t] = x[u]; }
    }
}

// Reverse segment [s, s+m): swap pairs (s + t, s + m - 1 - t) for t in
// [c0, c1).  A vector of pairs t..t+W-1 meets the mirrored vector ending at
// s+m-1-t, reversed element-wise; vectors that would overlap the mirror
// (the middle of the segment) or run past c1 fall back to elements.
template <typename E>
__device__ __forceinline__ void rev_chunk(E *__restrict__ p, int64_t s, int64_t m, int64_t c0,
                                          int64_t c1) {
    using V = Vec<E>;
    constexpr int W = V::N;
    constexpr int NV = kRotPer / W;
    V x[NV], y[NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        int64_t t = c0 + (int64_t)(threadIdx.x + u * kRotThreads) * W;
        if (t + W <= c1 && t + W - 1 < m - W - t) {
            x[u] = *reinterpret_cast<const V *>(p + s + t);
            y[u] = *reinterpret_cast<const V *>(p + s + m - W - t);
        }
    }
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        int64_t t = c0 + (int64_t)(threadIdx.x + u * kRotThreads) * W;
        if (t + W <= c1 && t + W - 1 < m - W - t) {
            V rx, ry;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                rx.v[j] = y[u].v[W - 1 - j];
                ry.v[j] = x[u].v[W - 1 - j];
            }
            *reinterpret_cast<V *>(p + s + t) = rx;
            *reinterpret_cast<V *>(p + s + m - W - t) = ry;
        } else {
            for (int j = 0; j < W; ++j) {
                const int64_t tt = t + j;
                if (tt < c1) {
                    E xa = p[s + tt], yb = p[s + m - 1 - tt];
                    p[s + tt] = yb;
                    p[s + m - 1 - tt] = xa;
                }
            }
        }
    }
}

template <typename E>
__device__ __forceinline__ void do_item(E *__restrict__ p, const Rot &R, int64_t local, int phase) {
    if (R.lx == R.ly) {
        if (phase != 0) return;
        int64_t c0 = local * kRotChunk, c1 = c0 + kRotChunk;
        if (c1 > R.lx) c1 = R.lx;
        if (c0 < c1) swap_chunk(p, R.pos, R.pos + R.lx, c0, c1);
        return;
    }
    if (phase == 0) {
        int64_t px = R.lx / 2, py = R.ly / 2;
        int64_t ix = (px + kRotChunk - 1) / kRotChunk;
        int64_t iy = (py + kRotChunk - 1) / kRotChunk;
        if (local < ix) {
            int64_t c0 = local * kRotChunk, c1 = c0 + kRotChunk;
            if (c1 > px) c1 = px;
            rev_chunk(p, R.pos, R.lx, c0, c1);
        } else if (local - ix < iy) {
            int64_t c0 = (local - ix) * kRotChunk, c1 = c0 + kRotChunk;
            if (c1 > py) c1 = py;
            rev_chunk(p, R.pos + R.lx, R.ly, c0, c1);
        }
    } else {
        int64_t m = R.lx + R.ly, pm = m / 2;
        int64_t c0 = local * kRotChunk, c1 = c0 + kRotChunk;
        if (c1 > pm) c1 = pm;
        if (c0 < c1) rev_chunk(p, R.pos, m, c0, c1);
    }
}

template <typename EK, typename EV>
__global__ __launch_bounds__(kRotThreads) void k_rotate(EK *__restrict__ keys, EV *__restrict__ vals,
                                                        const Rot *__restrict__ rot,
                                                        const Counters *__restrict__ ctr,
                                                        int64_t cap_rot, int level, int phase) {
    if (phase == 1 && ctr->level_rev[level] == 0) return;   // only block swaps
    const unsigned long long packed = ctr->level_rot[level];
    int64_t nrot = (int64_t)(packed >> kRotCountShift);
    if (nrot > cap_rot) nrot = cap_rot;
    const int64_t nitems = (int64_t)(packed & kRotWorkMask);
    if (nrot == 0 || nitems == 0) return;
    // Grid-stride over the items; the descriptor of the previous item is
    // reused while it still covers the current one (large exchanges).
    Rot R;
    R.w0 = 1;
    R.nw = 0;        // empty: forces a search for the first item
    for (int64_t wi = blockIdx.x; wi < nitems; wi += gridDim.x) {
        if (wi < R.w0 || wi >= R.w0 + R.nw) {
            // exchange holding item wi: last r with rot[r].w0 <= wi
            int64_t lo = 0, hi = nrot;
            while (hi - lo > 1) {
                int64_t mid = (lo + hi) >> 1;
                if (rot[mid].w0 <= wi) lo = mid; else hi = mid;
            }
            R = rot[lo];
            if (wi < R.w0 || wi >= R.w0 + R.nw) continue;   // a dropped exchange
        }
        const int64_t local = wi - R.w0;
        do_item<EK>(keys, R, local, phase);
        if constexpr (!std::is_same<EV, NoVal>::value) do_item<EV>(vals, R, local, phase);
    }
}

// Single exchange (stand-alone entry point): one descriptor built on the host.
template <typename E>
__global__ __launch_bounds__(kRotThreads) void k_rotate_one(E *__restrict__ p, int64_t lx,
                                                            int64_t ly, int phase, int64_t nitems) {
    Rot R;
    R.pos = 0; R.lx = lx; R.ly = ly; R.w0 = 0; R.nw = nitems;
    for (int64_t wi = blockIdx.x; wi < nitems; wi += gridDim.x) do_item<E>(p, R, wi, phase);
}

template <typename EK, typename EV>
static hipError_t rot_t(void *keys, void *vals, const Plan &pl, const Work &w, int level,
                        int phase, hipStream_t s) {
    int g = 2048;
    hipLaunchKernelGGL((k_rotate<EK, EV>), dim3(g), dim3(kRotThreads), 0, s, (EK *)keys,
                       (EV *)vals, w.rot, w.ctr, pl.cap_rot, level, phase);
    return hipGetLastError();
}

hipError_t launch_rotate(int esize_k, int esize_v, void *keys, void *vals, const Plan &pl,
                         const Work &w, int level, int phase, hipStream_t s) {
    if (esize_k == 4) {
        if (esize_v == 0) return rot_t<uint32_t, NoVal>(keys, vals, pl, w, level, phase, s);
        if (esize_v == 4) return rot_t<uint32_t, uint32_t>(keys, vals, pl, w, level, phase, s);
        if (esize_v == 8) return rot_t<uint32_t, uint64_t>(keys, vals, pl, w, level, phase, s);
    } else if (esize_k == 8) {
        if (esize_v == 0) return rot_t<uint64_t, NoVal>(keys, vals, pl, w, level, phase, s);
        if (esize_v == 4) return rot_t<uint64_t, uint32_t>(keys, vals, pl, w, level, phase, s);
        if (esize_v == 8) return rot_t<uint64_t, uint64_t>(keys, vals, pl, w, level, phase, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rotate_single(void *data, int64_t lx, int64_t ly, int esize, hipStream_t s) {
    if (lx <= 0 || ly <= 0) return hipSuccess;
    int64_t nw;
    if (lx == ly) {
        nw = (lx + kRotChunk - 1) / kRotChunk;
    } else {
        int64_t a = (lx / 2 + kRotChunk - 1) / kRotChunk + (ly / 2 + kRotChunk - 1) / kRotChunk;
        int64_t b = ((lx + ly) / 2 + kRotChunk - 1) / kRotChunk;
        nw = a > b ? a : b;
    }
    int g = (int)(nw < 2048 ? nw : 2048);
    int phases = lx == ly ? 1 : 2;
    for (int ph = 0; ph < phases; ++ph) {
        if (esize == 4)
            hipLaunchKernelGGL(k_rotate_one<uint32_t>, dim3(g), dim3(kRotThreads), 0, s,
                               (uint32_t *)data, lx, ly, ph, nw);
        else if (esize == 8)
            hipLaunchKernelGGL(k_rotate_one<uint64_t>, dim3(g), dim3(kRotThreads), 0, s,
                               (uint64_t *)data, lx, ly, ph, nw);
        else
            return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace imerge
