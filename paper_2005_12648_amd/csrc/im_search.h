// im_search.h -- device-side split searches.
//
// Co-rank (the exact split of Sec. 3.1 -- the "optimal" pivot search --
// generalised to an arbitrary output rank k): the number i of A elements
// among the first k outputs of the stable merge of A and B.  With
// P(m) := A[m] <= B[k-1-m], P is true then false on
// [max(0, k-L_B), min(k, L_A)), and i is the first m where it is false (or
// the upper bound).  Ties therefore take A first.
//
// The learned variant starts from a network prediction and brackets the
// answer by an exponential search before the same binary search; it returns
// exactly the same i.
#pragma once
#include "im_common.h"

namespace imerge {

// The searches read keys through `KP`: a plain pointer (packed keys), or
// RowKeys (rows of several words ordered by their leading key).
template <typename K>
struct RowKeys {
    const K *p;
    int64_t s;            // row length in key units
    __device__ __forceinline__ K operator[](int64_t m) const { return p[m * s]; }
    __device__ __forceinline__ RowKeys operator+(int64_t m) const { return RowKeys{p + m * s, s}; }
};

template <typename KP>
__device__ __forceinline__ int64_t corank_binary(KP A, int64_t la, KP B, int64_t lb,
                                                 int64_t k, int64_t lo, int64_t hi,
                                                 uint32_t &probes) {
    // Invariant: every m < lo has P(m) true, every m >= hi has P(m) false.
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        ++probes;
        if (A[mid] <= B[k - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <typename KP>
__device__ __forceinline__ int64_t corank_plain(KP A, int64_t la, KP B, int64_t lb, int64_t k,
                                                uint32_t &probes) {
    int64_t lo = k > lb ? k - lb : 0;
    int64_t hi = k < la ? k : la;
    return corank_binary(A, la, B, lb, k, lo, hi, probes);
}

// FindMedian (Sec. 3.3, Alg. 1): a pivot pair (pa, pb) with
// A[0,pa) <= B[pb,..) and B[0,pb) <= A[pa,..) that keeps the lower halves'
// size close to the upper halves', in O(log la + log lb) dependent looks.
// Each index bisects a window of its run and sits at the window's middle.
// A look at the two values decides which window shrinks: while the lower
// halves hold fewer elements than the upper ones the index on the smaller
// value moves up, otherwise the index on the larger value moves down (equal
// values rank A's as the larger).  The search ends on an empty window (both
// indexes then take their window's middle) or on a look at two equal values,
// which is a valid pivot by itself (the printed listing recomputes middles
// there, which breaks the pivot property when keys repeat).  One lane;
// `probes` counts the looks (value pairs read).
template <typename KP>
__device__ __forceinline__ void find_median(KP A, int64_t la, KP B, int64_t lb, int64_t &pa,
                                            int64_t &pb, uint32_t &probes) {
    if (la == 0 || lb == 0 || A[la - 1] <= B[0]) { pa = la; pb = 0; return; }   // in order
    if (!(A[0] <= B[lb - 1])) { pa = 0; pb = lb; return; }                    // reversed
    int64_t alo = 0, ahi = la, blo = 0, bhi = lb;
    for (bool first = true;; first = false) {
        pa = alo + ((ahi - alo) >> 1);
        pb = blo + ((bhi - blo) >> 1);
        const auto va = A[pa];
        const auto vb = B[pb];
        ++probes;
        const bool same = va == vb;
        if (first && same) return;
        const bool up = 2 * (pa + pb) < la + lb;     // lower halves the smaller
        const bool move_a = up == (va < vb);
        if (move_a) {
            if (up) alo = pa + 1;
            else ahi = pa;
        } else {
            if (up) blo = pb + 1;
            else bhi = pb;
        }
        if (alo >= ahi || blo >= bhi) break;
        if (same) return;
    }
    pa = alo + ((ahi - alo) >> 1);
    pb = blo + ((bhi - blo) >> 1);
}

// fp32 forward pass of the 1 -> H -> 1 ReLU network.
__device__ __forceinline__ float mlp_eval(const MlpDev *__restrict__ M, float x) {
    float y = M->p[3 * kMlpHidden];
#pragma unroll
    for (int h = 0; h < kMlpHidden; ++h) {
        float z = fmaf(M->p[h], x, M->p[kMlpHidden + h]);
        y = fmaf(M->p[2 * kMlpHidden + h], fmaxf(z, 0.0f), y);
    }
    return y;
}

// Half-width of the search bracket around a prediction at x = k/N.
__device__ __forceinline__ float mlp_halfwidth(const MlpDev *__restrict__ M, float x) {
    int b = (int)(x * (float)kErrBuckets);
    b = b < 0 ? 0 : (b >= kErrBuckets ? kErrBuckets - 1 : b);
    return M->err_b[b];
}

// Predicted local co-rank g of the searched sub-problem and its bracket
// half-width e (both in A elements of the sub-problem; g not clamped).
// False when the prediction is unusable (NaN) or its bracket would not be
// narrower than `frac` of the range [lo, hi]: the search then stays plain.
__device__ __forceinline__ bool mlp_bracket(const MlpDev *__restrict__ M, int64_t kg,
                                            int64_t n_inst, int64_t la_inst, int64_t i0,
                                            int64_t lo, int64_t hi, int frac, double &g,
                                            double &e) {
    const float x = n_inst > 0 ? (float)((double)kg / (double)n_inst) : 0.0f;
    g = (double)mlp_eval(M, x) * (double)la_inst - (double)i0;
    e = (double)mlp_halfwidth(M, x);
    if (!(g == g) || !(e >= 0.0)) return false;
    return (2.0 * e + 1.0) * (double)frac < (double)(hi - lo);
}

// Learned co-rank.  kg: global diagonal of the instance (size n_inst, A size
// la_inst); i0: global co-rank of the start of the searched sub-problem
// (A/B here are that sub-problem's parts), k: local diagonal.  The bracket
// [L, R] around the prediction holds the answer when P(L-1) holds and P(R)
// does not; both ends are probed together, then a binary search runs inside.
// A bracket end that fails gallops outward from it (doubling steps).  When
// the bracket is not 4x narrower than the range, plain binary search.
template <typename KP>
__device__ __forceinline__ int64_t corank_learned(KP A, int64_t la, KP B, int64_t lb, int64_t k,
                                                  const MlpDev *__restrict__ M, int64_t kg,
                                                  int64_t n_inst, int64_t la_inst, int64_t i0,
                                                  uint32_t &probes) {
    int64_t lo = k > lb ? k - lb : 0;
    int64_t hi = k < la ? k : la;
    double gd, e;
    if (hi - lo <= 1 || !mlp_bracket(M, kg, n_inst, la_inst, i0, lo, hi, 4, gd, e))
        return corank_binary(A, la, B, lb, k, lo, hi, probes);
    const double fl = floor(gd - e), fr = ceil(gd + e);
    const int64_t L = fl <= (double)lo ? lo : (fl >= (double)hi ? hi : (int64_t)fl);
    const int64_t R = fr <= (double)lo ? lo : (fr >= (double)hi ? hi : (int64_t)fr);
    // both ends in one round of loads
    const bool needL = L > lo, needR = R < hi;
    bool pl = true, pr = false;
    if (needL) {
        ++probes;
        pl = A[L - 1] <= B[k - L];
    }
    if (needR) {
        ++probes;
        pr = A[R] <= B[k - 1 - R];
    }
    int64_t blo = L, bhi = R;
    int64_t step = (int64_t)e + 1;
    if (!pl) {
        // the answer is below L: gallop down from L - 1
        bhi = L - 1;
        blo = lo;
        for (;;) {
            const int64_t m = bhi - step;
            if (m < lo) break;
            ++probes;
            if (A[m] <= B[k - 1 - m]) { blo = m + 1; break; }
            bhi = m;
            step <<= 1;
        }
    } else if (pr) {
        // the answer is above R: gallop up from R + 1
        blo = R + 1;
        bhi = hi;
        for (;;) {
            const int64_t m = blo + step - 1;
            if (m >= hi) break;
            ++probes;
            if (!(A[m] <= B[k - 1 - m])) { bhi = m; break; }
            blo = m + 1;
            step <<= 1;
        }
    }
    return corank_binary(A, la, B, lb, k, blo, bhi, probes);
}

// ---------------------------------------------------------------------------
// Group-cooperative searches.  The W lanes of an aligned group (W a power of
// two dividing 64) call with the same arguments and all get the same answer.
// Each round probes W points that cut [lo, hi) into W+1 nearly equal parts;
// the predicate is true on a prefix of them, so one ballot narrows the range
// (W+1)-fold: about 5 dependent rounds for 2^27 candidates with W = 64, 8
// with W = 8, instead of 27 for a binary search.  Different groups of a wave
// may search different ranges; the loop runs until every group is done
// (lanes of finished groups only take part in the ballots).  `rounds` counts
// the group's dependent probe rounds.
//
// Generic form: P(m) true then false on [lo, hi); returns the first m with
// P(m) false, or hi.
template <int W, typename Pred>
__device__ __forceinline__ int64_t group_search(int64_t lo, int64_t hi, Pred P, uint32_t &rounds) {
    static_assert(W >= 2 && W <= 64 && (W & (W - 1)) == 0, "group width");
    const int lane = threadIdx.x & 63;
    const int gl = lane & (W - 1);
    const int gbase = lane & ~(W - 1);
    const uint64_t gmask = W == 64 ? ~0ull : ((1ull << W) - 1);
    for (;;) {
        const bool wide = hi - lo > W;
        if (!__any(wide)) break;
        const int64_t span = hi - lo;             // < 2^47, so span * 65 fits
        bool p = false;
        if (wide) p = P(lo + span * (gl + 1) / (W + 1));
        const int c = __popcll((__ballot(p) >> gbase) & gmask);
        if (wide) {
            ++rounds;
            const int64_t nlo = c > 0 ? lo + span * c / (W + 1) + 1 : lo;
            const int64_t nhi = c < W ? lo + span * (c + 1) / (W + 1) : hi;
            lo = nlo;
            hi = nhi;
        }
    }
    const int64_t m = lo + gl;
    const bool p = m < hi && P(m);
    if (hi > lo) ++rounds;
    return lo + __popcll((__ballot(p) >> gbase) & gmask);
}

template <int W, typename KP>
__device__ __forceinline__ int64_t corank_group(KP A, int64_t la, KP B, int64_t lb, int64_t k,
                                                uint32_t &rounds) {
    const int64_t lo = k > lb ? k - lb : 0;
    const int64_t hi = k < la ? k : la;
    return group_search<W>(lo, hi, [&](int64_t m) { return A[m] <= B[k - 1 - m]; }, rounds);
}

// Learned group co-rank: the first round probes W points spread evenly over
// the bracket around the prediction (its half-width from the model's error
// table), then the plain rounds go on inside the bracket that round leaves
// (always exact: an answer outside the bracket leaves [lo, first point] or
// [last point, hi]).  A bracket not 8x narrower than the range: plain rounds.
template <int W, typename KP>
__device__ __forceinline__ int64_t corank_group_learned(KP A, int64_t la, KP B, int64_t lb,
                                                        int64_t k, const MlpDev *__restrict__ M,
                                                        int64_t kg, int64_t n_inst,
                                                        int64_t la_inst, int64_t i0,
                                                        uint32_t &rounds) {
    const int lane = threadIdx.x & 63;
    const int gl = lane & (W - 1);
    const int gbase = lane & ~(W - 1);
    const uint64_t gmask = W == 64 ? ~0ull : ((1ull << W) - 1);
    int64_t lo = k > lb ? k - lb : 0;
    int64_t hi = k < la ? k : la;
    double gd = 0.0, e = 0.0;
    // the same on every lane of the group (same arguments)
    const bool use = hi - lo > W && mlp_bracket(M, kg, n_inst, la_inst, i0, lo, hi, 8, gd, e);
    bool p = false;
    int64_t m = lo;
    if (use) {
        const int64_t g = gd <= (double)lo ? lo : (gd >= (double)hi ? hi : (int64_t)llrint(gd));
        int64_t step = (int64_t)ceil((2.0 * e + 1.0) / (double)(W - 1));
        if (step < 1) step = 1;
        // probe g + (gl - W/2) * step, clamped into [lo, hi-1]: non-decreasing in gl
        m = g + (int64_t)(gl - W / 2) * step;
        if (m < lo) m = lo;
        if (m > hi - 1) m = hi - 1;
        p = A[m] <= B[k - 1 - m];
    }
    const int c = __popcll((__ballot(p) >> gbase) & gmask);
    // every lane takes part in the shuffles; sources lie in the same group
    const int64_t m_prev = __shfl(m, gbase + (c > 0 ? c - 1 : 0), 64);
    const int64_t m_next = __shfl(m, gbase + (c < W ? c : W - 1), 64);
    if (use) {
        ++rounds;
        const int64_t nlo = c > 0 ? m_prev + 1 : lo;
        const int64_t nhi = c < W ? m_next : hi;
        lo = nlo;
        hi = nhi > nlo ? nhi : nlo;
    }
    return group_search<W>(lo, hi, [&](int64_t q) { return A[q] <= B[k - 1 - q]; }, rounds);
}

}  // namespace imerge
