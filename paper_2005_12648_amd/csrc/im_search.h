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

// FindMedian (Sec. 3.3, Alg. 1): a double binary search for a pivot pair
// (p_A, p_B) with A[0,p_A) <= B[p_B,..) and B[0,p_B) <= A[p_A,..) that keeps
// |A0|+|B0| close to |A1|+|B1|, in O(log L_A + log L_B) probes.  The probes
// start at the middles of A and B; when the loop stops because the probed
// values are equal, that probe pair is the result (the printed listing tests
// p_A, p_B before setting them and recomputes midpoints after such a stop).
// One lane, sequential dependent probes.  `probes` counts value pairs read.
template <typename KP>
__device__ __forceinline__ void find_median(KP A, int64_t la, KP B, int64_t lb, int64_t &pa,
                                            int64_t &pb, uint32_t &probes) {
    if (la == 0 || lb == 0 || A[la - 1] <= B[0]) { pa = la; pb = 0; return; }
    if (!(A[0] <= B[lb - 1])) { pa = 0; pb = lb; return; }
    int64_t left_a = 0, limit_a = la, left_b = 0, limit_b = lb;
    pa = la / 2;
    pb = lb / 2;
    auto va = A[pa], vb = B[pb];
    ++probes;
    while (left_a < limit_a && left_b < limit_b && va != vb) {
        pa = (limit_a - left_a) / 2 + left_a;
        pb = (limit_b - left_b) / 2 + left_b;
        va = A[pa];
        vb = B[pb];
        ++probes;
        const int64_t lo = pa + pb, hi = (la - pa) + (lb - pb);
        if (va < vb) {
            if (lo < hi) left_a = pa + 1;
            else limit_b = pb;
        } else {
            if (lo < hi) left_b = pb + 1;
            else limit_a = pa;
        }
        // the loop test reads the values at the current probe pair
    }
    if (left_a < limit_a && left_b < limit_b) return;   // stopped on an equal probe
    pa = (limit_a - left_a) / 2 + left_a;
    pb = (limit_b - left_b) / 2 + left_b;
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

// Learned co-rank.  kg: global diagonal of the instance (size n_inst, A size
// la_inst); i0: global co-rank of the start of the searched sub-problem
// (A/B here are that sub-problem's parts), k: local diagonal.
template <typename KP>
__device__ __forceinline__ int64_t corank_learned(KP A, int64_t la, KP B, int64_t lb, int64_t k,
                                                  const MlpDev *__restrict__ M, int64_t kg,
                                                  int64_t n_inst, int64_t la_inst, int64_t i0,
                                                  uint32_t &probes) {
    int64_t lo = k > lb ? k - lb : 0;
    int64_t hi = k < la ? k : la;
    if (hi - lo <= 1) return corank_binary(A, la, B, lb, k, lo, hi, probes);
    float x = n_inst > 0 ? (float)((double)kg / (double)n_inst) : 0.0f;
    float y = mlp_eval(M, x);
    double gd = (double)y * (double)la_inst - (double)i0;
    int64_t g;
    if (!(gd == gd)) g = lo;                     // NaN prediction: start at lo
    else if (gd <= (double)lo) g = lo;
    else if (gd >= (double)hi) g = hi;
    else g = (int64_t)llrint(gd);
    int64_t step = (int64_t)M->err_scale;
    if (step < 1) step = 1;
    int64_t blo, bhi;
    if (g < hi && (++probes, A[g] <= B[k - 1 - g])) {
        // answer > g: gallop to the right
        blo = g + 1;
        for (;;) {
            int64_t m = g + step;
            if (m >= hi) { bhi = hi; break; }
            ++probes;
            if (!(A[m] <= B[k - 1 - m])) { bhi = m; break; }
            blo = m + 1;
            step <<= 1;
        }
    } else {
        // answer <= g: gallop to the left
        bhi = g;
        for (;;) {
            int64_t m = g - step;
            if (m < lo) { blo = lo; break; }
            ++probes;
            if (A[m] <= B[k - 1 - m]) { blo = m + 1; break; }
            bhi = m;
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

// Learned group co-rank: the first round probes W points spaced by the
// model's typical error around its prediction, then the plain rounds go on
// inside the bracket that round leaves (always exact).
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
    const bool wide = hi - lo > W;
    bool p = false;
    int64_t m = lo;
    if (wide) {
        const float x = n_inst > 0 ? (float)((double)kg / (double)n_inst) : 0.0f;
        const double gd = (double)mlp_eval(M, x) * (double)la_inst - (double)i0;
        int64_t g;
        if (!(gd == gd) || gd <= (double)lo) g = lo;
        else if (gd >= (double)hi) g = hi;
        else g = (int64_t)llrint(gd);
        int64_t step = (int64_t)M->err_scale;
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
    if (wide) {
        ++rounds;
        const int64_t nlo = c > 0 ? m_prev + 1 : lo;
        const int64_t nhi = c < W ? m_next : hi;
        lo = nlo;
        hi = nhi > nlo ? nhi : nlo;
    }
    return group_search<W>(lo, hi, [&](int64_t q) { return A[q] <= B[k - 1 - q]; }, rounds);
}

}  // namespace imerge
