/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for the in-place
 * merge of Bramas & Bramas, "On the improvement of the in-place merge
 * algorithm parallelization" (arXiv 2005.12648).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or helper with the HIP library under
 * paper_2005_12648_amd/; neither side includes or links the other.
 *
 * What is computed, and where it is defined:
 *   - merge:    the problem statement (Sec. 1, Introduction): two sorted
 *               arrays A and B become one sorted array C holding both.  The
 *               paper does not discuss ties; the reading used everywhere in
 *               this project is the STABLE merge (ties take A first), which is
 *               what the per-pair std::inplace_merge of Alg. 2 and Alg. 3
 *               produces.  Written out as the textbook two-finger merge into a
 *               fresh buffer, then copied back (out-of-place on purpose).
 *   - co-rank:  i(k) = number of A elements among the first k outputs of that
 *               merge.  This is the split the paper calls the "optimal"
 *               pivot search (Sec. 3.1), generalised to any output rank k.
 *               Computed by walking the same two-finger merge, never by a
 *               search.
 *   - rotate:   the partition exchange of Sec. 3.4: X|Y becomes Y|X.  Given
 *               as the plain definition (copy) plus the two schedules the
 *               paper describes, each with counters, so that the counts the
 *               paper proves (Sec. 3.4 correctness proof, Sec. 3.5
 *               complexities) can be checked:
 *                 * linear shifting (LS, Sec. 3.4): swap the smaller block
 *                   with the far end of the larger one and repeat on what is
 *                   left;
 *                 * circular shifting (CS, Sec. 3.4): follow the cycles
 *                   i -> i+L_B (A side) / i -> i-L_A (B side) starting at
 *                   0, 1, ..., until every element has been placed once.
 *
 *   - FindMedian (Sec. 3.3, Alg. 1): the paper's double binary search for
 *               a pivot pair that splits A and B into A0 A1, B0 B1 with
 *               A0 <= B1, B0 <= A1 and |A0|+|B0| close to |A1|+|B1|, written
 *               from the moves Sec. 3.3 describes.  Where Alg. 1 is garbled
 *               (its loop test reads p_A, p_B before they are first set, and
 *               after a stop on equal values it recomputes middles, which can
 *               give an invalid split when keys repeat) the reading used here
 *               is: the indexes start at the middles of A and B (the text of
 *               Sec. 3.3 says so), and a stop on equal values returns that
 *               pair of indexes.
 *   - merge_par: the same stable merge computed by all host cores (OpenMP):
 *               the output is cut at equal ranks, each thread bisects for the
 *               co-rank of its own cut, merges its piece into the fresh
 *               buffer, then the buffer is copied back.  Only for timing
 *               beside the GPU; its result equals merge().
 *
 * Error behaviour: every function trusts its caller (the Python wrapper
 * validates shapes); on allocation failure the merge functions return -1.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Stable two-finger merge (problem statement, Sec. 1).  Ties take A.        */
/* ------------------------------------------------------------------------ */
#define DEFINE_MERGE(NAME, KT)                                                 \
    int NAME(KT *data, int64_t la, int64_t lb)                                 \
    {                                                                          \
        int64_t n = la + lb;                                                   \
        if (n == 0) return 0;                                                  \
        KT *out = (KT *)malloc((size_t)n * sizeof(KT));                        \
        if (!out) return -1;                                                   \
        const KT *a = data, *b = data + la;                                    \
        int64_t i = 0, j = 0, k = 0;                                           \
        while (i < la && j < lb) {                                             \
            if (a[i] <= b[j]) out[k++] = a[i++]; /* tie: A first */            \
            else              out[k++] = b[j++];                               \
        }                                                                      \
        while (i < la) out[k++] = a[i++];                                      \
        while (j < lb) out[k++] = b[j++];                                      \
        memcpy(data, out, (size_t)n * sizeof(KT));                             \
        free(out);                                                             \
        return 0;                                                              \
    }

DEFINE_MERGE(orc_merge_i32, int32_t)
DEFINE_MERGE(orc_merge_u32, uint32_t)
DEFINE_MERGE(orc_merge_i64, int64_t)
DEFINE_MERGE(orc_merge_u64, uint64_t)

/* Key+payload variant: keys decide, the payload (vsz bytes per element)
 * follows its key.  Ties take A, so payloads of equal keys keep their input
 * order. */
#define DEFINE_MERGE_KV(NAME, KT)                                              \
    int NAME(KT *keys, uint8_t *vals, int64_t vsz, int64_t la, int64_t lb)     \
    {                                                                          \
        int64_t n = la + lb;                                                   \
        if (n == 0) return 0;                                                  \
        KT *ko = (KT *)malloc((size_t)n * sizeof(KT));                         \
        uint8_t *vo = (uint8_t *)malloc((size_t)(n * vsz));                    \
        if (!ko || !vo) { free(ko); free(vo); return -1; }                     \
        const KT *a = keys, *b = keys + la;                                    \
        const uint8_t *va = vals, *vb = vals + la * vsz;                       \
        int64_t i = 0, j = 0, k = 0;                                           \
        while (i < la || j < lb) {                                             \
            int take_a = (j >= lb) || (i < la && a[i] <= b[j]);                \
            if (take_a) {                                                      \
                ko[k] = a[i];                                                  \
                memcpy(vo + k * vsz, va + i * vsz, (size_t)vsz);               \
                i++;                                                           \
            } else {                                                           \
                ko[k] = b[j];                                                  \
                memcpy(vo + k * vsz, vb + j * vsz, (size_t)vsz);               \
                j++;                                                           \
            }                                                                  \
            k++;                                                               \
        }                                                                      \
        memcpy(keys, ko, (size_t)n * sizeof(KT));                              \
        memcpy(vals, vo, (size_t)(n * vsz));                                   \
        free(ko); free(vo);                                                    \
        return 0;                                                              \
    }

DEFINE_MERGE_KV(orc_merge_kv_i32, int32_t)
DEFINE_MERGE_KV(orc_merge_kv_u32, uint32_t)
DEFINE_MERGE_KV(orc_merge_kv_i64, int64_t)
DEFINE_MERGE_KV(orc_merge_kv_u64, uint64_t)

/* ------------------------------------------------------------------------ */
/* Co-rank by definition: walk the stable merge and count how many of the    */
/* first k outputs came from A.  ks[] must be ascending, each in [0, la+lb]. */
/* ------------------------------------------------------------------------ */
#define DEFINE_CORANK(NAME, KT)                                                \
    void NAME(const KT *a, int64_t la, const KT *b, int64_t lb,                \
              const int64_t *ks, int64_t nk, int64_t *out)                     \
    {                                                                          \
        int64_t i = 0, j = 0, q = 0;                                           \
        for (q = 0; q < nk; q++) {                                             \
            int64_t k = ks[q];                                                 \
            while (i + j < k) {                                                \
                if (j >= lb || (i < la && a[i] <= b[j])) i++;                  \
                else j++;                                                      \
            }                                                                  \
            out[q] = i;                                                        \
        }                                                                      \
    }

DEFINE_CORANK(orc_corank_i32, int32_t)
DEFINE_CORANK(orc_corank_u32, uint32_t)
DEFINE_CORANK(orc_corank_i64, int64_t)
DEFINE_CORANK(orc_corank_u64, uint64_t)

/* ------------------------------------------------------------------------ */
/* Partition exchange X|Y -> Y|X (Sec. 3.4).                                 */
/* ------------------------------------------------------------------------ */

/* The definition: copy Y then X into a fresh buffer, copy back. */
int orc_rotate_def(int64_t *data, int64_t lx, int64_t ly)
{
    int64_t n = lx + ly;
    if (n == 0) return 0;
    int64_t *tmp = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!tmp) return -1;
    memcpy(tmp, data + lx, (size_t)ly * sizeof(int64_t));
    memcpy(tmp + ly, data, (size_t)lx * sizeof(int64_t));
    memcpy(data, tmp, (size_t)n * sizeof(int64_t));
    free(tmp);
    return 0;
}

/* Linear shifting (Sec. 3.4): move the smaller partition to its final place
 * by swapping it element-wise with what occupies that place, then repeat on
 * the two parts of the larger partition that remain.  Returns the number of
 * element swaps performed. */
int64_t orc_rotate_ls(int64_t *data, int64_t lx, int64_t ly)
{
    int64_t swaps = 0;
    int64_t *base = data;
    while (lx > 0 && ly > 0) {
        if (lx <= ly) {
            /* X is smaller: its final place is the last lx slots. */
            int64_t *dst = base + lx + ly - lx;
            for (int64_t t = 0; t < lx; t++) {
                int64_t v = base[t]; base[t] = dst[t]; dst[t] = v; swaps++;
            }
            /* Now [Y_tail | Y_head | X]; X is done.  What remains is the
             * exchange of Y_tail (lx, now at the front) and Y_head (ly-lx). */
            ly = ly - lx;
            /* remaining problem is base[0..lx) | base[lx..lx+ly), same base */
        } else {
            /* Y is smaller: its final place is the first ly slots. */
            int64_t *src = base + lx;
            for (int64_t t = 0; t < ly; t++) {
                int64_t v = base[t]; base[t] = src[t]; src[t] = v; swaps++;
            }
            /* X = [X_head (ly) | X_rest (lx-ly)].  Now the block reads
             * [Y | X_rest | X_head]; Y is done.  What remains is the
             * exchange of X_rest (lx-ly) and X_head (ly), right after Y. */
            base = base + ly;
            lx = lx - ly;
        }
    }
    return swaps;
}

/* Circular shifting (Sec. 3.4, after Dudzinski & Dydek): element at index i
 * of A|B (sizes la, lb) must go to i+lb if i < la, else to i-la.  Start a
 * cycle at 0, 1, 2, ... until every element has been placed; each element is
 * written exactly once.  Reports the number of cycles and of element moves. */
int orc_rotate_cs(int64_t *data, int64_t la, int64_t lb,
                  int64_t *cycles_out, int64_t *moves_out)
{
    int64_t n = la + lb, placed = 0, cycles = 0, moves = 0;
    if (la == 0 || lb == 0) { *cycles_out = 0; *moves_out = 0; return 0; }
    for (int64_t start = 0; placed < n; start++) {
        int64_t carry = data[start];
        int64_t pos = start;
        do {
            int64_t dst = (pos < la) ? pos + lb : pos - la;
            int64_t next = data[dst];
            data[dst] = carry;
            moves++; placed++;
            carry = next;
            pos = dst;
        } while (pos != start);
        cycles++;
    }
    *cycles_out = cycles;
    *moves_out = moves;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* FindMedian (Sec. 3.3, Alg. 1).  The pivot pair (p_A, p_B) cuts A into    */
/* A0 = A[0,p_A), A1 = A[p_A,L_A) and B into B0, B1 so that A0 <= B1 and     */
/* B0 <= A1 (Sec. 3.3), while |A0|+|B0| stays close to |A1|+|B1|.  It is a   */
/* double binary search: p_A and p_B each search a window [lo, hi) of their  */
/* run and sit at its middle.  After each look at A[p_A] and B[p_B] one      */
/* window shrinks, toward balance (Sec. 3.3):                                */
/*   - when the parts below the pivots are the smaller ones                  */
/*     (|A0|+|B0| < |A1|+|B1|), the index whose value is the smaller moves   */
/*     up (its window starts after it);                                      */
/*   - otherwise the index whose value is the larger moves down (its window  */
/*     ends at it).                                                          */
/* Equal values count as "A's value is the larger".  The search ends when a  */
/* window is empty (each index then takes its window's middle), or, reading */
/* stated at the top, on a look at two equal values: that pair is a valid    */
/* pivot by itself (A0 <= v <= B1 and B0 <= v <= A1 for the common value v). */
/* The runs placed entirely in order, or entirely reversed, are recognised  */
/* first (the two tests that open Alg. 1).                                   */
/* ------------------------------------------------------------------------ */
#define DEFINE_FIND_MEDIAN(NAME, KT)                                           \
void NAME(const KT *A, int64_t la, const KT *B, int64_t lb,                     \
          int64_t *pa_out, int64_t *pb_out)                                     \
{                                                                               \
    if (la == 0 || lb == 0 || A[la - 1] <= B[0]) {   /* A already below B */    \
        *pa_out = la; *pb_out = 0; return;                                      \
    }                                                                           \
    if (!(A[0] <= B[lb - 1])) {                      /* A entirely above B */   \
        *pa_out = 0; *pb_out = lb; return;                                      \
    }                                                                           \
    int64_t a_lo = 0, a_hi = la, b_lo = 0, b_hi = lb;                           \
    int64_t p_A = la / 2, p_B = lb / 2;               /* the two middles */     \
    if (A[p_A] == B[p_B]) { *pa_out = p_A; *pb_out = p_B; return; }             \
    for (;;) {                                                                  \
        int below_smaller = p_A + p_B < (la - p_A) + (lb - p_B);                \
        int a_value_smaller = A[p_A] < B[p_B];                                  \
        if (below_smaller) {                                                    \
            if (a_value_smaller) a_lo = p_A + 1; else b_lo = p_B + 1;           \
        } else {                                                                \
            if (a_value_smaller) b_hi = p_B; else a_hi = p_A;                   \
        }                                                                       \
        if (a_lo >= a_hi || b_lo >= b_hi) break;     /* a window is empty */    \
        if (A[p_A] == B[p_B]) {                      /* equal look: a pivot */  \
            *pa_out = p_A; *pb_out = p_B; return;                               \
        }                                                                       \
        p_A = a_lo + (a_hi - a_lo) / 2;                                         \
        p_B = b_lo + (b_hi - b_lo) / 2;                                         \
    }                                                                           \
    *pa_out = a_lo + (a_hi - a_lo) / 2;                                         \
    *pb_out = b_lo + (b_hi - b_lo) / 2;                                         \
}

DEFINE_FIND_MEDIAN(orc_find_median_i32, int32_t)
DEFINE_FIND_MEDIAN(orc_find_median_u32, uint32_t)
DEFINE_FIND_MEDIAN(orc_find_median_i64, int64_t)
DEFINE_FIND_MEDIAN(orc_find_median_u64, uint64_t)

/* ------------------------------------------------------------------------ */
/* All-cores stable merge (timing only).  Output rank k_t = t*N/P starts     */
/* thread t's piece; the thread finds the co-rank of k_t itself by bisection */
/* on the predicate A[m] <= B[k-1-m] (true, then false, over the admissible  */
/* m: the first false m is the number of A elements among the first k_t     */
/* outputs when ties take A), merges its piece into a fresh buffer, and the  */
/* buffer is copied back in parallel.  Returns the threads used, -1 on       */
/* allocation failure.                                                       */
/* ------------------------------------------------------------------------ */
#define DEFINE_MERGE_PAR(NAME, KT)                                             \
static int64_t NAME##_cut(const KT *A, int64_t la, const KT *B, int64_t lb,    \
                          int64_t k)                                            \
{                                                                               \
    int64_t lo = k > lb ? k - lb : 0, hi = k < la ? k : la;                     \
    while (lo < hi) {                                                           \
        int64_t m = lo + (hi - lo) / 2;                                         \
        if (A[m] <= B[k - 1 - m]) lo = m + 1; else hi = m;                      \
    }                                                                           \
    return lo;                                                                  \
}                                                                               \
int NAME(KT *data, int64_t la, int64_t lb)                                      \
{                                                                               \
    int64_t n = la + lb;                                                        \
    int P = 1;                                                                  \
    _Pragma("omp parallel") { _Pragma("omp single") P = OMP_THREADS(); }       \
    if (n == 0) return P;                                                       \
    KT *out = (KT *)malloc((size_t)n * sizeof(KT));                             \
    if (!out) return -1;                                                        \
    const KT *A = data, *B = data + la;                                         \
    _Pragma("omp parallel for schedule(static)")                                \
    for (int t = 0; t < P; t++) {                                               \
        int64_t k0 = (int64_t)((double)n * t / P);                              \
        int64_t k1 = (t + 1 == P) ? n : (int64_t)((double)n * (t + 1) / P);     \
        int64_t x = NAME##_cut(A, la, B, lb, k0);                               \
        int64_t y = k0 - x, o = k0;                                             \
        while (o < k1) {                                                        \
            if (y >= lb || (x < la && A[x] <= B[y])) out[o++] = A[x++];         \
            else out[o++] = B[y++];                                             \
        }                                                                       \
    }                                                                           \
    _Pragma("omp parallel for schedule(static)")                                \
    for (int64_t q = 0; q < n; q++) data[q] = out[q];                           \
    free(out);                                                                  \
    return P;                                                                   \
}

#ifdef _OPENMP
#define OMP_THREADS() omp_get_num_threads()
#else
#define OMP_THREADS() 1
#endif
DEFINE_MERGE_PAR(orc_merge_par_i32, int32_t)
DEFINE_MERGE_PAR(orc_merge_par_u32, uint32_t)
DEFINE_MERGE_PAR(orc_merge_par_i64, int64_t)
DEFINE_MERGE_PAR(orc_merge_par_u64, uint64_t)
