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
 * Error behaviour: every function trusts its caller (the Python wrapper
 * validates shapes); on allocation failure the merge functions return -1.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

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
