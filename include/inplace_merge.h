/*
 * inplace_merge.h -- C ABI of the MI355X (gfx950) parallel in-place merge.
 *
 * Method: Bramas & Bramas, "On the improvement of the in-place merge algorithm
 * parallelization" (arXiv 2005.12648).  Two sorted runs A|B that sit next to
 * each other in one buffer (Sec. 1, problem statement) are split into
 * independent pairs A_0 B_0 A_1 B_1 ... (Sec. 3, the division of A B into
 * pairs), the pairs are made contiguous by in-place partition exchanges
 * (Sec. 3.4, linear shifting), level by level as in the recursive strategy of
 * Alg. 3 (sRecPar), and each pair is merged independently (Alg. 2/3, the
 * per-pair merge).
 *
 * Conventions that hold for every entry point:
 *  - Pointers named d_* or documented as "device" are device pointers on the
 *    current HIP device.  The caller owns them; the library never frees or
 *    retains them after the call returns.
 *  - Work is enqueued on `stream` and is asynchronous: a return value of 0
 *    means "validated and enqueued", not "finished".  Kernel faults surface at
 *    the caller's next synchronisation; device-side error bits through
 *    inplace_merge_device_status() (see there).  A NULL stream means the
 *    default stream.
 *  - The result is the STABLE merge: equal keys keep A before B and keep their
 *    order inside a run (the paper does not discuss ties; this is the reading
 *    of the per-pair std::inplace_merge, which is stable).
 *  - Inputs must be two ascending runs.  This is not checked unless the
 *    environment variable IM_CHECK=1 is set (then the call synchronises the
 *    stream and returns IM_ERR_NOT_SORTED on unsorted input).  Unsorted input
 *    without checking yields an unspecified permutation of the input but never
 *    an access outside [data, data + L_A + L_B).
 *  - Return value: IM_OK (0) or a negative IM_ERR_* code.  Nothing throws
 *    across this boundary.  inplace_merge_last_error() returns a thread-local
 *    description of the last failure on the calling thread.
 *  - The merge entry points refuse a stream that is capturing a graph
 *    (IM_ERR_INVALID_ARG): a captured call would replay this call's flag
 *    epoch and workspace.  batched_inplace_merge_graph records a merge.
 *  - Concurrent calls on different streams of the same device share the
 *    library's workspace only through a per-device lock: they are safe but
 *    serialised at enqueue time; the enqueued work itself may overlap only if
 *    the caller supplies a private workspace per stream (see
 *    inplace_merge_set_workspace).
 */
#ifndef INPLACE_MERGE_H
#define INPLACE_MERGE_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Key / payload element types. Keys are compared as the named integer type. */
typedef enum {
    IM_INT32 = 0,
    IM_UINT32 = 1,
    IM_INT64 = 2,
    IM_UINT64 = 3
} im_dtype;

/* Status codes. */
enum {
    IM_OK = 0,
    IM_ERR_INVALID_ARG = -1,       /* NULL pointer, negative length, ...      */
    IM_ERR_UNSUPPORTED_DTYPE = -2, /* dtype outside im_dtype                  */
    IM_ERR_HIP = -3,               /* a HIP runtime call failed               */
    IM_ERR_WORKSPACE = -4,         /* workspace too small / allocation failed */
    IM_ERR_NOT_SORTED = -5,        /* IM_CHECK=1 and an input run is unsorted */
    IM_ERR_UNIMPLEMENTED = -6,
    IM_ERR_DEVICE = -7             /* a kernel raised a device-side error bit */
};

/* Statistics of the most recent merge enqueued by the calling thread.
 * Fields filled from device counters are only valid after the stream has
 * been synchronised and inplace_merge_fetch_stats() has been called. */
typedef struct {
    int64_t leaf_capacity;   /* largest pair merged without further division */
    int64_t tile;            /* elements per workgroup in the pair merge      */
    int32_t max_levels;      /* division levels enqueued                      */
    int32_t levels_used;     /* division levels that had work (device)        */
    int64_t leaves;          /* pairs merged (device)                         */
    int64_t tiles;           /* workgroup tiles in the pair merge (device)    */
    int64_t rotations;       /* partition exchanges performed (device)        */
    int64_t rotated_elems;   /* elements moved by partition exchanges (dev.)  */
    int64_t reversed_elems;  /* of which by three-reversal exchanges (dev.)   */
    int64_t leaf_elems;      /* elements merged by the leaf merge (device)    */
    int64_t search_probes;   /* key-pair probes in all split searches (dev.)  */
    int64_t searches;        /* split searches performed (device)             */
    int32_t leaf_config;     /* leaf-merge configuration used (0..3)           */
    int32_t leaf_grid;       /* resident workgroups of the leaf merge          */
    int64_t split_fallbacks; /* FindMedian splits replaced by co-rank (device) */
    int64_t fused_nodes;     /* nodes whose two division levels ran as one    */
                             /* exchange (cycles of contiguous pieces) (dev.) */
} im_stats;

/* ---------------------------------------------------------------------- */
/* Plain in-place merge (Sec. 1 problem; Sec. 3 division; Alg. 3 levels;  */
/* Sec. 3.4 linear shifting; per-pair merge of Alg. 2/3).                 */
/* ---------------------------------------------------------------------- */

/* Merge data[0, L_A) and data[L_A, L_A+L_B) in place (device buffer of
 * L_A+L_B elements of type `dtype`).  Early exits (Alg. 1 first lines and
 * the entry test of Alg. 2/3): nothing happens when L_A == 0, L_B == 0 or
 * A[last] <= B[0]; when A[0] > B[last] a single exchange B|A is done. */
int inplace_merge(void *data, int64_t L_A, int64_t L_B, int dtype, hipStream_t stream);

/* inplace_merge() for callers that cannot allocate device memory (code
 * recorded into a graph by the caller's own means, tight serving loops,
 * hosts that forbid allocation during operation).  It calls no hipMalloc,
 * hipFree, pinned-host or event allocation: its workspace is a static
 * device array of 4 MiB that the library holds on every device it runs on
 * until the process ends.  The result equals inplace_merge()'s.  A merge
 * whose workspace (descriptors, counters, per-tile co-ranks, flags and
 * geometry: about 80 bytes per 16,896 int32 or 8,704 int64 elements, plus a
 * few KiB) does not fit in the array is refused with IM_ERR_WORKSPACE before
 * any work is enqueued (int32 inputs of up to about 8*10^8 elements, int64
 * of about 4*10^8, fit).  Every call on a device shares that
 * device's array and leaves its last contents there: two such calls whose
 * work overlaps in time on one device (different streams, or different host
 * threads without ordering) race and give wrong results; calls on one
 * stream are ordered.  It does not share the workspace of the other entry
 * points, so it may overlap with them.  Device error bits reach the caller
 * only under IM_CHECK=1 or through inplace_merge_fetch_stats (the host
 * error word is pinned memory, allocated by the other entry points). */
int inplace_merge_noalloc(void *data, int64_t L_A, int64_t L_B, int dtype, hipStream_t stream);

/* Key + payload variant (structure of arrays): keys[] and vals[] have
 * L_A+L_B elements each; only keys are compared, every move carries the
 * payload.  val_dtype: any im_dtype (only its size, 4 or 8 bytes, matters). */
int inplace_merge_kv(void *keys, void *vals, int64_t L_A, int64_t L_B,
                     int key_dtype, int val_dtype, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Wide elements (Sec. 4 test cases: elements of 4 to 65540 bytes whose    */
/* first 4 bytes are the compared key; Sec. 5 on minimum data movement     */
/* for large elements).                                                    */
/* ---------------------------------------------------------------------- */

/* Merge rows in place: data holds L_A+L_B rows of row_bytes bytes each
 * (array of structures); rows [0, L_A) and [L_A, L_A+L_B) are each ascending
 * by the key stored in the first bytes of a row, of type key_dtype (4 or 8
 * bytes).  Stable: equal keys keep A's rows first, and every row moves as a
 * whole.  The division and the exchanges are those of inplace_merge (the
 * exchanges move 4-byte words); the leaves gather rows into registers in
 * merged order.  Requirements (else IM_ERR_INVALID_ARG): row_bytes a
 * multiple of 4 and of the key size; data aligned to the key size; at most
 * 81920 bytes per row, which admits the paper's largest element (a 4-byte
 * key and 16384 ints, 65540 bytes).  Rows move in 16-, 8- or 4-byte chunks
 * (the widest that divides the row and the address; rows above 64 KiB move
 * in 4-byte chunks).
 * IM_CHECK=1 checks the runs' keys.  The element counts of im_stats count
 * rows. */
int inplace_merge_rows(void *data, int64_t L_A, int64_t L_B, int64_t row_bytes,
                       int key_dtype, hipStream_t stream);

/* Workspace bytes a rows merge of `rows` rows needs (see
 * inplace_merge_workspace_bytes). */
size_t inplace_merge_rows_workspace_bytes(int64_t rows, int64_t row_bytes, int key_dtype);

/* ---------------------------------------------------------------------- */
/* Batched segmented merge: n independent instances in one buffer.         */
/* ---------------------------------------------------------------------- */

/* d_offsets: device int64[2n+1], non-decreasing.  Instance q has
 *   A = data[d_offsets[2q],   d_offsets[2q+1])
 *   B = data[d_offsets[2q+1], d_offsets[2q+2]).
 * The library reads d_offsets[2n] back to size its workspace: one 8-byte
 * copy on `stream` and a synchronisation of it (the _sized form below is
 * fully asynchronous).  Offsets are validated on the device only when
 * IM_CHECK=1.  IM_ERR_INVALID_ARG if n >= 2^31 or the stream is capturing. */
int batched_inplace_merge(void *data, const int64_t *d_offsets, int64_t n, int dtype,
                          hipStream_t stream);
int batched_inplace_merge_kv(void *keys, void *vals, const int64_t *d_offsets, int64_t n,
                             int key_dtype, int val_dtype, hipStream_t stream);

/* The same merges without a synchronisation: the caller states the sizes.
 * total_elems: an upper bound of d_offsets[2n] (sizes the workspace).
 * max_instance: an upper bound of the largest instance (A+B) or 0 if unknown
 * (then total_elems is used); it sets how many division levels are enqueued.
 * IM_ERR_INVALID_ARG if n >= 2^31, or if the leaf and tile capacities that n
 * and total_elems imply do not fit together in one 64-bit device counter
 * (only for n within a fraction of a percent of 2^31). */
int batched_inplace_merge_sized(void *data, const int64_t *d_offsets, int64_t n,
                                int64_t total_elems, int64_t max_instance, int dtype,
                                hipStream_t stream);
int batched_inplace_merge_kv_sized(void *keys, void *vals, const int64_t *d_offsets, int64_t n,
                                   int64_t total_elems, int64_t max_instance, int key_dtype,
                                   int val_dtype, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Captured batched merge: the whole launch sequence of one batched merge  */
/* (division levels of Alg. 3, exchanges of Sec. 3.4, per-pair merges)    */
/* recorded once in a HIP graph and replayed with one call.               */
/* ---------------------------------------------------------------------- */
typedef struct im_graph im_graph;

/* Record a batched merge of the given buffers into a new graph object.
 * data, d_offsets: device pointers baked into the graph; the caller keeps
 * ownership and must keep them alive until im_graph_destroy.  Between
 * replays the caller may change the data and the offsets' contents, as long
 * as n stays the same, d_offsets[2n] <= total_elems and every instance stays
 * within max_instance (0: total_elems).  The graph owns a private workspace
 * (allocated here), so replays do not touch the library's shared one; two
 * replays of the same graph that overlap in time race.  Capture runs on a
 * private stream; `stream` only orders the workspace set-up.  The leaf merge
 * node is marked cooperative when the runtime accepts the attribute (queried
 * by im_graph_cooperative).  IM_CHECK and stage profiling do not apply. */
int batched_inplace_merge_graph(im_graph **out, void *data, const int64_t *d_offsets,
                                int64_t n, int64_t total_elems, int64_t max_instance,
                                int dtype, hipStream_t stream);
/* Enqueue one replay on `stream`. */
int im_graph_launch(im_graph *g, hipStream_t stream);
/* 1 if the leaf merge node carries the cooperative attribute, else 0. */
int im_graph_cooperative(const im_graph *g);
/* Free the graph and its workspace (synchronises the device first). */
int im_graph_destroy(im_graph *g);

/* ---------------------------------------------------------------------- */
/* Leaf-merge configuration and its autotuner (not part of the paper).     */
/* ---------------------------------------------------------------------- */
/* Configurations of the per-pair merge: workgroup threads x items per
 * thread, and pipeline depth (tiles a workgroup reads ahead of the oldest
 * one it has not stored; a pair may span depth x resident-workgroups tiles,
 * so depth 3 needs fewer division levels and depth 2 keeps one register set):
 *   0 = 512 threads, large tiles (about 70 KB of LDS), depth 3;
 *   1 = 512 threads, large tiles, depth 2;
 *   2 = 256 threads, same items per thread, depth 2;
 *   3 = 256 threads, half the items per thread, depth 3. */
#define IM_LEAF_CONFIGS 4

/* Force a configuration for the calling process (0..IM_LEAF_CONFIGS-1), or
 * -1 to return to automatic choice (tuned table, else configuration 0). */
int inplace_merge_set_config(int cfg);

/* Time every configuration on a private copy of the given batched input
 * (data and d_offsets are only read) and remember the fastest one for this
 * workload class: (device, key size, payload size, floor(log2(mean instance
 * size))).  Later merges of that class use it unless a configuration is
 * forced.  val_dtype: -1 for keys only.  reps >= 1 timed runs per
 * configuration (plus one warm-up); ms_out (host, may be NULL) receives the
 * median milliseconds per configuration; *chosen (may be NULL) the winner.
 * Allocates and frees a scratch copy of the data; synchronises `stream`. */
int inplace_merge_autotune(const void *data, const int64_t *d_offsets, int64_t n,
                           int64_t total_elems, int64_t max_instance, int key_dtype,
                           int val_dtype, int reps, double *ms_out, int *chosen,
                           hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Method variants and comparators (the paper's alternatives).             */
/* ---------------------------------------------------------------------- */
#define IM_SPLIT_CORANK 0      /* exact co-rank split (Sec. 3.1, "optimal")      */
#define IM_SPLIT_FINDMEDIAN 1  /* FindMedian double binary search (Alg. 1)     */
#define IM_ROTATE_SWAP_REV 0   /* one block swap (a linear-shifting step) when   */
                               /* the parts are equal, else three reversals       */
#define IM_ROTATE_CS 1         /* circular shifting: cycles (Sec. 3.4)          */

/* inplace_merge() with the split and exchange methods chosen (keys only).
 * IM_SPLIT_FINDMEDIAN splits every division node with FindMedian (Sec. 3.3,
 * Alg. 1; probes start at the middles and a stop on an equal probe returns
 * that pair); a node whose FindMedian split is invalid or leaves a child
 * larger than 9/16 of the node is split by co-rank instead (counted in
 * im_stats.split_fallbacks), which keeps the level count bounded.
 * FindMedian splits satisfy A0 <= B1 and B0 <= A1, so the result equals the
 * stable merge for keys (payloads could not tell equal keys apart: no kv
 * form).  IM_ROTATE_CS does every exchange by circular shifting (Sec. 3.4):
 * gcd(|X|+|Y|, |Y|) cycles, each element moved once, strided access; it
 * needs a stash of 2*(L_A+L_B)/256 elements in the workspace. */
int inplace_merge_variant(void *data, int64_t L_A, int64_t L_B, int dtype, int split_method,
                          int rot_method, hipStream_t stream);

/* Division without data movement (the pivot searches of Sec. 3 applied
 * recursively, as in Alg. 3): split data[0,L_A) | data[L_A,L_A+L_B) into
 * 2^depth pairs (depth 0..24) with method IM_SPLIT_CORANK (exact co-rank at
 * the middle rank of each node) or IM_SPLIT_FINDMEDIAN (Alg. 1).  d_sizes
 * (device int64[2 * 2^depth]) receives (|A_p|, |B_p|) for every pair in
 * order.  Uses stream-ordered temporary memory. */
int im_divide(const void *data, int64_t L_A, int64_t L_B, int dtype, int method, int depth,
              int64_t *d_sizes, hipStream_t stream);

/* Partition exchange X|Y -> Y|X by circular shifting (Sec. 3.4): the
 * comparator of im_rotate.  elem_bytes 4 or 8; stream-ordered stash. */
int im_rotate_cs(void *data, int64_t lx, int64_t ly, int elem_bytes, hipStream_t stream);

/* Partition exchange X|Y -> Y|X by linear shifting, step by step (Sec. 3.4):
 * the smaller block is swapped with the block at the far end of the larger
 * one, which puts it in its final place, and the same is done on what
 * remains, until one part is empty.  Performs exactly the paper's element
 * swaps, L - gcd(lx, ly) of them for L = lx + ly (Sec. 3.5 counts up to
 * 2L).  The steps that keep the same smaller block (one quotient of
 * Euclid's algorithm on the two lengths) run as one launch, one lane per
 * column of the block and segment of its chain of swaps; such a column's
 * value between two swaps stays in a register, so the fixed block is
 * written once per run.  d_swaps (device int64, may be NULL) receives the
 * element swaps the kernels performed.  elem_bytes 4 or 8; uses a
 * stream-ordered stash of about 2L/256 elements when a run's chains are
 * longer than 256 swaps. */
int im_rotate_ls(void *data, int64_t lx, int64_t ly, int elem_bytes, int64_t *d_swaps,
                 hipStream_t stream);

/* The classic out-of-place merge (the paper's external-buffer comparator):
 * out = stable merge of in[0,L_A) and in[L_A,L_A+L_B); in and out must not
 * overlap.  inplace_merge_buffered() allocates the buffer, merges into it,
 * copies back and frees it (allocation, copy and free included, as in the
 * paper's comparison). */
int merge_out_of_place(const void *in, void *out, int64_t L_A, int64_t L_B, int dtype,
                       hipStream_t stream);
int inplace_merge_buffered(void *data, int64_t L_A, int64_t L_B, int dtype, hipStream_t stream);

/* In-place merge sort of data[0, n): each tile is sorted in LDS, then
 * bottom-up passes of the batched merge double the sorted run length; the
 * unpaired last run of a pass is carried over unchanged. */
int inplace_merge_sort(void *data, int64_t n, int dtype, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Workspace, errors, statistics.                                          */
/* ---------------------------------------------------------------------- */

/* Bytes of device workspace that any single merge of N elements of this
 * dtype needs (keys, key+payload, every leaf configuration, and the passes
 * of an in-place merge sort of N).  The library allocates its workspace
 * lazily per device if none is set.  The workspace holds split descriptors
 * and counters only: its size grows with the number of workgroup tiles,
 * never with the data itself (about 1.3 MB for 2^28 int32 elements).
 * Returns 0 for invalid arguments. */
size_t inplace_merge_workspace_bytes(int64_t N, int dtype);

/* The same for a batched merge of `total_elems` elements in `n_inst`
 * instances (the descriptor arrays grow with the instance count). */
size_t inplace_merge_workspace_bytes_batched(int64_t total_elems, int64_t n_inst, int dtype);

/* Use caller-owned device memory as the workspace of the current device
 * (NULL/0 returns to library-owned workspace).  The caller keeps ownership
 * and must keep it alive while enqueued work uses it. */
int inplace_merge_set_workspace(void *d_ws, size_t bytes);

const char *inplace_merge_last_error(void);

/* Copy the statistics of the last enqueued merge of this thread into *out.
 * Synchronises `stream` to read the device counters.  Returns IM_ERR_DEVICE
 * if that merge raised a device-side error bit. */
int inplace_merge_fetch_stats(im_stats *out, hipStream_t stream);

/* The same, synchronising the stream the last merge of this thread was
 * enqueued on. */
typedef im_stats merge_stats;
int inplace_merge_last_stats(merge_stats *out);

/* How a device-side failure reaches the caller.  An enqueued merge returns
 * IM_OK once validated and enqueued; the kernels that run later can still
 * fail in three ways, each of which leaves the data a permutation of the
 * input but not merged: a node still larger than a leaf at the last division
 * level (error bit 1), a bounded wait for another workgroup's flag that gave
 * up (bit 2), a descriptor array that overflowed (bit 4).  The kernel that
 * raises a bit also stores it into a word of pinned host memory owned by
 * the library (one per device).  inplace_merge_device_status() reads and
 * clears that word WITHOUT synchronising anything: it returns IM_ERR_DEVICE
 * (message: the bit) if any merge enqueued on the current device has raised
 * a bit that completed since the last query, else IM_OK.  Call it after the
 * caller's own synchronisation to learn about every merge before it.  The
 * same bits are returned by inplace_merge_fetch_stats / _last_stats for the
 * last merge, and by the merge itself under IM_CHECK=1. */
int inplace_merge_device_status(void);

/* Stage timing for the calling thread.  While enabled, every merge records
 * HIP events on its stream around its launch groups; _read synchronises
 * `stream`, adds the elapsed milliseconds per stage into ms[0..nstages)
 * (0: split searches, 1: partition exchanges, 2: leaf planning (no launch
 * of its own: leaves are laid out as they are emitted, so it reads 0),
 * 3: tile co-ranks, 4: leaf merge), the number of kernel launches into launches[]
 * (may be NULL), and forgets the recorded events. */
int inplace_merge_profile(int enable);
int inplace_merge_profile_read(double *ms, int64_t *launches, int nstages, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Stage entry points (used by the unit parity tests and the benchmark).   */
/* ---------------------------------------------------------------------- */

/* Co-rank (Sec. 3.1, the exact "optimal" split for any output rank): for
 * each diagonal d_k[p] in [0, L_A+L_B], d_out[p] = number of A elements among
 * the first d_k[p] outputs of the stable merge of data[0,L_A) and
 * data[L_A,L_A+L_B) (a diagonal outside that range gives -1).  One wavefront
 * lane per diagonal, binary search.  d_probes (may be NULL) receives the key
 * pairs compared per diagonal.  All device pointers. */
int im_corank(const void *data, int64_t L_A, int64_t L_B, int dtype,
              const int64_t *d_k, int64_t nk, int64_t *d_out, int32_t *d_probes,
              hipStream_t stream);

/* Partition exchange (Sec. 3.4): data[0, lx+ly) = X|Y becomes Y|X.  Equal
 * sizes use one block swap (one linear-shifting step); otherwise the
 * exchange is done by three reversals on the device. elem_bytes: 4 or 8. */
int im_rotate(void *data, int64_t lx, int64_t ly, int elem_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Learned split: a 1->H->1 ReLU network (H = 32, fp32) predicts co-ranks;  */
/* a search corrects every prediction to the exact co-rank, so results are */
/* identical to inplace_merge().  The search starts from a bracket around  */
/* the prediction (half-width from the model's error table), checks both   */
/* ends, gallops outward (doubling steps) from an end that fails, and      */
/* bisects inside; where the bracket is not clearly narrower than the      */
/* plain search range it is a plain search.  Not part of the paper.        */
/* ---------------------------------------------------------------------- */
typedef struct merge_model merge_model;

#define IM_MLP_HIDDEN 32
#define IM_MLP_PARAMS (3 * IM_MLP_HIDDEN + 1)   /* w1[H], b1[H], w2[H], b2 */

typedef struct {
    int64_t samples;    /* diagonals sampled for training labels (>= 2)  */
    int32_t steps;      /* optimiser steps                               */
    float lr;           /* Adam learning rate                            */
    uint64_t seed;      /* initialisation seed                           */
} merge_train_cfg;

/* Create a model from host parameters (IM_MLP_PARAMS floats) or, if
 * params == NULL, from a deterministic seeded initialisation. */
int merge_model_create(merge_model **m, const float *params, uint64_t seed);

/* Train on the GPU: labels are produced by the plain co-rank search at
 * `samples` evenly spaced diagonals k_p = floor((p + 1/2) N / samples) of
 * the given runs (x = k_p/N, target i(k_p)/L_A, both rounded to fp32), then
 * `steps` Adam steps run with the library's forward/backward/update kernels,
 * the learning rate decaying from cfg->lr to zero on a cosine
 * (lr_s = lr (1 + cos(pi s / steps)) / 2 at step s).  Last, the model's
 * error table is measured on the same diagonals: per bucket of x (128
 * buckets), the half-width of the bracket its searches start from.  If *m is
 * NULL a model is first created from cfg->seed (and freed again, *m reset
 * to NULL, if training fails); otherwise the model *m is trained further
 * (its Adam moments restart at zero).  Synchronises `stream` at the end
 * (the model lives on the device). */
int merge_model_train(merge_model **m, const void *data, int64_t L_A, int64_t L_B,
                      int dtype, const merge_train_cfg *cfg, hipStream_t stream);

/* One forward+backward pass of the mean squared error on device samples
 * d_x[M], d_t[M] (fp32) with the model's current parameters; writes the
 * gradient (IM_MLP_PARAMS floats) to d_grad and the loss to d_loss. */
int merge_model_grad(const merge_model *m, const float *d_x, const float *d_t, int64_t M,
                     float *d_grad, float *d_loss, hipStream_t stream);

/* Forward pass only: d_y[p] = network(d_x[p]). */
int merge_model_forward(const merge_model *m, const float *d_x, int64_t M, float *d_y,
                        hipStream_t stream);

/* Host copy of the parameters / replace them.  Replacing them forgets the
 * model's error table: its searches are plain binary searches until it is
 * trained again (results are exact either way). */
int merge_model_get_params(const merge_model *m, float *params_out);
int merge_model_set_params(merge_model *m, const float *params);

/* One Adam step (Kingma & Ba; beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrected, `step` counting from 1) of the model's device parameters with
 * the device gradient d_grad[IM_MLP_PARAMS]; the moments d_m, d_v
 * (device, IM_MLP_PARAMS floats each, zero before step 1) are updated in
 * place.  The same kernel runs every step of merge_model_train. */
int merge_model_adam_step(merge_model *m, const float *d_grad, float *d_m, float *d_v, float lr,
                          int step, hipStream_t stream);

/* Learned-split co-rank of diagonals d_k[0..nk): same result as im_corank;
 * d_probes (optional, may be NULL) receives the probes spent per diagonal. */
int im_corank_learned(const void *data, int64_t L_A, int64_t L_B, int dtype,
                      const merge_model *m, const int64_t *d_k, int64_t nk,
                      int64_t *d_out, int32_t *d_probes, hipStream_t stream);

/* In-place merge whose split searches use the model; bit-identical result. */
int inplace_merge_learned(void *data, int64_t L_A, int64_t L_B, int dtype,
                          const merge_model *m, hipStream_t stream);

int merge_model_save(const merge_model *m, const char *path);
int merge_model_load(merge_model **m, const char *path);
int merge_model_free(merge_model *m);

#ifdef __cplusplus
}
#endif
#endif /* INPLACE_MERGE_H */
