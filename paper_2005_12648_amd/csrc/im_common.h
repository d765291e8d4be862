// im_common.h -- internal declarations shared by the HIP translation units of
// the in-place merge library.  Not installed; the public ABI is
// include/inplace_merge.h.
//
// Pipeline (all on one stream, no host synchronisation):
//   k_init      roots of the division tree, one per instance; counters reset.
//   per level:  k_split   - per node: the early exits of Alg. 1 / Alg. 2-3,
//                           then a split diagonal and its co-rank (Sec. 3.1),
//                           children for the next level, one partition
//                           exchange descriptor (Alg. 3 "shift"), or a leaf.
//               k_rotate  - all exchanges of the level in one segmented
//                           launch (phase A: block swap or the first two
//                           reversals; phase B: the last reversal).
//   (leaves get their tiles as they are emitted: one atomic on a packed
//   leaf/tile counter gives each leaf its index and its first tile)
//   k_tilerank  co-rank of every tile diagonal inside its leaf.
//   k_tiledeps  per tile: the range of tiles of its leaf that read its window.
//   k_leafmerge persistent kernel: each workgroup merges tiles in LDS (Alg.
//               2/3 per-pair merge, several workgroups per pair); a tile
//               publishes "inputs read" once staged, and stores its output
//               only after the tiles that read its window have published.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace imerge {

constexpr int kMaxLevels = 48;          // hard cap on enqueued division levels
constexpr int kMlpHidden = 32;
constexpr int kMlpParams = 3 * kMlpHidden + 1;
constexpr int64_t kRotChunk = 4096;     // element pairs per exchange work item

// A pair still to be divided: region [base, base+la+lb) of the buffer holds
// the sorted A-part followed by the sorted B-part.  k0/i0 locate the node in
// its instance's merge (global diagonal and co-rank of the node start).
struct Node {
    int64_t base, la, lb, k0, i0;
    int32_t inst, pad;
};

// Partition exchange X|Y -> Y|X of [pos, pos+lx+ly).  lx == ly: one block
// swap (a single linear-shifting step).  Otherwise three reversals.
constexpr int kMaxCyc = 4;       // pieces of one cycle of a fused two-level exchange

// An exchange of a level.  c == 0: the partition exchange X|Y -> Y|X of
// [pos, pos+lx+ly).  c >= 2: a cycle of a fused two-level exchange: c
// pieces of len elements at start[0..c), the piece at start[k] moves to
// start[k+1 mod c].
struct Rot {
    int64_t pos, lx, ly;
    int64_t w0;       // first work item of this exchange in its level
    int64_t nw;       // work items
    int64_t stash0;   // circular shifting: first stash slot (-1: none needed)
    int64_t len;
    int64_t start[kMaxCyc];
    int32_t c;
    int32_t pad;
};

// A pair that is merged without further division.  Its tiles are processed
// in increasing order (dir 0: every A element moves right by at most
// leaf_span elements) or in decreasing order (dir 1: every B element moves
// left by at most leaf_span elements).
struct Leaf {
    int64_t base, la, lb, k0, i0;
    int32_t inst, ntiles;
    int32_t dir, pad;
};

// Device counters.  Zeroed by k_init at the start of every call.
struct Counters {
    unsigned long long level_nodes[kMaxLevels + 1];  // nodes at each level
    unsigned long long level_rot[kMaxLevels];        // (count << 40) | work items
    unsigned long long level_rev[kMaxLevels];        // exchanges needing phase B
    unsigned long long level_stash[kMaxLevels];      // circular shifting: stash slots used
    unsigned long long leaves;
    unsigned long long tiles;
    unsigned long long rotated;       // elements moved by exchanges
    unsigned long long rotated_rev;   // of which in three-reversal exchanges
    unsigned long long leaf_elems;    // elements of all leaves (merged in LDS)
    unsigned long long probes;        // key-pair probes of split searches
    unsigned long long searches;      // split searches
    unsigned long long levels_used;   // max level index that had nodes, +1
    unsigned long long split_fallbacks;  // FindMedian splits replaced by co-rank splits
    unsigned long long fused;            // nodes whose two levels ran as one exchange
    unsigned long long leaf_next;        // leaf merge: slots handed out beyond the static ones
    unsigned long long leaf_tiles;       // (leaves << Plan::leaf_shift) | tiles, as emitted
    unsigned long long rot_next[kMaxLevels][2];  // exchanges: items handed out per level and phase
    unsigned int error;               // nonzero: a device-side check failed
    unsigned int pad;
};

constexpr int kRotCountShift = 40;
constexpr unsigned long long kRotWorkMask = (1ull << kRotCountShift) - 1;

// Error bits of Counters::error.
constexpr unsigned kErrOversizeLeaf = 1u;   // a node still too large at the last level
constexpr unsigned kErrBarrierSpin = 2u;    // a leaf-merge wait for readers' flags gave up
constexpr unsigned kErrCapacity = 4u;       // a descriptor array overflowed
constexpr unsigned kErrNotSorted = 8u;      // checked mode: a run is unsorted
constexpr unsigned kErrOffsets = 16u;       // checked mode: offsets not monotone

// The learned split model as the kernels see it (device memory).  The
// prediction error is kept per bucket of the normalised diagonal x = k/N
// (kErrBuckets equal buckets): err_b[b] is the half-width, in A elements, of
// the bracket a search starts from when x falls in bucket b.
constexpr int kErrBuckets = 128;
constexpr float kErrUnknown = 1e30f;    // no bracket: searches stay plain
struct MlpDev {
    float p[kMlpParams];      // w1[H], b1[H], w2[H], b2
    float err_scale;          // mean |prediction error| in A elements (>= 1)
    float err_b[kErrBuckets];
    float pad[2];
};

// Parameters common to one pipeline run.
struct Plan {
    int64_t n_inst;
    int64_t total;          // bound of the elements in all instances
    int64_t leaf_cap;       // a pair of at most this many elements is a leaf
    int64_t leaf_span;      // ... and so is a pair whose smaller part has at most this many
    int64_t tile;           // elements per workgroup tile in the leaf merge
    int32_t max_levels;     // division levels enqueued
    int32_t grid_leaf;      // persistent grid of the leaf merge
    int64_t cap_nodes, cap_rot, cap_leaves, cap_tiles;
    uint32_t epoch;         // value a tile writes to its "inputs read" flag
    int32_t cfg;            // leaf-merge configuration (tile size per workgroup)
    int32_t split_method;   // kSplitCorank or kSplitFindMedian
    int32_t rot_method;     // kRotSwapRev or kRotCS
    int64_t cap_stash;      // circular shifting: stash slots per level
    int32_t fuse;           // fuse two division levels into one exchange where possible
    // Leaf tiles are the cells [m*tile, (m+1)*tile) of the instance's output
    // cut at leaf boundaries, and the co-ranks of the cell boundaries are
    // found on the input layout, beside the first division level (single
    // instance, exact co-rank splits, plain or learned searches): no tile
    // search after the division.
    // 0: tiles of `tile` outputs from each leaf's start, searched after it.
    int32_t cells;
    int32_t leaf_shift;     // bits of the tile count in the packed leaf/tile counter
                            // (0: the caps do not fit in 64 bits; the plan is refused)
    // Rows (elements of several words ordered by their leading key): the
    // row length in key units (0: packed keys), and the number of 4-byte
    // exchange units per element (1: exchanges move whole elements).
    int64_t row_stride;
    int64_t rot_scale;
    // Merge-sort pass: width of the sorted runs it pairs (0: not a sort
    // pass).  The pass's offsets are then written into the workspace.
    int64_t sort_width;
};

// Split of a division node: the exact co-rank (symmetric or middle diagonal),
// or FindMedian (Sec. 3.3, Alg. 1) guarded by a validity and balance check.
constexpr int kSplitCorank = 0;
constexpr int kSplitFindMedian = 1;
// Partition exchange of the merge: a block swap (one linear-shifting step)
// when the parts are equal, else three reversals; or circular shifting
// (cycles of Sec. 3.4).
constexpr int kRotSwapRev = 0;
constexpr int kRotCS = 1;
constexpr int kCsSeg = 256;      // cycle steps per lane in circular shifting
constexpr int kCsLanes = 256;    // lanes per circular-shifting work item

constexpr int kLeafCfgs = 4;   // leaf-merge tile configurations (im_leaf.hip)

// Geometry of one leaf tile, in the order the leaf pipeline takes its slots
// (written by the planning kernel, read in one round by the pipeline):
// output window [out0, out0+n), A-slice (na elements from a0) and B-slice
// (n - na elements from b0), all as element indices of the whole buffer; the
// leaf's first tile and tile count, the tile's leaf-local index, and the
// leaf-local tiles that read its window (A-slices [alo, ahi], B-slices
// [blo, bhi]; an empty range is [0, -1]).
struct TileGeo {
    int64_t out0, a0, b0, tbase;
    int n, na;
    int32_t ntiles, local;
    int32_t alo, ahi, blo, bhi;
};

// Workspace carve-up (device pointers).
struct Work {
    Counters *ctr;
    Node *nodes[3];          // node lists of levels l, l+1, l+2 (ring)
    Rot *rot;
    Leaf *leaves;
    int64_t *tile_start;     // per leaf: first tile index (exclusive scan)
    int64_t *tile_rank;      // per tile: co-rank at the tile's first diagonal
    int32_t *tile_leaf;      // per tile: its leaf
    int64_t *cell_rank;      // Plan::cells: co-rank at each cell boundary m*tile (m = 0..cells)
    TileGeo *tile_geo;       // per slot: the tile's geometry and readers
    unsigned int *tile_flag; // per tile: == epoch once its inputs are in LDS
    int64_t *offsets1;       // [3] offsets of a single-instance call
    void *cs_stash_k;        // circular shifting: first value of each cycle segment
    void *cs_stash_v;        // ... and its payload
    int64_t *sort_off;       // merge-sort pass: the pass's instance offsets (else null)
    unsigned int *host_err;  // device view of a host-memory word that receives the
                             // error bits as they are raised (may be null)
};

// Raise a device-side error bit: in the call's counters (read under IM_CHECK
// and by the statistics call) and in the host-memory word that the library
// reads without a synchronisation.  The host word takes a plain store at
// system scope (no read-modify-write over the host link): concurrent raisers
// may overwrite each other's bit, but the word stays nonzero.
__device__ __forceinline__ void raise_error(const Work &w, unsigned bit) {
    atomicOr(&w.ctr->error, bit);
    if (w.host_err)
        __hip_atomic_store(w.host_err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Key-type dispatch codes (match im_dtype of the public header).
enum KeyCode { kI32 = 0, kU32 = 1, kI64 = 2, kU64 = 3 };

// ---- launchers (defined in the .hip files) --------------------------------
hipError_t launch_init(const Plan &pl, const Work &w, const int64_t *d_offsets,
                       int64_t la, int64_t lb, hipStream_t s);
hipError_t launch_split(int key, void *data, const int64_t *d_offsets, const Plan &pl,
                        const Work &w, int level, const MlpDev *mlp, hipStream_t s);
hipError_t launch_rotate(int esize_k, int esize_v, void *keys, void *vals, const Plan &pl,
                         const Work &w, int level, int phase, hipStream_t s);
hipError_t launch_tilerank(int key, void *data, const int64_t *d_offsets, const Plan &pl,
                           const Work &w, const MlpDev *mlp, hipStream_t s);
hipError_t launch_leafmerge(int key, int esize_v, void *keys, void *vals, const Plan &pl,
                            const Work &w, hipStream_t s);
hipError_t launch_tiledeps(const Plan &pl, const Work &w, hipStream_t s);
hipError_t launch_fill32(unsigned *p, int64_t n, unsigned v, hipStream_t s);
// Tile geometry of the leaf merge for a (key size, payload size, config):
// threads per workgroup, items per thread, pipeline depth (tiles read ahead
// of the oldest unstored one: a leaf may have depth * grid tiles), LDS bytes.
void leaf_geometry(int esize_k, int esize_v, int cfg, int *threads, int *ipt, int *depth,
                   size_t *lds_bytes);
int leaf_grid(int esize_k, int esize_v, int cfg);   // persistent grid (resident workgroups)
// One-launch merge of a single small pair (configuration 0 tiles; the grid is
// one workgroup per tile, at most a quarter of the resident workgroups).
hipError_t launch_smallmerge(int key, int esize_v, void *keys, void *vals, int64_t la, int64_t lb,
                             const Plan &pl, const Work &w, hipStream_t s);
const void *leaf_kernel_ptr(int key, int esize_v, int cfg);

hipError_t launch_corank(int key, const void *data, int64_t la, int64_t lb, const int64_t *d_k,
                         int64_t nk, int64_t *d_out, const MlpDev *mlp, int32_t *d_probes,
                         hipStream_t s);
hipError_t launch_rotate_single(void *data, int64_t lx, int64_t ly, int esize, hipStream_t s);
// Circular-shifting exchange of one X|Y (stand-alone); stash: one element per
// lane of cs_lanes(lx, ly), device memory.
int64_t cs_lanes(int64_t lx, int64_t ly);
hipError_t launch_rotate_cs_single(void *data, int64_t lx, int64_t ly, int esize, void *stash,
                                   hipStream_t s);
// Linear shifting step by step (stand-alone): the stash holds
// ls_stash_elems(lx, ly) elements; d_swaps (may be null) accumulates the
// element swaps performed.
int64_t ls_stash_elems(int64_t lx, int64_t ly);
hipError_t launch_rotate_ls_single(void *data, int64_t lx, int64_t ly, int esize, void *stash,
                                   unsigned long long *d_swaps, hipStream_t s);
// Recursive division into 2^depth pairs without moving data (im_split.hip).
hipError_t launch_divide(int key, const void *data, int64_t la, int64_t lb, int method,
                         int level, const int64_t *nodes_in, int64_t *nodes_out, hipStream_t s);
// Out-of-place merge of in[0,la) and in[la,la+lb) into out (im_leaf.hip):
// d_rank[t] = co-rank of tile diagonal t*tile, t = 0..ntiles-1.
int merge_oop_tile(int esize);
hipError_t launch_tile_diagonals(int64_t n, int64_t tile, int64_t *d_k, hipStream_t s);
hipError_t launch_merge_oop(int key, const void *in, void *out, int64_t la, int64_t lb,
                            const int64_t *d_rank, hipStream_t s);
// Checked mode: flags runs that are not ascending (keys `stride` key units
// apart: 1 for packed keys, the row length for rows).
hipError_t launch_check_sorted(int key, const void *data, const int64_t *d_offsets,
                               int64_t n_inst, Counters *ctr, int64_t stride, hipStream_t s);
// Wide rows (im_leaf.hip).  A row kind 0 .. rows_kinds()-1 fixes the chunk
// bytes rows move in, the chunks a thread holds and the tiles a workgroup
// holds; for each: rows per tile for a row size (0: a row does not fit),
// the resident grid of the rows leaf merge, and its cooperative launch.
int rows_kinds();
int rows_chunk_bytes(int kind);
int rows_tile(int64_t row_bytes, int kind);
int rows_depth(int kind);      // tiles a rows workgroup holds (its read-ahead)
int rows_grid(int key, int kind);
hipError_t launch_leafrows(int key, int kind, void *data, int64_t row_bytes, const Plan &pl,
                           const Work &w, hipStream_t s);

// Merge sort helpers.
int sort_tile_elems(int esize);
hipError_t launch_tilesort(int key, void *data, int64_t n, hipStream_t s);
hipError_t launch_pass_offsets(int64_t n, int64_t width, int64_t *d_off, int64_t n_inst,
                               hipStream_t s);

// MLP kernels.
hipError_t launch_mlp_grad(const float *d_params, const float *d_x, const float *d_t, int64_t m,
                           float *d_partial, int nblocks, hipStream_t s);
hipError_t launch_mlp_reduce(const float *d_partial, int nblocks, float *d_grad, float *d_loss,
                             hipStream_t s);
hipError_t launch_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v,
                           float lr, int step, hipStream_t s);
hipError_t launch_mlp_forward(const float *d_params, const float *d_x, int64_t m, float *d_y,
                              hipStream_t s);
hipError_t launch_mlp_samples(int key, const void *data, int64_t la, int64_t lb, int64_t m,
                              int64_t *d_k, float *d_x, hipStream_t s);
hipError_t launch_mlp_targets(const int64_t *d_i, int64_t m, int64_t la, float *d_t,
                              hipStream_t s);
hipError_t launch_mlp_errscale(const float *d_params, const int64_t *d_k, const int64_t *d_i,
                               int64_t m, int64_t la, int64_t lb, MlpDev *d_model,
                               hipStream_t s);
int mlp_grad_blocks(int64_t m);

}  // namespace imerge
