// im_split.hip -- division stage: tree roots, per-level split of every node,
// tile co-ranks of the leaves, and the stand-alone co-rank entry point.
//
// Sec. 3 divides A B into pairs A_0 B_0 ... A_{T-1} B_{T-1} whose elements
// are ordered pair to pair.  Alg. 3 (sRecPar) does it recursively: find the
// split of the current pair, exchange the two middle partitions (A_1 | B_0),
// recurse on both halves.  Here every level of that recursion is one launch
// over all nodes of the level (all instances of a batch included), and the
// exchanges of a level are one segmented launch (im_rotate.hip).
//
// Split rule of a node with parts la, lb (S = la + lb):
//   * early exits first, exactly the tests of Alg. 1 (lines that return
//     before the search) and of the entry of Alg. 2/3: an empty part, or
//     A[last] <= B[0], leaves the node as it is; A[0] > B[last] needs a single
//     exchange B|A and no merge;
//   * S <= leaf capacity, or the smaller part within the leaf span: the node
//     is a leaf (merged tile by tile in LDS, im_leaf.hip);
//   * otherwise the split diagonal is k = la when max(la, lb) <= 9/16 S --
//     then the two exchanged partitions have the same length (la - i == j),
//     so the exchange is a single block swap -- else k = S/2 (balanced
//     halves, the balance goal of Sec. 3.1) and the exchange takes three
//     reversals.  Children are at most 9/16 of the parent either way.
#include "im_common.h"
#include "im_search.h"

namespace imerge {

constexpr int kSplitThreads = 256;

__global__ void k_init(Counters *ctr, Node *nodes0, const int64_t *__restrict__ offsets,
                       int64_t n_inst, int64_t la, int64_t lb, int64_t *off1) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    constexpr int64_t kWords = (int64_t)(sizeof(Counters) / sizeof(unsigned long long));
    static_assert(sizeof(Counters) % sizeof(unsigned long long) == 0, "whole words");
    for (int64_t q = gid; q < kWords; q += stride) {
        // level_nodes[0] is the first word: it starts at the number of roots.
        reinterpret_cast<unsigned long long *>(ctr)[q] = q == 0 ? (unsigned long long)n_inst : 0ull;
    }
    if (offsets == nullptr) {
        // single instance: A = [0, la), B = [la, la+lb)
        if (gid == 0) {
            off1[0] = 0;
            off1[1] = la;
            off1[2] = la + lb;
            Node nd;
            nd.base = 0; nd.la = la; nd.lb = lb; nd.k0 = 0; nd.i0 = 0; nd.inst = 0; nd.pad = 0;
            nodes0[0] = nd;
        }
        return;
    }
    for (int64_t q = gid; q < n_inst; q += stride) {
        int64_t o0 = offsets[2 * q], o1 = offsets[2 * q + 1], o2 = offsets[2 * q + 2];
        Node nd;
        nd.base = o0;
        nd.la = o1 - o0;
        nd.lb = o2 - o1;
        if (nd.la < 0 || nd.lb < 0) { nd.la = 0; nd.lb = 0; }   // never index a bad instance
        nd.k0 = 0; nd.i0 = 0; nd.inst = (int32_t)q; nd.pad = 0;
        nodes0[q] = nd;
    }
}

__device__ __forceinline__ int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Circular shifting of X|Y (n = lx+ly): gcd(n, ly) cycles of n/gcd steps,
// each cut into segments of kCsSeg steps, one lane per (cycle, segment).
__device__ __forceinline__ void cs_shape(int64_t lx, int64_t ly, int64_t &g, int64_t &nseg) {
    const int64_t n = lx + ly;
    g = gcd64(n, ly);
    const int64_t L = n / g;
    nseg = (L + kCsSeg - 1) / kCsSeg;
}

__device__ __forceinline__ void emit_rot(const Plan &pl, const Work &w, int level, int64_t pos,
                                         int64_t lx, int64_t ly) {
    // counters count elements; the descriptor is in exchange units
    const int64_t elems = lx + ly;
    const bool three_rev = lx != ly;
    pos *= pl.rot_scale;
    lx *= pl.rot_scale;
    ly *= pl.rot_scale;
    int64_t nw, stash0 = -1;
    if (pl.rot_method == kRotCS) {
        int64_t g, nseg;
        cs_shape(lx, ly, g, nseg);
        nw = (g * nseg + kCsLanes - 1) / kCsLanes;
        if (nseg > 1) {
            // cycles cut into several segments keep the first value of every
            // segment in the level's stash (fewer than 2*(lx+ly)/kCsSeg slots)
            const unsigned long long st =
                atomicAdd(&w.ctr->level_stash[level], (unsigned long long)(g * nseg));
            if ((int64_t)st + g * nseg > pl.cap_stash) {
                raise_error(w, kErrCapacity);
                return;
            }
            stash0 = (int64_t)st;
        }
    } else if (lx == ly) {
        nw = (lx + kRotChunk - 1) / kRotChunk;
    } else {
        int64_t a = (lx / 2 + kRotChunk - 1) / kRotChunk + (ly / 2 + kRotChunk - 1) / kRotChunk;
        int64_t b = ((lx + ly) / 2 + kRotChunk - 1) / kRotChunk;
        nw = a > b ? a : b;
    }
    unsigned long long packed = atomicAdd(&w.ctr->level_rot[level],
                                          (1ull << kRotCountShift) | (unsigned long long)nw);
    unsigned long long slot = packed >> kRotCountShift;
    if ((int64_t)slot >= pl.cap_rot) {
        raise_error(w, kErrCapacity);
        return;
    }
    Rot r;
    r.pos = pos; r.lx = lx; r.ly = ly;
    r.w0 = (int64_t)(packed & kRotWorkMask);
    r.nw = nw;
    r.stash0 = stash0;
    r.len = 0;
    for (int q = 0; q < kMaxCyc; ++q) r.start[q] = 0;
    r.c = 0;
    r.pad = 0;
    w.rot[slot] = r;
    atomicAdd(&w.ctr->rotated, (unsigned long long)elems);
    if (three_rev && pl.rot_method != kRotCS) {
        atomicAdd(&w.ctr->rotated_rev, (unsigned long long)elems);
        atomicAdd(&w.ctr->level_rev[level], 1ull);
    }
}

// A leaf and its tiles: one atomic on the packed leaf/tile counter gives the
// leaf its index and its first tile, so tile_start rises with the leaf index
// (the tile co-rank kernel finds a tile's leaf by bisection) without a scan
// over the leaves after the division.
__device__ __forceinline__ void emit_leaf(const Plan &pl, const Work &w, const Node &nd) {
    const int64_t S = nd.la + nd.lb;
    // tiles of `tile` outputs from the leaf's start, or the instance's cells
    // that the leaf meets (its first and last may be partial)
    const unsigned long long nt =
        pl.cells ? (S > 0 ? (unsigned long long)((nd.k0 + S - 1) / pl.tile - nd.k0 / pl.tile + 1)
                          : 0ull)
                 : (unsigned long long)((S + pl.tile - 1) / pl.tile);
    const int sh = pl.leaf_shift;
    const unsigned long long packed = atomicAdd(&w.ctr->leaf_tiles, (1ull << sh) + nt);
    const unsigned long long slot = packed >> sh;
    const unsigned long long tstart = packed & ((1ull << sh) - 1);
    atomicAdd(&w.ctr->leaves, 1ull);
    // The leaves below cap_leaves come first in the counter's order, and
    // their tiles number at most total / tile + cap_leaves <= cap_tiles <
    // 2^leaf_shift, so the two fields never carry into each other there.
    // Only those leaves are counted in tiles and leaf_elems: the tile kernels
    // never meet a tile of a dropped leaf.
    if ((int64_t)slot >= pl.cap_leaves) {
        raise_error(w, kErrCapacity);
        return;
    }
    if ((int64_t)(tstart + nt) > pl.cap_tiles) raise_error(w, kErrCapacity);
    atomicAdd(&w.ctr->tiles, nt);
    atomicAdd(&w.ctr->leaf_elems, (unsigned long long)S);
    Leaf lf;
    lf.base = nd.base; lf.la = nd.la; lf.lb = nd.lb; lf.k0 = nd.k0; lf.i0 = nd.i0;
    lf.inst = nd.inst;
    lf.ntiles = (int32_t)nt;
    // direction of the tile order: the part that bounds how far elements
    // travel must be the one within leaf_span (see im_leaf.hip)
    lf.dir = (nd.la + nd.lb <= pl.leaf_cap || nd.lb <= pl.leaf_span) ? 0 : 1;
    lf.pad = 0;
    w.leaves[slot] = lf;
    w.tile_start[slot] = (int64_t)tstart;
}

// Split node nd at (i, j): Alg. 3's "shift" exchanges A[i, la) and B[0, j),
// which turns A_0 A_1 B_0 B_1 into A_0 B_0 A_1 B_1, and both pairs go to the
// next level.
__device__ __forceinline__ void emit_split(const Plan &pl, const Work &w, int level, Node *out,
                                           const Node &nd, int64_t i, int64_t j) {
    const int64_t la = nd.la, lb = nd.lb, kk = i + j;
    if (la - i > 0 && j > 0) emit_rot(pl, w, level, nd.base + i, la - i, j);
    unsigned long long slot = atomicAdd(&w.ctr->level_nodes[level + 1], 2ull);
    if ((int64_t)slot + 1 >= pl.cap_nodes) {
        raise_error(w, kErrCapacity);
        return;
    }
    Node l, r;
    l.base = nd.base; l.la = i; l.lb = j; l.k0 = nd.k0; l.i0 = nd.i0; l.inst = nd.inst;
    l.pad = 0;
    r.base = nd.base + kk; r.la = la - i; r.lb = lb - j; r.k0 = nd.k0 + kk;
    r.i0 = nd.i0 + i; r.inst = nd.inst; r.pad = 0;
    out[slot] = l;
    out[slot + 1] = r;
}

// ---------------------------------------------------------------------------
// Fused two-level exchange.  With symmetric splits at a node and at both of
// its children, the two levels of exchanges (Alg. 3's shift at the node,
// then at each child) compose into one permutation of the node that takes
//   A_LL A_LR A_RL A_RR B_LL B_LR B_RL B_RR  to  A_LL B_LL A_LR B_LR A_RL B_RL A_RR B_RR.
// Cut into pieces that move as wholes (the block boundaries closed under the
// permutation and its inverse), it is a handful of cycles of equal-length
// contiguous pieces; moving each cycle once reads and writes every element
// that changes place once, instead of twice for the elements that both
// levels move (about 3/4 of the node moves instead of 2 x 1/2).
// ---------------------------------------------------------------------------
// The decomposition runs on the whole wave: lane q holds cut q (sorted, no
// duplicates; kCutNone above the last), so a membership test is a six-step
// lane binary search and an insert is one lane shift.  Every value below is
// the same on all lanes of the wave except the per-lane cut and candidates.
constexpr int kMaxCuts = 63;            // lane 63 always holds kCutNone
constexpr int64_t kCutNone = INT64_MAX;

// Blocks are given in source order (src[b] + len[b] == src[b + 1]); a block
// of length 0 matches nothing.
struct FusedPerm {
    int64_t src[8], dst[8], len[8];
};

__device__ __forceinline__ int64_t fz_fwd(const FusedPerm &f, int64_t x) {
    int64_t y = x;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        y = (x >= f.src[b] && x < f.src[b] + f.len[b]) ? f.dst[b] + (x - f.src[b]) : y;
    return y;
}
__device__ __forceinline__ int64_t fz_inv(const FusedPerm &f, int64_t y) {
    int64_t x = y;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        x = (y >= f.dst[b] && y < f.dst[b] + f.len[b]) ? f.src[b] + (y - f.dst[b]) : x;
    return x;
}

// Number of cuts below v (the lanes hold a sorted list padded with kCutNone).
__device__ __forceinline__ int wave_lower_bound(int64_t c, int64_t v) {
    int pos = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (__shfl(c, pos + step - 1, 64) < v) pos += step;
    return pos;
}

// Adds the valid candidates of all lanes to the cut list.  False if it would
// exceed kMaxCuts.
__device__ __forceinline__ bool fz_add(int64_t &c, int &nc, int64_t cand, bool valid,
                                       bool &changed) {
    const int lane = threadIdx.x & 63;
    // the search runs on every lane: a shuffle only reads lanes that execute it
    const int64_t at = __shfl(c, wave_lower_bound(c, cand), 64);
    bool fresh = valid && at != cand;
    for (unsigned long long m = __ballot(fresh); m != 0; m = __ballot(fresh)) {
        const int64_t v = __shfl(cand, __ffsll((long long)m) - 1, 64);
        fresh = fresh && cand != v;
        if (nc >= kMaxCuts) return false;
        const int pos = __popcll(__ballot(c < v));
        const int64_t below = __shfl(c, lane > 0 ? lane - 1 : 0, 64);
        c = lane < pos ? c : (lane == pos ? v : below);
        ++nc;
        changed = true;
    }
    return true;
}

// Piece boundaries of the fused permutation of a node of S elements: the
// block boundaries closed under the permutation (starts and ends of images)
// and its inverse.  False if more than kMaxCuts are needed.
__device__ __forceinline__ bool fz_closure(const FusedPerm &f, int64_t S, int64_t &c, int &nc) {
    const int lane = threadIdx.x & 63;
    c = kCutNone;
    nc = 0;
    bool changed = false;
    int64_t b0 = lane == 8 ? S : 0;
#pragma unroll
    for (int b = 1; b < 8; ++b) b0 = lane == b ? f.src[b] : b0;
    if (!fz_add(c, nc, b0, lane <= 8, changed)) return false;
    for (int pass = 0; pass < 8; ++pass) {
        changed = false;
#pragma unroll
        for (int col = 0; col < 4; ++col) {
            const int64_t x = c;
            const bool has = lane < nc;
            int64_t cand;
            bool valid;
            if (col == 0) { cand = fz_fwd(f, x); valid = has && x < S; }
            else if (col == 1) { cand = fz_inv(f, x); valid = has && x < S; }
            else if (col == 2) { cand = fz_fwd(f, x - 1) + 1; valid = has && x > 0; }
            else { cand = fz_inv(f, x - 1) + 1; valid = has && x > 0; }
            if (!fz_add(c, nc, cand, valid, changed)) return false;
        }
        if (!changed) return true;
    }
    return false;
}

// Cycles of equal-length pieces between the cuts, one lane per piece;
// written as exchange descriptors (slots and work items reserved at once, in
// lane order).  False (nothing moved) if an image is not a piece of the
// same length, a cycle is longer than kMaxCyc, or the descriptor array is
// full (an error bit is then raised).
__device__ __forceinline__ bool fz_emit_cycles(const Plan &pl, const Work &w, int level,
                                               int64_t base, const FusedPerm &f, int64_t c,
                                               int nc) {
    const int lane = threadIdx.x & 63;
    const int64_t hi = __shfl(c, lane < 63 ? lane + 1 : 63, 64);
    const bool piece = lane + 1 < nc;
    const int64_t L = piece ? hi - c : 0;
    const int64_t img = piece ? fz_fwd(f, c) : c;
    const bool moving = piece && img != c;
    const int t = wave_lower_bound(c, img);
    const int64_t ct = __shfl(c, t, 64);
    const int64_t Lt = __shfl(L, t, 64);
    if (__ballot(moving && (ct != img || t + 1 >= nc || Lt != L))) return false;
    const int n1 = moving ? t : lane;
    const int n2 = __shfl(n1, n1, 64);
    const int n3 = __shfl(n1, n2, 64);
    const int n4 = __shfl(n1, n3, 64);
    const int clen = n2 == lane ? 2 : n3 == lane ? 3 : n4 == lane ? 4 : 0;
    if (__ballot(moving && clen == 0)) return false;
    const bool leader = moving && lane < n1 && (clen < 3 || lane < n2) && (clen < 4 || lane < n3);
    const int64_t s1 = __shfl(c, n1, 64), s2 = __shfl(c, n2, 64), s3 = __shfl(c, n3, 64);
    // inclusive scans of work items and cycles over the leader lanes
    const int64_t us = pl.rot_scale;            // descriptors are in exchange units
    const int64_t nw = leader ? (L * us + kRotChunk - 1) / kRotChunk : 0;
    int64_t sw = nw, mv = leader ? (int64_t)clen * L : 0;
    int sc = leader ? 1 : 0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t tw = __shfl(sw, lane >= d ? lane - d : 0, 64);
        const int64_t tm = __shfl(mv, lane >= d ? lane - d : 0, 64);
        const int tc = __shfl(sc, lane >= d ? lane - d : 0, 64);
        if (lane >= d) { sw += tw; mv += tm; sc += tc; }
    }
    const int64_t total_w = __shfl(sw, 63, 64), moved = __shfl(mv, 63, 64);
    const int ncyc = __shfl(sc, 63, 64);
    if (ncyc == 0) return true;
    unsigned long long packed = 0;
    if (lane == 0) {
        packed = atomicAdd(&w.ctr->level_rot[level],
                           ((unsigned long long)ncyc << kRotCountShift) |
                               (unsigned long long)total_w);
        atomicAdd(&w.ctr->rotated, (unsigned long long)moved);
    }
    packed = __shfl(packed, 0, 64);
    const int64_t slot0 = (int64_t)(packed >> kRotCountShift);
    if (slot0 + ncyc > pl.cap_rot) {
        // The reservation cannot be undone: the slots of it that lie inside
        // the array get empty exchanges (no stale descriptor is ever read),
        // and the node falls back to its plain split.
        if (lane == 0) raise_error(w, kErrCapacity);
        if (leader && slot0 + sc - 1 < pl.cap_rot) {
            Rot r = {};
            r.w0 = (int64_t)(packed & kRotWorkMask) + sw - nw;
            r.nw = nw;
            r.stash0 = -1;
            w.rot[slot0 + sc - 1] = r;
        }
        return false;
    }
    if (leader) {
        Rot r;
        r.pos = base * us; r.lx = 0; r.ly = 0;
        r.w0 = (int64_t)(packed & kRotWorkMask) + sw - nw;
        r.nw = nw;
        r.stash0 = -1;
        r.len = L * us;
        r.start[0] = (base + c) * us;
        r.start[1] = (base + s1) * us;
        r.start[2] = clen > 2 ? (base + s2) * us : 0;
        r.start[3] = clen > 3 ? (base + s3) * us : 0;
        r.c = clen;
        r.pad = 0;
        w.rot[slot0 + sc - 1] = r;
    }
    return true;
}

// The fused exchange of a node (all lanes of the wave).  False (nothing
// emitted) if the permutation does not fit.
__device__ __forceinline__ bool emit_fused(const Plan &pl, const Work &w, int level, int64_t base,
                                           const FusedPerm &f, int64_t S) {
    int64_t c;
    int nc;
    if (!fz_closure(f, S, c, nc)) return false;
    return fz_emit_cycles(pl, w, level, base, f, c, nc);
}

__device__ __forceinline__ void emit_node(const Plan &pl, const Work &w, int level, Node *out,
                                          const Node &nd) {
    unsigned long long slot = atomicAdd(&w.ctr->level_nodes[level], 1ull);
    if ((int64_t)slot >= pl.cap_nodes) {
        raise_error(w, kErrCapacity);
        return;
    }
    out[slot] = nd;
}

// What a child of a fused node does at the next level, read on the original
// layout: 0 = nothing to split (empty part, in order, or a leaf), 1 = a
// symmetric split (block swap), 2 = anything else (not fusable).  The end
// keys are loaded by the caller (both children's at once: one round of
// loads instead of four dependent ones); an empty child's are not used.
template <typename K>
__device__ __forceinline__ int child_kind(const Plan &pl, int64_t la, int64_t lb, K a_first,
                                          K a_last, K b_first, K b_last) {
    if (la == 0 || lb == 0) return 0;
    if (a_last <= b_first) return 0;
    if (a_first > b_last) return 2;                    // a whole-child exchange
    if (la + lb <= pl.leaf_cap || (la < lb ? la : lb) <= pl.leaf_span) return 0;
    const int64_t S = la + lb, mx = la > lb ? la : lb;
    return (mx * 16 <= S * 9) ? 1 : 2;
}

// Co-ranks of the cell boundaries m*tile (m = 0..cells) of a single
// instance, on the layout before any exchange, one lane per boundary.  They
// run in the first division level's launch (workgroups past the split's
// own), beside its latency-bound searches.  The merge's leaves are ranges of
// the stable merge's output, so a cell boundary inside a leaf that starts at
// output k0 and A index i0 has the leaf-local co-rank cell_rank - i0 there.
// Nothing is searched when the input is already in order (no leaf then).
// With a merge model each search starts from the model's bracket (the
// learned split: fewer probes, so fewer lines fetched in this launch).
template <bool LEARNED, typename KP>
__device__ void cell_coranks(KP data, const int64_t *__restrict__ offsets, const Plan &pl,
                             const Work &w, const MlpDev *__restrict__ mlp, int64_t b,
                             int64_t nb) {
    const int64_t o0 = offsets[0], o1 = offsets[1], o2 = offsets[2];
    const int64_t la = o1 - o0, lb = o2 - o1;
    if (la <= 0 || lb <= 0) return;
    const KP A = data + o0;
    const KP B = A + la;
    if (A[la - 1] <= B[0]) return;
    const int64_t S = la + lb;
    const int64_t ncell = (S + pl.tile - 1) / pl.tile;
    uint32_t probes = 0, searches = 0;
    for (int64_t m = b * blockDim.x + threadIdx.x; m <= ncell; m += nb * blockDim.x) {
        int64_t i;
        if (m == 0) {
            i = 0;
        } else if (m == ncell) {
            i = la;
        } else {
            ++searches;
            const int64_t d = m * pl.tile;
            if (LEARNED)
                i = corank_learned(A, la, B, lb, d, mlp, d, S, la, 0, probes);
            else
                i = corank_plain(A, la, B, lb, d, probes);
        }
        w.cell_rank[m] = i;
    }
    if (searches) {
        atomicAdd(&w.ctr->searches, (unsigned long long)searches);
        atomicAdd(&w.ctr->probes, (unsigned long long)probes);
    }
}

// One lane per node classifies it (early exits, leaf); the nodes of a wave
// that must be split are then searched one after another by the whole wave
// with the cooperative 64-ary co-rank (a handful of dependent rounds).  A
// node whose children both split symmetrically has its two levels fused: the
// children's searches run in the same wave and the node emits the cycles of
// the composed exchange and its grandchildren (to level + 2).
template <typename K, typename KP, bool LEARNED>
__global__ __launch_bounds__(kSplitThreads) void k_split(KP data,
                                                         const int64_t *__restrict__ offsets,
                                                         Plan pl, Work w, int level,
                                                         const MlpDev *__restrict__ mlp,
                                                         int split_grid) {
    if ((int)blockIdx.x >= split_grid) {      // cell co-ranks (first level, Plan::cells)
        cell_coranks<LEARNED>(data, offsets, pl, w, mlp, (int64_t)blockIdx.x - split_grid,
                              (int64_t)gridDim.x - split_grid);
        return;
    }
    const unsigned long long cnt_raw = w.ctr->level_nodes[level];
    const int64_t cnt = (int64_t)cnt_raw < pl.cap_nodes ? (int64_t)cnt_raw : pl.cap_nodes;
    const Node *in = w.nodes[level % 3];
    Node *out = w.nodes[(level + 1) % 3];
    Node *out2 = w.nodes[(level + 2) % 3];
    // two levels fused only when the grandchildren still get a level of
    // their own (the last level only classifies)
    const bool may_fuse = pl.fuse && level + 2 <= pl.max_levels - 1;
    const int lane = threadIdx.x & 63;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)split_grid * blockDim.x;
    if (gid == 0 && cnt > 0) atomicMax(&w.ctr->levels_used, (unsigned long long)(level + 1));
    uint32_t rounds = 0, searches = 0;          // wave-uniform counts
    uint32_t fm_probes = 0, fm_searches = 0;    // per lane (FindMedian)
    // A level with no more nodes than waves gives each wave one node (lane
    // 0), so their searches run side by side instead of one after another in
    // one wave; otherwise a wave takes 64 consecutive nodes, one per lane.
    const int64_t wave = gid >> 6, nwaves = stride >> 6;
    const bool spread = cnt <= nwaves;
    for (int64_t idx0 = spread ? wave : gid - lane; idx0 < cnt;
         idx0 += spread ? cnt : stride) {                          // wave-uniform
        const int64_t idx = spread ? (lane == 0 ? idx0 : cnt) : idx0 + lane;
        Node nd;
        bool split = false;
        int64_t k = 0;
        if (idx < cnt) {
            nd = in[idx];
            const int64_t la = nd.la, lb = nd.lb;
            const KP A = data + nd.base;
            const KP B = A + la;
            // the four end keys in one round of loads
            bool in_order = true, reversed = false;
            if (la > 0 && lb > 0) {
                const K a_first = A[0], a_last = A[la - 1], b_first = B[0], b_last = B[lb - 1];
                in_order = a_last <= b_first;
                reversed = a_first > b_last;
            }
            if (in_order) {
                // nothing to merge (an empty part, or already in order)
            } else if (reversed && level + 1 < pl.max_levels) {
                // every B before every A: one exchange.  At the last level such
                // a pair is merged as a leaf instead (every node there is within
                // the leaf bounds), so that level never exchanges and its
                // exchange launches are not enqueued.
                emit_rot(pl, w, level, nd.base, la, lb);
            } else if (la + lb <= pl.leaf_cap || (la < lb ? la : lb) <= pl.leaf_span) {
                emit_leaf(pl, w, nd);
            } else if (level + 1 >= pl.max_levels) {
                raise_error(w, kErrOversizeLeaf);   // depth bound violated
            } else {
                const int64_t S = la + lb;
                const int64_t mx = la > lb ? la : lb;
                k = (mx * 16 <= S * 9) ? la : S / 2;
                split = true;
                if (pl.split_method == kSplitFindMedian) {
                    // FindMedian, kept when its split is valid and no child
                    // exceeds the 9/16 bound the level count assumes; else
                    // the exact co-rank split below
                    int64_t pa, pb;
                    find_median(A, la, B, lb, pa, pb, fm_probes);
                    ++fm_searches;
                    const int64_t kf = pa + pb;
                    const int64_t big = kf > S - kf ? kf : S - kf;
                    const bool valid =
                        (pa == 0 || pb == lb || A[pa - 1] <= B[pb]) &&
                        (pb == 0 || pa == la || B[pb - 1] <= A[pa]);
                    if (valid && big * 16 <= S * 9 + 16 && kf > 0 && kf < S) {
                        emit_split(pl, w, level, out, nd, pa, pb);
                        split = false;
                    } else {
                        atomicAdd(&w.ctr->split_fallbacks, 1ull);
                    }
                }
            }
        }
        unsigned long long todo = __ballot(split);
        while (todo) {
            const int src = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const int64_t base = __shfl(nd.base, src, 64);
            const int64_t la = __shfl(nd.la, src, 64);
            const int64_t lb = __shfl(nd.lb, src, 64);
            const int64_t kk = __shfl(k, src, 64);
            const KP A = data + base;
            const KP B = A + la;
            int64_t i;
            ++searches;
            if (LEARNED) {
                const int64_t k0 = __shfl(nd.k0, src, 64);
                const int64_t i0 = __shfl(nd.i0, src, 64);
                const int inst = __shfl(nd.inst, src, 64);
                int64_t o0 = offsets[2 * inst], o1 = offsets[2 * inst + 1],
                        o2 = offsets[2 * inst + 2];
                i = corank_group_learned<64>(A, la, B, lb, kk, mlp, k0 + kk, o2 - o0, o1 - o0,
                                             i0, rounds);
            } else {
                i = corank_group<64>(A, la, B, lb, kk, rounds);
            }
            const int64_t j = kk - i;
            bool fused = false;
            if (may_fuse && kk == la && la - i > 0 && j > 0) {
                // children on the original layout: L = A[0,i) | B[0,j),
                // R = A[i,la) | B[j,lb).  Their end keys, with an empty part's
                // indices moved to a key of the node (la, lb > 0; i < la here)
                // so that every load is in range
                const int64_t i1 = i > 0 ? i - 1 : 0, j1 = j > 0 ? j - 1 : 0;
                const int64_t jx = j < lb ? j : lb - 1;
                const K l_af = A[0], l_al = A[i1], l_bf = B[0], l_bl = B[j1];
                const K r_af = A[i], r_al = A[la - 1], r_bf = B[jx], r_bl = B[lb - 1];
                const int kl = child_kind(pl, i, j, l_af, l_al, l_bf, l_bl);
                const int kr = child_kind(pl, la - i, lb - j, r_af, r_al, r_bf, r_bl);
                if (kl != 2 && kr != 2) {
                    int64_t il = i, ir = la - i;          // kept whole: (|A_X|, |B_X|)
                    ++searches;
                    if (!LEARNED) {
                        // both children's searches at once: lanes 0-31 split
                        // L at its own A-length, lanes 32-63 split R (a
                        // child that is not split searches an empty range)
                        const bool left = lane < 32;
                        const bool need = left ? kl == 1 : kr == 1;
                        const KP A2 = left ? A : A + i;
                        const KP B2 = left ? B : B + j;
                        const int64_t a2 = need ? (left ? i : la - i) : 0;
                        const int64_t b2 = need ? (left ? j : lb - j) : 0;
                        const int64_t r2 = corank_group<32>(A2, a2, B2, b2, a2, rounds);
                        const int64_t rl = __shfl(r2, 0, 64), rr = __shfl(r2, 32, 64);
                        if (kl == 1) il = rl;
                        if (kr == 1) ir = rr;
                    } else {
                        // learned searches, one child after the other
                        const int64_t k0 = __shfl(nd.k0, src, 64);
                        const int64_t i0 = __shfl(nd.i0, src, 64);
                        const int inst = __shfl(nd.inst, src, 64);
                        const int64_t o0 = offsets[2 * inst], o1 = offsets[2 * inst + 1],
                                      o2 = offsets[2 * inst + 2];
                        if (kl == 1)
                            il = corank_group_learned<64>(A, i, B, j, i, mlp, k0 + i, o2 - o0,
                                                          o1 - o0, i0, rounds);
                        if (kr == 1)
                            ir = corank_group_learned<64>(A + i, la - i, B + j, lb - j, la - i, mlp,
                                                          k0 + kk + (la - i), o2 - o0, o1 - o0,
                                                          i0 + i, rounds);
                    }
                    // child splits (il, jl) of L and (ir, jr) of R; the
                    // whole wave decomposes the permutation
                    const int64_t jl = kl == 1 ? i - il : j;
                    const int64_t jr = kr == 1 ? (la - i) - ir : lb - j;
                    FusedPerm f;
                    f.src[0] = 0;            f.len[0] = il;               f.dst[0] = 0;
                    f.src[1] = il;           f.len[1] = i - il;           f.dst[1] = il + jl;
                    f.src[2] = i;            f.len[2] = ir;               f.dst[2] = i + j;
                    f.src[3] = i + ir;       f.len[3] = la - i - ir;      f.dst[3] = i + j + ir + jr;
                    f.src[4] = la;           f.len[4] = jl;               f.dst[4] = il;
                    f.src[5] = la + jl;      f.len[5] = j - jl;           f.dst[5] = i + jl;
                    f.src[6] = la + j;       f.len[6] = jr;               f.dst[6] = i + j + ir;
                    f.src[7] = la + j + jr;  f.len[7] = lb - j - jr;      f.dst[7] = la + j + jr;
                    fused = emit_fused(pl, w, level, base, f, la + lb);
                    if (fused && lane == src) {
                        atomicAdd(&w.ctr->fused, 1ull);
                        // grandchildren (or whole children) go to level + 2
                        Node g;
                        g.inst = nd.inst;
                        g.pad = 0;
                        if (kl == 1) {
                            g.base = nd.base; g.la = il; g.lb = jl; g.k0 = nd.k0; g.i0 = nd.i0;
                            emit_node(pl, w, level + 2, out2, g);
                            g.base = nd.base + il + jl; g.la = i - il; g.lb = j - jl;
                            g.k0 = nd.k0 + il + jl; g.i0 = nd.i0 + il;
                            emit_node(pl, w, level + 2, out2, g);
                        } else {
                            g.base = nd.base; g.la = i; g.lb = j; g.k0 = nd.k0; g.i0 = nd.i0;
                            emit_node(pl, w, level + 2, out2, g);
                        }
                        const int64_t rb = nd.base + kk;
                        if (kr == 1) {
                            g.base = rb; g.la = ir; g.lb = jr; g.k0 = nd.k0 + kk;
                            g.i0 = nd.i0 + i;
                            emit_node(pl, w, level + 2, out2, g);
                            g.base = rb + ir + jr; g.la = la - i - ir; g.lb = lb - j - jr;
                            g.k0 = nd.k0 + kk + ir + jr; g.i0 = nd.i0 + i + ir;
                            emit_node(pl, w, level + 2, out2, g);
                        } else {
                            g.base = rb; g.la = la - i; g.lb = lb - j; g.k0 = nd.k0 + kk;
                            g.i0 = nd.i0 + i;
                            emit_node(pl, w, level + 2, out2, g);
                        }
                    }
                }
            }
            if (lane != src) continue;
            if (!fused) emit_split(pl, w, level, out, nd, i, j);
        }
    }
    if (pl.split_method == kSplitFindMedian) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            fm_probes += __shfl_xor(fm_probes, o, 64);
            fm_searches += __shfl_xor(fm_searches, o, 64);
        }
        searches += fm_searches;
        rounds += fm_probes;
    }
    if (lane == 0 && searches) {
        atomicAdd(&w.ctr->searches, (unsigned long long)searches);
        atomicAdd(&w.ctr->probes, (unsigned long long)rounds);
    }
}

// Recursive division without data movement (the pivot search of every
// level of Sec. 3, as sOptMov does before it moves anything): node q of level
// `level` is (a_off, la, b_off, lb) in the original A and B; its children are
// 2q and 2q+1 of the next level.  One lane per node.
template <typename K>
__global__ __launch_bounds__(kSplitThreads) void k_divide(const K *__restrict__ A,
                                                          const K *__restrict__ B, int method,
                                                          int64_t nnodes,
                                                          const int64_t *__restrict__ in,
                                                          int64_t *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnodes) return;
    const int64_t ao = in[4 * q], la = in[4 * q + 1], bo = in[4 * q + 2], lb = in[4 * q + 3];
    int64_t i, j;
    uint32_t probes = 0;
    if (method == kSplitFindMedian) {
        find_median(A + ao, la, B + bo, lb, i, j, probes);
    } else {
        const int64_t k = (la + lb) / 2;
        i = corank_plain(A + ao, la, B + bo, lb, k, probes);
        j = k - i;
    }
    int64_t *c = out + 8 * q;
    c[0] = ao; c[1] = i; c[2] = bo; c[3] = j;
    c[4] = ao + i; c[5] = la - i; c[6] = bo + j; c[7] = lb - j;
}

template <typename K>
static hipError_t divide_t(const void *data, int64_t la, int method, int level,
                           const int64_t *in, int64_t *out, hipStream_t s) {
    const int64_t nn = (int64_t)1 << level;
    const int g = (int)((nn + kSplitThreads - 1) / kSplitThreads);
    const K *A = (const K *)data;
    hipLaunchKernelGGL(k_divide<K>, dim3(g), dim3(kSplitThreads), 0, s, A, A + la, method, nn,
                       in, out);
    return hipGetLastError();
}

hipError_t launch_divide(int key, const void *data, int64_t la, int64_t lb, int method,
                         int level, const int64_t *nodes_in, int64_t *nodes_out, hipStream_t s) {
    (void)lb;
    switch (key) {
        case kI32: return divide_t<int32_t>(data, la, method, level, nodes_in, nodes_out, s);
        case kU32: return divide_t<uint32_t>(data, la, method, level, nodes_in, nodes_out, s);
        case kI64: return divide_t<int64_t>(data, la, method, level, nodes_in, nodes_out, s);
        case kU64: return divide_t<uint64_t>(data, la, method, level, nodes_in, nodes_out, s);
    }
    return hipErrorInvalidValue;
}

// Tile co-ranks: tile t of leaf l starts at local diagonal (t - tile_start[l]) * tile.
// One lane per tile, binary searches.  (Measured: group-cooperative searches
// with 8 lanes per tile need fewer dependent rounds but 2-3x the loads, and
// are slower here: this stage is bound by the memory system, not latency.)
template <typename K, typename KP, bool LEARNED>
__global__ __launch_bounds__(kSplitThreads) void k_tilerank(KP data,
                                                            const int64_t *__restrict__ offsets,
                                                            Plan pl, Work w,
                                                            const MlpDev *__restrict__ mlp) {
    const int64_t ntiles = (int64_t)w.ctr->tiles;
    int64_t nleaves = (int64_t)w.ctr->leaves;
    if (nleaves > pl.cap_leaves) nleaves = pl.cap_leaves;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t probes = 0, searches = 0;
    for (int64_t t = gid; t < ntiles && t < pl.cap_tiles; t += stride) {
        // leaf = last l with tile_start[l] <= t
        int64_t lo = 0, hi = nleaves;
        while (hi - lo > 1) {
            int64_t mid = (lo + hi) >> 1;
            if (w.tile_start[mid] <= t) lo = mid; else hi = mid;
        }
        const Leaf lf = w.leaves[lo];
        const int64_t d = (t - w.tile_start[lo]) * pl.tile;
        int64_t i = 0;
        if (d > 0) {
            const KP A = data + lf.base;
            const KP B = A + lf.la;
            ++searches;
            if (LEARNED) {
                int64_t o0 = offsets[2 * lf.inst], o1 = offsets[2 * lf.inst + 1],
                        o2 = offsets[2 * lf.inst + 2];
                i = corank_learned(A, lf.la, B, lf.lb, d, mlp, lf.k0 + d, o2 - o0, o1 - o0,
                                   lf.i0, probes);
            } else {
                i = corank_plain(A, lf.la, B, lf.lb, d, probes);
            }
        }
        w.tile_rank[t] = i;
        w.tile_leaf[t] = (int32_t)lo;
    }
    if (searches) {
        atomicAdd(&w.ctr->searches, (unsigned long long)searches);
        atomicAdd(&w.ctr->probes, (unsigned long long)probes);
    }
}

// Stand-alone co-rank of a list of diagonals (one lane per diagonal).
template <typename K, bool LEARNED>
__global__ __launch_bounds__(kSplitThreads) void k_corank(const K *__restrict__ data, int64_t la,
                                                          int64_t lb, const int64_t *__restrict__ ks,
                                                          int64_t nk, int64_t *__restrict__ out,
                                                          const MlpDev *__restrict__ mlp,
                                                          int32_t *__restrict__ probes_out) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const K *A = data;
    const K *B = data + la;
    for (int64_t p = gid; p < nk; p += stride) {
        int64_t k = ks[p];
        uint32_t probes = 0;
        int64_t i;
        if (k < 0 || k > la + lb) {
            i = -1;                                  // out-of-range diagonal
        } else if (LEARNED) {
            i = corank_learned(A, la, B, lb, k, mlp, k, la + lb, la, 0, probes);
        } else {
            i = corank_plain(A, la, B, lb, k, probes);
        }
        out[p] = i;
        if (probes_out) probes_out[p] = (int32_t)probes;
    }
}

// Checked mode: every run ascending, every instance's offsets monotone.
template <typename K>
__global__ void k_check_sorted(const K *__restrict__ data, const int64_t *__restrict__ offsets,
                               int64_t n_inst, Counters *ctr, int64_t stride) {
    for (int64_t q = blockIdx.x; q < n_inst; q += gridDim.x) {
        int64_t o0 = offsets[2 * q], o1 = offsets[2 * q + 1], o2 = offsets[2 * q + 2];
        if (o1 < o0 || o2 < o1) {
            if (threadIdx.x == 0) atomicOr(&ctr->error, kErrOffsets);
            continue;
        }
        bool bad = false;
        for (int64_t x = o0 + threadIdx.x; x + 1 < o2; x += blockDim.x) {
            if (x + 1 == o1) continue;                       // the A|B seam is not a run
            if (data[(x + 1) * stride] < data[x * stride]) bad = true;
        }
        if (bad) atomicOr(&ctr->error, kErrNotSorted);
    }
}

static int grid_for(int64_t items, int threads, int cap) {
    int64_t g = (items + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_init(const Plan &pl, const Work &w, const int64_t *d_offsets, int64_t la,
                       int64_t lb, hipStream_t s) {
    int64_t items = pl.n_inst > 256 ? pl.n_inst : 256;
    int g = grid_for(items, 256, 4096);
    hipLaunchKernelGGL(k_init, dim3(g), dim3(256), 0, s, w.ctr, w.nodes[0], d_offsets, pl.n_inst,
                       la, lb, w.offsets1);
    return hipGetLastError();
}

template <typename K>
static hipError_t split_t(const void *data, const int64_t *offs, const Plan &pl, const Work &w,
                          int level, const MlpDev *mlp, hipStream_t s) {
    // few nodes: one-wave workgroups, one per possible node (up to 2048),
    // so the waves' searches run side by side on different CUs
    const bool few = pl.cap_nodes <= 128 * kSplitThreads;
    const int th = few ? 64 : kSplitThreads;
    const int g = few ? (int)(pl.cap_nodes < 2048 ? pl.cap_nodes : 2048)
                      : grid_for(pl.cap_nodes, th, 2048);
    // the first level of a cell-tiled merge also finds the cell co-ranks:
    // one lane per cell boundary in workgroups past the split's
    const int gc = (pl.cells && level == 0) ? (int)((pl.total / pl.tile + 2 + th - 1) / th) : 0;
    if (pl.row_stride > 0) {
        if (mlp || gc) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_split<K, RowKeys<K>, false>), dim3(g), dim3(th), 0, s,
                           RowKeys<K>{(const K *)data, pl.row_stride}, offs, pl, w, level, mlp, g);
    } else if (mlp) {
        hipLaunchKernelGGL((k_split<K, const K *, true>), dim3(g + gc), dim3(th), 0, s,
                           (const K *)data, offs, pl, w, level, mlp, g);
    } else {
        hipLaunchKernelGGL((k_split<K, const K *, false>), dim3(g + gc), dim3(th), 0, s,
                           (const K *)data, offs, pl, w, level, mlp, g);
    }
    return hipGetLastError();
}

hipError_t launch_split(int key, void *data, const int64_t *offs, const Plan &pl, const Work &w,
                        int level, const MlpDev *mlp, hipStream_t s) {
    switch (key) {
        case kI32: return split_t<int32_t>(data, offs, pl, w, level, mlp, s);
        case kU32: return split_t<uint32_t>(data, offs, pl, w, level, mlp, s);
        case kI64: return split_t<int64_t>(data, offs, pl, w, level, mlp, s);
        case kU64: return split_t<uint64_t>(data, offs, pl, w, level, mlp, s);
    }
    return hipErrorInvalidValue;
}

template <typename K>
static hipError_t tilerank_t(const void *data, const int64_t *offs, const Plan &pl, const Work &w,
                             const MlpDev *mlp, hipStream_t s) {
    // With few tiles, one wave per workgroup spreads the dependent searches
    // over every CU instead of piling their misses onto a few (measured on
    // 15k tiles: 57 -> 44 us); with many tiles, full workgroups do better.
    const int th = pl.cap_tiles <= 128 * kSplitThreads ? 64 : kSplitThreads;
    const int g = grid_for(pl.cap_tiles, th, 16384);
    if (pl.row_stride > 0) {
        if (mlp) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_tilerank<K, RowKeys<K>, false>), dim3(g), dim3(th), 0, s,
                           RowKeys<K>{(const K *)data, pl.row_stride}, offs, pl, w, mlp);
    } else if (mlp) {
        hipLaunchKernelGGL((k_tilerank<K, const K *, true>), dim3(g), dim3(th), 0, s,
                           (const K *)data, offs, pl, w, mlp);
    } else {
        hipLaunchKernelGGL((k_tilerank<K, const K *, false>), dim3(g), dim3(th), 0, s,
                           (const K *)data, offs, pl, w, mlp);
    }
    return hipGetLastError();
}

hipError_t launch_tilerank(int key, void *data, const int64_t *offs, const Plan &pl,
                           const Work &w, const MlpDev *mlp, hipStream_t s) {
    switch (key) {
        case kI32: return tilerank_t<int32_t>(data, offs, pl, w, mlp, s);
        case kU32: return tilerank_t<uint32_t>(data, offs, pl, w, mlp, s);
        case kI64: return tilerank_t<int64_t>(data, offs, pl, w, mlp, s);
        case kU64: return tilerank_t<uint64_t>(data, offs, pl, w, mlp, s);
    }
    return hipErrorInvalidValue;
}

template <typename K>
static hipError_t corank_t(const void *data, int64_t la, int64_t lb, const int64_t *ks, int64_t nk,
                           int64_t *out, const MlpDev *mlp, int32_t *probes, hipStream_t s) {
    int g = grid_for(nk, kSplitThreads, 8192);
    if (mlp)
        hipLaunchKernelGGL((k_corank<K, true>), dim3(g), dim3(kSplitThreads), 0, s,
                           (const K *)data, la, lb, ks, nk, out, mlp, probes);
    else
        hipLaunchKernelGGL((k_corank<K, false>), dim3(g), dim3(kSplitThreads), 0, s,
                           (const K *)data, la, lb, ks, nk, out, mlp, probes);
    return hipGetLastError();
}

hipError_t launch_corank(int key, const void *data, int64_t la, int64_t lb, const int64_t *d_k,
                         int64_t nk, int64_t *d_out, const MlpDev *mlp, int32_t *d_probes,
                         hipStream_t s) {
    switch (key) {
        case kI32: return corank_t<int32_t>(data, la, lb, d_k, nk, d_out, mlp, d_probes, s);
        case kU32: return corank_t<uint32_t>(data, la, lb, d_k, nk, d_out, mlp, d_probes, s);
        case kI64: return corank_t<int64_t>(data, la, lb, d_k, nk, d_out, mlp, d_probes, s);
        case kU64: return corank_t<uint64_t>(data, la, lb, d_k, nk, d_out, mlp, d_probes, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_check_sorted(int key, const void *data, const int64_t *d_offsets,
                               int64_t n_inst, Counters *ctr, int64_t stride, hipStream_t s) {
    int g = (int)(n_inst < 4096 ? (n_inst < 1 ? 1 : n_inst) : 4096);
    switch (key) {
        case kI32:
            hipLaunchKernelGGL(k_check_sorted<int32_t>, dim3(g), dim3(256), 0, s,
                               (const int32_t *)data, d_offsets, n_inst, ctr, stride);
            break;
        case kU32:
            hipLaunchKernelGGL(k_check_sorted<uint32_t>, dim3(g), dim3(256), 0, s,
                               (const uint32_t *)data, d_offsets, n_inst, ctr, stride);
            break;
        case kI64:
            hipLaunchKernelGGL(k_check_sorted<int64_t>, dim3(g), dim3(256), 0, s,
                               (const int64_t *)data, d_offsets, n_inst, ctr, stride);
            break;
        case kU64:
            hipLaunchKernelGGL(k_check_sorted<uint64_t>, dim3(g), dim3(256), 0, s,
                               (const uint64_t *)data, d_offsets, n_inst, ctr, stride);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace imerge
