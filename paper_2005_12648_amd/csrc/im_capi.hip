// im_capi.hip -- the extern "C" boundary (include/inplace_merge.h): argument
// validation, workspace management, plan sizing and the launch sequence.
// No host synchronisation on the merge path (only in checked mode, when
// statistics are fetched, and when a model is trained).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/inplace_merge.h"
#include "im_common.h"

using namespace imerge;

namespace {

thread_local std::string g_err = "";
thread_local im_stats g_stats = {};
thread_local Counters *g_last_ctr = nullptr;
thread_local hipStream_t g_last_stream = nullptr;

// Stage timing (inplace_merge_profile): events recorded on the caller's
// stream around each group of launches, read back by
// inplace_merge_profile_read.
// (stage 2, leaf planning, has had no launch since leaves get their tiles as
// they are emitted; it stays in the numbering of the public API and reads 0)
enum { kStSplit = 0, kStRotate = 1, kStPlan = 2, kStTileRank = 3, kStLeafMerge = 4, kStCount = 5 };
struct ProfRec {
    int stage;
    int launches;
    hipEvent_t a, b;
};
thread_local bool g_prof = false;
thread_local std::vector<ProfRec> g_prof_recs;
thread_local std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Returns the start event (or nullptr when profiling is off).
hipEvent_t prof_begin(hipStream_t s) {
    if (!g_prof) return nullptr;
    hipEvent_t a = prof_event();
    if (a && hipEventRecord(a, s) != hipSuccess) return nullptr;
    return a;
}

void prof_end(hipEvent_t a, int stage, int launches, hipStream_t s) {
    if (!a) return;
    hipEvent_t b = prof_event();
    if (!b || hipEventRecord(b, s) != hipSuccess) return;
    g_prof_recs.push_back(ProfRec{stage, launches, a, b});
}

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *where) {
    return fail(IM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define IM_HIP(call, where)                          \
    do {                                             \
        hipError_t _e = (call);                      \
        if (_e != hipSuccess) return hip_fail(_e, where); \
    } while (0)

int key_size(int dt) { return (dt == IM_INT32 || dt == IM_UINT32) ? 4 : 8; }
bool valid_dtype(int dt) { return dt >= IM_INT32 && dt <= IM_UINT64; }

bool checked_mode() {
    const char *v = std::getenv("IM_CHECK");
    return v && v[0] == '1';
}

struct DevState {
    std::mutex mu;
    void *ws = nullptr;          // library-owned workspace
    size_t ws_bytes = 0;
    void *user_ws = nullptr;     // caller-owned workspace (if set)
    size_t user_bytes = 0;
    hipEvent_t done = nullptr;   // last enqueued use of the workspace
    bool done_valid = false;
    int grid[kLeafCfgs][2][3] = {};   // leaf grid by (config, key 4/8, payload 0/4/8)
    int rows_grid[4][4] = {};         // rows leaf grid by (key code, row kind)
    // Autotuned leaf configuration by (key 4/8, payload 0/4/8, floor(log2 of
    // the mean instance size)); -1: not tuned.
    int tuned[2][3][64];
    // Host-memory word (pinned, mapped) that kernels raise error bits into
    // (Work::host_err); read without a synchronisation.
    unsigned *h_err = nullptr;
    unsigned *d_err = nullptr;
    bool err_tried = false;
    // Tile flags sit right after the counters.  flag_cap flags there are
    // known to hold only values < epoch (zeroed, or written by earlier
    // calls); the rest of the layout always starts after them.
    int64_t flag_cap = 0;
    uint32_t epoch = 0;
    // The allocation-free entry point's workspace: this device's copy of the
    // static `scratch` array (its address, looked up once), with its own
    // flag bookkeeping.
    void *scr_ptr = nullptr;
    int64_t scr_flag_cap = 0;
    uint32_t scr_epoch = 0;
    std::string cache_path;      // the IM_AUTOTUNE_CACHE file last read for this device
    DevState() {
        for (auto &a : tuned)
            for (auto &b : a)
                for (int &c : b) c = -1;
    }
};

std::atomic<int> g_force_cfg{-1};   // inplace_merge_set_config

// Workspace of inplace_merge_noalloc: a fixed device array, one copy per
// device, held until the process ends.  Host code never uses its name as an
// address: the device address comes from hipGetSymbolAddress (scratch_base).
constexpr size_t kScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

int size_class(int64_t n_inst, int64_t total) {
    int64_t mean = total / std::max<int64_t>(n_inst, 1);
    int c = 0;
    while (c < 63 && (int64_t(2) << c) <= mean) ++c;
    return c;
}

int key_index(int ek) { return ek == 4 ? 0 : 1; }
int val_index(int ev) { return ev == 0 ? 0 : (ev == 4 ? 1 : 2); }

// IM_LOG: 0 (default) silent; 1 one line per merge call (its plan); 2 also
// the autotuner's timings and the tune cache.
int log_level() {
    const char *v = std::getenv("IM_LOG");
    return v ? (int)std::strtol(v, nullptr, 10) : 0;
}

// IM_TILE (elements per leaf tile) and IM_WAVES (wavefronts per leaf
// workgroup) pick the first leaf configuration that matches both for the
// element sizes of the call, overriding the tuned table; -1 if unset or if
// no configuration matches (then a line is logged at IM_LOG >= 1).
int env_cfg(int ek, int ev) {
    const char *te = std::getenv("IM_TILE"), *we = std::getenv("IM_WAVES");
    if (!te && !we) return -1;
    const long tile = te ? std::strtol(te, nullptr, 10) : -1;
    const long waves = we ? std::strtol(we, nullptr, 10) : -1;
    for (int c = 0; c < kLeafCfgs; ++c) {
        int th, ipt, depth;
        size_t lds;
        leaf_geometry(ek, ev, c, &th, &ipt, &depth, &lds);
        if ((tile < 0 || tile == (long)th * ipt) && (waves < 0 || waves == th / 64)) return c;
    }
    if (log_level() >= 1)
        std::fprintf(stderr, "[inplace_merge] IM_TILE=%s IM_WAVES=%s match no leaf configuration "
                             "for %d-byte keys and %d-byte payloads; ignored\n",
                     te ? te : "-", we ? we : "-", ek, ev);
    return -1;
}

void load_tune_cache(DevState *ds, int dev);

// Leaf configuration of a run: forced, else IM_TILE / IM_WAVES, else tuned
// for the class (this process's autotuner runs, or the IM_AUTOTUNE_CACHE
// file), else 0.
int choose_cfg(DevState *ds, int ek, int ev, int64_t n_inst, int64_t total, int override_cfg) {
    if (override_cfg >= 0 && override_cfg < kLeafCfgs) return override_cfg;
    int f = g_force_cfg.load();
    if (f >= 0 && f < kLeafCfgs) return f;
    const int e = env_cfg(ek, ev);
    if (e >= 0) return e;
    int t = ds->tuned[key_index(ek)][val_index(ev)][size_class(n_inst, total)];
    return (t >= 0 && t < kLeafCfgs) ? t : 0;
}

DevState g_dev[64];

DevState *dev_state(int *dev_out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    if (dev_out) *dev_out = dev;
    return &g_dev[dev];
}

// The on-disk tune cache (IM_AUTOTUNE_CACHE=<path>): one line per tuned
// workload class, "imtune1 <gcn arch> <key bytes> <payload bytes> <class>
// <config>"; later lines win.  Read by a device's first merge after the
// variable names a file it has not read; the autotuner appends its result.
// Lines of other architectures, and malformed lines, are skipped.
std::string device_arch(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    for (char &c : a)
        if (c == ' ' || c == '\n' || c == '\t') c = '_';
    return a.empty() ? "unknown" : a;
}

void load_tune_cache(DevState *ds, int dev) {
    const char *path = std::getenv("IM_AUTOTUNE_CACHE");
    if (!path || !*path || ds->cache_path == path) return;
    ds->cache_path = path;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    const std::string arch = device_arch(dev);
    char tag[32], a[128];
    int ek, ev, cls, cfg, loaded = 0;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        if (std::sscanf(line, "%31s %127s %d %d %d %d", tag, a, &ek, &ev, &cls, &cfg) != 6) continue;
        if (std::strcmp(tag, "imtune1") != 0 || arch != a) continue;
        if ((ek != 4 && ek != 8) || (ev != 0 && ev != 4 && ev != 8) || cls < 0 || cls >= 64 ||
            cfg < 0 || cfg >= kLeafCfgs)
            continue;
        ds->tuned[key_index(ek)][val_index(ev)][cls] = cfg;
        ++loaded;
    }
    std::fclose(f);
    if (log_level() >= 2)
        std::fprintf(stderr, "[inplace_merge] tune cache %s: %d entries for %s\n", path, loaded,
                     arch.c_str());
}

void save_tune_entry(int dev, int ek, int ev, int cls, int cfg) {
    const char *path = std::getenv("IM_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) {
        if (log_level() >= 1) std::fprintf(stderr, "[inplace_merge] cannot append to %s\n", path);
        return;
    }
    std::fprintf(f, "imtune1 %s %d %d %d %d\n", device_arch(dev).c_str(), ek, ev, cls, cfg);
    std::fclose(f);
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Split of the packed leaf/tile counter: enough low bits for every tile of
// the leaves within cap_leaves, the high bits for the leaf index (one bit to
// spare).  0 when the two do not fit in 64 bits (about 2^31 instances at
// once); such a plan is refused.
int leaf_shift(const Plan &pl) {
    int tb = 1, lb = 1;
    while (tb < 62 && (int64_t(1) << tb) <= pl.cap_tiles) ++tb;
    while (lb < 62 && (int64_t(1) << lb) <= pl.cap_leaves) ++lb;
    return tb + lb + 1 <= 64 ? tb : 0;
}

// Division levels: children are at most 9/16 of the parent (plus one for
// rounding); a node of at most max(leaf_cap, 2*leaf_span) elements is a
// leaf; the last level only classifies.
int division_levels(const Plan &pl, int64_t max_inst) {
    const double stop = (double)std::max<int64_t>(pl.leaf_cap, 2 * pl.leaf_span);
    int lv = 1;
    double sz = (double)max_inst;
    while (sz > stop && lv < kMaxLevels) {
        sz = sz * 9.0 / 16.0 + 1.0;
        ++lv;
    }
    return lv;
}

// Descriptor capacities.  A node is split only when it exceeds the leaf
// capacity, so a level has fewer than `per` split nodes; a level's node
// list takes children of the level before (2 per split) and grandchildren of
// fused nodes two levels before (4 per split); a fused node emits at most
// kMaxCuts/2 cycles.  Cell tiles (Plan::cells) add up to one tile per leaf.
void size_caps(Plan *pl) {
    const int64_t per = pl->total / std::max<int64_t>(pl->leaf_cap, 1) + 1;
    pl->cap_nodes = std::max<int64_t>(pl->n_inst, 6 * per) + 16;
    pl->cap_rot = pl->cap_nodes + 20 * per + 16;
    pl->cap_leaves = pl->n_inst + 6 * (int64_t)pl->max_levels * per + 16;
    pl->cap_tiles = pl->total / pl->tile + (pl->cells ? 2 : 1) * pl->cap_leaves + 16;
    pl->leaf_shift = leaf_shift(*pl);
}

// Sizes and derived limits of one pipeline run.
bool make_plan(DevState *ds, int ek, int ev, int64_t n_inst, int64_t total, int64_t max_inst,
               int cfg, Plan *pl) {
    const int vi = val_index(ev), ki = key_index(ek);
    if (ds->grid[cfg][ki][vi] == 0) ds->grid[cfg][ki][vi] = leaf_grid(ek, ev, cfg);
    int G = ds->grid[cfg][ki][vi];
    if (G <= 0) return false;
    // test hook: a smaller persistent grid (more slots per workgroup, so the
    // read-ahead and the waits of the leaf merge are exercised on small inputs)
    if (const char *g_env = std::getenv("IM_LEAF_GRID")) {
        long v = std::strtol(g_env, nullptr, 10);
        if (v >= 1 && v < G) G = (int)v;
    }
    int th, ipt, depth;
    size_t lds;
    leaf_geometry(ek, ev, cfg, &th, &ipt, &depth, &lds);
    pl->cfg = cfg;
    // Every workgroup of the leaf merge reads `depth` tiles ahead of its
    // oldest unstored one (im_leaf.hip), so readers less than depth*G slots
    // ahead never block: a leaf may have depth*G tiles.  (Measured: the full
    // capacity beats one with a round of slack on balanced and skewed
    // merges.)  IM_LEAF_TILES (tests, tuning) sets any capacity from 1 to
    // depth*G tiles.
    int64_t tiles_per_leaf = (int64_t)depth * G;
    if (const char *cap_env = std::getenv("IM_LEAF_TILES")) {
        long v = std::strtol(cap_env, nullptr, 10);
        if (v >= 1 && v <= (int64_t)depth * G) tiles_per_leaf = v;
    }
    pl->n_inst = n_inst;
    pl->total = total;
    pl->tile = (int64_t)th * ipt;
    pl->leaf_cap = tiles_per_leaf * pl->tile;
    // A leaf may be larger still when its smaller part keeps every element
    // within tiles_per_leaf-2 tiles of its source (im_leaf.hip, slot order).
    pl->leaf_span = (tiles_per_leaf > 2 ? tiles_per_leaf - 2 : 0) * pl->tile;
    pl->grid_leaf = G;
    if (max_inst <= 0 || max_inst > total) max_inst = total;
    const int lv = division_levels(*pl, max_inst);
    pl->max_levels = lv;
    pl->split_method = kSplitCorank;
    pl->rot_method = kRotSwapRev;
    pl->cap_stash = 2 * (total / kCsSeg) + 16;
    // Two division levels are fused into one exchange where the splits are
    // symmetric (k_split); the rotation kernel cycles up to kMaxCyc pieces
    // only for elements of at most 12 bytes.  IM_FUSE=0 turns it off.
    const char *fz = std::getenv("IM_FUSE");
    pl->fuse = (ek + ev <= 12 && !(fz && fz[0] == '0')) ? 1 : 0;
    pl->leaf_shift = 0;
    pl->row_stride = 0;
    pl->rot_scale = 1;
    pl->sort_width = 0;
    pl->cells = 0;
    size_caps(pl);
    return true;
}

// Cell-aligned tiles whose co-ranks are found beside the first division
// level (im_split.hip, k_split), for a single instance of packed keys with
// exact co-rank splits, whose leaves are then the stable merge's own output
// ranges.  A leaf of S elements meets up to ceil(S/tile) + 1 cells, so the
// size bound of a leaf drops by one tile to keep every leaf within the
// read-ahead of the leaf merge; the tile bound grows by one per leaf.
// (Called for a single instance only: its size is the plan's total.)
void set_cells(Plan &pl, bool eligible) {
    pl.cells = (eligible && pl.leaf_cap >= 3 * pl.tile) ? 1 : 0;
    if (pl.cells) {
        pl.leaf_cap -= pl.tile;
        pl.max_levels = division_levels(pl, pl.total);
        size_caps(&pl);
    }
}

// Plan of a rows merge: the same division (keys read row_bytes apart,
// exchanges in 4-byte units), leaves merged by k_leafrows: tiles of R rows,
// depth tiles held per workgroup (2 or 3 by row kind), so a leaf may have
// depth x G tiles.
bool make_plan_rows(DevState *ds, int key_dt, int64_t row_bytes, int kind, int64_t total,
                    Plan *pl) {
    if (kind < 0 || kind >= rows_kinds()) return false;
    int &gc = ds->rows_grid[key_dt][kind];
    if (gc == 0) gc = rows_grid(key_dt, kind);
    int G = gc;
    const int R = rows_tile(row_bytes, kind);
    if (G <= 0 || R < 1) return false;
    if (const char *g_env = std::getenv("IM_LEAF_GRID")) {
        long v = std::strtol(g_env, nullptr, 10);
        if (v >= 1 && v < G) G = (int)v;
    }
    const int64_t depth = rows_depth(kind);
    int64_t tiles_per_leaf = depth * G;
    if (const char *cap_env = std::getenv("IM_LEAF_TILES")) {
        long v = std::strtol(cap_env, nullptr, 10);
        if (v >= 1 && v <= depth * G) tiles_per_leaf = v;
    }
    pl->cfg = 0;
    pl->n_inst = 1;
    pl->total = total;
    pl->tile = R;
    pl->leaf_cap = tiles_per_leaf * R;
    pl->leaf_span = (tiles_per_leaf > 2 ? tiles_per_leaf - 2 : 0) * R;
    pl->grid_leaf = G;
    const double stop = (double)std::max<int64_t>(pl->leaf_cap, 2 * pl->leaf_span);
    int lv = 1;
    double sz = (double)total;
    while (sz > stop && lv < kMaxLevels) {
        sz = sz * 9.0 / 16.0 + 1.0;
        ++lv;
    }
    pl->max_levels = lv;
    pl->split_method = kSplitCorank;
    pl->rot_method = kRotSwapRev;
    pl->cap_stash = 16;
    const char *fz = std::getenv("IM_FUSE");
    pl->fuse = (fz && fz[0] == '0') ? 0 : 1;   // exchanges move 4-byte units
    pl->leaf_shift = 0;
    pl->row_stride = row_bytes / key_size(key_dt);
    pl->rot_scale = row_bytes / 4;
    pl->sort_width = 0;
    int64_t per = total / std::max<int64_t>(pl->leaf_cap, 1) + 1;
    pl->cap_nodes = std::max<int64_t>(1, 6 * per) + 16;
    pl->cap_rot = pl->cap_nodes + 20 * per + 16;
    pl->cap_leaves = 1 + 6 * (int64_t)lv * per + 16;
    pl->cap_tiles = total / pl->tile + pl->cap_leaves + 16;
    pl->leaf_shift = leaf_shift(*pl);
    return true;
}

size_t carve(const Plan &pl, int64_t flag_slots, void *base, Work *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? (char *)base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    Work x;
    x.ctr = (Counters *)take(sizeof(Counters));
    x.tile_flag = (unsigned *)take(sizeof(unsigned) * std::max<int64_t>(flag_slots, pl.cap_tiles));
    x.nodes[0] = (Node *)take(sizeof(Node) * pl.cap_nodes);
    x.nodes[1] = (Node *)take(sizeof(Node) * pl.cap_nodes);
    x.nodes[2] = (Node *)take(sizeof(Node) * pl.cap_nodes);
    x.rot = (Rot *)take(sizeof(Rot) * pl.cap_rot);
    x.leaves = (Leaf *)take(sizeof(Leaf) * pl.cap_leaves);
    x.tile_start = (int64_t *)take(sizeof(int64_t) * pl.cap_leaves);
    x.tile_rank = (int64_t *)take(sizeof(int64_t) * pl.cap_tiles);
    x.tile_leaf = (int32_t *)take(sizeof(int32_t) * pl.cap_tiles);
    x.tile_geo = (TileGeo *)take(sizeof(TileGeo) * pl.cap_tiles);
    x.cell_rank = pl.cells ? (int64_t *)take(sizeof(int64_t) * (pl.total / pl.tile + 2)) : nullptr;
    x.offsets1 = (int64_t *)take(sizeof(int64_t) * 4);
    x.cs_stash_k = nullptr;
    x.cs_stash_v = nullptr;
    x.sort_off = pl.sort_width > 0 ? (int64_t *)take(sizeof(int64_t) * (2 * pl.n_inst + 1))
                                   : nullptr;
    x.host_err = nullptr;
    if (pl.rot_method == kRotCS) {
        x.cs_stash_k = take((size_t)8 * pl.cap_stash);
        x.cs_stash_v = take((size_t)8 * pl.cap_stash);
    }
    if (w) *w = x;
    return off;
}

int acquire_ws(DevState *ds, size_t need, void **out) {
    // IM_FAULT=alloc simulates a failed workspace allocation (tests of the
    // error path); it applies whether or not the workspace must grow.
    if (std::getenv("IM_FAULT") && std::strcmp(std::getenv("IM_FAULT"), "alloc") == 0)
        return fail(IM_ERR_WORKSPACE, "workspace allocation failed (injected)");
    if (ds->user_ws) {
        if (ds->user_bytes < need)
            return fail(IM_ERR_WORKSPACE, "workspace set by the caller is too small: need " +
                                              std::to_string(need) + " bytes");
        *out = ds->user_ws;
        return IM_OK;
    }
    if (ds->ws_bytes < need) {
        if (ds->ws) {
            // earlier enqueued work may still use it
            if (hipDeviceSynchronize() != hipSuccess) return fail(IM_ERR_HIP, "sync before realloc");
            (void)hipFree(ds->ws);
            ds->ws = nullptr;
            ds->ws_bytes = 0;
        }
        size_t bytes = std::max(need, (size_t)1 << 20);
        if (hipMalloc(&ds->ws, bytes) != hipSuccess) {
            ds->ws = nullptr;
            return fail(IM_ERR_WORKSPACE, "workspace allocation of " + std::to_string(bytes) +
                                              " bytes failed");
        }
        ds->ws_bytes = bytes;
        ds->flag_cap = 0;          // new memory: no flag is known to be clear
    }
    *out = ds->ws;
    return IM_OK;
}

// The host word of the device's error bits (allocated once; null if pinned
// memory is unavailable, and errors then reach the host only through the
// counters).
void ensure_err_word(DevState *ds) {
    if (ds->err_tried) return;
    ds->err_tried = true;
    void *h = nullptr;
    if (hipHostMalloc(&h, 256, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(h);
        return;
    }
    std::memset(h, 0, 256);
    ds->h_err = (unsigned *)h;
    ds->d_err = (unsigned *)d;
}

// This device's address of `scratch` (looked up on the device's first
// allocation-free call, with the device current and its lock held).
int scratch_base(DevState *ds, void **out) {
    if (!ds->scr_ptr) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "address of the static scratch array");
        if (p == nullptr) return fail(IM_ERR_HIP, "null address of the static scratch array");
        ds->scr_ptr = p;
    }
    *out = ds->scr_ptr;
    return IM_OK;
}

bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

// Order this call after the previous use of the shared workspace (other
// streams) and record this use.
int ws_enter(DevState *ds, hipStream_t s) {
    if (ds->done == nullptr) {
        if (hipEventCreateWithFlags(&ds->done, hipEventDisableTiming) != hipSuccess)
            return fail(IM_ERR_HIP, "event create");
    }
    if (ds->done_valid && !stream_capturing(s)) IM_HIP(hipStreamWaitEvent(s, ds->done, 0), "stream wait");
    return IM_OK;
}

int ws_leave(DevState *ds, hipStream_t s) {
    if (!stream_capturing(s)) {
        IM_HIP(hipEventRecord(ds->done, s), "event record");
        ds->done_valid = true;
    }
    return IM_OK;
}

int read_error_bits(Counters *ctr, hipStream_t s, unsigned *bits) {
    IM_HIP(hipStreamSynchronize(s), "synchronise (checked mode)");
    unsigned v = 0;
    IM_HIP(hipMemcpy(&v, &ctr->error, sizeof(v), hipMemcpyDeviceToHost), "read error flag");
    *bits = v;
    return IM_OK;
}

// Everything up to the leaf merge: counters and roots, division levels
// (which also lay the leaves out in tiles), tile co-ranks and dependencies.
// `offs` is the caller's offsets or null for a single pair (la, lb).
int enqueue_division(int key_dt, int ev, void *keys, void *vals, const int64_t *d_offsets,
                     int64_t n_inst, int64_t la, int64_t lb, const MlpDev *mlp, const Plan &pl,
                     const Work &w, bool check, bool prof, hipStream_t s) {
    // rows are exchanged as 4-byte units (the descriptors are scaled)
    const int ek = pl.row_stride > 0 ? 4 : key_size(key_dt);
    IM_HIP(launch_init(pl, w, d_offsets, la, lb, s), "launch init");
    const int64_t *offs = d_offsets ? d_offsets : w.offsets1;
    if (check) {
        IM_HIP(launch_check_sorted(key_dt, keys, offs, n_inst, w.ctr,
                                   pl.row_stride > 0 ? pl.row_stride : 1, s),
               "launch check");
        unsigned bits = 0;
        int rc = read_error_bits(w.ctr, s, &bits);
        if (rc) return rc;
        if (bits & kErrOffsets) return fail(IM_ERR_INVALID_ARG, "offsets are not monotone");
        if (bits & kErrNotSorted) return fail(IM_ERR_NOT_SORTED, "an input run is not ascending");
    }
    // A single pair with L_A == L_B splits at the symmetric diagonal (or is
    // one exchange of two equal parts): the first level has block swaps or
    // cycles only, never the second pass of three reversals.
    const bool equal_root = n_inst == 1 && d_offsets == nullptr && la == lb &&
                            pl.split_method == kSplitCorank && pl.rot_method == kRotSwapRev;
    for (int lv = 0; lv < pl.max_levels; ++lv) {
        hipEvent_t e0 = prof ? prof_begin(s) : nullptr;
        IM_HIP(launch_split(key_dt, keys, offs, pl, w, lv, mlp, s), "launch split");
        prof_end(e0, kStSplit, 1, s);
        if (lv + 1 == pl.max_levels) break;   // the last level only classifies
        hipEvent_t e1 = prof ? prof_begin(s) : nullptr;
        IM_HIP(launch_rotate(ek, ev, keys, vals, pl, w, lv, 0, s), "launch rotate A");
        const bool phase_b = !(lv == 0 && equal_root);
        if (phase_b)
            IM_HIP(launch_rotate(ek, ev, keys, vals, pl, w, lv, 1, s), "launch rotate B");
        prof_end(e1, kStRotate, phase_b ? 2 : 1, s);
    }
    hipEvent_t e3 = prof ? prof_begin(s) : nullptr;
    if (!pl.cells)
        IM_HIP(launch_tilerank(key_dt, keys, offs, pl, w, mlp, s), "launch tile co-rank");
    IM_HIP(launch_tiledeps(pl, w, s), "launch tile dependencies");
    prof_end(e3, kStTileRank, pl.cells ? 1 : 2, s);
    return IM_OK;
}

void record_stats(const Plan &pl, const Work &w) {
    g_stats = im_stats{};
    g_stats.leaf_capacity = pl.leaf_cap;
    g_stats.tile = pl.tile;
    g_stats.max_levels = pl.max_levels;
    g_stats.leaf_config = pl.cfg;
    g_stats.leaf_grid = pl.grid_leaf;
    g_last_ctr = w.ctr;
}

// The whole merge: division levels, tile co-ranks, leaf merge.
// cfg_override >= 0 forces a leaf configuration (autotuner).
// Rows mode of run_pipeline: row bytes (0: packed keys) and row kind.
struct RowsArg {
    int64_t bytes;
    int kind;
};

// sort_width > 0: a merge-sort pass over runs of that width (its offsets are
// written into the workspace, in stream order after the workspace's earlier
// users; d_offsets is then ignored).
int run_pipeline(int key_dt, int ev, void *keys, void *vals, const int64_t *d_offsets,
                 int64_t n_inst, int64_t total, int64_t max_inst, int64_t la, int64_t lb,
                 const MlpDev *mlp, hipStream_t s, int cfg_override = -1,
                 int split_method = kSplitCorank, int rot_method = kRotSwapRev,
                 RowsArg rows = RowsArg{0, 0}, int64_t sort_width = 0,
                 bool static_scratch = false) {
    int dev = 0;
    DevState *ds = dev_state(&dev);
    if (!ds) return fail(IM_ERR_HIP, "no current HIP device");
    // A captured call would bake this call's epoch and workspace into the
    // graph: later replays would find every tile flag already set.  Graphs
    // are recorded by batched_inplace_merge_graph, which owns its workspace.
    if (stream_capturing(s))
        return fail(IM_ERR_INVALID_ARG, "the stream is capturing a graph: record the merge "
                                        "with batched_inplace_merge_graph instead");
    std::lock_guard<std::mutex> lock(ds->mu);
    if (!static_scratch) ensure_err_word(ds);    // (pinned host memory: an allocation)
    load_tune_cache(ds, dev);
    const int ek = key_size(key_dt);
    Plan pl = {};
    if (rows.bytes > 0) {
        if (!make_plan_rows(ds, key_dt, rows.bytes, rows.kind, total, &pl))
            return fail(IM_ERR_HIP, "could not size the rows leaf merge grid");
    } else {
        const int cfg = choose_cfg(ds, ek, ev, n_inst, total, cfg_override);
        if (!make_plan(ds, ek, ev, n_inst, total, max_inst, cfg, &pl))
            return fail(IM_ERR_HIP, "could not size the leaf merge grid (occupancy query failed)");
    }
    pl.split_method = split_method;
    pl.rot_method = rot_method;
    pl.sort_width = sort_width;
    if (split_method != kSplitCorank || rot_method != kRotSwapRev) pl.fuse = 0;   // the paper's modes as such
    set_cells(pl, n_inst == 1 && rows.bytes == 0 && sort_width == 0 &&
                      split_method == kSplitCorank);
    if (pl.leaf_shift == 0)
        return fail(IM_ERR_INVALID_ARG, "too many instances for the 64-bit leaf/tile counter");
    int64_t &flag_cap = static_scratch ? ds->scr_flag_cap : ds->flag_cap;
    uint32_t &epoch = static_scratch ? ds->scr_epoch : ds->epoch;
    size_t need = carve(pl, flag_cap, nullptr, nullptr);
    void *base = nullptr;
    int rc = IM_OK;
    if (static_scratch) {
        // the flag region only grows, so a plan that fits now fits with it
        if (carve(pl, pl.cap_tiles, nullptr, nullptr) > kScratchBytes || need > kScratchBytes)
            return fail(IM_ERR_WORKSPACE, "this merge needs " +
                                              std::to_string(std::max(need, carve(pl, pl.cap_tiles,
                                                                                  nullptr, nullptr))) +
                                              " bytes of workspace; the static scratch holds " +
                                              std::to_string(kScratchBytes));
        rc = scratch_base(ds, &base);
        if (rc) return rc;
    } else {
        rc = acquire_ws(ds, need, &base);
        if (rc) return rc;
        if (carve(pl, flag_cap, nullptr, nullptr) > need) {
            // the buffer was replaced (flag_cap reset): size again
            need = carve(pl, flag_cap, nullptr, nullptr);
            rc = acquire_ws(ds, need, &base);
            if (rc) return rc;
        }
    }
    Work w;
    carve(pl, flag_cap, base, &w);
    w.host_err = ds->d_err;
    if (!static_scratch) {
        // the static scratch is private to the allocation-free calls (they
        // race with each other by contract), so only the shared workspace
        // is ordered across streams
        rc = ws_enter(ds, s);
        if (rc) return rc;
    }
    if (sort_width > 0) {
        IM_HIP(launch_pass_offsets(total, sort_width, w.sort_off, n_inst, s), "launch pass offsets");
        d_offsets = w.sort_off;
    }
    // Tile flags: a tile is "read" when its flag equals this call's epoch.
    // Flags beyond flag_cap may hold stale data of other arrays, so they are
    // cleared (with a kernel: graph-capture safe) before first use.
    if (pl.cap_tiles > flag_cap || epoch == 0xFFFFFFFFu) {
        int64_t nflags = std::max<int64_t>(flag_cap, pl.cap_tiles);
        IM_HIP(launch_fill32(w.tile_flag, nflags, 0u, s), "clear tile flags");
        flag_cap = nflags;
        if (epoch == 0xFFFFFFFFu) epoch = 0;
    }
    pl.epoch = ++epoch;

    const bool check = checked_mode();
    if (std::getenv("IM_FAULT") && std::strcmp(std::getenv("IM_FAULT"), "launch") == 0)
        return fail(IM_ERR_HIP, "kernel launch failed (injected)");
    const bool prof = g_prof && !static_scratch;    // (events are created lazily)
    // A single small pair: one launch (im_leaf.hip, k_smallmerge) when it has
    // at most a quarter of the resident tiles.  Not in checked mode, for the
    // paper's split and exchange modes, for the learned split (its searches
    // are the point there), or under the test hooks that force division
    // levels or a small grid; IM_SMALL=0 turns it off.
    const char *sm = std::getenv("IM_SMALL");
    const bool small = !(sm && sm[0] == '0') && n_inst == 1 && d_offsets == nullptr &&
                       rows.bytes == 0 && mlp == nullptr && sort_width == 0 && !check &&
                       split_method == kSplitCorank && rot_method == kRotSwapRev && pl.cfg == 0 &&
                       !std::getenv("IM_LEAF_TILES") && !std::getenv("IM_LEAF_GRID") &&
                       (total + pl.tile - 1) / pl.tile <= pl.grid_leaf / 4;
    if (small) {
        hipEvent_t e4 = prof ? prof_begin(s) : nullptr;
        IM_HIP(launch_smallmerge(key_dt, ev, keys, vals, la, lb, pl, w, s), "launch small merge");
        prof_end(e4, kStLeafMerge, 1, s);
    } else {
        rc = enqueue_division(key_dt, ev, keys, vals, d_offsets, n_inst, la, lb, mlp, pl, w, check,
                              prof, s);
        if (rc) return rc;
        hipEvent_t e4 = prof ? prof_begin(s) : nullptr;
        if (rows.bytes > 0)
            IM_HIP(launch_leafrows(key_dt, rows.kind, keys, rows.bytes, pl, w, s), "launch rows merge");
        else
            IM_HIP(launch_leafmerge(key_dt, ev, keys, vals, pl, w, s), "launch leaf merge");
        prof_end(e4, kStLeafMerge, 1, s);
    }
    if (!static_scratch) {
        rc = ws_leave(ds, s);
        if (rc) return rc;
    }

    record_stats(pl, w);
    g_last_stream = s;
    if (log_level() >= 1)
        std::fprintf(stderr,
                     "[inplace_merge] dev %d: %lld instance(s), %lld elements, key %d B, payload "
                     "%d B%s; leaf config %d (tile %lld, grid %d), leaf capacity %lld, span %lld, "
                     "%d level(s) enqueued, fusion %s, workspace %zu B%s%s\n",
                     dev, (long long)n_inst, (long long)total, ek, ev,
                     rows.bytes > 0 ? " (rows)" : "", pl.cfg, (long long)pl.tile, pl.grid_leaf,
                     (long long)pl.leaf_cap, (long long)pl.leaf_span, pl.max_levels,
                     pl.fuse ? "on" : "off", need, static_scratch ? " (static scratch)" : "",
                     small ? ", one launch" : "");
    if (check) {
        unsigned bits = 0;
        rc = read_error_bits(w.ctr, s, &bits);
        if (rc) return rc;
        if (bits) return fail(IM_ERR_DEVICE, "device-side check failed, error bits " +
                                                 std::to_string(bits));
    }
    return IM_OK;
}

int check_common(const void *p, int64_t la, int64_t lb, int dt) {
    if (!valid_dtype(dt)) return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported key dtype");
    if (la < 0 || lb < 0) return fail(IM_ERR_INVALID_ARG, "negative run length");
    if (la + lb > 0 && p == nullptr) return fail(IM_ERR_INVALID_ARG, "null data pointer");
    if (la > (int64_t(1) << 46) || lb > (int64_t(1) << 46))
        return fail(IM_ERR_INVALID_ARG, "run length too large");
    return IM_OK;
}

}  // namespace

// Captured batched merge: the executable graph and its private workspace.
struct im_graph {
    int device = 0;
    Plan plan = {};
    void *ws = nullptr;
    size_t ws_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool coop = false;
};

// ---------------------------------------------------------------------------
// Learned model object.
// ---------------------------------------------------------------------------
struct merge_model {
    int device = 0;
    MlpDev *d = nullptr;       // device copy used by the kernels
    float *d_m = nullptr;      // Adam moments
    float *d_v = nullptr;
    float host[kMlpParams] = {};
    float err_scale = 1.0f;
    float err_b[kErrBuckets];    // bracket half-widths (kErrUnknown: untrained)
    merge_model() {
        for (float &v : err_b) v = kErrUnknown;
    }
};

static uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int model_upload(merge_model *m) {
    MlpDev h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.p, m->host, sizeof(m->host));
    h.err_scale = m->err_scale;
    std::memcpy(h.err_b, m->err_b, sizeof(m->err_b));
    IM_HIP(hipMemcpy(m->d, &h, sizeof(h), hipMemcpyHostToDevice), "model upload");
    return IM_OK;
}

extern "C" {

const char *inplace_merge_last_error(void) { return g_err.c_str(); }

int inplace_merge(void *data, int64_t L_A, int64_t L_B, int dtype, hipStream_t stream) {
    int rc = check_common(data, L_A, L_B, dtype);
    if (rc) return rc;
    if (L_A == 0 || L_B == 0) { g_err.clear(); return IM_OK; }
    return run_pipeline(dtype, 0, data, nullptr, nullptr, 1, L_A + L_B, L_A + L_B, L_A, L_B,
                        nullptr, stream);
}

int inplace_merge_noalloc(void *data, int64_t L_A, int64_t L_B, int dtype, hipStream_t stream) {
    int rc = check_common(data, L_A, L_B, dtype);
    if (rc) return rc;
    if (L_A == 0 || L_B == 0) { g_err.clear(); return IM_OK; }
    return run_pipeline(dtype, 0, data, nullptr, nullptr, 1, L_A + L_B, L_A + L_B, L_A, L_B,
                        nullptr, stream, -1, kSplitCorank, kRotSwapRev, RowsArg{0, 0}, 0, true);
}

int inplace_merge_kv(void *keys, void *vals, int64_t L_A, int64_t L_B, int key_dtype,
                     int val_dtype, hipStream_t stream) {
    int rc = check_common(keys, L_A, L_B, key_dtype);
    if (rc) return rc;
    if (!valid_dtype(val_dtype)) return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported payload dtype");
    if (L_A + L_B > 0 && vals == nullptr) return fail(IM_ERR_INVALID_ARG, "null payload pointer");
    if (L_A == 0 || L_B == 0) { g_err.clear(); return IM_OK; }
    return run_pipeline(key_dtype, key_size(val_dtype), keys, vals, nullptr, 1, L_A + L_B,
                        L_A + L_B, L_A, L_B, nullptr, stream);
}

// Row kind of a rows merge, -1 (with *why) if the rows cannot be merged:
// the widest chunk that divides the row and the address and still puts a
// whole row in a tile; of the 16-byte kinds, the one whose workgroup holds
// more bytes of whole rows (depth x rows per tile x row bytes).
static int rows_kind(const void *data, int64_t row_bytes, int key_dtype, const char **why) {
    const int kb = key_size(key_dtype);
    if (row_bytes < kb || row_bytes % kb != 0 || row_bytes % 4 != 0) {
        *why = "row bytes must be a positive multiple of the key size and of 4";
        return -1;
    }
    const uintptr_t a = (uintptr_t)data;
    if (a % (uintptr_t)kb != 0) {
        *why = "data must be aligned to the key size";
        return -1;
    }
    int best = -1, best_ch = 0;
    int64_t best_hold = 0;
    for (int k = 0; k < rows_kinds(); ++k) {
        const int ch = rows_chunk_bytes(k);
        const int R = rows_tile(row_bytes, k);
        if (R < 1 || row_bytes % ch != 0 || a % (uintptr_t)ch != 0) continue;
        const int64_t hold = (int64_t)rows_depth(k) * R * row_bytes;
        if (ch > best_ch || (ch == best_ch && hold > best_hold)) {
            best = k;
            best_ch = ch;
            best_hold = hold;
        }
    }
    if (best < 0) *why = "row too large: at most 81920 bytes";
    return best;
}

int inplace_merge_rows(void *data, int64_t L_A, int64_t L_B, int64_t row_bytes, int key_dtype,
                       hipStream_t stream) {
    int rc = check_common(data, L_A, L_B, key_dtype);
    if (rc) return rc;
    if (row_bytes <= 0) return fail(IM_ERR_INVALID_ARG, "row bytes must be positive");
    if (L_A + L_B > 0 && (L_A + L_B) > (int64_t(1) << 46) / row_bytes)
        return fail(IM_ERR_INVALID_ARG, "array too large");
    if (L_A == 0 || L_B == 0) { g_err.clear(); return IM_OK; }
    const char *why = "";
    const int kind = rows_kind(data, row_bytes, key_dtype, &why);
    if (kind < 0) return fail(IM_ERR_INVALID_ARG, why);
    return run_pipeline(key_dtype, 0, data, nullptr, nullptr, 1, L_A + L_B, L_A + L_B, L_A, L_B,
                        nullptr, stream, -1, kSplitCorank, kRotSwapRev, RowsArg{row_bytes, kind});
}

size_t inplace_merge_rows_workspace_bytes(int64_t rows, int64_t row_bytes, int key_dtype) {
    if (!valid_dtype(key_dtype) || rows < 0 || row_bytes <= 0) return 0;
    DevState *ds = dev_state(nullptr);
    if (!ds) return 0;
    std::lock_guard<std::mutex> lock(ds->mu);
    size_t need = 0;
    for (int k = 0; k < rows_kinds(); ++k) {
        if (row_bytes % rows_chunk_bytes(k) != 0 || rows_tile(row_bytes, k) < 1) continue;
        Plan pl = {};
        if (!make_plan_rows(ds, key_dtype, row_bytes, k, std::max<int64_t>(rows, 1), &pl))
            return 0;
        need = std::max(need, carve(pl, 0, nullptr, nullptr));
    }
    return need;
}

int batched_inplace_merge_sized(void *data, const int64_t *d_offsets, int64_t n,
                                int64_t total_elems, int64_t max_instance, int dtype,
                                hipStream_t stream) {
    if (!valid_dtype(dtype)) return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported key dtype");
    if (n < 0 || total_elems < 0 || max_instance < 0)
        return fail(IM_ERR_INVALID_ARG, "negative count");
    if (n == 0 || total_elems == 0) { g_err.clear(); return IM_OK; }
    if (data == nullptr || d_offsets == nullptr) return fail(IM_ERR_INVALID_ARG, "null pointer");
    if (n >= (int64_t(1) << 31)) return fail(IM_ERR_INVALID_ARG, "too many instances");
    return run_pipeline(dtype, 0, data, nullptr, d_offsets, n, total_elems, max_instance, 0, 0,
                        nullptr, stream);
}

int batched_inplace_merge_kv_sized(void *keys, void *vals, const int64_t *d_offsets, int64_t n,
                                   int64_t total_elems, int64_t max_instance, int key_dtype,
                                   int val_dtype, hipStream_t stream) {
    if (!valid_dtype(key_dtype)) return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported key dtype");
    if (!valid_dtype(val_dtype)) return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported payload dtype");
    if (n < 0 || total_elems < 0 || max_instance < 0)
        return fail(IM_ERR_INVALID_ARG, "negative count");
    if (n == 0 || total_elems == 0) { g_err.clear(); return IM_OK; }
    if (keys == nullptr || vals == nullptr || d_offsets == nullptr)
        return fail(IM_ERR_INVALID_ARG, "null pointer");
    if (n >= (int64_t(1) << 31)) return fail(IM_ERR_INVALID_ARG, "too many instances");
    return run_pipeline(key_dtype, key_size(val_dtype), keys, vals, d_offsets, n, total_elems,
                        max_instance, 0, 0, nullptr, stream);
}

// The offsets-only forms read the total d_offsets[2n] back to size the
// workspace (one 8-byte copy on the stream, then a synchronisation).
static int read_total(const int64_t *d_offsets, int64_t n, hipStream_t stream, int64_t *total) {
    if (stream_capturing(stream))
        return fail(IM_ERR_INVALID_ARG, "the stream is capturing a graph: use the _sized form "
                                        "through batched_inplace_merge_graph");
    int64_t v = 0;
    IM_HIP(hipMemcpyAsync(&v, d_offsets + 2 * n, sizeof(v), hipMemcpyDeviceToHost, stream),
           "read the offsets' total");
    IM_HIP(hipStreamSynchronize(stream), "read the offsets' total");
    if (v < 0 || v > (int64_t(1) << 46)) return fail(IM_ERR_INVALID_ARG, "offsets' total out of range");
    *total = v;
    return IM_OK;
}

int batched_inplace_merge(void *data, const int64_t *d_offsets, int64_t n, int dtype,
                          hipStream_t stream) {
    if (!valid_dtype(dtype)) return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported key dtype");
    if (n < 0) return fail(IM_ERR_INVALID_ARG, "negative count");
    if (n == 0) { g_err.clear(); return IM_OK; }
    if (data == nullptr || d_offsets == nullptr) return fail(IM_ERR_INVALID_ARG, "null pointer");
    if (n >= (int64_t(1) << 31)) return fail(IM_ERR_INVALID_ARG, "too many instances");
    int64_t total = 0;
    int rc = read_total(d_offsets, n, stream, &total);
    if (rc) return rc;
    return batched_inplace_merge_sized(data, d_offsets, n, total, 0, dtype, stream);
}

int batched_inplace_merge_kv(void *keys, void *vals, const int64_t *d_offsets, int64_t n,
                             int key_dtype, int val_dtype, hipStream_t stream) {
    if (!valid_dtype(key_dtype)) return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported key dtype");
    if (!valid_dtype(val_dtype)) return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported payload dtype");
    if (n < 0) return fail(IM_ERR_INVALID_ARG, "negative count");
    if (n == 0) { g_err.clear(); return IM_OK; }
    if (keys == nullptr || vals == nullptr || d_offsets == nullptr)
        return fail(IM_ERR_INVALID_ARG, "null pointer");
    if (n >= (int64_t(1) << 31)) return fail(IM_ERR_INVALID_ARG, "too many instances");
    int64_t total = 0;
    int rc = read_total(d_offsets, n, stream, &total);
    if (rc) return rc;
    return batched_inplace_merge_kv_sized(keys, vals, d_offsets, n, total, 0, key_dtype,
                                          val_dtype, stream);
}

int inplace_merge_sort(void *data, int64_t n, int dtype, hipStream_t stream) {
    if (!valid_dtype(dtype)) return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported key dtype");
    if (n < 0) return fail(IM_ERR_INVALID_ARG, "negative length");
    if (n <= 1) { g_err.clear(); return IM_OK; }
    if (data == nullptr) return fail(IM_ERR_INVALID_ARG, "null data pointer");
    if (n > (int64_t(1) << 46)) return fail(IM_ERR_INVALID_ARG, "length too large");
    if (stream_capturing(stream))
        return fail(IM_ERR_INVALID_ARG, "the stream is capturing a graph");
    const int64_t tile = sort_tile_elems(key_size(dtype));
    IM_HIP(launch_tilesort(dtype, data, n, stream), "launch tile sort");
    // each pass writes its offsets into the shared workspace, after the
    // workspace's earlier users on other streams (inside run_pipeline)
    for (int64_t w = tile; w < n; w *= 2) {
        const int64_t ni = (n + 2 * w - 1) / (2 * w);
        int rc = run_pipeline(dtype, 0, data, nullptr, nullptr, ni, n, std::min(n, 2 * w), 0, 0,
                              nullptr, stream, -1, kSplitCorank, kRotSwapRev, RowsArg{0, 0}, w);
        if (rc) return rc;
    }
    return IM_OK;
}

size_t inplace_merge_workspace_bytes_batched(int64_t total_elems, int64_t n_inst, int dtype) {
    if (!valid_dtype(dtype) || total_elems < 0 || n_inst < 0) return 0;
    DevState *ds = dev_state(nullptr);
    if (!ds) return 0;
    std::lock_guard<std::mutex> lock(ds->mu);
    // the largest need over payload sizes and leaf configurations
    size_t need = 0;
    for (int cfg = 0; cfg < kLeafCfgs; ++cfg) {
        for (int ev : {0, 4, 8}) {
            Plan pl = {};
            if (!make_plan(ds, key_size(dtype), ev, std::max<int64_t>(n_inst, 1),
                           std::max<int64_t>(total_elems, 1), 0, cfg, &pl))
                return 0;
            need = std::max(need, carve(pl, 0, nullptr, nullptr));
            if (n_inst <= 1) {           // a single pair may run with cell tiles
                set_cells(pl, true);
                need = std::max(need, carve(pl, 0, nullptr, nullptr));
            }
        }
    }
    return need;
}

size_t inplace_merge_workspace_bytes(int64_t N, int dtype) {
    if (!valid_dtype(dtype) || N < 0) return 0;
    // one pair, or the first (widest in instances) pass of a sort of N
    size_t need = inplace_merge_workspace_bytes_batched(N, 1, dtype);
    const int64_t tile = sort_tile_elems(key_size(dtype));
    const int64_t ni = std::max<int64_t>((N + 2 * tile - 1) / (2 * tile), 1);
    const size_t sort = inplace_merge_workspace_bytes_batched(N, ni, dtype);
    if (need == 0 || sort == 0) return 0;
    return std::max(need, sort) + align_up(sizeof(int64_t) * (2 * ni + 1));
}

int inplace_merge_set_workspace(void *d_ws, size_t bytes) {
    DevState *ds = dev_state(nullptr);
    if (!ds) return fail(IM_ERR_HIP, "no current HIP device");
    std::lock_guard<std::mutex> lock(ds->mu);
    if (d_ws != nullptr && bytes < 4096) return fail(IM_ERR_WORKSPACE, "workspace too small");
    ds->user_ws = d_ws;
    ds->user_bytes = d_ws ? bytes : 0;
    ds->flag_cap = 0;              // a different buffer: no flag is known clear
    g_err.clear();
    return IM_OK;
}

int inplace_merge_fetch_stats(im_stats *out, hipStream_t stream) {
    if (!out) return fail(IM_ERR_INVALID_ARG, "null output");
    *out = g_stats;
    if (!g_last_ctr) return IM_OK;
    IM_HIP(hipStreamSynchronize(stream), "synchronise for statistics");
    Counters c;
    IM_HIP(hipMemcpy(&c, g_last_ctr, sizeof(c), hipMemcpyDeviceToHost), "read counters");
    out->levels_used = (int32_t)c.levels_used;
    out->leaves = (int64_t)c.leaves;
    out->tiles = (int64_t)c.tiles;
    int64_t nrot = 0;
    for (int l = 0; l < kMaxLevels; ++l) nrot += (int64_t)(c.level_rot[l] >> kRotCountShift);
    out->rotations = nrot;
    out->rotated_elems = (int64_t)c.rotated;
    out->reversed_elems = (int64_t)c.rotated_rev;
    out->leaf_elems = (int64_t)c.leaf_elems;
    out->search_probes = (int64_t)c.probes;
    out->searches = (int64_t)c.searches;
    out->split_fallbacks = (int64_t)c.split_fallbacks;
    out->fused_nodes = (int64_t)c.fused;
    if (c.error) return fail(IM_ERR_DEVICE, "device error bits " + std::to_string(c.error));
    return IM_OK;
}

int inplace_merge_last_stats(merge_stats *out) {
    return inplace_merge_fetch_stats(out, g_last_stream);
}

int inplace_merge_device_status(void) {
    DevState *ds = dev_state(nullptr);
    if (!ds) return fail(IM_ERR_HIP, "no current HIP device");
    if (!ds->h_err) return IM_OK;
    const unsigned bits = __atomic_exchange_n(ds->h_err, 0u, __ATOMIC_ACQ_REL);
    if (bits == 0) return IM_OK;
    return fail(IM_ERR_DEVICE, "an enqueued merge raised device error bit " + std::to_string(bits) +
                                   " (1: a node too large at the last level, 2: a bounded wait "
                                   "gave up, 4: a descriptor array overflowed)");
}

int inplace_merge_profile(int enable) {
    g_prof = enable != 0;
    return IM_OK;
}

int inplace_merge_profile_read(double *ms, int64_t *launches, int nstages, hipStream_t stream) {
    if (!ms || nstages < 0) return fail(IM_ERR_INVALID_ARG, "null output");
    for (int i = 0; i < nstages; ++i) {
        ms[i] = 0.0;
        if (launches) launches[i] = 0;
    }
    if (!g_prof_recs.empty()) IM_HIP(hipStreamSynchronize(stream), "synchronise for profile");
    for (const ProfRec &r : g_prof_recs) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess && r.stage < nstages) {
            ms[r.stage] += t;
            if (launches) launches[r.stage] += r.launches;
        }
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_prof_recs.clear();
    return IM_OK;
}

int im_corank(const void *data, int64_t L_A, int64_t L_B, int dtype, const int64_t *d_k,
              int64_t nk, int64_t *d_out, int32_t *d_probes, hipStream_t stream) {
    int rc = check_common(data, L_A, L_B, dtype);
    if (rc) return rc;
    if (nk < 0) return fail(IM_ERR_INVALID_ARG, "negative count");
    if (nk == 0) return IM_OK;
    if (!d_k || !d_out) return fail(IM_ERR_INVALID_ARG, "null pointer");
    IM_HIP(launch_corank(dtype, data, L_A, L_B, d_k, nk, d_out, nullptr, d_probes, stream),
           "launch co-rank");
    return IM_OK;
}

int im_rotate(void *data, int64_t lx, int64_t ly, int elem_bytes, hipStream_t stream) {
    if (lx < 0 || ly < 0) return fail(IM_ERR_INVALID_ARG, "negative length");
    if (elem_bytes != 4 && elem_bytes != 8) return fail(IM_ERR_UNSUPPORTED_DTYPE, "element size");
    if (lx == 0 || ly == 0) return IM_OK;
    if (!data) return fail(IM_ERR_INVALID_ARG, "null data pointer");
    IM_HIP(launch_rotate_single(data, lx, ly, elem_bytes, stream), "launch rotate");
    return IM_OK;
}

// ---------------------------------------------------------------------------
// Method variants and comparators.
// ---------------------------------------------------------------------------
int inplace_merge_variant(void *data, int64_t L_A, int64_t L_B, int dtype, int split_method,
                          int rot_method, hipStream_t stream) {
    int rc = check_common(data, L_A, L_B, dtype);
    if (rc) return rc;
    if (split_method != IM_SPLIT_CORANK && split_method != IM_SPLIT_FINDMEDIAN)
        return fail(IM_ERR_INVALID_ARG, "unknown split method");
    if (rot_method != IM_ROTATE_SWAP_REV && rot_method != IM_ROTATE_CS)
        return fail(IM_ERR_INVALID_ARG, "unknown exchange method");
    if (L_A == 0 || L_B == 0) { g_err.clear(); return IM_OK; }
    return run_pipeline(dtype, 0, data, nullptr, nullptr, 1, L_A + L_B, L_A + L_B, L_A, L_B,
                        nullptr, stream, -1,
                        split_method == IM_SPLIT_FINDMEDIAN ? kSplitFindMedian : kSplitCorank,
                        rot_method == IM_ROTATE_CS ? kRotCS : kRotSwapRev);
}

int im_divide(const void *data, int64_t L_A, int64_t L_B, int dtype, int method, int depth,
              int64_t *d_sizes, hipStream_t stream) {
    int rc = check_common(data, L_A, L_B, dtype);
    if (rc) return rc;
    if (method != IM_SPLIT_CORANK && method != IM_SPLIT_FINDMEDIAN)
        return fail(IM_ERR_INVALID_ARG, "unknown split method");
    if (depth < 0 || depth > 24) return fail(IM_ERR_INVALID_ARG, "depth outside [0, 24]");
    if (!d_sizes) return fail(IM_ERR_INVALID_ARG, "null output");
    const int64_t leaves = (int64_t)1 << depth;
    int64_t *buf = nullptr;
    IM_HIP(hipMallocAsync((void **)&buf, sizeof(int64_t) * 8 * leaves, stream), "division buffers");
    int64_t *nodes[2] = {buf, buf + 4 * leaves};
    const int64_t root[4] = {0, L_A, 0, L_B};
    hipError_t e = hipMemcpyAsync(nodes[0], root, sizeof(root), hipMemcpyHostToDevice, stream);
    const int m = method == IM_SPLIT_FINDMEDIAN ? kSplitFindMedian : kSplitCorank;
    for (int lv = 0; lv < depth && e == hipSuccess; ++lv)
        e = launch_divide(dtype, data, L_A, L_B, m, lv, nodes[lv & 1], nodes[(lv + 1) & 1], stream);
    // (a_off, la, b_off, lb) per pair -> (la, lb)
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(d_sizes, 2 * sizeof(int64_t), nodes[depth & 1] + 1,
                             4 * sizeof(int64_t), sizeof(int64_t), leaves,
                             hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(d_sizes + 1, 2 * sizeof(int64_t), nodes[depth & 1] + 3,
                             4 * sizeof(int64_t), sizeof(int64_t), leaves,
                             hipMemcpyDeviceToDevice, stream);
    hipError_t ef = hipFreeAsync(buf, stream);
    if (e != hipSuccess) return hip_fail(e, "division");
    if (ef != hipSuccess) return hip_fail(ef, "division buffers");
    return IM_OK;
}

int im_rotate_cs(void *data, int64_t lx, int64_t ly, int elem_bytes, hipStream_t stream) {
    if (lx < 0 || ly < 0) return fail(IM_ERR_INVALID_ARG, "negative length");
    if (elem_bytes != 4 && elem_bytes != 8) return fail(IM_ERR_UNSUPPORTED_DTYPE, "element size");
    if (lx == 0 || ly == 0) return IM_OK;
    if (!data) return fail(IM_ERR_INVALID_ARG, "null data pointer");
    if (lx > (int64_t(1) << 46) || ly > (int64_t(1) << 46))
        return fail(IM_ERR_INVALID_ARG, "length too large");
    const int64_t lanes = cs_lanes(lx, ly);
    void *stash = nullptr;
    IM_HIP(hipMallocAsync(&stash, (size_t)elem_bytes * std::max<int64_t>(lanes, 1), stream),
           "stash allocation");
    hipError_t e = launch_rotate_cs_single(data, lx, ly, elem_bytes, stash, stream);
    hipError_t ef = hipFreeAsync(stash, stream);
    if (e != hipSuccess) return hip_fail(e, "launch circular shifting");
    if (ef != hipSuccess) return hip_fail(ef, "stash free");
    return IM_OK;
}

int im_rotate_ls(void *data, int64_t lx, int64_t ly, int elem_bytes, int64_t *d_swaps,
                 hipStream_t stream) {
    if (lx < 0 || ly < 0) return fail(IM_ERR_INVALID_ARG, "negative length");
    if (elem_bytes != 4 && elem_bytes != 8) return fail(IM_ERR_UNSUPPORTED_DTYPE, "element size");
    if (lx > (int64_t(1) << 46) || ly > (int64_t(1) << 46))
        return fail(IM_ERR_INVALID_ARG, "length too large");
    if (d_swaps) IM_HIP(hipMemsetAsync(d_swaps, 0, sizeof(int64_t), stream), "clear swap count");
    if (lx == 0 || ly == 0) return IM_OK;
    if (!data) return fail(IM_ERR_INVALID_ARG, "null data pointer");
    const int64_t ns = ls_stash_elems(lx, ly);
    void *stash = nullptr;
    if (ns > 0)
        IM_HIP(hipMallocAsync(&stash, (size_t)elem_bytes * ns, stream), "stash allocation");
    hipError_t e = launch_rotate_ls_single(data, lx, ly, elem_bytes, stash,
                                           (unsigned long long *)d_swaps, stream);
    hipError_t ef = stash ? hipFreeAsync(stash, stream) : hipSuccess;
    if (e != hipSuccess) return hip_fail(e, "launch linear shifting");
    if (ef != hipSuccess) return hip_fail(ef, "stash free");
    return IM_OK;
}

int merge_out_of_place(const void *in, void *out, int64_t L_A, int64_t L_B, int dtype,
                       hipStream_t stream) {
    int rc = check_common(in, L_A, L_B, dtype);
    if (rc) return rc;
    const int64_t n = L_A + L_B;
    if (n == 0) return IM_OK;
    if (!out) return fail(IM_ERR_INVALID_ARG, "null output");
    const char *ib = (const char *)in, *ob = (const char *)out;
    const int64_t bytes = n * key_size(dtype);
    if (ib < ob + bytes && ob < ib + bytes)
        return fail(IM_ERR_INVALID_ARG, "input and output overlap");
    const int64_t T = merge_oop_tile(key_size(dtype));
    const int64_t nt = (n + T - 1) / T;
    int64_t *buf = nullptr;
    IM_HIP(hipMallocAsync((void **)&buf, sizeof(int64_t) * 2 * nt, stream), "tile buffers");
    hipError_t e = launch_tile_diagonals(n, T, buf, stream);
    if (e == hipSuccess)
        e = launch_corank(dtype, in, L_A, L_B, buf, nt, buf + nt, nullptr, nullptr, stream);
    if (e == hipSuccess) e = launch_merge_oop(dtype, in, out, L_A, L_B, buf + nt, stream);
    hipError_t ef = hipFreeAsync(buf, stream);
    if (e != hipSuccess) return hip_fail(e, "out-of-place merge");
    if (ef != hipSuccess) return hip_fail(ef, "tile buffers");
    return IM_OK;
}

int inplace_merge_buffered(void *data, int64_t L_A, int64_t L_B, int dtype, hipStream_t stream) {
    int rc = check_common(data, L_A, L_B, dtype);
    if (rc) return rc;
    if (L_A == 0 || L_B == 0) { g_err.clear(); return IM_OK; }
    const size_t bytes = (size_t)(L_A + L_B) * key_size(dtype);
    void *tmp = nullptr;
    IM_HIP(hipMallocAsync(&tmp, bytes, stream), "merge buffer allocation");
    rc = merge_out_of_place(data, tmp, L_A, L_B, dtype, stream);
    hipError_t e = rc == IM_OK ? hipMemcpyAsync(data, tmp, bytes, hipMemcpyDeviceToDevice, stream)
                               : hipSuccess;
    hipError_t ef = hipFreeAsync(tmp, stream);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "copy back");
    if (ef != hipSuccess) return hip_fail(ef, "merge buffer free");
    return IM_OK;
}

// ---------------------------------------------------------------------------
// Captured batched merge.
// ---------------------------------------------------------------------------
int batched_inplace_merge_graph(im_graph **out, void *data, const int64_t *d_offsets, int64_t n,
                                int64_t total_elems, int64_t max_instance, int dtype,
                                hipStream_t stream) {
    if (!out) return fail(IM_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    if (!valid_dtype(dtype)) return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported key dtype");
    if (n <= 0 || total_elems <= 0 || max_instance < 0)
        return fail(IM_ERR_INVALID_ARG, "a graph needs n > 0 and total_elems > 0");
    if (data == nullptr || d_offsets == nullptr) return fail(IM_ERR_INVALID_ARG, "null pointer");
    if (n >= (int64_t(1) << 31)) return fail(IM_ERR_INVALID_ARG, "too many instances");
    DevState *ds = dev_state(nullptr);
    if (!ds) return fail(IM_ERR_HIP, "no current HIP device");
    const int ek = key_size(dtype);
    Plan pl = {};
    {
        std::lock_guard<std::mutex> lock(ds->mu);
        int dev = 0;
        (void)hipGetDevice(&dev);
        load_tune_cache(ds, dev);
        const int cfg = choose_cfg(ds, ek, 0, n, total_elems, -1);
        if (!make_plan(ds, ek, 0, n, total_elems, max_instance, cfg, &pl))
            return fail(IM_ERR_HIP, "could not size the leaf merge grid");
        ensure_err_word(ds);
    }
    set_cells(pl, n == 1);   // a single pair is tiled by output cells, as in the eager call
    if (pl.leaf_shift == 0)
        return fail(IM_ERR_INVALID_ARG, "too many instances for the 64-bit leaf/tile counter");
    pl.epoch = 1;   // every replay clears the flags first
    im_graph *g = new (std::nothrow) im_graph();
    if (!g) return fail(IM_ERR_WORKSPACE, "out of host memory");
    (void)hipGetDevice(&g->device);
    g->plan = pl;
    g->ws_bytes = carve(pl, 0, nullptr, nullptr);
    if (hipMalloc(&g->ws, g->ws_bytes) != hipSuccess) {
        g->ws = nullptr;
        im_graph_destroy(g);
        return fail(IM_ERR_WORKSPACE, "graph workspace allocation failed");
    }
    Work w;
    carve(pl, 0, g->ws, &w);
    w.host_err = ds->d_err;
    int th, ipt, depth;
    size_t lds;
    leaf_geometry(ek, 0, pl.cfg, &th, &ipt, &depth, &lds);
    const void *leaf_fn = leaf_kernel_ptr(dtype, 0, pl.cfg);
    hipError_t e = leaf_fn ? hipFuncSetAttribute(leaf_fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds)
                           : hipErrorInvalidValue;
    hipStream_t cs = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    // the caller's stream may still be writing the inputs: order the capture
    // stream's (non-captured) set-up after it
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        if (cs) (void)hipStreamDestroy(cs);
        im_graph_destroy(g);
        return hip_fail(e, "graph set-up");
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    int rc = IM_OK;
    if (e == hipSuccess) {
        e = launch_fill32(w.tile_flag, pl.cap_tiles, 0u, cs);
        if (e == hipSuccess)
            rc = enqueue_division(dtype, 0, data, nullptr, d_offsets, n, 0, 0, nullptr, pl, w,
                                  false, false, cs);
    }
    // the leaf merge is added by hand after the captured chain so that it can
    // carry the cooperative attribute
    std::vector<hipGraphNode_t> deps;
    if (e == hipSuccess && rc == IM_OK) {
        hipStreamCaptureStatus st;
        unsigned long long id = 0;
        hipGraph_t cg = nullptr;
        const hipGraphNode_t *dp = nullptr;
        size_t nd = 0;
        e = hipStreamGetCaptureInfo_v2(cs, &st, &id, &cg, &dp, &nd);
        if (e == hipSuccess) deps.assign(dp, dp + nd);
    }
    hipGraph_t graph = nullptr;
    hipError_t e_end = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (rc != IM_OK || e != hipSuccess || e_end != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        im_graph_destroy(g);
        if (rc != IM_OK) return rc;
        return hip_fail(e != hipSuccess ? e : e_end, "graph capture");
    }
    g->graph = graph;
    void *keys = data, *vals = nullptr;
    Plan plc = pl;
    Work wc = w;
    void *args[] = {&keys, &vals, &plc, &wc};
    hipKernelNodeParams kp = {};
    kp.func = const_cast<void *>(leaf_fn);
    kp.gridDim = dim3(pl.grid_leaf);
    kp.blockDim = dim3(th);
    kp.sharedMemBytes = (unsigned)lds;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t leaf_node = nullptr;
    e = hipGraphAddKernelNode(&leaf_node, graph, deps.empty() ? nullptr : deps.data(), deps.size(),
                              &kp);
    if (e != hipSuccess) {
        im_graph_destroy(g);
        return hip_fail(e, "graph leaf node");
    }
    hipKernelNodeAttrValue av;
    std::memset(&av, 0, sizeof(av));
    av.cooperative = 1;
    g->coop = hipGraphKernelNodeSetAttribute(leaf_node, hipKernelNodeAttributeCooperative, &av) ==
              hipSuccess;
    (void)hipGetLastError();   // an unsupported attribute leaves no sticky error
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        g->exec = nullptr;
        im_graph_destroy(g);
        return hip_fail(e, "graph instantiate");
    }
    record_stats(pl, w);
    g_last_ctr = nullptr;   // counters live in the graph's workspace
    *out = g;
    g_err.clear();
    return IM_OK;
}

int im_graph_launch(im_graph *g, hipStream_t stream) {
    if (!g || !g->exec) return fail(IM_ERR_INVALID_ARG, "null graph");
    IM_HIP(hipGraphLaunch(g->exec, stream), "graph launch");
    g_stats = im_stats{};
    g_stats.leaf_capacity = g->plan.leaf_cap;
    g_stats.tile = g->plan.tile;
    g_stats.max_levels = g->plan.max_levels;
    g_stats.leaf_config = g->plan.cfg;
    g_stats.leaf_grid = g->plan.grid_leaf;
    g_last_ctr = reinterpret_cast<Counters *>(g->ws);   // first carve slot
    return IM_OK;
}

int im_graph_cooperative(const im_graph *g) { return (g && g->coop) ? 1 : 0; }

int im_graph_destroy(im_graph *g) {
    if (!g) return IM_OK;
    (void)hipDeviceSynchronize();
    if (g_last_ctr == reinterpret_cast<Counters *>(g->ws)) g_last_ctr = nullptr;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ws) (void)hipFree(g->ws);
    delete g;
    return IM_OK;
}

// ---------------------------------------------------------------------------
// Leaf configuration and autotuner.
// ---------------------------------------------------------------------------
int inplace_merge_set_config(int cfg) {
    if (cfg < -1 || cfg >= kLeafCfgs) return fail(IM_ERR_INVALID_ARG, "no such leaf configuration");
    g_force_cfg.store(cfg);
    return IM_OK;
}

int inplace_merge_autotune(const void *data, const int64_t *d_offsets, int64_t n,
                           int64_t total_elems, int64_t max_instance, int key_dtype,
                           int val_dtype, int reps, double *ms_out, int *chosen,
                           hipStream_t stream) {
    if (!valid_dtype(key_dtype)) return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported key dtype");
    if (val_dtype != -1 && !valid_dtype(val_dtype))
        return fail(IM_ERR_UNSUPPORTED_DTYPE, "unsupported payload dtype");
    if (n <= 0 || total_elems <= 0 || max_instance < 0 || reps < 1)
        return fail(IM_ERR_INVALID_ARG, "autotune needs n > 0, total_elems > 0, reps >= 1");
    if (!data || !d_offsets) return fail(IM_ERR_INVALID_ARG, "null pointer");
    if (n >= (int64_t(1) << 31)) return fail(IM_ERR_INVALID_ARG, "too many instances");
    DevState *ds = dev_state(nullptr);
    if (!ds) return fail(IM_ERR_HIP, "no current HIP device");
    const int ek = key_size(key_dtype);
    const int ev = val_dtype < 0 ? 0 : key_size(val_dtype);
    // the data buffer holds exactly d_offsets[2n] elements
    int64_t used = 0;
    IM_HIP(hipStreamSynchronize(stream), "autotune sync");
    IM_HIP(hipMemcpy(&used, d_offsets + 2 * n, sizeof(used), hipMemcpyDeviceToHost),
           "read offsets");
    if (used < 0 || used > total_elems)
        return fail(IM_ERR_INVALID_ARG, "d_offsets[2n] outside [0, total_elems]");
    void *sk = nullptr, *sv = nullptr;
    hipEvent_t ea = nullptr, eb = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(stream);
        if (sk) (void)hipFree(sk);
        if (sv) (void)hipFree(sv);
        if (ea) (void)hipEventDestroy(ea);
        if (eb) (void)hipEventDestroy(eb);
    };
    const size_t nb = (size_t)std::max<int64_t>(used, 1);
    if (hipMalloc(&sk, nb * ek) != hipSuccess || (ev && hipMalloc(&sv, nb * ev) != hipSuccess)) {
        cleanup();
        return fail(IM_ERR_WORKSPACE, "autotune scratch allocation failed");
    }
    if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
        cleanup();
        return fail(IM_ERR_HIP, "event create");
    }
    if (ev) (void)hipMemsetAsync(sv, 0, nb * ev, stream);
    double med[kLeafCfgs];
    int best = 0;
    for (int cfg = 0; cfg < kLeafCfgs; ++cfg) {
        std::vector<double> t;
        for (int r = 0; r <= reps; ++r) {
            hipError_t e = hipMemcpyAsync(sk, data, (size_t)used * ek, hipMemcpyDeviceToDevice, stream);
            if (e == hipSuccess) e = hipEventRecord(ea, stream);
            if (e != hipSuccess) { cleanup(); return hip_fail(e, "autotune copy"); }
            int rc = run_pipeline(key_dtype, ev, sk, sv, d_offsets, n, total_elems, max_instance,
                                  0, 0, nullptr, stream, cfg);
            if (rc) { cleanup(); return rc; }
            e = hipEventRecord(eb, stream);
            if (e == hipSuccess) e = hipEventSynchronize(eb);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ea, eb);
            if (e != hipSuccess) { cleanup(); return hip_fail(e, "autotune timing"); }
            if (r > 0) t.push_back(ms);
        }
        std::sort(t.begin(), t.end());
        med[cfg] = t[t.size() / 2];
        if (ms_out) ms_out[cfg] = med[cfg];
        if (med[cfg] < med[best]) best = cfg;
    }
    cleanup();
    {
        std::lock_guard<std::mutex> lock(ds->mu);
        ds->tuned[key_index(ek)][val_index(ev)][size_class(n, total_elems)] = best;
        int dev = 0;
        (void)hipGetDevice(&dev);
        save_tune_entry(dev, ek, ev, size_class(n, total_elems), best);
    }
    if (log_level() >= 2) {
        std::fprintf(stderr, "[inplace_merge] autotune: class %d, median ms",
                     size_class(n, total_elems));
        for (int c = 0; c < kLeafCfgs; ++c) std::fprintf(stderr, " %.4f", med[c]);
        std::fprintf(stderr, ", chosen %d\n", best);
    }
    if (chosen) *chosen = best;
    g_err.clear();
    return IM_OK;
}

// ---------------------------------------------------------------------------
// Learned split.
// ---------------------------------------------------------------------------
int merge_model_create(merge_model **out, const float *params, uint64_t seed) {
    if (!out) return fail(IM_ERR_INVALID_ARG, "null output");
    merge_model *m = new (std::nothrow) merge_model();
    if (!m) return fail(IM_ERR_WORKSPACE, "out of host memory");
    if (hipGetDevice(&m->device) != hipSuccess) { delete m; return fail(IM_ERR_HIP, "no device"); }
    if (params) {
        std::memcpy(m->host, params, sizeof(m->host));
    } else {
        // ReLU hinges spread over [0, 1): unit slopes, knots at h/H, small
        // seeded output weights.
        uint64_t st = seed;
        for (int h = 0; h < kMlpHidden; ++h) {
            double u = (double)(splitmix(st) >> 11) / 9007199254740992.0;
            double v = (double)(splitmix(st) >> 11) / 9007199254740992.0;
            m->host[h] = (float)(1.0 + 0.1 * (u - 0.5));
            m->host[kMlpHidden + h] = (float)(-(double)h / kMlpHidden);
            m->host[2 * kMlpHidden + h] = (float)(0.2 * (v - 0.5));
        }
        m->host[3 * kMlpHidden] = 0.0f;
    }
    if (hipMalloc(&m->d, sizeof(MlpDev)) != hipSuccess ||
        hipMalloc(&m->d_m, sizeof(float) * kMlpParams) != hipSuccess ||
        hipMalloc(&m->d_v, sizeof(float) * kMlpParams) != hipSuccess) {
        merge_model_free(m);
        return fail(IM_ERR_WORKSPACE, "model allocation failed");
    }
    int rc = model_upload(m);
    if (rc) { merge_model_free(m); return rc; }
    *out = m;
    return IM_OK;
}

int merge_model_free(merge_model *m) {
    if (!m) return IM_OK;
    if (m->d) (void)hipFree(m->d);
    if (m->d_m) (void)hipFree(m->d_m);
    if (m->d_v) (void)hipFree(m->d_v);
    delete m;
    return IM_OK;
}

int merge_model_get_params(const merge_model *m, float *params_out) {
    if (!m || !params_out) return fail(IM_ERR_INVALID_ARG, "null pointer");
    MlpDev h;
    IM_HIP(hipMemcpy(&h, m->d, sizeof(h), hipMemcpyDeviceToHost), "model download");
    std::memcpy(params_out, h.p, sizeof(h.p));
    return IM_OK;
}

int merge_model_set_params(merge_model *m, const float *params) {
    if (!m || !params) return fail(IM_ERR_INVALID_ARG, "null pointer");
    std::memcpy(m->host, params, sizeof(m->host));
    // the error table described the old parameters: searches stay plain
    // until the model is trained again
    for (float &v : m->err_b) v = kErrUnknown;
    m->err_scale = 1.0f;
    return model_upload(m);
}

int merge_model_adam_step(merge_model *m, const float *d_grad, float *d_m, float *d_v, float lr,
                          int step, hipStream_t stream) {
    if (!m || !d_grad || !d_m || !d_v) return fail(IM_ERR_INVALID_ARG, "null pointer");
    if (step < 1) return fail(IM_ERR_INVALID_ARG, "Adam steps count from 1");
    if (!(lr >= 0.0f)) return fail(IM_ERR_INVALID_ARG, "bad learning rate");
    IM_HIP(launch_mlp_adam(m->d->p, d_grad, d_m, d_v, lr, step, stream), "launch Adam step");
    return IM_OK;
}

int merge_model_grad(const merge_model *m, const float *d_x, const float *d_t, int64_t M,
                     float *d_grad, float *d_loss, hipStream_t stream) {
    if (!m || !d_x || !d_t || !d_grad) return fail(IM_ERR_INVALID_ARG, "null pointer");
    if (M <= 0) return fail(IM_ERR_INVALID_ARG, "no samples");
    int nb = mlp_grad_blocks(M);
    float *partial = nullptr;
    IM_HIP(hipMallocAsync((void **)&partial, sizeof(float) * (kMlpParams + 1) * nb, stream),
           "alloc partials");
    IM_HIP(launch_mlp_grad(m->d->p, d_x, d_t, M, partial, nb, stream), "launch grad");
    IM_HIP(launch_mlp_reduce(partial, nb, d_grad, d_loss, stream), "launch reduce");
    IM_HIP(hipFreeAsync(partial, stream), "free partials");
    return IM_OK;
}

int merge_model_forward(const merge_model *m, const float *d_x, int64_t M, float *d_y,
                        hipStream_t stream) {
    if (!m || !d_x || !d_y) return fail(IM_ERR_INVALID_ARG, "null pointer");
    if (M <= 0) return IM_OK;
    IM_HIP(launch_mlp_forward(m->d->p, d_x, M, d_y, stream), "launch forward");
    return IM_OK;
}

static int train_model(merge_model *m, const void *data, int64_t L_A, int64_t L_B, int dtype,
                       const merge_train_cfg *cfg, hipStream_t stream);

int merge_model_train(merge_model **pm, const void *data, int64_t L_A, int64_t L_B, int dtype,
                      const merge_train_cfg *cfg, hipStream_t stream) {
    if (!pm || !cfg) return fail(IM_ERR_INVALID_ARG, "null pointer");
    int rc = check_common(data, L_A, L_B, dtype);
    if (rc) return rc;
    if (L_A == 0 || L_B == 0) return fail(IM_ERR_INVALID_ARG, "both runs must be non-empty");
    if (cfg->samples < 2 || cfg->steps < 0 || !(cfg->lr > 0.0f))
        return fail(IM_ERR_INVALID_ARG, "bad config");
    const bool created = *pm == nullptr;
    if (created) {
        rc = merge_model_create(pm, nullptr, cfg->seed);
        if (rc) return rc;
    }
    rc = train_model(*pm, data, L_A, L_B, dtype, cfg, stream);
    if (rc && created) {
        merge_model_free(*pm);
        *pm = nullptr;
    }
    return rc;
}

static int train_model(merge_model *m, const void *data, int64_t L_A, int64_t L_B, int dtype,
                       const merge_train_cfg *cfg, hipStream_t stream) {
    const int64_t M = cfg->samples;
    const int nb = mlp_grad_blocks(M);
    int64_t *d_k = nullptr, *d_i = nullptr;
    float *d_x = nullptr, *d_t = nullptr, *d_g = nullptr, *d_part = nullptr;
    auto cleanup = [&]() {
        if (d_k) (void)hipFree(d_k);
        if (d_i) (void)hipFree(d_i);
        if (d_x) (void)hipFree(d_x);
        if (d_t) (void)hipFree(d_t);
        if (d_g) (void)hipFree(d_g);
        if (d_part) (void)hipFree(d_part);
    };
    if (hipMalloc(&d_k, sizeof(int64_t) * M) != hipSuccess ||
        hipMalloc(&d_i, sizeof(int64_t) * M) != hipSuccess ||
        hipMalloc(&d_x, sizeof(float) * M) != hipSuccess ||
        hipMalloc(&d_t, sizeof(float) * M) != hipSuccess ||
        hipMalloc(&d_g, sizeof(float) * kMlpParams) != hipSuccess ||
        hipMalloc(&d_part, sizeof(float) * (kMlpParams + 1) * nb) != hipSuccess) {
        cleanup();
        return fail(IM_ERR_WORKSPACE, "training buffers");
    }
    hipError_t e = hipSuccess;
    e = launch_mlp_samples(dtype, data, L_A, L_B, M, d_k, d_x, stream);
    if (e == hipSuccess) e = launch_corank(dtype, data, L_A, L_B, d_k, M, d_i, nullptr, nullptr, stream);
    if (e == hipSuccess) e = launch_mlp_targets(d_i, M, L_A, d_t, stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->d_m, 0, sizeof(float) * kMlpParams, stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->d_v, 0, sizeof(float) * kMlpParams, stream);
    // cosine decay of the learning rate to zero over the steps
    for (int st = 1; st <= cfg->steps && e == hipSuccess; ++st) {
        const float lr = (float)((double)cfg->lr * 0.5 *
                                 (1.0 + std::cos(M_PI * (double)st / (double)cfg->steps)));
        e = launch_mlp_grad(m->d->p, d_x, d_t, M, d_part, nb, stream);
        if (e == hipSuccess) e = launch_mlp_reduce(d_part, nb, d_g, nullptr, stream);
        if (e == hipSuccess) e = launch_mlp_adam(m->d->p, d_g, m->d_m, m->d_v, lr, st, stream);
    }
    if (e == hipSuccess) e = launch_mlp_errscale(m->d->p, d_k, d_i, M, L_A, L_B, m->d, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    MlpDev h;
    if (e == hipSuccess) e = hipMemcpy(&h, m->d, sizeof(h), hipMemcpyDeviceToHost);
    cleanup();
    if (e != hipSuccess) return hip_fail(e, "training");
    std::memcpy(m->host, h.p, sizeof(m->host));
    m->err_scale = h.err_scale;
    std::memcpy(m->err_b, h.err_b, sizeof(m->err_b));
    return IM_OK;
}

int im_corank_learned(const void *data, int64_t L_A, int64_t L_B, int dtype, const merge_model *m,
                      const int64_t *d_k, int64_t nk, int64_t *d_out, int32_t *d_probes,
                      hipStream_t stream) {
    int rc = check_common(data, L_A, L_B, dtype);
    if (rc) return rc;
    if (!m) return fail(IM_ERR_INVALID_ARG, "null model");
    if (nk < 0) return fail(IM_ERR_INVALID_ARG, "negative count");
    if (nk == 0) return IM_OK;
    if (!d_k || !d_out) return fail(IM_ERR_INVALID_ARG, "null pointer");
    IM_HIP(launch_corank(dtype, data, L_A, L_B, d_k, nk, d_out, m->d, d_probes, stream),
           "launch learned co-rank");
    return IM_OK;
}

int inplace_merge_learned(void *data, int64_t L_A, int64_t L_B, int dtype, const merge_model *m,
                          hipStream_t stream) {
    int rc = check_common(data, L_A, L_B, dtype);
    if (rc) return rc;
    if (!m) return fail(IM_ERR_INVALID_ARG, "null model");
    if (L_A == 0 || L_B == 0) { g_err.clear(); return IM_OK; }
    return run_pipeline(dtype, 0, data, nullptr, nullptr, 1, L_A + L_B, L_A + L_B, L_A, L_B, m->d,
                        stream);
}

int merge_model_save(const merge_model *m, const char *path) {
    if (!m || !path) return fail(IM_ERR_INVALID_ARG, "null pointer");
    float p[kMlpParams];
    int rc = merge_model_get_params(m, p);
    if (rc) return rc;
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(IM_ERR_INVALID_ARG, std::string("cannot open ") + path);
    // IMMLP2: parameters, mean error, the bracket table
    const char magic[8] = {'I', 'M', 'M', 'L', 'P', '2', 0, 0};
    int32_t hdr[3] = {kMlpHidden, kMlpParams, kErrBuckets};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
              std::fwrite(p, sizeof(p), 1, f) == 1 &&
              std::fwrite(&m->err_scale, sizeof(float), 1, f) == 1 &&
              std::fwrite(m->err_b, sizeof(m->err_b), 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(IM_ERR_INVALID_ARG, "write failed");
    return IM_OK;
}

int merge_model_load(merge_model **out, const char *path) {
    if (!out || !path) return fail(IM_ERR_INVALID_ARG, "null pointer");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(IM_ERR_INVALID_ARG, std::string("cannot open ") + path);
    char magic[8];
    int32_t hdr[3];
    float p[kMlpParams];
    float es = 1.0f;
    float eb[kErrBuckets];
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "IMMLP2", 6) == 0 &&
              std::fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == kMlpHidden &&
              hdr[1] == kMlpParams && hdr[2] == kErrBuckets &&
              std::fread(p, sizeof(p), 1, f) == 1 && std::fread(&es, sizeof(float), 1, f) == 1 &&
              std::fread(eb, sizeof(eb), 1, f) == 1;
    std::fclose(f);
    if (!ok) return fail(IM_ERR_INVALID_ARG, "not a model file of this shape");
    int rc = merge_model_create(out, p, 0);
    if (rc) return rc;
    (*out)->err_scale = es;
    std::memcpy((*out)->err_b, eb, sizeof(eb));
    return model_upload(*out);
}

}  // extern "C"
