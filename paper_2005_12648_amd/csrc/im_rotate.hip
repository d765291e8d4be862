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

template <typename EV> struct ValBytes { static constexpr int v = sizeof(EV); };

struct NoVal {};
template <> struct ValBytes<NoVal> { static constexpr int v = 0; };

// Per element width (key + payload bytes): threads per workgroup, the most
// pieces an item may cycle (fused two-level exchanges need up to kMaxCyc;
// 16-byte elements run only pairs, and their levels are not fused), and the
// elements per thread and piece.  Every lane holds MAXC x PER elements per
// item, twice (software pipeline).
template <int BYTES>
struct RotGeom {
    static constexpr int threads = BYTES <= 4 ? 512 : 1024;
    static constexpr int maxc = BYTES <= 12 ? kMaxCyc : 2;
    static constexpr int per = (int)(kRotChunk / threads);
};

// One work item moves `lim` elements of each of c pieces: the element at
// P_k[dir_k * t] goes to P_{k+1 mod c}[dir_{k+1} * t], t in [0, lim).  A
// block swap is a cycle of two pieces running upwards; the two ends of a
// reversal are two pieces, the second running downwards; a cycle of a fused
// two-level exchange has up to kMaxCyc pieces running upwards.  The starts
// are the same for every lane: only a 32-bit offset varies per lane.
struct CycItem {
    int64_t start[kMaxCyc];
    int32_t dir[kMaxCyc];
    int32_t c, lim;
};

// Item `local` of exchange R in this phase; lim = 0 if the phase has no such
// item.
//   cycle (R.c >= 2): phase 0 moves chunk `local` of its pieces;
//   |X| == |Y|: phase 0 swaps X with Y (one linear-shifting step);
//   |X| != |Y|: phase 0 reverses X and Y (items of X first), phase 1
//   reverses X|Y.
__device__ __forceinline__ CycItem make_item(const Rot &R, int64_t local, int phase) {
    CycItem it;
#pragma unroll
    for (int k = 0; k < kMaxCyc; ++k) {
        it.start[k] = 0;
        it.dir[k] = 1;
    }
    it.c = 2;
    it.lim = 0;
    if (R.c >= 2) {
        if (phase != 0) return it;
        const int64_t c0 = local * kRotChunk;
        const int64_t n = R.len - c0;
        if (n <= 0) return it;
        it.c = R.c;
#pragma unroll
        for (int k = 0; k < kMaxCyc; ++k) it.start[k] = R.start[k] + c0;
        it.lim = (int32_t)(n < kRotChunk ? n : kRotChunk);
        return it;
    }
    if (R.lx == R.ly) {
        if (phase != 0) return it;
        const int64_t c0 = local * kRotChunk;
        const int64_t n = R.lx - c0;
        if (n <= 0) return it;
        it.start[0] = R.pos + c0;
        it.start[1] = R.pos + R.lx + c0;
        it.lim = (int32_t)(n < kRotChunk ? n : kRotChunk);
        return it;
    }
    int64_t s, m, c0;
    if (phase == 0) {
        const int64_t ix = (R.lx / 2 + kRotChunk - 1) / kRotChunk;
        if (local < ix) {
            s = R.pos; m = R.lx; c0 = local * kRotChunk;
        } else {
            s = R.pos + R.lx; m = R.ly; c0 = (local - ix) * kRotChunk;
        }
    } else {
        s = R.pos; m = R.lx + R.ly; c0 = local * kRotChunk;
    }
    const int64_t n = m / 2 - c0;          // pairs (t, m-1-t) for t < m/2
    if (n <= 0) return it;
    it.start[0] = s + c0;
    it.start[1] = s + m - 1 - c0;
    it.dir[1] = -1;
    it.lim = (int32_t)(n < kRotChunk ? n : kRotChunk);
    return it;
}

template <typename E, int MAXC, int PER>
struct CycRegs {
    E v[MAXC][PER];
};

__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename E, int TH, int MAXC, int PER>
__device__ __forceinline__ void item_load(const E *__restrict__ p, const CycItem &it,
                                          CycRegs<E, MAXC, PER> &r) {
    const int c = __builtin_amdgcn_readfirstlane(it.c);
    const int lim = __builtin_amdgcn_readfirstlane(it.lim);
#pragma unroll
    for (int k = 0; k < MAXC; ++k) {
        if (k < c) {
            const E *P = p + uni64(it.start[k]);
            const int dir = __builtin_amdgcn_readfirstlane(it.dir[k]);
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int t = (int)threadIdx.x + u * TH;
                if (t < lim) r.v[k][u] = P[dir * t];
            }
        }
    }
}

template <typename E, int TH, int MAXC, int PER>
__device__ __forceinline__ void item_store(E *__restrict__ p, const CycItem &it,
                                           const CycRegs<E, MAXC, PER> &r) {
    const int c = __builtin_amdgcn_readfirstlane(it.c);
    const int lim = __builtin_amdgcn_readfirstlane(it.lim);
#pragma unroll
    for (int k = 0; k < MAXC; ++k) {
        if (k < c) {
            const int d = k + 1 == c ? 0 : k + 1;      // piece k moves to piece d
            E *P = p + uni64(it.start[d]);
            const int dir = __builtin_amdgcn_readfirstlane(it.dir[d]);
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int t = (int)threadIdx.x + u * TH;
                if (t < lim) P[dir * t] = r.v[k][u];
            }
        }
    }
}

template <typename EV, int MAXC, int PER>
struct ValRegs { CycRegs<EV, MAXC, PER> r; };
template <int MAXC, int PER>
struct ValRegs<NoVal, MAXC, PER> {};

// A persistent grid walks the level's items, software pipelined: the loads
// of the workgroup's next item are issued before the stores of the current
// one, so one item's stores drain while the next one's loads are in flight.
// (Measured on MI355X, 2^27-pair swap: plain grid-stride loop 4.2 TB/s,
// pipelined 5.1-5.3 TB/s; one workgroup per item reaches 5.2 TB/s, but an
// empty launch of such a grid costs about 18 us against 6 us, and the
// phase-1 launch is empty whenever a level has only block swaps.)
// Items go to workgroups in grid-stride order for 512-thread workgroups
// (elements of 4 bytes).  1024-thread workgroups (wider elements) take their
// first item by index and the rest from a per-level, per-phase counter:
// thread 0 takes the next index one item ahead and hands it over through
// LDS, so the counter's latency hides behind an item.  (Measured: the
// counter makes the 2^26+2^26 int64+uint32 merge 4% faster at a grid of
// 1024 and the 2^27+2^27 int32 merge 7-23% slower at grids of 2048-6144.)
template <typename EK, typename EV,
          typename G = RotGeom<(int)sizeof(EK) + ValBytes<EV>::v>>
__global__ __launch_bounds__(G::threads) void k_rotate(EK *__restrict__ keys, EV *__restrict__ vals,
                                                       const Rot *__restrict__ rot,
                                                       Counters *__restrict__ ctr,
                                                       int64_t cap_rot, int level, int phase) {
    constexpr bool HAS_V = !std::is_same<EV, NoVal>::value;
    constexpr int TH = G::threads, MAXC = G::maxc, PER = G::per;
    constexpr bool DYN = TH >= 1024;   // items from the counter after the first
    __shared__ int64_t s_item[2];
    if (phase == 1 && ctr->level_rev[level] == 0) return;   // only swaps and cycles
    const unsigned long long packed = ctr->level_rot[level];
    int64_t nrot = (int64_t)(packed >> kRotCountShift);
    if (nrot > cap_rot) nrot = cap_rot;
    const int64_t nitems = (int64_t)(packed & kRotWorkMask);
    if (nrot == 0 || nitems == 0) return;

    Rot R;                 // descriptor of the exchange holding the item
    R.w0 = 1;
    R.nw = 0;              // empty: forces a search for the first item
    bool have = false;     // an item is loaded and waits for its stores
    CycItem cur;
    CycRegs<EK, MAXC, PER> kr;
    ValRegs<EV, MAXC, PER> vr;
    unsigned long long pend = 0;   // thread 0: counter value for the item after next
    if (DYN && threadIdx.x == 0) pend = atomicAdd(&ctr->rot_next[level][phase], 1ull);
    int par = 0;
    for (int64_t wi = blockIdx.x;;) {
        CycItem nx;
        nx.lim = 0;
        if (wi < nitems) {
            if (wi < R.w0 || wi >= R.w0 + R.nw) {
                // exchange holding item wi: last r with rot[r].w0 <= wi
                int64_t lo = 0, hi = nrot;
                while (hi - lo > 1) {
                    int64_t mid = (lo + hi) >> 1;
                    if (rot[mid].w0 <= wi) lo = mid; else hi = mid;
                }
                R = rot[lo];
            }
            if (wi >= R.w0 && wi < R.w0 + R.nw && R.c <= MAXC)   // else dropped / unsupported
                nx = make_item(R, wi - R.w0, phase);
        }
        if (nx.lim > 0) {
            CycRegs<EK, MAXC, PER> kn;
            ValRegs<EV, MAXC, PER> vn;
            item_load<EK, TH, MAXC, PER>(keys, nx, kn);
            if constexpr (HAS_V) item_load<EV, TH, MAXC, PER>(vals, nx, vn.r);
            if (have) {
                item_store<EK, TH, MAXC, PER>(keys, cur, kr);
                if constexpr (HAS_V) item_store<EV, TH, MAXC, PER>(vals, cur, vr.r);
            }
            kr = kn;
            vr = vn;
            cur = nx;
            have = true;
        }
        if (wi >= nitems) break;
        if constexpr (DYN) {
            // an index taken after one at or past nitems is past it too, so
            // an unused last take loses no item
            if (threadIdx.x == 0) {
                s_item[par] = (int64_t)gridDim.x + (int64_t)pend;
                pend = atomicAdd(&ctr->rot_next[level][phase], 1ull);
            }
            __syncthreads();
            wi = s_item[par];
            par ^= 1;
        } else {
            wi += gridDim.x;
        }
    }
    if (have) {
        item_store<EK, TH, MAXC, PER>(keys, cur, kr);
        if constexpr (HAS_V) item_store<EV, TH, MAXC, PER>(vals, cur, vr.r);
    }
}

// Single exchange (stand-alone entry point): one descriptor built on the host.
template <typename E, typename G = RotGeom<(int)sizeof(E)>>
__global__ __launch_bounds__(G::threads) void k_rotate_one(E *__restrict__ p, int64_t lx, int64_t ly,
                                                          int phase, int64_t nitems) {
    Rot R;
    R.pos = 0; R.lx = lx; R.ly = ly; R.w0 = 0; R.nw = nitems; R.c = 0; R.len = 0;
    for (int64_t wi = blockIdx.x; wi < nitems; wi += gridDim.x) {
        const CycItem it = make_item(R, wi, phase);
        if (it.lim <= 0) continue;
        CycRegs<E, 2, G::per> r;
        item_load<E, G::threads, 2, G::per>(p, it, r);
        item_store<E, G::threads, 2, G::per>(p, it, r);
    }
}

// ---------------------------------------------------------------------------
// Circular shifting (Sec. 3.4, the comparator of linear shifting): element p
// of X|Y (n = lx+ly) belongs at (p + ly) mod n.  The permutation has
// gcd(n, ly) cycles of n/gcd steps; every element is read once and written
// once, but a lane's successive accesses jump by ly.  Lane l of an exchange
// takes cycle l mod g and segment l / g of kCsSeg steps; consecutive lanes
// take consecutive cycles, so a wave's accesses are contiguous when there
// are many cycles and scattered when there are few.  A cycle held by one lane
// runs in phase 0; a cycle cut into segments needs the first value of every
// segment saved before any lane writes (phase 0: stash, phase 1: walk).
__device__ __forceinline__ int64_t cs_gcd(int64_t a, int64_t b) {
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// (a * b) mod n without overflow (n < 2^47): double and add.
__device__ __forceinline__ int64_t cs_mulmod(int64_t a, int64_t b, int64_t n) {
    int64_t r = 0;
    a %= n;
    while (b > 0) {
        if (b & 1) {
            r += a;
            if (r >= n) r -= n;
        }
        a += a;
        if (a >= n) a -= n;
        b >>= 1;
    }
    return r;
}

// Walk `steps` steps of a cycle from position x (element values v carried):
// reads run kCsBatch positions ahead of the writes (distinct positions of the
// same cycle), so a batch of loads is in flight at once.
constexpr int kCsBatch = 8;

template <typename E>
__device__ __forceinline__ void cs_walk(E *__restrict__ p, int64_t n, int64_t ly, int64_t x,
                                        int64_t steps, E v, bool read_last) {
    int64_t q = 0;
    while (q < steps) {
        int64_t pos[kCsBatch];
        E nxt[kCsBatch];
        const int64_t m = steps - q < kCsBatch ? steps - q : kCsBatch;
#pragma unroll
        for (int b = 0; b < kCsBatch; ++b) {
            if (b < m) {
                x += ly;
                if (x >= n) x -= n;
                pos[b] = x;
                const bool last = q + b + 1 == steps;
                if (!last || read_last) nxt[b] = p[x];
            }
        }
#pragma unroll
        for (int b = 0; b < kCsBatch; ++b) {
            if (b < m) {
                p[pos[b]] = v;
                v = nxt[b];
            }
        }
        q += m;
    }
}

// Lane `lane` of exchange R in phase `phase` (one array).
template <typename E>
__device__ __forceinline__ void cs_lane(E *__restrict__ base, const Rot &R, int64_t lane,
                                        int phase, E *__restrict__ stash) {
    const int64_t n = R.lx + R.ly;
    const int64_t g = cs_gcd(n, R.ly);
    const int64_t L = n / g;
    const int64_t nseg = (L + kCsSeg - 1) / kCsSeg;
    if (lane >= g * nseg) return;
    E *p = base + R.pos;
    const int64_t c = lane % g, sg = lane / g;
    if (nseg == 1) {
        // the whole cycle: its start is read first and written last
        if (phase != 0) return;
        cs_walk<E>(p, n, R.ly, c, L, p[c], false);
        return;
    }
    const int64_t q0 = sg * kCsSeg;
    const int64_t q1 = q0 + kCsSeg < L ? q0 + kCsSeg : L;
    int64_t x0 = c + cs_mulmod(q0, R.ly, n);
    if (x0 >= n) x0 -= n;
    if (phase == 0) {
        stash[R.stash0 + lane] = p[x0];
    } else {
        // writes reach the next segment's start, whose value is in the stash
        cs_walk<E>(p, n, R.ly, x0, q1 - q0, stash[R.stash0 + lane], false);
    }
}

template <typename EK, typename EV>
__global__ __launch_bounds__(kCsLanes) void k_rotate_cs(EK *__restrict__ keys, EV *__restrict__ vals,
                                                        const Rot *__restrict__ rot,
                                                        const Counters *__restrict__ ctr,
                                                        int64_t cap_rot, int level, int phase,
                                                        EK *__restrict__ sk, EV *__restrict__ sv) {
    const unsigned long long packed = ctr->level_rot[level];
    int64_t nrot = (int64_t)(packed >> kRotCountShift);
    if (nrot > cap_rot) nrot = cap_rot;
    const int64_t nitems = (int64_t)(packed & kRotWorkMask);
    for (int64_t wi = blockIdx.x; wi < nitems; wi += gridDim.x) {
        int64_t lo = 0, hi = nrot;
        while (hi - lo > 1) {
            int64_t mid = (lo + hi) >> 1;
            if (rot[mid].w0 <= wi) lo = mid; else hi = mid;
        }
        if (nrot == 0) break;
        const Rot R = rot[lo];
        if (wi < R.w0 || wi >= R.w0 + R.nw) continue;   // a dropped exchange
        const int64_t lane = (wi - R.w0) * kCsLanes + threadIdx.x;
        cs_lane<EK>(keys, R, lane, phase, sk);
        if constexpr (!std::is_same<EV, NoVal>::value) cs_lane<EV>(vals, R, lane, phase, sv);
    }
}

template <typename E>
__global__ __launch_bounds__(kCsLanes) void k_rotate_cs_one(E *__restrict__ p, Rot R, int phase,
                                                            E *__restrict__ stash) {
    for (int64_t wi = blockIdx.x; wi < R.nw; wi += gridDim.x)
        cs_lane<E>(p, R, wi * kCsLanes + threadIdx.x, phase, stash);
}

template <typename EK, typename EV>
static hipError_t rot_cs_t(void *keys, void *vals, const Plan &pl, const Work &w, int level,
                           int phase, hipStream_t s) {
    hipLaunchKernelGGL((k_rotate_cs<EK, EV>), dim3(2048), dim3(kCsLanes), 0, s, (EK *)keys,
                       (EV *)vals, w.rot, w.ctr, pl.cap_rot, level, phase, (EK *)w.cs_stash_k,
                       (EV *)w.cs_stash_v);
    return hipGetLastError();
}

int64_t cs_lanes(int64_t lx, int64_t ly) {
    int64_t n = lx + ly, a = n, b = ly;
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    const int64_t L = n / a;
    return a * ((L + kCsSeg - 1) / kCsSeg);
}

hipError_t launch_rotate_cs_single(void *data, int64_t lx, int64_t ly, int esize, void *stash,
                                   hipStream_t s) {
    if (lx <= 0 || ly <= 0) return hipSuccess;
    Rot R;
    R.pos = 0; R.lx = lx; R.ly = ly; R.w0 = 0;
    const int64_t lanes = cs_lanes(lx, ly);
    R.nw = (lanes + kCsLanes - 1) / kCsLanes;
    R.stash0 = 0;
    const int g = (int)(R.nw < 2048 ? R.nw : 2048);
    for (int ph = 0; ph < 2; ++ph) {
        if (esize == 4)
            hipLaunchKernelGGL(k_rotate_cs_one<uint32_t>, dim3(g), dim3(kCsLanes), 0, s,
                               (uint32_t *)data, R, ph, (uint32_t *)stash);
        else if (esize == 8)
            hipLaunchKernelGGL(k_rotate_cs_one<uint64_t>, dim3(g), dim3(kCsLanes), 0, s,
                               (uint64_t *)data, R, ph, (uint64_t *)stash);
        else
            return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Linear shifting step by step (Sec. 3.4): the stand-alone exchange that
// performs the paper's swaps.  X|Y with |X| != |Y|: the smaller block is
// swapped, element pair by element pair, with the block at the far end of
// the larger one, which puts it in its final place; the rest is the same
// problem on what remains.  A run of q such steps with the same smaller
// block size s (one quotient of Euclid's algorithm on the two lengths) keeps
// one block F fixed and swaps it with B_1, B_2, ..., B_q in turn:
//   |X| <= |Y|: F = X at the front, B_t = the t-th block of s from the end;
//   |X| >  |Y|: F = Y's place (right after X), B_t = the t-th block of s
//               from the front.
// Column j of a run is a chain: F[j] <-> B_1[j], then F[j] <-> B_2[j], ...
// Columns are independent, so one lane per (column, segment of kLsSeg
// chain positions) performs those swaps in order; the value held at F[j]
// between two swaps stays in the lane's register, so F[j] is written once
// per run.  A lane's segment starts from the value the chain carries into
// it: F[j] for the first segment, else the old value at the last position of
// the segment before, which phase 0 copies to a stash before phase 1 walks.
// Every run is one launch (two with a stash); runs are in Euclid's order.
// Lanes count the swaps they perform: Sigma q*s = L_A + L_B - gcd.
constexpr int kLsSeg = 256;
constexpr int kLsThreads = 256;
constexpr int kLsBatch = 8;

struct LsRun {
    int64_t f;       // first element of the fixed block
    int64_t b1;      // first element of B_1
    int64_t bstep;   // B_t = b1 + (t - 1) * bstep  (+s or -s)
    int64_t s, q;    // block size, swaps per column
    int64_t nseg;    // segments per column (ceil(q / kLsSeg))
};

template <typename E>
__global__ __launch_bounds__(kLsThreads) void k_ls_run(E *__restrict__ p, LsRun r, int phase,
                                                      E *__restrict__ stash,
                                                      unsigned long long *__restrict__ swaps) {
    const int64_t lanes = r.s * r.nseg;
    unsigned long long done = 0;
    for (int64_t lane = (int64_t)blockIdx.x * kLsThreads + threadIdx.x; lane < lanes;
         lane += (int64_t)gridDim.x * kLsThreads) {
        const int64_t j = lane % r.s, k = lane / r.s;
        const int64_t t0 = k * kLsSeg + 1;
        const int64_t t1 = (k + 1) * kLsSeg < r.q ? (k + 1) * kLsSeg : r.q;
        if (phase == 0) {
            stash[lane] = k == 0 ? p[r.f + j] : p[r.b1 + (t0 - 2) * r.bstep + j];
            continue;
        }
        E carry = r.nseg == 1 ? p[r.f + j] : stash[lane];
        for (int64_t t = t0; t <= t1; t += kLsBatch) {
            E v[kLsBatch];
#pragma unroll
            for (int b = 0; b < kLsBatch; ++b)
                if (t + b <= t1) v[b] = p[r.b1 + (t + b - 1) * r.bstep + j];
#pragma unroll
            for (int b = 0; b < kLsBatch; ++b) {
                if (t + b <= t1) {
                    p[r.b1 + (t + b - 1) * r.bstep + j] = carry;
                    carry = v[b];
                }
            }
        }
        done += (unsigned long long)(t1 - t0 + 1);
        if (k == r.nseg - 1) p[r.f + j] = carry;
    }
    if (phase == 0 || swaps == nullptr) return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) done += __shfl_xor(done, o, 64);
    if ((threadIdx.x & 63) == 0 && done) atomicAdd(swaps, done);
}

// The runs of linear shifting on X|Y, in order (host side).
static void ls_runs(int64_t lx, int64_t ly, void (*emit)(const LsRun &, void *), void *ctx) {
    int64_t base = 0;
    while (lx > 0 && ly > 0) {
        LsRun r;
        if (lx <= ly) {
            r.s = lx;
            r.q = ly / lx;
            r.f = base;
            r.b1 = base + lx + ly - lx;
            r.bstep = -lx;
            ly -= r.q * lx;
        } else {
            r.s = ly;
            r.q = lx / ly;
            r.f = base + lx;
            r.b1 = base;
            r.bstep = ly;
            base += r.q * ly;
            lx -= r.q * ly;
        }
        r.nseg = (r.q + kLsSeg - 1) / kLsSeg;
        emit(r, ctx);
    }
}

int64_t ls_stash_elems(int64_t lx, int64_t ly) {
    int64_t need = 0;
    ls_runs(lx, ly, [](const LsRun &r, void *c) {
        int64_t *n = (int64_t *)c;
        if (r.nseg > 1 && r.s * r.nseg > *n) *n = r.s * r.nseg;
    }, &need);
    return need;
}

struct LsLaunch {
    void *data, *stash;
    unsigned long long *swaps;
    int esize;
    hipStream_t s;
    hipError_t err;
};

template <typename E>
static void ls_launch_run(const LsRun &r, LsLaunch *L) {
    const int64_t lanes = r.s * r.nseg;
    const int64_t g64 = (lanes + kLsThreads - 1) / kLsThreads;
    const int g = (int)(g64 < 8192 ? g64 : 8192);
    for (int ph = r.nseg > 1 ? 0 : 1; ph < 2 && L->err == hipSuccess; ++ph) {
        hipLaunchKernelGGL(k_ls_run<E>, dim3(g), dim3(kLsThreads), 0, L->s, (E *)L->data, r, ph,
                           (E *)L->stash, L->swaps);
        L->err = hipGetLastError();
    }
}

hipError_t launch_rotate_ls_single(void *data, int64_t lx, int64_t ly, int esize, void *stash,
                                   unsigned long long *d_swaps, hipStream_t s) {
    if (esize != 4 && esize != 8) return hipErrorInvalidValue;
    LsLaunch L{data, stash, d_swaps, esize, s, hipSuccess};
    ls_runs(lx, ly, [](const LsRun &r, void *c) {
        LsLaunch *l = (LsLaunch *)c;
        if (l->err != hipSuccess) return;
        if (l->esize == 4) ls_launch_run<uint32_t>(r, l);
        else ls_launch_run<uint64_t>(r, l);
    }, &L);
    return L.err;
}

template <typename EK, typename EV>
static hipError_t rot_t(void *keys, void *vals, const Plan &pl, const Work &w, int level,
                        int phase, hipStream_t s) {
    // 512-thread workgroups (grid-stride items): a grid several times larger
    // than the chip holds at once, so that workgroups that finish early are
    // replaced, which balances the items.  (Measured on the exchange stage
    // of the 2^27+2^27 int32 merge, about 16k items per level: grids of
    // 6144 / 12288 / 16384 / 24576 / 32768 take 0.490 / 0.480 / 0.473 /
    // 0.483 / 0.498 ms, the empty launches included; exactly the resident
    // workgroups was 6-13% slower than 2048 in an earlier version.)
    // 1024-thread workgroups take items from a counter, which balances them
    // without replacement: 1024 (best of 1024, 2048 and 4096).  Phase 1 (the
    // last reversal of three-reversal exchanges) is empty on balanced levels,
    // and an empty launch costs about its dispatch: 1024 workgroups there
    // (measured: int32 2^27+2^27 merge -0.7%, 64-byte rows -1.2%, the
    // 4096-instance batch, which has phase-1 work, unchanged).
    constexpr int TH = RotGeom<(int)sizeof(EK) + ValBytes<EV>::v>::threads;
    const int g = phase == 1 ? 1024 : (TH == 512 ? 16384 : 1024);
    hipLaunchKernelGGL((k_rotate<EK, EV>), dim3(g), dim3(TH), 0, s, (EK *)keys, (EV *)vals,
                       w.rot, w.ctr, pl.cap_rot, level, phase);
    return hipGetLastError();
}

hipError_t launch_rotate(int esize_k, int esize_v, void *keys, void *vals, const Plan &pl,
                         const Work &w, int level, int phase, hipStream_t s) {
    if (pl.rot_method == kRotCS) {
        if (esize_k == 4) {
            if (esize_v == 0) return rot_cs_t<uint32_t, NoVal>(keys, vals, pl, w, level, phase, s);
            if (esize_v == 4) return rot_cs_t<uint32_t, uint32_t>(keys, vals, pl, w, level, phase, s);
            if (esize_v == 8) return rot_cs_t<uint32_t, uint64_t>(keys, vals, pl, w, level, phase, s);
        } else if (esize_k == 8) {
            if (esize_v == 0) return rot_cs_t<uint64_t, NoVal>(keys, vals, pl, w, level, phase, s);
            if (esize_v == 4) return rot_cs_t<uint64_t, uint32_t>(keys, vals, pl, w, level, phase, s);
            if (esize_v == 8) return rot_cs_t<uint64_t, uint64_t>(keys, vals, pl, w, level, phase, s);
        }
        return hipErrorInvalidValue;
    }
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
            hipLaunchKernelGGL(k_rotate_one<uint32_t>, dim3(g), dim3(RotGeom<4>::threads), 0, s,
                               (uint32_t *)data, lx, ly, ph, nw);
        else if (esize == 8)
            hipLaunchKernelGGL(k_rotate_one<uint64_t>, dim3(g), dim3(RotGeom<8>::threads), 0, s,
                               (uint64_t *)data, lx, ly, ph, nw);
        else
            return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace imerge
