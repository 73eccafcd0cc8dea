// Step kernels of the per-timestep vehicle update on gfx950 (wave64).
//
// Layout.  Active vehicles live in a structure-of-arrays "slot" buffer sorted
// by (edge, lane, x descending, id descending), so every lane is a contiguous
// run with its front first.  The buffer is double-buffered: step t reads
// slots[t & 1] and the scatter kernel writes slots[(t + 1) & 1].  Per-lane
// tables carry the rear of each lane at the start of the step (look-ahead,
// stamped with the step they are valid for), the rear after the move
// (admission), and the post-lane-change run of each lane (scatter).
//
// One step = 4 launches (5 on networks above 262,144 edges), all reading the
// step number from device memory, so a captured graph of one step can be
// replayed for every step:
//   k_tile_step   Phases 1-2 per tile of whole edges, staged in LDS
//   k_big_admit   the same for tiles above 384 vehicles (1,024 threads), then
//                 eligibility + atomicMin of a 64-bit priority key per lane
//   k_commit      one thread per edge, over its lanes: winners, losers,
//                 arrivals, departures, travel-time sums, new lane counts and
//                 edge offsets within the workgroup
//   (k_blkscan    offsets of the commit workgroups, on large networks)
//   k_scatter     offsets of the commit workgroups (in LDS), the next layout
//                 and the next look-ahead table; the step counter advances
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>

#include "device_math.hpp"

namespace manta {

constexpr int kNT = 256;                 // threads per workgroup (4 waves)
constexpr int kWaves = kNT / 64;
constexpr int kTileWindowMax = 256;      // a tile = the edges whose first slot lies in a window of
constexpr int kTileWindowMin = 64;       // tile_window slots (a schedule parameter, 64..256, a multiple of 16)
constexpr int kTileCapLds = 304;         // tiles up to this size are staged in LDS (6 workgroups per CU)
constexpr int kTileIndexMax = 32767;     // vehicles of a tile at most (16-bit indices in LDS)
constexpr int kTileNT = 256;             // threads per tile workgroup
constexpr int kTileGroups = 8;           // tile counters of k_tile_step (one per group of workgroups)
constexpr int kTileCtrRounds = 8;        // the counters hand out tiles above this many rounds per step
constexpr int kTileCtrStride = 32;       // ints between two counters: one 128-byte line each
constexpr int kTileCtrInts = 2 * kTileGroups * kTileCtrStride;   // [step parity][group] counters
constexpr int kTileWindowAuto = 192;     // largest window the per-step choice takes
constexpr int kTileDrawTasks = 384;      // listed Philox blocks per tile round (more are computed in place)
constexpr int kCommitLanes = 8;         // lanes of an edge at most
constexpr int kCommitNT = 256;           // threads per commit workgroup
constexpr int kEdgeBlock = kCommitNT;    // edges per commit workgroup (one thread per edge)
constexpr int kBigNT = 1024;             // threads per workgroup for tiles above kTileCapLds
constexpr int kBigCapLds = 1408;         // vehicles per big tile piece staged in LDS (110 KiB)
constexpr unsigned long long kBarrierTimeout = 20000000ull;   // 0.2 s of the 100 MHz clock
constexpr int kScanLdsMax = 8192;        // edge blocks whose offsets k_scatter scans in LDS (32 KiB)
constexpr int kCounterCopies = 1024;     // each counter is spread over 1,024 slots (few colliding atomics)

// ---- vehicle meta word ---------------------------------------------------
// bits 0-3 lane | 4 mandatory | 5 held at stop line | 8-14 wrong-lane wait |
// 16-19 class | 24-31 lane mask of the move to the next edge
__host__ __device__ inline int m_lane(uint32_t m) { return (int)(m & 15u); }
__host__ __device__ inline bool m_mand(uint32_t m) { return (m >> 4) & 1u; }
__host__ __device__ inline bool m_held(uint32_t m) { return (m >> 5) & 1u; }
__host__ __device__ inline int m_ww(uint32_t m) { return (int)((m >> 8) & 127u); }
__host__ __device__ inline int m_cls(uint32_t m) { return (int)((m >> 16) & 15u); }
__host__ __device__ inline uint32_t m_mask(uint32_t m) { return m >> 24; }
__host__ __device__ inline uint32_t m_make(int lane, bool mand, bool held, int ww, int cls, uint32_t mask) {
    return (uint32_t)lane | ((uint32_t)mand << 4) | ((uint32_t)held << 5) | ((uint32_t)ww << 8) |
           ((uint32_t)cls << 16) | (mask << 24);
}
__host__ __device__ inline uint32_t m_set_lane(uint32_t m, int lane) { return (m & ~15u) | (uint32_t)lane; }

enum Status : uint8_t { kWaiting = 0, kActive = 1, kArrived = 2 };

enum Counter {
    cActiveSum = 0, cDeparted, cArrived, cLaneChanges, cTransfers, cHolds, cInsertDenied,
    cMandTriggers, cStopBranch, cClamp, cWrongLaneHolds, cWaivedExits, cGridlock, cNumCounters
};
// Gridlock detector (failure detection): a step stalls when vehicles were
// active at its start and none of them changed position or lane, crossed to
// another edge or arrived, and none departed; cGridlock counts the steps that
// end a run of at least kGridlockSteps stalled steps (5 minutes at dt = 0.5 s).
constexpr int kGridlockSteps = 600;
constexpr int kMovedSlots = 64;          // one wavefront reads them all

struct Ctl {
    // The step number, kept twice so that no kernel has to change a value its
    // own workgroups are still reading: the tile kernels and admission read t_a,
    // k_commit and k_scatter read t_b.  k_tile_step sets t_b = t_a; the
    // workgroup that finishes the step (finish_step) sets t_a = t + 1.
    int t_a;
    int t_b;
    int n_act[2];
    int n_big[2];     // tiles above kTileCapLds, listed for k_big_admit
    int err;          // non-zero: a layout bound check failed (see kErr*)
    int n_departed;   // vehicles admitted from the departure queues so far
    unsigned big_done;   // workgroups of k_big_admit past their admission pass or their big tiles
    int n_defer;      // admission items left to the workgroups of the big tiles (this step)
    unsigned long long big_updates;   // vehicle-updates done in big tiles (measurement)
    int stall_run;    // consecutive stalled steps before this one (gridlock detector)
    int pad1;
};

// t_a, t_b, n_act[0], n_act[1] in one 16-byte load (the step number and both
// active counts), so no read of the control block waits for another
struct StepHead {
    int t_a, t_b, n0, n1;
};
__device__ inline StepHead step_head(const Ctl* c) {
    const int4 v = *(const int4*)c;
    return StepHead{v.x, v.y, v.z, v.w};
}

enum : int { kErrTileTooBig = 1, kErrNewPos = 2, kErrScatter = 4, kErrPermutation = 8, kErrBarrier = 16,
             kErrTrace = 32 };

struct Slots {
    float* x;
    float* v;
    uint32_t* vid;
    int32_t* edge;
    uint32_t* meta;
    int32_t* nxt;     // next route edge, -1 on the last edge
    int32_t* gl;      // global lane after the lane change, written by the tile kernels for k_scatter
};

struct LaneRear {     // rear of a lane at the start of step `stamp`
    float xm;         // x - length of the rear vehicle
    float v;
    int stamp;
    uint32_t vid;     // the rear vehicle
};

// One vehicle in one step of a traced re-run (differentiable form): every
// discrete decision of the step, and the continuous inputs of Eq. (1).
struct TraceRec {
    uint32_t vid;
    int partner;      // leader (VEH, clamp) or look-ahead rear (LOOK), -1
    float x, v;       // start of the step
    float s, vl;      // gap and leader speed of Eq. (1)
    float xn;         // position after Phase 2
    int edge;
    uint32_t kb;      // kind | branch bits << 8 (TB_*)
    int look_gl;      // LOOK: the global lane whose start-of-step rear is the partner; else -1
};
enum : uint32_t { TB_F = 1, TB_D = 2, TB_S = 4, TB_B = 8, TB_C = 16, TB_W = 32, TB_EXIT = 64, TB_ARRIVE = 128,
                  TB_HELD = 256 };

struct LanePost {     // post-lane-change run of a lane in step `stamp`
    int stamp;
    int start;        // first slot of the run
    int cnt;
    float rear_xm;    // rear after Phase 2 (x_new - length)
};

struct Outbox {       // end-of-edge request of a lane's front vehicle
    int stamp;
    int slot;
    uint32_t vid;
    int target;       // global lane on the next edge, -1 for an arrival
    float xp;         // position on the next edge
    float phi;        // fraction of the step at which the stop line was crossed
    uint64_t key;     // admission priority (smaller first); case 1: the node key set by admission
    int elig;         // set by admission: 0 = refused; else 1 (case 2) or 1 + the node (case 1)
    uint32_t tl_cls;  // lane on the next edge | class << 8 | (case 1) (in, out) pair << 16
    float v;          // speed after the step
    int nxt;          // next edge (-1 for an arrival)
};

struct EntryRec {
    float x, v;
    uint32_t vid;
    int edge;
    uint32_t meta;
    int nxt;
    int gl;
    int pad;
};

// The constants of one edge in one 16-byte record: a vehicle's edge and its
// next edge cost one load each in the tile kernel.
struct EdgeC {
    float L;          // length, m
    float lim;        // speed limit, m/s
    int lane_base;    // first global lane
    int lanes;
};

struct Dev {
    Ctl* ctl;
    unsigned long long* counters;
    // network
    int n_edges, n_lanes_total;
    const float* L;
    const float* lim;
    const int* lanes;
    const int* lane_base;
    const EdgeC* ec;            // the four above, packed per edge
    // vehicles (static)
    int n_veh;
    const int64_t* roff;
    const int* redges;
    const uint8_t* rmask;       // per route entry: lane mask of the move to the next route edge (0xFF last)
    const uint8_t* cls;
    const float* alpha;
    const int* due;             // due[t] = vehicles with departure step <= t, t <= max_dep
    // departure queues, one per (entry lane, class), sorted by (departure
    // step, id): all members share the admission test, so only the head can
    // hold the smallest eligible key of its queue
    int* qhead;                 // next vehicle of each queue
    int2* qhd;                  // head of each queue: {departure step, id}, {INT_MAX, -1} once empty
    const int* qlane;           // global entry lane of each queue
    const float* qs0;           // s0 of the queue's class (insertion test)
    const int4* vq;             // per vehicle: {queue, index in the queue order, next vehicle of the queue or -1,
                                //   its departure step}
    int nq;
    const uint32_t* rid;        // id used in the random-number counter
    const int* scen_voff;       // first vehicle of each scenario (the id of the draws is the id within it)
    int max_dep;
    const ClassParams* cp;
    float dt;
    uint64_t seed;
    float v0_spread;    // per-driver free-flow speed spread (0: off)
    int edge_period;    // draws keyed by an edge use edge % edge_period (one scenario's edges)
    // case 1 intersections (flashing red); imode 0 = case 2 (all green)
    int imode;
    int stop_steps;             // steps a vehicle stands at the line before it may cross (2 s)
    int n_nodes;
    const int* efrom;           // [edge] tail node
    const int* pair_base;       // [edge] index among its head node's in-edges x that node's out-degree
    const int* out_idx;         // [edge] index among its tail node's out-edges
    const int* nm;              // [node] in-degree x out-degree (<= 64)
    int* rr;                    // [node] pair served last, -1 before the first (state)
    unsigned long long* win_node;   // [node] smallest eligible crossing key of the step
    // layout
    Slots s[2];
    // per vehicle (id-indexed)
    uint8_t* status;
    int* cursor;
    int* held_since;
    double* tau_in;
    double* t_arr;
    float* fin_x;
    float* fin_v;
    uint32_t* fin_meta;
    // per lane
    LaneRear* rear;
    LanePost* post;
    Outbox* outbox;
    int* req_stamp;             // the step in which the lane's front last wrote its Outbox
    unsigned long long* win;
    int* exit_stamp;
    int* enter_stamp;
    int* lane_off;              // next layout: lane start relative to its commit block
    int* lane_newcnt;
    // per edge
    int* blk_sum;
    int* blk_off;
    int n_blk;
    double* tt_sum;
    unsigned long long* tt_cnt;
    EntryRec* ent;              // per lane: the record entering it this step (where enter_stamp == t)
    // big tiles: (first, end) slot pairs, and global scratch for single
    // edges beyond the LDS of a workgroup
    int* big_list;
    int2* big_lane;             // [lane] {step, big tile} of the last step the lane's edge was in a big tile
    int* moved_at;              // [kMovedSlots] last step in which a workgroup hashed to the slot saw a vehicle move,
                                //   then in the same allocation the tile counters (tile_counters)
    unsigned long long* big_defer;   // admission items whose target lane is in a big tile: tile << 32 | item
    int tile_window;            // slots per tile window, or 0: chosen per step from tile_target
    int tile_target;            // tiles per step that run in one round of resident workgroups
    // traced re-run of a segment that starts at a multiple of trace_period:
    // record of step t at trace[(t % trace_period) * trace_stride + slot], so one
    // captured graph serves every segment
    TraceRec* trace;
    int trace_period;
    int trace_stride;
    int* nact_hist;
    char* big;
    int big_cap;                // vehicles per workgroup region
};

// k_tile_step's tile counters: after the movement stamps, 128-byte aligned
// (the stamps take 256 bytes), in the same allocation
__host__ __device__ inline int* tile_counters(const Dev& d) { return d.moved_at + kMovedSlots; }

// ---- per-tile working set -----------------------------------------------
struct TileBuf {
    float* x;
    float* v;
    uint32_t* vid;
    uint32_t* el;       // edge << 4 | lane (S_t)
    uint32_t* meta;
    int* nxt;
    int* pm;            // Phase 1: insertion point in the target lane's run | decision code << 16;
                        //   Phase 2: start of the post-change lane's run
    int* mpref;         // movers before index q (n + 1 entries)
    int* lml;           // last mover (low 16 bits) and last stayer (high 16 bits) at or before q, or -1
    int* rk;            // index of q's run (maximal group of one edge and lane in S_t)
    uint32_t* run_el;   // per run: edge << 4 | lane; run_el[nruns] = ~0
    int* run_st;        // per run: first index; run_st[nruns] = n
    int* nruns;         // [1]
    float* xn;          // Phase 2 position
    uint32_t* fl;       // Phase 2 flags
    uint32_t* pel;      // post-change (edge, lane), permuted to the new order
    int* inv;           // new order -> q
    // per-vehicle copies of its edge's constants, loaded with the vehicle so
    // that later phases find them in LDS
    float* L;           // edge length
    float* lim;         // edge speed limit; after Phase 2 the vehicle's new speed
    uint32_t* lbe;      // first global lane of the edge | its lanes << 24
    uint32_t* lbf;      // the same for the next edge (0 if none)
};

// lane words: first global lane (below 2^24) and lane count in one word
constexpr int kLaneBaseBits = 24;
__device__ inline int lw_base(uint32_t w) { return (int)(w & ((1u << kLaneBaseBits) - 1u)); }
__device__ inline int lw_lanes(uint32_t w) { return (int)(w >> kLaneBaseBits); }
__device__ inline int lastm_of(const int* lml, int i) { return (int)(short)(lml[i] & 0xFFFF); }
__device__ inline int lasts_of(const int* lml, int i) { return lml[i] >> 16; }

constexpr int kTileBytesPerVeh = 80;   // 20 four-byte arrays (plus a few words within the 64-byte slack)
__host__ __device__ inline size_t tile_bytes(int cap) { return (size_t)cap * kTileBytesPerVeh + 64; }

__device__ inline TileBuf carve(char* base, int cap) {
    TileBuf b;
    size_t o = 0;
    auto take = [&](size_t n) { char* p = base + o; o += n * 4; return p; };
    b.x = (float*)take(cap);
    b.v = (float*)take(cap);
    b.vid = (uint32_t*)take(cap);
    b.el = (uint32_t*)take(cap);
    b.meta = (uint32_t*)take(cap);
    b.nxt = (int*)take(cap);
    b.pm = (int*)take(cap);
    b.mpref = (int*)take(cap + 1);
    b.lml = (int*)take(cap);
    b.rk = (int*)take(cap);
    b.run_el = (uint32_t*)take(cap + 1);
    b.run_st = (int*)take(cap + 1);
    b.nruns = (int*)take(1);
    b.xn = (float*)take(cap);
    b.fl = (uint32_t*)take(cap);
    b.pel = (uint32_t*)take(cap);
    b.inv = (int*)take(cap);
    b.L = (float*)take(cap);
    b.lim = (float*)take(cap);
    b.lbe = (uint32_t*)take(cap);
    b.lbf = (uint32_t*)take(cap);
    return b;
}

// flags of Phase 2
constexpr uint32_t F_WHOLD = 1u, F_VEH = 2u;

// Index of the first run whose key is not below `key`, where key is a lane
// of the edge of run k0 or one past its last lane.  An edge has at most 8
// lanes, so that run lies within 8 runs of k0: a few independent LDS reads
// instead of a search of the tile.
__device__ inline int run_lower(const TileBuf& b, int nruns, int k0, uint32_t key) {
    int k = k0;
    if (key > b.run_el[k0]) {
#pragma unroll
        for (int j = 1; j <= 8; ++j) {
            const int kk = k0 + j;
            if (kk <= nruns && b.run_el[kk] < key) k = kk;
        }
        return k + 1;
    }
#pragma unroll
    for (int j = 1; j <= 8; ++j) {
        const int kk = k0 - j;
        if (kk >= 0 && b.run_el[kk] >= key) k = kk;
    }
    return k;
}

// first index in [lo, hi), part of one run, that does not precede (x, id)
// in the tile order (x descending, id descending)
__device__ inline int run_insert(const TileBuf& b, int lo, int hi, float x, uint32_t id) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const float x2 = b.x[mid];
        if ((x2 > x) || (x2 == x && b.vid[mid] > id)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ---- workgroup helpers ---------------------------------------------------
struct Scan4 {
    int s, a, b, c;     // s: sum; a, b, c: max
};

__device__ inline Scan4 scan4_op(Scan4 x, Scan4 y) {
    return Scan4{x.s + y.s, max(x.a, y.a), max(x.b, y.b), max(x.c, y.c)};
}

// Inclusive wavefront scans with DPP moves (register to register, no LDS
// round trip): Hillis-Steele over row shifts of 1, 2, 4 and 8 lanes within
// each row of 16, then the last lane of row 0 broadcast into row 1 and of
// row 2 into row 3 (row_bcast:15), then lane 31 into rows 2 and 3
// (row_bcast:31).  A lane whose source is outside its row, or whose row is
// masked off, takes the identity (the `old` operand).
constexpr int kDppRowShr = 0x110, kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;

__device__ inline int wave_incl_sum(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr + 1, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr + 2, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr + 4, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr + 8, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowBcast15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kDppRowBcast31, 0xc, 0xf, false);
    return x;
}

// the same for max with identity -1 (the values scanned are indices >= -1)
__device__ inline int wave_incl_max(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, kDppRowShr + 1, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, kDppRowShr + 2, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, kDppRowShr + 4, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, kDppRowShr + 8, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, kDppRowBcast15, 0xa, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, kDppRowBcast31, 0xc, 0xf, false));
    return x;
}

// exclusive workgroup scan of one Scan4 per thread (all NT threads take
// part); wsh: NT/64 Scan4 in LDS
template <int NT = kNT>
__device__ inline Scan4 wg_exclusive_scan4(Scan4 v, Scan4* wsh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    Scan4 inc;
    inc.s = wave_incl_sum(v.s);
    inc.a = wave_incl_max(v.a);
    inc.b = wave_incl_max(v.b);
    inc.c = wave_incl_max(v.c);
    if (lane == 63) wsh[wave] = inc;
    __syncthreads();
    Scan4 carry{0, -1, -1, -1};
    for (int w = 0; w < wave; ++w) carry = scan4_op(carry, wsh[w]);
    __syncthreads();
    Scan4 exc;
    exc.s = inc.s - v.s;
    exc.a = __builtin_amdgcn_update_dpp(-1, inc.a, kDppWaveShr1, 0xf, 0xf, false);   // lane 0 gets -1
    exc.b = __builtin_amdgcn_update_dpp(-1, inc.b, kDppWaveShr1, 0xf, 0xf, false);
    exc.c = __builtin_amdgcn_update_dpp(-1, inc.c, kDppWaveShr1, 0xf, 0xf, false);
    return scan4_op(carry, exc);
}

// Gridlock detector: a workgroup that saw a vehicle move stamps the step
// into one of kMovedSlots slots (spread so that thousands of workgroups do
// not store to one address), from an LDS flag (a register held across the
// kernel would spill in the tile kernel); call after a barrier that follows
// every write of the flag.
__device__ inline void publish_moved(const Dev& d, const int* smoved, int t) {
    if (threadIdx.x == 0 && *smoved) d.moved_at[blockIdx.x % kMovedSlots] = t;
}

// per-workgroup counter accumulation, flushed with one atomic per counter
struct CounterAcc {
    unsigned c[cNumCounters];
    __device__ void zero() {
        for (int k = 0; k < cNumCounters; ++k) c[k] = 0;
    }
};

// counters: per-thread registers -> wavefront sums -> LDS atomics -> one
// global atomic each.  The wavefront sum is a fixed-cost DPP reduction; an
// atomic on a per-thread value would be split by the compiler into a loop
// over the lanes holding a non-zero count, which at the end of a busy tile
// costs microseconds.  Counters that no lane of the wavefront touched are
// skipped on a ballot (all of them, where the kernel never updates one).
__device__ inline void flush_counters_lds(const Dev& d, const CounterAcc& acc, unsigned* shc) {
#pragma unroll
    for (int k = 0; k < cNumCounters; ++k) {
        if (__ballot(acc.c[k] != 0u) == 0ull) continue;   // uniform across the wavefront
        const unsigned s = __ockl_wfred_add_u32(acc.c[k]);
        if ((threadIdx.x & 63) == 0) atomicAdd(&shc[k], s);
    }
    __syncthreads();
    if (threadIdx.x < cNumCounters && shc[threadIdx.x])
        atomicAdd(&d.counters[threadIdx.x * kCounterCopies + (blockIdx.x % kCounterCopies)],
                  (unsigned long long)shc[threadIdx.x]);
}

__device__ inline bool lane_allowed(uint32_t meta, int nxt, int l) {
    return nxt < 0 || ((m_mask(meta) >> l) & 1u);
}

// ---- tile search ---------------------------------------------------------
// first slot s in [lo, hi) that starts an edge (s == 0 or edge differs from
// s - 1), or hi if none; every thread of the workgroup gets the answer
template <int NT>
__device__ inline int first_edge_start(const int32_t* edge, int lo, int hi, int* wsh) {
    constexpr int kW = NT / 64;
    for (int base = lo; base < hi; base += NT) {
        const int s = base + (int)threadIdx.x;
        bool f = false;
        if (s < hi) f = (s == 0) || (edge[s] != edge[s - 1]);
        const unsigned long long bal = __ballot(f);
        const int wave = threadIdx.x >> 6;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) wsh[wave] = bal ? (base + wave * 64 + (__ffsll((long long)bal) - 1)) : INT32_MAX;
        __syncthreads();
        int m = INT32_MAX;
        for (int w = 0; w < kW; ++w) m = min(m, wsh[w]);
        __syncthreads();
        if (m != INT32_MAX) return m;
    }
    return hi;
}

// Both ends of a tile in one pass over the slots [w0, w0 + NT): a0 = the
// first edge start in [w0, w1) (w1 if none), a1 = the first edge start at or
// after w1 (n if none).  Windows are at most NT / 2 slots, so the pass also
// covers NT / 2 slots past w1; a longer edge continues with first_edge_start.
struct TileSpan {   // a tile's slots [a0, a1) and the end of its window
    int a0, a1, w1;
};

template <int NT>
__device__ inline void tile_bounds(const int32_t* edge, int w0, int w1, int n, int* wsh2, int& a0, int& a1) {
    constexpr int kW = NT / 64;
    const int s = w0 + (int)threadIdx.x;
    const bool f = s < n && (s == 0 || edge[s] != edge[s - 1]);
    const bool in0 = f && s < w1, in1 = f && s >= w1;
    const unsigned long long b0 = __ballot(in0), b1 = __ballot(in1);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        wsh2[wave] = b0 ? (w0 + wave * 64 + (__ffsll((long long)b0) - 1)) : INT32_MAX;
        wsh2[kW + wave] = b1 ? (w0 + wave * 64 + (__ffsll((long long)b1) - 1)) : INT32_MAX;
    }
    __syncthreads();
    int m0 = INT32_MAX, m1 = INT32_MAX;
    for (int w = 0; w < kW; ++w) {
        m0 = min(m0, wsh2[w]);
        m1 = min(m1, wsh2[kW + w]);
    }
    __syncthreads();
    a0 = m0 == INT32_MAX ? w1 : m0;
    if (m1 != INT32_MAX) a1 = m1;
    else a1 = (w0 + NT >= n) ? n : first_edge_start<NT>(edge, w0 + NT, n, wsh2);
}

// ---- lane-change draws computed by the whole workgroup -------------------
// A task is one Philox block (vehicle q of the tile, stream, block index).
// Its 24-bit words are added into the vehicle's slot with an LDS atomic; the
// sums are integers, so the order of the additions does not matter and the
// result equals draw_uniform / draw_normal exactly.
struct DrawQ {
    uint32_t* task;   // [cap] q << 4 | stream << 2 | block
    int* n;           // [2] tasks listed in each round
    int cap;
};

__device__ inline uint32_t philox_words(uint64_t seed, int t, uint32_t rid, int stream, int blk) {
    const U64x4 r = philox4x64_10((uint64_t)(int64_t)t, rid, (uint64_t)stream, (uint64_t)blk, seed, 0);
    if (stream == 1) return (uint32_t)(r.w[0] >> 40);
    return (uint32_t)((r.w[0] >> 40) + (r.w[1] >> 40) + (r.w[2] >> 40) + (r.w[3] >> 40));
}

// list one task; a full list computes it in place
__device__ inline void draw_task(const DrawQ& dq, int round, uint32_t rid, int q, int stream, int blk, int* slot,
                                 uint64_t seed, int t) {
    const int k = atomicAdd(&dq.n[round], 1);
    if (k < dq.cap) dq.task[k] = ((uint32_t)q << 4) | ((uint32_t)stream << 2) | (uint32_t)blk;
    else atomicAdd(&slot[q], (int)philox_words(seed, t, rid, stream, blk));
}

// The counter id of a vehicle's draws: its id within its scenario (the
// scenario of an ensemble member is its edge's copy of the network).
__device__ inline uint32_t draw_id(const Dev& d, uint32_t vid, int e) {
    return vid - (uint32_t)d.scen_voff[e / d.edge_period];
}

template <int NT>
__device__ inline void draw_run(const Dev& d, const DrawQ& dq, int round, int t, const TileBuf& b, int* u1,
                                int* na, int* nb) {
    const int nt = min(dq.n[round], dq.cap);
    for (int i = threadIdx.x; i < nt; i += NT) {
        const uint32_t tk = dq.task[i];
        const int q = (int)(tk >> 4), st = (int)((tk >> 2) & 3u), blk = (int)(tk & 3u);
        int* slot = st == 1 ? u1 : (st == 2 ? na : nb);
        const uint32_t rid = draw_id(d, b.vid[q], (int)(b.el[q] >> 4));
        atomicAdd(&slot[q], (int)philox_words(d.seed, t, rid, st, blk));
    }
}

__device__ inline float uniform_of_word(uint32_t w) {
    return (float)w * 5.9604644775390625e-08f;   // * 2^-24, exact
}

// Eqs. (3)-(4): G >= max(c + eps, 0).  eps lies in [-6, 6] (Irwin-Hall of
// twelve uniforms minus 6) and binary32 rounding is monotone, so the noise
// decides only when G is within 6 m of c.
constexpr int kGapNo = 0, kGapYes = 1, kGapDraw = 2;
constexpr int kPending = 2, kDrawA = 4, kDrawB = 8;   // Phase 1 decision codes (b.pm >> 16)

__device__ inline int gap_outcome(float G, float c) {
    if (G < c - 6.0f) return kGapNo;
    if (G >= c + 6.0f && G >= 0.0f) return kGapYes;
    return kGapDraw;
}

__device__ inline bool gap_with_noise(float G, float c, int word_sum) {
    const int32_t z = (int32_t)((int64_t)(uint32_t)word_sum - 6ll * 16777216ll);
    const float g = c + (float)z * 5.9604644775390625e-08f;
    const float need = g > 0.0f ? g : 0.0f;
    return G >= need;
}

// The lane-change decision of vehicle q once its noise is drawn (Eqs. (3)-(4)):
// its decision code becomes 0 or 1.
__device__ inline void finish_pending(const TileBuf& b, int q, int dir, const float* Ga, const float* ca,
                                      const float* Gb, const float* cb, const int* na, const int* nb,
                                      CounterAcc& acc) {
    const int code = b.pm[q] >> 16;
    if (!(code & kPending)) return;
    bool ok = true;
    if (code & kDrawA) ok = gap_with_noise(Ga[q], ca[q], na[q]);
    if (code & kDrawB) ok = ok && gap_with_noise(Gb[q], cb[q], nb[q]);
    int moved = 0;
    if (ok) {
        moved = 1;
        acc.c[cLaneChanges]++;
        const uint32_t m = b.meta[q];
        const int lp = (int)(b.el[q] & 15u) + dir;
        if (lane_allowed(m, b.nxt[q], lp)) b.meta[q] = m & ~((1u << 4) | (127u << 8));
    }
    b.pm[q] = (b.pm[q] & 0xFFFF) | (moved << 16);
}

// ---- Phases 1-2 for one tile ----------------------------------------------
// kSpread: the per-driver limits may be on (a kernel of its own, so that the
// common case carries none of their code)
template <int NT, bool kSpread>
__device__ inline void process_tile(const Dev& d, const TileBuf& b, int a0, int n, int t, int par,
                                    CounterAcc& acc, Scan4* wsh4, const ClassParams* scp, const DrawQ& dq,
                                    int* smoved) {
    const Slots S = d.s[par];
    const int tid = threadIdx.x;
    const int dir = (t % 2 == 0) ? -1 : 1;

    // Phase 1 keeps its scratch in arrays that the scans fill later.  Few
    // vehicles need a Philox draw, and a block costs thousands of cycles, so
    // a wavefront in which one lane draws would make the other 63 wait.
    // Instead the draws are listed as tasks and computed by the whole
    // workgroup at once, in two rounds: the uniforms of Eq. (2), listed while
    // S_t is loaded, then the noise of Eqs. (3)-(4), whose need depends on the
    // mandatory flag.
    int* const u1 = b.pm;                         // Eq. (2) uniform words (read before Phase 1 writes pm)
    int* const na = b.mpref;                      // noise word sums, leading side (scratch until the scans)
    int* const nb = b.lml;                        // noise word sums, lagging side
    float* const Ga = b.xn;                       // gaps and critical gaps of pending decisions
    float* const ca = (float*)b.fl;               // (scratch until Phase 2)
    float* const Gb = (float*)b.pel;
    float* const cb = (float*)b.inv;

    // load S_t (coalesced) and list the Eq. (2) draws
    for (int q = tid; q < n; q += NT) {
        const int s = a0 + q;
        const uint32_t m = S.meta[s];
        const int e = S.edge[s], f = S.nxt[s];
        const float x = S.x[s];
        b.x[q] = x;
        b.v[q] = S.v[s];
        b.vid[q] = S.vid[s];
        b.el[q] = ((uint32_t)e << 4) | (uint32_t)m_lane(m);
        b.meta[q] = m;
        b.nxt[q] = f;
        const EdgeC ce = d.ec[e];
        const EdgeC cf = f >= 0 ? d.ec[f] : EdgeC{0.0f, 0.0f, 0, 0};
        const float L = ce.L;
        b.L[q] = L;
        b.lbe[q] = (uint32_t)ce.lane_base | ((uint32_t)ce.lanes << kLaneBaseBits);
        b.lbf[q] = (uint32_t)cf.lane_base | ((uint32_t)cf.lanes << kLaneBaseBits);
        b.lim[q] = ce.lim;
        u1[q] = 0;
        na[q] = 0;
        nb[q] = 0;
        if (!m_held(m) && !m_mand(m) && !lane_allowed(m, f, m_lane(m))) {   // Eq. (2) may trigger
            const float dd = L - x;
            if (dd > kX0) {
                const float dm = dd - kX0;
                if (dm * dm < kZCut) draw_task(dq, 0, draw_id(d, b.vid[q], e), q, 1, 0, u1, d.seed, t);
            }
        }
    }
    __syncthreads();
    draw_run<NT>(d, dq, 0, t, b, u1, na, nb);
    if (kSpread && d.v0_spread != 0.0f)   // each driver's own limit on its edge (Sec. IV)
        for (int q = tid; q < n; q += NT) {
            const int e = (int)(b.el[q] >> 4);
            b.lim[q] = driver_limit(b.lim[q], d.v0_spread, d.seed, e, d.edge_period, draw_id(d, b.vid[q], e));
        }

    // ---- runs of S_t (tile order: edge, lane, then x and id descending)
    {
        const int chunk = (n + NT - 1) / NT;
        const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
        int loc = 0;
        for (int q = lo; q < hi; ++q) loc += (q == 0 || b.el[q] != b.el[q - 1]) ? 1 : 0;
        const Scan4 r = wg_exclusive_scan4<NT>(Scan4{loc, -1, -1, -1}, wsh4);
        int k = r.s - 1;
        for (int q = lo; q < hi; ++q) {
            if (q == 0 || b.el[q] != b.el[q - 1]) {
                ++k;
                b.run_el[k] = b.el[q];
                b.run_st[k] = q;
            }
            b.rk[q] = k;
        }
        if (hi == n && lo < hi) {
            b.run_el[k + 1] = ~0u;
            b.run_st[k + 1] = n;
            *b.nruns = k + 1;
        }
        if (n == 0 && tid == 0) {
            b.run_el[0] = ~0u;
            b.run_st[0] = 0;
            *b.nruns = 0;
        }
    }
    __syncthreads();
    const int nruns = *b.nruns;

    // ---- Phase 1: lane-change decisions (Eqs. (2)-(4)) against S_t
    for (int q = tid; q < n; q += NT) {
        uint32_t m = b.meta[q];
        int moved = 0, pos = 0;
        if (!m_held(m)) {
            const uint32_t el = b.el[q];
            const int l = (int)(el & 15u);
            const int f = b.nxt[q];
            const float xi = b.x[q], vi = b.v[q];
            const bool allowed_l = lane_allowed(m, f, l);
            const ClassParams cpi = scp[m_cls(m)];
            if (!allowed_l && !m_mand(m)) {                              // Eq. (2)
                const float dd = b.L[q] - xi;
                bool trig = false;
                if (dd <= kX0) {
                    trig = true;
                } else {
                    const float dm = dd - kX0;
                    const float z = dm * dm;
                    if (z < kZCut && uniform_of_word((uint32_t)u1[q]) < exp_eq2(-z)) trig = true;
                }
                if (trig) {
                    m |= 1u << 4;
                    acc.c[cMandTriggers]++;
                }
            }
            const int lp = l + dir;
            if (lp >= 0 && lp < lw_lanes(b.lbe[q])) {
                const uint32_t elp = (el & ~15u) | (uint32_t)lp;
                const int kp = run_lower(b, nruns, b.rk[q], elp);
                pos = b.run_st[kp];
                if (b.run_el[kp] == elp) pos = run_insert(b, pos, b.run_st[kp + 1], xi, b.vid[q]);
                const int la = (pos > 0 && b.el[pos - 1] == elp) ? pos - 1 : -1;
                const int lb = (pos < n && b.el[pos] == elp) ? pos : -1;
                const uint32_t mask = f < 0 ? 0xFFu : m_mask(m);
                bool desire = !allowed_l && (lane_distance(mask, lp) < lane_distance(mask, l));
                const bool allowed_lp = lane_allowed(m, f, lp);
                const int lc = (q > 0 && b.el[q - 1] == el) ? q - 1 : -1;
                // with no leader in its own lane a vehicle already has the free
                // acceleration, which no leader in the other lane can beat
                // (Eq. (1) only subtracts from it): no incentive to compute
                if (!desire && allowed_lp && !(m_mand(m) && !allowed_l) && lc >= 0) {
                    const float v0 = cpi.v0f * b.lim[q];
                    unsigned br = 0;
                    float acc_cur, acc_new;
                    if (lc >= 0) {
                        const float s = (b.x[lc] - scp[m_cls(b.meta[lc])].len) - xi;
                        acc_cur = idm_acc(vi, v0, b.v[lc], s, cpi, kVeh, br);
                    } else {
                        acc_cur = idm_acc(vi, v0, 0.0f, 0.0f, cpi, kFree, br);
                    }
                    if (la >= 0) {
                        const float s = (b.x[la] - scp[m_cls(b.meta[la])].len) - xi;
                        acc_new = idm_acc(vi, v0, b.v[la], s, cpi, kVeh, br);
                    } else {
                        acc_new = idm_acc(vi, v0, 0.0f, 0.0f, cpi, kFree, br);
                    }
                    desire = (acc_new - acc_cur) > kIncentive;
                }
                if (desire) {                                            // Eqs. (3)-(4)
                    const float g0 = desired_gap(vi);
                    // anticipation times, loaded only by the vehicles that get here
                    const float ai = d.alpha[b.vid[q]];
                    const float a_la = la >= 0 ? d.alpha[b.vid[la]] : 0.0f;
                    const float a_lb = lb >= 0 ? d.alpha[b.vid[lb]] : 0.0f;
                    int ra = kGapYes, rb = kGapYes;
                    if (la >= 0) {
                        const float G = (b.x[la] - scp[m_cls(b.meta[la])].len) - xi;
                        const float c = crit_gap(g0, a_la, vi, ai, b.v[la]);
                        ra = gap_outcome(G, c);
                        Ga[q] = G;
                        ca[q] = c;
                    }
                    if (lb >= 0) {
                        const float G = (xi - cpi.len) - b.x[lb];
                        const float c = crit_gap(g0, ai, vi, a_lb, b.v[lb]);
                        rb = gap_outcome(G, c);
                        Gb[q] = G;
                        cb[q] = c;
                    }
                    if (ra != kGapNo && rb != kGapNo) {
                        if (ra == kGapYes && rb == kGapYes) {
                            moved = 1;
                            acc.c[cLaneChanges]++;
                            if (allowed_lp) m &= ~((1u << 4) | (127u << 8));   // mand = 0, ww = 0
                        } else {                                 // decided by the noise
                            moved = kPending | (ra == kGapDraw ? kDrawA : 0) | (rb == kGapDraw ? kDrawB : 0);
                            const uint32_t rid = draw_id(d, b.vid[q], (int)(el >> 4));
                            for (int k = 0; k < 3; ++k) {
                                if (ra == kGapDraw) draw_task(dq, 1, rid, q, 2, k, na, d.seed, t);
                                if (rb == kGapDraw) draw_task(dq, 1, rid, q, 3, k, nb, d.seed, t);
                            }
                        }
                    }
                }
            }
        }
        b.pm[q] = pos | (moved << 16);   // u1[q] (the same word) was read above
        // only this vehicle's own mandatory/wait bits change; its class bits,
        // which neighbours read, stay the same
        b.meta[q] = m;
    }
    __syncthreads();
    draw_run<NT>(d, dq, 1, t, b, u1, na, nb);
    __syncthreads();
    if (tid < 2) dq.n[tid] = 0;   // lists of the next tile (several barriers away)

    // ---- mover prefix sums and last-mover / last-stayer / run-start maxima
    {
        const int chunk = (n + NT - 1) / NT;
        const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
        Scan4 loc{0, -1, -1, -1};
        for (int q = lo; q < hi; ++q) {
            // the decisions waiting for noise are finished by the thread that scans them
            finish_pending(b, q, dir, Ga, ca, Gb, cb, na, nb, acc);
            const int mv = b.pm[q] >> 16;
            loc.s += mv;
            if (mv) loc.a = q; else loc.b = q;
        }
        Scan4 run = wg_exclusive_scan4<NT>(loc, wsh4);
        for (int q = lo; q < hi; ++q) {
            const int mv = b.pm[q] >> 16;
            b.mpref[q] = run.s;
            run.s += mv;
            if (mv) run.a = q; else run.b = q;
            b.lml[q] = (int)(((uint32_t)run.a & 0xFFFFu) | ((uint32_t)run.b << 16));
        }
        if (hi == n && lo < hi) b.mpref[n] = run.s;
        if (n == 0 && tid == 0) b.mpref[0] = 0;
    }
    for (int q = tid; q < n; q += NT) b.inv[q] = -1;
    __syncthreads();

    // ---- Phase 2: leader on the post-change lane, Eq. (1), integration
    for (int q = tid; q < n; q += NT) {
        const uint32_t el = b.el[q];
        const int e = (int)(el >> 4), l = (int)(el & 15u);
        const int mv = b.pm[q] >> 16;
        const int lam = mv ? l + dir : l;
        const uint32_t elam = (el & ~15u) | (uint32_t)lam;
        const float xi = b.x[q], vi = b.v[q];
        const uint32_t id = b.vid[q];
        uint32_t m = b.meta[q];
        const int f = b.nxt[q];
        const int lanes_e = lw_lanes(b.lbe[q]);
        const uint32_t e0 = el & ~15u;
        // leader and position in the post-change order.  On an edge where no
        // vehicle changes lanes (most edges of a step) both stay as in S_t:
        // the leader is the vehicle before in the same run, the position q.
        const int k0 = b.rk[q];
        const int rs = b.run_st[k0];
        // the start-of-step rear of the lane it would look into with no leader
        // on the tile, loaded now so that the round trip overlaps the leader
        // search: for a lane's first vehicle and for the movers, the vehicles
        // that most often have none (any other loads it where it is used)
        const int look_i = lw_base(b.lbf[q]) + min(lam, lw_lanes(b.lbf[q]) - 1);
        const bool pre = f >= 0 && (mv != 0 || q == rs);
        LaneRear rp{0.0f, 0.0f, -1, 0u};
        if (pre) rp = d.rear[look_i];
        int j, newpos, lane_start;
        bool quiet = false;
        if (!mv) {
            const int es_q = b.run_st[run_lower(b, nruns, k0, e0)];
            const int ee_q = b.run_st[run_lower(b, nruns, k0, e0 + 16u)];   // first slot of the next edge
            quiet = b.mpref[ee_q] == b.mpref[es_q];
            if (quiet) {
                j = q > rs ? q - 1 : -1;
                newpos = q;
                lane_start = rs;
            }
        }
        if (!quiet) {
            // leader candidates and rank in the post-change lane
            int c1 = -1, c2 = -1, rank;
            const int mu = lam - dir;   // lane whose movers enter lam
            int sl;                     // start of lam's run in S_t (lower bound if empty)
            if (!mv) {
                sl = rs;
                if (q > 0 && lasts_of(b.lml, q - 1) >= rs) c1 = lasts_of(b.lml, q - 1);
                int mov_ahead = 0;
                if (mu >= 0 && mu < lanes_e) {
                    const uint32_t emu = e0 | (uint32_t)mu;
                    const int kmu = run_lower(b, nruns, k0, emu);
                    const int st = b.run_st[kmu];
                    const int p2 = (b.run_el[kmu] == emu) ? run_insert(b, st, b.run_st[kmu + 1], xi, id) : st;
                    if (p2 > 0 && lastm_of(b.lml, p2 - 1) >= st) c2 = lastm_of(b.lml, p2 - 1);
                    mov_ahead = b.mpref[p2] - b.mpref[st];
                }
                rank = ((q - rs) - (b.mpref[q] - b.mpref[rs])) + mov_ahead;
            } else {
                const int p = b.pm[q] & 0xFFFF;
                const int st = b.run_st[run_lower(b, nruns, k0, elam)];
                sl = st;
                if (p > 0 && lasts_of(b.lml, p - 1) >= st) c1 = lasts_of(b.lml, p - 1);
                if (q > 0 && lastm_of(b.lml, q - 1) >= rs) c2 = lastm_of(b.lml, q - 1);
                rank = ((p - st) - (b.mpref[p] - b.mpref[st])) + (b.mpref[q] - b.mpref[rs]);
            }
            j = c1;
            if (c2 >= 0) {
                if (j < 0) j = c2;
                else if (b.x[c2] < b.x[j] || (b.x[c2] == b.x[j] && b.vid[c2] < b.vid[j])) j = c2;
            }
            // post-change vehicles of this edge in lanes below lam
            const int es = b.run_st[run_lower(b, nruns, k0, e0)];
            int below = sl - es;
            if (dir < 0) {
                const int ee = b.run_st[run_lower(b, nruns, k0, elam + 1)];
                below += b.mpref[ee] - b.mpref[sl];
            } else if (lam >= 1) {
                const int s0 = b.run_st[run_lower(b, nruns, k0, elam - 1)];
                below -= b.mpref[sl] - b.mpref[s0];
            }
            newpos = es + below + rank;
            lane_start = es + below;
        }
        if (newpos < 0 || newpos >= n) {   // cannot happen if the layout is consistent
            atomicOr(&d.ctl->err, kErrNewPos);
            continue;
        }
        b.pm[q] = lane_start;   // start of the post-change lane's run (pm[q] is not read again)

        // kind and gap (A1-A8, A17)
        const ClassParams cpi = scp[m_cls(m)];
        const bool allowed_l = lane_allowed(m, f, lam);
        int kind;
        int partner = -1, look_gl = -1;
        float s = 0.0f, vl = 0.0f, rear_j = 0.0f;
        if (j >= 0) {
            kind = kVeh;
            partner = (int)b.vid[j];
            rear_j = b.x[j] - scp[m_cls(b.meta[j])].len;
            s = rear_j - xi;
            vl = b.v[j];
        } else if (f < 0) {
            kind = kFree;
        } else if (m_mand(m) && !allowed_l && m_ww(m) < kPatience) {
            kind = kStop;
            s = b.L[q] - xi;
            vl = 0.0f;
        } else {
            const LaneRear r = pre ? rp : d.rear[look_i];
            if (r.stamp == t) {
                kind = kLook;
                s = (b.L[q] - xi) + r.xm;
                vl = r.v;
                partner = (int)r.vid;
                look_gl = look_i;
            } else {
                kind = kFree;
            }
        }
        unsigned br = 0;
        const float v0 = cpi.v0f * b.lim[q];
        const float a = idm_acc(vi, v0, vl, s, cpi, kind, br);
        const float dt = d.dt;
        float vnew = vi + (a * dt);
        float xnew;
        uint32_t tb = br;
        if (vnew >= 0.0f) {
            xnew = (xi + (vi * dt)) + ((0.5f * a) * (dt * dt));
        } else {
            xnew = xi - ((vi * vi) / (2.0f * a));
            vnew = 0.0f;
            acc.c[cStopBranch]++;
            tb |= TB_B;
        }
        uint32_t fl = 0;
        if (kind == kVeh && xnew > rear_j) {
            xnew = rear_j;
            acc.c[cClamp]++;
            tb |= TB_C;
        }
        if (f >= 0 && !allowed_l && m_ww(m) < kPatience && xnew >= b.L[q]) {
            xnew = b.L[q];
            vnew = 0.0f;
            m = (m | (1u << 4));
            m = (m & ~(127u << 8)) | ((uint32_t)(m_ww(m) + 1) << 8);
            fl |= F_WHOLD;
            acc.c[cWrongLaneHolds]++;
            tb |= TB_W;
        }
        m = m_set_lane(m, lam);
        // write the post-step record in the post-change order.  newpos stays
        // inside this edge's slot range, so the edge id stored at every slot
        // is unchanged and other workgroups may read it concurrently.
        const int dst = a0 + newpos;
        S.x[dst] = xnew;
        S.v[dst] = vnew;
        S.vid[dst] = id;
        S.edge[dst] = e;
        S.meta[dst] = m;
        S.nxt[dst] = f;
        S.gl[dst] = lw_base(b.lbe[q]) + lam;
        b.xn[q] = xnew;
        b.fl[q] = fl;
        b.lim[q] = vnew;   // lim[q] is read only by this thread, above
        if (d.trace) {
            TraceRec tr;
            tr.vid = id;
            tr.partner = partner;
            tr.x = xi;
            tr.v = vi;
            tr.s = s;
            tr.vl = vl;
            tr.xn = xnew;
            tr.edge = e;
            tr.kb = (uint32_t)kind | (tb << 8);
            tr.look_gl = look_gl;
            d.trace[(size_t)(t % d.trace_period) * d.trace_stride + dst] = tr;
        }
        b.pel[newpos] = elam;
        b.inv[newpos] = q;
    }
    __syncthreads();

    // ---- lane fronts (requests) and rears (admission and scatter tables)
    // (and, for the gridlock detector, whether any vehicle changed position,
    // x_new against x of slot index r, or lane: the movers' count mpref[n])
    bool moved = tid == 0 && n > 0 && b.mpref[n] > 0;
    for (int r = tid; r < n; r += NT) {
        moved = moved || (b.xn[r] != b.x[r]);
        const uint32_t el = b.pel[r];
        const bool front = (r == 0) || (b.pel[r - 1] != el);
        const bool rear = (r == n - 1) || (b.pel[r + 1] != el);
        if (front || rear) {
            const int q = b.inv[r];
            if (q < 0 || q >= n) {
                atomicOr(&d.ctl->err, kErrPermutation);
            } else {
                const int lam = (int)(el & 15u);
                const int gl = lw_base(b.lbe[q]) + lam;
                const float xnew = b.xn[q];
                if (rear) {
                    const int fr = b.pm[q];
                    LanePost lp;
                    lp.stamp = t;
                    lp.start = a0 + fr;
                    lp.cnt = r - fr + 1;
                    lp.rear_xm = xnew - scp[m_cls(b.meta[q])].len;
                    d.post[gl] = lp;
                }
                if (front && xnew >= b.L[q] && !(b.fl[q] & F_WHOLD)) {
                    const int f = b.nxt[q];
                    const float xo = b.x[q];
                    Outbox ob;
                    ob.stamp = t;
                    ob.elig = 0;
                    ob.slot = a0 + r;
                    ob.vid = b.vid[q];
                    ob.phi = (xnew == xo) ? 0.0f : (b.L[q] - xo) / (xnew - xo);
                    ob.v = b.lim[q];
                    ob.nxt = f;
                    if (f < 0) {
                        ob.target = -1;
                        ob.xp = 0.0f;
                        ob.key = 0;
                        ob.tl_cls = 0;
                    } else {
                        const int tl = min(lam, lw_lanes(b.lbf[q]) - 1);
                        ob.target = lw_base(b.lbf[q]) + tl;
                        ob.tl_cls = (uint32_t)tl | (m_cls(b.meta[q]) << 8);
                        ob.xp = xnew - b.L[q];
                        const int hs = m_held(b.meta[q]) ? d.held_since[ob.vid] : t;
                        ob.key = ((unsigned long long)(uint32_t)hs << 32) | ob.vid;
                    }
                    d.outbox[gl] = ob;
                    d.req_stamp[gl] = t;
                }
            }
        }
    }
    if (__ballot(moved) && (tid & 63) == 0) *smoved = 1;
    __syncthreads();
}

// The lanes of a big tile's edges, stamped with the step and the tile's index
// in the big-tile list: admission leaves requests into them to the
// workgroup of that tile, which writes their post-move rears.
template <int NT>
__device__ inline void mark_big_lanes(const Dev& d, const int32_t* edge, int a0, int a1, int t, int k) {
    for (int s = a0 + (int)threadIdx.x; s < a1; s += NT) {
        const int e = edge[s];
        if (s == a0 || edge[s - 1] != e) {
            const EdgeC c = d.ec[e];
            for (int l = 0; l < c.lanes; ++l) d.big_lane[c.lane_base + l] = make_int2(t, k);
        }
    }
}

// Tile window of a step with n active vehicles: fixed by the schedule, or
// (0) chosen for the fewest rounds of the tile workgroups: a workgroup
// runs its tiles one after another, so the step lasts as many tile chains as
// the busiest workgroup has tiles.  R = the fewest rounds that windows of at
// most kTileWindowAuto slots allow; the window is the smallest multiple of
// 16 slots (at least kTileWindowMin) whose tiles fit in R rounds, since
// larger windows make larger tiles and more of them above the LDS cap.
__device__ inline int tile_window(const Dev& d, int n) {
    int W = d.tile_window;
    if (W == 0) {
        const long long tgt = gridDim.x;   // the tile workgroups (persistent: all resident)
        const long long R = max(1LL, ((long long)n + kTileWindowAuto * tgt - 1) / (kTileWindowAuto * tgt));
        const int w = (int)(((long long)n + R * tgt - 1) / (R * tgt));
        W = max(kTileWindowMin, (w + 15) / 16 * 16);
    }
    return W;
}

// Small tiles (<= kTileCapLds vehicles) in 256-thread workgroups; larger
// tiles go to a list for k_big_admit.
template <bool kSpread>
__device__ inline void tile_step(const Dev& d) {
    __shared__ __align__(16) char lds[kTileCapLds * kTileBytesPerVeh + 64];
    __shared__ Scan4 wsh4[kTileNT / 64];
    __shared__ int wsh[2 * (kTileNT / 64)];
    __shared__ unsigned shc[cNumCounters];
    __shared__ ClassParams scp[16];
    __shared__ uint32_t dtask[kTileDrawTasks];
    __shared__ int dcount[2];
    __shared__ int smoved;                      // gridlock detector: a vehicle of this workgroup moved
    __shared__ int snext;                       // the workgroup's next tile
    const DrawQ dq{dtask, dcount, kTileDrawTasks};
    if (threadIdx.x < cNumCounters) shc[threadIdx.x] = 0;
    if (threadIdx.x < 2) dcount[threadIdx.x] = 0;
    if (threadIdx.x == 0) smoved = 0;
    if (threadIdx.x < 16) scp[threadIdx.x] = d.cp[threadIdx.x];
    const StepHead sh = step_head(d.ctl);
    const int t = sh.t_a, par = t & 1;
    const int n = par ? sh.n1 : sh.n0;
    CounterAcc acc;
    acc.zero();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        atomicAdd(&d.counters[cActiveSum * kCounterCopies], (unsigned long long)n);
        // the later kernels of this step read t_b; lists of the next step
        // are unused during this one
        d.ctl->t_b = t;
        d.ctl->n_big[par ^ 1] = 0;
        d.ctl->big_done = 0;
        d.ctl->n_defer = 0;
        if (d.trace) d.nact_hist[t % d.trace_period] = n;
    }
    // the next step's tile counters (this step's were cleared by the previous one)
    if (blockIdx.x == 0 && threadIdx.x < kTileGroups)
        tile_counters(d)[((par ^ 1) * kTileGroups + (int)threadIdx.x) * kTileCtrStride] = 0;
    __syncthreads();
    // a tile is the set of edges whose first slot lies in one window
    const int W = tile_window(d, n);
    const int ntile = (n + W - 1) / W;
    const int32_t* edge = d.s[par].edge;
    // A tile is the set of edges whose first slot lies in one window: its
    // bounds (run_tile), then its phases or its listing as a big tile (do_tile)
    auto run_tile = [&](int k) {
        const int w0 = k * W, w1 = min(n, w0 + W);
        int a0, a1;
        tile_bounds<kTileNT>(edge, w0, w1, n, wsh, a0, a1);
        return TileSpan{a0, a1, w1};
    };
    auto do_tile = [&](const TileSpan& sp) {
        const int a0 = sp.a0, a1 = sp.a1;
        if (a0 >= sp.w1) return;   // window inside one long edge: handled by an earlier tile
        const int cnt = a1 - a0;
        if (cnt > d.big_cap) {     // more vehicles than the edges can physically hold
            if (threadIdx.x == 0) atomicOr(&d.ctl->err, kErrTileTooBig);
            return;
        }
        if (cnt <= kTileCapLds) {
            process_tile<kTileNT, kSpread>(d, carve(lds, kTileCapLds), a0, cnt, t, par, acc, wsh4, scp, dq, &smoved);
        } else {
            if (threadIdx.x == 0) {
                const int q = atomicAdd(&d.ctl->n_big[par], 1);
                d.big_list[2 * q] = a0;
                d.big_list[2 * q + 1] = a1;
                wsh[0] = q;
            }
            __syncthreads();
            mark_big_lanes<kTileNT>(d, edge, a0, a1, t, wsh[0]);
            __syncthreads();                        // wsh is reused by the next tile
        }
    };
    // A workgroup's first tile is its index.  With few rounds per step each
    // later one is G further (G the workgroups).  With many, the imbalance of
    // tile lengths adds up over the rounds, so the later tiles are split into
    // kTileGroups groups (tile G + g + j * groups), each handed out by a
    // counter of its own to the workgroups of index g modulo the groups: a
    // workgroup whose tiles ran short takes the next, and each counter sees
    // one workgroup in eight.  The counter is read before the bounds probe,
    // whose loads its round trip overlaps, and the index is shared after the
    // probe (which begins with a barrier, so every thread has read the
    // previous one).
    const int G = (int)gridDim.x;
    if (ntile > kTileCtrRounds * G) {
        const int ng = min(kTileGroups, G);
        const int grp = (int)blockIdx.x % ng;
        int* const ctr = tile_counters(d) + (par * kTileGroups + grp) * kTileCtrStride;
        int k = blockIdx.x;
        while (k < ntile) {
            int nk = 0;
            if (threadIdx.x == 0) nk = G + grp + ng * atomicAdd(ctr, 1);
            const TileSpan sp = run_tile(k);
            if (threadIdx.x == 0) snext = nk;
            do_tile(sp);
            __syncthreads();                        // snext written
            k = __builtin_amdgcn_readfirstlane(snext);
        }
    } else {
        for (int k = blockIdx.x; k < ntile; k += G) do_tile(run_tile(k));
    }
    flush_counters_lds(d, acc, shc);
    publish_moved(d, &smoved, t);
}

// six workgroups per CU: at most 80 VGPRs, which the kernel fits without spills
__global__ void __launch_bounds__(kTileNT) __attribute__((amdgpu_waves_per_eu(6))) k_tile_step(Dev d) {
    tile_step<false>(d);
}
// the same with per-driver free-flow limits (v0_spread > 0)
__global__ void __launch_bounds__(kTileNT) __attribute__((amdgpu_waves_per_eu(6))) k_tile_step_v0spread(Dev d) {
    tile_step<true>(d);
}

// Tiles above kTileCapLds: 1,024-thread workgroups with kBigCapLds vehicles
// of LDS; a tile is cut at edge boundaries into pieces that fit, and only a
// single edge larger than the LDS runs from the global-memory scratch.
__device__ __forceinline__ void big_tiles(const Dev& d, int t, int par, int nbig) {
    __shared__ __align__(16) char lds[kBigCapLds * kTileBytesPerVeh + 64];
    __shared__ Scan4 wsh4[kBigNT / 64];
    __shared__ int wsh[kBigNT / 64];
    __shared__ unsigned shc[cNumCounters];
    __shared__ ClassParams scp[16];
    __shared__ uint32_t dtask[2 * kBigNT];
    __shared__ int dcount[2];
    __shared__ int smoved;                      // gridlock detector: a vehicle of this workgroup moved
    const DrawQ dq{dtask, dcount, 2 * kBigNT};
    if (threadIdx.x < cNumCounters) shc[threadIdx.x] = 0;
    if (threadIdx.x < 2) dcount[threadIdx.x] = 0;
    if (threadIdx.x == 0) smoved = 0;
    if (threadIdx.x < 16) scp[threadIdx.x] = d.cp[threadIdx.x];
    __syncthreads();
    const int32_t* edge = d.s[par].edge;
    CounterAcc acc;
    acc.zero();
    for (int k = blockIdx.x; k < nbig; k += gridDim.x) {
        const int a0 = d.big_list[2 * k], a1 = d.big_list[2 * k + 1];
        int pos = a0;
        while (pos < a1) {
            const int lim = min(a1, pos + kBigCapLds);
            int end;
            if (lim == a1) {
                end = a1;
            } else {
                // last edge start in (pos, lim]
                end = -1;
                for (int base = lim; base > pos && end < 0; base -= kBigNT) {
                    const int s = base - (int)threadIdx.x;
                    const bool f = (s > pos) && (s < a1) && edge[s] != edge[s - 1];
                    const unsigned long long bal = __ballot(f);
                    const int wave = threadIdx.x >> 6;
                    __syncthreads();
                    if ((threadIdx.x & 63) == 0) wsh[wave] = bal ? (base - wave * 64 - (__ffsll((long long)bal) - 1)) : -1;
                    __syncthreads();
                    int m = -1;
                    for (int w = 0; w < kBigNT / 64; ++w) m = max(m, wsh[w]);
                    __syncthreads();
                    end = m;
                }
                if (end < 0) end = first_edge_start<kBigNT>(edge, lim, a1, wsh);   // one edge beyond the LDS
            }
            const int cnt = end - pos;
            if (threadIdx.x == 0) atomicAdd(&d.ctl->big_updates, (unsigned long long)cnt);
            if (cnt <= kBigCapLds) {
                process_tile<kBigNT, true>(d, carve(lds, kBigCapLds), pos, cnt, t, par, acc, wsh4, scp, dq, &smoved);
            } else {
                char* mine = d.big + (size_t)blockIdx.x * tile_bytes(d.big_cap);
                process_tile<kBigNT, true>(d, carve(mine, d.big_cap), pos, cnt, t, par, acc, wsh4, scp, dq, &smoved);
            }
            pos = end;
        }
    }
    flush_counters_lds(d, acc, shc);
    publish_moved(d, &smoved, t);
}

// ---- admission -------------------------------------------------------------
__device__ inline bool transfer_eligible(const Dev& d, const Outbox& ob, int t) {
    const LanePost p = d.post[ob.target];
    return p.stamp != t || (p.rear_xm - ob.xp >= 0.0f);
}

// An eligible request lowers the lane's 64-bit key with atomicMin; the
// smallest key wins whatever the order of the atomics.  The lane is marked
// claimed for this step.
__device__ inline void claim(const Dev& d, int gl, unsigned long long key, int t) {
    atomicMin(&d.win[gl], key);
    d.enter_stamp[gl] = t;   // every claimant stores the same step
}

// Grid barrier of k_big_admit: every workgroup is resident (one per CU at
// most, checked at launch), and the wait ends after kBarrierTimeout of the
// 100 MHz clock at the latest, with an error flag instead of a hang.  Only a
// workgroup that wrote something (release) makes its writes device-wide
// first: on a GPU whose XCDs have separate L2 caches that fence writes the
// L2 back, the costly part of the barrier.
__device__ inline void grid_barrier(const Dev& d, unsigned* counter, bool release) {
    // A workgroup barrier waits for LDS operations only: every wave first
    // waits for its own global stores, so that the fence of thread 0 below
    // releases the whole workgroup's writes.
    if (release) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (release) __threadfence();
        atomicAdd(counter, 1u);
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x) {
            if (__builtin_amdgcn_s_memrealtime() - t0 > kBarrierTimeout) {
                atomicOr(&d.ctl->err, kErrBarrier);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
    }
    __syncthreads();
}

// An item whose target lane is in big tile k: listed for that tile's workgroup.
__device__ inline void defer_item(const Dev& d, int k, int item) {
    const int slot = atomicAdd(&d.ctl->n_defer, 1);
    __hip_atomic_store(&d.big_defer[slot], ((unsigned long long)(uint32_t)k << 32) | (uint32_t)item,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Admission of the request of lane i's front (eligibility, then the claim
// of the target lane, or in case 1 the node's crossing key).  kDefer: lane i
// in a big tile is left out (that tile's workgroup writes its request and
// admits it), and a target lane in a big tile is left to that tile's
// workgroup.
template <int NT, bool kDefer>
__device__ inline void admit_request(const Dev& d, int i, int t) {
    if (kDefer && d.big_lane[i].x == t) return;
    const Outbox ob = d.outbox[i];
    if (ob.target < 0) return;                    // an arrival
    if (kDefer) {
        const int2 bl = d.big_lane[ob.target];
        if (bl.x == t) {
            defer_item(d, bl.y, i);
            return;
        }
    }
    bool ok = transfer_eligible(d, ob, t);
    if (d.imode == 1) {
        // case 1: only after standing stop_steps at the line (the key's
        // step is the held-since step, t if not held); one crossing per
        // node, its (in, out) pairs served round-robin after the last
        // served one: key = (distance in the cycle, held since, source lane)
        const int e = d.s[t & 1].edge[ob.slot], f = ob.nxt;
        const int node = d.efrom[f], nmv = d.nm[node];
        const int pr = d.pair_base[e] + d.out_idx[f];
        int dd = (pr - d.rr[node] - 1) % nmv;
        if (dd < 0) dd += nmv;
        const int hs = (int)(ob.key >> 32);
        ok = ok && t - hs >= d.stop_steps;
        const unsigned long long nk = ((unsigned long long)dd << 58) |
                                      ((unsigned long long)(uint32_t)hs << 26) | (unsigned long long)i;
        d.outbox[i].key = nk;
        d.outbox[i].elig = ok ? 1 + node : 0;
        d.outbox[i].tl_cls = ob.tl_cls | ((uint32_t)pr << 16);
        if (ok) atomicMin(&d.win_node[node], nk);
        return;
    }
    d.outbox[i].elig = ok ? 1 : 0;
    if (ok) claim(d, ob.target, ob.key, t);
}

// Admission of a due departure-queue head (departure step hd.x, id hd.y):
// it claims the queue's lane if the lane's rear leaves it s0 at x = 0.
template <bool kDefer>
__device__ inline void admit_head(const Dev& d, int q, int2 hd, int t) {
    const int gl = d.qlane[q];
    if (kDefer) {
        const int2 bl = d.big_lane[gl];
        if (bl.x == t) {
            defer_item(d, bl.y, d.n_lanes_total + q);
            return;
        }
    }
    const LanePost p = d.post[gl];
    if (p.stamp != t || p.rear_xm >= d.qs0[q])
        claim(d, gl, (1ull << 63) | ((unsigned long long)(uint32_t)hd.x << 32) | (uint32_t)hd.y, t);
}

// One item per lane (its front may have asked to leave the edge this step)
// and one per departure queue, over workgroups wg of nwg.  A request is
// eligible if it does not overlap the target lane's rear after the move; a
// due queue head if the lane's rear leaves it s0 at x = 0.  Each thread takes
// its items four at a time and loads their stamps (queue heads) together, so
// that the loads overlap.
// The four stamps are read into one bit mask of due items, so that no
// per-thread array is indexed by a runtime value (which would put it in
// scratch memory).
template <int NT, bool kDefer>
__device__ inline void admit_items(const Dev& d, int t, int wg, int nwg) {
    constexpr int kU = 4;
    const int nl = d.n_lanes_total, nq = d.nq;
    const int stride = nwg * NT;
    for (int i0 = wg * NT + threadIdx.x; i0 < nl; i0 += kU * stride) {
        unsigned due = 0;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = i0 + u * stride;
            if (i < nl && d.req_stamp[i] == t) due |= 1u << u;
        }
        while (due) {
            const int u = __builtin_ctz(due);
            due &= due - 1;
            admit_request<NT, kDefer>(d, i0 + u * stride, t);
        }
    }
    for (int q0 = wg * NT + threadIdx.x; q0 < nq; q0 += kU * stride) {
        unsigned due = 0;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int q = q0 + u * stride;
            if (q < nq && d.qhd[q].x <= t) due |= 1u << u;
        }
        while (due) {
            const int q = q0 + __builtin_ctz(due) * stride;
            due &= due - 1;
            admit_head<kDefer>(d, q, d.qhd[q], t);
        }
    }
}

// Admission that waits for big tile k: the requests of the tile's own lanes
// and the items other workgroups left to it.  The workgroup first counts
// itself done and waits until every workgroup has (the admission workgroups
// after listing their items, the other big tiles after writing their
// requests and rears), like the grid barrier and bounded the same way.
__device__ inline void admit_big_tile(const Dev& d, int t, int par, int k) {
    grid_barrier(d, &d.ctl->big_done, true);
    const int a0 = d.big_list[2 * k], a1 = d.big_list[2 * k + 1];
    const int32_t* edge = d.s[par].edge;
    for (int s = a0 + (int)threadIdx.x; s < a1; s += kBigNT) {
        const int e = edge[s];
        if (s == a0 || edge[s - 1] != e) {
            const EdgeC c = d.ec[e];
            for (int l = 0; l < c.lanes; ++l)
                if (d.req_stamp[c.lane_base + l] == t) admit_request<kBigNT, false>(d, c.lane_base + l, t);
        }
    }
    const int nd = __hip_atomic_load(&d.ctl->n_defer, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int nl = d.n_lanes_total;
    for (int j = threadIdx.x; j < nd; j += kBigNT) {
        const unsigned long long en = __hip_atomic_load(&d.big_defer[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((int)(en >> 32) != k) continue;
        const int item = (int)(uint32_t)en;
        if (item < nl) admit_request<kBigNT, false>(d, item, t);
        else admit_head<false>(d, item - nl, d.qhd[item - nl], t);
    }
}

// The tiles above one workgroup's LDS, and admission, in one launch (one
// launch less per step).  Admission reads the requests of the source lanes
// and the post-move rears of the target lanes, which big tiles write.  With
// fewer big tiles than workgroups, the workgroups past the big tiles take the
// admission items of every other lane and queue, leave those whose target
// lane is in a big tile to that tile's workgroup, make the list visible and
// count themselves done without waiting; each big-tile workgroup, after its
// tile, waits until all have counted and admits its own lanes' requests and
// the items left to it.  Otherwise (every workgroup has a big tile) all of
// them meet at a grid barrier between the tiles and admission.
__global__ void __launch_bounds__(kBigNT) k_big_admit(Dev d) {
    const int2 nb2 = *(const int2*)d.ctl->n_big;   // independent of the step number load
    const int t = d.ctl->t_a, par = t & 1;
    const int nbig = par ? nb2.y : nb2.x;
    const bool all_big = nbig >= (int)gridDim.x;
    if (nbig == 0) {
        admit_items<kBigNT, false>(d, t, blockIdx.x, gridDim.x);
    } else if (all_big || (int)blockIdx.x < nbig) {
        big_tiles(d, t, par, nbig);                 // one call site: inlined, no call frame
        if (all_big) {
            grid_barrier(d, &d.ctl->big_done, true);
            admit_items<kBigNT, false>(d, t, blockIdx.x, gridDim.x);
        } else {
            admit_big_tile(d, t, par, blockIdx.x);  // tile blockIdx.x
        }
    } else {
        admit_items<kBigNT, true>(d, t, blockIdx.x - nbig, gridDim.x - nbig);
        __builtin_amdgcn_s_waitcnt(0);              // every wave's listed items and stores first
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(&d.ctl->big_done, 1u);
        }
    }
}

// One thread per edge, over its lanes (most edges have one or two).  For a
// lane the thread
//   * settles its front's end-of-edge request: arrival, admitted transfer
//     (an entry record on the next edge), or held at the stop line;
//   * inserts the departure whose key won the lane;
//   * counts its vehicles for the next layout.
// The edge's travel-time sum adds the exits in ascending vehicle id (at most
// one per lane; kept in LDS and sorted there when an edge has several).
// Lanes without a request cost three 4-byte stamps and their post-move count.
__device__ inline void commit_block(const Dev& d, int blk, int t, int par, CounterAcc& acc, Scan4* wsh4,
                                    uint32_t* xid, double* xtt, uint16_t* xnc, int* smoved) {
    const Slots S = d.s[par];
    const int e = blk * kEdgeBlock + (int)threadIdx.x;
    uint32_t* myid = xid + threadIdx.x * kCommitLanes;
    double* mytt = xtt + threadIdx.x * kCommitLanes;
    uint16_t* mync = xnc + threadIdx.x * kCommitLanes;
    int c = 0, nex = 0, nl = 0, base = 0;
    if (e < d.n_edges) {
        const EdgeC ce = d.ec[e];
        nl = ce.lanes;
        base = ce.lane_base;
        int node_win = -1;                         // case 1: lane index of this node's winning crossing
        if (d.imode == 1) {
            const unsigned long long wn = d.win_node[d.efrom[e]];
            if (wn != ~0ull) node_win = d.outbox[(int)(wn & ((1ull << 26) - 1))].target;
        }
        // each lane's three stamps are loaded one lane ahead
        LanePost pn = d.post[base];
        int rn = d.req_stamp[base], en = d.enter_stamp[base];
        for (int l = 0; l < nl; ++l) {
            const int gl = base + l;
            const LanePost p = pn;
            const bool req = rn == t;
            bool claimed = en == t;
            if (l + 1 < nl) {
                pn = d.post[gl + 1];
                rn = d.req_stamp[gl + 1];
                en = d.enter_stamp[gl + 1];
            }
            const int pcnt = p.stamp == t ? p.cnt : 0;
            bool exits = false;
            if (req) {
                const Outbox ob = d.outbox[gl];
                // every load of this request first, then the decisions and stores
                const uint32_t m = S.meta[ob.slot];
                const float xs = S.x[ob.slot], vs = S.v[ob.slot];
                const int hs = d.held_since[ob.vid];
                const double tin = d.tau_in[ob.vid];
                int kk = 0;
                int64_t r0 = 0;
                if (ob.target >= 0) {              // the route, for an entry record
                    kk = d.cursor[ob.vid] + 1;
                    r0 = d.roff[ob.vid];
                }
                bool won;
                if (d.imode == 1) {
                    won = ob.target >= 0 && ob.elig && d.win_node[ob.elig - 1] == ob.key;
                    if (won) d.rr[ob.elig - 1] = (int)((ob.tl_cls >> 16) & 255u);   // the pair just served
                } else {
                    won = ob.target >= 0 && ob.elig && d.win[ob.target] == ob.key;
                }
                const bool arrived = ob.target < 0;
                if (d.trace)
                    d.trace[(size_t)(t % d.trace_period) * d.trace_stride + ob.slot].kb |=
                        (arrived ? TB_ARRIVE : (won ? TB_EXIT : TB_HELD)) << 8;
                exits = arrived || won;
                if (arrived) {                     // arrival at the route end
                    d.status[ob.vid] = kArrived;
                    d.fin_x[ob.vid] = xs;
                    d.fin_v[ob.vid] = vs;
                    d.fin_meta[ob.vid] = m;
                } else if (!won) {                 // held at the stop line
                    S.x[ob.slot] = ce.L;
                    S.v[ob.slot] = 0.0f;
                    S.meta[ob.slot] = m | (1u << 5);
                    if (hs < 0) d.held_since[ob.vid] = t;
                }
                // counted outside the branches: an increment of a different
                // counter in each branch would be merged into one store through
                // a computed index, which moves the counters to scratch memory
                acc.c[cArrived] += arrived ? 1u : 0u;
                acc.c[cTransfers] += won ? 1u : 0u;
                acc.c[cWaivedExits] += (won && !lane_allowed(m, ob.nxt, l)) ? 1u : 0u;
                acc.c[cHolds] += exits ? 0u : 1u;
                if (exits) *smoved = 1;                 // gridlock detector
                if (exits) {
                    d.exit_stamp[gl] = t;
                    const double tau = ((double)t + (double)ob.phi) * (double)d.dt;
                    myid[nex] = ob.vid;
                    mytt[nex] = tau - tin;
                    ++nex;
                    if (arrived) d.t_arr[ob.vid] = tau;
                    else d.tau_in[ob.vid] = tau;
                }
                if (won) {                         // entry record, stored at the target lane
                    const int64_t pos = r0 + kk + 1;   // route index of the edge after ob.nxt
                    EntryRec r;
                    r.x = ob.xp;
                    r.v = ob.v;
                    r.vid = ob.vid;
                    r.edge = ob.nxt;
                    r.gl = ob.target;
                    r.meta = m_make((int)(ob.tl_cls & 255u), false, false, 0, (int)((ob.tl_cls >> 8) & 255u),
                                    d.rmask[r0 + kk]);
                    r.nxt = pos < d.roff[ob.vid + 1] ? d.redges[pos] : -1;
                    r.pad = 0;
                    d.cursor[ob.vid] = kk;
                    d.held_since[ob.vid] = -1;
                    d.ent[ob.target] = r;
                }
            }
            // the departure whose key won this lane; in case 1 only departures
            // claim lanes, and this node's crossing into the lane comes first
            const bool transfer_in = node_win == gl;
            if (claimed && !transfer_in) {
                const unsigned long long w = d.win[gl];
                if (w >> 63) {
                    const int vid = (int)(uint32_t)w;
                    const int4 vq = d.vq[vid];     // vid is the head of queue vq.x
                    const int64_t q0 = d.roff[vid];
                    d.qhead[vq.x] = vq.y + 1;
                    d.qhd[vq.x] = vq.z >= 0 ? make_int2(vq.w, vq.z) : make_int2(INT_MAX, -1);
                    EntryRec r;
                    r.x = 0.0f;
                    r.v = 0.0f;
                    r.vid = (uint32_t)vid;
                    r.edge = e;                    // the queue's lane is on the first route edge
                    r.gl = gl;
                    r.meta = m_make(l, false, false, 0, d.cls[vid], d.rmask[q0]);
                    r.nxt = (q0 + 1 < d.roff[vid + 1]) ? d.redges[q0 + 1] : -1;
                    r.pad = 0;
                    d.status[vid] = kActive;
                    d.cursor[vid] = 0;
                    d.held_since[vid] = -1;
                    d.tau_in[vid] = (double)(t + 1) * (double)d.dt;
                    d.ent[gl] = r;
                    acc.c[cDeparted]++;
                    *smoved = 1;
                }
            }
            if (transfer_in && !claimed) d.enter_stamp[gl] = t;   // the scatter takes the crossing's record
            claimed = claimed || transfer_in;
            // next layout: this lane's count (its offset follows the block scan)
            const int nc = pcnt - (exits ? 1 : 0) + (claimed ? 1 : 0);
            mync[l] = (uint16_t)nc;
            d.lane_newcnt[gl] = nc;
            c += nc;
        }
        if (nex > 0) {
            // travel times of the edge's exits, added in ascending vehicle id
            for (int i = 1; i < nex; ++i)
                for (int j = i; j > 0 && myid[j - 1] > myid[j]; --j) {
                    const uint32_t ti = myid[j];
                    myid[j] = myid[j - 1];
                    myid[j - 1] = ti;
                    const double tt = mytt[j];
                    mytt[j] = mytt[j - 1];
                    mytt[j - 1] = tt;
                }
            double sum = d.tt_sum[e];
            for (int i = 0; i < nex; ++i) sum += mytt[i];
            d.tt_sum[e] = sum;
            d.tt_cnt[e] += (unsigned long long)nex;
        }
    }
    // offsets of the edges in the workgroup, then of their lanes
    const Scan4 run = wg_exclusive_scan4<kCommitNT>(Scan4{c, -1, -1, -1}, wsh4);
    int o = run.s;
    for (int l = 0; l < nl; ++l) {
        d.lane_off[base + l] = o;
        o += mync[l];
    }
    if (threadIdx.x == kCommitNT - 1) d.blk_sum[blk] = run.s + c;
}

__device__ inline void flush_commit_counters(const Dev& d, const CounterAcc& acc, unsigned* shc) {
    flush_counters_lds(d, acc, shc);   // ends with a barrier: shc is complete
    if (threadIdx.x == 0 && shc[cDeparted]) atomicAdd(&d.ctl->n_departed, (int)shc[cDeparted]);
}

__global__ void __launch_bounds__(kCommitNT) k_commit(Dev d) {
    __shared__ unsigned shc[cNumCounters];
    __shared__ Scan4 wsh4[kCommitNT / 64];
    __shared__ uint32_t xid[kCommitNT * kCommitLanes];     // exits of each thread's edge
    __shared__ double xtt[kCommitNT * kCommitLanes];
    __shared__ uint16_t xnc[kCommitNT * kCommitLanes];   // new counts of each thread's lanes
    __shared__ int smoved;                                // gridlock detector: an exit or a departure here
    if (threadIdx.x < cNumCounters) shc[threadIdx.x] = 0;
    if (threadIdx.x == 0) smoved = 0;
    __syncthreads();
    const int t = d.ctl->t_b, par = t & 1;
    CounterAcc acc;
    acc.zero();
    commit_block(d, blockIdx.x, t, par, acc, wsh4, xid, xtt, xnc, &smoved);
    flush_commit_counters(d, acc, shc);
    publish_moved(d, &smoved, t);
}

// ---- offsets of the edge blocks and the end of the step --------------------
// Exclusive scan of the commit workgroups' vehicle counts into off[0, nb);
// returns the total (the active vehicles of the next step).  The sums were
// written by k_commit, a previous kernel, so no fence is needed: no workgroup
// waits for another inside a kernel, which on a GPU of several L2 caches
// would cost a write-back of the L2 at every release.
template <int NT>
__device__ inline int scan_block_sums(const int* blk_sum, int nb, int* off, Scan4* wsh4, int* tot) {
    const int chunk = (nb + NT - 1) / NT;
    const int lo = min(nb, (int)threadIdx.x * chunk), hi = min(nb, lo + chunk);
    int loc = 0;
    for (int i = lo; i < hi; ++i) loc += blk_sum[i];
    const Scan4 r = wg_exclusive_scan4<NT>(Scan4{loc, -1, -1, -1}, wsh4);
    int o = r.s;
    for (int i = lo; i < hi; ++i) {
        off[i] = o;
        o += blk_sum[i];
    }
    if (hi == nb && lo < hi) *tot = o;
    __syncthreads();
    return *tot;
}

// The same for many blocks (one workgroup, global output): the counts go
// through `stage` (LDS, cap entries per round), read coalesced with every
// load of a thread in flight together, scanned there by contiguous chunks
// and written back coalesced.  With tens of blocks per thread, reading each
// thread's contiguous chunk straight from memory would wait for one load
// after another.
template <int NT>
__device__ inline int scan_block_sums_staged(const int* blk_sum, int nb, int* off, int* stage, int cap,
                                             Scan4* wsh4, int* tot) {
    int carry = 0;
    for (int r0 = 0; r0 < nb; r0 += cap) {
        const int m = min(cap, nb - r0);
        // coalesced loads, every one of a thread in flight before the first use
#pragma unroll 8
        for (int i = (int)threadIdx.x; i < m; i += NT) stage[i] = blk_sum[r0 + i];
        __syncthreads();
        const int chunk = (m + NT - 1) / NT;
        const int lo = min(m, (int)threadIdx.x * chunk), hi = min(m, lo + chunk);
        int loc = 0;
        for (int i = lo; i < hi; ++i) loc += stage[i];
        const Scan4 r = wg_exclusive_scan4<NT>(Scan4{loc, -1, -1, -1}, wsh4);
        int o = carry + r.s;
        for (int i = lo; i < hi; ++i) {
            const int v = stage[i];
            stage[i] = o;
            o += v;
        }
        if (hi == m && lo < hi) *tot = o;
        __syncthreads();
        for (int i = (int)threadIdx.x; i < m; i += NT) off[r0 + i] = stage[i];
        carry = *tot;
        __syncthreads();                            // stage and *tot are reused by the next round
    }
    return carry;
}

// n_act of the next step, refused departures of this one (every due vehicle
// still waiting asked for a lane and was refused), and the step counter
// Called by the first wavefront of one workgroup; its lane 0 writes.
__device__ inline void finish_step(const Dev& d, int t, int par, int total) {
    const bool moved = __ballot(d.moved_at[threadIdx.x] == t) != 0ull;   // gridlock detector
    if (threadIdx.x != 0) return;
    const int run = (d.ctl->n_act[par] > 0 && !moved) ? d.ctl->stall_run + 1 : 0;
    d.ctl->stall_run = run;
    if (run >= kGridlockSteps) d.counters[cGridlock * kCounterCopies] += 1ull;
    d.ctl->n_act[par ^ 1] = total;
    const int due_now = d.max_dep < 0 ? 0 : d.due[min(t, d.max_dep)];
    const int departed = d.ctl->n_departed;
    if (due_now > departed)
        atomicAdd(&d.counters[cInsertDenied * kCounterCopies], (unsigned long long)(due_now - departed));
    d.ctl->t_a = t + 1;   // the tile kernels and admission of this step are done
}

// Networks with more edge blocks than kScanLdsMax: one workgroup scans the
// block offsets into global memory before k_scatter.
__global__ void __launch_bounds__(kBigNT) k_blkscan(Dev d) {
    __shared__ Scan4 wsh4[kBigNT / 64];
    __shared__ int tot;
    __shared__ int stage[kScanLdsMax];
    const int t = d.ctl->t_b, par = t & 1;
    const int total = scan_block_sums_staged<kBigNT>(d.blk_sum, d.n_blk, d.blk_off, stage, kScanLdsMax, wsh4, &tot);
    if (threadIdx.x < 64) finish_step(d, t, par, total);
}

// ---- next layout -----------------------------------------------------------
// One record of the next layout at slot dst, and the lane's rear for the
// next step's look-ahead if it is the lane's last vehicle.
__device__ inline void put_record(const Dev& d, const Slots& B, int dst, int nnew, float x, float v, uint32_t vid,
                                  int edge, uint32_t meta, int nxt, bool is_rear, int gl, int t, const float* slen) {
    if (dst < 0 || dst >= nnew) {
        atomicOr(&d.ctl->err, kErrScatter);
        return;
    }
    B.x[dst] = x;
    B.v[dst] = v;
    B.vid[dst] = vid;
    B.edge[dst] = edge;
    B.meta[dst] = meta;
    B.nxt[dst] = nxt;
    if (is_rear) {
        LaneRear lr;
        lr.xm = x - slen[m_cls(meta)];
        lr.v = v;
        lr.stamp = t + 1;
        lr.vid = vid;
        d.rear[gl] = lr;
    }
}

// slot of a vehicle in the next layout:
//   block offset + edge offset in block + lane offset in edge + rank in lane
// kLds: the workgroup scans the block offsets itself into LDS (at most
// kScanLdsMax edge blocks), and workgroup 0 finishes the step; otherwise
// k_blkscan has done both.
template <bool kLds>
__device__ inline void scatter_items(const Dev& d, int* soff, Scan4* wsh4, int* totp, float* slen) {
    if (threadIdx.x < 16) slen[threadIdx.x] = d.cp[threadIdx.x].len;
    const StepHead sh = step_head(d.ctl);
    const int t = sh.t_b, par = t & 1;
    const int nold = par ? sh.n1 : sh.n0;
    const int nl = d.n_lanes_total;
    const int* boff;
    int nnew;
    if (kLds) {
        // every block sum loaded at once into LDS and scanned there (one round:
        // at most kScanLdsMax blocks take this path)
        nnew = scan_block_sums_staged<kNT>(d.blk_sum, d.n_blk, soff, soff, kScanLdsMax, wsh4, totp);
        boff = soff;
        if (blockIdx.x == 0 && threadIdx.x < 64) finish_step(d, t, par, nnew);
    } else {
        boff = d.blk_off;
        nnew = d.ctl->n_act[par ^ 1];
        __syncthreads();                          // slen
    }
    const Slots A = d.s[par], B = d.s[par ^ 1];
    // Item k is the record in slot k (k < nold) and lane k (k < nl), which
    // takes the record that entered it if it was claimed this step.  Each
    // round of loads of the two is issued together: the record with its lane
    // and the lane's claim stamp; then the tables of the record's lane and
    // the entry of a claimed lane.
    const int nit = max(nold, nl);
    for (int k = blockIdx.x * kNT + threadIdx.x; k < nit; k += gridDim.x * kNT) {
        const bool hv = k < nold;
        float x = 0.0f, v = 0.0f;
        uint32_t vid = 0, meta = 0;
        int edge = 0, nxt = 0, gl = 0;
        if (hv) {
            meta = A.meta[k];
            edge = A.edge[k];
            x = A.x[k];
            v = A.v[k];
            vid = A.vid[k];
            nxt = A.nxt[k];
            gl = A.gl[k];
        }
        const bool claimed = k < nl && d.enter_stamp[k] == t;
        LanePost lp{};
        int ex = 0, ncnt = 0, loff = 0;
        bool entered = false;
        if (hv) {
            lp = d.post[gl];
            ex = d.exit_stamp[gl] == t ? 1 : 0;
            ncnt = d.lane_newcnt[gl];
            entered = d.enter_stamp[gl] == t;
            loff = d.lane_off[gl];
        }
        EntryRec en{};
        int encnt = 0, enoff = 0;
        if (claimed) {
            en = d.ent[k];
            encnt = d.lane_newcnt[k];
            enoff = d.lane_off[k];
        }
        if (hv) {
            const int r = k - lp.start;
            if (lp.stamp != t) {
                atomicOr(&d.ctl->err, kErrScatter);
            } else if (!(ex && r == 0)) {         // unless the lane's front left the edge
                const int nr = r - ex;
                put_record(d, B, boff[edge / kEdgeBlock] + loff + nr, nnew, x, v, vid, edge, meta, nxt,
                           (nr == ncnt - 1) && !entered, gl, t, slen);
            }
        }
        if (claimed) {                            // the entry is the lane's new rear
            put_record(d, B, boff[en.edge / kEdgeBlock] + enoff + encnt - 1, nnew, en.x, en.v, en.vid, en.edge,
                       en.meta, en.nxt, true, k, t, slen);
            d.win[k] = ~0ull;                     // lane free for the next step's claims
        }
    }
}

template <bool kLds>
__global__ void __launch_bounds__(kNT) k_scatter(Dev d) {
    // kLds: the block offsets, d.n_blk ints of dynamic LDS sized at launch
    // (so a network with few edge blocks leaves room for more workgroups)
    extern __shared__ int soff[];
    __shared__ Scan4 wsh4[kWaves];
    __shared__ int tot;
    __shared__ float slen[16];                    // vehicle length per class
    scatter_items<kLds>(d, soff, wsh4, &tot, slen);
    if (d.imode == 1)                             // case 1: nodes free for the next step's crossings
        for (int v = blockIdx.x * kNT + threadIdx.x; v < d.n_nodes; v += gridDim.x * kNT) d.win_node[v] = ~0ull;
}


// ---- differentiable form: reverse sweep of one step ----------------------
// With the step's discrete decisions frozen (trace records), the state at
// t + 1 is a smooth function of the state at t and of the class parameters.
// lx, lv: adjoints of (x, v) at t + 1 by vehicle id; nx, nv (zeroed): at t.
// lt: adjoint of each vehicle's current edge-entry time.  w: dL/d(edge mean
// travel time) / (traversals of the edge).  Parameter gradients of the
// workgroup's records are reduced in a fixed tree and added to its own slot
// gpart[blockIdx][5 * classes] (one workgroup per slot, kernels in order).
constexpr int kParamMax = 5 * 16;

__device__ inline double idm_partials(double v, double v0, double vl, double s, const ClassParams& p, int kind,
                                      uint32_t bits, double d[8]) {
    for (int k = 0; k < 8; ++k) d[k] = 0.0;   // d acc / d (v, vl, s, v0, T, a, b, s0)
    const double a = p.a, b = p.b, T = p.T, s0 = p.s0;
    const double r = v / v0, r2 = r * r;
    double phi;
    if (bits & TB_F) {
        phi = -b;
        d[6] = -1.0;
    } else {
        phi = a * (1.0 - r2 * r2);
        d[0] = -4.0 * a * r2 * r / v0;
        d[3] = 4.0 * a * r2 * r2 / v0;
        d[5] = 1.0 - r2 * r2;
    }
    if (kind == kFree) return phi;
    const double den = 2.0 * sqrt(a * b);
    double dyn = 0.0, dyv = 0.0, dyvl = 0.0, dyT = 0.0, dyden = 0.0;
    if (!(bits & TB_D)) {
        dyn = v * T + v * (v - vl) / den;
        dyv = T + (2.0 * v - vl) / den;
        dyvl = -v / den;
        dyT = v;
        dyden = -v * (v - vl) / (den * den);
    }
    const double sst = s0 + dyn;
    const double se = (bits & TB_S) ? (double)kSMin : s;
    const double q = sst / se;
    const double dsst = -2.0 * a * q / se;
    if (!(bits & TB_S)) d[2] = 2.0 * a * q * q / se;
    d[0] += dsst * dyv;
    d[1] = dsst * dyvl;
    d[4] = dsst * dyT;
    d[5] += -q * q + dsst * dyden * (den / (2.0 * a));
    d[6] += dsst * dyden * (den / (2.0 * b));
    d[7] = dsst;
    return phi - a * q * q;
}

// The reverse sweep of one step in three kernels, with no floating-point
// atomics, so the result is the same bit for bit on every run:
//   k_backward   each record's own part of (nx, nv) and its part for its
//                partner (leader, or look-ahead rear), written per record;
//                a look-ahead record joins the list of the lane it looked into;
//   k_bw_looks   the first record of each such list adds the list's parts in
//                record order for the lane's start-of-step rear;
//   k_bw_gather  every vehicle: own part + the part of the record behind it
//                in its lane (its follower, whose leader it is) + its
//                look-ahead sum.
// A VEH or clamp record's leader is the record just before it in the traced
// layout (the post-lane-change order of edge, lane, x and id); k_backward
// checks this and flags a layout error otherwise.
constexpr int kLookListCap = 16;   // look-ahead records into one lane in one step, at most

struct BwPart {
    double sx, sv;    // the record's own vehicle
    double px, pv;    // its partner
};

__global__ void __launch_bounds__(kNT) k_backward(Dev d, const TraceRec* rec, const int* n_ptr, int t, int n_classes,
                                                 const double* lx, const double* lv, BwPart* part, int* lk_cnt,
                                                 int* lk_rec, double* lt, const double* w, double* gpart,
                                                 double* ox, double* ov, int n_all) {
    __shared__ double red[kNT];
    double g[kParamMax];
    const int np = 5 * n_classes;
    for (int k = 0; k < np; ++k) g[k] = 0.0;
    const double dt = (double)d.dt;
    const int n = *n_ptr;
    // the step's output adjoints start at zero (k_bw_gather writes those of
    // the vehicles active at the step's start)
    for (int i = blockIdx.x * kNT + threadIdx.x; i < n_all; i += gridDim.x * kNT) {
        ox[i] = 0.0;
        ov[i] = 0.0;
    }
    for (int r = blockIdx.x * kNT + threadIdx.x; r < n; r += gridDim.x * kNT) {
        const TraceRec R = rec[r];
        const uint32_t bits = R.kb >> 8;
        const int kind = (int)(R.kb & 255u);
        const int i = (int)R.vid, e = R.edge, j = R.partner;
        const double L = (double)d.L[e];
        const double x = R.x, v = R.v, xn = R.xn;
        double mx = lx[i], mv = lv[i];
        BwPart P{0.0, 0.0, 0.0, 0.0};
        if (bits & (TB_HELD | TB_W | TB_ARRIVE)) {
            mx = 0.0;
            mv = 0.0;
        }
        if (bits & (TB_EXIT | TB_ARRIVE)) {       // crossing time (t + phi) dt, phi = (L - x) / (xn - x)
            const double gt = w[e] + lt[i];
            if (xn != x) {
                const double dd = xn - x;
                mx += gt * dt * (-(L - x) / (dd * dd));
                P.sx = gt * dt * ((L - xn) / (dd * dd));
            }
            lt[i] = -w[e];
        }
        if (!(bits & (TB_HELD | TB_W))) {
            const int c = d.cls[i];
            const ClassParams cp = d.cp[c];
            const double lim = (double)driver_limit(d.lim[e], d.v0_spread, d.seed, e, d.edge_period, d.rid[i]);
            const double v0 = (double)cp.v0f * lim;
            double pd[8];
            const double acc = idm_partials(v, v0, (double)R.vl, (double)R.s, cp, kind, bits, pd);
            double macc = 0.0, ax = 0.0, av = 0.0;
            if (bits & TB_C) {                     // clamped to the leader's rear
                P.px = mx;
                mx = 0.0;
            }
            if (bits & TB_B) {                     // exact stop
                ax += mx;
                av += mx * (-v / acc);
                macc += mx * (v * v / (2.0 * acc * acc));
            } else {
                ax += mx;
                av += mx * dt + mv;
                macc += mx * 0.5 * dt * dt + mv * dt;
            }
            av += macc * pd[0];
            if (kind == kVeh || kind == kLook) {
                ax -= macc * pd[2];
                P.px += macc * pd[2];
                P.pv += macc * pd[1];
            } else if (kind == kStop) {
                ax -= macc * pd[2];
            }
            P.sx += ax;
            P.sv += av;
            g[5 * c + 0] += macc * pd[3] * lim;
            g[5 * c + 1] += macc * pd[4];
            g[5 * c + 2] += macc * pd[5];
            g[5 * c + 3] += macc * pd[6];
            g[5 * c + 4] += macc * pd[7];
        }
        part[r] = P;
        if ((kind == kVeh || (bits & TB_C)) && !(bits & (TB_HELD | TB_W)) && (r == 0 || (int)rec[r - 1].vid != j))
            atomicOr(&d.ctl->err, kErrTrace);     // the leader is not the record just before
        if (kind == kLook && !(bits & (TB_HELD | TB_W))) {
            const int k = atomicAdd(&lk_cnt[R.look_gl], 1);
            if (k < kLookListCap) lk_rec[(size_t)R.look_gl * kLookListCap + k] = r;
            else atomicOr(&d.ctl->err, kErrTrace);
        }
    }
    for (int k = 0; k < np; ++k) {                 // fixed-order tree per parameter
        red[threadIdx.x] = g[k];
        __syncthreads();
        for (int h = kNT / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) gpart[(size_t)blockIdx.x * np + k] += red[0];
        __syncthreads();
    }
}

// Look-ahead sums: the list of a lane is sorted by record index and added in
// that order by its first record, for the lane's start-of-step rear (the
// partner of every record in the list); the list is then emptied.
__global__ void __launch_bounds__(kNT) k_bw_looks(const TraceRec* rec, const int* n_ptr, int t, const BwPart* part,
                                                  int* lk_cnt, const int* lk_rec, double* lkx, double* lkv,
                                                  int* lk_stamp) {
    const int n = *n_ptr;
    for (int r = blockIdx.x * kNT + threadIdx.x; r < n; r += gridDim.x * kNT) {
        const TraceRec R = rec[r];
        if ((int)(R.kb & 255u) != kLook || ((R.kb >> 8) & (TB_HELD | TB_W))) continue;
        const int g = R.look_gl;
        const int m = min(lk_cnt[g], kLookListCap);
        int lst[kLookListCap];
        int first = r;
        for (int k = 0; k < kLookListCap; ++k) {
            lst[k] = k < m ? lk_rec[(size_t)g * kLookListCap + k] : INT_MAX;
            first = min(first, lst[k]);
        }
        if (first != r) continue;                  // another record of the list sums it
        for (int a = 1; a < kLookListCap; ++a)     // insertion sort of the (few) record indices
            for (int b = a; b > 0 && lst[b - 1] > lst[b]; --b) {
                const int tmp = lst[b];
                lst[b] = lst[b - 1];
                lst[b - 1] = tmp;
            }
        double sx = 0.0, sv = 0.0;
        for (int k = 0; k < m; ++k) {
            sx += part[lst[k]].px;
            sv += part[lst[k]].pv;
        }
        const int j = R.partner;
        lkx[j] = sx;
        lkv[j] = sv;
        lk_stamp[j] = t;
        lk_cnt[g] = 0;
    }
}

// (nx, nv) of every vehicle that was active at the step's start, in a fixed
// order: own part, then its follower's part, then its look-ahead sum.
__global__ void __launch_bounds__(kNT) k_bw_gather(const TraceRec* rec, const int* n_ptr, int t, const BwPart* part,
                                                   const double* lkx, const double* lkv, int* lk_stamp,
                                                   double* nx, double* nv) {
    const int n = *n_ptr;
    for (int r = blockIdx.x * kNT + threadIdx.x; r < n; r += gridDim.x * kNT) {
        const int i = (int)rec[r].vid;
        const BwPart P = part[r];
        double ax = P.sx, av = P.sv;
        if (r + 1 < n) {
            const TraceRec F = rec[r + 1];
            const uint32_t fb = F.kb >> 8;
            if (F.partner == i && ((int)(F.kb & 255u) == kVeh || (fb & TB_C)) && !(fb & (TB_HELD | TB_W))) {
                const BwPart Q = part[r + 1];
                ax += Q.px;
                av += Q.pv;
            }
        }
        if (lk_stamp[i] == t) {                    // consumed here: stamps repeat from segment to segment
            ax += lkx[i];
            av += lkv[i];
            lk_stamp[i] = -1;
        }
        nx[i] = ax;
        nv[i] = av;
    }
}

// ---- diagnostics ---------------------------------------------------------
__global__ void k_probe_fp32(int op, const float* a, const float* b, float* out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = a[i], y = b ? b[i] : 0.0f;
        float r;
        switch (op) {
            case 0: r = x / y; break;
            case 1: r = sqrtf(x); break;
            case 2: r = x * y; break;
            case 3: r = x + y; break;
            default: r = exp_eq2(x); break;
        }
        out[i] = r;
    }
}

// Per-edge mean completed traversal time: the sum over the count (FP64,
// correctly rounded), 0 where nothing completed a traversal.
__global__ void __launch_bounds__(kNT) k_edge_means(const double* sum, const unsigned long long* cnt, double* mean,
                                                    int n) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i < n) {
        const unsigned long long c = cnt[i];
        mean[i] = c ? sum[i] / (double)c : 0.0;
    }
}

__global__ void k_probe_philox(const uint64_t* ctr, uint64_t k0, uint64_t k1, uint64_t* out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const U64x4 r = philox4x64_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
        for (int j = 0; j < 4; ++j) out[4 * i + j] = r.w[j];
    }
}

__global__ void k_probe_draws(uint64_t seed, const int64_t* t, const int64_t* id, float* u, float* e2, float* e3,
                              int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        u[i] = draw_uniform(seed, (int)t[i], (uint32_t)id[i], 1);
        e2[i] = draw_normal(seed, (int)t[i], (uint32_t)id[i], 2);
        e3[i] = draw_normal(seed, (int)t[i], (uint32_t)id[i], 3);
    }
}

}  // namespace manta
