// libmanta host side: input validation, device layout, the step launch
// sequence (replayed from a captured HIP graph), and state I/O.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/manta.h"
#include "routing.hpp"
#include "step_kernels.hpp"

static_assert(manta::cNumCounters == SIM_N_COUNTERS, "device counters and sim_state.counters differ");

using namespace manta;

namespace {

// ---- allocator -----------------------------------------------------------
void* (*g_alloc)(size_t, void*) = nullptr;
void (*g_release)(void*, void*) = nullptr;
void* g_ctx = nullptr;
thread_local std::string g_create_error;

struct Alloc {
    void* (*alloc)(size_t, void*);
    void (*release)(void*, void*);
    void* ctx;
    void* get(size_t bytes) {
        if (bytes == 0) bytes = 16;
        bytes = (bytes + 255) & ~(size_t)255;
        if (alloc) return alloc(bytes, ctx);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        return p;
    }
    void put(void* p) {
        if (!p) return;
        if (release) release(p, ctx);
        else (void)hipFree(p);
    }
};

struct Fail {
    sim_status st;
    std::string msg;
};

std::string fmt(const char* f, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof(buf), f, ap);
    va_end(ap);
    return buf;
}

#define HIP_OK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) throw Fail{SIM_EDEVICE, fmt("%s: %s", #expr, hipGetErrorString(e_))}; \
    } while (0)

}  // namespace

struct sim_handle {
    Alloc al{};
    std::vector<void*> bufs;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph_k = nullptr;     // kGraphSteps steps in one graph (fewer graph launches)
    hipGraphExec_t exec_k = nullptr;
    std::string err;
    Dev d{};
    int t = 0;
    int n_veh = 0, n_edges = 0, n_lanes = 0, n_classes = 0;
    int g_tile = 1, g_big = 1, g_scatter = 1, n_blk = 1;
    size_t scatter_lds = 0;   // dynamic LDS of k_scatter<true>: the block offsets
    int g_big_min = 1, g_big_max = 1, g_scatter_max = 1, g_scatter_res = 1;
    int n_scen = 1;
    double* tt_mean = nullptr;      // per-edge means (sim_read_edge_means), allocated at first use
    std::vector<int32_t> veh_off;   // ensemble: vehicles of scenario k
    // differentiable form: a snapshot of the dynamic state every rec_every steps
    int rec_every = 0;
    bool rec_broken = false;
    std::vector<void*> snaps;
    size_t snap_bytes = 0;
    int nq = 0;
    // host copies of the static inputs needed for state I/O
    std::vector<int64_t> roff;
    std::vector<int32_t> redges, dep, lanes, lane_base, conn_off, conn_to, ins_lane;
    std::vector<int32_t> qveh, qoff;   // departure queues (host copy, for state writes)
    std::vector<uint8_t> conn_mask, cls;
    std::vector<float> L, len_c, s0_c;

    template <class T>
    T* dev(size_t count) {
        void* p = al.get(count * sizeof(T));
        if (!p) throw Fail{SIM_ENOMEM, fmt("device allocation of %zu bytes failed", count * sizeof(T))};
        bufs.push_back(p);
        return (T*)p;
    }
    template <class T>
    T* upload(const T* host, size_t count) {
        T* p = dev<T>(count);
        if (count) HIP_OK(hipMemcpy(p, host, count * sizeof(T), hipMemcpyHostToDevice));
        return p;
    }
    void release_all() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (exec_k) (void)hipGraphExecDestroy(exec_k);
        if (graph_k) (void)hipGraphDestroy(graph_k);
        exec = nullptr;
        graph = nullptr;
        exec_k = nullptr;
        graph_k = nullptr;
        for (void* p : bufs) al.put(p);
        bufs.clear();
        for (void* p : snaps) al.put(p);
        snaps.clear();
    }
    uint32_t mask_of(int e, int f) const {
        if (f < 0) return 0xFFu;
        for (int c = conn_off[e]; c < conn_off[e + 1]; ++c)
            if (conn_to[c] == f) return conn_mask[c];
        return 0u;
    }
};

namespace {

bool finite_in(float v, float lo, float hi) { return std::isfinite(v) && v >= lo && v <= hi; }

void validate(const sim_network* net, const sim_routes* r, const sim_idm_params* p) {
    auto bad = [](std::string m) { throw Fail{SIM_EINVAL, std::move(m)}; };
    if (!net || !r || !p) bad("null argument");
    if (net->n_nodes <= 0 || net->n_edges <= 0) bad("network must have nodes and edges");
    if (!net->edge_from || !net->edge_to || !net->length_m || !net->speed_limit_mps || !net->n_lanes ||
        !net->conn_off || !net->conn_to || !net->conn_lane_mask)
        bad("network array missing");
    const int E = net->n_edges;
    if (net->conn_off[0] != 0) bad("conn_off[0] != 0");
    for (int e = 0; e < E; ++e) {
        if (net->edge_from[e] < 0 || net->edge_from[e] >= net->n_nodes || net->edge_to[e] < 0 ||
            net->edge_to[e] >= net->n_nodes)
            bad(fmt("edge %d: node id out of range", e));
        if (net->n_lanes[e] < 1 || net->n_lanes[e] > 8) bad(fmt("edge %d: lanes %d not in 1..8", e, net->n_lanes[e]));
        if (!(std::isfinite(net->length_m[e]) && net->length_m[e] >= 20.0f))
            bad(fmt("edge %d: length must be >= 20 m", e));
        if (!(std::isfinite(net->speed_limit_mps[e]) && net->speed_limit_mps[e] > 0.0f))
            bad(fmt("edge %d: speed limit must be > 0", e));
        if (net->conn_off[e + 1] < net->conn_off[e]) bad("conn_off must be non-decreasing");
    }
    for (int e = 0; e < E; ++e)
        for (int c = net->conn_off[e]; c < net->conn_off[e + 1]; ++c) {
            const int f = net->conn_to[c];
            if (f < 0 || f >= E) bad(fmt("move %d: target edge out of range", c));
            if (net->edge_from[f] != net->edge_to[e]) bad(fmt("move %d: edges %d -> %d do not meet", c, e, f));
            const unsigned m = net->conn_lane_mask[c];
            if (m == 0 || (m >> net->n_lanes[e]) != 0) bad(fmt("move %d: lane mask invalid", c));
        }
    if (p->n_classes < 1 || p->n_classes > 16) bad("n_classes must be in 1..16");
    if (!p->v0_factor || !p->T || !p->a || !p->b || !p->s0 || !p->length_m) bad("parameter array missing");
    for (int c = 0; c < p->n_classes; ++c) {
        if (!finite_in(p->a[c], 1.0f, 10.0f)) bad(fmt("class %d: a outside [1, 10]", c));
        if (!finite_in(p->b[c], 1.0f, 10.0f)) bad(fmt("class %d: b outside [1, 10]", c));
        if (!finite_in(p->T[c], 0.1f, 2.0f)) bad(fmt("class %d: T outside [0.1, 2]", c));
        if (!finite_in(p->s0[c], 1.0f, 5.0f)) bad(fmt("class %d: s0 outside [1, 5]", c));
        if (!(std::isfinite(p->v0_factor[c]) && p->v0_factor[c] > 0.0f && p->v0_factor[c] <= 2.0f))
            bad(fmt("class %d: v0_factor outside (0, 2]", c));
        if (!(std::isfinite(p->length_m[c]) && p->length_m[c] > 0.0f && p->length_m[c] <= 20.0f))
            bad(fmt("class %d: length outside (0, 20]", c));
    }
    if (!(std::isfinite(p->dt) && p->dt > 0.0f && p->dt <= 1.0f)) bad("dt outside (0, 1]");
    if (p->intersection_mode != 0 && p->intersection_mode != 1) bad("intersection_mode must be 0 or 1");
    if (p->intersection_mode == 1) {
        // case 1 keys hold the source lane in 26 bits and the round-robin distance in 6
        if ((int64_t)net->n_nodes <= 0) bad("case 1 needs the node count");
        std::vector<int> indeg((size_t)net->n_nodes, 0), outdeg((size_t)net->n_nodes, 0);
        int64_t nl = 0;
        for (int e = 0; e < E; ++e) {
            if (net->edge_from[e] < 0 || net->edge_from[e] >= net->n_nodes || net->edge_to[e] < 0 ||
                net->edge_to[e] >= net->n_nodes)
                bad(fmt("edge %d: node out of range", e));
            ++indeg[net->edge_to[e]];
            ++outdeg[net->edge_from[e]];
            nl += net->n_lanes[e];
        }
        for (int v = 0; v < net->n_nodes; ++v)
            if (indeg[v] * outdeg[v] > 64)
                throw Fail{SIM_EUNSUPPORTED, fmt("case 1: node %d has more than 64 (in, out) pairs", v)};
        if (nl >= (1ll << 26)) throw Fail{SIM_EUNSUPPORTED, "case 1: more than 2^26 lanes"};
    }
    if (p->record_every < 0) bad("record_every must be >= 0");
    if (!finite_in(p->v0_spread, 0.0f, 0.25f)) bad("v0_spread outside [0, 0.25]");
    // a vehicle entering an edge must land behind everything on it: the
    // overshoot of one step stays below the shortest edge minus a length
    float vmax = 0, amax = 0, lmax = 0, lmin = 1e30f, limmax = 0;
    for (int c = 0; c < p->n_classes; ++c) {
        vmax = std::max(vmax, p->v0_factor[c]);
        amax = std::max(amax, p->a[c]);
        lmax = std::max(lmax, p->length_m[c]);
    }
    for (int e = 0; e < E; ++e) {
        lmin = std::min(lmin, net->length_m[e]);
        limmax = std::max(limmax, net->speed_limit_mps[e]);
    }
    // a driver's limit is at most 1 + 12 v0_spread times the edge's (|z| <= 6)
    const double reach = ((double)vmax * limmax * (1.0 + 12.0 * (double)p->v0_spread) + (double)amax * p->dt) * p->dt +
                         lmax;
    if (lmin < reach) bad(fmt("shortest edge %.2f m is below one step's reach %.2f m", lmin, reach));

    if (r->n_vehicles < 0) bad("n_vehicles < 0");
    if (r->n_vehicles > 0 && (!r->route_off || !r->route_edges || !r->depart_step || !r->vclass || !r->alpha_s))
        bad("route array missing");
    if (r->n_vehicles > 0 && r->route_off[0] != 0) bad("route_off[0] != 0");
    for (int i = 0; i < r->n_vehicles; ++i) {
        const int64_t a = r->route_off[i], b = r->route_off[i + 1];
        if (b <= a) bad(fmt("vehicle %d: empty route", i));
        if (r->depart_step[i] < 0) bad(fmt("vehicle %d: negative departure step", i));
        if (r->vclass[i] >= p->n_classes) bad(fmt("vehicle %d: class out of range", i));
        if (!finite_in(r->alpha_s[i], 0.0f, 0.40f)) bad(fmt("vehicle %d: alpha outside [0, 0.40]", i));
        for (int64_t k = a; k < b; ++k) {
            const int e = r->route_edges[k];
            if (e < 0 || e >= E) bad(fmt("vehicle %d: route edge out of range", i));
            if (k + 1 < b) {
                const int f = r->route_edges[k + 1];
                if (f < 0 || f >= E) bad(fmt("vehicle %d: route edge out of range", i));
                bool ok = false;
                for (int c = net->conn_off[e]; c < net->conn_off[e + 1]; ++c) ok = ok || net->conn_to[c] == f;
                if (!ok) bad(fmt("vehicle %d: route is not continuous at edge %d -> %d", i, e, f));
            }
        }
    }
}

// The kernels of one step, in order.  ev (optional): 2 events per kernel,
// recorded by the runtime at the kernel's start and end.
void launch_step(sim_handle* h, hipStream_t s, hipEvent_t* ev = nullptr) {
    const Dev& d = h->d;
    const dim3 b(kNT);
    const bool lds_scan = h->n_blk <= kScanLdsMax;
    if (!ev) {
        hipLaunchKernelGGL(d.v0_spread != 0.0f ? k_tile_step_v0spread : k_tile_step, dim3(h->g_tile), dim3(kTileNT),
                           0, s, d);
        hipLaunchKernelGGL(k_big_admit, dim3(h->g_big), dim3(kBigNT), 0, s, d);
        hipLaunchKernelGGL(k_commit, dim3(h->n_blk), dim3(kCommitNT), 0, s, d);
        if (lds_scan) {
            hipLaunchKernelGGL(k_scatter<true>, dim3(h->g_scatter), b, h->scatter_lds, s, d);
        } else {
            hipLaunchKernelGGL(k_blkscan, dim3(1), dim3(kBigNT), 0, s, d);
            hipLaunchKernelGGL(k_scatter<false>, dim3(h->g_scatter), b, 0, s, d);
        }
        return;
    }
    hipExtLaunchKernelGGL(d.v0_spread != 0.0f ? k_tile_step_v0spread : k_tile_step, dim3(h->g_tile), dim3(kTileNT),
                          0, s, ev[0], ev[1], 0, d);
    hipExtLaunchKernelGGL(k_big_admit, dim3(h->g_big), dim3(kBigNT), 0, s, ev[2], ev[3], 0, d);
    if (lds_scan) {
        hipExtLaunchKernelGGL(k_commit, dim3(h->n_blk), dim3(kCommitNT), 0, s, ev[4], ev[5], 0, d);
        hipExtLaunchKernelGGL(k_scatter<true>, dim3(h->g_scatter), b, h->scatter_lds, s, ev[6], ev[7], 0, d);
    } else {   // the block scan is counted with commit
        hipExtLaunchKernelGGL(k_commit, dim3(h->n_blk), dim3(kCommitNT), 0, s, ev[4], nullptr, 0, d);
        hipExtLaunchKernelGGL(k_blkscan, dim3(1), dim3(kBigNT), 0, s, nullptr, ev[5], 0, d);
        hipExtLaunchKernelGGL(k_scatter<false>, dim3(h->g_scatter), b, 0, s, ev[6], ev[7], 0, d);
    }
}

// The dynamic state at a step boundary, as (device pointer, bytes) pieces.
template <class F>
void for_each_state_piece(sim_handle* h, F&& f) {
    Dev& d = h->d;
    const size_t N = (size_t)std::max(h->n_veh, 1), E = (size_t)h->n_edges, NL = (size_t)h->n_lanes;
    for (int b = 0; b < 2; ++b) {
        f((void*)d.s[b].x, 4 * N);
        f((void*)d.s[b].v, 4 * N);
        f((void*)d.s[b].vid, 4 * N);
        f((void*)d.s[b].edge, 4 * N);
        f((void*)d.s[b].meta, 4 * N);
        f((void*)d.s[b].nxt, 4 * N);
    }
    f((void*)d.status, N);
    f((void*)d.cursor, 4 * N);
    f((void*)d.held_since, 4 * N);
    f((void*)d.tau_in, 8 * N);
    f((void*)d.t_arr, 8 * N);
    f((void*)d.fin_x, 4 * N);
    f((void*)d.fin_v, 4 * N);
    f((void*)d.fin_meta, 4 * N);
    f((void*)d.rear, sizeof(LaneRear) * NL);
    f((void*)d.qhead, 4 * ((size_t)h->nq + 1));
    f((void*)d.qhd, sizeof(int2) * (size_t)std::max(h->nq, 1));
    f((void*)d.tt_sum, 8 * E);
    f((void*)d.tt_cnt, 8 * E);
    f((void*)d.ctl, sizeof(Ctl));
    f((void*)d.counters, sizeof(unsigned long long) * cNumCounters * kCounterCopies);
    if (d.imode == 1) f((void*)d.rr, 4 * (size_t)d.n_nodes);   // case 1 round-robin pointers
}

size_t state_bytes(sim_handle* h) {
    size_t tot = 0;
    for_each_state_piece(h, [&](void*, size_t b) { tot += (b + 255) & ~(size_t)255; });
    return tot;
}

void save_state(sim_handle* h, void* dst) {
    size_t o = 0;
    for_each_state_piece(h, [&](void* p, size_t b) {
        HIP_OK(hipMemcpyAsync((char*)dst + o, p, b, hipMemcpyDeviceToDevice, h->stream));
        o += (b + 255) & ~(size_t)255;
    });
}

void load_state(sim_handle* h, const void* src, int t) {
    size_t o = 0;
    for_each_state_piece(h, [&](void* p, size_t b) {
        HIP_OK(hipMemcpyAsync(p, (const char*)src + o, b, hipMemcpyDeviceToDevice, h->stream));
        o += (b + 255) & ~(size_t)255;
    });
    // big-tile marks of steps at or after t belong to the run being replaced
    HIP_OK(hipMemsetAsync(h->d.big_lane, 0xFF, sizeof(int2) * (size_t)h->n_lanes, h->stream));
    HIP_OK(hipMemsetAsync(h->d.moved_at, 0xFF, sizeof(int) * kMovedSlots, h->stream));
    // a step at t clears the counters of t + 1: those of t may hold a later step's count
    HIP_OK(hipMemsetAsync(tile_counters(h->d), 0, sizeof(int) * kTileCtrInts, h->stream));
    h->t = t;
}

// Graphs of one step and of kGraphSteps steps.  Every kernel reads the step
// number from the control block, so the launches of consecutive steps are the
// same and one captured sequence serves any step.
constexpr int kGraphSteps = 8;

void capture_graph(sim_handle* h) {
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->exec_k) (void)hipGraphExecDestroy(h->exec_k);
    if (h->graph_k) (void)hipGraphDestroy(h->graph_k);
    h->exec = nullptr;
    h->graph = nullptr;
    h->exec_k = nullptr;
    h->graph_k = nullptr;
    for (int which = 0; which < 2; ++which) {
        hipStream_t cs;
        HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int q = 0; q < (which ? kGraphSteps : 1); ++q) launch_step(h, cs);
            e = hipStreamEndCapture(cs, &g);
        }
        (void)hipStreamDestroy(cs);
        HIP_OK(e);
        (which ? h->graph_k : h->graph) = g;
        HIP_OK(hipGraphInstantiate(which ? &h->exec_k : &h->exec, g, nullptr, nullptr, 0));
    }
}

template <class F>
sim_status guarded(sim_handle* h, F&& f) {
    try {
        f();
        if (h) h->err.clear();
        return SIM_OK;
    } catch (const Fail& x) {
        if (h) h->err = x.msg;
        else g_create_error = x.msg;
        return x.st;
    } catch (const std::bad_alloc&) {
        if (h) h->err = "host allocation failed";
        else g_create_error = "host allocation failed";
        return SIM_ENOMEM;
    }
}

}  // namespace

extern "C" {

sim_status sim_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx) {
    if ((alloc == nullptr) != (release == nullptr)) return SIM_EINVAL;
    g_alloc = alloc;
    g_release = release;
    g_ctx = ctx;
    return SIM_OK;
}

namespace {
sim_status create_impl(const sim_network* net, const sim_routes* r, const sim_idm_params* p, const uint32_t* rng_id,
                       int32_t edge_period, sim_handle** out);
}

sim_status sim_create(const sim_network* net, const sim_routes* r, const sim_idm_params* p, sim_handle** out) {
    return create_impl(net, r, p, nullptr, net ? net->n_edges : 1, out);
}

}  // extern "C"

namespace {
// Workgroups of a kernel whose LDS fits one CU, with each workgroup's LDS
// rounded up to 1 KiB: the occupancy query alone has reported one workgroup
// more than fits for a tile kernel just below a sixth of the CU's LDS, and a
// persistent grid sized on that runs its surplus workgroups in a second wave.
int lds_fit(const void* kernel, int dev, size_t dyn = 0) {
    hipFuncAttributes fa;
    HIP_OK(hipFuncGetAttributes(&fa, kernel));
    int lds_cu = 0;
    HIP_OK(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
    const size_t per = (fa.sharedSizeBytes + dyn + 1023) / 1024 * 1024;
    if (per == 0 || lds_cu <= 0) return INT_MAX;
    return std::max(1, (int)((size_t)lds_cu / per));
}

// rng_id: per-vehicle draw id (null: the vehicle id); edge_period: the
// draws keyed by an edge use the edge id modulo this (the edges of one
// scenario in an ensemble's union network, else the edge count)
sim_status create_impl(const sim_network* net, const sim_routes* r, const sim_idm_params* p, const uint32_t* rng_id,
                       int32_t edge_period, sim_handle** out) {
    if (!out) return SIM_EINVAL;
    *out = nullptr;
    sim_handle* h = nullptr;
    sim_status st = guarded(nullptr, [&] {
        validate(net, r, p);
        h = new sim_handle();
        h->al = Alloc{g_alloc, g_release, g_ctx};
        try {
            const int E = net->n_edges, N = r->n_vehicles;
            h->n_veh = N;
            h->n_edges = E;
            h->n_classes = p->n_classes;
            Dev& d = h->d;
            // ---- network
            h->lanes.assign(E, 0);
            h->lane_base.assign(E + 1, 0);
            for (int e = 0; e < E; ++e) {
                h->lanes[e] = net->n_lanes[e];
                h->lane_base[e + 1] = h->lane_base[e] + net->n_lanes[e];
            }
            const int NL = h->lane_base[E];
            if (NL >= (1 << kLaneBaseBits))   // a lane index and a lane count share one word in the tiles
                throw Fail{SIM_EUNSUPPORTED, fmt("%d lanes: at most %d", NL, (1 << kLaneBaseBits) - 1)};
            h->n_lanes = NL;
            const int NC = net->conn_off[E];
            h->conn_off.assign(net->conn_off, net->conn_off + E + 1);
            h->conn_to.assign(net->conn_to, net->conn_to + NC);
            h->conn_mask.assign(net->conn_lane_mask, net->conn_lane_mask + NC);
            h->L.assign(net->length_m, net->length_m + E);
            d.n_edges = E;
            d.edge_period = std::max(1, edge_period);
            d.imode = p->intersection_mode;
            d.n_nodes = net->n_nodes;
            if (d.imode == 1) {
                // pairs numbered in-edge major, both in edge-id order within a node
                const int V = net->n_nodes;
                std::vector<int> indeg(V, 0), outdeg(V, 0), in_idx(E), out_idx(E), pb(E), nmv(V), rr0(V, -1);
                for (int e = 0; e < E; ++e) {
                    in_idx[e] = indeg[net->edge_to[e]]++;
                    out_idx[e] = outdeg[net->edge_from[e]]++;
                }
                for (int e = 0; e < E; ++e) pb[e] = in_idx[e] * outdeg[net->edge_to[e]];
                for (int v = 0; v < V; ++v) nmv[v] = std::max(1, indeg[v] * outdeg[v]);
                d.stop_steps = (int)std::ceil(2.0 / (double)p->dt - 1e-6);
                d.efrom = h->upload(net->edge_from, E);
                d.pair_base = h->upload(pb.data(), E);
                d.out_idx = h->upload(out_idx.data(), E);
                d.nm = h->upload(nmv.data(), V);
                d.rr = h->dev<int>(V);
                HIP_OK(hipMemcpy(d.rr, rr0.data(), sizeof(int) * V, hipMemcpyHostToDevice));
                d.win_node = h->dev<unsigned long long>(V);
                HIP_OK(hipMemset(d.win_node, 0xFF, sizeof(unsigned long long) * V));
            }
            d.n_lanes_total = NL;
            d.L = h->upload(net->length_m, E);
            d.lim = h->upload(net->speed_limit_mps, E);
            d.lanes = h->upload(h->lanes.data(), E);
            d.lane_base = h->upload(h->lane_base.data(), E + 1);
            {
                std::vector<EdgeC> ec(std::max(E, 1));
                for (int e = 0; e < E; ++e)
                    ec[e] = EdgeC{net->length_m[e], net->speed_limit_mps[e], h->lane_base[e], h->lanes[e]};
                d.ec = h->upload(ec.data(), ec.size());
            }
            // ---- classes (den = 2 sqrt(ab), rounded once in binary32)
            std::vector<ClassParams> cp(16);
            h->len_c.assign(p->n_classes, 0.f);
            h->s0_c.assign(p->n_classes, 0.f);
            float len_min = 1e30f;
            for (int c = 0; c < p->n_classes; ++c) {
                ClassParams& q = cp[c];
                q.v0f = p->v0_factor[c];
                q.T = p->T[c];
                q.a = p->a[c];
                q.b = p->b[c];
                q.s0 = p->s0[c];
                q.len = p->length_m[c];
                const float ab = q.a * q.b;
                q.den = 2.0f * sqrtf(ab);
                q.pad = 0.f;
                h->len_c[c] = q.len;
                h->s0_c[c] = q.s0;
                len_min = std::min(len_min, q.len);
            }
            d.cp = h->upload(cp.data(), 16);
            d.dt = p->dt;
            d.seed = p->seed;
            d.v0_spread = p->v0_spread;
            // ---- vehicles
            d.n_veh = N;
            h->roff.assign(r->route_off, r->route_off + N + 1);
            const int64_t NR = N ? r->route_off[N] : 0;
            h->redges.assign(r->route_edges, r->route_edges + NR);
            h->dep.assign(r->depart_step, r->depart_step + N);
            h->cls.assign(r->vclass, r->vclass + N);
            h->ins_lane.assign(N, 0);
            std::vector<int> ins_gl(N);
            for (int i = 0; i < N; ++i) {
                const int e0 = h->redges[h->roff[i]];
                int il = 0;
                if (h->roff[i + 1] - h->roff[i] > 1) {
                    const uint32_t m = h->mask_of(e0, h->redges[h->roff[i] + 1]);
                    while (il < 7 && !((m >> il) & 1u)) ++il;
                }
                h->ins_lane[i] = il;
                ins_gl[i] = h->lane_base[e0] + il;
            }
            int max_dep = -1;
            for (int i = 0; i < N; ++i) max_dep = std::max(max_dep, h->dep[i]);
            std::vector<int> due(std::max(1, max_dep + 1), 0);
            for (int i = 0; i < N; ++i) due[h->dep[i]]++;
            for (int k = 1; k <= max_dep; ++k) due[k] += due[k - 1];
            // departure queues: (entry lane, class), each sorted by (step, id)
            std::vector<int> order(N);
            for (int i = 0; i < N; ++i) order[i] = i;
            std::sort(order.begin(), order.end(), [&](int a, int b) {
                if (ins_gl[a] != ins_gl[b]) return ins_gl[a] < ins_gl[b];
                if (h->cls[a] != h->cls[b]) return h->cls[a] < h->cls[b];
                if (h->dep[a] != h->dep[b]) return h->dep[a] < h->dep[b];
                return a < b;
            });
            h->qveh = order;
            h->qoff.assign(1, 0);
            std::vector<int> qlane;
            for (int k = 0; k < N; ++k) {
                const int i = order[k];
                if (k == 0 || ins_gl[i] != ins_gl[order[k - 1]] || h->cls[i] != h->cls[order[k - 1]]) {
                    if (k > 0) h->qoff.push_back(k);
                    qlane.push_back(ins_gl[i]);
                }
            }
            if (N > 0) h->qoff.push_back(N);
            const int NQ = (int)qlane.size();
            std::vector<int4> vq(std::max(N, 1));
            for (int q = 0; q < NQ; ++q)
                for (int k = h->qoff[q]; k < h->qoff[q + 1]; ++k) {
                    const int nv = k + 1 < h->qoff[q + 1] ? h->qveh[k + 1] : -1;
                    vq[h->qveh[k]] = make_int4(q, k, nv, nv >= 0 ? h->dep[nv] : 0);
                }
            std::vector<int2> qhd(std::max(NQ, 1));
            std::vector<float> qs0(std::max(NQ, 1));
            for (int q = 0; q < NQ; ++q) {
                const int v0 = h->qveh[h->qoff[q]];
                qhd[q] = make_int2(h->dep[v0], v0);
                qs0[q] = p->s0[h->cls[v0]];
            }
            d.roff = h->upload(h->roff.data(), N + 1);
            d.redges = h->upload(h->redges.data(), (size_t)NR);
            std::vector<uint8_t> rmask(std::max<int64_t>(NR, 1), 0xFFu);
            for (int i = 0; i < N; ++i)
                for (int64_t k = h->roff[i]; k + 1 < h->roff[i + 1]; ++k)
                    rmask[k] = (uint8_t)h->mask_of(h->redges[k], h->redges[k + 1]);
            d.rmask = h->upload(rmask.data(), rmask.size());
            d.cls = h->upload(h->cls.data(), N);
            d.alpha = h->upload(r->alpha_s, N);
            d.due = h->upload(due.data(), due.size());
            d.max_dep = max_dep;
            d.qhead = h->upload(h->qoff.data(), NQ + 1);
            d.qlane = NQ ? h->upload(qlane.data(), NQ) : h->dev<int>(1);
            d.qhd = h->upload(qhd.data(), qhd.size());
            d.qs0 = h->upload(qs0.data(), qs0.size());
            d.vq = h->upload(vq.data(), vq.size());
            d.nq = NQ;
            h->nq = NQ;
            h->rec_every = p->record_every;
            std::vector<uint32_t> rid(N);
            for (int i = 0; i < N; ++i) rid[i] = rng_id ? rng_id[i] : (uint32_t)i;
            d.rid = h->upload(rid.data(), N);
            {   // the tile kernels compute a draw id as vehicle id - first vehicle of its scenario
                const int np = d.edge_period;
                const int ns = std::max(1, (E + np - 1) / np);
                std::vector<int> voff(ns + 1, INT_MAX);
                for (int i = 0; i < N; ++i) {
                    const int k = h->redges[h->roff[i]] / np;
                    voff[k] = std::min(voff[k], i);
                }
                for (int k = 0; k <= ns; ++k)
                    if (voff[k] == INT_MAX) voff[k] = 0;
                for (int i = 0; i < N; ++i)
                    if (rid[i] != (uint32_t)(i - voff[h->redges[h->roff[i]] / np]))
                        throw Fail{SIM_EUNSUPPORTED, "draw ids are not consecutive within a scenario"};
                d.scen_voff = h->upload(voff.data(), voff.size());
            }
            // ---- capacity of the largest edge (vehicles never overlap)
            long long max_edge = 1;
            for (int e = 0; e < E; ++e)
                max_edge = std::max(max_edge, (long long)h->lanes[e] * ((long long)(h->L[e] / len_min) + 1));
            const long long cap_all = std::min<long long>(std::max(N, 1), (long long)kTileWindowMax - 1 + max_edge);
            if (cap_all > kTileIndexMax)
                throw Fail{SIM_EUNSUPPORTED, fmt("a tile may hold %lld vehicles: at most %d", cap_all, kTileIndexMax)};
            d.big_cap = (int)std::max<long long>(kTileCapLds + 1, cap_all);
            {   // tile workgroups resident at once on this device
                int dev = 0, cus = 0, per_cu = 0;
                HIP_OK(hipGetDevice(&dev));
                HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
                HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tile_step, kTileNT, 0));
                per_cu = std::min(per_cu, lds_fit((const void*)k_tile_step, dev));
                d.tile_target = std::max(1, cus * std::max(per_cu, 1));
            }
            d.tile_window = 0;
            h->g_tile = std::max(1, std::min(d.tile_target, (N + kTileWindowMin - 1) / kTileWindowMin));
            {   // k_big_admit: every workgroup resident (its grid barrier), enough threads
                // for one admission item each where that fits
                int dev = 0, cus = 0, per_cu = 0;
                HIP_OK(hipGetDevice(&dev));
                HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
                HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_big_admit, kBigNT, 0));
                per_cu = std::min(per_cu, lds_fit((const void*)k_big_admit, dev));
                h->g_big_max = std::max(1, cus * std::max(per_cu, 1));
                const long long items = (long long)NL + (long long)h->nq;
                h->g_big_min = (int)std::max(1LL, std::min<long long>(h->g_big_max, (items + kBigNT - 1) / kBigNT));
                h->g_big = h->g_big_min;
            }
            h->n_blk = (E + kEdgeBlock - 1) / kEdgeBlock;
            d.n_blk = h->n_blk;
            h->scatter_lds = h->n_blk <= kScanLdsMax ? sizeof(int) * (size_t)h->n_blk : 0;
            h->g_scatter_max = std::max(1, std::min(4096, (N + kNT - 1) / kNT));
            {   // k_scatter: the workgroups resident at once, each scanning the block sums once.
                // Without the LDS scan (above kScanLdsMax blocks: tens of millions of
                // vehicles) as many as the LDS scan allows at its largest: more
                // workgroups were slower there (2,048 against 1,024 on the 4.39M-edge
                // roofline probe: 1.02 against 0.98 ms), as more scattered stores wait at once
                int dev = 0, cus = 0, per_cu = 0;
                HIP_OK(hipGetDevice(&dev));
                HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
                const size_t dyn = h->scatter_lds ? h->scatter_lds : sizeof(int) * (size_t)kScanLdsMax;
                HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_scatter<true>, kNT, dyn));
                per_cu = std::min(per_cu, lds_fit((const void*)k_scatter<true>, dev, dyn));
                h->g_scatter_res = std::max(1, std::min(cus * std::max(per_cu, 1), h->g_scatter_max));
                h->g_scatter = h->g_scatter_res;
            }
            // ---- dynamic state
            const size_t NV = std::max(N, 1);
            for (int b = 0; b < 2; ++b) {
                d.s[b].x = h->dev<float>(NV);
                d.s[b].v = h->dev<float>(NV);
                d.s[b].vid = h->dev<uint32_t>(NV);
                d.s[b].edge = h->dev<int32_t>(NV);
                d.s[b].meta = h->dev<uint32_t>(NV);
                d.s[b].nxt = h->dev<int32_t>(NV);
                d.s[b].gl = h->dev<int32_t>(NV);
            }
            d.ent = h->dev<EntryRec>(NL);
            d.status = h->dev<uint8_t>(NV);
            d.cursor = h->dev<int>(NV);
            d.held_since = h->dev<int>(NV);
            d.tau_in = h->dev<double>(NV);
            d.t_arr = h->dev<double>(NV);
            d.fin_x = h->dev<float>(NV);
            d.fin_v = h->dev<float>(NV);
            d.fin_meta = h->dev<uint32_t>(NV);
            d.rear = h->dev<LaneRear>(NL);
            d.post = h->dev<LanePost>(NL);
            d.outbox = h->dev<Outbox>(NL);
            d.req_stamp = h->dev<int>(NL);
            d.win = h->dev<unsigned long long>(NL);
            d.exit_stamp = h->dev<int>(NL);
            d.enter_stamp = h->dev<int>(NL);
            d.lane_off = h->dev<int>(NL);
            d.lane_newcnt = h->dev<int>(NL);
            d.blk_sum = h->dev<int>(h->n_blk);
            d.blk_off = h->dev<int>(h->n_blk);
            d.tt_sum = h->dev<double>(E);
            d.tt_cnt = h->dev<unsigned long long>(E);
            d.ctl = h->dev<Ctl>(1);
            d.counters = h->dev<unsigned long long>(cNumCounters * kCounterCopies);
            d.big_list = h->dev<int>(2 * ((size_t)N / kTileWindowMin + 2));
            d.big_lane = h->dev<int2>(NL);
            d.moved_at = h->dev<int>(kMovedSlots + kTileCtrInts);   // then the tile counters
            d.big_defer = h->dev<unsigned long long>((size_t)NL + (size_t)h->nq);   // each item at most once
            d.big = h->dev<char>(tile_bytes(d.big_cap) * (size_t)h->g_big_max);
            // ---- initial values
            HIP_OK(hipMemset(d.rear, 0xFF, sizeof(LaneRear) * NL));
            HIP_OK(hipMemset(d.post, 0xFF, sizeof(LanePost) * NL));
            HIP_OK(hipMemset(d.outbox, 0xFF, sizeof(Outbox) * NL));
            HIP_OK(hipMemset(d.req_stamp, 0xFF, sizeof(int) * NL));
            HIP_OK(hipMemset(d.win, 0xFF, sizeof(unsigned long long) * NL));
            HIP_OK(hipMemset(d.exit_stamp, 0xFF, sizeof(int) * NL));
            HIP_OK(hipMemset(d.enter_stamp, 0xFF, sizeof(int) * NL));
            HIP_OK(hipMemset(d.big_lane, 0xFF, sizeof(int2) * NL));
            HIP_OK(hipMemset(d.moved_at, 0xFF, sizeof(int) * kMovedSlots));
            HIP_OK(hipMemset(tile_counters(d), 0, sizeof(int) * kTileCtrInts));
            HIP_OK(hipMemset(d.tt_sum, 0, sizeof(double) * E));
            HIP_OK(hipMemset(d.tt_cnt, 0, sizeof(unsigned long long) * E));
            HIP_OK(hipMemset(d.ctl, 0, sizeof(Ctl)));
            HIP_OK(hipMemset(d.counters, 0, sizeof(unsigned long long) * cNumCounters * kCounterCopies));
            HIP_OK(hipMemset(d.status, 0, NV));
            HIP_OK(hipMemset(d.cursor, 0, sizeof(int) * NV));
            HIP_OK(hipMemset(d.held_since, 0xFF, sizeof(int) * NV));
            std::vector<double> neg1(NV, -1.0);
            HIP_OK(hipMemcpy(d.tau_in, neg1.data(), sizeof(double) * NV, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d.t_arr, neg1.data(), sizeof(double) * NV, hipMemcpyHostToDevice));
            HIP_OK(hipDeviceSynchronize());
            capture_graph(h);
        } catch (...) {
            h->release_all();
            delete h;
            h = nullptr;
            throw;
        }
    });
    if (st == SIM_OK) *out = h;
    return st;
}
}  // namespace

extern "C" {

sim_status sim_set_stream(sim_handle* h, void* stream) {
    if (!h) return SIM_EINVAL;
    return guarded(h, [&] {
        h->stream = (hipStream_t)stream;
    });
}

sim_status sim_step(sim_handle* h, int32_t n) {
    if (!h) return SIM_EINVAL;
    if (n < 0) {
        h->err = "n must be >= 0";
        return SIM_EINVAL;
    }
    return guarded(h, [&] {
        const bool rec = h->rec_every > 0 && !h->rec_broken;
        for (int q = 0; q < n;) {
            if (rec && h->t % h->rec_every == 0 && (size_t)(h->t / h->rec_every) == h->snaps.size()) {
                if (!h->snap_bytes) h->snap_bytes = state_bytes(h);
                void* p = h->al.get(h->snap_bytes);
                if (!p) throw Fail{SIM_ENOMEM, "no device memory for a checkpoint"};
                h->snaps.push_back(p);
                save_state(h, p);
            }
            // kGraphSteps at once unless a checkpoint falls strictly inside them
            const bool batch = n - q >= kGraphSteps &&
                               (!rec || (h->t / h->rec_every + 1) * h->rec_every >= h->t + kGraphSteps);
            HIP_OK(hipGraphLaunch(batch ? h->exec_k : h->exec, h->stream));
            h->t += batch ? kGraphSteps : 1;
            q += batch ? kGraphSteps : 1;
        }
        HIP_OK(hipGetLastError());
    });
}

sim_status sim_step_timed(sim_handle* h, int32_t n, double* kernel_ms, double* total_ms) {
    if (!h) return SIM_EINVAL;
    if (n < 0) {
        h->err = "n must be >= 0";
        return SIM_EINVAL;
    }
    std::vector<hipEvent_t> ev;
    sim_status st = guarded(h, [&] {
        const size_t per = 2 * SIM_N_KERNELS;
        ev.resize((size_t)n * per, nullptr);
        for (auto& e : ev) HIP_OK(hipEventCreate(&e));
        for (int q = 0; q < n; ++q) launch_step(h, h->stream, &ev[(size_t)q * per]);
        HIP_OK(hipGetLastError());
        h->t += n;
        if (h->rec_every > 0 && n > 0) h->rec_broken = true;   // timed steps take no checkpoints
        double ks[SIM_N_KERNELS] = {0};
        if (n > 0) {
            HIP_OK(hipEventSynchronize(ev.back()));
            for (int q = 0; q < n; ++q)
                for (int k = 0; k < SIM_N_KERNELS; ++k) {
                    float ms = 0.f;
                    HIP_OK(hipEventElapsedTime(&ms, ev[(size_t)q * per + 2 * k], ev[(size_t)q * per + 2 * k + 1]));
                    ks[k] += ms;
                }
        }
        if (kernel_ms)
            for (int k = 0; k < SIM_N_KERNELS; ++k) kernel_ms[k] = ks[k];
        if (total_ms) {
            float ms = 0.f;
            if (n > 0) HIP_OK(hipEventElapsedTime(&ms, ev.front(), ev.back()));
            *total_ms = ms;
        }
    });
    for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
    return st;
}

sim_status sim_n_active(sim_handle* h, int32_t* out) {
    if (!h || !out) return SIM_EINVAL;
    return guarded(h, [&] {
        Ctl c;
        HIP_OK(hipStreamSynchronize(h->stream));
        HIP_OK(hipMemcpy(&c, h->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
        if (c.err) throw Fail{SIM_EDEVICE, fmt("device layout check failed (code %d)", c.err)};
        *out = c.n_act[c.t_a & 1];
    });
}

sim_status sim_read_state(sim_handle* h, sim_state* o) {
    if (!h || !o) return SIM_EINVAL;
    return guarded(h, [&] {
        const Dev& d = h->d;
        const int N = h->n_veh;
        HIP_OK(hipStreamSynchronize(h->stream));
        Ctl c;
        HIP_OK(hipMemcpy(&c, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
        if (c.err) throw Fail{SIM_EDEVICE, fmt("device layout check failed (code %d)", c.err)};
        const int par = c.t_a & 1, na = c.n_act[par];
        std::vector<float> sx(na), sv(na), fx(N), fv(N);
        std::vector<uint32_t> svid(na), smeta(na), fmeta(N);
        std::vector<int32_t> sedge(na), cur(N), hs(N);
        std::vector<uint8_t> st(N);
        std::vector<double> tin(N), tar(N);
        const Slots S = d.s[par];
        if (na) {
            HIP_OK(hipMemcpy(sx.data(), S.x, 4 * (size_t)na, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(sv.data(), S.v, 4 * (size_t)na, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(svid.data(), S.vid, 4 * (size_t)na, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(smeta.data(), S.meta, 4 * (size_t)na, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(sedge.data(), S.edge, 4 * (size_t)na, hipMemcpyDeviceToHost));
        }
        if (N) {
            HIP_OK(hipMemcpy(st.data(), d.status, (size_t)N, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(cur.data(), d.cursor, 4 * (size_t)N, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(hs.data(), d.held_since, 4 * (size_t)N, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(tin.data(), d.tau_in, 8 * (size_t)N, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(tar.data(), d.t_arr, 8 * (size_t)N, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(fx.data(), d.fin_x, 4 * (size_t)N, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(fv.data(), d.fin_v, 4 * (size_t)N, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(fmeta.data(), d.fin_meta, 4 * (size_t)N, hipMemcpyDeviceToHost));
        }
        std::vector<int> slot_of(N, -1);
        for (int s = 0; s < na; ++s) {
            if (svid[s] >= (uint32_t)N) throw Fail{SIM_EDEVICE, "corrupt layout: vehicle id out of range"};
            slot_of[svid[s]] = s;
        }
        for (int i = 0; i < N; ++i) {
            float x = 0.f, v = 0.f;
            int edge, lane, ww = 0;
            uint8_t mand = 0;
            if (st[i] == kActive) {
                const int s = slot_of[i];
                if (s < 0) throw Fail{SIM_EDEVICE, fmt("corrupt layout: active vehicle %d has no slot", i)};
                x = sx[s];
                v = sv[s];
                edge = sedge[s];
                lane = m_lane(smeta[s]);
                mand = m_mand(smeta[s]);
                ww = m_ww(smeta[s]);
            } else if (st[i] == kArrived) {
                x = fx[i];
                v = fv[i];
                edge = h->redges[h->roff[i] + cur[i]];
                lane = m_lane(fmeta[i]);
                mand = m_mand(fmeta[i]);
                ww = m_ww(fmeta[i]);
            } else {
                edge = h->redges[h->roff[i]];
                lane = h->ins_lane[i];
            }
            if (o->status) o->status[i] = st[i];
            if (o->edge) o->edge[i] = edge;
            if (o->lane) o->lane[i] = lane;
            if (o->cursor) o->cursor[i] = cur[i];
            if (o->x) o->x[i] = x;
            if (o->v) o->v[i] = v;
            if (o->held_since) o->held_since[i] = hs[i];
            if (o->mand) o->mand[i] = mand;
            if (o->ww) o->ww[i] = ww;
            if (o->tau_in) o->tau_in[i] = tin[i];
            if (o->t_arr) o->t_arr[i] = tar[i];
        }
        if (o->counters) {
            std::vector<unsigned long long> cc((size_t)cNumCounters * kCounterCopies);
            HIP_OK(hipMemcpy(cc.data(), d.counters, 8 * cc.size(), hipMemcpyDeviceToHost));
            for (int k = 0; k < cNumCounters; ++k) {
                unsigned long long v = 0;
                for (int q = 0; q < kCounterCopies; ++q) v += cc[k * kCounterCopies + q];
                o->counters[k] = (int64_t)v;
            }
        }
        o->t = c.t_a;
    });
}

sim_status sim_write_state(sim_handle* h, const sim_state* in) {
    if (!h || !in) return SIM_EINVAL;
    return guarded(h, [&] {
        const int N = h->n_veh;
        if (!in->status || !in->edge || !in->lane || !in->cursor || !in->x || !in->v || !in->held_since ||
            !in->mand || !in->ww || !in->tau_in || !in->t_arr)
            throw Fail{SIM_EINVAL, "every state field is required"};
        if (in->t < 0) throw Fail{SIM_EINVAL, "t < 0"};
        const Dev& d = h->d;
        struct Rec {
            int edge, lane;
            float x;
            int id;
        };
        std::vector<Rec> act;
        for (int i = 0; i < N; ++i) {
            const uint8_t s = in->status[i];
            if (s > 2) throw Fail{SIM_EINVAL, fmt("vehicle %d: bad status", i)};
            const int64_t rl = h->roff[i + 1] - h->roff[i];
            if (in->cursor[i] < 0 || in->cursor[i] >= rl) throw Fail{SIM_EINVAL, fmt("vehicle %d: bad cursor", i)};
            if (s == kActive) {
                const int e = h->redges[h->roff[i] + in->cursor[i]];
                if (in->edge[i] != e) throw Fail{SIM_EINVAL, fmt("vehicle %d: edge is not the route edge", i)};
                if (in->lane[i] < 0 || in->lane[i] >= h->lanes[e]) throw Fail{SIM_EINVAL, fmt("vehicle %d: lane", i)};
                if (!(in->x[i] >= 0.f && in->x[i] <= h->L[e]) || !(in->v[i] >= 0.f) || !std::isfinite(in->v[i]))
                    throw Fail{SIM_EINVAL, fmt("vehicle %d: x or v out of range", i)};
                if (in->ww[i] < 0 || in->ww[i] > kPatience) throw Fail{SIM_EINVAL, fmt("vehicle %d: ww", i)};
                act.push_back(Rec{e, in->lane[i], in->x[i], i});
            }
        }
        std::sort(act.begin(), act.end(), [](const Rec& a, const Rec& b) {
            if (a.edge != b.edge) return a.edge < b.edge;
            if (a.lane != b.lane) return a.lane < b.lane;
            if (a.x != b.x) return a.x > b.x;
            return a.id > b.id;
        });
        for (size_t k = 1; k < act.size(); ++k)
            if (act[k].edge == act[k - 1].edge && act[k].lane == act[k - 1].lane &&
                act[k - 1].x - h->len_c[h->cls[act[k - 1].id]] < act[k].x)
                throw Fail{SIM_EINVAL, fmt("vehicles %d and %d overlap", act[k - 1].id, act[k].id)};
        const int na = (int)act.size(), t = in->t, par = t & 1;
        std::vector<float> sx(na), sv(na);
        std::vector<uint32_t> svid(na), smeta(na);
        std::vector<int32_t> sedge(na), snxt(na);
        std::vector<LaneRear> rear(h->n_lanes);
        for (auto& r : rear) r = LaneRear{0.f, 0.f, -1, 0u};
        for (int k = 0; k < na; ++k) {
            const int i = act[k].id, e = act[k].edge;
            const int64_t pos = h->roff[i] + in->cursor[i] + 1;
            const int nx = pos < h->roff[i + 1] ? h->redges[pos] : -1;
            sx[k] = in->x[i];
            sv[k] = in->v[i];
            svid[k] = (uint32_t)i;
            sedge[k] = e;
            snxt[k] = nx;
            smeta[k] = m_make(in->lane[i], in->mand[i] != 0, in->held_since[i] >= 0, in->ww[i], h->cls[i],
                              h->mask_of(e, nx));
            const bool last = (k + 1 == na) || act[k + 1].edge != e || act[k + 1].lane != act[k].lane;
            if (last) rear[h->lane_base[e] + act[k].lane] = LaneRear{in->x[i] - h->len_c[h->cls[i]], in->v[i], t, (uint32_t)i};
        }
        // departure queues: the vehicles that have left a queue must be a prefix of it
        std::vector<int> qhead(h->qoff.begin(), h->qoff.end());
        int departed = 0;
        for (size_t q = 0; q + 1 < h->qoff.size(); ++q) {
            int k = h->qoff[q];
            while (k < h->qoff[q + 1] && in->status[h->qveh[k]] != kWaiting) ++k;
            for (int k2 = k; k2 < h->qoff[q + 1]; ++k2)
                if (in->status[h->qveh[k2]] != kWaiting)
                    throw Fail{SIM_EINVAL, fmt("vehicle %d departed before an earlier vehicle of its entry lane",
                                               h->qveh[k2])};
            qhead[q] = k;
            departed += k - h->qoff[q];
        }
        std::vector<uint8_t> st(in->status, in->status + N);
        std::vector<float> fx(N, 0.f), fv(N, 0.f);
        std::vector<uint32_t> fmeta(N, 0);
        for (int i = 0; i < N; ++i)
            if (st[i] == kArrived) {
                fx[i] = in->x[i];
                fv[i] = in->v[i];
                fmeta[i] = m_make(in->lane[i], in->mand[i] != 0, false, in->ww[i], h->cls[i], 0);
            }
        HIP_OK(hipStreamSynchronize(h->stream));
        const Slots S = d.s[par];
        if (na) {
            HIP_OK(hipMemcpy(S.x, sx.data(), 4 * (size_t)na, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(S.v, sv.data(), 4 * (size_t)na, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(S.vid, svid.data(), 4 * (size_t)na, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(S.meta, smeta.data(), 4 * (size_t)na, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(S.edge, sedge.data(), 4 * (size_t)na, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(S.nxt, snxt.data(), 4 * (size_t)na, hipMemcpyHostToDevice));
        }
        if (N) {
            HIP_OK(hipMemcpy(d.status, st.data(), (size_t)N, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d.cursor, in->cursor, 4 * (size_t)N, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d.held_since, in->held_since, 4 * (size_t)N, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d.tau_in, in->tau_in, 8 * (size_t)N, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d.t_arr, in->t_arr, 8 * (size_t)N, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d.fin_x, fx.data(), 4 * (size_t)N, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d.fin_v, fv.data(), 4 * (size_t)N, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d.fin_meta, fmeta.data(), 4 * (size_t)N, hipMemcpyHostToDevice));
        }
        HIP_OK(hipMemcpy(d.qhead, qhead.data(), 4 * qhead.size(), hipMemcpyHostToDevice));
        if (h->nq > 0) {
            std::vector<int2> qhd(h->nq);
            for (int q = 0; q < h->nq; ++q)
                qhd[q] = qhead[q] < h->qoff[q + 1] ? make_int2(h->dep[h->qveh[qhead[q]]], h->qveh[qhead[q]])
                                                   : make_int2(INT_MAX, -1);
            HIP_OK(hipMemcpy(d.qhd, qhd.data(), sizeof(int2) * qhd.size(), hipMemcpyHostToDevice));
        }
        HIP_OK(hipMemcpy(d.rear, rear.data(), sizeof(LaneRear) * h->n_lanes, hipMemcpyHostToDevice));
        HIP_OK(hipMemset(d.post, 0xFF, sizeof(LanePost) * h->n_lanes));
        HIP_OK(hipMemset(d.outbox, 0xFF, sizeof(Outbox) * h->n_lanes));
        HIP_OK(hipMemset(d.req_stamp, 0xFF, sizeof(int) * h->n_lanes));
        HIP_OK(hipMemset(d.win, 0xFF, sizeof(unsigned long long) * h->n_lanes));
        HIP_OK(hipMemset(d.exit_stamp, 0xFF, sizeof(int) * h->n_lanes));
        HIP_OK(hipMemset(d.enter_stamp, 0xFF, sizeof(int) * h->n_lanes));
        HIP_OK(hipMemset(d.big_lane, 0xFF, sizeof(int2) * h->n_lanes));   // no big-tile marks of other runs
        HIP_OK(hipMemset(d.moved_at, 0xFF, sizeof(int) * kMovedSlots));     // nor movement stamps
        HIP_OK(hipMemset(tile_counters(d), 0, sizeof(int) * kTileCtrInts));   // nor tile counts
        if (d.imode == 1) {                        // the round-robin restarts
            HIP_OK(hipMemset(d.rr, 0xFF, sizeof(int) * (size_t)d.n_nodes));
            HIP_OK(hipMemset(d.win_node, 0xFF, sizeof(unsigned long long) * (size_t)d.n_nodes));
        }
        Ctl c{};
        c.t_a = t;
        c.t_b = t;
        c.n_act[par] = na;
        c.n_departed = departed;
        HIP_OK(hipMemcpy(d.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice));
        if (in->counters) {
            std::vector<unsigned long long> cc((size_t)cNumCounters * kCounterCopies, 0ull);
            for (int k = 0; k < cNumCounters; ++k) cc[(size_t)k * kCounterCopies] = (unsigned long long)in->counters[k];
            HIP_OK(hipMemcpy(d.counters, cc.data(), 8 * cc.size(), hipMemcpyHostToDevice));
        }
        HIP_OK(hipDeviceSynchronize());
        h->t = t;
        for (void* p : h->snaps) h->al.put(p);
        h->snaps.clear();
        h->rec_broken = (t != 0);
    });
}

sim_status sim_read_edge_stats(sim_handle* h, double* tt_sum, int64_t* tt_count) {
    if (!h) return SIM_EINVAL;
    return guarded(h, [&] {
        HIP_OK(hipStreamSynchronize(h->stream));
        if (tt_sum) HIP_OK(hipMemcpy(tt_sum, h->d.tt_sum, 8 * (size_t)h->n_edges, hipMemcpyDeviceToHost));
        if (tt_count) HIP_OK(hipMemcpy(tt_count, h->d.tt_cnt, 8 * (size_t)h->n_edges, hipMemcpyDeviceToHost));
    });
}

sim_status sim_read_edge_means(sim_handle* h, double* mean_s, int64_t* tt_count) {
    if (!h || !mean_s) return SIM_EINVAL;
    return guarded(h, [&] {
        const int E = h->n_edges;
        if (!h->tt_mean) h->tt_mean = h->dev<double>((size_t)E);
        hipLaunchKernelGGL(k_edge_means, dim3((E + kNT - 1) / kNT), dim3(kNT), 0, h->stream, h->d.tt_sum, h->d.tt_cnt,
                           h->tt_mean, E);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(h->stream));
        HIP_OK(hipMemcpy(mean_s, h->tt_mean, 8 * (size_t)E, hipMemcpyDeviceToHost));
        if (tt_count) HIP_OK(hipMemcpy(tt_count, h->d.tt_cnt, 8 * (size_t)E, hipMemcpyDeviceToHost));
    });
}

sim_status sim_destroy(sim_handle* h) {
    if (!h) return SIM_OK;
    (void)hipStreamSynchronize(h->stream);
    h->release_all();
    delete h;
    return SIM_OK;
}

const char* sim_last_error(const sim_handle* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

// ---- differentiable form ----------------------------------------------------
sim_status sim_backward(sim_handle* h, const double* dL_dmean_tt, double* dL_dparams) {
    if (!h || !dL_dmean_tt || !dL_dparams) return SIM_EINVAL;
    if (h->rec_every <= 0) {
        h->err = "the handle was created with record_every = 0";
        return SIM_ESTATE;
    }
    if (h->rec_broken) {
        h->err = "the forward run was not recorded from step 0 (state written or timed steps)";
        return SIM_ESTATE;
    }
    std::vector<void*> tmp;
    auto get = [&](size_t bytes) {
        void* p = h->al.get(bytes);
        if (!p) throw Fail{SIM_ENOMEM, "no device memory for the reverse sweep"};
        tmp.push_back(p);
        return p;
    };
    const Dev saved = h->d;
    const int T = h->t;
    sim_status st = guarded(h, [&] {
        const int N = std::max(h->n_veh, 1), E = h->n_edges, R = h->rec_every, NC = h->n_classes;
        const int np = 5 * NC;
        HIP_OK(hipStreamSynchronize(h->stream));
        std::vector<unsigned long long> cnt(E);
        HIP_OK(hipMemcpy(cnt.data(), h->d.tt_cnt, 8 * (size_t)E, hipMemcpyDeviceToHost));
        std::vector<double> w(E, 0.0);
        for (int e = 0; e < E; ++e) {
            if (!std::isfinite(dL_dmean_tt[e])) throw Fail{SIM_EINVAL, fmt("dL_dmean_tt[%d] is not finite", e)};
            if (cnt[e]) w[e] = dL_dmean_tt[e] / (double)cnt[e];
        }
        const int gbw = std::max(1, std::min(256, (N + kNT - 1) / kNT));
        double* dw = (double*)get(8 * (size_t)E);
        HIP_OK(hipMemcpy(dw, w.data(), 8 * (size_t)E, hipMemcpyHostToDevice));
        double* lam[5];
        for (auto& q : lam) {
            q = (double*)get(8 * (size_t)N);
            HIP_OK(hipMemsetAsync(q, 0, 8 * (size_t)N, h->stream));
        }
        double* lt = lam[4];   // lam[0..3]: the two (x, v) adjoint pairs, swapped every step
        double* gpart = (double*)get(8 * (size_t)gbw * np);
        HIP_OK(hipMemsetAsync(gpart, 0, 8 * (size_t)gbw * np, h->stream));
        TraceRec* trace = (TraceRec*)get(sizeof(TraceRec) * (size_t)R * N);
        int* nact = (int*)get(4 * (size_t)R);
        void* end_state = get(h->snap_bytes ? h->snap_bytes : (h->snap_bytes = state_bytes(h)));
        save_state(h, end_state);
        const int nseg = (T + R - 1) / R;
        if ((int)h->snaps.size() < nseg) throw Fail{SIM_ESTATE, "missing checkpoints"};
        Dev traced = saved;
        traced.trace = trace;
        traced.trace_period = R;
        traced.trace_stride = N;
        traced.nact_hist = nact;
        // per-record parts and the look-ahead lists of one reverse step
        const size_t NLs = (size_t)std::max(h->n_lanes, 1);
        BwPart* part = (BwPart*)get(sizeof(BwPart) * (size_t)N);
        int* lk_cnt = (int*)get(4 * NLs);
        int* lk_rec = (int*)get(4 * NLs * kLookListCap);
        double* lkx = (double*)get(8 * (size_t)N);
        double* lkv = (double*)get(8 * (size_t)N);
        int* lk_stamp = (int*)get(4 * (size_t)N);
        HIP_OK(hipMemsetAsync(lk_cnt, 0, 4 * NLs, h->stream));
        HIP_OK(hipMemsetAsync(lk_stamp, 0xFF, 4 * (size_t)N, h->stream));
        // one reverse step: (lx, lv) -> (nx, nv) for step index i of a segment
        auto reverse_step = [&](hipStream_t s, int i, double* ix, double* iv, double* ox, double* ov) {
            const TraceRec* tr = trace + (size_t)i * N;
            hipLaunchKernelGGL(k_backward, dim3(gbw), dim3(kNT), 0, s, saved, tr, nact + i, i, NC, ix, iv, part,
                               lk_cnt, lk_rec, lt, dw, gpart, ox, ov, N);
            hipLaunchKernelGGL(k_bw_looks, dim3(gbw), dim3(kNT), 0, s, tr, nact + i, i, part, lk_cnt, lk_rec, lkx,
                               lkv, lk_stamp);
            hipLaunchKernelGGL(k_bw_gather, dim3(gbw), dim3(kNT), 0, s, tr, nact + i, i, part, lkx, lkv, lk_stamp,
                               ox, ov);
        };
        // Full segments replay captured graphs: the traced re-run (kGraphSteps
        // steps at a time) and the whole reverse sweep of R steps, for either
        // assignment of the two adjoint buffer pairs (they swap every step).
        // The last segment may be shorter and runs launch by launch.
        hipGraph_t gg[4] = {nullptr, nullptr, nullptr, nullptr};
        hipGraphExec_t ge[4] = {nullptr, nullptr, nullptr, nullptr};   // fwd 1 step, fwd k steps, rev A, rev B
        auto capture = [&](int which) {
            hipStream_t cs;
            HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                if (which < 2) {
                    h->d = traced;
                    for (int q = 0; q < (which ? kGraphSteps : 1); ++q) launch_step(h, cs);
                    h->d = saved;
                } else {
                    double *ax = lam[0], *av = lam[1], *bx = lam[2], *bv = lam[3];
                    if (which == 3) {
                        std::swap(ax, bx);
                        std::swap(av, bv);
                    }
                    for (int i = R - 1; i >= 0; --i) {
                        reverse_step(cs, i, ax, av, bx, bv);
                        std::swap(ax, bx);
                        std::swap(av, bv);
                    }
                }
                e = hipStreamEndCapture(cs, &gg[which]);
            }
            (void)hipStreamDestroy(cs);
            HIP_OK(e);
            HIP_OK(hipGraphInstantiate(&ge[which], gg[which], nullptr, nullptr, 0));
        };
        try {
            for (int wch = 0; wch < 4; ++wch) capture(wch);
            bool a_is_in = true;                       // lx/lv are lam[0]/lam[1]
            for (int sg = nseg - 1; sg >= 0; --sg) {
                const int t0 = sg * R, t1 = std::min(T, t0 + R);
                load_state(h, h->snaps[sg], t0);
                for (int t = t0; t < t1;) {
                    const bool batch = t1 - t >= kGraphSteps;
                    HIP_OK(hipGraphLaunch(ge[batch ? 1 : 0], h->stream));
                    t += batch ? kGraphSteps : 1;
                }
                double *ix = a_is_in ? lam[0] : lam[2], *iv = a_is_in ? lam[1] : lam[3];
                double *ox = a_is_in ? lam[2] : lam[0], *ov = a_is_in ? lam[3] : lam[1];
                if (t1 - t0 == R) {
                    HIP_OK(hipGraphLaunch(ge[a_is_in ? 2 : 3], h->stream));
                } else {
                    for (int t = t1 - 1; t >= t0; --t) {
                        reverse_step(h->stream, t - t0, ix, iv, ox, ov);
                        std::swap(ix, ox);
                        std::swap(iv, ov);
                    }
                }
                if ((t1 - t0) & 1) a_is_in = !a_is_in;
            }
            HIP_OK(hipGetLastError());
        } catch (...) {
            h->d = saved;
            for (int q = 0; q < 4; ++q) {
                if (ge[q]) (void)hipGraphExecDestroy(ge[q]);
                if (gg[q]) (void)hipGraphDestroy(gg[q]);
            }
            throw;
        }
        HIP_OK(hipStreamSynchronize(h->stream));
        for (int q = 0; q < 4; ++q) {
            if (ge[q]) (void)hipGraphExecDestroy(ge[q]);
            if (gg[q]) (void)hipGraphDestroy(gg[q]);
        }
        {   // a layout or trace check of the re-runs or of the sweep failed
            Ctl c;
            HIP_OK(hipMemcpy(&c, h->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
            if (c.err) {
                load_state(h, end_state, T);
                throw Fail{SIM_EDEVICE, fmt("device check failed in the reverse sweep (code %d)", c.err)};
            }
        }
        load_state(h, end_state, T);
        std::vector<double> gp((size_t)gbw * np);
        HIP_OK(hipMemcpyAsync(gp.data(), gpart, 8 * gp.size(), hipMemcpyDeviceToHost, h->stream));
        HIP_OK(hipStreamSynchronize(h->stream));
        for (int k = 0; k < np; ++k) {
            double acc = 0.0;
            for (int b = 0; b < gbw; ++b) acc += gp[(size_t)b * np + k];
            dL_dparams[k] = acc;
        }
    });
    h->d = saved;
    h->t = T;
    (void)hipStreamSynchronize(h->stream);
    for (void* p : tmp) h->al.put(p);
    return st;
}

// ---- ensembles -----------------------------------------------------------
sim_status sim_create_ensemble(const sim_network* net, const sim_routes* m, const sim_scenario* sc, int32_t ns,
                               const sim_idm_params* p, sim_handle** out) {
    if (!out) return SIM_EINVAL;
    *out = nullptr;
    std::vector<int32_t> ef, et, co, ct, dp, re, vo;
    std::vector<float> ln, li, al;
    std::vector<uint8_t> la, cm, vc;
    std::vector<int64_t> ro;
    std::vector<uint32_t> rid;
    std::vector<float> cv0, cT, ca, cb, cs0, clen;   // classes of all scenarios (per-scenario parameters)
    sim_idm_params up{};
    bool per_scen = false;
    sim_network un{};
    sim_routes ur{};
    sim_status st = guarded(nullptr, [&] {
        auto bad = [](std::string msg) { throw Fail{SIM_EINVAL, std::move(msg)}; };
        if (!net || !m || !p || !sc) bad("null argument");
        if (ns < 1) bad("n_scen must be >= 1");
        if (net->n_edges <= 0 || net->n_nodes <= 0 || !net->conn_off || !net->n_lanes) bad("network missing");
        if (m->n_vehicles < 0 || (m->n_vehicles > 0 && (!m->route_off || !m->route_edges))) bad("master demand missing");
        const int64_t E = net->n_edges, V = net->n_nodes, NC = net->conn_off[E];
        if (E * ns >= (1ll << 27) || V * ns >= (1ll << 31)) bad("ensemble too large for 32-bit ids");
        int64_t ntot = 0;
        for (int k = 0; k < ns; ++k) {
            if (sc[k].n_vehicles < 0 || sc[k].n_vehicles > m->n_vehicles)
                bad(fmt("scenario %d: n_vehicles outside [0, master]", k));
            if (sc[k].n_reduced < 0 || (sc[k].n_reduced > 0 && !sc[k].reduced_edges))
                bad(fmt("scenario %d: reduced edges missing", k));
            for (int q = 0; q < sc[k].n_reduced; ++q)
                if (sc[k].reduced_edges[q] < 0 || sc[k].reduced_edges[q] >= E)
                    bad(fmt("scenario %d: reduced edge out of range", k));
            ntot += sc[k].n_vehicles;
        }
        if (ntot >= (1ll << 31)) bad("ensemble has too many vehicles");
        for (int k = 0; k < ns; ++k) per_scen = per_scen || sc[k].class_params != nullptr;
        const int nc = p->n_classes;
        if (per_scen) {
            // scenario k's class c becomes class k * nc + c; create_impl checks the bounds
            if (nc < 1 || !p->v0_factor || !p->T || !p->a || !p->b || !p->s0 || !p->length_m)
                bad("parameter array missing");
            if ((int64_t)ns * nc > 16) throw Fail{SIM_EUNSUPPORTED, "n_scen * n_classes above 16"};
            for (int k = 0; k < ns; ++k)
                for (int c = 0; c < nc; ++c) {
                    const float* q = sc[k].class_params ? sc[k].class_params + 5 * c : nullptr;
                    cv0.push_back(q ? q[0] : p->v0_factor[c]);
                    cT.push_back(q ? q[1] : p->T[c]);
                    ca.push_back(q ? q[2] : p->a[c]);
                    cb.push_back(q ? q[3] : p->b[c]);
                    cs0.push_back(q ? q[4] : p->s0[c]);
                    clen.push_back(p->length_m[c]);
                }
            up = *p;
            up.n_classes = ns * nc;
            up.v0_factor = cv0.data();
            up.T = cT.data();
            up.a = ca.data();
            up.b = cb.data();
            up.s0 = cs0.data();
            up.length_m = clen.data();
            for (int i = 0; i < m->n_vehicles; ++i)
                if (!m->vclass || m->vclass[i] >= nc) bad(fmt("vehicle %d: class out of range", i));
        }
        const size_t EU = (size_t)(E * ns);
        ef.resize(EU); et.resize(EU); ln.resize(EU); li.resize(EU); la.resize(EU);
        co.resize(EU + 1); ct.resize((size_t)NC * ns); cm.resize((size_t)NC * ns);
        co[0] = 0;
        for (int k = 0; k < ns; ++k) {
            std::vector<uint8_t> red((size_t)E, 0);
            for (int q = 0; q < sc[k].n_reduced; ++q) red[sc[k].reduced_edges[q]] = 1;
            for (int64_t e = 0; e < E; ++e) {
                const size_t u = (size_t)(k * E + e);
                ef[u] = (int32_t)(net->edge_from[e] + k * V);
                et[u] = (int32_t)(net->edge_to[e] + k * V);
                ln[u] = net->length_m[e];
                li[u] = net->speed_limit_mps[e];
                la[u] = red[e] ? 1 : net->n_lanes[e];
                for (int c = net->conn_off[e]; c < net->conn_off[e + 1]; ++c) {
                    const size_t cu = (size_t)(k * NC + c);
                    ct[cu] = (int32_t)(net->conn_to[c] + k * E);
                    cm[cu] = red[e] ? 1 : net->conn_lane_mask[c];
                }
                co[u + 1] = (int32_t)(k * NC + net->conn_off[e + 1]);
            }
        }
        vo.assign(ns + 1, 0);
        ro.assign(1, 0);
        for (int k = 0; k < ns; ++k) {
            const int n = sc[k].n_vehicles;
            for (int i = 0; i < n; ++i) {
                for (int64_t q = m->route_off[i]; q < m->route_off[i + 1]; ++q)
                    re.push_back((int32_t)(m->route_edges[q] + k * E));
                ro.push_back((int64_t)re.size());
                dp.push_back(m->depart_step[i]);
                vc.push_back(per_scen ? (uint8_t)(k * nc + m->vclass[i]) : m->vclass[i]);
                al.push_back(m->alpha_s[i]);
                rid.push_back((uint32_t)i);
            }
            vo[k + 1] = vo[k] + n;
        }
        un = sim_network{(int32_t)(V * ns), (int32_t)EU, ef.data(), et.data(), ln.data(), li.data(), la.data(),
                         co.data(), ct.data(), cm.data()};
        ur = sim_routes{(int32_t)ntot, ro.data(), re.data(), dp.data(), vc.data(), al.data()};
    });
    if (st != SIM_OK) return st;
    st = create_impl(&un, &ur, per_scen ? &up : p, rid.data(), net ? net->n_edges : 1, out);
    if (st == SIM_OK) {
        (*out)->n_scen = ns;
        (*out)->veh_off = vo;
    }
    return st;
}

sim_status sim_ensemble_offsets(const sim_handle* h, int32_t* n_scen, int32_t* veh_off) {
    if (!h) return SIM_EINVAL;
    if (n_scen) *n_scen = h->n_scen;
    if (veh_off) {
        if (h->veh_off.empty()) {
            veh_off[0] = 0;
            veh_off[1] = h->n_veh;
        } else {
            for (size_t k = 0; k < h->veh_off.size(); ++k) veh_off[k] = h->veh_off[k];
        }
    }
    return SIM_OK;
}

// ---- schedule and autotuner -----------------------------------------------
sim_status sim_get_schedule(const sim_handle* h, int32_t* sched) {
    if (!h || !sched) return SIM_EINVAL;
    sched[0] = h->d.tile_window;
    sched[1] = h->g_tile;
    sched[2] = h->g_big;
    sched[3] = h->g_scatter;
    return SIM_OK;
}

namespace {
bool set_schedule(sim_handle* h, int w, int g1, int g2, int g4) {
    if (w != 0 && (w < kTileWindowMin || w > kTileWindowMax || (w % 16) != 0)) return false;
    if (g1 < 1 || g2 < h->g_big_min || g2 > h->g_big_max || g4 < 1 || g4 > h->g_scatter_max) return false;
    h->d.tile_window = w;
    h->g_tile = g1;
    h->g_big = g2;
    h->g_scatter = g4;
    return true;
}
}  // namespace

sim_status sim_autotune(sim_handle* h, const char* cache_path) { return sim_autotune_steps(h, cache_path, 20); }

sim_status sim_autotune_steps(sim_handle* h, const char* cache_path, int32_t steps) {
    if (!h || steps < 1) return SIM_EINVAL;
    return guarded(h, [&] {
        char key[160];
        snprintf(key, sizeof(key), "manta-schedule E=%d L=%d N=%d S=%d", h->n_edges, h->n_lanes, h->n_veh, h->n_scen);
        if (cache_path) {
            if (FILE* f = fopen(cache_path, "r")) {
                char line[256];
                int w, g1, g2, g4;
                bool hit = false;
                while (fgets(line, sizeof(line), f)) {
                    if (strncmp(line, key, strlen(key)) == 0 && line[strlen(key)] == ' ' &&
                        sscanf(line + strlen(key), " -> %d %d %d %d", &w, &g1, &g2, &g4) == 4 &&
                        set_schedule(h, w, g1, g2, g4))
                        hit = true;
                }
                fclose(f);
                if (hit) {
                    capture_graph(h);
                    return;
                }
            }
        }
        // snapshot of the state (restored after every trial)
        const int N = h->n_veh;
        std::vector<uint8_t> st(N), mand(N);
        std::vector<int32_t> edge(N), lane(N), cur(N), hs(N), ww(N);
        std::vector<float> x(N), v(N);
        std::vector<double> tin(N), tar(N);
        std::vector<int64_t> cnt(SIM_N_COUNTERS);
        sim_state snap{st.data(), edge.data(), lane.data(), cur.data(), x.data(), v.data(), hs.data(),
                       mand.data(), ww.data(), tin.data(), tar.data(), cnt.data(), 0};
        if (sim_read_state(h, &snap) != SIM_OK) throw Fail{SIM_EDEVICE, h->err};
        const size_t E = (size_t)h->n_edges;
        std::vector<double> tts(E);
        std::vector<unsigned long long> ttc(E);
        HIP_OK(hipMemcpy(tts.data(), h->d.tt_sum, 8 * E, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(ttc.data(), h->d.tt_cnt, 8 * E, hipMemcpyDeviceToHost));
        const int w0 = h->d.tile_window, g10 = h->g_tile, g20 = h->g_big, g40 = h->g_scatter;
        struct Cand {
            int w, g1, g2, g4;
        };
        std::vector<Cand> cands;
        for (int w : {0, 64, 128, 256})
            for (int g1 : {std::max(1, h->d.tile_target / 2), h->d.tile_target})
                for (int g2 : {h->g_big_min, h->g_big_max})
                    for (int g4 : {h->g_scatter_res, 4096}) {
                        const int g1c = std::max(1, std::min(g1, (N + (w ? w : kTileWindowMin) - 1) /
                                                                     (w ? w : kTileWindowMin)));
                        const int g4c = std::max(1, std::min(g4, h->g_scatter_max));
                        bool dup = false;
                        for (auto& c : cands) dup = dup || (c.w == w && c.g1 == g1c && c.g2 == g2 && c.g4 == g4c);
                        if (!dup) cands.push_back(Cand{w, g1c, g2, g4c});
                    }
        double best_ms = 1e30;
        Cand best{w0, g10, g20, g40};
        hipEvent_t e0, e1;
        HIP_OK(hipEventCreate(&e0));
        HIP_OK(hipEventCreate(&e1));
        for (const Cand& c : cands) {
            if (!set_schedule(h, c.w, c.g1, c.g2, c.g4)) continue;
            if (sim_write_state(h, &snap) != SIM_OK) throw Fail{SIM_EDEVICE, h->err};
            launch_step(h, h->stream);   // first launch of a schedule is not timed
            HIP_OK(hipEventRecord(e0, h->stream));
            for (int q = 0; q < steps; ++q) launch_step(h, h->stream);
            HIP_OK(hipEventRecord(e1, h->stream));
            HIP_OK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        set_schedule(h, best.w, best.g1, best.g2, best.g4);
        if (sim_write_state(h, &snap) != SIM_OK) throw Fail{SIM_EDEVICE, h->err};
        HIP_OK(hipMemcpy(h->d.tt_sum, tts.data(), 8 * E, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(h->d.tt_cnt, ttc.data(), 8 * E, hipMemcpyHostToDevice));
        capture_graph(h);
        if (cache_path) {
            if (FILE* f = fopen(cache_path, "a")) {
                fprintf(f, "%s -> %d %d %d %d\n", key, best.w, best.g1, best.g2, best.g4);
                fclose(f);
            }
        }
    });
}

sim_status sim_big_tile_updates(sim_handle* h, int64_t* updates) {
    if (!h || !updates) return SIM_EINVAL;
    return guarded(h, [&] {
        Ctl c;
        HIP_OK(hipStreamSynchronize(h->stream));
        HIP_OK(hipMemcpy(&c, h->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
        *updates = (int64_t)c.big_updates;
    });
}

// ---- diagnostics ---------------------------------------------------------
sim_status sim_probe_fp32(int32_t op, const float* a, const float* b, float* out, int64_t n) {
    if (!a || !out || n < 0 || op < 0 || op > 4 || ((op == 0 || op == 2 || op == 3) && !b)) return SIM_EINVAL;
    if (n == 0) return SIM_OK;
    float *da = nullptr, *db = nullptr, *dout = nullptr;
    sim_status st = guarded(nullptr, [&] {
        HIP_OK(hipMalloc(&da, 4 * n));
        HIP_OK(hipMalloc(&dout, 4 * n));
        HIP_OK(hipMemcpy(da, a, 4 * n, hipMemcpyHostToDevice));
        if (b) {
            HIP_OK(hipMalloc(&db, 4 * n));
            HIP_OK(hipMemcpy(db, b, 4 * n, hipMemcpyHostToDevice));
        }
        const int g = (int)std::min<int64_t>(4096, (n + 255) / 256);
        hipLaunchKernelGGL(k_probe_fp32, dim3(g), dim3(256), 0, 0, op, da, db, dout, n);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpy(out, dout, 4 * n, hipMemcpyDeviceToHost));
    });
    (void)hipFree(da);
    (void)hipFree(db);
    (void)hipFree(dout);
    return st;
}

sim_status sim_probe_philox(const uint64_t* counters, const uint64_t* key, uint64_t* out, int64_t n) {
    if (!counters || !key || !out || n < 0) return SIM_EINVAL;
    if (n == 0) return SIM_OK;
    uint64_t *dc = nullptr, *dout = nullptr;
    sim_status st = guarded(nullptr, [&] {
        HIP_OK(hipMalloc(&dc, 32 * n));
        HIP_OK(hipMalloc(&dout, 32 * n));
        HIP_OK(hipMemcpy(dc, counters, 32 * n, hipMemcpyHostToDevice));
        const int g = (int)std::min<int64_t>(4096, (n + 255) / 256);
        hipLaunchKernelGGL(k_probe_philox, dim3(g), dim3(256), 0, 0, dc, key[0], key[1], dout, n);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpy(out, dout, 32 * n, hipMemcpyDeviceToHost));
    });
    (void)hipFree(dc);
    (void)hipFree(dout);
    return st;
}

sim_status sim_probe_draws(uint64_t seed, const int64_t* t, const int64_t* id, float* u, float* e2, float* e3,
                           int64_t n) {
    if (!t || !id || !u || !e2 || !e3 || n < 0) return SIM_EINVAL;
    if (n == 0) return SIM_OK;
    int64_t *dt = nullptr, *did = nullptr;
    float* dout = nullptr;
    sim_status st = guarded(nullptr, [&] {
        HIP_OK(hipMalloc(&dt, 8 * n));
        HIP_OK(hipMalloc(&did, 8 * n));
        HIP_OK(hipMalloc(&dout, 12 * n));
        HIP_OK(hipMemcpy(dt, t, 8 * n, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(did, id, 8 * n, hipMemcpyHostToDevice));
        const int g = (int)std::min<int64_t>(4096, (n + 255) / 256);
        hipLaunchKernelGGL(k_probe_draws, dim3(g), dim3(256), 0, 0, seed, dt, did, dout, dout + n, dout + 2 * n, n);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpy(u, dout, 4 * n, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(e2, dout + n, 4 * n, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(e3, dout + 2 * n, 4 * n, hipMemcpyDeviceToHost));
    });
    (void)hipFree(dt);
    (void)hipFree(did);
    (void)hipFree(dout);
    return st;
}

}  // extern "C"

// ---- routes on travel times ------------------------------------------------
namespace {
// Device buffers of one routing call, from the allocator set by
// sim_set_allocator (hipMalloc without one), returned on every exit; the call
// has synchronized the device before it returns them.
struct DevBufs {
    Alloc al{g_alloc, g_release, g_ctx};
    std::vector<void*> p;
    size_t left() const { return SIZE_MAX; }
    template <class T>
    T* get(size_t n) {
        const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
        void* q = al.get(bytes);
        if (!q) throw Fail{SIM_ENOMEM, fmt("device allocation of %zu bytes failed", bytes)};
        p.push_back(q);
        return (T*)q;
    }
    ~DevBufs() {
        for (void* q : p) al.put(q);
    }
};
}  // namespace

namespace {
// Device memory of one routing call carved out of a fixed region (the
// no-allocation entry point): 256-byte aligned pieces, SIM_EINVAL past its end.
struct ScratchBufs {
    char* base;
    size_t cap, used = 0;
    size_t left() const { return cap - used; }
    template <class T>
    T* get(size_t n) {
        const size_t bytes = (std::max<size_t>(n, 1) * sizeof(T) + 255) & ~(size_t)255;
        if (used + bytes > cap)
            throw Fail{SIM_EINVAL, fmt("the call needs more than the %zu bytes of scratch of "
                                       "sim_shortest_routes_noalloc", cap)};
        T* q = (T*)(base + used);
        used += bytes;
        return q;
    }
};

// The routes of Sec. II-C on the GPU; B provides the call's device buffers.
template <class B>
void shortest_routes_impl(B& b, const sim_network* net, const float* edge_cost, int32_t n_queries,
                          const int32_t* origin, const int32_t* dest, int64_t* route_off, int32_t* route_edges,
                          int64_t capacity, int64_t* n_route_edges) {
    {
        auto bad = [](std::string m) { throw Fail{SIM_EINVAL, std::move(m)}; };
        if (!net || !edge_cost || !route_off || !n_route_edges || n_queries < 0) bad("null argument");
        if (n_queries > 0 && (!origin || !dest)) bad("null argument");
        const int V = net->n_nodes, E = net->n_edges;
        if (V <= 0 || E <= 0 || !net->edge_from || !net->edge_to) bad("network must have nodes and edges");
        for (int e = 0; e < E; ++e) {
            if (net->edge_from[e] < 0 || net->edge_from[e] >= V || net->edge_to[e] < 0 || net->edge_to[e] >= V)
                bad(fmt("edge %d: node out of range", e));
            if (!(std::isfinite(edge_cost[e]) && edge_cost[e] > 0.0f)) bad(fmt("edge %d: cost not finite and > 0", e));
        }
        for (int q = 0; q < n_queries; ++q)
            if (origin[q] < 0 || origin[q] >= V || dest[q] < 0 || dest[q] >= V) bad(fmt("query %d: node out of range", q));
        route_off[0] = 0;
        if (n_queries == 0) {
            *n_route_edges = 0;
            return;
        }
        // out-edges per node, ascending edge id
        std::vector<int> out_off(V + 1, 0), out_edge(E), fill(V, 0);
        for (int e = 0; e < E; ++e) ++out_off[net->edge_from[e] + 1];
        for (int v = 0; v < V; ++v) out_off[v + 1] += out_off[v];
        for (int e = 0; e < E; ++e) out_edge[out_off[net->edge_from[e]] + fill[net->edge_from[e]]++] = e;
        // one label array per distinct destination
        std::vector<int> slot_of(V, -1), dests, slot(n_queries);
        for (int q = 0; q < n_queries; ++q) {
            if (slot_of[dest[q]] < 0) {
                slot_of[dest[q]] = (int)dests.size();
                dests.push_back(dest[q]);
            }
            slot[q] = slot_of[dest[q]];
        }
        const int nd = (int)dests.size();
        if ((double)nd * V * 4.0 > 16e9) throw Fail{SIM_EUNSUPPORTED, "labels of all destinations above 16 GB"};
        int* d_off = b.template get<int>(V + 1);
        int* d_oe = b.template get<int>(E);
        int* d_to = b.template get<int>(E);
        float* d_cost = b.template get<float>(E);
        int* d_dest = b.template get<int>(nd);
        float* d_dist = b.template get<float>((size_t)nd * V);
        int* d_slot = b.template get<int>(n_queries);
        int* d_o = b.template get<int>(n_queries);
        int* d_d = b.template get<int>(n_queries);
        int* d_len = b.template get<int>(n_queries);
        HIP_OK(hipMemcpy(d_off, out_off.data(), 4 * (size_t)(V + 1), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d_oe, out_edge.data(), 4 * (size_t)E, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d_to, net->edge_to, 4 * (size_t)E, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d_cost, edge_cost, 4 * (size_t)E, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d_dest, dests.data(), 4 * (size_t)nd, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d_slot, slot.data(), 4 * (size_t)n_queries, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d_o, origin, 4 * (size_t)n_queries, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d_d, dest, 4 * (size_t)n_queries, hipMemcpyHostToDevice));
        int max_deg = 0;
        for (int v = 0; v < V; ++v) max_deg = std::max(max_deg, out_off[v + 1] - out_off[v]);
        const dim3 gd(std::min(nd, 2048));
        if (V > kRouteMaxNodes) {   // labels in global memory, relaxed from a frontier
            std::vector<int> in_off(V + 1, 0), in_edge(E), fill_in(V, 0);
            for (int e = 0; e < E; ++e) ++in_off[net->edge_to[e] + 1];
            for (int v = 0; v < V; ++v) in_off[v + 1] += in_off[v];
            for (int e = 0; e < E; ++e) in_edge[in_off[net->edge_to[e]] + fill_in[net->edge_to[e]]++] = e;
            int* d_ioff = b.template get<int>(V + 1);
            int* d_iedge = b.template get<int>(E);
            int* d_from = b.template get<int>(E);
            HIP_OK(hipMemcpy(d_ioff, in_off.data(), 4 * (size_t)(V + 1), hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d_iedge, in_edge.data(), 4 * (size_t)E, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d_from, net->edge_from, 4 * (size_t)E, hipMemcpyHostToDevice));
            // frontier (2 V) and marks (V) per workgroup, as many workgroups as fit
            const size_t per_wg = 3 * 4 * (size_t)V + 512;
            const int g = (int)std::max<size_t>(1, std::min<size_t>({(size_t)nd, (size_t)1024, b.left() / per_wg}));
            int* d_fq = b.template get<int>((size_t)g * 2 * V);
            int* d_mk = b.template get<int>((size_t)g * V);
            hipLaunchKernelGGL(k_route_dist_global, dim3(g), dim3(kRouteNT), 0, 0, V, d_ioff, d_iedge, d_from, d_cost,
                               d_dest, nd, d_dist, d_fq, d_mk);
        } else if (max_deg <= 8) {   // padded adjacency, slot-major: [j * V + v]
            const int km = max_deg <= 4 ? 4 : 8;
            std::vector<int> pto((size_t)km * V);
            std::vector<float> pcost((size_t)km * V);
            for (int v = 0; v < V; ++v)
                for (int j = 0; j < km; ++j) {
                    const int k = out_off[v] + j;
                    const bool has = k < out_off[v + 1];
                    pto[(size_t)j * V + v] = has ? net->edge_to[out_edge[k]] : v;
                    pcost[(size_t)j * V + v] = has ? edge_cost[out_edge[k]] : INFINITY;
                }
            int* d_pto = b.template get<int>((size_t)km * V);
            float* d_pcost = b.template get<float>((size_t)km * V);
            HIP_OK(hipMemcpy(d_pto, pto.data(), 4 * (size_t)km * V, hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d_pcost, pcost.data(), 4 * (size_t)km * V, hipMemcpyHostToDevice));
            if (km == 4 && V <= 10 * kRouteNT)   // adjacency in registers
                hipLaunchKernelGGL((k_route_dist_regs<4, 10>), gd, dim3(kRouteNT), 0, 0, V, d_pto, d_pcost, d_dest, nd,
                                   d_dist);
            else if (km == 4)
                hipLaunchKernelGGL(k_route_dist_padded<4>, gd, dim3(kRouteNT), 0, 0, V, d_pto, d_pcost, d_dest, nd, d_dist);
            else
                hipLaunchKernelGGL(k_route_dist_padded<8>, gd, dim3(kRouteNT), 0, 0, V, d_pto, d_pcost, d_dest, nd, d_dist);
        } else {
            hipLaunchKernelGGL(k_route_dist, gd, dim3(kRouteNT), 0, 0, V, d_off, d_oe, d_to, d_cost, d_dest, nd, d_dist);
        }
        HIP_OK(hipGetLastError());
        const int gw = std::max(1, std::min(4096, (n_queries + 255) / 256));
        hipLaunchKernelGGL(k_route_walk, dim3(gw), dim3(256), 0, 0, V, d_off, d_oe, d_to, d_cost, d_dist, d_slot, d_o,
                           d_d, n_queries, 0, d_len, (const int64_t*)nullptr, (int*)nullptr);
        HIP_OK(hipGetLastError());
        std::vector<int> len(n_queries);
        HIP_OK(hipMemcpy(len.data(), d_len, 4 * (size_t)n_queries, hipMemcpyDeviceToHost));
        for (int q = 0; q < n_queries; ++q) {
            if (len[q] < 0) bad(fmt("query %d: no route from node %d to node %d", q, origin[q], dest[q]));
            route_off[q + 1] = route_off[q] + len[q];
        }
        *n_route_edges = route_off[n_queries];
        if (!route_edges || capacity < route_off[n_queries])
            bad(fmt("route_edges holds %lld edges, the routes need %lld", (long long)capacity,
                    (long long)route_off[n_queries]));
        int64_t* d_roff = b.template get<int64_t>(n_queries + 1);
        int* d_re = b.template get<int>((size_t)route_off[n_queries]);
        HIP_OK(hipMemcpy(d_roff, route_off, 8 * (size_t)(n_queries + 1), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_route_walk, dim3(gw), dim3(256), 0, 0, V, d_off, d_oe, d_to, d_cost, d_dist, d_slot, d_o,
                           d_d, n_queries, 1, d_len, (const int64_t*)d_roff, d_re);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpy(route_edges, d_re, 4 * (size_t)route_off[n_queries], hipMemcpyDeviceToHost));
    }
}

// Scratch of sim_shortest_routes_noalloc: every device that runs it holds one
// copy until the process ends.  Host code reaches a device's copy through the
// address hipGetSymbolAddress returns on that device, never through the name.
constexpr size_t kRouteScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kRouteScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* route_scratch() {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Fail{SIM_EUNSUPPORTED, fmt("device %d: too many devices", dev)};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw Fail{SIM_EDEVICE, "no address for the routing scratch"};
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" sim_status sim_shortest_routes(const sim_network* net, const float* edge_cost, int32_t n_queries,
                                          const int32_t* origin, const int32_t* dest, int64_t* route_off,
                                          int32_t* route_edges, int64_t capacity, int64_t* n_route_edges) {
    return guarded(nullptr, [&] {
        DevBufs b;
        shortest_routes_impl(b, net, edge_cost, n_queries, origin, dest, route_off, route_edges, capacity,
                             n_route_edges);
    });
}

extern "C" sim_status sim_shortest_routes_noalloc(const sim_network* net, const float* edge_cost, int32_t n_queries,
                                                  const int32_t* origin, const int32_t* dest, int64_t* route_off,
                                                  int32_t* route_edges, int64_t capacity, int64_t* n_route_edges) {
    return guarded(nullptr, [&] {
        ScratchBufs b{(char*)route_scratch(), kRouteScratchBytes};
        shortest_routes_impl(b, net, edge_cost, n_queries, origin, dest, route_off, route_edges, capacity,
                             n_route_edges);
    });
}
