/*
 * libmanta — per-timestep vehicle update of the MANTA traffic microsimulation
 * (Yedavalli, Kumar, Waddell, arXiv 2007.03614) on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  Unless a comment says "device",
 * every pointer argument is a HOST pointer: inputs are borrowed for the call
 * and deep-copied; outputs are caller-owned buffers of the stated length.
 *
 * Conventions
 *   - Every call returns sim_status; nothing throws or aborts across the ABI.
 *   - On error the handle is left unchanged and sim_last_error() describes it.
 *   - One handle is not thread-safe; separate handles are independent.
 *   - Device memory comes from the allocator registered with
 *     sim_set_allocator() (default: hipMalloc/hipFree).  All device work of a
 *     handle runs on its stream (sim_set_stream; default: the null stream).
 *
 * What one step computes (Sec. II-D of the paper, with dt = 0.5 s):
 *   for every active vehicle, find its leader on its lane, evaluate the
 *   Intelligent Driver Model (Eq. (1)), decide lane changes (mandatory-change
 *   probability Eq. (2), critical lead/lag gaps Eqs. (3)-(4)), advance
 *   position and speed, and hand vehicles that reach the end of their edge
 *   to the next edge of their fixed route through intersection admission
 *   (case 2: every node green, finite lane capacity).
 */
#ifndef MANTA_H
#define MANTA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sim_handle sim_handle;   /* opaque; owns all its device memory */

typedef enum {
    SIM_OK = 0,
    SIM_EINVAL = -1,        /* an argument or input array is invalid */
    SIM_ENOMEM = -2,        /* the allocator returned NULL */
    SIM_EDEVICE = -3,       /* a HIP runtime call failed */
    SIM_ESTATE = -4,        /* call not valid in the handle's current state */
    SIM_EUNSUPPORTED = -5   /* a documented option that is not implemented */
} sim_status;

/* Road network (Sec. II-A): directed edges with lanes, length and speed limit;
 * a CSR of allowed moves e -> f with a per-move lane mask (bit l set: lane l
 * of e, counted from the right, may proceed to f). */
typedef struct {
    int32_t n_nodes, n_edges;
    const int32_t *edge_from, *edge_to;   /* [n_edges] node ids */
    const float *length_m;                /* [n_edges], >= 20 m */
    const float *speed_limit_mps;         /* [n_edges], > 0 */
    const uint8_t *n_lanes;               /* [n_edges], 1..8 */
    const int32_t *conn_off;              /* [n_edges + 1], non-decreasing, conn_off[0] = 0 */
    const int32_t *conn_to;               /* [conn_off[n_edges]] edge ids, from(f) == to(e) */
    const uint8_t *conn_lane_mask;        /* [conn_off[n_edges]], non-zero, < 2^n_lanes[e] */
} sim_network;

/* Fixed routes computed before the simulation (Sec. II-C) and departures
 * (Sec. II-D).  Vehicle id == index. */
typedef struct {
    int32_t n_vehicles;                   /* >= 0, < 2^31 */
    const int64_t *route_off;             /* [n_vehicles + 1], route_off[0] = 0, strictly increasing */
    const int32_t *route_edges;           /* consecutive edges connected by an allowed move */
    const int32_t *depart_step;           /* [n_vehicles], >= 0: enters at the end of this step */
    const uint8_t *vclass;                /* [n_vehicles], < n_classes */
    const float *alpha_s;                 /* [n_vehicles], anticipation time, [0, 0.40] (Eqs. (3)-(4)) */
} sim_routes;

/* Car-following parameters per vehicle class (Eq. (1), Table I), bounds of
 * Sec. IV-A: a, b in [1, 10] m/s^2, T in [0.1, 2] s, s0 in [1, 5] m;
 * v0 = v0_factor * edge speed limit, v0_factor in (0, 2]; length in (0, 20] m. */
typedef struct {
    int32_t n_classes;                    /* 1..16 */
    const float *v0_factor, *T, *a, *b, *s0, *length_m;   /* [n_classes] */
    float dt;                             /* (0, 1]; the paper uses 0.5 s */
    uint64_t seed;                        /* Philox key for the lane-change draws */
    int32_t intersection_mode;            /* Sec. II-D traffic control.  0 = case 2, all green: a front crosses
                                           * when the target lane has room.  1 = case 1, flashing red: a front
                                           * crosses only after standing ceil(2 s / dt) steps at the stop line,
                                           * and each node passes one vehicle per step, its (in, out) pairs
                                           * served round-robin (in-edge major, edge-id order; within a pair,
                                           * earliest at the line, then lowest source lane).  Case 1 needs at
                                           * most 64 pairs per node and fewer than 2^26 lanes, else
                                           * SIM_EUNSUPPORTED; other values SIM_EINVAL.  sim_write_state
                                           * restarts the round-robin. */
    int32_t record_every;                 /* >= 0; > 0: keep a checkpoint every record_every steps for sim_backward */
    float v0_spread;                      /* [0, 0.25]; per-driver free-flow speed (Sec. IV, model validation):
                                           * driver i on edge e drives at v0_factor * limit_e * f_i,e with
                                           * f = max(1 + 2 v0_spread z, 0.1), z ~ N(0, 1) (Irwin-Hall of twelve
                                           * Philox uniforms, stream 4, counter (edge, vehicle, 4, block)) fixed
                                           * per driver and edge; 0 = every driver at the limit */
} sim_idm_params;

/* Per-vehicle state, all arrays [n_vehicles] indexed by vehicle id; any
 * pointer may be NULL to skip that field.  status: 0 waiting, 1 active,
 * 2 arrived.  For a waiting vehicle edge/lane are its first edge and entry
 * lane and x = v = 0.  counters: [SIM_N_COUNTERS] (cumulative). */
typedef struct {
    uint8_t *status;
    int32_t *edge, *lane, *cursor;
    float *x, *v;                         /* metres from the edge start (front bumper), m/s */
    int32_t *held_since;                  /* -1, or the step a held transfer was first refused */
    uint8_t *mand;                        /* mandatory lane change pending (Eq. (2)) */
    int32_t *ww;                          /* steps held at the stop line in a wrong lane */
    double *tau_in;                       /* time the current edge was entered, s (-1 waiting) */
    double *t_arr;                        /* arrival time, s (-1 not arrived) */
    int64_t *counters;
    int32_t t;                            /* out: current step */
} sim_state;

/* Cumulative counters (sim_state.counters order). */
enum {
    SIM_C_ACTIVE_SUM = 0,     /* sum over steps of vehicles active at the step's start */
    SIM_C_DEPARTED,           /* admitted departures */
    SIM_C_ARRIVED,
    SIM_C_LANE_CHANGES,
    SIM_C_TRANSFERS,          /* admitted edge-to-edge transfers */
    SIM_C_HOLDS,              /* transfer requests refused (vehicle held at the stop line) */
    SIM_C_INSERT_DENIED,      /* departure requests refused */
    SIM_C_MAND_TRIGGERS,      /* mandatory lane-change flags raised by Eq. (2) */
    SIM_C_STOP_BRANCH,        /* integration steps that ended in a stop */
    SIM_C_CLAMP,              /* positions clamped to the leader's rear */
    SIM_C_WRONG_LANE_HOLDS,   /* steps held at the stop line in a wrong lane */
    SIM_C_WAIVED_EXITS,       /* transfers from a wrong lane after the patience ran out */
    SIM_C_GRIDLOCK_STEPS,     /* gridlock detector (failure detection, not part of the method): steps that end
                               * a run of at least 600 consecutive stalled steps, a stalled step being one with
                               * active vehicles at its start of which none changed position (in the update of
                               * Eq. (1)) or lane, crossed to another edge or arrived, and with no departure.
                               * sim_write_state restarts the run; in an ensemble the run is over all scenarios */
    SIM_N_COUNTERS
};

/* Process-wide device allocator used by handles created afterwards.
 * alloc(bytes, ctx) returns a device pointer or NULL; release(ptr, ctx).
 * Pass NULL, NULL to restore hipMalloc/hipFree.  Both are called only from
 * the thread calling sim_create or sim_destroy. */
sim_status sim_set_allocator(void *(*alloc)(size_t bytes, void *ctx),
                             void (*release)(void *ptr, void *ctx), void *ctx);

/* Validate and deep-copy the inputs, build the device layout, and leave the
 * simulation at step 0 with every vehicle waiting.  Validation: node ids in
 * range, lanes 1..8, length >= 20 m, limit > 0 and finite, moves connect
 * (from(f) == to(e)) with a non-empty lane mask inside the lanes of e, every
 * route non-empty with consecutive edges joined by a move, depart_step >= 0,
 * class ids in range, alpha finite in [0, 0.40], parameters finite and in the
 * bounds above.  Errors: SIM_EINVAL, SIM_ENOMEM, SIM_EDEVICE, SIM_EUNSUPPORTED (also for
 * 2^24 lanes or more in all, or an edge that could hold more than 32,767
 * vehicles at the shortest vehicle length). */
sim_status sim_create(const sim_network *net, const sim_routes *routes, const sim_idm_params *params,
                      sim_handle **out);

/* What-if scenario of an ensemble: a demand subset and capacity cuts on the
 * shared network (the paper's use case of quickly comparing scenarios,
 * Sec. I; calibration runs several parameter sets per iteration, Sec. IV-A). */
typedef struct {
    int32_t n_vehicles;                   /* the first n_vehicles of the master demand, 0..master */
    int32_t n_reduced;                    /* >= 0 */
    const int32_t *reduced_edges;         /* [n_reduced] edge ids forced to 1 lane (all moves from lane 0) */
    const float *class_params;            /* optional [5 * n_classes]: this scenario's (v0_factor, T, a, b, s0)
                                           * per class (Sec. IV-A runs several parameter sets per calibration
                                           * iteration); NULL: the shared parameters.  If any scenario gives
                                           * them, class c of scenario k is class k * n_classes + c of the
                                           * handle (state, sim_backward), n_scen * n_classes <= 16 (else
                                           * SIM_EUNSUPPORTED), each value within the bounds of sim_create */
} sim_scenario;

/* One handle running n_scen >= 1 scenarios in the same kernels: the device
 * network is the disjoint union of the scenario copies (edge k*n_edges + e,
 * node k*n_nodes + v, vehicle ids scenario after scenario), so every launch of
 * a step covers all scenarios.  The lane-change draws use each vehicle's id
 * within its scenario, so member k evolves exactly like sim_create on its own
 * network and demand.  State and edge statistics are read in the union
 * numbering (sim_ensemble_offsets gives the vehicle ranges).  Errors as
 * sim_create, plus SIM_EINVAL for an empty scenario list, n_vehicles outside
 * [0, master], or a reduced edge out of range. */
sim_status sim_create_ensemble(const sim_network *net, const sim_routes *master, const sim_scenario *scen,
                               int32_t n_scen, const sim_idm_params *params, sim_handle **out);

/* Gradient of a loss of the per-edge mean traversal times with respect to
 * the class parameters, by the adjoint of the step with every discrete
 * decision of the recorded forward run held fixed (leaders, lane changes,
 * IDM branches, stops, clamps, admissions, arrivals).  Needs a handle created
 * with record_every > 0 whose steps since step 0 all went through sim_step;
 * the segments between checkpoints are re-run with a trace and swept in
 * reverse (continuous parts of Eq. (1), the integration, the leader coupling
 * and the crossing-time interpolation of Sec. IV-A's per-edge outputs).
 * dL_dmean_tt: [n_edges] (edges without a completed traversal are ignored);
 * dL_dparams: [5 * n_classes] out, per class (v0_factor, T, a, b, s0).
 * The handle's state is left as it was.  Adjoint arithmetic is FP64 with
 * atomic accumulation into leaders; parameter sums are reduced in a fixed
 * order.  Errors: SIM_ESTATE (not recorded), SIM_EINVAL, SIM_ENOMEM. */
sim_status sim_backward(sim_handle *h, const double *dL_dmean_tt, double *dL_dparams);

/* veh_off[n_scen + 1]: vehicles of scenario k are [veh_off[k], veh_off[k+1]). */
sim_status sim_ensemble_offsets(const sim_handle *h, int32_t *n_scen, int32_t *veh_off);

/* Pick the launch schedule (tile window, workgroups per kernel) by timing
 * 20 steps of each candidate from the current state, which is restored
 * afterwards.  The choice is appended to cache_path (text, one line per
 * network/demand size) and reused from there when the same sizes come back;
 * cache_path may be NULL.  Results of the simulation never depend on the
 * schedule. */
sim_status sim_autotune(sim_handle *h, const char *cache_path);

/* The same with steps_per_trial (>= 1) steps per candidate. */
sim_status sim_autotune_steps(sim_handle *h, const char *cache_path, int32_t steps_per_trial);

/* Current schedule, sched[4]: [tile_window, tile_workgroups,
 * big_tile_and_admission_workgroups, scatter_workgroups].  tile_window 0 (the
 * default) picks the window at every step: the fewest rounds of the tile
 * workgroups the device holds at once that windows of at most 192 slots
 * allow, with the smallest window (a multiple of 16, at least 64) that gives
 * them.  A fixed window is a multiple of 16 in 64..256. */
sim_status sim_get_schedule(const sim_handle *h, int32_t *sched);

/* Stream for all later device work of h (a hipStream_t; NULL = null stream).
 * The captured step graph is launched on this stream. */
sim_status sim_set_stream(sim_handle *h, void *hip_stream);

/* Enqueue n >= 0 steps on the handle's stream and return (asynchronous). */
sim_status sim_step(sim_handle *h, int32_t n);

/* Measurement form of sim_step: the n steps are launched kernel by kernel
 * (not from the captured graph), each kernel between a start and a stop HIP
 * event recorded on the handle's stream at the kernel's own start and end;
 * then the stream is synchronized.  kernel_ms[SIM_N_KERNELS] (may be NULL)
 * receives each kernel's summed duration over the n steps, total_ms (may be
 * NULL) the time from the first start to the last stop.  Results are
 * identical to sim_step. */
enum {
    SIM_K_TILE_STEP = 0,   /* lane changes, leaders, Eq. (1), integration */
    SIM_K_BIG_ADMIT,       /* the same for tiles above 384 vehicles, then intersection
                              admission: eligibility + priority claim */
    SIM_K_COMMIT,          /* transfers, arrivals, departures, travel times, new counts */
    SIM_K_SCATTER,         /* next sorted layout and look-ahead table */
    SIM_N_KERNELS
};
sim_status sim_step_timed(sim_handle *h, int32_t n, double *kernel_ms, double *total_ms);

/* Synchronize the stream and copy the state out (vehicle-id order). */
sim_status sim_read_state(sim_handle *h, sim_state *out);

/* Replace the dynamic state (resume from a state read earlier).  Every
 * non-NULL field is required except counters (kept if NULL).  The edge
 * travel-time sums are kept.  SIM_EINVAL if the state is inconsistent
 * (edge not at the cursor of the route, lane out of range, x outside
 * [0, length], overlapping vehicles in a lane). */
sim_status sim_write_state(sim_handle *h, const sim_state *in);

/* Per-edge sums of completed traversal times (s, FP64, accumulated each step
 * in ascending vehicle id) and traversal counts: [n_edges] each. */
sim_status sim_read_edge_stats(sim_handle *h, double *tt_sum, int64_t *tt_count);

/* Per-edge mean completed traversal time, the per-edge output that the
 * calibration compares with observations (Sec. IV-A) and whose gradient
 * sim_backward takes: sum / count computed on the device in FP64 (correctly
 * rounded), 0 where nothing completed a traversal.  mean_s: [n_edges]
 * (caller-owned, required); tt_count: [n_edges] or NULL.  Synchronizes the
 * stream.  Errors: SIM_EINVAL (null handle or mean_s), SIM_ENOMEM (the
 * handle's mean buffer, allocated at the first call), SIM_EDEVICE. */
sim_status sim_read_edge_means(sim_handle *h, double *mean_s, int64_t *tt_count);

/* Number of vehicles active at the start of the current step (synchronizes). */
sim_status sim_n_active(sim_handle *h, int32_t *out);

/* Release every device buffer of h.  NULL is a no-op. */
sim_status sim_destroy(sim_handle *h);

/* Message of the last failed call on h (or of the last failed sim_create when
 * h is NULL).  Valid until the next call on the same handle. */
/* Shortest routes on travel times (the routes of Sec. II-C, which the paper
 * computes once on CPUs, re-computed on the GPU from current per-edge costs,
 * e.g. the mean traversal times of sim_read_edge_stats).  edge_cost: [n_edges]
 * binary32 seconds, finite and > 0.  For each query q the route from node
 * origin[q] to node dest[q] minimises the cost summed, in binary32, from the
 * destination back (dist(d) = 0, dist(v) = min over out-edges e of
 * cost_e + dist(head e)) and leaves every node by the out-edge of smallest
 * (cost_e + dist(head e), edge id).  No move restrictions are applied: a
 * shortest route never turns back, so on networks whose moves exclude only
 * U-turns every route is a valid route for sim_create.
 * Output (host memory): route_off [n_queries + 1] and route_edges [capacity];
 * *n_route_edges is set to the total even when capacity is too small (then
 * SIM_EINVAL).  Up to 16,000 nodes the labels of a destination sit in one
 * workgroup's LDS; above, in device memory (4 bytes x nodes x distinct
 * destinations, at most 16 GB).  Errors: SIM_EINVAL (bad input, origin ==
 * destination, no route), SIM_EUNSUPPORTED (labels above 16 GB), SIM_ENOMEM,
 * SIM_EDEVICE.
 * Needs no handle; runs on the current device and synchronises it.  Its
 * device buffers come from the allocator of sim_set_allocator (hipMalloc
 * without one) and are returned before the call returns. */
sim_status sim_shortest_routes(const sim_network *net, const float *edge_cost, int32_t n_queries,
                               const int32_t *origin, const int32_t *dest, int64_t *route_off,
                               int32_t *route_edges, int64_t capacity, int64_t *n_route_edges);

/* The same routes for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, results and errors as sim_shortest_routes, but every device
 * buffer of the call (network copy, labels, queries, routes) is carved out of
 * one fixed 64 MiB region that the library holds on each device it runs on
 * until the process ends; no allocation is made.  A call that needs more
 * (roughly: 4 bytes x nodes x distinct destinations, plus the network, the
 * queries and 4 bytes per route edge) returns SIM_EINVAL and says so in
 * sim_last_error(NULL).  Calls on one device share the region: calls that
 * overlap in time on the same device (other host threads) race and must be
 * serialised by the caller. */
sim_status sim_shortest_routes_noalloc(const sim_network *net, const float *edge_cost, int32_t n_queries,
                                       const int32_t *origin, const int32_t *dest, int64_t *route_off,
                                       int32_t *route_edges, int64_t capacity, int64_t *n_route_edges);

const char *sim_last_error(const sim_handle *h);

/* Vehicle-updates done in tiles above one workgroup's LDS (inside
 * k_big_admit) since the handle's state was last written; the rest were done
 * by k_tile_step.  Synchronizes the handle's stream.  For measurement only. */
sim_status sim_big_tile_updates(sim_handle *h, int64_t *updates);

/* ------------------------------------------------------------------ diagnostics
 * Device-side evaluation of the arithmetic building blocks, for checking that
 * the GPU rounds exactly like IEEE-754 binary32 on the host.  op: 0 a/b,
 * 1 sqrt(a), 2 a*b, 3 a+b, 4 exp of Eq. (2)'s evaluator on a (a in (-17, 0]).
 * a, b, out: [n] host arrays. */
sim_status sim_probe_fp32(int32_t op, const float *a, const float *b, float *out, int64_t n);

/* Device Philox4x64-10 blocks: counters [n][4], key [2] -> out [n][4]. */
sim_status sim_probe_philox(const uint64_t *counters, const uint64_t *key, uint64_t *out, int64_t n);

/* Device lane-change draws: uniform (stream 1) and normal (streams 2, 3)
 * for n (t, id) pairs -> u [n], e2 [n], e3 [n]. */
sim_status sim_probe_draws(uint64_t seed, const int64_t *t, const int64_t *id, float *u, float *e2, float *e3,
                           int64_t n);

#ifdef __cplusplus
}
#endif
#endif /* MANTA_H */
