/*
 * CPU ORACLE for the per-timestep vehicle update of the MANTA traffic
 * microsimulation (Yedavalli, Kumar, Waddell, arXiv 2007.03614).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product imports, links or calls
 * this file; it is built and used by the test-suite, by the smoke check and by
 * the CPU-baseline leg of the benchmark.  It shares no code with the HIP path:
 * both are written separately from the same written step contract.
 *
 * It is deliberately plain: per-lane vehicle lists rebuilt by bucket + insertion
 * sort every phase, brute-force admission, one vehicle at a time in id order.
 * Phases 1 and 2 decide each vehicle from S_t alone and write only that
 * vehicle's entries, so built with OpenMP they run over vehicles in parallel;
 * their event counts are integer sums, so every thread count gives the same
 * result bit for bit.  Everything else runs in id order on one thread.
 *
 * Precision.  The paper fixes none.  Compiled with REAL=float (default) it is
 * the parity oracle: every FP32 operation in the order written below, no
 * contraction (-ffp-contract=off), so that discrete events can be compared
 * bit for bit.  Compiled with REAL=double it is the FP64 twin used to report
 * how far FP32 trajectories drift (same algorithm, same random integers).
 *
 * Paper passages followed (sections of the paper):
 *   Sec. II-D  time step dt = 0.5 s;
 *   Sec. II-D  lanes are 1-D rows where a vehicle finds its neighbours by
 *              lookup (the traffic atlas), at most one vehicle per place;
 *   Eq. (1)    Intelligent Driver Model acceleration; position and speed from
 *              integrating it twice;
 *   Table I and Sec. IV-A  parameter bounds and delta = 4;
 *   Eq. (2)    probability of a mandatory lane change, x0 = 1;
 *   Eqs. (3)-(4) critical lead and lag gaps with anticipation times
 *              alpha in [0.05, 0.40] and N(0,1) noise in metres;
 *   Sec. II-D (intersections, case 2)  all-green nodes, finite edge capacity.
 * Where the paper is silent, ambiguous or garbled, the reading taken is stated
 * in a comment at the place it is used (tags A1..A35 name the readings).
 *
 * Parity pins: see tests/test_oracle_*.py (closed forms of Eq. (1), the
 * platoon equilibrium gap, Eq. (2) frequencies, Philox against numpy,
 * exp against libm, brute-force leader and admission checks, invariants).
 * The crossing time inside a step (per-edge traversal times) is pinned by
 * exact cruise kinematics (each traversal lasts L/v0), by first-order
 * convergence to the closed-form free-road time from rest, and by a hold
 * released at the stop line (crossing at the step start).  Phase 2's kind
 * tree (VEH, FREE, STOP, LOOK with its partner from the start-of-step
 * table), the integration with its clamp and wrong-lane hold, and the
 * mandatory flag and wrong-lane wait are pinned by a plain re-derivation
 * from S_t; the 60-step patience by a hand-built deadlock at a junction.
 * Lane-change behaviour and the admission policy follow readings of the
 * paper, which prints no values for them; they are pinned by brute-force
 * re-derivations of those readings in plain Python (leaders, Phase-1
 * decisions, admission winners, case-1 round-robin), not by paper values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef REAL
#define REAL float
#endif
#define RL(c) ((REAL)(c))

#ifdef ORACLE_FP64
#define ORC_EXP(y) exp(y)
#else
#define ORC_EXP(y) orc_expf_c(y)
#endif

enum { WAITING = 0, ACTIVE = 1, ARRIVED = 2 };
enum { K_FREE = 0, K_VEH = 1, K_STOP = 2, K_LOOK = 3 };
enum {
    C_ACTIVE_SUM, C_DEPARTED, C_ARRIVED, C_LANE_CHANGES, C_TRANSFERS, C_HOLDS,
    C_INSERT_DENIED, C_MAND_TRIGGERS, C_STOP_BRANCH, C_CLAMP, C_WRONG_LANE_HOLDS,
    C_WAIVED_EXITS, C_GRIDLOCK, C_N
};
/* Gridlock detector (failure detection; the paper describes none): a step
 * stalls when vehicles were active at its start and none of them changed
 * position or lane, none crossed to another edge or arrived, and none
 * departed.  C_GRIDLOCK counts the steps that end a run of at least
 * GRIDLOCK_STEPS stalled steps (5 minutes at dt = 0.5 s). */
#define GRIDLOCK_STEPS 600
/* event flags of the last step (for brute-force tests) */
enum {
    EV_REQ = 1, EV_WIN = 2, EV_ARRIVE = 4, EV_WHOLD = 8, EV_CLAMP = 16, EV_STOPB = 32,
    EV_ELIG = 64, EV_INSERT_REQ = 128, EV_MOVED = 256, EV_MAND_TRIG = 512
};

#define PATIENCE 60          /* A19: wrong-lane hold waived after 60 held steps */
#define X0 1.0               /* Eq. (2): critical distance x0 = 1 (metres, A8) */
#define Z_CUT 17.0           /* exp(-17) < 5e-8: no trigger beyond this */
#define INCENTIVE 0.2        /* A9: discretionary incentive threshold, m/s^2 */
#define V_25MPH 11.176       /* Eqs. (3)-(4) text: 25 mph in m/s */
#define G_SLOW 3.0           /* A12: midpoint of 1-5 m below 25 mph */
#define G_FAST 7.5           /* A12: midpoint of 5-10 m above 25 mph */
#define S_MIN 0.1            /* A4: gap floor in the interaction term */

/* ------------------------------------------------------------------ random numbers
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11), counter-based: no state is carried between steps.
 * key = (seed, 0); counter = (t, vehicle id, stream, block).               */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ULL, c0, &hi0, &lo0);
        mulhilo64(0xCA5A826395121157ULL, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw_block(uint64_t seed, int64_t t, int64_t id, int s, int blk, uint64_t w[4]) {
    uint64_t c[4] = {(uint64_t)t, (uint64_t)id, (uint64_t)s, (uint64_t)blk};
    uint64_t k[2] = {seed, 0};
    orc_philox4x64(c, k, w);
}

/* U(t, id, s): top 24 bits of the first word, scaled to [0, 1). */
REAL orc_uniform(uint64_t seed, int64_t t, int64_t id, int s) {
    uint64_t w[4];
    draw_block(seed, t, id, s, 0, w);
    return (REAL)(w[0] >> 40) * RL(5.9604644775390625e-08); /* 2^-24, exact */
}

/* N(t, id, s): Irwin-Hall sum of twelve 24-bit uniforms, minus 6 (A14).
 * Integers: S = sum of (w >> 40) over blocks 0..2 (12 words); the value is
 * (S - 6*2^24) * 2^-24, converted once to REAL. */
REAL orc_normal(uint64_t seed, int64_t t, int64_t id, int s) {
    int64_t S = 0;
    for (int blk = 0; blk < 3; blk++) {
        uint64_t w[4];
        draw_block(seed, t, id, s, blk, w);
        for (int j = 0; j < 4; j++) S += (int64_t)(w[j] >> 40);
    }
    int32_t c = (int32_t)(S - 6 * 16777216LL);
    return (REAL)c * RL(5.9604644775390625e-08);
}

/* ------------------------------------------------------------------ per-driver v0 (Sec. IV)
 * Each driver's free-flow speed on an edge is drawn around the edge's limit
 * with standard deviation 2 sigma_s, sigma_s the spread of observed speeds at
 * that limit; here sigma_s = spread * limit (A28).  The draw is the
 * Irwin-Hall normal of stream 4 with the edge in place of the step, so it is
 * fixed for one driver on one edge, and the factor is floored at 0.1 (A29):
 *   limit_i,e = limit_e * max(1 + (2 spread) z, 0.1).                       */
REAL orc_driver_limit(uint64_t seed, int64_t edge, int64_t id, REAL lim, REAL spread) {
    if (spread == RL(0.0)) return lim;
    REAL f = RL(1.0) + (RL(2.0) * spread) * orc_normal(seed, edge, id, 4);
    if (f < RL(0.1)) f = RL(0.1);
    return lim * f;
}

/* ------------------------------------------------------------------ exp for Eq. (2)
 * exp(y) for y in (-17, 0], FP32, every operation in this order:
 * Cody-Waite reduction y = k ln2 + r with a two-part ln 2, a degree-7 Taylor
 * polynomial of e^r in Horner form, and an exact scaling by 2^k.          */
float orc_expf_c(float y) {
    const float log2e = 1.44269502162933349609375f;       /* nearest float to 1/ln2 */
    const float ln2_hi = 0.693145751953125f;               /* 0x3F317200, 16 bits */
    const float ln2_lo = 1.428606765330187045e-06f;        /* ln2 - ln2_hi, rounded */
    float kf = floorf(y * log2e + 0.5f);
    float r = (y - kf * ln2_hi) - kf * ln2_lo;
    float p = 1.0f / 5040.0f;
    p = p * r + 1.0f / 720.0f;
    p = p * r + 1.0f / 120.0f;
    p = p * r + 1.0f / 24.0f;
    p = p * r + 1.0f / 6.0f;
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    int k = (int)kf;
    union { uint32_t u; float f; } sc;
    sc.u = (uint32_t)(k + 127) << 23;   /* 2^k, normal for k >= -126 */
    return p * sc.f;
}

void orc_expf_c_batch(const float *in, float *out, int64_t n) {
    for (int64_t i = 0; i < n; i++) out[i] = orc_expf_c(in[i]);
}

/* ------------------------------------------------------------------ Eq. (1)
 * IDM acceleration, the order of operations fixed:
 *   r = v/v0, r4 = (r*r)*(r*r), phi = a(1 - r4), floored at -b  (A3)
 *   FREE: acc = phi
 *   else: s_star = s0 + max(0, vT + v(v - vl)/(2 sqrt(ab)))       (A1)
 *         acc = phi - a (s_star / max(s, 0.1))^2                  (A4)
 * den = 2 sqrt(ab) is per class.  flags: bit0 free term floored, bit1 dyn
 * term clipped at 0, bit2 gap floored. */
REAL orc_idm(REAL v, REAL v0, REAL vl, REAL s, REAL T, REAL a, REAL b, REAL s0, REAL den,
             int kind, int *flags) {
    int fl = 0;
    REAL r = v / v0;
    REAL r2 = r * r;
    REAL r4 = r2 * r2;
    REAL phi = a * (RL(1.0) - r4);
    if (phi < -b) { phi = -b; fl |= 1; }
    REAL acc;
    if (kind == K_FREE) {
        acc = phi;
    } else {
        REAL dv = v - vl;
        REAL dyn = (v * T) + ((v * dv) / den);
        if (dyn < RL(0.0)) { dyn = RL(0.0); fl |= 2; }
        REAL sst = s0 + dyn;
        REAL se = s;
        if (s < RL(S_MIN)) { se = RL(S_MIN); fl |= 4; }
        REAL q = sst / se;
        acc = phi - (a * (q * q));
    }
    if (flags) *flags = fl;
    return acc;
}

/* Eqs. (3)-(4): critical gap before the noise is added, the max taken first,
 * with g0 the desired gap at the merging vehicle's speed (A12).
 *   lead: max(g0, (g0 + alpha_a v_i) + alpha_i (v_i - v_a))
 *   lag:  max(g0, (g0 + alpha_i v_i) + alpha_b (v_i - v_b))              */
REAL orc_crit_gap(REAL g0, REAL alpha_first, REAL v_i, REAL alpha_second, REAL v_other) {
    REAL e = (g0 + alpha_first * v_i) + alpha_second * (v_i - v_other);
    return e > g0 ? e : g0;
}

REAL orc_desired_gap(REAL v_i) { return v_i < RL(V_25MPH) ? RL(G_SLOW) : RL(G_FAST); }

/* ------------------------------------------------------------------ simulation */
typedef struct {
    int *a;
    int n, cap;
} ivec;

static int iv_push(ivec *v, int x) {
    if (v->n == v->cap) {
        int nc = v->cap ? 2 * v->cap : 8;
        int *na = (int *)realloc(v->a, (size_t)nc * sizeof(int));
        if (!na) return -1;
        v->a = na;
        v->cap = nc;
    }
    v->a[v->n++] = x;
    return 0;
}

typedef struct orc_sim {
    /* network */
    int n_nodes, n_edges, n_lanes_total;
    int *efrom, *eto, *lanes, *lane_base;
    REAL *L, *lim;
    int *conn_off, *conn_to;
    uint8_t *conn_mask;
    /* vehicles (static) */
    int n;
    int64_t *roff;
    int *redges, *dep, *cls, *ins_lane;
    REAL *alpha;
    /* classes */
    int nc;
    REAL *v0f, *T, *a, *b, *s0, *len, *den;
    REAL dt;
    uint64_t seed;
    REAL spread;        /* per-driver v0 spread (0: every driver drives at v0f * limit) */
    /* dynamic state, indexed by vehicle id */
    int t;
    uint8_t *status;
    int *edge, *k, *lane, *mand, *held, *ww;
    REAL *x, *v;
    double *tau_in, *t_arr;
    int64_t cnt[C_N];
    int stall_run;      /* consecutive stalled steps (gridlock detector) */
    double *tt_sum;
    int64_t *tt_cnt;
    /* per-step scratch */
    ivec *lst;          /* per global lane: vehicle ids, front first */
    int *nlane;         /* post-LC lane */
    REAL *xn, *vn;      /* post-Phase-2 position and speed */
    int *tgt, *elig;    /* admission target lane (global) and eligibility */
    uint64_t *key;
    uint64_t *best;     /* per global lane: smallest eligible key */
    /* last-step events */
    int *ev_leader, *ev_kind, *ev_flags;
    int *ev_partner, *ev_bits;
    /* record of discrete decisions for the differentiable form (optional) */
    int recording;
    struct orc_drec *rec;
    int64_t n_rec, cap_rec;
    int64_t *rec_off;          /* [steps + 1]: records of step t */
    int *ins_step;             /* step at whose end a vehicle was admitted, -1 */
    int rec_t0;                /* first recorded step */
    /* case 1 intersections (flashing red; 0 = case 2, all green) */
    int imode;
    int stop_steps;            /* steps of the stop at the line: 2 s, rounded up */
    int *pair_base;            /* [edge]: its index among the in-edges of its head node x out-degree */
    int *out_idx;              /* [edge]: its index among the out-edges of its tail node */
    int *nm;                   /* [node]: in-degree x out-degree, the round-robin length */
    int *rr;                   /* [node]: pair served last, -1 before the first */
    uint64_t *bestnode;        /* [node]: smallest eligible transfer key of the step */
    int *tin;                  /* [lane]: a transfer enters it this step */
} orc_sim;

/* one active vehicle in one step, with every discrete decision frozen */
typedef struct orc_drec {
    int32_t vid;
    int32_t partner;           /* leader (VEH, clamp) or look-ahead rear (LOOK), -1 */
    int16_t kind;
    uint16_t bits;             /* RB_* */
} orc_drec;
enum { RB_F = 1, RB_D = 2, RB_S = 4, RB_B = 8, RB_C = 16, RB_W = 32, RB_EXIT = 64, RB_ARRIVE = 128,
       RB_HELD = 256 };

static int next_edge(const orc_sim *S, int i) {
    int64_t pos = S->roff[i] + S->k[i] + 1;
    return pos < S->roff[i + 1] ? S->redges[pos] : -1;
}

static int conn_mask_of(const orc_sim *S, int e, int f) {
    for (int c = S->conn_off[e]; c < S->conn_off[e + 1]; c++)
        if (S->conn_to[c] == f) return S->conn_mask[c];
    return 0;
}

/* lane l of e may proceed to f (any lane may, if e is the last route edge) */
static int allowed_lane(const orc_sim *S, int e, int f, int l) {
    if (f < 0) return 1;
    return (conn_mask_of(S, e, f) >> l) & 1;
}

static int lane_dist(const orc_sim *S, int e, int f, int l) {
    int m = conn_mask_of(S, e, f), best = 1 << 20;
    for (int q = 0; q < 8; q++)
        if ((m >> q) & 1) { int d = q > l ? q - l : l - q; if (d < best) best = d; }
    return best;
}

/* (x_j, id_j) > (x_i, id_i): j is ahead of i */
static int ahead(REAL xj, int j, REAL xi, int i) { return xj > xi || (xj == xi && j > i); }

/* rebuild every lane list from a lane assignment, front first */
static void build_lanes(orc_sim *S, const int *lane_of, const REAL *pos) {
    for (int g = 0; g < S->n_lanes_total; g++) S->lst[g].n = 0;
    for (int i = 0; i < S->n; i++) {
        if (S->status[i] != ACTIVE) continue;
        iv_push(&S->lst[S->lane_base[S->edge[i]] + lane_of[i]], i);
    }
    for (int g = 0; g < S->n_lanes_total; g++) {
        int *a = S->lst[g].a, n = S->lst[g].n;
        for (int p = 1; p < n; p++) {
            int cur = a[p], q = p - 1;
            while (q >= 0 && ahead(pos[cur], cur, pos[a[q]], a[q])) { a[q + 1] = a[q]; q--; }
            a[q + 1] = cur;
        }
    }
}

static void free_sim(orc_sim *S) {
    if (!S) return;
    void *ptrs[] = {S->efrom, S->eto, S->lanes, S->lane_base, S->L, S->lim, S->conn_off, S->conn_to,
                    S->conn_mask, S->roff, S->redges, S->dep, S->cls, S->ins_lane, S->alpha, S->v0f,
                    S->T, S->a, S->b, S->s0, S->len, S->den, S->status, S->edge, S->k, S->lane,
                    S->mand, S->held, S->ww, S->x, S->v, S->tau_in, S->t_arr, S->tt_sum, S->tt_cnt,
                    S->nlane, S->xn, S->vn, S->tgt, S->elig, S->key, S->best, S->ev_leader,
                    S->ev_kind, S->ev_flags, S->ev_partner, S->ev_bits, S->rec, S->rec_off, S->ins_step,
                    S->pair_base, S->out_idx, S->nm, S->rr, S->bestnode, S->tin};
    for (size_t q = 0; q < sizeof(ptrs) / sizeof(ptrs[0]); q++) free(ptrs[q]);
    if (S->lst) {
        for (int g = 0; g < S->n_lanes_total; g++) free(S->lst[g].a);
        free(S->lst);
    }
    free(S);
}

void orc_destroy(orc_sim *S) { free_sim(S); }

#define ALLOC(p, cnt) do { (p) = calloc((size_t)((cnt) > 0 ? (cnt) : 1), sizeof(*(p))); if (!(p)) { free_sim(S); return NULL; } } while (0)

/* The oracle trusts its inputs (the product validates); tests feed it only
 * generator output. */
orc_sim *orc_create(int32_t n_nodes, int32_t n_edges, const int32_t *edge_from, const int32_t *edge_to,
                    const float *length, const float *limit, const uint8_t *lanes,
                    const int32_t *conn_off, const int32_t *conn_to, const uint8_t *conn_mask,
                    int32_t n_veh, const int64_t *route_off, const int32_t *route_edges,
                    const int32_t *depart_step, const uint8_t *vclass, const float *alpha,
                    int32_t n_classes, const float *v0f, const float *T, const float *a,
                    const float *b, const float *s0, const float *vlen, float dt, uint64_t seed) {
    orc_sim *S = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!S) return NULL;
    S->n_nodes = n_nodes;
    S->n_edges = n_edges;
    ALLOC(S->efrom, n_edges); ALLOC(S->eto, n_edges); ALLOC(S->lanes, n_edges);
    ALLOC(S->lane_base, n_edges + 1); ALLOC(S->L, n_edges); ALLOC(S->lim, n_edges);
    ALLOC(S->conn_off, n_edges + 1);
    int n_conn = conn_off[n_edges];
    ALLOC(S->conn_to, n_conn); ALLOC(S->conn_mask, n_conn);
    for (int e = 0; e < n_edges; e++) {
        S->efrom[e] = edge_from[e]; S->eto[e] = edge_to[e]; S->lanes[e] = lanes[e];
        S->L[e] = (REAL)length[e]; S->lim[e] = (REAL)limit[e];
        S->lane_base[e + 1] = S->lane_base[e] + lanes[e];
    }
    S->n_lanes_total = S->lane_base[n_edges];
    for (int e = 0; e <= n_edges; e++) S->conn_off[e] = conn_off[e];
    for (int c = 0; c < n_conn; c++) { S->conn_to[c] = conn_to[c]; S->conn_mask[c] = conn_mask[c]; }
    S->n = n_veh;
    ALLOC(S->roff, n_veh + 1);
    int64_t n_re = route_off[n_veh];
    ALLOC(S->redges, n_re);
    for (int i = 0; i <= n_veh; i++) S->roff[i] = route_off[i];
    for (int64_t q = 0; q < n_re; q++) S->redges[q] = route_edges[q];
    ALLOC(S->dep, n_veh); ALLOC(S->cls, n_veh); ALLOC(S->alpha, n_veh); ALLOC(S->ins_lane, n_veh);
    S->nc = n_classes;
    ALLOC(S->v0f, n_classes); ALLOC(S->T, n_classes); ALLOC(S->a, n_classes); ALLOC(S->b, n_classes);
    ALLOC(S->s0, n_classes); ALLOC(S->len, n_classes); ALLOC(S->den, n_classes);
    for (int c = 0; c < n_classes; c++) {
        S->v0f[c] = (REAL)v0f[c]; S->T[c] = (REAL)T[c]; S->a[c] = (REAL)a[c];
        S->b[c] = (REAL)b[c]; S->s0[c] = (REAL)s0[c]; S->len[c] = (REAL)vlen[c];
#ifdef ORACLE_FP64
        S->den[c] = 2.0 * sqrt(S->a[c] * S->b[c]);
#else
        S->den[c] = 2.0f * sqrtf(S->a[c] * S->b[c]);
#endif
    }
    S->dt = (REAL)dt;
    S->seed = seed;
    ALLOC(S->status, n_veh); ALLOC(S->edge, n_veh); ALLOC(S->k, n_veh); ALLOC(S->lane, n_veh);
    ALLOC(S->mand, n_veh); ALLOC(S->held, n_veh); ALLOC(S->ww, n_veh); ALLOC(S->x, n_veh);
    ALLOC(S->v, n_veh); ALLOC(S->tau_in, n_veh); ALLOC(S->t_arr, n_veh);
    ALLOC(S->tt_sum, n_edges); ALLOC(S->tt_cnt, n_edges);
    ALLOC(S->nlane, n_veh); ALLOC(S->xn, n_veh); ALLOC(S->vn, n_veh); ALLOC(S->tgt, n_veh);
    ALLOC(S->elig, n_veh); ALLOC(S->key, n_veh); ALLOC(S->best, S->n_lanes_total);
    ALLOC(S->ev_leader, n_veh); ALLOC(S->ev_kind, n_veh); ALLOC(S->ev_flags, n_veh);
    ALLOC(S->ev_partner, n_veh); ALLOC(S->ev_bits, n_veh); ALLOC(S->ins_step, n_veh);
    for (int i = 0; i < n_veh; i++) S->ins_step[i] = -1;
    S->lst = (ivec *)calloc((size_t)(S->n_lanes_total > 0 ? S->n_lanes_total : 1), sizeof(ivec));
    if (!S->lst) { free_sim(S); return NULL; }
    for (int i = 0; i < n_veh; i++) {
        S->dep[i] = depart_step[i];
        S->cls[i] = vclass[i];
        S->alpha[i] = (REAL)alpha[i];
        S->status[i] = WAITING;
        S->edge[i] = route_edges[route_off[i]];
        S->k[i] = 0;
        S->held[i] = -1;
        S->tau_in[i] = -1.0;
        S->t_arr[i] = -1.0;
        /* A18: departures enter the lowest lane that may take the second route
         * edge (lane 0 for a one-edge route) */
        int e0 = route_edges[route_off[i]];
        int il = 0;
        if (route_off[i + 1] - route_off[i] > 1) {
            int m = conn_mask_of(S, e0, route_edges[route_off[i] + 1]);
            while (il < 7 && !((m >> il) & 1)) il++;
        }
        S->ins_lane[i] = il;
        S->lane[i] = il;
    }
    return S;
}

/* ------------------------------------------------------------------ one step
 * Four phases over the synchronous state S_t (every read below is of S_t
 * unless it says otherwise); S_{t+1} is written only in Phase 4.          */
static void step_once(orc_sim *S) {
    const int t = S->t;
    const int n = S->n;
    int n_active = 0;
    for (int i = 0; i < n; i++) {
        S->ev_leader[i] = -1; S->ev_kind[i] = -1; S->ev_flags[i] = 0;
        S->ev_partner[i] = -1; S->ev_bits[i] = 0;
        if (S->status[i] == ACTIVE) n_active++;
    }
    S->cnt[C_ACTIVE_SUM] += n_active;
    const int64_t c_moves0 = S->cnt[C_TRANSFERS] + S->cnt[C_ARRIVED] + S->cnt[C_DEPARTED];

    /* S_t lane lists (front first); M_t rear of a lane = its last entry */
    build_lanes(S, S->lane, S->x);

    /* ---- Phase 1: lane changes (Eqs. (2)-(4); A8-A15).  All changes in a
     * step go the same direction (A15), so checking both gaps >= 0 against the
     * S_t neighbours keeps the post-change lanes free of overlap. */
    const int dir = (t % 2 == 0) ? -1 : +1;
    int64_t n_mand = 0, n_lc = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : n_mand, n_lc)
    for (int i = 0; i < n; i++) {
        S->nlane[i] = S->lane[i];
        if (S->status[i] != ACTIVE || S->held[i] >= 0) continue;
        const int e = S->edge[i], l = S->lane[i], f = next_edge(S, i), c = S->cls[i];
        const int allowed_l = allowed_lane(S, e, f, l);
        /* Eq. (2): mandatory with probability exp(-(d - x0)^2), 1 within x0 */
        if (!allowed_l && !S->mand[i]) {
            REAL d = S->L[e] - S->x[i];
            if (d <= RL(X0)) {
                S->mand[i] = 1; n_mand++; S->ev_flags[i] |= EV_MAND_TRIG;
            } else {
                REAL dm = d - RL(X0);
                REAL z = dm * dm;
                if (z < RL(Z_CUT) && orc_uniform(S->seed, t, i, 1) < (REAL)ORC_EXP(-z)) {
                    S->mand[i] = 1; n_mand++; S->ev_flags[i] |= EV_MAND_TRIG;
                }
            }
        }
        const int lp = l + dir;
        if (lp < 0 || lp >= S->lanes[e]) continue;
        const int allowed_lp = allowed_lane(S, e, f, lp);
        /* S_t neighbours: same-lane leader, and lead a / lag b in lane lp */
        ivec *own = &S->lst[S->lane_base[e] + l];
        int lead_cur = -1;
        for (int p = 0; p < own->n; p++)
            if (own->a[p] == i) { if (p > 0) lead_cur = own->a[p - 1]; break; }
        ivec *tl = &S->lst[S->lane_base[e] + lp];
        int la = -1, lb = -1;
        for (int p = 0; p < tl->n; p++) {
            int j = tl->a[p];
            if (ahead(S->x[j], j, S->x[i], i)) la = j;
            else { lb = j; break; }
        }
        /* desire: route-motivated (towards the allowed lanes) or incentive */
        int desire = (!allowed_l) && (lane_dist(S, e, f, lp) < lane_dist(S, e, f, l));
        if (!desire && allowed_lp && !(S->mand[i] && !allowed_l)) {
            REAL v0 = S->v0f[c] * orc_driver_limit(S->seed, e, i, S->lim[e], S->spread);
            REAL acc_cur, acc_new;
            if (lead_cur >= 0) {
                REAL s = (S->x[lead_cur] - S->len[S->cls[lead_cur]]) - S->x[i];
                acc_cur = orc_idm(S->v[i], v0, S->v[lead_cur], s, S->T[c], S->a[c], S->b[c], S->s0[c],
                                  S->den[c], K_VEH, NULL);
            } else {
                acc_cur = orc_idm(S->v[i], v0, RL(0), RL(0), S->T[c], S->a[c], S->b[c], S->s0[c],
                                  S->den[c], K_FREE, NULL);
            }
            if (la >= 0) {
                REAL s = (S->x[la] - S->len[S->cls[la]]) - S->x[i];
                acc_new = orc_idm(S->v[i], v0, S->v[la], s, S->T[c], S->a[c], S->b[c], S->s0[c],
                                  S->den[c], K_VEH, NULL);
            } else {
                acc_new = orc_idm(S->v[i], v0, RL(0), RL(0), S->T[c], S->a[c], S->b[c], S->s0[c],
                                  S->den[c], K_FREE, NULL);
            }
            desire = (acc_new - acc_cur) > RL(INCENTIVE);
        }
        if (!desire) continue;
        /* Eqs. (3)-(4): gap acceptance with N(0,1) noise (A11-A14) */
        const REAL vi = S->v[i];
        const REAL g0 = orc_desired_gap(vi);
        int ok = 1;
        if (la >= 0) {
            REAL G = (S->x[la] - S->len[S->cls[la]]) - S->x[i];
            REAL g = orc_crit_gap(g0, S->alpha[la], vi, S->alpha[i], S->v[la]) + orc_normal(S->seed, t, i, 2);
            REAL need = g > RL(0) ? g : RL(0);
            ok = ok && (G >= need);
        }
        if (lb >= 0) {
            REAL G = (S->x[i] - S->len[c]) - S->x[lb];
            REAL g = orc_crit_gap(g0, S->alpha[i], vi, S->alpha[lb], S->v[lb]) + orc_normal(S->seed, t, i, 3);
            REAL need = g > RL(0) ? g : RL(0);
            ok = ok && (G >= need);
        }
        if (!ok) continue;
        S->nlane[i] = lp;
        S->ev_flags[i] |= EV_MOVED;
        n_lc++;
        if (allowed_lp) { S->mand[i] = 0; S->ww[i] = 0; }
    }
    S->cnt[C_MAND_TRIGGERS] += n_mand;
    S->cnt[C_LANE_CHANGES] += n_lc;

    /* M_t rears (pre-change lanes) are needed for look-ahead: keep them */
    int *mrear = (int *)malloc((size_t)(S->n_lanes_total > 0 ? S->n_lanes_total : 1) * sizeof(int));
    for (int g = 0; g < S->n_lanes_total; g++)
        mrear[g] = S->lst[g].n ? S->lst[g].a[S->lst[g].n - 1] : -1;

    /* ---- Phase 2: leader on the post-change lane, Eq. (1), integration */
    build_lanes(S, S->nlane, S->x);
    int64_t n_stopb = 0, n_clamp = 0, n_whold = 0, n_moved = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : n_stopb, n_clamp, n_whold, n_moved)
    for (int i = 0; i < n; i++) {
        if (S->status[i] != ACTIVE) continue;
        const int e = S->edge[i], l = S->nlane[i], f = next_edge(S, i), c = S->cls[i];
        const int allowed_l = allowed_lane(S, e, f, l);
        ivec *own = &S->lst[S->lane_base[e] + l];
        int j = -1;
        for (int p = 0; p < own->n; p++)
            if (own->a[p] == i) { if (p > 0) j = own->a[p - 1]; break; }
        int kind;
        REAL s = RL(0), vl = RL(0);
        if (j >= 0) {
            kind = K_VEH;
            s = (S->x[j] - S->len[S->cls[j]]) - S->x[i];
            vl = S->v[j];
        } else if (f < 0) {
            kind = K_FREE;
        } else if (S->mand[i] && !allowed_l && S->ww[i] < PATIENCE) {
            kind = K_STOP;                       /* A8: stop at the stop line */
            s = S->L[e] - S->x[i];
            vl = RL(0);
        } else {
            /* look ahead into (f, min(l, lanes_f - 1)) of M_t (A17) */
            int lam = l < S->lanes[f] - 1 ? l : S->lanes[f] - 1;
            int r = mrear[S->lane_base[f] + lam];
            if (r >= 0) {
                kind = K_LOOK;
                s = (S->L[e] - S->x[i]) + (S->x[r] - S->len[S->cls[r]]);
                vl = S->v[r];
            } else {
                kind = K_FREE;
            }
        }
        S->ev_leader[i] = j;
        S->ev_kind[i] = kind;
        S->ev_partner[i] = (kind == K_VEH) ? j : (kind == K_LOOK ? mrear[S->lane_base[f] + (S->nlane[i] < S->lanes[f] - 1 ? S->nlane[i] : S->lanes[f] - 1)] : -1);
        REAL v0 = S->v0f[c] * orc_driver_limit(S->seed, e, i, S->lim[e], S->spread);
        int idm_fl = 0;
        REAL acc = orc_idm(S->v[i], v0, vl, s, S->T[c], S->a[c], S->b[c], S->s0[c], S->den[c], kind, &idm_fl);
        S->ev_bits[i] = idm_fl;
        /* A5: ballistic update with an exact stop */
        const REAL dt = S->dt;
        REAL vnew = S->v[i] + (acc * dt);
        REAL xnew;
        if (vnew >= RL(0)) {
            xnew = (S->x[i] + (S->v[i] * dt)) + ((RL(0.5) * acc) * (dt * dt));
        } else {
            xnew = S->x[i] - ((S->v[i] * S->v[i]) / (RL(2.0) * acc));
            vnew = RL(0);
            n_stopb++;
            S->ev_flags[i] |= EV_STOPB;
            S->ev_bits[i] |= RB_B;
        }
        /* A7: never past the leader's S_t rear */
        if (kind == K_VEH) {
            REAL rear = S->x[j] - S->len[S->cls[j]];
            if (xnew > rear) { xnew = rear; n_clamp++; S->ev_flags[i] |= EV_CLAMP; S->ev_bits[i] |= RB_C; }
        }
        /* A8/A19: a wrong-lane vehicle waits at the stop line */
        if (f >= 0 && !allowed_l && S->ww[i] < PATIENCE && xnew >= S->L[e]) {
            xnew = S->L[e];
            vnew = RL(0);
            S->mand[i] = 1;
            S->ww[i] += 1;
            n_whold++;
            S->ev_flags[i] |= EV_WHOLD;
            S->ev_bits[i] |= RB_W;
        }
        S->xn[i] = xnew;
        S->vn[i] = vnew;
        if (xnew != S->x[i]) n_moved++;
    }
    S->cnt[C_STOP_BRANCH] += n_stopb;
    S->cnt[C_CLAMP] += n_clamp;
    S->cnt[C_WRONG_LANE_HOLDS] += n_whold;
    free(mrear);

    /* ---- Phase 3: end of edge and admission (case 2 intersections, A16-A18).
     * rear'(g, lam) = the active vehicle with the smallest (x_new, id) in the
     * post-change lane; it still counts if it is leaving itself. */
    for (int g = 0; g < S->n_lanes_total; g++) S->best[g] = UINT64_MAX;
    if (S->imode == 1)
        for (int v = 0; v < S->n_nodes; v++) S->bestnode[v] = UINT64_MAX;
    int *rearp = (int *)malloc((size_t)(S->n_lanes_total > 0 ? S->n_lanes_total : 1) * sizeof(int));
    for (int g = 0; g < S->n_lanes_total; g++) {
        int r = -1;
        for (int p = 0; p < S->lst[g].n; p++) {
            int q = S->lst[g].a[p];
            if (r < 0 || ahead(S->xn[r], r, S->xn[q], q)) r = q;
        }
        rearp[g] = r;
    }
    for (int i = 0; i < n; i++) {
        S->tgt[i] = -1;
        S->elig[i] = 0;
        if (S->status[i] == ACTIVE) {
            const int e = S->edge[i], f = next_edge(S, i);
            if (S->xn[i] >= S->L[e] && !(S->ev_flags[i] & EV_WHOLD)) {
                if (f < 0) {
                    S->ev_flags[i] |= EV_ARRIVE;
                } else {
                    int lam = S->nlane[i] < S->lanes[f] - 1 ? S->nlane[i] : S->lanes[f] - 1;
                    int g = S->lane_base[f] + lam;
                    REAL xp = S->xn[i] - S->L[e];
                    int r = rearp[g];
                    int ok = (r < 0) || ((S->xn[r] - S->len[S->cls[r]]) - xp >= RL(0));
                    uint64_t hs = (uint64_t)(S->held[i] >= 0 ? S->held[i] : t);
                    S->tgt[i] = g;
                    S->key[i] = (hs << 32) | (uint64_t)(uint32_t)i;
                    if (S->imode == 1) {
                        /* case 1: a vehicle crosses only after a 2 s stop at the line
                         * (held for ceil(2 s / dt) steps, A30); one crossing per node and step, the
                         * (in, out) pairs served round-robin after the last served one
                         * (A31): key = (distance in the cycle, held since, source lane) */
                        const int node = S->efrom[f];
                        const int pr = S->pair_base[e] + S->out_idx[f];
                        int dd = (pr - S->rr[node] - 1) % S->nm[node];
                        if (dd < 0) dd += S->nm[node];
                        ok = ok && S->held[i] >= 0 && t - S->held[i] >= S->stop_steps;
                        S->key[i] = ((uint64_t)dd << 58) | (hs << 26) | (uint64_t)(S->lane_base[e] + S->nlane[i]);
                        if (ok && S->key[i] < S->bestnode[node]) S->bestnode[node] = S->key[i];
                    }
                    S->elig[i] = ok;
                    S->ev_flags[i] |= EV_REQ | (ok ? EV_ELIG : 0);
                }
            }
        } else if (S->status[i] == WAITING && S->dep[i] <= t) {
            int g0e = S->redges[S->roff[i]];
            int g = S->lane_base[g0e] + S->ins_lane[i];
            int r = rearp[g];
            int ok = (r < 0) || ((S->xn[r] - S->len[S->cls[r]]) >= S->s0[S->cls[i]]);
            S->tgt[i] = g;
            S->elig[i] = ok;
            S->key[i] = (1ULL << 63) | ((uint64_t)(uint32_t)S->dep[i] << 32) | (uint64_t)(uint32_t)i;
            S->ev_flags[i] |= EV_INSERT_REQ | (ok ? EV_ELIG : 0);
        }
        /* transfers of case 1 are arbitrated per node above, not per lane */
        const int per_node = S->imode == 1 && S->status[i] == ACTIVE;
        if (!per_node && S->tgt[i] >= 0 && S->elig[i] && S->key[i] < S->best[S->tgt[i]]) S->best[S->tgt[i]] = S->key[i];
    }
    free(rearp);
    if (S->imode == 1) {
        /* the node winners: their lanes take no departure this step */
        for (int g = 0; g < S->n_lanes_total; g++) S->tin[g] = 0;
        for (int i = 0; i < n; i++)
            if (S->status[i] == ACTIVE && S->tgt[i] >= 0 && S->elig[i] &&
                S->bestnode[S->efrom[next_edge(S, i)]] == S->key[i])
                S->tin[S->tgt[i]] = 1;
    }

    /* ---- Phase 4: commit, in ascending vehicle id (this is also the order of
     * the per-edge travel-time sums, A22). */
    for (int i = 0; i < n; i++) {
        if (S->status[i] == ACTIVE) {
            const int e = S->edge[i];
            int won = S->tgt[i] >= 0 && S->elig[i] && S->best[S->tgt[i]] == S->key[i];
            if (S->imode == 1 && S->tgt[i] >= 0) {
                const int f = next_edge(S, i), node = S->efrom[f];
                won = S->elig[i] && S->bestnode[node] == S->key[i];
                if (won) S->rr[node] = S->pair_base[e] + S->out_idx[f];
            }
            if ((S->ev_flags[i] & EV_ARRIVE) || won) {
                /* crossing time interpolated inside the step */
                REAL phi = (S->xn[i] == S->x[i]) ? RL(0) : (S->L[e] - S->x[i]) / (S->xn[i] - S->x[i]);
                double tau = ((double)t + (double)phi) * (double)S->dt;
                S->tt_sum[e] += tau - S->tau_in[i];
                S->tt_cnt[e] += 1;
                if (S->ev_flags[i] & EV_ARRIVE) {
                    S->status[i] = ARRIVED;
                    S->t_arr[i] = tau;
                    S->x[i] = S->xn[i];
                    S->v[i] = S->vn[i];
                    S->lane[i] = S->nlane[i];
                    S->cnt[C_ARRIVED]++;
                } else {
                    const int f = next_edge(S, i);
                    if (!allowed_lane(S, e, f, S->nlane[i])) S->cnt[C_WAIVED_EXITS]++;
                    S->ev_flags[i] |= EV_WIN;
                    S->x[i] = S->xn[i] - S->L[e];
                    S->v[i] = S->vn[i];
                    S->edge[i] = f;
                    S->k[i] += 1;
                    S->lane[i] = S->tgt[i] - S->lane_base[f];
                    S->held[i] = -1;
                    S->mand[i] = 0;
                    S->ww[i] = 0;
                    S->tau_in[i] = tau;
                    S->cnt[C_TRANSFERS]++;
                }
            } else if (S->tgt[i] >= 0) {
                /* a losing transfer waits at the stop line */
                S->x[i] = S->L[e];
                S->v[i] = RL(0);
                S->lane[i] = S->nlane[i];
                if (S->held[i] < 0) S->held[i] = t;
                S->cnt[C_HOLDS]++;
            } else {
                S->x[i] = S->xn[i];
                S->v[i] = S->vn[i];
                S->lane[i] = S->nlane[i];
            }
        } else if (S->status[i] == WAITING && S->tgt[i] >= 0) {
            if (S->elig[i] && S->best[S->tgt[i]] == S->key[i] && !(S->imode == 1 && S->tin[S->tgt[i]])) {
                int e0 = S->redges[S->roff[i]];
                S->status[i] = ACTIVE;
                S->edge[i] = e0;
                S->k[i] = 0;
                S->lane[i] = S->tgt[i] - S->lane_base[e0];
                S->x[i] = RL(0);
                S->v[i] = RL(0);
                S->held[i] = -1;
                S->mand[i] = 0;
                S->ww[i] = 0;
                S->tau_in[i] = (double)(t + 1) * (double)S->dt;
                S->ev_flags[i] |= EV_WIN;
                S->cnt[C_DEPARTED]++;
            } else {
                S->cnt[C_INSERT_DENIED]++;
            }
        }
    }
    if (S->recording) {
        for (int i = 0; i < n; i++) {
            if (!(S->ev_kind[i] >= 0)) continue;     /* active at the start of the step */
            int bits = S->ev_bits[i];
            if (S->ev_flags[i] & EV_ARRIVE) bits |= RB_ARRIVE;
            else if ((S->ev_flags[i] & EV_REQ) && (S->ev_flags[i] & EV_WIN)) bits |= RB_EXIT;
            else if (S->ev_flags[i] & EV_REQ) bits |= RB_HELD;
            if (S->n_rec == S->cap_rec) {
                int64_t nc = S->cap_rec ? 2 * S->cap_rec : 4096;
                orc_drec *nr = (orc_drec *)realloc(S->rec, (size_t)nc * sizeof(orc_drec));
                if (!nr) { S->recording = 0; break; }
                S->rec = nr;
                S->cap_rec = nc;
            }
            orc_drec *r = &S->rec[S->n_rec++];
            r->vid = i;
            r->partner = S->ev_partner[i];
            r->kind = (int16_t)S->ev_kind[i];
            r->bits = (uint16_t)bits;
        }
        for (int i = 0; i < n; i++)
            if ((S->ev_flags[i] & EV_INSERT_REQ) && (S->ev_flags[i] & EV_WIN)) S->ins_step[i] = t;
        S->rec_off[t - S->rec_t0 + 1] = S->n_rec;
    }
    /* gridlock detector */
    const int moved = n_moved > 0 || n_lc > 0 ||
                      S->cnt[C_TRANSFERS] + S->cnt[C_ARRIVED] + S->cnt[C_DEPARTED] != c_moves0;
    S->stall_run = (n_active > 0 && !moved) ? S->stall_run + 1 : 0;
    if (S->stall_run >= GRIDLOCK_STEPS) S->cnt[C_GRIDLOCK]++;
    S->t = t + 1;
}

int orc_step(orc_sim *S, int32_t n_steps) {
    if (S->recording) {
        int64_t *no = (int64_t *)realloc(S->rec_off, (size_t)(S->t + n_steps - S->rec_t0 + 1) * sizeof(int64_t));
        if (!no) return -1;
        S->rec_off = no;
    }
    for (int q = 0; q < n_steps; q++) step_once(S);
    return 0;
}

/* ------------------------------------------------------------------ differentiable form
 * With every discrete decision of a recorded forward run held fixed (leader
 * or look-ahead partner, kind, IDM branches, stop, clamp, wrong-lane hold,
 * admissions, arrivals), the trajectory is a smooth function of the class
 * parameters theta = (v0_factor, T, a, b, s0) per class.  orc_replay
 * recomputes it in FP64 and returns the loss
 *     L = sum over used edges of (mean completed traversal time - target)^2
 * (Sec. IV-A calibrates the IDM parameters against per-edge observations;
 * here the observations are per-edge mean travel times).  With grad != NULL
 * it also runs the reverse sweep (the adjoint of Eq. (1) and of the
 * integration, the crossing-time interpolation and the leader coupling) and
 * writes dL/dtheta.  Central differences of orc_replay pin the adjoint. */
int32_t orc_enable_record(orc_sim *S) {
    if (S->t != 0) return -1;
    S->recording = 1;
    S->rec_t0 = 0;
    S->n_rec = 0;
    free(S->rec_off);
    S->rec_off = (int64_t *)calloc(1, sizeof(int64_t));
    return S->rec_off ? 0 : -1;
}

/* IDM in FP64 on frozen branches, with its partial derivatives
 * d[0..7] = d acc / d (v, vl, s, v0, T, a, b, s0) */
static double idm64(double v, double v0, double vl, double s, double T, double a, double b, double s0, int kind,
                    int bits, double d[8]) {
    for (int k = 0; k < 8; k++) d[k] = 0.0;
    const double r = v / v0;
    double phi;
    if (bits & RB_F) {
        phi = -b;
        d[6] = -1.0;
    } else {
        phi = a * (1.0 - r * r * r * r);
        d[0] = -4.0 * a * r * r * r / v0;
        d[3] = 4.0 * a * r * r * r * r / v0;
        d[5] = 1.0 - r * r * r * r;
    }
    if (kind == K_FREE) return phi;
    const double den = 2.0 * sqrt(a * b);
    double dyn = 0.0, ddyn_dv = 0.0, ddyn_dvl = 0.0, ddyn_dT = 0.0, ddyn_dden = 0.0;
    if (!(bits & RB_D)) {
        dyn = v * T + v * (v - vl) / den;
        ddyn_dv = T + (2.0 * v - vl) / den;
        ddyn_dvl = -v / den;
        ddyn_dT = v;
        ddyn_dden = -v * (v - vl) / (den * den);
    }
    const double sst = s0 + dyn;
    const double se = (bits & RB_S) ? S_MIN : s;
    const double q = sst / se;
    const double acc = phi - a * q * q;
    const double dsst = -2.0 * a * q / se;
    if (!(bits & RB_S)) d[2] = 2.0 * a * q * q / se;
    d[0] += dsst * ddyn_dv;
    d[1] = dsst * ddyn_dvl;
    d[4] = dsst * ddyn_dT;
    d[5] += -q * q + dsst * ddyn_dden * (den / (2.0 * a));
    d[6] += dsst * ddyn_dden * (den / (2.0 * b));
    d[7] = dsst;
    return acc;
}

double orc_replay(orc_sim *S, const double *theta, const double *target, const uint8_t *use, double *mean_out,
                  double *grad) {
    if (!S->recording || S->rec_t0 != 0) return NAN;
    const int n = S->n, E = S->n_edges, steps = S->t - S->rec_t0;
    const double dt = (double)S->dt;
    double *x = calloc((size_t)n + 1, sizeof(double)), *v = calloc((size_t)n + 1, sizeof(double));
    double *tin = calloc((size_t)n + 1, sizeof(double));
    int *cur = calloc((size_t)n + 1, sizeof(int));
    double *sum = calloc((size_t)E, sizeof(double));
    int64_t *cnt = calloc((size_t)E, sizeof(int64_t));
    const int64_t NR = S->n_rec;
    /* per record: x, v, xn, acc, partials[8], edge */
    double *tx = calloc((size_t)NR + 1, sizeof(double)), *tv = calloc((size_t)NR + 1, sizeof(double));
    double *txn = calloc((size_t)NR + 1, sizeof(double)), *tac = calloc((size_t)NR + 1, sizeof(double));
    double *tpd = grad ? calloc((size_t)(NR + 1) * 8, sizeof(double)) : NULL;
    int *ted = calloc((size_t)NR + 1, sizeof(int));
    double *vn = calloc((size_t)NR + 1, sizeof(double));
    if (!x || !v || !tin || !cur || !sum || !cnt || !tx || !tv || !txn || !tac || !ted || !vn || (grad && !tpd)) {
        free(x); free(v); free(tin); free(cur); free(sum); free(cnt); free(tx); free(tv); free(txn); free(tac);
        free(tpd); free(ted); free(vn);
        return NAN;
    }
    for (int t = 0; t < steps; t++) {
        const int64_t r0 = S->rec_off[t], r1 = S->rec_off[t + 1];
        for (int64_t k = r0; k < r1; k++) {          /* all reads of S_t */
            const orc_drec *R = &S->rec[k];
            const int i = R->vid, c = S->cls[i];
            const int e = S->redges[S->roff[i] + cur[i]];
            const double L = (double)S->L[e];
            double sgap = 0.0, vl = 0.0;
            const int j = R->partner;
            if (R->kind == K_VEH) { sgap = (x[j] - (double)S->len[S->cls[j]]) - x[i]; vl = v[j]; }
            else if (R->kind == K_STOP) { sgap = L - x[i]; }
            else if (R->kind == K_LOOK) { sgap = (L - x[i]) + (x[j] - (double)S->len[S->cls[j]]); vl = v[j]; }
            const double *th = theta + 5 * c;
            const double v0 = th[0] * (double)orc_driver_limit(S->seed, e, i, S->lim[e], S->spread);
            double pd[8];
            const double acc = idm64(v[i], v0, vl, sgap, th[1], th[2], th[3], th[4], R->kind, R->bits, pd);
            double xnew, vnew;
            if (R->bits & RB_B) { xnew = x[i] - v[i] * v[i] / (2.0 * acc); vnew = 0.0; }
            else { xnew = x[i] + v[i] * dt + 0.5 * acc * dt * dt; vnew = v[i] + acc * dt; }
            if (R->bits & RB_C) xnew = x[j] - (double)S->len[S->cls[j]];
            if (R->bits & RB_W) { xnew = L; vnew = 0.0; }
            tx[k] = x[i]; tv[k] = v[i]; txn[k] = xnew; tac[k] = acc; ted[k] = e; vn[k] = vnew;
            if (tpd) for (int q = 0; q < 8; q++) tpd[8 * k + q] = pd[q];
        }
        for (int64_t k = r0; k < r1; k++) {          /* commit */
            const orc_drec *R = &S->rec[k];
            const int i = R->vid, e = ted[k];
            const double L = (double)S->L[e];
            if (R->bits & (RB_EXIT | RB_ARRIVE)) {
                const double phi = (txn[k] == tx[k]) ? 0.0 : (L - tx[k]) / (txn[k] - tx[k]);
                const double tau = ((double)t + phi) * dt;
                sum[e] += tau - tin[i];
                cnt[e] += 1;
                tin[i] = tau;
                x[i] = txn[k] - L;
                v[i] = vn[k];
                cur[i] += 1;
            } else if (R->bits & RB_HELD) {
                x[i] = L;
                v[i] = 0.0;
            } else {
                x[i] = txn[k];
                v[i] = vn[k];
            }
        }
        for (int i = 0; i < n; i++)
            if (S->ins_step[i] == t) { x[i] = 0.0; v[i] = 0.0; cur[i] = 0; tin[i] = (double)(t + 1) * dt; }
    }
    double loss = 0.0;
    double *w = calloc((size_t)E, sizeof(double));
    for (int e = 0; e < E; e++) {
        const double m = cnt[e] ? sum[e] / (double)cnt[e] : 0.0;
        if (mean_out) mean_out[e] = m;
        if (cnt[e] && (!use || use[e])) {
            const double g = m - (target ? target[e] : 0.0);
            loss += g * g;
            if (w) w[e] = 2.0 * g / (double)cnt[e];
        }
    }
    if (grad && w) {
        for (int q = 0; q < 5 * S->nc; q++) grad[q] = 0.0;
        double *lx = calloc((size_t)n + 1, sizeof(double)), *lv = calloc((size_t)n + 1, sizeof(double));
        double *nx = calloc((size_t)n + 1, sizeof(double)), *nv = calloc((size_t)n + 1, sizeof(double));
        double *lt = calloc((size_t)n + 1, sizeof(double));
        int *cr = calloc((size_t)n + 1, sizeof(int));
        if (lx && lv && nx && nv && lt && cr) {
            for (int t = steps - 1; t >= 0; t--) {
                for (int i = 0; i < n; i++)
                    if (S->ins_step[i] == t) { lx[i] = 0.0; lv[i] = 0.0; lt[i] = 0.0; }
                for (int i = 0; i < n; i++) { nx[i] = 0.0; nv[i] = 0.0; }
                const int64_t r0 = S->rec_off[t], r1 = S->rec_off[t + 1];
                for (int64_t k = r0; k < r1; k++) {
                    const orc_drec *R = &S->rec[k];
                    const int i = R->vid, c = S->cls[i], e = ted[k], j = R->partner;
                    const double L = (double)S->L[e];
                    double mx = lx[i], mv = lv[i];
                    if (R->bits & (RB_HELD | RB_W)) { mx = 0.0; mv = 0.0; }
                    if (R->bits & RB_ARRIVE) { mx = 0.0; mv = 0.0; }
                    if (R->bits & (RB_EXIT | RB_ARRIVE)) {
                        const double gt = w[e] + lt[i];
                        if (txn[k] != tx[k]) {
                            const double dd = txn[k] - tx[k];
                            mx += gt * dt * (-(L - tx[k]) / (dd * dd));
                            nx[i] += gt * dt * ((L - txn[k]) / (dd * dd));
                        }
                        lt[i] = -w[e];
                    }
                    if (R->bits & (RB_HELD | RB_W)) continue;
                    double macc = 0.0;
                    if (R->bits & RB_C) {
                        nx[j] += mx;
                        mx = 0.0;
                    }
                    if (R->bits & RB_B) {
                        nx[i] += mx;
                        nv[i] += mx * (-tv[k] / tac[k]);
                        macc += mx * (tv[k] * tv[k] / (2.0 * tac[k] * tac[k]));
                    } else {
                        nx[i] += mx;
                        nv[i] += mx * dt + mv;
                        macc += mx * 0.5 * dt * dt + mv * dt;
                    }
                    const double *pd = tpd + 8 * k;
                    nv[i] += macc * pd[0];
                    if (R->kind == K_VEH) { nx[j] += macc * pd[2]; nx[i] -= macc * pd[2]; nv[j] += macc * pd[1]; }
                    else if (R->kind == K_STOP) { nx[i] -= macc * pd[2]; }
                    else if (R->kind == K_LOOK) { nx[i] -= macc * pd[2]; nx[j] += macc * pd[2]; nv[j] += macc * pd[1]; }
                    grad[5 * c + 0] += macc * pd[3] * (double)orc_driver_limit(S->seed, e, i, S->lim[e], S->spread);
                    grad[5 * c + 1] += macc * pd[4];
                    grad[5 * c + 2] += macc * pd[5];
                    grad[5 * c + 3] += macc * pd[6];
                    grad[5 * c + 4] += macc * pd[7];
                }
                for (int i = 0; i < n; i++) { lx[i] = nx[i]; lv[i] = nv[i]; }
            }
        } else {
            loss = NAN;
        }
        free(lx); free(lv); free(nx); free(nv); free(lt); free(cr);
    }
    free(w);
    free(x); free(v); free(tin); free(cur); free(sum); free(cnt); free(tx); free(tv); free(txn); free(tac);
    free(tpd); free(ted); free(vn);
    return loss;
}

int32_t orc_time(const orc_sim *S) { return S->t; }

/* state out, indexed by vehicle id (x, v widened to double exactly) */
void orc_read_state(const orc_sim *S, uint8_t *status, int32_t *edge, int32_t *lane, int32_t *cursor,
                    double *x, double *v, int32_t *held_since, uint8_t *mand, int32_t *ww,
                    double *tau_in, double *t_arr) {
    for (int i = 0; i < S->n; i++) {
        status[i] = S->status[i];
        edge[i] = S->edge[i];
        lane[i] = S->lane[i];
        cursor[i] = S->k[i];
        x[i] = (double)S->x[i];
        v[i] = (double)S->v[i];
        held_since[i] = S->held[i];
        mand[i] = (uint8_t)S->mand[i];
        ww[i] = S->ww[i];
        tau_in[i] = S->tau_in[i];
        t_arr[i] = S->t_arr[i];
    }
}

/* overwrite the dynamic state (test scenarios built by hand) */
void orc_write_state(orc_sim *S, int32_t t, const uint8_t *status, const int32_t *edge,
                     const int32_t *lane, const int32_t *cursor, const double *x, const double *v,
                     const int32_t *held_since, const uint8_t *mand, const int32_t *ww,
                     const double *tau_in, const double *t_arr) {
    S->t = t;
    for (int i = 0; i < S->n; i++) {
        S->status[i] = status[i];
        S->edge[i] = edge[i];
        S->lane[i] = lane[i];
        if (status[i] == WAITING) {   /* a waiting vehicle sits at its first route edge and entry lane (A18) */
            S->edge[i] = S->redges[S->roff[i]];
            S->lane[i] = S->ins_lane[i];
        }
        S->k[i] = cursor[i];
        S->x[i] = (REAL)x[i];
        S->v[i] = (REAL)v[i];
        S->held[i] = held_since[i];
        S->mand[i] = mand[i];
        S->ww[i] = ww[i];
        S->tau_in[i] = tau_in[i];
        if (t_arr) S->t_arr[i] = t_arr[i];
    }
    if (S->rr)
        for (int v = 0; v < S->n_nodes; v++) S->rr[v] = -1;   /* the round-robin restarts */
    S->stall_run = 0;                                         /* so does the gridlock detector */
}

void orc_counters(const orc_sim *S, int64_t *out) {
    for (int q = 0; q < C_N; q++) out[q] = S->cnt[q];
}

int32_t orc_n_counters(void) { return C_N; }

void orc_edge_stats(const orc_sim *S, double *tt_sum, int64_t *tt_cnt) {
    for (int e = 0; e < S->n_edges; e++) { tt_sum[e] = S->tt_sum[e]; tt_cnt[e] = S->tt_cnt[e]; }
}

/* events of the last step: Phase-2 leader id (-1 none), kind, flags, and the
 * post-Phase-2 position/speed before commit */
void orc_last_events(const orc_sim *S, int32_t *leader, int32_t *kind, int32_t *flags, int32_t *post_lane,
                     double *xnew, double *vnew, int32_t *target_lane) {
    for (int i = 0; i < S->n; i++) {
        leader[i] = S->ev_leader[i];
        kind[i] = S->ev_kind[i];
        flags[i] = S->ev_flags[i];
        post_lane[i] = S->nlane[i];
        xnew[i] = (double)S->xn[i];
        vnew[i] = (double)S->vn[i];
        target_lane[i] = S->tgt[i];
    }
}

/* Phase-2 partner of the last step: the same-lane leader (VEH) or the rear
 * of the look-ahead lane in the start-of-step table (LOOK), -1 otherwise */
void orc_last_partner(const orc_sim *S, int32_t *partner) {
    for (int i = 0; i < S->n; i++) partner[i] = S->ev_partner[i];
}

int32_t orc_real_bytes(void) { return (int32_t)sizeof(REAL); }

/* threads of the parallel phases (0: leave the OpenMP default); returns the
 * count in use, 1 in a build without OpenMP */
int32_t orc_set_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return (int32_t)omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Eq. (2) trigger test hook: does the draw at (t, id) fire at distance d? */
int32_t orc_mand_trigger(uint64_t seed, int64_t t, int64_t id, double d_in) {
    REAL d = (REAL)d_in;
    if (d <= RL(X0)) return 1;
    REAL dm = d - RL(X0);
    REAL z = dm * dm;
    return (z < RL(Z_CUT) && orc_uniform(seed, t, id, 1) < (REAL)ORC_EXP(-z)) ? 1 : 0;
}

/* scalar wrappers with double arguments, for the tests' ctypes layer */
double orc_idm_d(double v, double v0, double vl, double s, double T, double a, double b, double s0,
                 int32_t kind, int32_t *flags) {
    REAL A = (REAL)a, B = (REAL)b;
#ifdef ORACLE_FP64
    REAL den = 2.0 * sqrt(A * B);
#else
    REAL den = 2.0f * sqrtf(A * B);
#endif
    return (double)orc_idm((REAL)v, (REAL)v0, (REAL)vl, (REAL)s, (REAL)T, A, B, (REAL)s0, den, kind, flags);
}

double orc_crit_gap_d(double g0, double af, double vi, double as, double vo) {
    return (double)orc_crit_gap((REAL)g0, (REAL)af, (REAL)vi, (REAL)as, (REAL)vo);
}

double orc_desired_gap_d(double vi) { return (double)orc_desired_gap((REAL)vi); }
double orc_uniform_d(uint64_t seed, int64_t t, int64_t id, int32_t s) { return (double)orc_uniform(seed, t, id, s); }
double orc_normal_d(uint64_t seed, int64_t t, int64_t id, int32_t s) { return (double)orc_normal(seed, t, id, s); }
void orc_set_v0_spread(orc_sim *S, float spread) { S->spread = (REAL)spread; }
double orc_driver_limit_d(uint64_t seed, int64_t edge, int64_t id, float lim, float spread) {
    return (double)orc_driver_limit(seed, edge, id, (REAL)lim, (REAL)spread);
}

/* Case 1 intersections (flashing red).  The (in, out) pairs of a node are
 * numbered in-edge major, both in edge-id order.  Returns -1 if a node has
 * more than 64 pairs or memory runs out. */
int32_t orc_set_intersection_mode(orc_sim *S, int32_t mode) {
    S->imode = mode;
    if (mode != 1) return 0;
    S->stop_steps = (int)ceil(2.0 / (double)S->dt - 1e-6);
    const int E = S->n_edges, V = S->n_nodes;
    int *indeg = calloc((size_t)V + 1, sizeof(int)), *outdeg = calloc((size_t)V + 1, sizeof(int));
    S->pair_base = calloc((size_t)E + 1, sizeof(int));
    S->out_idx = calloc((size_t)E + 1, sizeof(int));
    S->nm = calloc((size_t)V + 1, sizeof(int));
    S->rr = calloc((size_t)V + 1, sizeof(int));
    S->bestnode = calloc((size_t)V + 1, sizeof(uint64_t));
    S->tin = calloc((size_t)S->n_lanes_total + 1, sizeof(int));
    if (!indeg || !outdeg || !S->pair_base || !S->out_idx || !S->nm || !S->rr || !S->bestnode || !S->tin) {
        free(indeg); free(outdeg);
        return -1;
    }
    int *in_idx = calloc((size_t)E + 1, sizeof(int));
    if (!in_idx) { free(indeg); free(outdeg); return -1; }
    for (int e = 0; e < E; e++) {                 /* edge-id order within each node */
        in_idx[e] = indeg[S->eto[e]]++;
        S->out_idx[e] = outdeg[S->efrom[e]]++;
    }
    int rc = 0;
    for (int v = 0; v < V; v++) {
        S->nm[v] = indeg[v] * outdeg[v];
        if (S->nm[v] > 64) rc = -1;
        S->rr[v] = -1;
    }
    for (int e = 0; e < E; e++) S->pair_base[e] = in_idx[e] * outdeg[S->eto[e]];
    free(in_idx); free(indeg); free(outdeg);
    return rc;
}

/* ------------------------------------------------------------------ routes on travel times
 * Shortest routes (Sec. II-C, re-computed on current edge costs) in binary32:
 * dist_d(v) = min over out-edges e = (v -> u) of fl(cost_e + dist_d(u)),
 * dist_d(d) = 0, by Dijkstra from d over the reversed edges (plain O(V^2)
 * selection of the smallest label, ties to the lower node id).  The route
 * from o leaves every node by the out-edge of smallest (fl(cost_e + dist(head
 * e)), edge id) until it reaches d.  Returns the number of edges written, or
 * -1 (o == d, d unreachable, or more than cap edges). */
int32_t orc_route(int32_t n_nodes, int32_t n_edges, const int32_t *edge_from, const int32_t *edge_to,
                  const float *cost, int32_t o, int32_t d, int32_t *out, int32_t cap) {
    if (o == d) return -1;
    float *dist = malloc(sizeof(float) * (size_t)n_nodes);
    uint8_t *done = calloc((size_t)n_nodes, 1);
    if (!dist || !done) { free(dist); free(done); return -1; }
    for (int v = 0; v < n_nodes; v++) dist[v] = INFINITY;
    dist[d] = 0.0f;
    for (int it = 0; it < n_nodes; it++) {
        int best = -1;
        for (int v = 0; v < n_nodes; v++)
            if (!done[v] && dist[v] < INFINITY && (best < 0 || dist[v] < dist[best])) best = v;
        if (best < 0) break;
        done[best] = 1;
        for (int e = 0; e < n_edges; e++)          /* edges into best */
            if (edge_to[e] == best && !done[edge_from[e]]) {
                const float c = cost[e] + dist[best];
                if (c < dist[edge_from[e]]) dist[edge_from[e]] = c;
            }
    }
    int n = -1;
    if (dist[o] < INFINITY) {
        n = 0;
        int v = o;
        while (v != d) {
            int be = -1;
            float bc = INFINITY;
            for (int e = 0; e < n_edges; e++)
                if (edge_from[e] == v) {
                    const float c = cost[e] + dist[edge_to[e]];
                    if (be < 0 || c < bc) { be = e; bc = c; }   /* edges scanned in id order: ties to the lower id */
                }
            if (be < 0 || n >= cap) { n = -1; break; }
            out[n++] = be;
            v = edge_to[be];
        }
    }
    free(dist); free(done);
    return n;
}

/* dist_d(v) of the above for every node (pins) */
void orc_route_dist(int32_t n_nodes, int32_t n_edges, const int32_t *edge_from, const int32_t *edge_to,
                    const float *cost, int32_t d, float *dist) {
    uint8_t *done = calloc((size_t)n_nodes, 1);
    if (!done) return;
    for (int v = 0; v < n_nodes; v++) dist[v] = INFINITY;
    dist[d] = 0.0f;
    for (int it = 0; it < n_nodes; it++) {
        int best = -1;
        for (int v = 0; v < n_nodes; v++)
            if (!done[v] && dist[v] < INFINITY && (best < 0 || dist[v] < dist[best])) best = v;
        if (best < 0) break;
        done[best] = 1;
        for (int e = 0; e < n_edges; e++)
            if (edge_to[e] == best && !done[edge_from[e]]) {
                const float c = cost[e] + dist[best];
                if (c < dist[edge_from[e]]) dist[edge_from[e]] = c;
            }
    }
    free(done);
}
