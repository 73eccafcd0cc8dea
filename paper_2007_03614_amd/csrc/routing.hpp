// Routes on travel times (the fixed routes of Sec. II-C, re-computed on the
// GPU from current per-edge costs, e.g. the mean traversal times of the step
// statistics).  Binary32 costs; for a destination d
//   dist(d) = 0,  dist(v) = min over out-edges e = (v -> u) of fl(cost_e + dist(u)),
// and a route leaves every node by the out-edge of smallest
// (fl(cost_e + dist(head e)), edge id).  Any order of relaxation reaches the
// same least fixed point as Dijkstra from d when every cost is positive, so
// the result does not depend on the schedule of the sweeps.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace manta {

constexpr int kRouteNT = 1024;
constexpr int kRouteMaxNodes = 16000;   // one binary32 label per node, within 64 KiB of LDS

// One workgroup per destination: labels in LDS, Bellman-Ford sweeps in
// place until one changes nothing (at most V sweeps).  Out-edges of node v
// are out_edge[out_off[v] .. out_off[v + 1]).
__global__ void __launch_bounds__(kRouteNT) k_route_dist(int V, const int* out_off, const int* out_edge,
                                                        const int* edge_to, const float* cost, const int* dests,
                                                        int nd, float* dist_out) {
    __shared__ float dist[kRouteMaxNodes];
    __shared__ int changed;
    for (int q = blockIdx.x; q < nd; q += gridDim.x) {
        const int d = dests[q];
        for (int v = threadIdx.x; v < V; v += kRouteNT) dist[v] = v == d ? 0.0f : INFINITY;
        __syncthreads();
        for (int it = 0; it < V; ++it) {
            if (threadIdx.x == 0) changed = 0;
            __syncthreads();
            bool ch = false;
            for (int v = threadIdx.x; v < V; v += kRouteNT) {
                float best = dist[v];
                for (int k = out_off[v]; k < out_off[v + 1]; ++k) {
                    const int e = out_edge[k];
                    const float c = cost[e] + dist[edge_to[e]];
                    if (c < best) best = c;
                }
                if (best < dist[v]) {
                    dist[v] = best;
                    ch = true;
                }
            }
            if (ch) changed = 1;
            __syncthreads();
            const bool more = changed != 0;
            __syncthreads();   // every thread has read the flag before it is reset
            if (!more) break;
        }
        for (int v = threadIdx.x; v < V; v += kRouteNT) dist_out[(size_t)q * V + v] = dist[v];
        __syncthreads();
    }
}

// The same sweeps over a padded adjacency: slot j of node v holds its j-th
// out-edge's head and cost at [j * V + v] (unused slots: head v, cost +inf,
// which never improves a label).  A node's KM loads are independent of each
// other and of the labels, so they are in flight together, and neighbouring
// threads read neighbouring words; the CSR form above chains out_off ->
// out_edge -> edge_to for every edge.  Same labels: each is the minimum of
// the same fl(cost + dist(head)) values, in any order.
template <int KM>
__global__ void __launch_bounds__(kRouteNT) k_route_dist_padded(int V, const int* __restrict__ adj_to,
                                                               const float* __restrict__ adj_cost,
                                                               const int* __restrict__ dests, int nd,
                                                               float* __restrict__ dist_out) {
    __shared__ float dist[kRouteMaxNodes];
    __shared__ int changed;
    for (int q = blockIdx.x; q < nd; q += gridDim.x) {
        const int d = dests[q];
        for (int v = threadIdx.x; v < V; v += kRouteNT) dist[v] = v == d ? 0.0f : INFINITY;
        __syncthreads();
        for (int it = 0; it < V; ++it) {
            if (threadIdx.x == 0) changed = 0;
            __syncthreads();
            bool ch = false;
            for (int v = threadIdx.x; v < V; v += kRouteNT) {
                int to[KM];
                float c[KM];
#pragma unroll
                for (int j = 0; j < KM; ++j) {
                    to[j] = adj_to[(size_t)j * V + v];
                    c[j] = adj_cost[(size_t)j * V + v];
                }
                float best = dist[v];
#pragma unroll
                for (int j = 0; j < KM; ++j) {
                    const float cj = c[j] + dist[to[j]];
                    if (cj < best) best = cj;
                }
                if (best < dist[v]) {
                    dist[v] = best;
                    ch = true;
                }
            }
            if (ch) changed = 1;
            __syncthreads();
            const bool more = changed != 0;
            __syncthreads();   // every thread has read the flag before it is reset
            if (!more) break;
        }
        for (int v = threadIdx.x; v < V; v += kRouteNT) dist_out[(size_t)q * V + v] = dist[v];
        __syncthreads();
    }
}

// The padded sweeps with the adjacency held in registers: thread x owns
// nodes x + i * kRouteNT (i < NPT) and loads their KM (head, cost) slots once
// per workgroup, before its first destination; a sweep then touches only
// the labels in LDS.  For networks of at most NPT * kRouteNT nodes.
template <int KM, int NPT>
__global__ void __launch_bounds__(kRouteNT) k_route_dist_regs(int V, const int* __restrict__ adj_to,
                                                             const float* __restrict__ adj_cost,
                                                             const int* __restrict__ dests, int nd,
                                                             float* __restrict__ dist_out) {
    __shared__ float dist[kRouteMaxNodes];
    __shared__ int changed;
    int to[NPT][KM];
    float c[NPT][KM];
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int v = (int)threadIdx.x + i * kRouteNT;
#pragma unroll
        for (int j = 0; j < KM; ++j) {
            to[i][j] = v < V ? adj_to[(size_t)j * V + v] : 0;
            c[i][j] = v < V ? adj_cost[(size_t)j * V + v] : INFINITY;
        }
    }
    for (int q = blockIdx.x; q < nd; q += gridDim.x) {
        const int d = dests[q];
        for (int v = threadIdx.x; v < V; v += kRouteNT) dist[v] = v == d ? 0.0f : INFINITY;
        __syncthreads();
        for (int it = 0; it < V; ++it) {
            if (threadIdx.x == 0) changed = 0;
            __syncthreads();
            bool ch = false;
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                const int v = (int)threadIdx.x + i * kRouteNT;
                if (v < V) {
                    float best = dist[v];
#pragma unroll
                    for (int j = 0; j < KM; ++j) {
                        const float cj = c[i][j] + dist[to[i][j]];
                        if (cj < best) best = cj;
                    }
                    if (best < dist[v]) {
                        dist[v] = best;
                        ch = true;
                    }
                }
            }
            if (ch) changed = 1;
            __syncthreads();
            const bool more = changed != 0;
            __syncthreads();   // every thread has read the flag before it is reset
            if (!more) break;
        }
        for (int v = threadIdx.x; v < V; v += kRouteNT) dist_out[(size_t)q * V + v] = dist[v];
        __syncthreads();
    }
}

// Networks above kRouteMaxNodes: one workgroup per destination with its
// labels in global memory (row q of dist_out), relaxed from a frontier -- the
// nodes whose label dropped in the last round push the drop to the tails of
// their in-edges (a label-correcting search; with positive costs it ends at
// the same binary32 fixed point as any other relaxation order, see above).
// A node enters the next frontier once per round (mark holds the round of
// its last push).  Labels are positive floats, so their bit patterns order
// like the values and atomicMin on the integer view takes the minimum.
// Labels, marks and frontier entries are read and written only by atomics
// at device scope (performed in L2, never served stale from a CU's L1), and
// every thread waits for its memory operations before each barrier.
// Per workgroup: frontier space 2 * V and marks V (fq, mk at blockIdx * V).
__device__ inline int ld_l2(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_l2(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void settle_and_sync() {
    __builtin_amdgcn_s_waitcnt(0);   // this thread's loads, stores and atomics are done
    __syncthreads();
}

__global__ void __launch_bounds__(kRouteNT) k_route_dist_global(int V, const int* in_off, const int* in_edge,
                                                               const int* edge_from, const float* cost,
                                                               const int* dests, int nd, float* dist_out, int* fq,
                                                               int* mk) {
    __shared__ int n_next;
    int* fa = fq + (size_t)blockIdx.x * 2 * V;
    int* fb = fa + V;
    int* mark = mk + (size_t)blockIdx.x * V;
    for (int q = blockIdx.x; q < nd; q += gridDim.x) {
        const int d = dests[q];
        int* idist = (int*)(dist_out + (size_t)q * V);
        for (int v = threadIdx.x; v < V; v += kRouteNT) {
            st_l2(&idist[v], __float_as_int(v == d ? 0.0f : INFINITY));
            st_l2(&mark[v], -1);
        }
        if (threadIdx.x == 0) {
            st_l2(&fa[0], d);
            n_next = 0;
        }
        settle_and_sync();
        int n_cur = 1;
        int* cur = fa;
        int* nxt = fb;
        for (int round = 0; n_cur > 0; ++round) {
            for (int i = threadIdx.x; i < n_cur; i += kRouteNT) {
                const int u = ld_l2(&cur[i]);
                const float du = __int_as_float(ld_l2(&idist[u]));
                for (int k = in_off[u]; k < in_off[u + 1]; ++k) {
                    const int e = in_edge[k];
                    const int v = edge_from[e];
                    const float c = cost[e] + du;
                    const int old = atomicMin(&idist[v], __float_as_int(c));
                    if (c < __int_as_float(old) && atomicExch(&mark[v], round) != round)
                        st_l2(&nxt[atomicAdd(&n_next, 1)], v);
                }
            }
            settle_and_sync();
            n_cur = n_next;
            __syncthreads();   // every thread has read the count before it is reset
            if (threadIdx.x == 0) n_next = 0;
            int* t = cur;
            cur = nxt;
            nxt = t;
        }
        __syncthreads();
    }
}

// One thread per query: walk from the origin to the destination over the
// labels of its destination (slot).  fill == 0: write the number of edges to
// len[q] (-1: origin == destination, unreachable, or longer than V edges);
// fill == 1: write the edges at route_edges[off[q] ...].
__global__ void __launch_bounds__(256) k_route_walk(int V, const int* out_off, const int* out_edge,
                                                   const int* edge_to, const float* cost, const float* dist_all,
                                                   const int* slot, const int* origin, const int* dest, int nq,
                                                   int fill, int* len, const int64_t* off, int* route_edges) {
    for (int q = blockIdx.x * 256 + threadIdx.x; q < nq; q += gridDim.x * 256) {
        const float* dist = dist_all + (size_t)slot[q] * V;
        const int o = origin[q], d = dest[q];
        int n = 0;
        bool ok = o != d && dist[o] < INFINITY;
        int v = o;
        while (ok && v != d) {
            int be = -1;
            float bc = INFINITY;
            for (int k = out_off[v]; k < out_off[v + 1]; ++k) {   // ascending edge id within a node
                const int e = out_edge[k];
                const float c = cost[e] + dist[edge_to[e]];
                if (be < 0 || c < bc) {
                    be = e;
                    bc = c;
                }
            }
            if (be < 0 || n >= V) {
                ok = false;
                break;
            }
            if (fill) route_edges[off[q] + n] = be;
            ++n;
            v = edge_to[be];
        }
        if (!fill) len[q] = ok ? n : -1;
    }
}

}  // namespace manta
