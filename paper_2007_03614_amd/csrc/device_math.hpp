// Device arithmetic of the per-timestep vehicle update (gfx950).
//
// Everything here is FP32 with contraction off (the build passes
// -ffp-contract=off) and IEEE-correct division, so each expression rounds
// exactly as binary32 on any conforming host; the operation order is part of
// the step contract and must not be rearranged.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace manta {

// ---- step contract constants --------------------------------------------
constexpr int kPatience = 60;            // wrong-lane hold waived after 60 held steps
constexpr float kX0 = 1.0f;              // Eq. (2): critical distance x0 = 1 m
constexpr float kZCut = 17.0f;           // exp(-17) < 5e-8: no Eq. (2) draw beyond this
constexpr float kIncentive = 0.2f;       // discretionary lane-change threshold, m/s^2
constexpr float kV25mph = 11.176f;       // Eqs. (3)-(4): desired gap switches at 25 mph
constexpr float kGSlow = 3.0f;           // desired gap below 25 mph (middle of 1-5 m)
constexpr float kGFast = 7.5f;           // desired gap above 25 mph (middle of 5-10 m)
constexpr float kSMin = 0.1f;            // gap floor in the IDM interaction term

enum Kind : int { kFree = 0, kVeh = 1, kStop = 2, kLook = 3 };

// ---- Philox4x64-10 (Salmon et al., SC'11) -------------------------------
// Counter-based: a draw is a pure function of (key, counter), so every
// vehicle can draw independently with no generator state in memory.
struct U64x4 {
    uint64_t w[4];
};

__host__ __device__ inline void mul_hilo(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
#if defined(__HIP_DEVICE_COMPILE__)
    hi = __umul64hi(a, b);
    lo = a * b;
#else
    unsigned __int128 p = (unsigned __int128)a * b;
    hi = (uint64_t)(p >> 64);
    lo = (uint64_t)p;
#endif
}

__host__ __device__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                 uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t h0, l0, h1, l1;
        mul_hilo(M0, c0, h0, l0);
        mul_hilo(M1, c2, h1, l1);
        const uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0;
        c1 = l1;
        c2 = n2;
        c3 = l0;
        k0 += W0;
        k1 += W1;
    }
    return U64x4{{c0, c1, c2, c3}};
}

// counter = (step, vehicle id, stream, block); key = (seed, 0)
__device__ inline float draw_uniform(uint64_t seed, int t, uint32_t vid, int stream) {
    U64x4 r = philox4x64_10((uint64_t)(int64_t)t, vid, (uint64_t)stream, 0, seed, 0);
    return (float)(uint32_t)(r.w[0] >> 40) * 5.9604644775390625e-08f;   // * 2^-24, exact
}

// Irwin-Hall(12) - 6 on 24-bit grids: 12 words from blocks 0..2, integer sum,
// one rounding to binary32 at the end.
__device__ inline float draw_normal(uint64_t seed, int t, uint32_t vid, int stream) {
    int64_t s = 0;
#pragma unroll
    for (int blk = 0; blk < 3; ++blk) {
        U64x4 r = philox4x64_10((uint64_t)(int64_t)t, vid, (uint64_t)stream, (uint64_t)blk, seed, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) s += (int64_t)(r.w[j] >> 40);
    }
    const int32_t c = (int32_t)(s - 6ll * 16777216ll);
    return (float)c * 5.9604644775390625e-08f;
}

// A driver's free-flow limit on an edge (Sec. IV, model validation): the
// edge's limit times max(1 + 2 spread z, 0.1), z the Irwin-Hall normal of
// stream 4 with the edge (modulo period: one scenario's edges in an
// ensemble) in place of the step, so it is fixed for one driver on one edge.
// spread = 0 returns the limit itself.
__device__ inline float driver_limit(float lim, float spread, uint64_t seed, int edge, int period, uint32_t rid) {
    if (spread == 0.0f) return lim;
    float f = 1.0f + (2.0f * spread) * draw_normal(seed, edge % period, rid, 4);
    f = f < 0.1f ? 0.1f : f;
    return lim * f;
}

// exp(y) for y in (-17, 0] (Eq. (2)): Cody-Waite split y = k ln2 + r with
// ln2 = 0x3F317200 + 1.4286068e-6, degree-7 Taylor polynomial of e^r by
// Horner, then multiplication by 2^k built from its exponent bits (exact).
__device__ inline float exp_eq2(float y) {
    const float kf = floorf(y * 1.44269502162933349609375f + 0.5f);
    const float r = (y - kf * 0.693145751953125f) - kf * 1.428606765330187045e-06f;
    float p = 1.0f / 5040.0f;
    p = p * r + 1.0f / 720.0f;
    p = p * r + 1.0f / 120.0f;
    p = p * r + 1.0f / 24.0f;
    p = p * r + 1.0f / 6.0f;
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    const int k = (int)kf;
    return p * __int_as_float((k + 127) << 23);
}

// ---- Eq. (1): IDM with delta = 4 ----------------------------------------
// phi = a (1 - (v/v0)^4) floored at -b; interaction s* = s0 + max(0, vT +
// v(v - vl)/den) with den = 2 sqrt(ab); gap floored at 0.1 m.
struct ClassParams {
    float v0f, T, a, b, s0, len, den, pad;
};

__device__ inline float idm_acc(float v, float v0, float vl, float s, const ClassParams& p, int kind,
                                unsigned& branches) {
    const float r = v / v0;
    const float r2 = r * r;
    const float r4 = r2 * r2;
    float phi = p.a * (1.0f - r4);
    if (phi < -p.b) {
        phi = -p.b;
        branches |= 1u;
    }
    if (kind == kFree) return phi;
    const float dv = v - vl;
    float dyn = (v * p.T) + ((v * dv) / p.den);
    if (dyn < 0.0f) {
        dyn = 0.0f;
        branches |= 2u;
    }
    const float sst = p.s0 + dyn;
    float se = s;
    if (s < kSMin) {
        se = kSMin;
        branches |= 4u;
    }
    const float q = sst / se;
    return phi - (p.a * (q * q));
}

// Eqs. (3)-(4) before the noise: max(g0, (g0 + alpha_1 v_i) + alpha_2 (v_i - v_o))
__device__ inline float crit_gap(float g0, float alpha1, float vi, float alpha2, float vo) {
    const float e = (g0 + alpha1 * vi) + alpha2 * (vi - vo);
    return e > g0 ? e : g0;
}

__device__ inline float desired_gap(float vi) { return vi < kV25mph ? kGSlow : kGFast; }

// distance from lane l to the nearest lane whose bit is set in mask (mask != 0)
__device__ inline int lane_distance(unsigned mask, int l) {
    if ((mask >> l) & 1u) return 0;
    int best = 64;
    const unsigned below = mask & ((1u << l) - 1u);
    if (below) best = l - (31 - __clz((int)below));
    const unsigned above = mask >> (l + 1);
    if (above) {
        const int d = __ffs((int)above);   // 1-based position of the lowest set bit
        if (d < best) best = d;
    }
    return best;
}

}  // namespace manta
