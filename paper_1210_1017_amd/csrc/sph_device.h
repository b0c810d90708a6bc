// Device helpers shared by the HIP kernels of libsph.so.
#pragma once

#include "sph_internal.h"

namespace sph {

// Tait equation of state (Sec. 2.2), gamma = 7, in FP32 without the
// cancellation of (rho/rho0)^7 - 1 near rho0: with s = rho/rho0,
// s^7 - 1 = (s - 1)(1 + s + ... + s^6), and rho - rho0 is exact in FP32.
__device__ __forceinline__ float tait_p(const KParams &kp, float rho) {
    const float e = (rho - kp.rho0) * kp.inv_rho0;
    const float s = rho * kp.inv_rho0;
    float q = s + 1.0f;
    q = fmaf(q, s, 1.0f);
    q = fmaf(q, s, 1.0f);
    q = fmaf(q, s, 1.0f);
    q = fmaf(q, s, 1.0f);
    q = fmaf(q, s, 1.0f);
    return kp.B * e * q;
}

// p / rho^2, the pressure factor of the symmetric momentum equation.
__device__ __forceinline__ float tait_p_over_rho2(const KParams &kp, float rho) {
    return tait_p(kp, rho) / (rho * rho);
}

// Sound speed c = sqrt(dp/drho) = c0 (rho/rho0)^3 for gamma = 7.
__device__ __forceinline__ float sound_speed(const KParams &kp, float rho) {
    const float s = rho * kp.inv_rho0;
    return kp.c0 * (s * s * s);
}

// Cell key of one particle (Sec. 3.1 cells of side 2h; Sec. 4.3 migration
// label): FP32 cell coordinates floor((x - o) * (1/cs)); outside the grid on
// any axis (or NaN) -> label 3; in slab mode a non-ghost particle left of
// slab_xlo -> 1, at or right of slab_xhi -> 2. key = label << Bc | cell.
__device__ __forceinline__ uint32_t cell_key(const KParams &kp, float px, float py, float pz,
                                             uint8_t type) {
#pragma clang fp contract(off)
    const float tx = (px - kp.ox) * kp.inv_cs;
    const float ty = (py - kp.oy) * kp.inv_cs;
    const float tz = (pz - kp.oz) * kp.inv_cs;
    // no short-circuit and no early return: every input is needed up front,
    // so a caller's loads of x, y, z and type are issued together instead of
    // one after another behind branches
    const bool inside = (tx >= 0.0f) & (tx < (float)kp.ncx) & (ty >= 0.0f) &
                        (ty < (float)kp.ncy) & (tz >= 0.0f) & (tz < (float)kp.ncz);
    // clamped only so that the conversions of an outside (or NaN) coordinate
    // stay defined; inside particles are unchanged by the clamp
    const uint32_t cx = (uint32_t)(int)floorf(fminf(fmaxf(tx, 0.0f), (float)(kp.ncx - 1)));
    const uint32_t cy = (uint32_t)(int)floorf(fminf(fmaxf(ty, 0.0f), (float)(kp.ncy - 1)));
    const uint32_t cz = (uint32_t)(int)floorf(fminf(fmaxf(tz, 0.0f), (float)(kp.ncz - 1)));
    const uint32_t cell = (cx * (uint32_t)kp.ncy + cy) * (uint32_t)kp.ncz + cz;
    const uint32_t lab = px < kp.slab_xlo ? 1u : (px >= kp.slab_xhi ? 2u : 0u);
    const uint32_t label = (kp.slab_mode && type != kGhost) ? lab : 0u;
    return inside ? (label << kp.cell_bits) | cell : 3u << kp.cell_bits;
}

// Workgroups are handed to the 8 XCDs of the chip round-robin. Renumber them
// so that each XCD receives stretches of kXcdChunk consecutive blocks (the
// neighbour data of a stretch then stays in one XCD's L2) dealt out in turn
// over the whole domain (the cost per particle varies along x: dealing
// stretches keeps the XCDs evenly loaded). A bijection of [0, nb); the last
// partial round keeps the hardware order.
#ifndef SPH_XCD_CHUNK
#define SPH_XCD_CHUNK 16
#endif
constexpr uint32_t kXcdChunk = SPH_XCD_CHUNK;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
    constexpr uint32_t X = 8;
    const uint32_t round = X * kXcdChunk;
    const uint32_t full = nb / round * round;
    if (kXcdChunk <= 1 || b >= full) return b;
    const uint32_t x = b % X, k = b / X;  // k-th block that XCD x receives
    return (k / kXcdChunk) * round + x * kXcdChunk + k % kXcdChunk;
}

// Block order of the interaction kernels (blocks of kInteractThreads
// particles): the hardware hands block b to XCD b % 8. In the sorted
// order, the blocks whose first particle lies in x-layer X of cells form a
// range [s0, s1); of these, each XCD receives as many as it would in index
// order, but as one contiguous group (XCD 0 the first group, and so on).
// All XCDs then work through the same layer at the same time, each on its
// own range of rows, and the neighbour rows in layers X - 1 and X + 1 of a
// group are the same XCD's groups there, read shortly before and after
// (its L2 keeps them). Blocks past the label-0 prefix keep their index.
__device__ __forceinline__ uint32_t layer_block(uint32_t b, uint32_t nb0,
                                                const uint32_t *__restrict__ sk,
                                                const uint32_t *__restrict__ cbeg,
                                                const KParams &kp) {
    if (b >= nb0) return b;
    const uint32_t lay = (uint32_t)kp.ncy * (uint32_t)kp.ncz;
    const uint32_t X = (sk[b * kInteractThreads] & kp.cell_mask) / lay;
    auto start = [&](uint32_t x) -> uint32_t {  // first block of layer x
        return x >= (uint32_t)kp.ncx ? nb0
                                     : min((cbeg[x * lay] + kInteractThreads - 1) / kInteractThreads, nb0);
    };
    const uint32_t s0 = start(X), s1 = start(X + 1);
    auto cnt = [](uint32_t a, uint32_t x) { return (a + 7u - x) / 8u; };  // j < a with j % 8 == x
    const uint32_t x = b % 8u;
    uint32_t g = s0;
    for (uint32_t y = 0; y < x; y++) g += cnt(s1, y) - cnt(s0, y);
    return g + cnt(b, x) - cnt(s0, x);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive prefix sum over a block of NT threads (NT a multiple of 64).
// s_w must hold NT/64 words of shared memory. Every thread must call it.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_w,
                                                    uint32_t *total = nullptr) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; k++) {
        const uint32_t t = s_w[k];
        if (k < w) pre += t;
        tot += t;
    }
    __syncthreads();
    if (total) *total = tot;
    return pre + incl - v;
}

}  // namespace sph
