// Particle interaction of the WCSPH step (Sec. 3.2) with the SPH continuity
// and momentum equations, artificial viscosity and Tait equation of state of
// Sec. 2.2 and the dynamic boundaries of Sec. 2.3; plus the CFL time-step
// reduction (Sec. 3.3): block-local min, then one atomic min per block.
#include "sph_device.h"

namespace sph {

#ifndef SPH_INTERACT_ENT
#define SPH_INTERACT_ENT 19
#endif
#ifndef SPH_TEST_UNROLL
#define SPH_TEST_UNROLL 8
#endif
#ifndef SPH_ENT_SLACK
#define SPH_ENT_SLACK 3
#endif
#ifndef SPH_STAGE
#define SPH_STAGE 768
#endif
#ifndef SPH_INTERACT_WAVES_PER_EU
#define SPH_INTERACT_WAVES_PER_EU 3
#endif
// Hit-mask entries per lane: a lane's list holds up to kEnt - 1 entries and
// one sentinel slot.
constexpr int kEnt = SPH_INTERACT_ENT;
// At each run boundary the whole wave flushes together if any lane could not
// take kEntSlack more entries (a converged flush); inside a run a lane
// flushes alone only if its list fills (a run longer than 32 kEntSlack
// candidates).
constexpr int kEntSlack = SPH_ENT_SLACK;
constexpr int kUnroll = SPH_TEST_UNROLL;  // candidates loaded together in the support test
constexpr int kStage = SPH_STAGE;  // candidate positions a block stages in LDS per column offset
static_assert(32 % kUnroll == 0, "a hit mask covers whole groups of candidates");
constexpr uint32_t kRsrcWord3 = 0x00020000u;  // gfx9 buffer resource: 32-bit raw dwords

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v3f __attribute__((ext_vector_type(3)));
typedef uint32_t v3u __attribute__((ext_vector_type(3)));

// One lane per particle i of the label-0 prefix (Sec. 3.2: one thread per
// particle, neighbours in its own cell and the 26 adjacent ones). With an
// x-major cell index the three cells z-1..z+1 of each of the 9 (x, y) columns
// are one contiguous run of the sorted arrays, so the search is 9 runs.
//
// Two phases per lane keep the wave converged on the expensive part:
//   test:    every candidate of the 9 runs gets the FP32 support test
//            |r_ij|^2 < 4h^2 (groups of kUnroll bounds-checked buffer loads
//            in flight). The outcome is shifted into a 32-bit hit mask, one
//            bit per candidate (the sign of r_ij^2 - 4h^2, which is exact);
//            every 32 candidates of a run (and at its end) the mask and the
//            index of its first candidate go to the lane's list in LDS if any
//            bit is set;
//   compute: the pair terms are evaluated for the set bits only, each lane
//            walking its own list; a lane whose list is used up evaluates its
//            own particle (the sentinel entry), which adds exactly zero.
// The list is flushed early if it fills (dense regions), so any neighbour
// count and any run length are handled. The gradient constant and the mass
// are applied once per particle after the sums: grad_i W_ij = kgrad G(q) r_ij
// with
//   Wendland C2:   G = (1 - q/2)^3,                         kgrad = -5 aD / h^2;
//   cubic spline:  G = 4 - 3q (q < 1), (2 - q)^2 / q (q >= 1), kgrad = -3 aD / (4 h^2)
// (the two aD of the kernels' definitions differ).
template <bool kCubic>
__global__ __launch_bounds__(kInteractThreads) __attribute__((amdgpu_waves_per_eu(
    SPH_INTERACT_WAVES_PER_EU, SPH_INTERACT_WAVES_PER_EU))) void k_interact(
    KParams kp, const float4 *__restrict__ pos4, const float4 *__restrict__ vel4, uint32_t n,
    const uint8_t *__restrict__ type, const uint32_t *__restrict__ sk,
    const uint32_t *__restrict__ cbeg, const uint32_t *__restrict__ cend,
    DevInfo *__restrict__ info, float *__restrict__ oax, float *__restrict__ oay,
    float *__restrict__ oaz, float *__restrict__ orho, float *__restrict__ opress,
    float *__restrict__ onu, uint32_t *__restrict__ onpair) {
    constexpr int kWaves = kInteractThreads / 64;
    // entry = (byte offset 16 j of the first candidate of the mask, hit mask
    // with the first candidate in bit 31); [slot][lane]: a wave's 64 lanes
    // touch 512 consecutive bytes
    __shared__ uint2 s_ent[kEnt][kInteractThreads];
    // positions of the block's candidates of one column offset (the index
    // range spanned by the 256 lanes' runs), padded for a group past the end
    __shared__ float4 s_stage[kStage + kUnroll];
    __shared__ uint32_t s_lo[kWaves], s_hi[kWaves];
    __shared__ float s_rdt[kWaves];
    __shared__ uint32_t s_rnp[kWaves];
    __shared__ uint32_t s_rnc[kWaves];

    const int tid = threadIdx.x;
    const uint32_t n0 = info->n_label[0];
    const uint32_t blk = layer_block(blockIdx.x, (n0 + kInteractThreads - 1) / kInteractThreads, sk, cbeg, kp);
    const uint32_t i = blk * kInteractThreads + tid;
    const bool inrange = i < n0;
    const uint8_t ti = inrange ? type[i] : (uint8_t)kGhost;
    const bool act = ti != kGhost;  // this lane searches (in range and not a ghost)
    float dtmin = INFINITY;
    uint32_t npair = 0, ncand = 0;

    float4 pi = make_float4(0.f, 0.f, 0.f, 0.f), vi = pi;
    if (inrange) {
        pi = pos4[i];
        vi = vel4[i];
    }
    const float rhoi = vi.w, Pi = pi.w;
    const float si = rhoi * kp.inv_rho0;
    const float si3 = si * si * si;
    const float ci = kp.c0 * si3;
    float axs = 0.f, ays = 0.f, azs = 0.f, drho = 0.f, nu = 0.f;
    const __amdgpu_buffer_rsrc_t rp =
        __builtin_amdgcn_make_buffer_rsrc((void *)pos4, 0, (int)(n * 16u), kRsrcWord3);
    const __amdgpu_buffer_rsrc_t rv =
        __builtin_amdgcn_make_buffer_rsrc((void *)vel4, 0, (int)(n * 16u), kRsrcWord3);
    const uint32_t ncz = (uint32_t)kp.ncz, ncy = (uint32_t)kp.ncy;
    int cx = 0, cy = 0, cz = 0;
    if (act) {
        const uint32_t cell = sk[i] & kp.cell_mask;
        cz = (int)(cell % ncz);
        cy = (int)((cell / ncz) % ncy);
        cx = (int)(cell / (ncz * ncy));
    }
    const uint32_t zlo = (uint32_t)(cz > 0 ? cz - 1 : 0);
    const uint32_t zhi = (uint32_t)(cz + 1 < kp.ncz ? cz + 1 : kp.ncz - 1);
    const float hinv2 = -0.5f * kp.inv_h;
    const float eta2 = kp.eta2, h = kp.h;
    // Pi_ij = kvis (s_i^2 - s_i s_j + s_j^2) vr / (r^2 + eta^2) with s = rho/rho0,
    // evaluated as kvis2 (rho_i^2 - rho_i rho_j + rho_j^2) vr / (r^2 + eta^2)
    const float kvis2 = -kp.alpha * kp.h * kp.c0 * kp.inv_rho0 * kp.inv_rho0 * kp.inv_rho0;
    const float rhoi2 = rhoi * rhoi;

    auto pair = [&](const v4f pj, const v4f vj) {
        const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        float F;  // grad W / (kgrad r_ij)
        if (kCubic) {
            const float q = __builtin_amdgcn_sqrtf(r2) * kp.inv_h;
            const float t = 2.0f - q;
            // both sides first, then the choice: the compiler keeps it a
            // select (a conditional expression here became a branch)
            const float outer = t * t * __builtin_amdgcn_rcpf(q);
            const float inner = fmaf(-3.0f, q, 4.0f);
            F = q < 1.0f ? inner : outer;
        } else {
            const float t = fmaf(hinv2, __builtin_amdgcn_sqrtf(r2), 1.0f);  // 1 - q/2
            F = t * t * t;
        }
        const float ux = vi.x - vj.x, uy = vi.y - vj.y, uz = vi.z - vj.z;
        const float vr = fmaf(uz, dz, fmaf(uy, dy, ux * dx));
        drho = fmaf(F, vr, drho);
        // mu = h vr / (r^2 + eta^2) and the viscous term -alpha cbar mu /
        // rhobar with cbar = c0 (s_i^3 + s_j^3) / 2, rhobar = rho0 (s_i + s_j) / 2:
        // (s_i^3 + s_j^3) / (s_i + s_j) = s_i^2 - s_i s_j + s_j^2, so one
        // reciprocal serves both; h (in nu) and -alpha c0 h / rho0^3 (in the
        // force factor) are applied outside the sums. vR has the sign of vr:
        // min(vR, 0) is the approaching-pair switch (Pi = 0 when vr >= 0).
        const float vR = vr * __builtin_amdgcn_rcpf(r2 + eta2);
        nu = fmaxf(nu, fabsf(vR));  // |mu| / h
        const float visc = fmaf(vj.w, vj.w - rhoi, rhoi2) * fminf(vR, 0.0f);  // Pi / kvis2
        const float f = fmaf(kvis2, visc, Pi + pj.w) * F;
        axs = fmaf(f, dx, axs);
        ays = fmaf(f, dy, ays);
        azs = fmaf(f, dz, azs);
    };

    // compute phase over the cnt entries of the lane's list holding
    // nhit set bits. The sentinel (16 i, bit 31) after the last entry
    // stands in for every position past the end, so a group of four
    // never needs a mask. The next group's indices are drawn from the
    // masks while the current group's neighbour data is in flight.
    auto flush = [&](uint32_t cnt, uint32_t nhit) {
        s_ent[cnt][tid] = make_uint2(i * 16u, 0x80000000u);
        uint32_t pk = 0, cb = 0, cj = 0;
        uint2 nx = s_ent[0][tid];
        auto draw = [&](uint32_t (&jj)[4]) {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const bool empty = cb == 0u;  // take the prefetched entry
                cb = empty ? nx.y : cb;
                cj = empty ? nx.x : cj;
                pk = min(pk + (empty ? 1u : 0u), cnt);
                nx = s_ent[pk][tid];
                const uint32_t off = (uint32_t)__builtin_clz(cb);
                jj[u] = cj + (off << 4);  // byte offset of j
                cb &= 0x7fffffffu >> off;
            }
        };
        // two groups in flight: the next group's data loads while the
        // current one is evaluated (past the end the sentinel's own index)
        uint32_t jn[4];
        draw(jn);
        v4f qp[4], qv[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            qp[u] = __builtin_amdgcn_raw_buffer_load_b128(rp, jn[u], 0, 0);
            qv[u] = __builtin_amdgcn_raw_buffer_load_b128(rv, jn[u], 0, 0);
        }
        draw(jn);
        for (uint32_t t = 0; t < nhit; t += 4) {
            v4f np[4], nv[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                np[u] = __builtin_amdgcn_raw_buffer_load_b128(rp, jn[u], 0, 0);
                nv[u] = __builtin_amdgcn_raw_buffer_load_b128(rv, jn[u], 0, 0);
            }
            draw(jn);
#pragma unroll
            for (int u = 0; u < 4; u++) {
                pair(qp[u], qv[u]);
                qp[u] = np[u];
                qv[u] = nv[u];
            }
        }
    };

    // The list keeps i itself (found in its own run): the self pair has
    // r_ij = v_ij = 0 and adds exactly zero to every sum and to nu, so
    // it costs one bit instead of a j != i test per candidate.
    uint32_t lp = 0;    // entries in the lane's list
    uint32_t nhit = 0;  // set bits in them
    uint32_t listed = 0;
    auto put = [&](uint32_t j16, uint32_t b) {
        s_ent[lp][tid] = make_uint2(j16, b);
        lp += b != 0u ? 1u : 0u;
        nhit += (uint32_t)__builtin_popcount(b);
        if (lp >= (uint32_t)(kEnt - 1)) {  // full: this lane alone
            flush(lp, nhit);
            listed += nhit;
            lp = 0;
            nhit = 0;
        }
    };
    // every lane of the block runs the column loop (it holds barriers);
    // lanes that do not search have empty runs
    for (int col = 0; col < 9; col++) {
        if (__any(act && lp > (uint32_t)(kEnt - 1 - kEntSlack))) {
            if (act) {
                flush(lp, nhit);
                listed += nhit;
                lp = 0;
                nhit = 0;
            }
        }
        const int X = cx + col / 3 - 1, Y = cy + col % 3 - 1;
        uint32_t jb = 0, je = 0;
        if (act && X >= 0 && X < kp.ncx && Y >= 0 && Y < kp.ncy) {
            const uint32_t c0 = ((uint32_t)X * ncy + (uint32_t)Y) * ncz;
            jb = cbeg[c0 + zlo];
            je = cend[c0 + zhi];
        }
        const uint32_t len = je - jb;
        ncand += len;
        // index range [lo, hi) of the block's runs of this column offset:
        // consecutive particles lie in one (x, y) column or in neighbouring
        // ones, whose neighbour columns are neighbours in the x-major order
        // too, so the range is compact except where the block crosses an
        // x-layer of cells. For a fixed offset the neighbour cell of a later
        // particle (in sorted order) is never an earlier cell, so jb and je
        // never decrease along the lanes: the wave's range runs from the jb
        // of its first lane with a run to the je of its last.
        const unsigned long long wm = __ballot(len != 0u);
        uint32_t lo = 0xffffffffu, hi = 0u;
        if (wm) {
            lo = (uint32_t)__builtin_amdgcn_readlane((int)jb, __builtin_ctzll(wm));
            hi = (uint32_t)__builtin_amdgcn_readlane((int)je, 63 - __builtin_clzll(wm));
        }
        if ((tid & 63) == 0) {
            s_lo[tid >> 6] = lo;
            s_hi[tid >> 6] = hi;
        }
        __syncthreads();  // also: every wave is done with the previous staging
#pragma unroll
        for (int w = 0; w < kWaves; w++) {
            lo = min(lo, s_lo[w]);
            hi = max(hi, s_hi[w]);
        }
        const bool staged = hi > lo && hi - lo <= (uint32_t)kStage;  // the same in every lane
        if (staged) {
            for (uint32_t t = tid; t < hi - lo; t += kInteractThreads) s_stage[t] = pos4[lo + t];
        }
        __syncthreads();
        if (!len) continue;
        const uint32_t voff = jb * 16u;
        uint32_t bits = 0;
        uint32_t k0 = 0;
        auto test = [&](const v3f (&q)[kUnroll], uint32_t k) {
#pragma unroll
            for (int u = 0; u < kUnroll; u++) {
                const float dx = pi.x - q[u].x, dy = pi.y - q[u].y, dz = pi.z - q[u].z;
                // e = r^2 - 4h^2 as one chain of fused multiply-adds from
                // -4h^2; bits = bits << 1 | (e < 0) (a zero sum is +0)
                const float e = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, -kp.r2max)));
                bits = __builtin_amdgcn_alignbit(bits, __float_as_uint(e), 31);
            }
            if ((k & 31u) == 32u - kUnroll) {  // 32 candidates tested
                const uint32_t c0 = k + kUnroll - 32u;
                const uint32_t v = len - c0;  // of which inside the run
                put(voff + c0 * 16u, v >= 32u ? bits : bits & ~(0xffffffffu >> v));
                bits = 0;
            }
        };
        // k0 is the same for every lane still in its run (the group counter
        // of the wave). Candidates past the run give garbage that the mask
        // of valid candidates drops.
        if (staged) {
            const float4 *sp = s_stage + (jb - lo);
            for (; k0 < len; k0 += kUnroll) {
                v3f q[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; u++) {
                    const float4 t = sp[k0 + u];
                    q[u] = v3f{t.x, t.y, t.z};
                }
                test(q, k0);
            }
        } else {  // range too wide to stage (a block across an x-layer): bounds-checked loads
            for (; k0 < len; k0 += kUnroll) {
                v3f q[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; u++)  // past the run: in-bounds data or 0
                    q[u] = __builtin_bit_cast(
                        v3f, __builtin_amdgcn_raw_buffer_load_b96(rp, voff, (int)(k0 * 16u + 16u * u), 0));
                test(q, k0);
            }
        }
        const uint32_t tail = k0 & 31u;  // candidates tested since the last mask
        if (tail) {
            const uint32_t c0 = k0 - tail;
            const uint32_t v = len - c0;  // 1 .. tail
            put(voff + c0 * 16u, (bits << (32u - tail)) & ~(0xffffffffu >> v));
        }
    }
    if (act) {
        flush(lp, nhit);
        npair = listed + nhit - 1u;  // minus the self entry
        nu *= h;
    }
    if (inrange) {
        const float mk = kp.mass * (kCubic ? kp.kgrad_cubic : kp.kgrad);
        float ax = 0.f, ay = 0.f, az = 0.f, ar = 0.f;
        if (ti == kFluid) {
            ax = fmaf(-mk, axs, kp.gx);
            ay = fmaf(-mk, ays, kp.gy);
            az = fmaf(-mk, azs, kp.gz);
        }
        if (ti != kGhost) {
            ar = mk * drho;
            // CFL limits (Sec. 3.3): h / (c_i + nu_i), and sqrt(h/|a_i|) for fluid
            dtmin = kp.h / (ci + nu);
            if (ti == kFluid) {
                const float a2 = fmaf(az, az, fmaf(ay, ay, ax * ax));
                if (a2 > 0.0f) dtmin = fminf(dtmin, sqrtf(kp.h / sqrtf(a2)));
            }
        }
        oax[i] = ax;
        oay[i] = ay;
        oaz[i] = az;
        orho[i] = ar;
        if (opress) opress[i] = tait_p(kp, rhoi);
        if (onu) onu[i] = nu;
        if (onpair) onpair[i] = npair;
    }

    // block-local reduction of the dt limit, the pair and candidate counts
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        dtmin = fminf(dtmin, __shfl_xor(dtmin, o, 64));
        npair += __shfl_xor(npair, o, 64);
        ncand += __shfl_xor(ncand, o, 64);
    }
    if ((tid & 63) == 0) {
        s_rdt[tid >> 6] = dtmin;
        s_rnp[tid >> 6] = npair;
        s_rnc[tid >> 6] = ncand;
    }
    __syncthreads();
    if (tid == 0) {
        float d = s_rdt[0];
        uint32_t np = s_rnp[0], nc = s_rnc[0];
        for (int k = 1; k < kWaves; k++) {
            d = fminf(d, s_rdt[k]);
            np += s_rnp[k];
            nc += s_rnc[k];
        }
        // device-wide min and sums; positive floats order like their bits, and
        // neither min nor integer sums depend on the order of the blocks
        if (d < INFINITY) atomicMin(&info->dtmin_bits, __float_as_uint(d));
        if (np) {
            atomicAdd(&info->pairs, (unsigned long long)np);
            atomicAdd(&info->pairs_total, (unsigned long long)np);
        }
        if (nc) atomicAdd(&info->cand_total, (unsigned long long)nc);
    }
}

hipError_t launch_interact(sph_ctx *c, const uint8_t *type, uint32_t n, const sph_rates &out,
                           hipStream_t s, hipEvent_t after_kernel) {
    const uint32_t nb = n == 0 ? 1 : (n + kInteractThreads - 1) / kInteractThreads;
    auto kern = (c->kp.options & SPH_O_CUBIC) ? k_interact<true> : k_interact<false>;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kInteractThreads), 0, s, c->kp, c->pos4, c->vel4, n,
                       type, c->keys_sorted, c->cell_begin, c->cell_end, c->info, out.ax, out.ay,
                       out.az, out.arho, out.press, out.nu, out.npair);
    if (after_kernel) (void)hipEventRecord(after_kernel, s);
    return hipGetLastError();
}

}  // namespace sph
