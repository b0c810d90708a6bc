// Particle interaction of the WCSPH step (Sec. 3.2) with the SPH continuity
// and momentum equations, artificial viscosity and Tait equation of state of
// Sec. 2.2 and the dynamic boundaries of Sec. 2.3; plus the per-block parts of
// the CFL time-step reduction (Sec. 3.3).
#include "sph_device.h"

namespace sph {

constexpr int kCap = 128;  // neighbour entries buffered per lane before a flush

// One lane per particle i of the label-0 prefix (Sec. 3.2: one thread per
// particle, neighbours in its own cell and the 26 adjacent ones). With an
// x-major cell index the three cells z-1..z+1 of each of the 9 (x, y) columns
// are one contiguous run of the sorted arrays, so the search is 9 runs.
//
// Two phases per lane keep the wave converged on the expensive part:
//   test:    every candidate of the 9 runs gets the FP32 support test
//            |r_ij|^2 < 4h^2; hits are appended to the lane's own list in LDS
//            as 16-bit (run, offset) entries;
//   compute: the pair terms are evaluated for the listed neighbours only.
// The list is flushed early if it fills (dense regions), so any neighbour
// count is handled.
__global__ __launch_bounds__(kInteractThreads) void k_interact(
    KParams kp, const float4 *__restrict__ pos4, const float4 *__restrict__ vel4,
    const uint8_t *__restrict__ type, const uint32_t *__restrict__ sk,
    const uint32_t *__restrict__ cbeg, const uint32_t *__restrict__ cend,
    DevInfo *__restrict__ info, float *__restrict__ oax, float *__restrict__ oay,
    float *__restrict__ oaz, float *__restrict__ orho, float *__restrict__ opress,
    float *__restrict__ onu, float *__restrict__ dt_part, uint32_t *__restrict__ pair_part) {
    __shared__ uint16_t s_list[kCap][kInteractThreads];
    __shared__ uint32_t s_base[9][kInteractThreads];
    __shared__ float s_rdt[kInteractThreads / 64];
    __shared__ uint32_t s_rnp[kInteractThreads / 64];

    const int tid = threadIdx.x;
    const uint32_t n0 = info->n_label[0];
    const uint32_t i = blockIdx.x * kInteractThreads + tid;
    const bool inrange = i < n0;
    const uint8_t ti = inrange ? type[i] : (uint8_t)kGhost;
    float dtmin = INFINITY;
    uint32_t npair = 0;

    if (inrange) {
        const float4 pi = pos4[i], vi = vel4[i];
        const float rhoi = vi.w, Pi = pi.w;
        const float si = rhoi * kp.inv_rho0;
        const float ci = kp.c0 * (si * si * si);
        float axs = 0.f, ays = 0.f, azs = 0.f, drho = 0.f, nu = 0.f;
        if (ti != kGhost) {
            const uint32_t cell = sk[i] & kp.cell_mask;
            const uint32_t ncz = (uint32_t)kp.ncz, ncy = (uint32_t)kp.ncy;
            const int cz = (int)(cell % ncz);
            const int cy = (int)((cell / ncz) % ncy);
            const int cx = (int)(cell / (ncz * ncy));
            const uint32_t zlo = (uint32_t)(cz > 0 ? cz - 1 : 0);
            const uint32_t zhi = (uint32_t)(cz + 1 < kp.ncz ? cz + 1 : kp.ncz - 1);
            const float hinv2 = -0.5f * kp.inv_h;
            const float vr_h = kp.h;

            auto flush = [&](int cnt) {
                for (int k = 0; k < cnt; k++) {
                    const uint32_t e = s_list[k][tid];
                    const uint32_t j = s_base[e >> kRunBits][tid] + (e & kRunMax);
                    const float4 pj = pos4[j];
                    const float4 vj = vel4[j];
                    const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
                    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    const float r = __builtin_amdgcn_sqrtf(r2);
                    const float t = fmaf(hinv2, r, 1.0f);  // 1 - q/2
                    const float F = kp.kgrad * (t * t * t);
                    const float ux = vi.x - vj.x, uy = vi.y - vj.y, uz = vi.z - vj.z;
                    const float vr = fmaf(uz, dz, fmaf(uy, dy, ux * dx));
                    drho = fmaf(F, vr, drho);
                    const float mu = vr_h * vr * __builtin_amdgcn_rcpf(r2 + kp.eta2);
                    nu = fmaxf(nu, fabsf(mu));
                    const float sj = vj.w * kp.inv_rho0;
                    const float cj = kp.c0 * (sj * sj * sj);
                    const float visc =
                        vr < 0.0f ? -kp.alpha * (ci + cj) * mu * __builtin_amdgcn_rcpf(rhoi + vj.w)
                                  : 0.0f;
                    const float f = (Pi + pj.w + visc) * F;
                    axs = fmaf(f, dx, axs);
                    ays = fmaf(f, dy, ays);
                    azs = fmaf(f, dz, azs);
                }
            };

            int cnt = 0;
            for (int col = 0; col < 9; col++) {
                const int X = cx + col / 3 - 1, Y = cy + col % 3 - 1;
                uint32_t jb = 0, je = 0;
                if (X >= 0 && X < kp.ncx && Y >= 0 && Y < kp.ncy) {
                    const uint32_t c0 = ((uint32_t)X * ncy + (uint32_t)Y) * ncz;
                    jb = cbeg[c0 + zlo];
                    je = cend[c0 + zhi];
                }
                if (je - jb > kRunMax + 1u) {
                    atomicOr(&info->flags, (uint32_t)SPH_S_RUN_OVERFLOW);
                    je = jb + kRunMax + 1u;
                }
                s_base[col][tid] = jb;
                for (uint32_t j = jb; j < je; j++) {
                    const float4 pj = pos4[j];
                    const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
                    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    if (r2 < kp.r2max && j != i) {
                        s_list[cnt][tid] = (uint16_t)(((uint32_t)col << kRunBits) | (j - jb));
                        npair++;
                        if (++cnt == kCap) {
                            flush(cnt);
                            cnt = 0;
                        }
                    }
                }
            }
            flush(cnt);
        }
        const float m = kp.mass;
        float ax = 0.f, ay = 0.f, az = 0.f, ar = 0.f;
        if (ti == kFluid) {
            ax = fmaf(-m, axs, kp.gx);
            ay = fmaf(-m, ays, kp.gy);
            az = fmaf(-m, azs, kp.gz);
        }
        if (ti != kGhost) {
            ar = m * drho;
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
    }

    // block-local reduction of the dt limit and of the pair count
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        dtmin = fminf(dtmin, __shfl_xor(dtmin, o, 64));
        npair += __shfl_xor(npair, o, 64);
    }
    if ((tid & 63) == 0) {
        s_rdt[tid >> 6] = dtmin;
        s_rnp[tid >> 6] = npair;
    }
    __syncthreads();
    if (tid == 0) {
        float d = s_rdt[0];
        uint32_t np = s_rnp[0];
        for (int k = 1; k < kInteractThreads / 64; k++) {
            d = fminf(d, s_rdt[k]);
            np += s_rnp[k];
        }
        dt_part[blockIdx.x] = d;
        pair_part[blockIdx.x] = np;
    }
}

// dt = CFL * min over blocks; total neighbour pairs.
__global__ __launch_bounds__(256) void k_dt_final(KParams kp, const float *__restrict__ dt_part,
                                                  const uint32_t *__restrict__ pair_part,
                                                  uint32_t nblocks, DevInfo *__restrict__ info) {
    __shared__ float s_d[4];
    __shared__ unsigned long long s_p[4];
    const int tid = threadIdx.x;
    float d = INFINITY;
    unsigned long long np = 0;
    for (uint32_t b = tid; b < nblocks; b += 256) {
        d = fminf(d, dt_part[b]);
        np += pair_part[b];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        d = fminf(d, __shfl_xor(d, o, 64));
        np += __shfl_xor(np, o, 64);
    }
    if ((tid & 63) == 0) {
        s_d[tid >> 6] = d;
        s_p[tid >> 6] = np;
    }
    __syncthreads();
    if (tid == 0) {
        d = fminf(fminf(s_d[0], s_d[1]), fminf(s_d[2], s_d[3]));
        np = s_p[0] + s_p[1] + s_p[2] + s_p[3];
        const float dt = kp.cfl * d;
        info->dt = dt;
        info->pairs = np;
        info->pairs_total += np;
        if (!(dt > 0.0f) || !(dt < INFINITY)) atomicOr(&info->flags, (uint32_t)SPH_S_DT);
    }
}

hipError_t launch_interact(sph_ctx *c, const uint8_t *type, uint32_t n, const sph_rates &out,
                           hipStream_t s, hipEvent_t after_kernel) {
    const uint32_t nb = n == 0 ? 1 : (n + kInteractThreads - 1) / kInteractThreads;
    hipLaunchKernelGGL(k_interact, dim3(nb), dim3(kInteractThreads), 0, s, c->kp, c->pos4,
                       c->vel4, type, c->keys_sorted, c->cell_begin, c->cell_end, c->info,
                       out.ax, out.ay, out.az, out.arho, out.press, out.nu, c->dt_part,
                       c->pair_part);
    if (after_kernel) (void)hipEventRecord(after_kernel, s);
    hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(256), 0, s, c->kp, c->dt_part, c->pair_part, nb,
                       c->info);
    return hipGetLastError();
}

}  // namespace sph
