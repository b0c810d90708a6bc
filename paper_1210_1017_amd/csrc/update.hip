// Verlet update of the WCSPH step (Sec. 3.3) with the dynamic-boundary rule
// of Sec. 2.3: fluid advances position, velocity and density; boundary
// particles advance density only; ghosts are not updated.
#include "sph_device.h"

namespace sph {

// Leapfrog form of the second-order Verlet scheme, with an Euler step every
// euler_every steps (step 0 included):
//   Euler:    v' = v + dt a,        rho' = rho + dt D
//   leapfrog: v' = v_prev + 2dt a,  rho' = rho_prev + 2dt D
//   r' = r + dt v + dt^2 a / 2, then (v_prev, rho_prev) <- (v, rho).
// With SPH_O_RHO_FLOOR a boundary particle's new density is at least rho0.
// PACKED (inside sph_step): r, v and rho are read from the interaction's
// packed inputs (pos4, vel4), which hold the same bits, and written for every
// particle, updated or not, since the reorder left them out of the state.
template <bool PACKED>
__global__ __launch_bounds__(256) void k_verlet(KParams kp, sph_soa st,
                                                const float *__restrict__ ax,
                                                const float *__restrict__ ay,
                                                const float *__restrict__ az,
                                                const float *__restrict__ arho,
                                                const float4 *__restrict__ pos4,
                                                const float4 *__restrict__ vel4, uint32_t n,
                                                DevInfo *__restrict__ info, int euler) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    // dt = CFL * (smallest per-particle limit of the interaction), Sec. 3.3
    const float dt = kp.cfl * __uint_as_float(info->dtmin_bits);
    if (k == 0) {
        info->dt = dt;
        if (!(dt > 0.0f) || !(dt < INFINITY)) atomicOr(&info->flags, (uint32_t)SPH_S_DT);
    }
    const uint32_t n0 = info->n_label[0];
    if (k >= (PACKED ? n : n0)) return;
    const uint8_t t = st.type[k];
    float r[3], v[3], rho;
    if (PACKED) {
        const float4 p4 = pos4[k], v4 = vel4[k];
        r[0] = p4.x; r[1] = p4.y; r[2] = p4.z;
        v[0] = v4.x; v[1] = v4.y; v[2] = v4.z;
        rho = v4.w;
    }
    const bool upd = k < n0 && t != kGhost;
    if (upd) {
        if (!PACKED) rho = st.rho[k];
        float rn = euler ? fmaf(dt, arho[k], rho) : fmaf(2.0f * dt, arho[k], st.rhop[k]);
        if ((kp.options & SPH_O_RHO_FLOOR) && t == kBoundary && rn < kp.rho0) rn = kp.rho0;
        st.rhop[k] = rho;
        rho = rn;
        bool ok = isfinite(rn);
        if (t == kFluid) {
            const float a[3] = {ax[k], ay[k], az[k]};
            const float *pos[3] = {st.x, st.y, st.z};
            const float *vel[3] = {st.vx, st.vy, st.vz};
            float *velp[3] = {st.vxp, st.vyp, st.vzp};
            const float hdt2 = 0.5f * dt * dt;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                if (!PACKED) {
                    r[d] = pos[d][k];
                    v[d] = vel[d][k];
                }
                const float vn = euler ? fmaf(dt, a[d], v[d]) : fmaf(2.0f * dt, a[d], velp[d][k]);
                const float xn = r[d] + fmaf(hdt2, a[d], dt * v[d]);
                velp[d][k] = v[d];
                r[d] = xn;
                v[d] = vn;
                ok = ok && isfinite(vn) && isfinite(xn);
            }
            if (!PACKED) {
                st.x[k] = r[0]; st.y[k] = r[1]; st.z[k] = r[2];
                st.vx[k] = v[0]; st.vy[k] = v[1]; st.vz[k] = v[2];
            }
        }
        if (!PACKED) st.rho[k] = rho;
        if (!ok) atomicOr(&info->flags, (uint32_t)SPH_S_NONFINITE);
    }
    if (PACKED) {
        st.x[k] = r[0]; st.y[k] = r[1]; st.z[k] = r[2];
        st.vx[k] = v[0]; st.vy[k] = v[1]; st.vz[k] = v[2];
        st.rho[k] = rho;
    }
}

// Symplectic variant (SPH_O_SYMPLECTIC, not in the paper): a kick-drift
// position-Verlet step with dt from the rates at n.
//   k_sym_half: the half state r + dt/2 v, v + dt/2 a (fluid), rho + dt/2 D
//     (fluid and boundary), written straight into the packed interaction
//     inputs (pos4 with the EOS term p/rho^2 of rho_h, vel4 with rho_h), so
//     the second interaction reads it with the cell tables of the sort at n;
//     the sorted state arrays keep the values at n.
//   k_sym_full: v' = v + dt a_h, r' = r + dt (v + v')/2 (fluid);
//     rho' = rho (2 - e)/(2 + e), e = -(D_h / rho_h) dt (fluid and boundary);
//     (v_prev, rho_prev) <- (v, rho).
__global__ __launch_bounds__(256) void k_sym_half(KParams kp, sph_soa st,
                                                  const float *__restrict__ ax,
                                                  const float *__restrict__ ay,
                                                  const float *__restrict__ az,
                                                  const float *__restrict__ arho,
                                                  float4 *__restrict__ pos4,
                                                  float4 *__restrict__ vel4,
                                                  DevInfo *__restrict__ info) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const float dt = kp.cfl * __uint_as_float(info->dtmin_bits);
    if (k == 0) {
        info->dt = dt;
        info->pairs = 0ull;  // the pair count of the step is the half state's
        if (!(dt > 0.0f) || !(dt < INFINITY)) atomicOr(&info->flags, (uint32_t)SPH_S_DT);
    }
    if (k >= info->n_label[0]) return;
    const uint8_t t = st.type[k];
    if (t == kGhost) return;  // pos4 / vel4 keep the gathered values
    const float hdt = 0.5f * dt;
    const float rh = fmaf(hdt, arho[k], st.rho[k]);
    float x = st.x[k], y = st.y[k], z = st.z[k];
    float vx = st.vx[k], vy = st.vy[k], vz = st.vz[k];
    if (t == kFluid) {
        const float ux = vx, uy = vy, uz = vz;
        vx = fmaf(hdt, ax[k], vx);
        vy = fmaf(hdt, ay[k], vy);
        vz = fmaf(hdt, az[k], vz);
        x = fmaf(hdt, ux, x);
        y = fmaf(hdt, uy, y);
        z = fmaf(hdt, uz, z);
    }
    pos4[k] = make_float4(x, y, z, tait_p_over_rho2(kp, rh));
    vel4[k] = make_float4(vx, vy, vz, rh);
    if (!isfinite(rh) || !isfinite(x) || !isfinite(y) || !isfinite(z))
        atomicOr(&info->flags, (uint32_t)SPH_S_NONFINITE);
}

__global__ __launch_bounds__(256) void k_sym_full(KParams kp, sph_soa st,
                                                  const float *__restrict__ ax,
                                                  const float *__restrict__ ay,
                                                  const float *__restrict__ az,
                                                  const float *__restrict__ arho,
                                                  const float4 *__restrict__ vel4,
                                                  DevInfo *__restrict__ info) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= info->n_label[0]) return;
    const uint8_t t = st.type[k];
    if (t == kGhost) return;
    const float dt = info->dt;
    const float rho = st.rho[k];
    const float e = -(arho[k] / vel4[k].w) * dt;
    float rn = rho * (2.0f - e) / (2.0f + e);
    if ((kp.options & SPH_O_RHO_FLOOR) && t == kBoundary && rn < kp.rho0) rn = kp.rho0;
    st.rhop[k] = rho;
    st.rho[k] = rn;
    bool ok = isfinite(rn);
    if (t == kFluid) {
        const float a[3] = {ax[k], ay[k], az[k]};
        float *pos[3] = {st.x, st.y, st.z};
        float *vel[3] = {st.vx, st.vy, st.vz};
        float *velp[3] = {st.vxp, st.vyp, st.vzp};
        const float hdt = 0.5f * dt;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const float v = vel[d][k];
            const float vn = fmaf(dt, a[d], v);
            const float xn = fmaf(hdt, v + vn, pos[d][k]);
            pos[d][k] = xn;
            velp[d][k] = v;
            vel[d][k] = vn;
            ok = ok && isfinite(vn) && isfinite(xn);
        }
    }
    if (!ok) atomicOr(&info->flags, (uint32_t)SPH_S_NONFINITE);
}

hipError_t launch_sym_half(sph_ctx *c, const sph_soa &st, const float *ax, const float *ay,
                           const float *az, const float *arho, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_sym_half, dim3(n == 0 ? 1 : (n + 255) / 256), dim3(256), 0, s, c->kp, st,
                       ax, ay, az, arho, c->pos4, c->vel4, c->info);
    return hipGetLastError();
}

hipError_t launch_sym_full(sph_ctx *c, const sph_soa &st, const float *ax, const float *ay,
                           const float *az, const float *arho, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_sym_full, dim3(n == 0 ? 1 : (n + 255) / 256), dim3(256), 0, s, c->kp, st,
                       ax, ay, az, arho, c->vel4, c->info);
    return hipGetLastError();
}

hipError_t launch_update(sph_ctx *c, const sph_soa &st, const float *ax, const float *ay,
                         const float *az, const float *arho, uint32_t n, uint64_t step,
                         hipStream_t s, bool packed) {
    const int E = c->kp.euler_every;
    const int euler = E > 0 ? (step % (uint64_t)E == 0) : (step == 0);
    const dim3 grid(n == 0 ? 1 : (n + 255) / 256);
    if (packed)
        hipLaunchKernelGGL(k_verlet<true>, grid, dim3(256), 0, s, c->kp, st, ax, ay, az, arho,
                           c->pos4, c->vel4, n, c->info, euler);
    else
        hipLaunchKernelGGL(k_verlet<false>, grid, dim3(256), 0, s, c->kp, st, ax, ay, az, arho,
                           c->pos4, c->vel4, n, c->info, euler);
    return hipGetLastError();
}

}  // namespace sph
