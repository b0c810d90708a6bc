// Variant paths of the WCSPH step:
//  * cell + offset positions (int32 cell, FP32 offset from the cell centre),
//    FP32 interaction on separations formed from offsets and cell
//    differences, FP64 dt minimum and FP64 global totals;
//  * an FP64 reference path (every state array, the interaction and the
//    update in FP64).
// The sort machinery (radix sort, cell tables, counts) is shared with the
// plain path; only the key, reorder, interaction and update kernels differ.
#include "sph_device.h"

namespace sph {

constexpr uint64_t kInf64Bits = 0x7ff0000000000000ull;  // +inf as FP64 bits
constexpr uint32_t kRsrc3 = 0x00020000u;
typedef float v4f __attribute__((ext_vector_type(4)));

GridD grid_d(const sph_ctx *c) {
    GridD g;
    g.ox = c->prm.origin[0];
    g.oy = c->prm.origin[1];
    g.oz = c->prm.origin[2];
    g.cs = 2.0 * c->prm.h;
    g.ncx = c->prm.ncell[0];
    g.ncy = c->prm.ncell[1];
    g.ncz = c->prm.ncell[2];
    return g;
}

__device__ __forceinline__ void reset_variant_reductions(DevInfo *info) {
    info->dtmin_bits = 0x7f800000u;
    info->dtmin64_bits = kInf64Bits;
    info->pairs = 0ull;
}

// positive doubles order like their bits
__device__ __forceinline__ void atomic_min_pos_double(unsigned long long *a, double v) {
    atomicMin(a, (unsigned long long)__double_as_longlong(v));
}

// ------------------------------------------------------------- conversions
__global__ __launch_bounds__(256) void k_cell_from_pos(GridD g, const double *__restrict__ x,
                                                       const double *__restrict__ y,
                                                       const double *__restrict__ z, uint32_t n,
                                                       sph_cstate out) {
#pragma clang fp contract(off)
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t[3] = {(x[i] - g.ox) / g.cs, (y[i] - g.oy) / g.cs, (z[i] - g.oz) / g.cs};
    const int nc[3] = {g.ncx, g.ncy, g.ncz};
    int c[3];
    float o[3];
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (!(t[a] >= 0.0 && t[a] < (double)nc[a])) {
            inside = false;
            c[a] = 0;
            o[a] = 0.0f;
        } else {
            const double f = floor(t[a]);
            c[a] = (int)f;
            o[a] = (float)((t[a] - f - 0.5) * g.cs);
        }
    }
    out.cell[i] = inside ? (c[0] * g.ncy + c[1]) * g.ncz + c[2] : -1;
    out.ox[i] = inside ? o[0] : 0.0f;
    out.oy[i] = inside ? o[1] : 0.0f;
    out.oz[i] = inside ? o[2] : 0.0f;
}

__device__ __forceinline__ void cell_coords(int32_t cell, int32_t ncy, int32_t ncz, int *cx,
                                            int *cy, int *cz) {
    *cz = cell % ncz;
    *cy = (cell / ncz) % ncy;
    *cx = cell / (ncz * ncy);
}

__device__ __forceinline__ void pos_of(const GridD &g, int32_t cell, float ox, float oy, float oz,
                                       double *x, double *y, double *z) {
#pragma clang fp contract(off)
    int cx, cy, cz;
    cell_coords(cell, g.ncy, g.ncz, &cx, &cy, &cz);
    *x = g.ox + ((double)cx + 0.5) * g.cs + (double)ox;
    *y = g.oy + ((double)cy + 0.5) * g.cs + (double)oy;
    *z = g.oz + ((double)cz + 0.5) * g.cs + (double)oz;
}

__global__ __launch_bounds__(256) void k_pos_from_cell(GridD g, sph_cstate st, uint32_t n,
                                                       double *__restrict__ x,
                                                       double *__restrict__ y,
                                                       double *__restrict__ z) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = st.cell[i];
    if (c < 0) {
        x[i] = y[i] = z[i] = __longlong_as_double(0x7ff8000000000000ll);
        return;
    }
    pos_of(g, c, st.ox[i], st.oy[i], st.oz[i], &x[i], &y[i], &z[i]);
}

hipError_t launch_cell_from_pos(sph_ctx *c, const double *x, const double *y, const double *z,
                                const sph_cstate &out, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_from_pos, dim3((n + 255) / 256), dim3(256), 0, s, grid_d(c), x, y, z,
                       n, out);
    return hipGetLastError();
}

hipError_t launch_pos_from_cell(sph_ctx *c, const sph_cstate &st, double *x, double *y,
                                double *z, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pos_from_cell, dim3((n + 255) / 256), dim3(256), 0, s, grid_d(c), st, n,
                       x, y, z);
    return hipGetLastError();
}

// ------------------------------------------------------------ cell path
// Keys straight from the stored cells: label 3 for cell -1; in slab mode the
// halo layers x = 0 and x = ncx-1 are exactly "left of slab_xlo" and "at or
// right of slab_xhi" (the slab faces are cell faces), so non-ghosts there get
// labels 1 and 2.
__global__ __launch_bounds__(256) void k_keys_cell(KParams kp, const int32_t *__restrict__ cell,
                                                   const uint8_t *__restrict__ type, uint32_t n,
                                                   uint32_t *__restrict__ keys,
                                                   int32_t *__restrict__ vals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = cell[i];
    uint32_t key;
    if (c < 0 || (uint32_t)c >= kp.ncells) {
        key = 3u << kp.cell_bits;
    } else {
        uint32_t label = 0;
        if (kp.slab_mode && type[i] != kGhost) {
            const int cx = c / (kp.ncy * kp.ncz);
            label = cx == 0 ? 1u : (cx == kp.ncx - 1 ? 2u : 0u);
        }
        key = (label << kp.cell_bits) | (uint32_t)c;
    }
    keys[i] = key;
    vals[i] = (int32_t)i;
}

hipError_t launch_keys_cell(sph_ctx *c, const sph_cstate &in, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys_cell, dim3((n + 255) / 256), dim3(256), 0, s, c->kp, in.cell,
                       in.type, n, c->keys_a, c->vals_a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_gather_cell(KParams kp, sph_cstate in, sph_cstate out,
                                                     const int32_t *__restrict__ perm, uint32_t n,
                                                     float4 *__restrict__ pos4,
                                                     float4 *__restrict__ vel4,
                                                     DevInfo *__restrict__ info) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) reset_variant_reductions(info);
    if (k >= n) return;
    const uint32_t s = (uint32_t)perm[k];
    const float ox = in.ox[s], oy = in.oy[s], oz = in.oz[s];
    const float vx = in.vx[s], vy = in.vy[s], vz = in.vz[s], rho = in.rho[s];
    out.cell[k] = in.cell[s];
    out.ox[k] = ox; out.oy[k] = oy; out.oz[k] = oz;
    out.vx[k] = vx; out.vy[k] = vy; out.vz[k] = vz;
    out.rho[k] = rho;
    out.vxp[k] = in.vxp[s]; out.vyp[k] = in.vyp[s]; out.vzp[k] = in.vzp[s];
    out.rhop[k] = in.rhop[s];
    out.type[k] = in.type[s];
    out.id[k] = in.id[s];
    pos4[k] = make_float4(ox, oy, oz, tait_p_over_rho2(kp, rho));
    vel4[k] = make_float4(vx, vy, vz, rho);
}

hipError_t launch_gather_cell(sph_ctx *c, const sph_cstate &in, const sph_cstate &out,
                              uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_cell, dim3(n == 0 ? 1 : (n + 255) / 256), dim3(256), 0, s, c->kp,
                       in, out, c->perm, n, c->pos4, c->vel4, c->info);
    return hipGetLastError();
}

// Interaction on cell + offset positions. The structure is that of the plain
// kernel (lane per particle, 9 contiguous z-runs, the candidates of each
// column offset staged in LDS, FP32 support test into 32-bit hit masks in a
// per-lane LDS list, four pairs per step of the compute phase); what
// differs is the separation: r_ij = (o_i + s) - o_j with s = (c_i - c_j) cs,
// the cell difference being the run's (x, y) column offset and, along z,
// which of the run's three cells j lies in (from the run's cell
// boundaries). A list entry is (j << 5 | 3 column, mask) and, beside it, the
// two positions in the mask where the z cell changes (l1: first candidate
// not in cell z - 1, l2: first one in cell z + 1); the compute phase takes
// the shift-table index 3 column + z cell of each drawn candidate from
// them.
constexpr int kCEnt = 15;       // list slots per lane (one for the sentinel)
constexpr int kCUnroll = 8;     // candidates tested per group
constexpr int kCStage = 768;    // staged candidate positions per column offset
constexpr int kCSlack = 3;      // converged flush when a lane cannot take this many more

__global__ __launch_bounds__(kInteractThreads) __attribute__((amdgpu_waves_per_eu(3, 3))) void
k_interact_cell(KParams kp, const float4 *__restrict__ pos4, const float4 *__restrict__ vel4,
                uint32_t n, const uint8_t *__restrict__ type, const uint32_t *__restrict__ sk,
                const uint32_t *__restrict__ cbeg, const uint32_t *__restrict__ cend,
                DevInfo *__restrict__ info, float *__restrict__ oax, float *__restrict__ oay,
                float *__restrict__ oaz, float *__restrict__ orho, float *__restrict__ opress,
                float *__restrict__ onu, uint32_t *__restrict__ onpair) {
    constexpr int kWaves = kInteractThreads / 64;
    __shared__ uint2 s_ent[kCEnt][kInteractThreads];
    __shared__ uint16_t s_zs[kCEnt][kInteractThreads];  // l1 | l2 << 6 of each entry
    __shared__ float4 s_stage[kCStage + kCUnroll];
    __shared__ float4 s_sh[27];  // (x, y, z) shift of tag 3 col + zc
    __shared__ uint32_t s_lo[kWaves], s_hi[kWaves];
    __shared__ double s_rdt[kWaves];
    __shared__ uint32_t s_rnp[kWaves];
    __shared__ uint32_t s_rnc[kWaves];

    const int tid = threadIdx.x;
    const float cs = 2.0f * kp.h;
    if (tid < 27) {
        const int col = tid / 3, zc = tid % 3;
        s_sh[tid] = make_float4((float)(1 - col / 3) * cs, (float)(1 - col % 3) * cs,
                                (float)(1 - zc) * cs, 0.0f);
    }
    const uint32_t n0 = info->n_label[0];
    const uint32_t i =
        layer_block(blockIdx.x, (n0 + kInteractThreads - 1) / kInteractThreads, sk, cbeg, kp) *
            kInteractThreads + tid;
    const bool inrange = i < n0;
    const uint8_t ti = inrange ? type[i] : (uint8_t)kGhost;
    const bool act = ti != kGhost;
    double dtmin = INFINITY;
    uint32_t npair = 0, ncand = 0;

    float4 pi = make_float4(0.f, 0.f, 0.f, 0.f), vi = pi;
    if (inrange) {
        pi = pos4[i];
        vi = vel4[i];
    }
    const float rhoi = vi.w, Pi = pi.w;
    float axs = 0.f, ays = 0.f, azs = 0.f, drho = 0.f, nu = 0.f;
    const __amdgpu_buffer_rsrc_t rp =
        __builtin_amdgcn_make_buffer_rsrc((void *)pos4, 0, (int)(n * 16u), kRsrc3);
    const __amdgpu_buffer_rsrc_t rv =
        __builtin_amdgcn_make_buffer_rsrc((void *)vel4, 0, (int)(n * 16u), kRsrc3);
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
    const float eta2 = kp.eta2;
    // Pi_ij as in the plain kernel: kvis2 (rho_i^2 - rho_i rho_j + rho_j^2) vr / (r^2 + eta^2)
    const float kvis2 = -kp.alpha * kp.h * kp.c0 * kp.inv_rho0 * kp.inv_rho0 * kp.inv_rho0;
    const float rhoi2 = rhoi * rhoi;
    const float zm = pi.z + cs, zp = pi.z - cs;  // i's z relative to the cells z-1, z+1
    const float zabs = pi.z + (float)cz * cs;    // i's z against staged candidates

    auto pair = [&](const v4f pj, const v4f vj, const float4 sh) {
        const float dx = (pi.x + sh.x) - pj.x, dy = (pi.y + sh.y) - pj.y, dz = (pi.z + sh.z) - pj.z;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float t = fmaf(hinv2, __builtin_amdgcn_sqrtf(r2), 1.0f);  // 1 - q/2
        const float F = t * t * t;
        const float ux = vi.x - vj.x, uy = vi.y - vj.y, uz = vi.z - vj.z;
        const float vr = fmaf(uz, dz, fmaf(uy, dy, ux * dx));
        drho = fmaf(F, vr, drho);
        const float vR = vr * __builtin_amdgcn_rcpf(r2 + eta2);
        nu = fmaxf(nu, fabsf(vR));  // |mu| / h
        const float visc = fmaf(vj.w, vj.w - rhoi, rhoi2) * fminf(vR, 0.0f);
        const float f = fmaf(kvis2, visc, Pi + pj.w) * F;
        axs = fmaf(f, dx, axs);
        ays = fmaf(f, dy, ays);
        azs = fmaf(f, dz, azs);
    };

    // compute phase over the cnt entries of the lane's list holding nhit
    // set bits; the sentinel (i in the own cell: column 4, z cell 1 for
    // every position, bit 31) after the last entry stands in for every
    // position past the end (the self pair adds exactly zero)
    auto flush = [&](uint32_t cnt, uint32_t nhit) {
        s_ent[cnt][tid] = make_uint2(i << 5 | 12u, 0x80000000u);
        s_zs[cnt][tid] = (uint16_t)(32u << 6);
        uint32_t pk = 0, cb = 0, ce = 0, cz = 0;
        uint2 nx = s_ent[0][tid];
        uint32_t nz = s_zs[0][tid];
        auto draw = [&](uint32_t (&jj)[4], uint32_t (&tt)[4]) {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const bool empty = cb == 0u;
                cb = empty ? nx.y : cb;
                ce = empty ? nx.x : ce;
                cz = empty ? nz : cz;
                pk = min(pk + (empty ? 1u : 0u), cnt);
                nx = s_ent[pk][tid];
                nz = s_zs[pk][tid];
                const uint32_t off = (uint32_t)__builtin_clz(cb);
                jj[u] = ((ce >> 5) + off) << 4;  // byte offset of j
                tt[u] = (ce & 31u) + (off >= (cz & 63u) ? 1u : 0u) + (off >= (cz >> 6) ? 1u : 0u);
                cb &= 0x7fffffffu >> off;
            }
        };
        uint32_t jn[4], tn[4];
        draw(jn, tn);
        for (uint32_t t = 0; t < nhit; t += 4) {
            v4f qp[4], qv[4];
            float4 sh[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                qp[u] = __builtin_amdgcn_raw_buffer_load_b128(rp, jn[u], 0, 0);
                qv[u] = __builtin_amdgcn_raw_buffer_load_b128(rv, jn[u], 0, 0);
                sh[u] = s_sh[tn[u]];
            }
            draw(jn, tn);
#pragma unroll
            for (int u = 0; u < 4; u++) pair(qp[u], qv[u], sh[u]);
        }
    };

    uint32_t lp = 0, nhit = 0, listed = 0;
    for (int col = 0; col < 9; col++) {
        if (__any(act && lp > (uint32_t)(kCEnt - 1 - kCSlack))) {
            if (act) {
                flush(lp, nhit);
                listed += nhit;
                lp = 0;
                nhit = 0;
            }
        }
        const int X = cx + col / 3 - 1, Y = cy + col % 3 - 1;
        uint32_t jb = 0, je = 0, b1 = 0, b2 = 0;
        if (act && X >= 0 && X < kp.ncx && Y >= 0 && Y < kp.ncy) {
            const uint32_t c0 = ((uint32_t)X * ncy + (uint32_t)Y) * ncz;
            jb = cbeg[c0 + zlo];
            je = cend[c0 + zhi];
            b1 = cbeg[c0 + (uint32_t)cz];
            b2 = (uint32_t)cz + 1 < ncz ? cbeg[c0 + (uint32_t)cz + 1] : je;
        }
        const uint32_t len = je - jb;
        const uint32_t kb1 = min(b1 - jb, len), kb2 = min(b2 - jb, len);
        ncand += len;
        // the block's index range of this column offset, staged in LDS when
        // it fits (as in the plain kernel: jb, je never decrease along the lanes)
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
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kWaves; w++) {
            lo = min(lo, s_lo[w]);
            hi = max(hi, s_hi[w]);
        }
        const bool staged = hi > lo && hi - lo <= (uint32_t)kCStage;
        if (staged) {
            // z of a staged candidate as o_z + c_z cs (its cell's z index
            // from its key): the lanes then test every candidate of a run
            // against one z, o_z,i + c_z,i cs, without choosing the z cell
            // per candidate. Only the support test sees these sums; the pair
            // terms use the offsets and the exact cell shifts.
            for (uint32_t t = tid; t < hi - lo; t += kInteractThreads) {
                float4 q = pos4[lo + t];
                q.z += (float)((sk[lo + t] & kp.cell_mask) % ncz) * cs;
                s_stage[t] = q;
            }
        }
        __syncthreads();
        if (!len) continue;
        const float pix = pi.x + (float)(1 - col / 3) * cs;
        const float piy = pi.y + (float)(1 - col % 3) * cs;
        const uint32_t tag0 = (uint32_t)col * 3u;
        uint32_t bits = 0, k0 = 0;
        // a full or final mask of 32 candidates from c0 is listed with the
        // positions where its z cell changes (candidates below kb1 lie in
        // cell z - 1, below kb2 in cell z, the rest in z + 1); a lane
        // flushes alone when its list is full
        auto put = [&](uint32_t c0, uint32_t b) {
            const uint32_t l1 = kb1 > c0 ? min(kb1 - c0, 32u) : 0u;
            const uint32_t l2 = kb2 > c0 ? min(kb2 - c0, 32u) : 0u;
            s_ent[lp][tid] = make_uint2((jb + c0) << 5 | tag0, b);
            s_zs[lp][tid] = (uint16_t)(l1 | l2 << 6);
            lp += b != 0u ? 1u : 0u;
            nhit += (uint32_t)__builtin_popcount(b);
            if (lp >= (uint32_t)(kCEnt - 1)) {
                flush(lp, nhit);
                listed += nhit;
                lp = 0;
                nhit = 0;
            }
        };
        auto test = [&](const v4f (&q)[kCUnroll], uint32_t k, const bool absz) {
#pragma unroll
            for (int u = 0; u < kCUnroll; u++) {
                const uint32_t kk = k + (uint32_t)u;
                const float ziz = absz ? zabs : (kk < kb1 ? zm : (kk < kb2 ? pi.z : zp));
                const float dx = pix - q[u].x, dy = piy - q[u].y, dz = ziz - q[u].z;
                const float e = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, -kp.r2max)));  // r^2 - 4h^2
                bits = __builtin_amdgcn_alignbit(bits, __float_as_uint(e), 31);
            }
            if ((k & 31u) == 32u - kCUnroll) {
                const uint32_t c0 = k + kCUnroll - 32u;
                const uint32_t v = len - c0;
                put(c0, v >= 32u ? bits : bits & ~(0xffffffffu >> v));
                bits = 0;
            }
        };
        if (staged) {
            const float4 *sp = s_stage + (jb - lo);
            for (; k0 < len; k0 += kCUnroll) {
                v4f q[kCUnroll];
#pragma unroll
                for (int u = 0; u < kCUnroll; u++) {
                    const float4 t = sp[k0 + u];
                    q[u] = v4f{t.x, t.y, t.z, 0.0f};
                }
                test(q, k0, true);
            }
        } else {
            const uint32_t voff = jb * 16u;
            for (; k0 < len; k0 += kCUnroll) {
                v4f q[kCUnroll];
#pragma unroll
                for (int u = 0; u < kCUnroll; u++)
                    q[u] = __builtin_amdgcn_raw_buffer_load_b128(rp, voff, (int)(k0 * 16u + 16u * u), 0);
                test(q, k0, false);
            }
        }
        const uint32_t tail = k0 & 31u;
        if (tail) {
            const uint32_t c0 = k0 - tail;
            const uint32_t v = len - c0;
            put(c0, (bits << (32u - tail)) & ~(0xffffffffu >> v));
        }
    }
    if (act) {
        flush(lp, nhit);
        npair = listed + nhit - 1u;  // minus the self entry
        nu *= kp.h;
    }
    if (inrange) {
        const float mk = kp.mass * kp.kgrad;
        float ax = 0.f, ay = 0.f, az = 0.f, ar = 0.f;
        if (ti == kFluid) {
            ax = fmaf(-mk, axs, kp.gx);
            ay = fmaf(-mk, ays, kp.gy);
            az = fmaf(-mk, azs, kp.gz);
        }
        if (ti != kGhost) {
            ar = mk * drho;
            // CFL limits (Sec. 3.3) in FP64
            const double s = (double)rhoi / (double)kp.rho0;
            const double c = (double)kp.c0 * s * s * s;
            dtmin = (double)kp.h / (c + (double)nu);
            if (ti == kFluid) {
                const double a2 = (double)ax * ax + (double)ay * ay + (double)az * az;
                if (a2 > 0.0) dtmin = fmin(dtmin, sqrt((double)kp.h / sqrt(a2)));
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
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        dtmin = fmin(dtmin, __shfl_xor(dtmin, o, 64));
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
        double d = s_rdt[0];
        uint32_t np = s_rnp[0], nc = s_rnc[0];
        for (int k = 1; k < kWaves; k++) {
            d = fmin(d, s_rdt[k]);
            np += s_rnp[k];
            nc += s_rnc[k];
        }
        if (d < INFINITY) atomic_min_pos_double(&info->dtmin64_bits, d);
        if (np) {
            atomicAdd(&info->pairs, (unsigned long long)np);
            atomicAdd(&info->pairs_total, (unsigned long long)np);
        }
        if (nc) atomicAdd(&info->cand_total, (unsigned long long)nc);
    }
}

hipError_t launch_interact_cell(sph_ctx *c, const sph_cstate &st, uint32_t n,
                                const sph_rates &out, hipStream_t s) {
    const uint32_t nb = n == 0 ? 1 : (n + kInteractThreads - 1) / kInteractThreads;
    hipLaunchKernelGGL(k_interact_cell, dim3(nb), dim3(kInteractThreads), 0, s, c->kp, c->pos4,
                       c->vel4, n, st.type, c->keys_sorted, c->cell_begin, c->cell_end, c->info,
                       out.ax, out.ay, out.az, out.arho, out.press, out.nu, out.npair);
    return hipGetLastError();
}

// Verlet update on cell + offset positions (same scheme as the plain path);
// dt = (float)(CFL * FP64 minimum). After the move an offset outside [-h, h)
// hands the particle to the neighbouring cell (offset -/+ cs, exact in FP32
// for |offset| < 3h); leaving the grid gives cell -1.
__global__ __launch_bounds__(256) void k_verlet_cell(KParams kp, sph_cstate st,
                                                     const float *__restrict__ ax,
                                                     const float *__restrict__ ay,
                                                     const float *__restrict__ az,
                                                     const float *__restrict__ arho,
                                                     DevInfo *__restrict__ info, int euler) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const double dt64 = (double)kp.cfl * __longlong_as_double((long long)info->dtmin64_bits);
    const float dt = (float)dt64;
    if (k == 0) {
        info->dt = dt;
        if (!(dt > 0.0f) || !(dt < INFINITY)) atomicOr(&info->flags, (uint32_t)SPH_S_DT);
    }
    if (k >= info->n_label[0]) return;
    const uint8_t t = st.type[k];
    if (t == kGhost) return;
    const float rho = st.rho[k];
    const float rn = euler ? fmaf(dt, arho[k], rho) : fmaf(2.0f * dt, arho[k], st.rhop[k]);
    st.rhop[k] = rho;
    st.rho[k] = rn;
    bool ok = isfinite(rn);
    if (t == kFluid) {
        const float cs = 2.0f * kp.h, hh = kp.h;
        const float a[3] = {ax[k], ay[k], az[k]};
        float *off[3] = {st.ox, st.oy, st.oz};
        float *vel[3] = {st.vx, st.vy, st.vz};
        float *velp[3] = {st.vxp, st.vyp, st.vzp};
        const float hdt2 = 0.5f * dt * dt;
        int32_t cell = st.cell[k];
        int cc[3];
        cell_coords(cell, kp.ncy, kp.ncz, &cc[0], &cc[1], &cc[2]);
        const int nc[3] = {kp.ncx, kp.ncy, kp.ncz};
        bool inside = cell >= 0;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const float v = vel[d][k];
            const float vn = euler ? fmaf(dt, a[d], v) : fmaf(2.0f * dt, a[d], velp[d][k]);
            float o = off[d][k] + fmaf(hdt2, a[d], dt * v);
            for (int it = 0; it < 4 && o >= hh; it++) { o -= cs; cc[d]++; }
            for (int it = 0; it < 4 && o < -hh; it++) { o += cs; cc[d]--; }
            ok = ok && isfinite(vn) && isfinite(o) && o >= -hh && o < hh;
            off[d][k] = o;
            velp[d][k] = v;
            vel[d][k] = vn;
            inside = inside && cc[d] >= 0 && cc[d] < nc[d];
        }
        st.cell[k] = inside ? (cc[0] * kp.ncy + cc[1]) * kp.ncz + cc[2] : -1;
    }
    if (!ok) atomicOr(&info->flags, (uint32_t)SPH_S_NONFINITE);
}

hipError_t launch_update_cell(sph_ctx *c, const sph_cstate &st, const float *ax, const float *ay,
                              const float *az, const float *arho, uint32_t n, uint64_t step,
                              hipStream_t s) {
    const int E = c->kp.euler_every;
    const int euler = E > 0 ? (step % (uint64_t)E == 0) : (step == 0);
    hipLaunchKernelGGL(k_verlet_cell, dim3(n == 0 ? 1 : (n + 255) / 256), dim3(256), 0, s, c->kp,
                       st, ax, ay, az, arho, c->info, euler);
    return hipGetLastError();
}

// ----------------------------------------------------------- FP64 totals
// Per-particle: mass, momentum, kinetic energy, potential energy -m g.r and
// internal energy m e(rho), e = B[(s^6 - 1)/(6 rho0) + 1/rho - 1/rho0],
// s = rho/rho0 (gamma = 7); block sums in a fixed tree order, then one block
// adds the block sums in index order: the totals are reproducible.
struct TotParams {
    GridD g;
    double mass, B, rho0, gx, gy, gz;
};

__device__ __forceinline__ void add_particle(const TotParams &tp, double x, double y, double z,
                                             double vx, double vy, double vz, double rho,
                                             double acc[8]) {
    const double m = tp.mass;
    const double s = rho / tp.rho0;
    const double s2 = s * s, s6 = s2 * s2 * s2;
    const double e = tp.B * ((s6 - 1.0) / (6.0 * tp.rho0) + (1.0 / rho - 1.0 / tp.rho0));
    acc[0] += m;
    acc[1] += m * vx;
    acc[2] += m * vy;
    acc[3] += m * vz;
    acc[4] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
    acc[5] += -m * (tp.gx * x + tp.gy * y + tp.gz * z);
    acc[6] += m * e;
    acc[7] += 1.0;
}

__device__ __forceinline__ void block_sum8(double acc[8], double *part) {
    __shared__ double s_acc[kTotThreads][8];
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 8; q++) s_acc[tid][q] = acc[q];
    __syncthreads();
    for (int w = kTotThreads / 2; w > 0; w >>= 1) {
        if (tid < w)
#pragma unroll
            for (int q = 0; q < 8; q++) s_acc[tid][q] += s_acc[tid + w][q];
        __syncthreads();
    }
    if (tid < 8) part[blockIdx.x * 8 + tid] = s_acc[0][tid];
}

__global__ __launch_bounds__(kTotThreads) void k_totals_cell(TotParams tp, sph_cstate st,
                                                             uint32_t n,
                                                             double *__restrict__ part) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t k = blockIdx.x * kTotThreads + threadIdx.x; k < n; k += gridDim.x * kTotThreads) {
        const int32_t c = st.cell[k];
        if (c < 0 || st.type[k] == kGhost) continue;
        double x, y, z;
        pos_of(tp.g, c, st.ox[k], st.oy[k], st.oz[k], &x, &y, &z);
        add_particle(tp, x, y, z, st.vx[k], st.vy[k], st.vz[k], st.rho[k], acc);
    }
    block_sum8(acc, part);
}

__global__ __launch_bounds__(kTotThreads) void k_totals_d(TotParams tp, sph_dstate st, uint32_t n,
                                                          double *__restrict__ part) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t k = blockIdx.x * kTotThreads + threadIdx.x; k < n; k += gridDim.x * kTotThreads) {
        if (st.type[k] == kGhost || !(st.x[k] == st.x[k])) continue;
        add_particle(tp, st.x[k], st.y[k], st.z[k], st.vx[k], st.vy[k], st.vz[k], st.rho[k], acc);
    }
    block_sum8(acc, part);
}

__global__ __launch_bounds__(kTotThreads) void k_totals_final(const double *__restrict__ part,
                                                              uint32_t nb,
                                                              double *__restrict__ out) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t b = threadIdx.x; b < nb; b += kTotThreads)
#pragma unroll
        for (int q = 0; q < 8; q++) acc[q] += part[b * 8 + q];
    block_sum8(acc, out);  // gridDim.x == 1: writes out[0..7]
}

static TotParams tot_params(const sph_ctx *c) {
    TotParams tp;
    tp.g = grid_d(c);
    tp.mass = c->prm.mass;
    tp.B = c->prm.c0 * c->prm.c0 * c->prm.rho0 / c->prm.gamma;
    tp.rho0 = c->prm.rho0;
    tp.gx = c->prm.g[0];
    tp.gy = c->prm.g[1];
    tp.gz = c->prm.g[2];
    return tp;
}

static hipError_t finish_totals(sph_ctx *c, double *out_host, hipStream_t s) {
    double *res = c->tot_part + 8 * c->tot_blocks;
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(kTotThreads), 0, s, c->tot_part,
                       c->tot_blocks, res);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, res, 8 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

hipError_t launch_totals_cell(sph_ctx *c, const sph_cstate &st, uint32_t n, double *out_host,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_totals_cell, dim3(c->tot_blocks), dim3(kTotThreads), 0, s, tot_params(c),
                       st, n, c->tot_part);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? finish_totals(c, out_host, s) : e;
}

hipError_t launch_totals_d(sph_ctx *c, const sph_dstate &st, uint32_t n, double *out_host,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_totals_d, dim3(c->tot_blocks), dim3(kTotThreads), 0, s, tot_params(c), st,
                       n, c->tot_part);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? finish_totals(c, out_host, s) : e;
}

// ------------------------------------------------------------ FP64 path
__global__ __launch_bounds__(256) void k_keys_d(KParams kp, const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                const double *__restrict__ z,
                                                const uint8_t *__restrict__ type, uint32_t n,
                                                uint32_t *__restrict__ keys,
                                                int32_t *__restrict__ vals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = cell_key(kp, (float)x[i], (float)y[i], (float)z[i], type[i]);
    vals[i] = (int32_t)i;
}

hipError_t launch_keys_d(sph_ctx *c, const sph_dstate &in, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys_d, dim3((n + 255) / 256), dim3(256), 0, s, c->kp, in.x, in.y, in.z,
                       in.type, n, c->keys_a, c->vals_a);
    return hipGetLastError();
}

struct DParams {
    double h, r2max, eta2, mass, alpha, rho0, B, c0, gx, gy, gz, kgrad, cfl;
};

static DParams dparams(const sph_ctx *c) {
    const sph_params &p = c->prm;
    DParams d;
    d.h = p.h;
    d.r2max = 4.0 * p.h * p.h;
    const double eta = p.eta_over_h * p.h;
    d.eta2 = eta * eta;
    d.mass = p.mass;
    d.alpha = p.alpha;
    d.rho0 = p.rho0;
    d.B = p.c0 * p.c0 * p.rho0 / p.gamma;
    d.c0 = p.c0;
    d.gx = p.g[0];
    d.gy = p.g[1];
    d.gz = p.g[2];
    d.kgrad = -5.0 * (21.0 / (16.0 * M_PI * p.h * p.h * p.h)) / (p.h * p.h);
    d.cfl = p.cfl;
    return d;
}

__device__ __forceinline__ double tait_p64(const DParams &d, double rho) {
    const double s = rho / d.rho0, e = (rho - d.rho0) / d.rho0;
    double q = s + 1.0;
    for (int k = 0; k < 5; k++) q = q * s + 1.0;  // 1 + s + ... + s^6
    return d.B * e * q;
}

__global__ __launch_bounds__(256) void k_gather_d(DParams dp, sph_dstate in, sph_dstate out,
                                                  const int32_t *__restrict__ perm, uint32_t n,
                                                  double4 *__restrict__ pos8,
                                                  double4 *__restrict__ vel8,
                                                  DevInfo *__restrict__ info) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) reset_variant_reductions(info);
    if (k >= n) return;
    const uint32_t s = (uint32_t)perm[k];
    const double rho = in.rho[s];
    const double x = in.x[s], y = in.y[s], z = in.z[s];
    const double vx = in.vx[s], vy = in.vy[s], vz = in.vz[s];
    out.x[k] = x; out.y[k] = y; out.z[k] = z;
    out.vx[k] = vx; out.vy[k] = vy; out.vz[k] = vz;
    out.rho[k] = rho;
    out.vxp[k] = in.vxp[s]; out.vyp[k] = in.vyp[s]; out.vzp[k] = in.vzp[s];
    out.rhop[k] = in.rhop[s];
    out.type[k] = in.type[s];
    out.id[k] = in.id[s];
    // the interaction's packed inputs: (x, y, z, p / rho^2), (v, rho)
    pos8[k] = make_double4(x, y, z, tait_p64(dp, rho) / (rho * rho));
    vel8[k] = make_double4(vx, vy, vz, rho);
}

hipError_t launch_gather_d(sph_ctx *c, const sph_dstate &in, const sph_dstate &out, uint32_t n,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_gather_d, dim3(n == 0 ? 1 : (n + 255) / 256), dim3(256), 0, s, dparams(c),
                       in, out, c->perm, n, c->pos8, c->vel8, c->info);
    return hipGetLastError();
}

// Interaction in FP64 (the reference path): the pair terms of Sec. 2.2
// written as plainly as the oracle's, with the search of the FP32 kernels:
// lane per particle, the 9 contiguous z-runs, the candidates of each column
// offset staged in LDS, the FP64 support test |r_ij|^2 < 4h^2 into 32-bit hit
// masks in a per-lane LDS list, then the pair terms for the hits only. Pairs
// are summed in the order of a direct loop over the runs (the list keeps it);
// the particle itself is in the list and adds exactly zero.
constexpr int kDEnt = 19;     // list slots per lane (one for the sentinel)
constexpr int kDSlack = 3;    // converged flush when a lane cannot take this many more
constexpr int kDUnroll = 8;   // candidates tested per group
constexpr int kDStage = 512;  // staged candidate positions per column offset
struct DPos {
    double x, y, z;
};

__global__ __launch_bounds__(kInteractThreads) __attribute__((amdgpu_waves_per_eu(3, 3))) void
k_interact_d(DParams dp, KParams kp, const double4 *__restrict__ pos8,
             const double4 *__restrict__ vel8, const uint8_t *__restrict__ type,
             const uint32_t *__restrict__ sk, const uint32_t *__restrict__ cbeg,
             const uint32_t *__restrict__ cend, DevInfo *__restrict__ info, sph_drates out) {
    constexpr int kWaves = kInteractThreads / 64;
    __shared__ uint2 s_ent[kDEnt][kInteractThreads];  // (j, mask with the first candidate in bit 31)
    __shared__ DPos s_stage[kDStage + kDUnroll];
    __shared__ uint32_t s_lo[kWaves], s_hi[kWaves];
    __shared__ double s_rdt[kWaves];
    __shared__ uint32_t s_rnp[kWaves];

    const int tid = threadIdx.x;
    const uint32_t n0 = info->n_label[0];
    const uint32_t i =
        layer_block(blockIdx.x, (n0 + kInteractThreads - 1) / kInteractThreads, sk, cbeg, kp) *
            kInteractThreads + tid;
    const bool inrange = i < n0;
    const uint8_t ti = inrange ? type[i] : (uint8_t)kGhost;
    const bool act = ti != kGhost;
    double dtmin = INFINITY;
    uint32_t npair = 0;

    double4 pi = make_double4(0.0, 0.0, 0.0, 0.0), vi = pi;
    if (inrange) {
        pi = pos8[i];
        vi = vel8[i];
    }
    const double rhoi = vi.w, Pi = pi.w;
    const double ci = dp.c0 * (rhoi / dp.rho0) * (rhoi / dp.rho0) * (rhoi / dp.rho0);
    double axs = 0.0, ays = 0.0, azs = 0.0, drho = 0.0, nu = 0.0;
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

    auto pair = [&](const double4 pj, const double4 vj) {
        const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double rhoj = vj.w;
        const double t = 1.0 - 0.5 * sqrt(r2) / dp.h;
        const double F = t * t * t;
        const double ux = vi.x - vj.x, uy = vi.y - vj.y, uz = vi.z - vj.z;
        const double vr = ux * dx + uy * dy + uz * dz;
        drho += F * vr;
        const double mu = dp.h * vr / (r2 + dp.eta2);
        nu = fmax(nu, fabs(mu));
        const double sj = rhoj / dp.rho0;
        const double cj = dp.c0 * sj * sj * sj;
        const double pv = -dp.alpha * 0.5 * (ci + cj) * mu / (0.5 * (rhoi + rhoj));
        const double visc = vr < 0.0 ? pv : 0.0;
        const double f = (Pi + pj.w + visc) * F;
        axs += f * dx;
        ays += f * dy;
        azs += f * dz;
    };

    // compute phase over the cnt entries of the lane's list holding nhit set
    // bits; the sentinel (i, bit 31) after the last entry stands in for every
    // position past the end
    auto flush = [&](uint32_t cnt, uint32_t nhit) {
        s_ent[cnt][tid] = make_uint2(i, 0x80000000u);
        uint32_t pk = 0, cb = 0, cj = 0;
        uint2 nx = s_ent[0][tid];
        auto draw = [&](uint32_t (&jj)[2]) {
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const bool empty = cb == 0u;
                cb = empty ? nx.y : cb;
                cj = empty ? nx.x : cj;
                pk = min(pk + (empty ? 1u : 0u), cnt);
                nx = s_ent[pk][tid];
                const uint32_t off = (uint32_t)__builtin_clz(cb);
                jj[u] = cj + off;
                cb &= 0x7fffffffu >> off;
            }
        };
        uint32_t jn[2];
        draw(jn);
        for (uint32_t t = 0; t < nhit; t += 2) {
            double4 qp[2], qv[2];
#pragma unroll
            for (int u = 0; u < 2; u++) {
                qp[u] = pos8[jn[u]];
                qv[u] = vel8[jn[u]];
            }
            draw(jn);
#pragma unroll
            for (int u = 0; u < 2; u++) pair(qp[u], qv[u]);
        }
    };

    uint32_t lp = 0, nhit = 0, listed = 0;
    auto put = [&](uint32_t j0, uint32_t b) {
        s_ent[lp][tid] = make_uint2(j0, b);
        lp += b != 0u ? 1u : 0u;
        nhit += (uint32_t)__builtin_popcount(b);
        if (lp >= (uint32_t)(kDEnt - 1)) {  // full: this lane alone
            flush(lp, nhit);
            listed += nhit;
            lp = 0;
            nhit = 0;
        }
    };
    for (int col = 0; col < 9; col++) {
        if (__any(act && lp > (uint32_t)(kDEnt - 1 - kDSlack))) {
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
        // the block's index range of this column offset (jb, je never
        // decrease along the lanes), staged when it fits
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
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kWaves; w++) {
            lo = min(lo, s_lo[w]);
            hi = max(hi, s_hi[w]);
        }
        const bool staged = hi > lo && hi - lo <= (uint32_t)kDStage;
        if (staged) {
            for (uint32_t t = tid; t < hi - lo; t += kInteractThreads) {
                const double4 q = pos8[lo + t];
                s_stage[t] = DPos{q.x, q.y, q.z};
            }
        }
        __syncthreads();
        if (!len) continue;
        uint32_t bits = 0, k0 = 0;
        auto test = [&](const DPos (&q)[kDUnroll], uint32_t k) {
#pragma unroll
            for (int u = 0; u < kDUnroll; u++) {
                const double dx = pi.x - q[u].x, dy = pi.y - q[u].y, dz = pi.z - q[u].z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                // bits = bits << 1 | (r2 < 4h^2): the sign of the difference
                const double e = r2 - dp.r2max;
                bits = __builtin_amdgcn_alignbit(bits, (uint32_t)(__double_as_longlong(e) >> 32), 31);
            }
            if ((k & 31u) == 32u - kDUnroll) {
                const uint32_t c0 = k + kDUnroll - 32u;
                const uint32_t v = len - c0;
                put(jb + c0, v >= 32u ? bits : bits & ~(0xffffffffu >> v));
                bits = 0;
            }
        };
        if (staged) {
            const DPos *sp = s_stage + (jb - lo);
            for (; k0 < len; k0 += kDUnroll) {
                DPos q[kDUnroll];
#pragma unroll
                for (int u = 0; u < kDUnroll; u++) q[u] = sp[k0 + u];
                test(q, k0);
            }
        } else {  // a range too wide to stage: loads clamped to the run
            for (; k0 < len; k0 += kDUnroll) {
                DPos q[kDUnroll];
#pragma unroll
                for (int u = 0; u < kDUnroll; u++) {
                    const uint32_t kk = k0 + (uint32_t)u;
                    const double4 t = pos8[jb + (kk < len ? kk : len - 1u)];
                    q[u] = DPos{t.x, t.y, t.z};
                }
                test(q, k0);
            }
        }
        const uint32_t tail = k0 & 31u;
        if (tail) {
            const uint32_t c0 = k0 - tail;
            const uint32_t v = len - c0;
            put(jb + c0, (bits << (32u - tail)) & ~(0xffffffffu >> v));
        }
    }
    if (act) {
        flush(lp, nhit);
        npair = listed + nhit - 1u;  // minus the self entry
    }
    if (inrange) {
        const double mk = dp.mass * dp.kgrad;
        double ax = 0, ay = 0, az = 0, ar = 0;
        if (ti == kFluid) {
            ax = -mk * axs + dp.gx;
            ay = -mk * ays + dp.gy;
            az = -mk * azs + dp.gz;
        }
        if (ti != kGhost) {
            ar = mk * drho;
            dtmin = dp.h / (ci + nu);
            if (ti == kFluid) {
                const double amag = sqrt(ax * ax + ay * ay + az * az);
                if (amag > 0.0) dtmin = fmin(dtmin, sqrt(dp.h / amag));
            }
        }
        out.ax[i] = ax;
        out.ay[i] = ay;
        out.az[i] = az;
        out.arho[i] = ar;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        dtmin = fmin(dtmin, __shfl_xor(dtmin, o, 64));
        npair += __shfl_xor(npair, o, 64);
    }
    if ((tid & 63) == 0) {
        s_rdt[tid >> 6] = dtmin;
        s_rnp[tid >> 6] = npair;
    }
    __syncthreads();
    if (tid == 0) {
        double d = s_rdt[0];
        uint32_t np = s_rnp[0];
        for (int k = 1; k < kWaves; k++) {
            d = fmin(d, s_rdt[k]);
            np += s_rnp[k];
        }
        if (d < INFINITY) atomic_min_pos_double(&info->dtmin64_bits, d);
        if (np) {
            atomicAdd(&info->pairs, (unsigned long long)np);
            atomicAdd(&info->pairs_total, (unsigned long long)np);
        }
    }
}

hipError_t launch_interact_d(sph_ctx *c, const sph_dstate &st, uint32_t n, const sph_drates &out,
                             hipStream_t s) {
    const uint32_t nb = n == 0 ? 1 : (n + kInteractThreads - 1) / kInteractThreads;
    hipLaunchKernelGGL(k_interact_d, dim3(nb), dim3(kInteractThreads), 0, s, dparams(c), c->kp,
                       c->pos8, c->vel8, st.type, c->keys_sorted, c->cell_begin, c->cell_end,
                       c->info, out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_verlet_d(DParams dp, sph_dstate st, sph_drates r,
                                                  DevInfo *__restrict__ info, int euler) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const double dt = dp.cfl * __longlong_as_double((long long)info->dtmin64_bits);
    if (k == 0) {
        info->dt = (float)dt;
        if (!(dt > 0.0) || !(dt < INFINITY)) atomicOr(&info->flags, (uint32_t)SPH_S_DT);
    }
    if (k >= info->n_label[0]) return;
    const uint8_t t = st.type[k];
    if (t == kGhost) return;
    const double rho = st.rho[k];
    const double rn = euler ? rho + dt * r.arho[k] : st.rhop[k] + 2.0 * dt * r.arho[k];
    st.rhop[k] = rho;
    st.rho[k] = rn;
    bool ok = isfinite(rn);
    if (t == kFluid) {
        const double a[3] = {r.ax[k], r.ay[k], r.az[k]};
        double *pos[3] = {st.x, st.y, st.z};
        double *vel[3] = {st.vx, st.vy, st.vz};
        double *velp[3] = {st.vxp, st.vyp, st.vzp};
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const double v = vel[d][k];
            const double vn = euler ? v + dt * a[d] : velp[d][k] + 2.0 * dt * a[d];
            pos[d][k] += dt * v + 0.5 * dt * dt * a[d];
            velp[d][k] = v;
            vel[d][k] = vn;
            ok = ok && isfinite(vn) && isfinite(pos[d][k]);
        }
    }
    if (!ok) atomicOr(&info->flags, (uint32_t)SPH_S_NONFINITE);
}

hipError_t launch_update_d(sph_ctx *c, const sph_dstate &st, const sph_drates &r, uint32_t n,
                           uint64_t step, hipStream_t s) {
    const int E = c->kp.euler_every;
    const int euler = E > 0 ? (step % (uint64_t)E == 0) : (step == 0);
    hipLaunchKernelGGL(k_verlet_d, dim3(n == 0 ? 1 : (n + 255) / 256), dim3(256), 0, s, dparams(c),
                       st, r, c->info, euler);
    return hipGetLastError();
}

}  // namespace sph
