// Sort step of the WCSPH time step: cell keys with migration labels, stable
// LSD radix sort, reorder of the particle arrays, cell tables and packing
// ranges (Sec. 3.1 neighbour search; Sec. 4.2-4.3 migration and halo packing).
#include "sph_device.h"

namespace sph {

// ------------------------------------------------------------------ keys
// One thread per particle (Sec. 3.1). Cell coordinates in FP32:
// c = floor((x - o) * (1/cs)); a coordinate outside [0, ncell) on any axis
// gives label 3 (outside the grid). In slab mode a non-ghost particle left of
// slab_xlo gets label 1 and one at or right of slab_xhi label 2 (Sec. 4.3).
__global__ __launch_bounds__(256) void k_keys(KParams kp, const float *__restrict__ x,
                                              const float *__restrict__ y,
                                              const float *__restrict__ z,
                                              const uint8_t *__restrict__ type, uint32_t n,
                                              uint32_t *__restrict__ keys,
                                              int32_t *__restrict__ vals) {
#pragma clang fp contract(off)
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float px = x[i], py = y[i], pz = z[i];
    const float tx = (px - kp.ox) * kp.inv_cs;
    const float ty = (py - kp.oy) * kp.inv_cs;
    const float tz = (pz - kp.oz) * kp.inv_cs;
    const bool inside = (tx >= 0.0f && tx < (float)kp.ncx) && (ty >= 0.0f && ty < (float)kp.ncy) &&
                        (tz >= 0.0f && tz < (float)kp.ncz);
    uint32_t key;
    if (!inside) {
        key = 3u << kp.cell_bits;
    } else {
        const uint32_t cx = (uint32_t)(int)floorf(tx), cy = (uint32_t)(int)floorf(ty),
                       cz = (uint32_t)(int)floorf(tz);
        const uint32_t cell = (cx * (uint32_t)kp.ncy + cy) * (uint32_t)kp.ncz + cz;
        uint32_t label = 0;
        if (kp.slab_mode && type[i] != kGhost) label = px < kp.slab_xlo ? 1u : (px >= kp.slab_xhi ? 2u : 0u);
        key = (label << kp.cell_bits) | cell;
    }
    keys[i] = key;
    vals[i] = (int32_t)i;
}

hipError_t launch_keys(const KParams &kp, const sph_soa &in, uint32_t n, uint32_t *keys,
                       int32_t *vals, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys, dim3((n + 255) / 256), dim3(256), 0, s, kp, in.x, in.y, in.z,
                       in.type, n, keys, vals);
    return hipGetLastError();
}

// ------------------------------------------------------------ radix sort
// LSD radix sort with 8-bit digits, three kernels per digit:
//   hist:    per-tile digit counts, stored digit-major (hist[d * ntiles + t]);
//   scan:    per digit, exclusive scan over tiles, and the digit total;
//   scatter: per tile, a stable rank of each key among the tile's keys with
//            the same digit (wave ballots over the 8 digit bits give the
//            lanes holding the same digit), a reorder through LDS by digit,
//            and coalesced runs written to their global positions.
// Stability: keys are ranked in input order (round, wave, lane), so equal
// keys keep their relative order in every pass.

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                             uint32_t n, int shift,
                                                             uint32_t ntiles,
                                                             uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * (uint32_t)kSortTile;
#pragma unroll 4
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t idx = base + r * kSortThreads + tid;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint32_t)tid * ntiles + blockIdx.x] = h[tid];
}

__global__ __launch_bounds__(256) void k_radix_scan(uint32_t *__restrict__ hist, uint32_t ntiles,
                                                    uint32_t *__restrict__ tot) {
    __shared__ uint32_t s_w[4];
    uint32_t *row = hist + (size_t)blockIdx.x * ntiles;
    const int tid = threadIdx.x;
    uint32_t running = 0;
    for (uint32_t start = 0; start < ntiles; start += 256 * 4) {
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint32_t idx = start + tid * 4 + k;
            v[k] = idx < ntiles ? row[idx] : 0u;
            sum += v[k];
        }
        uint32_t total;
        uint32_t pre = block_excl_scan<256>(sum, s_w, &total) + running;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint32_t idx = start + tid * 4 + k;
            if (idx < ntiles) row[idx] = pre;
            pre += v[k];
        }
        running += total;
    }
    if (tid == 0) tot[blockIdx.x] = running;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    int32_t *__restrict__ vout, uint32_t n, int shift, uint32_t ntiles,
    const uint32_t *__restrict__ hist, const uint32_t *__restrict__ tot) {
    __shared__ uint32_t s_k[kSortTile];
    __shared__ int32_t s_v[kSortTile];
    __shared__ uint32_t s_cnt[kSortThreads / 64][256];
    __shared__ uint32_t s_run[256];
    __shared__ uint32_t s_off[256];
    __shared__ uint32_t s_glob[256];
    __shared__ uint32_t s_w[kSortThreads / 64];
    constexpr int NW = kSortThreads / 64;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t tile = blockIdx.x;
    const uint32_t base = tile * (uint32_t)kSortTile;

    // global start of each digit's run for this tile
    const uint32_t gbase = block_excl_scan<kSortThreads>(tot[tid], s_w);
    s_glob[tid] = gbase + hist[(uint32_t)tid * ntiles + tile];
    s_run[tid] = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) s_cnt[k][tid] = 0;
    __syncthreads();

    const unsigned long long lt = (1ull << lane) - 1ull;
    uint32_t key[kSortItems];
    int32_t val[kSortItems];
    uint32_t rank[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t idx = base + r * kSortThreads + tid;
        const bool valid = idx < n;
        key[r] = valid ? kin[idx] : 0xffffffffu;
        val[r] = valid ? vin[idx] : 0;
        const uint32_t d = (key[r] >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t wr = (uint32_t)__popcll(peers & lt);
        if (valid && wr == 0) s_cnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        uint32_t pre = s_run[d];
#pragma unroll
        for (int k = 0; k < NW; k++)
            if (k < w) pre += s_cnt[k][d];
        rank[r] = pre + wr;
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int k = 0; k < NW; k++) {
            add += s_cnt[k][tid];
            s_cnt[k][tid] = 0;
        }
        s_run[tid] += add;
        __syncthreads();
    }
    s_off[tid] = block_excl_scan<kSortThreads>(s_run[tid], s_w);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t idx = base + r * kSortThreads + tid;
        if (idx < n) {
            const uint32_t d = (key[r] >> shift) & 255u;
            const uint32_t pos = s_off[d] + rank[r];
            s_k[pos] = key[r];
            s_v[pos] = val[r];
        }
    }
    __syncthreads();
    const uint32_t tile_n = (n - base) < (uint32_t)kSortTile ? (n - base) : (uint32_t)kSortTile;
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t idx = r * kSortThreads + tid;
        if (idx < tile_n) {
            const uint32_t k = s_k[idx];
            const uint32_t d = (k >> shift) & 255u;
            const uint32_t o = s_glob[d] + (idx - s_off[d]);
            kout[o] = k;
            vout[o] = s_v[idx];
        }
    }
}

hipError_t radix_sort(sph_ctx *c, const uint32_t *keys_in, const int32_t *vals_in,
                      uint32_t *keys_out, int32_t *vals_out, uint32_t n, int key_bits,
                      hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int passes = (key_bits + 7) / 8;
    const uint32_t ntiles = (n + kSortTile - 1) / kSortTile;
    const uint32_t *ksrc = keys_in;
    const int32_t *vsrc = vals_in;
    for (int p = 0; p < passes; p++) {
        uint32_t *kdst;
        int32_t *vdst;
        if (p == passes - 1) {
            kdst = keys_out;
            vdst = vals_out;
        } else {
            // ping-pong between two scratch buffers, never onto the source
            kdst = (ksrc == c->keys_a) ? c->keys_b : c->keys_a;
            vdst = (vsrc == c->vals_a) ? c->vals_b : c->vals_a;
        }
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kSortThreads), 0, s, ksrc, n, shift,
                           ntiles, c->hist);
        hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(256), 0, s, c->hist, ntiles,
                           c->digit_tot);
        hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kSortThreads), 0, s, ksrc, vsrc,
                           kdst, vdst, n, shift, ntiles, c->hist, c->digit_tot);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        ksrc = kdst;
        vsrc = vdst;
    }
    return hipSuccess;
}

// ---------------------------------------------------- counts and ranges
__device__ __forceinline__ uint32_t lower_bound_dev(const uint32_t *a, uint32_t n, uint32_t v) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Label counts from the label boundaries of the sorted keys, and the packing
// ranges: x-layers 0, 1, ncx-2, ncx-1 of the x-major cell order are each one
// contiguous range of the label-0 prefix (Sec. 4.2-4.3).
__global__ void k_counts(KParams kp, const uint32_t *__restrict__ sk, uint32_t n,
                         DevInfo *__restrict__ info) {
    __shared__ uint32_t st[5];
    const int t = threadIdx.x;
    if (t < 4) st[t] = t == 0 ? 0u : lower_bound_dev(sk, n, (uint32_t)t << kp.cell_bits);
    if (t == 4) st[4] = n;
    __syncthreads();
    const uint32_t n0 = st[1];
    if (t < 4) info->n_label[t] = st[t + 1] - st[t];
    if (t < 8) {
        const uint32_t L = (uint32_t)kp.ncy * (uint32_t)kp.ncz;
        int lay;
        switch (t >> 1) {
            case 0: lay = 0; break;
            case 1: lay = 1; break;
            case 2: lay = kp.ncx - 2; break;
            default: lay = kp.ncx - 1; break;
        }
        lay = lay < 0 ? 0 : (lay >= kp.ncx ? kp.ncx - 1 : lay);
        const uint32_t bound = (uint32_t)(lay + (t & 1)) * L;
        info->ranges[t] = lower_bound_dev(sk, n0, bound);
    }
    if (t == 8) {
        info->ranges[8] = st[1];
        info->ranges[9] = st[2];
        info->ranges[10] = st[2];
        info->ranges[11] = st[3];
        info->ranges[12] = st[3];
        info->ranges[13] = st[4];
        if (st[4] > st[3]) atomicOr(&info->flags, (uint32_t)SPH_S_EXCLUDED);
    }
}

// Cell begin/end tables over the label-0 prefix. Thread k (0..n0) owns the
// gap between sorted particles k-1 and k: every cell c in (cell(k-1), cell(k)]
// starts at k, every cell in [cell(k-1), cell(k)) ends at k. Each table entry
// is written exactly once; empty cells get begin = end = lower_bound(c).
__global__ __launch_bounds__(256) void k_cell_tables(KParams kp, const uint32_t *__restrict__ sk,
                                                     const DevInfo *__restrict__ info,
                                                     uint32_t nthreads,
                                                     uint32_t *__restrict__ begin,
                                                     uint32_t *__restrict__ end) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nthreads) return;
    const uint32_t n0 = info->n_label[0];
    if (k > n0) return;
    const int64_t cprev = k == 0 ? -1 : (int64_t)(sk[k - 1] & kp.cell_mask);
    const int64_t ccur = k == n0 ? (int64_t)kp.ncells : (int64_t)(sk[k] & kp.cell_mask);
    for (int64_t c = cprev + 1; c <= ccur && c < (int64_t)kp.ncells; c++) begin[c] = k;
    for (int64_t c = cprev < 0 ? 0 : cprev; c < ccur; c++) end[c] = k;
}

hipError_t launch_tables(sph_ctx *c, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, s, c->kp, c->keys_sorted, n, c->info);
    const uint32_t nt = n + 1;
    hipLaunchKernelGGL(k_cell_tables, dim3((nt + 255) / 256), dim3(256), 0, s, c->kp,
                       c->keys_sorted, c->info, nt, c->cell_begin, c->cell_end);
    return hipGetLastError();
}

// ------------------------------------------------------- gather / pack
// Reorder every state array by the sorted permutation (Sec. 3.1: all arrays
// are ordered according to the sorted IDs) and write the packed interaction
// inputs (x, y, z, p/rho^2) and (vx, vy, vz, rho).
__global__ __launch_bounds__(256) void k_gather(KParams kp, sph_soa in, sph_soa out,
                                                const int32_t *__restrict__ perm, uint32_t n,
                                                float4 *__restrict__ pos4,
                                                float4 *__restrict__ vel4) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t s = (uint32_t)perm[k];
    const float x = in.x[s], y = in.y[s], z = in.z[s];
    const float vx = in.vx[s], vy = in.vy[s], vz = in.vz[s], rho = in.rho[s];
    out.x[k] = x; out.y[k] = y; out.z[k] = z;
    out.vx[k] = vx; out.vy[k] = vy; out.vz[k] = vz;
    out.rho[k] = rho;
    out.vxp[k] = in.vxp[s]; out.vyp[k] = in.vyp[s]; out.vzp[k] = in.vzp[s];
    out.rhop[k] = in.rhop[s];
    out.type[k] = in.type[s];
    out.id[k] = in.id[s];
    pos4[k] = make_float4(x, y, z, tait_p_over_rho2(kp, rho));
    vel4[k] = make_float4(vx, vy, vz, rho);
}

hipError_t launch_gather(sph_ctx *c, const sph_soa &in, const sph_soa &out, uint32_t n,
                         hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3((n + 255) / 256), dim3(256), 0, s, c->kp, in, out, c->perm,
                       n, c->pos4, c->vel4);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_pack(KParams kp, sph_soa in, uint32_t n,
                                              float4 *__restrict__ pos4,
                                              float4 *__restrict__ vel4) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float rho = in.rho[k];
    pos4[k] = make_float4(in.x[k], in.y[k], in.z[k], tait_p_over_rho2(kp, rho));
    vel4[k] = make_float4(in.vx[k], in.vy[k], in.vz[k], rho);
}

hipError_t launch_pack(sph_ctx *c, const sph_soa &in, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, s, c->kp, in, n, c->pos4,
                       c->vel4);
    return hipGetLastError();
}

}  // namespace sph
