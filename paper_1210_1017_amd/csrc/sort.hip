// Sort step of the WCSPH time step: cell keys with migration labels, stable
// LSD radix sort, reorder of the particle arrays, cell tables and packing
// ranges (Sec. 3.1 neighbour search; Sec. 4.2-4.3 migration and halo packing).
#include "sph_device.h"

namespace sph {

// ------------------------------------------------------------------ keys
// One thread per particle (Sec. 3.1): key = label << Bc | cell (cell_key).
__global__ __launch_bounds__(256) void k_keys(KParams kp, const float *__restrict__ x,
                                              const float *__restrict__ y,
                                              const float *__restrict__ z,
                                              const uint8_t *__restrict__ type, uint32_t n,
                                              uint32_t *__restrict__ keys,
                                              int32_t *__restrict__ vals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = cell_key(kp, x[i], y[i], z[i], type[i]);
    vals[i] = (int32_t)i;
}

// Keys fused with the digit histogram of the first radix pass (one radix
// tile per block, as k_radix_hist): saves a kernel and a pass over the keys.
__global__ __launch_bounds__(kSortThreads) void k_keys_hist(KParams kp, const float *__restrict__ x,
                                                            const float *__restrict__ y,
                                                            const float *__restrict__ z,
                                                            const uint8_t *__restrict__ type,
                                                            uint32_t n, uint32_t ntiles,
                                                            uint32_t *__restrict__ keys,
                                                            int32_t *__restrict__ vals,
                                                            uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * (uint32_t)kSortTile;
    // all of the thread's positions and types first (clamped index: in bounds
    // for every lane), then the keys
    float px[kSortItems], py[kSortItems], pz[kSortItems];
    uint8_t pt[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t idx = base + r * kSortThreads + tid;
        const uint32_t ic = idx < n ? idx : n - 1u;
        px[r] = x[ic];
        py[r] = y[ic];
        pz[r] = z[ic];
        pt[r] = type[ic];
    }
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t idx = base + r * kSortThreads + tid;
        if (idx < n) {
            const uint32_t key = cell_key(kp, px[r], py[r], pz[r], pt[r]);
            keys[idx] = key;
            vals[idx] = (int32_t)idx;
            atomicAdd(&h[key & 255u], 1u);
        }
    }
    __syncthreads();
    hist[(uint32_t)tid * ntiles + blockIdx.x] = h[tid];
}

hipError_t launch_keys_hist(sph_ctx *c, const sph_soa &in, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t ntiles = (n + kSortTile - 1) / kSortTile;
    hipLaunchKernelGGL(k_keys_hist, dim3(ntiles), dim3(kSortThreads), 0, s, c->kp, in.x, in.y,
                       in.z, in.type, n, ntiles, c->keys_a, c->vals_a, c->hist);
    return hipGetLastError();
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
//            lanes holding the same digit; one count per round, wave and
//            digit, then one prefix per digit over the tile), a reorder
//            through LDS by digit, and coalesced runs written to their global
//            positions.
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
    uint32_t k[kSortItems];  // all loads first (clamped index), then the counts
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t idx = base + r * kSortThreads + tid;
        k[r] = keys[idx < n ? idx : n - 1u];
    }
#pragma unroll
    for (int r = 0; r < kSortItems; r++)
        if (base + r * kSortThreads + tid < n) atomicAdd(&h[(k[r] >> shift) & 255u], 1u);
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
    constexpr int NW = kSortThreads / 64;
    __shared__ uint32_t s_k[kSortTile];
    __shared__ int32_t s_v[kSortTile];
    __shared__ uint32_t s_cnt[kSortItems][NW][256];  // per (round, wave, digit) count, then prefix
    __shared__ uint32_t s_off[256];
    __shared__ uint32_t s_glob[256];
    __shared__ uint32_t s_w[NW];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t tile = blockIdx.x;
    const uint32_t base = tile * (uint32_t)kSortTile;

    // global start of each digit's run for this tile
    const uint32_t gbase = block_excl_scan<kSortThreads>(tot[tid], s_w);
    s_glob[tid] = gbase + hist[(uint32_t)tid * ntiles + tile];
#pragma unroll
    for (int r = 0; r < kSortItems; r++)
#pragma unroll
        for (int k = 0; k < NW; k++) s_cnt[r][k][tid] = 0;

    // all of the tile's loads first
    uint32_t key[kSortItems];
    int32_t val[kSortItems];
    uint32_t rank[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t idx = base + r * kSortThreads + tid;
        const bool valid = idx < n;
        key[r] = valid ? kin[idx] : 0xffffffffu;
        val[r] = valid ? vin[idx] : 0;
    }
    __syncthreads();
    // rank among the wave's lanes with the same digit in this round (ballots
    // over the 8 digit bits); the first such lane records the count
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const bool valid = base + r * kSortThreads + tid < n;
        const uint32_t d = (key[r] >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        rank[r] = (uint32_t)__popcll(peers & lt);
        if (valid && rank[r] == 0) s_cnt[r][w][d] = (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit (one thread each): exclusive prefix over (round, wave), the
    // input order of the tile, so equal digits keep their order
    uint32_t run = 0;
#pragma unroll
    for (int r = 0; r < kSortItems; r++)
#pragma unroll
        for (int k = 0; k < NW; k++) {
            const uint32_t c = s_cnt[r][k][tid];
            s_cnt[r][k][tid] = run;
            run += c;
        }
    s_off[tid] = block_excl_scan<kSortThreads>(run, s_w);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t idx = base + r * kSortThreads + tid;
        if (idx < n) {
            const uint32_t d = (key[r] >> shift) & 255u;
            const uint32_t pos = s_off[d] + s_cnt[r][w][d] + rank[r];
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
                      hipStream_t s, bool first_hist_done) {
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
        if (p > 0 || !first_hist_done)
            hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kSortThreads), 0, s, ksrc, n,
                               shift, ntiles, c->hist);
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

// The same passes with explicit buffers: one scratch pair (ks, vs) and the
// output. The last pass writes the output; the passes before it alternate
// between the scratch pair and the output so that no pass writes onto its own
// source (the input is only read).
hipError_t radix_sort_bufs(const uint32_t *keys_in, const int32_t *vals_in, uint32_t *keys_out,
                           int32_t *vals_out, uint32_t n, int key_bits, uint32_t *ks,
                           int32_t *vs, uint32_t *hist, uint32_t *tot, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int passes = (key_bits + 7) / 8;
    const uint32_t ntiles = (n + kSortTile - 1) / kSortTile;
    const uint32_t *ksrc = keys_in;
    const int32_t *vsrc = vals_in;
    for (int p = 0; p < passes; p++) {
        const bool to_out = ((passes - 1 - p) & 1) == 0;
        uint32_t *kdst = to_out ? keys_out : ks;
        int32_t *vdst = to_out ? vals_out : vs;
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kSortThreads), 0, s, ksrc, n, shift,
                           ntiles, hist);
        hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(256), 0, s, hist, ntiles, tot);
        hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kSortThreads), 0, s, ksrc, vsrc,
                           kdst, vdst, n, shift, ntiles, hist, tot);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        ksrc = kdst;
        vsrc = vdst;
    }
    return hipSuccess;
}

// ---------------------------------------------------- counts and ranges
// Cell tables over the label-0 prefix of the sorted keys (Sec. 3.1 first
// index of each cell; Sec. 4.4 first and last of a region) and label counts.
// Every label-0 key is its cell index and every key of a label l > 0 is at
// least l << Bc, so one search of the sorted keys gives each bound:
//   k_tables: thread c < ncells: begin[c] = lower_bound(c), and
//             end[c - 1] = begin[c]; three more threads: lstart[l] =
//             lower_bound(l << Bc) for l = 1..3 (lstart[1] = n0 also ends
//             the last cell). An empty cell gets begin = end = lower_bound(c).
//             The search starts from the previous table's value (particles
//             move little between sorts, so the bound is usually a few
//             places away); the exponential-then-binary search is correct
//             from any start, including uninitialised tables.
//   k_counts: label counts, and the packing ranges of x-layers 0, 1,
//             ncx-2, ncx-1 read off begin[] (each layer is one contiguous
//             range of the x-major order, Sec. 4.2-4.3).
__device__ __forceinline__ uint32_t lower_bound_from(const uint32_t *__restrict__ sk, uint32_t n,
                                                     uint32_t key, uint32_t hint) {
    hint = hint < n ? hint : n;
    uint32_t lo, hi;  // answer in [lo, hi]: sk[< lo] < key, hi == n or sk[hi] >= key
    if (hint < n && sk[hint] < key) {
        lo = hint + 1;
        hi = n;
        for (uint32_t step = 1;; step <<= 1) {
            const uint32_t q = lo + step - 1;
            if (q >= n) break;
            if (sk[q] >= key) {
                hi = q;
                break;
            }
            lo = q + 1;
        }
    } else {
        hi = hint;
        lo = 0;
        for (uint32_t step = 1;; step <<= 1) {
            if (hi < step) break;
            const uint32_t q = hi - step;
            if (sk[q] < key) {
                lo = q + 1;
                break;
            }
            hi = q;
        }
    }
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (sk[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_tables(KParams kp, const uint32_t *__restrict__ sk,
                                                uint32_t n, DevInfo *__restrict__ info,
                                                uint32_t *__restrict__ begin,
                                                uint32_t *__restrict__ end) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nc = kp.ncells;
    if (t < nc) {
        const uint32_t b = lower_bound_from(sk, n, t, begin[t]);
        begin[t] = b;
        if (t > 0) end[t - 1] = b;
    } else if (t < nc + 3) {
        const uint32_t l = t - nc + 1;
        const uint32_t b = lower_bound_from(sk, n, l << kp.cell_bits, info->lstart[l]);
        info->lstart[l] = b;
        if (l == 1) {
            info->lstart[0] = 0;
            if (nc > 0) end[nc - 1] = b;
        }
    }
}

// Thread t < 9 of one block: label counts and packing ranges.
__device__ __forceinline__ void table_counts(const KParams &kp, const uint32_t *__restrict__ begin,
                                             uint32_t n, DevInfo *__restrict__ info, int t) {
    const uint32_t n0 = info->lstart[1];
    if (t < 4) info->n_label[t] = (t < 3 ? info->lstart[t + 1] : n) - info->lstart[t];
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
        const uint32_t c = (uint32_t)(lay + (t & 1)) * L;
        info->ranges[t] = c < kp.ncells ? begin[c] : n0;
    }
    if (t == 8) {
        info->ranges[8] = info->lstart[1];
        info->ranges[9] = info->lstart[2];
        info->ranges[10] = info->lstart[2];
        info->ranges[11] = info->lstart[3];
        info->ranges[12] = info->lstart[3];
        info->ranges[13] = n;
        if (n > info->lstart[3]) atomicOr(&info->flags, (uint32_t)SPH_S_EXCLUDED);
    }
}

__global__ void k_counts(KParams kp, const uint32_t *__restrict__ begin, uint32_t n,
                         DevInfo *__restrict__ info) {
    table_counts(kp, begin, n, info, (int)threadIdx.x);
}

hipError_t launch_tables(sph_ctx *c, uint32_t n, hipStream_t s, bool counts) {
    const uint32_t threads = c->ncells + 3;
    hipLaunchKernelGGL(k_tables, dim3((threads + 255) / 256), dim3(256), 0, s, c->kp, c->keys_sorted,
                       n, c->info, c->cell_begin, c->cell_end);
    if (counts)
        hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, s, c->kp, c->cell_begin, n, c->info);
    return hipGetLastError();
}

// ------------------------------------------------------- gather / pack
// The interaction that follows a reorder (or a pack) reduces into these.
__device__ __forceinline__ void reset_step_reductions(DevInfo *info) {
    info->dtmin_bits = 0x7f800000u;  // +inf
    info->pairs = 0ull;
}

// Reorder every state array by the sorted permutation (Sec. 3.1: all arrays
// are ordered according to the sorted IDs) and write the packed interaction
// inputs (x, y, z, p/rho^2) and (vx, vy, vz, rho).
// Block 0 also forms the label counts and packing ranges from the cell
// tables (no separate kernel).
__global__ __launch_bounds__(256) void k_gather(KParams kp, sph_soa in, sph_soa out,
                                                const int32_t *__restrict__ perm, uint32_t n,
                                                float4 *__restrict__ pos4,
                                                float4 *__restrict__ vel4,
                                                const uint32_t *__restrict__ cbegin,
                                                DevInfo *__restrict__ info) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) reset_step_reductions(info);
    if (k < 9) table_counts(kp, cbegin, n, info, (int)k);
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
    hipLaunchKernelGGL(k_gather, dim3(n == 0 ? 1 : (n + 255) / 256), dim3(256), 0, s, c->kp, in,
                       out, c->perm, n, c->pos4, c->vel4, c->cell_begin, c->info);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_pack(KParams kp, sph_soa in, uint32_t n,
                                              float4 *__restrict__ pos4,
                                              float4 *__restrict__ vel4,
                                              DevInfo *__restrict__ info) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) reset_step_reductions(info);
    if (k >= n) return;
    const float rho = in.rho[k];
    pos4[k] = make_float4(in.x[k], in.y[k], in.z[k], tait_p_over_rho2(kp, rho));
    vel4[k] = make_float4(in.vx[k], in.vy[k], in.vz[k], rho);
}

hipError_t launch_pack(sph_ctx *c, const sph_soa &in, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_pack, dim3(n == 0 ? 1 : (n + 255) / 256), dim3(256), 0, s, c->kp, in, n,
                       c->pos4, c->vel4, c->info);
    return hipGetLastError();
}

__global__ void k_clear_flags(DevInfo *__restrict__ info) {
    if (threadIdx.x == 0) info->flags = 0u;
}

hipError_t launch_clear_flags(sph_ctx *c, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, c->info);
    return hipGetLastError();
}

}  // namespace sph
