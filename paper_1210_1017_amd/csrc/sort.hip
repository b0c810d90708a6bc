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
// Cell tables over the label-0 prefix of the sorted keys (Sec. 3.1 first
// index of each cell; Sec. 4.4 first and last of a region) and label counts:
//   k_fill:        begin[c] = EMPTY for every cell;
//   k_mark:        thread k marks the label boundaries around k (label starts
//                  lstart[l] = lower_bound(l << Bc)) and, for label 0, the first
//                  and one-past-last index of k's cell;
//   k_cells_min:   per block of cells, the minimum begin (EMPTY if all empty);
//   k_cells_carry: suffix minimum over the blocks (n0 past the last one);
//   k_cells_apply: an empty cell c gets begin = end = min over cells >= c of
//                  begin, i.e. lower_bound(c) (begins rise with the cell index);
//   k_counts:      label counts, and the packing ranges of x-layers 0, 1,
//                  ncx-2, ncx-1 read off begin[] (each layer is one contiguous
//                  range of the x-major order, Sec. 4.2-4.3).
constexpr uint32_t kEmpty = 0xffffffffu;

__global__ __launch_bounds__(256) void k_fill(uint32_t *__restrict__ a, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ __launch_bounds__(256) void k_mark(KParams kp, const uint32_t *__restrict__ sk,
                                              uint32_t n, DevInfo *__restrict__ info,
                                              uint32_t *__restrict__ begin,
                                              uint32_t *__restrict__ end) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > n) return;
    const uint32_t kc = k < n ? sk[k] : 0u;
    const int lprev = k == 0 ? -1 : (int)(sk[k - 1] >> kp.cell_bits);
    const int lcur = k == n ? 4 : (int)(kc >> kp.cell_bits);
    for (int l = lprev + 1; l <= lcur && l < 4; l++) info->lstart[l] = k;
    if (k < n && lcur == 0) {
        const uint32_t c = kc & kp.cell_mask;
        if (k == 0 || sk[k - 1] != kc) begin[c] = k;
        if (k + 1 == n || sk[k + 1] != kc) end[c] = k + 1;
    }
}

__device__ __forceinline__ uint32_t wave_suffix_min(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_down(v, o, 64);
        if (lane + o < 64) v = min(v, t);
    }
    return v;
}

__global__ __launch_bounds__(kCellScanThreads) void k_cells_min(const uint32_t *__restrict__ begin,
                                                               uint32_t ncells,
                                                               uint32_t *__restrict__ bmin) {
    __shared__ uint32_t s_w[kCellScanThreads / 64];
    const uint32_t base = blockIdx.x * (uint32_t)kCellScanBlock;
    uint32_t m = kEmpty;
#pragma unroll
    for (int r = 0; r < kCellScanItems; r++) {
        const uint32_t c = base + r * kCellScanThreads + threadIdx.x;
        if (c < ncells) m = min(m, begin[c]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = min(m, (uint32_t)__shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kCellScanThreads / 64; w++) m = min(m, s_w[w]);
        bmin[blockIdx.x] = m;
    }
}

// One block: bmin[b] <- min(n0, bmin[b+1], bmin[b+2], ...) (exclusive suffix).
__global__ __launch_bounds__(256) void k_cells_carry(uint32_t *__restrict__ bmin, uint32_t nb,
                                                     const DevInfo *__restrict__ info) {
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_carry;
    const uint32_t n0 = info->lstart[1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_carry = n0;
    __syncthreads();
    // chunks of 256 blocks, from the last chunk down
    const uint32_t nchunk = (nb + 255) / 256;
    for (uint32_t ch = nchunk; ch-- > 0;) {
        const uint32_t b = ch * 256 + tid;
        const uint32_t v = b < nb ? bmin[b] : kEmpty;
        const uint32_t wsuf = wave_suffix_min(v);  // min over lanes >= lane
        if (lane == 0) s_w[w] = wsuf;
        __syncthreads();
        uint32_t later = s_carry;  // min over chunks after this one
        for (int q = w + 1; q < 4; q++) later = min(later, s_w[q]);
        const uint32_t nxt = __shfl_down(wsuf, 1, 64);
        const uint32_t excl = min(later, lane < 63 ? nxt : kEmpty);
        __syncthreads();
        if (b < nb) bmin[b] = excl;
        if (tid == 0) {
            uint32_t all = s_carry;
            for (int q = 0; q < 4; q++) all = min(all, s_w[q]);
            s_carry = all;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kCellScanThreads) void k_cells_apply(uint32_t *__restrict__ begin,
                                                                 uint32_t *__restrict__ end,
                                                                 uint32_t ncells,
                                                                 const uint32_t *__restrict__ carry) {
    __shared__ uint32_t s_w[kCellScanThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // thread t owns cells base + t*4 .. base + t*4 + 3 (contiguous, in order)
    const uint32_t base = blockIdx.x * (uint32_t)kCellScanBlock + (uint32_t)tid * kCellScanItems;
    uint32_t v[kCellScanItems];
#pragma unroll
    for (int r = 0; r < kCellScanItems; r++) v[r] = base + r < ncells ? begin[base + r] : kEmpty;
    uint32_t tmin = kEmpty;
#pragma unroll
    for (int r = 0; r < kCellScanItems; r++) tmin = min(tmin, v[r]);
    const uint32_t wsuf = wave_suffix_min(tmin);
    if (lane == 0) s_w[w] = wsuf;
    __syncthreads();
    uint32_t after = carry[blockIdx.x];
    for (int q = w + 1; q < kCellScanThreads / 64; q++) after = min(after, s_w[q]);
    const uint32_t nxt = __shfl_down(wsuf, 1, 64);
    after = min(after, lane < 63 ? nxt : kEmpty);  // min over cells after this thread's
#pragma unroll
    for (int r = kCellScanItems - 1; r >= 0; r--) {
        if (v[r] == kEmpty) {
            if (base + r < ncells) {
                begin[base + r] = after;
                end[base + r] = after;
            }
        } else {
            after = v[r];
        }
    }
}

__global__ void k_counts(KParams kp, const uint32_t *__restrict__ begin, uint32_t n,
                         DevInfo *__restrict__ info) {
    const int t = threadIdx.x;
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

hipError_t launch_tables(sph_ctx *c, uint32_t n, hipStream_t s) {
    const uint32_t nc = c->ncells;
    const uint32_t nb = (nc + kCellScanBlock - 1) / kCellScanBlock;
    hipLaunchKernelGGL(k_fill, dim3((nc + 255) / 256), dim3(256), 0, s, c->cell_begin, nc, kEmpty);
    hipLaunchKernelGGL(k_mark, dim3((n + 1 + 255) / 256), dim3(256), 0, s, c->kp, c->keys_sorted,
                       n, c->info, c->cell_begin, c->cell_end);
    hipLaunchKernelGGL(k_cells_min, dim3(nb), dim3(kCellScanThreads), 0, s, c->cell_begin, nc,
                       c->cell_blockmin);
    hipLaunchKernelGGL(k_cells_carry, dim3(1), dim3(256), 0, s, c->cell_blockmin, nb, c->info);
    hipLaunchKernelGGL(k_cells_apply, dim3(nb), dim3(kCellScanThreads), 0, s, c->cell_begin,
                       c->cell_end, nc, c->cell_blockmin);
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
__global__ __launch_bounds__(256) void k_gather(KParams kp, sph_soa in, sph_soa out,
                                                const int32_t *__restrict__ perm, uint32_t n,
                                                float4 *__restrict__ pos4,
                                                float4 *__restrict__ vel4,
                                                DevInfo *__restrict__ info) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) reset_step_reductions(info);
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
                       out, c->perm, n, c->pos4, c->vel4, c->info);
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
