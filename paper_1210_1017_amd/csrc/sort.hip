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

// One radix tile per block, with twice the threads of the radix kernels (more
// waves in flight for the loads; the tile and its mask words are the same).
constexpr int kKeysThreads = 2 * kSortThreads;
constexpr int kKeysItems = kSortTile / kKeysThreads;

// Keys fused with the digit histogram of the first radix pass (one radix
// tile per block, as k_radix_hist) and with the mover flags of the
// incremental sort: particle i is a mover when i >= nprev or its key differs
// from prev[i], the key the previous sort left at index i. Per 64 particles
// (one wave of one round) the mover bits and the movers before that word in
// the tile; per tile the mover count, the smallest and largest key, and its
// movers' (key, index) in index order at the tile's own place of
// (segk, segi).
__global__ __launch_bounds__(kKeysThreads) void k_keys_move(
    KParams kp, const float *__restrict__ x, const float *__restrict__ y,
    const float *__restrict__ z, const uint8_t *__restrict__ type, uint32_t n, uint32_t ntiles,
    uint32_t *__restrict__ keys, uint32_t *__restrict__ hist,  // null: not stored / counted
    const uint32_t *__restrict__ prev, uint32_t nprev, unsigned long long *__restrict__ mmask,
    uint32_t *__restrict__ mwpre, uint32_t *__restrict__ mcnt, uint32_t *__restrict__ segk,
    uint32_t *__restrict__ segi, uint2 *__restrict__ mtile) {
    constexpr int NW = kKeysThreads / 64;
    constexpr int WPT = kSortTile / 64;  // mask words per tile
    static_assert(WPT <= 64, "one wave scans a tile's words");
    __shared__ uint32_t h[256];
    __shared__ uint32_t s_wc[WPT];
    __shared__ uint32_t s_kmin, s_kmax;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid < 256) h[tid] = 0;
    if (tid == 0) {
        s_kmin = 0xffffffffu;
        s_kmax = 0u;
    }
    __syncthreads();
    const uint32_t base = blockIdx.x * (uint32_t)kSortTile;
    // all of the thread's loads first (clamped index: in bounds for every
    // lane), then the keys
    float px[kKeysItems], py[kKeysItems], pz[kKeysItems];
    uint8_t pt[kKeysItems];
    uint32_t pk[kKeysItems];
#pragma unroll
    for (int r = 0; r < kKeysItems; r++) {
        const uint32_t idx = base + r * kKeysThreads + tid;
        const uint32_t ic = idx < n ? idx : n - 1u;
        px[r] = x[ic];
        py[r] = y[ic];
        pz[r] = z[ic];
        pt[r] = type[ic];
        pk[r] = nprev ? prev[idx < nprev ? idx : nprev - 1u] : 0u;
    }
    uint32_t key[kKeysItems];
    unsigned long long bm[kKeysItems];
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint32_t kmin = 0xffffffffu, kmax = 0u;
#pragma unroll
    for (int r = 0; r < kKeysItems; r++) {
        const uint32_t idx = base + r * kKeysThreads + tid;
        const bool valid = idx < n;
        key[r] = cell_key(kp, px[r], py[r], pz[r], pt[r]);
        if (valid) {
            if (keys) keys[idx] = key[r];
            if (hist) atomicAdd(&h[key[r] & 255u], 1u);
            kmin = key[r] < kmin ? key[r] : kmin;
            kmax = key[r] > kmax ? key[r] : kmax;
        }
        bm[r] = __ballot(valid && (idx >= nprev || key[r] != pk[r]));
        if (lane == 0) {
            s_wc[r * NW + w] = (uint32_t)__popcll(bm[r]);
            if (base + (uint32_t)(r * kKeysThreads + w * 64) < n)
                mmask[(base >> 6) + (uint32_t)(r * NW + w)] = bm[r];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t a = (uint32_t)__shfl_xor((int)kmin, o), c = (uint32_t)__shfl_xor((int)kmax, o);
        kmin = a < kmin ? a : kmin;
        kmax = c > kmax ? c : kmax;
    }
    if (lane == 0) {
        atomicMin(&s_kmin, kmin);
        atomicMax(&s_kmax, kmax);
    }
    __syncthreads();
    if (hist && tid < 256) hist[(uint32_t)tid * ntiles + blockIdx.x] = h[tid];
    if (tid == 0) mtile[blockIdx.x] = make_uint2(s_kmin, s_kmax);
    if (tid < 64) {  // word r * NW + w covers particles base + 64 (r * NW + w) + [0, 64)
        const uint32_t v = tid < WPT ? s_wc[tid] : 0u;
        const uint32_t inc = wave_incl_scan(v);
        if (tid < WPT) {
            s_wc[tid] = inc - v;
            if (base + 64u * (uint32_t)tid < n) mwpre[(base >> 6) + tid] = inc - v;
        }
        if (tid == 63) mcnt[blockIdx.x] = inc;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kKeysItems; r++) {
        if ((bm[r] >> lane) & 1ull) {
            const uint32_t at = base + s_wc[r * NW + w] + (uint32_t)__popcll(bm[r] & lt);
            segk[at] = key[r];
            segi[at] = base + r * kKeysThreads + tid;
        }
    }
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

// Gating and size of the passes: with `skip`, a pass runs only when the
// sort's mode (*skip) is `run_mode`; with `n_dev`, the key count is *n_dev
// (at most ntiles tiles; tiles past it count nothing and write nothing).
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                             uint32_t n, int shift,
                                                             uint32_t ntiles,
                                                             uint32_t *__restrict__ hist,
                                                             const uint32_t *__restrict__ skip,
                                                             uint32_t run_mode,
                                                             const uint32_t *__restrict__ n_dev) {
    if (skip && *skip != run_mode) return;
    if (n_dev) n = *n_dev;
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * (uint32_t)kSortTile;
    if (base < n) {
        uint32_t k[kSortItems];  // all loads first (clamped index), then the counts
#pragma unroll
        for (int r = 0; r < kSortItems; r++) {
            const uint32_t idx = base + r * kSortThreads + tid;
            k[r] = keys[idx < n ? idx : n - 1u];
        }
#pragma unroll
        for (int r = 0; r < kSortItems; r++)
            if (base + r * kSortThreads + tid < n) atomicAdd(&h[(k[r] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint32_t)tid * ntiles + blockIdx.x] = h[tid];
}

__global__ __launch_bounds__(256) void k_radix_scan(uint32_t *__restrict__ hist, uint32_t ntiles,
                                                    uint32_t *__restrict__ tot,
                                                    const uint32_t *__restrict__ skip,
                                                    uint32_t run_mode) {
    if (skip && *skip != run_mode) return;
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
    const uint32_t *__restrict__ hist, const uint32_t *__restrict__ tot,
    const uint32_t *__restrict__ skip, uint32_t run_mode, const uint32_t *__restrict__ n_dev) {
    if (skip && *skip != run_mode) return;
    if (n_dev) n = *n_dev;
    if (blockIdx.x * (uint32_t)kSortTile >= n) return;  // a tile past the keys
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
        val[r] = valid ? (vin ? vin[idx] : (int32_t)idx) : 0;  // no values: the index
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

// vals_in may be null: the first pass then takes each key's index as its value.
hipError_t radix_sort(sph_ctx *c, const uint32_t *keys_in, const int32_t *vals_in,
                      uint32_t *keys_out, int32_t *vals_out, uint32_t n, int key_bits,
                      hipStream_t s, bool first_hist_done, const uint32_t *skip) {
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
                               shift, ntiles, c->hist, skip, kModeFull, nullptr);
        hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(256), 0, s, c->hist, ntiles,
                           c->digit_tot, skip, kModeFull);
        hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kSortThreads), 0, s, ksrc, vsrc,
                           kdst, vdst, n, shift, ntiles, c->hist, c->digit_tot, skip, kModeFull,
                           nullptr);
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
                           int32_t *vs, uint32_t *hist, uint32_t *tot, hipStream_t s,
                           const uint32_t *skip, uint32_t run_mode, const uint32_t *n_dev) {
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
                           ntiles, hist, skip, run_mode, n_dev);
        hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(256), 0, s, hist, ntiles, tot, skip,
                           run_mode);
        hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kSortThreads), 0, s, ksrc, vsrc,
                           kdst, vdst, n, shift, ntiles, hist, tot, skip, run_mode, n_dev);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        ksrc = kdst;
        vsrc = vdst;
    }
    return hipSuccess;
}

// ------------------------------------------------------ incremental sort
// Between two sorts of one simulation most particles keep their cell, so the
// key of the particle at index i usually equals prev[i], the key the previous
// sort left at index i. Such a particle is a stayer; every other one (and
// every index at or beyond the previous sort's n) is a mover. The stayers'
// keys are the previous sorted keys at their indices, so in index order they
// never decrease, and the stable sort of all keys is the merge, by
// (key, index), of the stayers in index order with the movers stably sorted
// by key (the stable order is unique, so the result is the radix sort's):
//   stayer i:  dest = i - (movers before index i) + (movers below (key_i, i))
//   mover k (k-th in (key, index) order):
//              dest = (stayers below (key, index)) + k,
// where the stayers below (key, j) are the non-movers before
// P = clamp(j, lower_bound(prev, key), upper_bound(prev, key)): the pairs
// (prev[p], p) increase with p. Both bounds come from the previous sort's
// cell tables (label 0), the label's first index and the previous n
// (label 3: one key), or a search of prev within the label's range (labels
// 1 and 2). k_keys_move flags the movers; k_move_plan sorts up to kIncCap of
// them in LDS (with more it selects the radix passes, whose kernels then run
// while the merge work is skipped, and vice versa); k_gather moves every
// particle to its place.

// Movers at indices below q (q <= n).
__device__ __forceinline__ uint32_t movers_before(uint32_t q, uint32_t n, uint32_t m,
                                                  const unsigned long long *__restrict__ mmask,
                                                  const uint32_t *__restrict__ mwpre,
                                                  const uint32_t *__restrict__ moff) {
    if (q >= n) return m;
    const uint32_t wd = q >> 6;
    return moff[q / (uint32_t)kSortTile] + mwpre[wd] +
           (uint32_t)__popcll(mmask[wd] & ((1ull << (q & 63u)) - 1ull));
}

__device__ __forceinline__ uint32_t upper_in(const uint32_t *__restrict__ a, uint32_t lo,
                                             uint32_t hi, uint32_t key) {
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (a[mid] <= key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t lower_in(const uint32_t *__restrict__ a, uint32_t lo,
                                             uint32_t hi, uint32_t key) {
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (a[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// The index q below which the stayers precede (key, j) in (key, index)
// order: P = clamp(j, lower_bound, upper_bound) over the previous keys, at
// most ns (no stayer at or beyond ns). lb and ub as found for the key.
__device__ __forceinline__ uint32_t stayer_split(uint32_t j, uint32_t lb, uint32_t ub,
                                                 uint32_t nprev, uint32_t ns) {
    lb = lb < nprev ? lb : nprev;
    ub = ub < lb ? lb : (ub < nprev ? ub : nprev);
    const uint32_t P = j < lb ? lb : (j > ub ? ub : j);
    return P < ns ? P : ns;
}

constexpr int kPlanThreads = 1024;
constexpr int kPlanWaves = kPlanThreads / 64;
constexpr uint32_t kNoSplit = 0xffffffffu;

// One round of a stable LSD radix pass over (sk, si)[c0, c0 + 1024) into
// (dk, di) (LDS or global): ranks among the wave's lanes with the same digit
// from 8 ballots, per-(wave, digit) counts stamped (high half) with the
// round, one prefix per digit over the waves. The prefixes overwrite every
// entry and are relative to the round's start of the digit (below 1024, so
// their high half is 0 and never a stamp); that start is kept in s_b0 and
// the running digit starts in s_base advance by the round's counts.
__device__ __forceinline__ void lsd_round(const uint32_t *sk, const uint32_t *si, uint32_t *dk,
                                          uint32_t *di, uint32_t m, uint32_t c0, int shift,
                                          uint32_t stamp, uint32_t (*s_wc)[256],
                                          uint32_t *s_base, uint32_t *s_b0) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t k = c0 + (uint32_t)tid;
    const bool valid = k < m;
    const uint32_t key = valid ? sk[k] : 0u;
    const uint32_t idx = valid ? si[k] : 0u;
    const uint32_t d = (key >> shift) & 255u;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const bool bit = (d >> b) & 1u;
        const unsigned long long mb = __ballot(bit);
        peers &= bit ? mb : ~mb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
    if (valid && rank == 0) s_wc[w][d] = stamp << 16 | (uint32_t)__popcll(peers);
    __syncthreads();
    if (tid < 256) {  // per digit: prefix over the waves in order
        uint32_t c[kPlanWaves];
#pragma unroll
        for (int q = 0; q < kPlanWaves; q++) {
            const uint32_t e = s_wc[q][tid];
            c[q] = (e >> 16) == stamp ? (e & 0xffffu) : 0u;
        }
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < kPlanWaves; q++) {
            s_wc[q][tid] = run;
            run += c[q];
        }
        const uint32_t b0 = s_base[tid];
        s_b0[tid] = b0;
        s_base[tid] = b0 + run;
    }
    __syncthreads();
    if (valid) {
        const uint32_t pos = s_b0[d] + s_wc[w][d] + rank;
        dk[pos] = key;
        di[pos] = idx;
    }
    __syncthreads();
}

// Stable LSD sort of (key, index) pairs by key: `passes` 8-bit digits, the
// digit counts of all passes in s_hist. Returns the buffer (0 or 1) that
// holds the result.
__device__ __forceinline__ int lsd_sort(uint32_t *k0, uint32_t *i0, uint32_t *k1, uint32_t *i1,
                                        uint32_t m, int passes, uint32_t (*s_wc)[256],
                                        uint32_t *s_base, uint32_t *s_b0,
                                        uint32_t (*s_hist)[256], uint32_t *stamp) {
    const int tid = threadIdx.x;
    int src = 0;
    for (int p = 0; p < passes; p++) {
        if (tid < 64) {  // digit starts: one wave, 4 digits per lane; the first
                         // round's barrier orders them before their reads
            uint32_t c[4], sum = 0;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                c[e] = s_hist[p][4 * tid + e];
                sum += c[e];
            }
            uint32_t ex = wave_incl_scan(sum) - sum;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                s_base[4 * tid + e] = ex;
                ex += c[e];
            }
        }
        uint32_t *sk = src ? k1 : k0, *si = src ? i1 : i0;
        uint32_t *dk = src ? k0 : k1, *di = src ? i0 : i1;
        for (uint32_t c0 = 0; c0 < m; c0 += kPlanThreads) {
            uint32_t st = ++*stamp & 0xffffu;
            if (st == 0) {  // the stamps wrapped: clear, and skip stamp 0
                for (int q = tid; q < kPlanWaves * 256; q += kPlanThreads) (&s_wc[0][0])[q] = 0u;
                __syncthreads();
                st = ++*stamp & 0xffffu;
            }
            lsd_round(sk, si, dk, di, m, c0, 8 * p, st, s_wc, s_base, s_b0);
        }
        src ^= 1;
    }
    return src;
}

// Lower bounds of (k0, j0) and (k1, j1) in the (key, index)-sorted (sk, si)
// of length m, searched in step (the same halving sequence).
__device__ __forceinline__ uint2 lower_bound2(const uint32_t *sk, const uint32_t *si, uint32_t m,
                                              uint32_t k0, uint32_t j0, uint32_t k1, uint32_t j1) {
    uint32_t b0 = 0, b1 = 0;
    for (uint32_t len = m; len > 1;) {
        const uint32_t half = len / 2;
        const uint32_t ka = sk[b0 + half], ia = si[b0 + half];
        const uint32_t kb = sk[b1 + half], ib = si[b1 + half];
        if (ka < k0 || (ka == k0 && ia < j0)) b0 += half;
        if (kb < k1 || (kb == k1 && ib < j1)) b1 += half;
        len -= half;
    }
    if (m > 0) {
        const uint32_t ka = sk[b0], ia = si[b0];
        const uint32_t kb = sk[b1], ib = si[b1];
        b0 += (ka < k0 || (ka == k0 && ia < j0)) ? 1u : 0u;
        b1 += (kb < k1 || (kb == k1 && ib < j1)) ? 1u : 0u;
    }
    return make_uint2(b0, b1);
}

// Lower bound of (key, idx) in the (key, index)-sorted (sk, si) of length m,
// by the 64 lanes of a wave together (every lane gets it): each step tests 64
// evenly spaced pivots of [lo, hi) and keeps the gap after the last one below.
__device__ __forceinline__ uint32_t wave_lower_bound(const uint32_t *sk, const uint32_t *si,
                                                     uint32_t m, uint32_t key, uint32_t idx,
                                                     uint32_t lane) {
    uint32_t lo = 0, hi = m;  // the answer lies in [lo, hi]
    while (hi > lo) {
        const uint32_t step = (hi - lo + 63u) / 64u;
        const uint32_t p = lo + lane * step;
        bool below = false;
        if (p < hi) {
            const uint32_t k = sk[p], j = si[p];
            below = k < key || (k == key && j < idx);
        }
        const uint32_t c = (uint32_t)__popcll(__ballot(below));  // pivots below: lanes 0..c-1
        if (c == 0) return lo;
        const uint32_t last = lo + (c - 1u) * step;  // below the target
        const uint32_t next = lo + c * step;          // at or above it, when < hi
        lo = last + 1u;
        hi = next < hi ? next : hi;
        if (step == 1u) return lo;
    }
    return lo;
}

// Wave-cooperative copy of the tiles' mover segments with more than `above`
// movers to (dk, di) at the tiles' offsets: wave w takes tiles w, w + NW,
// ... (lane j reads the offsets of the j-th of them), 64 movers per load and
// eight loads in flight.
__device__ __forceinline__ void copy_segments(const uint32_t *__restrict__ segk,
                                              const uint32_t *__restrict__ segi,
                                              const uint32_t *__restrict__ moff, uint32_t ntiles,
                                              uint32_t m, uint32_t above, uint32_t *dk,
                                              uint32_t *di) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (uint32_t g = 0; g * (uint32_t)(kPlanWaves * 64) < ntiles; g++) {
        const uint32_t t = (uint32_t)w + (uint32_t)kPlanWaves * ((uint32_t)lane + 64u * g);
        const uint32_t off = t < ntiles ? moff[t] : m;
        const uint32_t nxt = t + 1 < ntiles ? moff[t + 1] : m;
        unsigned long long big = __ballot(t < ntiles && nxt - off > above);
        while (big) {
            const int src = __builtin_ctzll(big);
            big &= big - 1ull;
            const uint32_t tt = (uint32_t)w + (uint32_t)kPlanWaves * ((uint32_t)src + 64u * g);
            const uint32_t toff = __shfl(off, src), tcnt = __shfl(nxt - off, src);
            const uint32_t sb = tt * (uint32_t)kSortTile;
            for (uint32_t j0 = 0; j0 < tcnt; j0 += 512) {
                uint32_t kk[8], ii[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const uint32_t j = j0 + (uint32_t)(u * 64 + lane);
                    const uint32_t jc = j < tcnt ? j : tcnt - 1u;
                    kk[u] = segk[sb + jc];
                    ii[u] = segi[sb + jc];
                }
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const uint32_t j = j0 + (uint32_t)(u * 64 + lane);
                    if (j < tcnt) {
                        dk[toff + j] = kk[u];
                        di[toff + j] = ii[u];
                    }
                }
            }
        }
    }
}

// One block. Per-tile mover counts -> exclusive offsets (in place) and the
// total m, reported to the host word fb (m and whether there was a previous
// sort) when fb is set. Then:
//  * m <= kIncCap: the movers (index order, from the tiles' segments) into
//    LDS at their tiles' offsets, sorted stably by key there;
//  * m > kIncCap and allow_full: the movers' own radix passes are chosen
//    when m <= mid (kModeMid: k_move_compact, the passes and k_move_split
//    do the rest), else the radix passes over all keys; nothing more here;
//  * m > kIncCap otherwise (the host expected few movers): the movers are
//    copied to global memory and sorted there by the same passes, slowly
//    but exactly.
// The offsets end with moff[ntiles] = m.
// Out: the movers sorted by (key, index) in (outk, outi); per tile the range
// of sorted movers its particles can fall between; the stayer split of the
// label-1 and label-2 movers (a search of the previous keys; the gather
// finds the others' from the cell tables) in tmpk. (tmpk, tmpi) is the
// second buffer of the global sort; the one of (outk, outi) and (tmpk, tmpi)
// that the pass count makes the start of the global sort must not be the
// segments' buffer.
__global__ __launch_bounds__(kPlanThreads) void k_move_plan(
    uint32_t n, uint32_t ntiles, int passes, const uint32_t *__restrict__ segk,
    const uint32_t *__restrict__ segi, uint32_t *__restrict__ mcnt, const uint32_t *__restrict__ prev,
    uint32_t nprev, uint32_t cell_bits, uint32_t *outk, uint32_t *outi, uint32_t *tmpk,
    uint32_t *tmpi, uint2 *__restrict__ mtile,
    DevInfo *__restrict__ info, int allow_full, uint32_t mid, unsigned long long *fb) {
    __shared__ uint32_t s_k[2][kIncCap];
    __shared__ uint32_t s_i[2][kIncCap];
    __shared__ uint32_t s_wc[kPlanWaves][256];
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_b0[256];
    __shared__ uint32_t s_w[kPlanWaves];
    __shared__ uint32_t s_hist[4][256];  // digit counts of every pass
    __shared__ uint32_t s_big;  // a tile with more movers than one thread copies was seen
    const int tid = threadIdx.x;
    if (tid == 0) s_big = 0u;
    (&s_hist[0][0])[tid] = 0u;
    for (int q = tid; q < kPlanWaves * 256; q += kPlanThreads) (&s_wc[0][0])[q] = 0u;
    // the first tiles' key ranges, needed at the end: loaded now
    const uint2 kr0 = (uint32_t)tid < ntiles ? mtile[tid] : make_uint2(0u, 0u);

    // offsets, one tile per thread per round; a thread copies the movers of
    // its tile to LDS when there are at most kSmall (loads in flight
    // together), a wave those of larger tiles below
    constexpr uint32_t kSmall = 32;
    uint32_t running = 0;
    for (uint32_t start = 0; start < ntiles; start += kPlanThreads) {
        const uint32_t t = start + (uint32_t)tid;
        const uint32_t v = t < ntiles ? mcnt[t] : 0u;
        uint32_t total;
        const uint32_t pre = block_excl_scan<kPlanThreads>(v, s_w, &total) + running;
        running += total;
        const bool fits = running <= kIncCap;  // the same in every thread
        if (t < ntiles) mcnt[t] = pre;
        if (fits && v > kSmall) s_big = 1u;
        if (fits && v > 0u && v <= kSmall) {
            // 16-byte loads from the tile's segment (8 KB aligned), only as
            // many as hold its movers: one cache line per lane and load
            const uint4 *gk = (const uint4 *)(segk + t * (uint32_t)kSortTile);
            const uint4 *gi = (const uint4 *)(segi + t * (uint32_t)kSortTile);
            uint4 kk[kSmall / 4], ii[kSmall / 4];
#pragma unroll
            for (uint32_t u = 0; u < kSmall / 4; u++)
                if (4u * u < v) {
                    kk[u] = gk[u];
                    ii[u] = gi[u];
                }
#pragma unroll
            for (uint32_t u = 0; u < kSmall / 4; u++) {
                const uint32_t kv[4] = {kk[u].x, kk[u].y, kk[u].z, kk[u].w};
                const uint32_t iv[4] = {ii[u].x, ii[u].y, ii[u].z, ii[u].w};
#pragma unroll
                for (uint32_t e = 0; e < 4; e++)
                    if (4u * u + e < v) {
                        s_k[0][pre + 4u * u + e] = kv[e];
                        s_i[0][pre + 4u * u + e] = iv[e];
                    }
            }
        }
    }
    const uint32_t m = running;  // the same in every thread
    if (tid == 0) mcnt[ntiles] = m;
    if (tid == 0 && fb)
        __hip_atomic_store(fb, (unsigned long long)m << 1 | (nprev > 0 ? 1ull : 0ull),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const bool small = m <= kIncCap;
    if (!small && allow_full) {
        if (tid == 0) {
            info->sort_mode = m <= mid ? kModeMid : kModeFull;
            info->movers = m;
        }
        return;
    }
    __syncthreads();  // offsets (global) and s_big
    uint32_t stamp = 0;
    const uint32_t *fk, *fi;  // the sorted movers
    if (small) {
        if (s_big) copy_segments(segk, segi, mcnt, ntiles, m, kSmall, s_k[0], s_i[0]);
        __syncthreads();
        for (uint32_t k = (uint32_t)tid; k < m; k += kPlanThreads) {  // digit counts of all passes
            const uint32_t key = s_k[0][k];
            for (int p = 0; p < passes; p++) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255u], 1u);
        }
        __syncthreads();
        const int r = lsd_sort(s_k[0], s_i[0], s_k[1], s_i[1], m, passes, s_wc, s_base, s_b0,
                               s_hist, &stamp);
        for (uint32_t k = (uint32_t)tid; k < m; k += kPlanThreads) {
            outk[k] = s_k[r][k];
            outi[k] = s_i[r][k];
        }
        fk = s_k[r];
        fi = s_i[r];
    } else {
        // the pass count decides where to start so that the result lands in
        // (outk, outi)
        uint32_t *ak = (passes & 1) ? tmpk : outk, *ai = (passes & 1) ? tmpi : outi;
        uint32_t *bk = (passes & 1) ? outk : tmpk, *bi = (passes & 1) ? outi : tmpi;
        copy_segments(segk, segi, mcnt, ntiles, m, 0u, ak, ai);
        __syncthreads();
        for (uint32_t k = (uint32_t)tid; k < m; k += kPlanThreads) {
            const uint32_t key = ak[k];
            for (int p = 0; p < passes; p++) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255u], 1u);
        }
        __syncthreads();
        lsd_sort(ak, ai, bk, bi, m, passes, s_wc, s_base, s_b0, s_hist, &stamp);
        fk = outk;
        fi = outi;
    }
    // per tile: the range of the sorted movers that can lie below its
    // particles, [movers below (kmin, first index), movers below (kmax, end)]
    for (uint32_t t = (uint32_t)tid; t < ntiles; t += kPlanThreads) {
        const uint2 kr = t == (uint32_t)tid ? kr0 : mtile[t];
        const uint32_t i0 = t * (uint32_t)kSortTile;
        mtile[t] = lower_bound2(fk, fi, m, kr.x, i0, kr.y, i0 + (uint32_t)kSortTile);
    }
    const uint32_t ns = nprev < n ? nprev : n;
    for (uint32_t k = (uint32_t)tid; k < m; k += kPlanThreads) {
        const uint32_t key = fk[k], idx = fi[k];
        const uint32_t l = key >> cell_bits;
        uint32_t split = kNoSplit;
        if ((l == 1u || l == 2u) && ns > 0) {
            uint32_t hi = info->lstart[l + 1];
            hi = hi < nprev ? hi : nprev;
            uint32_t lo = info->lstart[l];
            lo = lo < hi ? lo : hi;
            const uint32_t lb = lower_in(prev, lo, hi, key);
            split = stayer_split(idx, lb, upper_in(prev, lb, hi, key), nprev, ns);
        }
        tmpk[k] = split;
    }
    if (tid == 0) {
        info->sort_mode = kModeIncr;
        info->movers = m;
    }
}

// kModeMid, before the movers' radix passes: the movers of each tile's
// segment (index order) to their offsets in (ck, ci), one wave per tile.
__global__ __launch_bounds__(64) void k_move_compact(const uint32_t *__restrict__ segk,
                                                     const uint32_t *__restrict__ segi,
                                                     const uint32_t *__restrict__ moff,
                                                     uint32_t ntiles, uint32_t *__restrict__ ck,
                                                     uint32_t *__restrict__ ci,
                                                     const uint32_t *__restrict__ mode) {
    if (*mode != kModeMid) return;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t o = moff[t], cnt = moff[t + 1] - o;
        const uint32_t sb = t * (uint32_t)kSortTile;
        for (uint32_t r = threadIdx.x; r < cnt; r += 64u) {
            ck[o + r] = segk[sb + r];
            ci[o + r] = segi[sb + r];
        }
    }
}

// kModeMid, after the passes: what the plan's block does for few movers, over
// the grid: per tile the range of the sorted movers (fk, fi) its particles
// can fall between, and the stayer split of the label-1 and label-2 movers
// into split[].
__global__ __launch_bounds__(256) void k_move_split(const uint32_t *__restrict__ fk,
                                                    const uint32_t *__restrict__ fi,
                                                    uint32_t n, uint32_t ntiles,
                                                    const uint32_t *__restrict__ prev,
                                                    uint32_t nprev, uint32_t cell_bits,
                                                    uint2 *__restrict__ mtile,
                                                    uint32_t *__restrict__ split,
                                                    const DevInfo *__restrict__ info) {
    if (info->sort_mode != kModeMid) return;
    const uint32_t m = info->movers;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x, gs = gridDim.x * blockDim.x;
    // one wave per tile: 64-way search steps (ballot over 64 pivots) instead
    // of a chain of dependent halvings
    const uint32_t lane = threadIdx.x & 63u;
    for (uint32_t t = g >> 6; t < ntiles; t += gs >> 6) {
        const uint2 kr = mtile[t];
        const uint32_t i0 = t * (uint32_t)kSortTile;
        const uint32_t a = wave_lower_bound(fk, fi, m, kr.x, i0, lane);
        const uint32_t b = wave_lower_bound(fk, fi, m, kr.y, i0 + (uint32_t)kSortTile, lane);
        if (lane == 0) mtile[t] = make_uint2(a, b);
    }
    const uint32_t ns = nprev < n ? nprev : n;
    for (uint32_t k = g; k < m; k += gs) {
        const uint32_t key = fk[k], idx = fi[k];
        const uint32_t l = key >> cell_bits;
        uint32_t q = kNoSplit;
        if ((l == 1u || l == 2u) && ns > 0) {
            uint32_t hi = info->lstart[l + 1];
            hi = hi < nprev ? hi : nprev;
            uint32_t lo = info->lstart[l];
            lo = lo < hi ? lo : hi;
            const uint32_t lb = lower_in(prev, lo, hi, key);
            q = stayer_split(idx, lb, upper_in(prev, lb, hi, key), nprev, ns);
        }
        split[k] = q;
    }
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
//             With counts: label counts, and the packing ranges of x-layers
//             0, 1, ncx-2, ncx-1, each the begin of a layer's first cell
//             (each layer is one contiguous range of the x-major order,
//             Sec. 4.2-4.3).
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

// Cell of the packing range bound t < 8 (Sec. 4.2-4.3): the first cell of
// x-layer 0, 1, ncx-2, ncx-1 (even t) or of the layer after it (odd t).
__device__ __forceinline__ uint32_t layer_cell(const KParams &kp, int t) {
    int lay;
    switch (t >> 1) {
        case 0: lay = 0; break;
        case 1: lay = 1; break;
        case 2: lay = kp.ncx - 2; break;
        default: lay = kp.ncx - 1; break;
    }
    lay = lay < 0 ? 0 : (lay >= kp.ncx ? kp.ncx - 1 : lay);
    return (uint32_t)(lay + (t & 1)) * (uint32_t)kp.ncy * (uint32_t)kp.ncz;
}

// With `counts`, each thread also writes the counts and ranges that its own
// bounds decide: a cell thread the packing bounds at its cell, label thread
// l the first index of label l, the size of label l and the ranges that
// start or end there (no thread waits for another).
__global__ __launch_bounds__(256) void k_tables(KParams kp, const uint32_t *__restrict__ sk,
                                                uint32_t n, DevInfo *__restrict__ info,
                                                uint32_t *__restrict__ begin,
                                                uint32_t *__restrict__ end, int counts) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nc = kp.ncells;
    if (t < nc) {
        const uint32_t b = lower_bound_from(sk, n, t, begin[t]);
        begin[t] = b;
        if (t > 0) end[t - 1] = b;
        if (counts)
#pragma unroll
            for (int r = 0; r < 8; r++)
                if (layer_cell(kp, r) == t) info->ranges[r] = b;
    } else if (t < nc + 3) {
        const uint32_t l = t - nc + 1;
        const uint32_t hint = info->lstart[l];
        const uint32_t b = lower_bound_from(sk, n, l << kp.cell_bits, hint);
        // the next label's first index (n after label 3), for the count
        const uint32_t b1 = l < 3 ? lower_bound_from(sk, n, (l + 1) << kp.cell_bits, b) : n;
        info->lstart[l] = b;
        if (l == 1) {
            info->lstart[0] = 0;
            if (nc > 0) end[nc - 1] = b;
        }
        if (counts) {
            info->n_label[l] = b1 - b;
            if (l == 1) {
                info->n_label[0] = b;
                info->ranges[8] = b;
#pragma unroll
                for (int r = 0; r < 8; r++)
                    if (layer_cell(kp, r) >= nc) info->ranges[r] = b;
            } else if (l == 2) {
                info->ranges[9] = b;
                info->ranges[10] = b;
            } else {
                info->ranges[11] = b;
                info->ranges[12] = b;
                info->ranges[13] = n;
                if (n > b) atomicOr(&info->flags, (uint32_t)SPH_S_EXCLUDED);
            }
        }
    }
}

hipError_t launch_tables(sph_ctx *c, uint32_t n, hipStream_t s, bool counts) {
    const uint32_t threads = c->ncells + 3;
    hipLaunchKernelGGL(k_tables, dim3((threads + 255) / 256), dim3(256), 0, s, c->kp, c->keys_sorted,
                       n, c->info, c->cell_begin, c->cell_end, counts ? 1 : 0);
    return hipGetLastError();
}

// ------------------------------------------------------- gather / pack
// The interaction that follows a reorder (or a pack) reduces into these.
__device__ __forceinline__ void reset_step_reductions(DevInfo *info) {
    info->dtmin_bits = 0x7f800000u;  // +inf
    info->pairs = 0ull;
}

// Reorder every state array by the sort (Sec. 3.1: all arrays are ordered
// according to the sorted IDs) and write the packed interaction inputs
// (x, y, z, p/rho^2) and (vx, vy, vz, rho). After the radix passes thread k
// pulls particle perm[k] into place k; after the merge path thread i pushes
// particle i to its destination and writes its key there (the sorted keys).
struct MoveArgs {
    const uint32_t *keys;  // unsorted keys (index order); null: formed again from the particle
    uint32_t *skeys;       // sorted keys: read as the previous ones, written by the merge
    const uint32_t *mk, *mi;  // the movers sorted by (key, index)
    const uint2 *mtile;       // per tile: the range of them its particles fall between
    const uint32_t *msplit;
    const unsigned long long *mmask;
    const uint32_t *mwpre, *moff;
    const uint32_t *cbegin, *cend;  // the previous sort's cell tables
    uint32_t nprev;
};

// With skip_rv the position, velocity and density go to the packed arrays
// only (the step's update writes them to the state from there).
__device__ __forceinline__ void move_particle(const KParams &kp, const sph_soa &in,
                                              const sph_soa &out, uint32_t s, uint32_t k,
                                              float4 *__restrict__ pos4,
                                              float4 *__restrict__ vel4, bool skip_rv) {
    const float x = in.x[s], y = in.y[s], z = in.z[s];
    const float vx = in.vx[s], vy = in.vy[s], vz = in.vz[s], rho = in.rho[s];
    const float vxp = in.vxp[s], vyp = in.vyp[s], vzp = in.vzp[s], rhop = in.rhop[s];
    const uint8_t ty = in.type[s];
    const int32_t id = in.id[s];
    if (!skip_rv) {
        out.x[k] = x; out.y[k] = y; out.z[k] = z;
        out.vx[k] = vx; out.vy[k] = vy; out.vz[k] = vz;
        out.rho[k] = rho;
    }
    out.vxp[k] = vxp; out.vyp[k] = vyp; out.vzp[k] = vzp;
    out.rhop[k] = rhop;
    out.type[k] = ty;
    out.id[k] = id;
    pos4[k] = make_float4(x, y, z, tait_p_over_rho2(kp, rho));
    vel4[k] = make_float4(vx, vy, vz, rho);
}

__global__ __launch_bounds__(256) void k_gather(KParams kp, sph_soa in, sph_soa out,
                                                const int32_t *__restrict__ perm, uint32_t n,
                                                float4 *__restrict__ pos4,
                                                float4 *__restrict__ vel4,
                                                DevInfo *__restrict__ info, MoveArgs mv,
                                                int skip_rv) {
    // the sorted movers that a block's particles (one tile's) can fall
    // between, staged when they are few
    constexpr uint32_t kStageMovers = 1024;
    __shared__ uint32_t s_mk[kStageMovers], s_mi[kStageMovers];
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) reset_step_reductions(info);
    if (n == 0) return;
    if (info->sort_mode == kModeFull) {
        if (k < n) move_particle(kp, in, out, (uint32_t)perm[k], k, pos4, vel4, skip_rv != 0);
        return;
    }
    const uint32_t b0 = blockIdx.x * blockDim.x;  // 256 | kSortTile: one tile per block
    const uint2 range = mv.mtile[b0 / (uint32_t)kSortTile];
    const uint32_t len = range.y - range.x;
    const bool staged = len <= kStageMovers;  // the same in every thread
    if (staged) {
        for (uint32_t r = threadIdx.x; r < len; r += blockDim.x) {
            s_mk[r] = mv.mk[range.x + r];
            s_mi[r] = mv.mi[range.x + r];
        }
    }
    __syncthreads();
    if (k >= n) return;
    const uint32_t i = k, m = info->movers;
    // the key from the particle's own data when the keys kernel did not
    // store it (the same function of the same values)
    const uint32_t key = mv.keys ? mv.keys[i] : cell_key(kp, in.x[i], in.y[i], in.z[i], in.type[i]);
    uint32_t lo = range.x, hi = range.y;  // movers below (key, i) in (key, index) order
    if (staged) {
        lo = 0;
        hi = len;
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            const uint32_t ek = s_mk[mid], ei = s_mi[mid];
            if (ek < key || (ek == key && ei < i))
                lo = mid + 1;
            else
                hi = mid;
        }
        lo += range.x;
    } else {
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            const uint32_t ek = mv.mk[mid], ei = mv.mi[mid];
            if (ek < key || (ek == key && ei < i))
                lo = mid + 1;
            else
                hi = mid;
        }
    }
    const uint32_t wd = i >> 6;
    const unsigned long long bits = mv.mmask[wd];
    uint32_t dest;
    if ((bits >> (i & 63u)) & 1ull) {  // a mover: lo is its own rank
        const uint32_t ns = mv.nprev < n ? mv.nprev : n;
        uint32_t q = mv.msplit[lo];
        if (q == kNoSplit) {
            if (ns == 0)
                q = 0;
            else if (key < kp.ncells)
                q = stayer_split(i, mv.cbegin[key], mv.cend[key], mv.nprev, ns);
            else  // label 3: a single key, from its first index to the end
                q = stayer_split(i, info->lstart[3], mv.nprev, mv.nprev, ns);
        }
        dest = q - movers_before(q, n, m, mv.mmask, mv.mwpre, mv.moff) + lo;
    } else {
        const uint32_t before = mv.moff[i / (uint32_t)kSortTile] + mv.mwpre[wd] +
                                (uint32_t)__popcll(bits & ((1ull << (i & 63u)) - 1ull));
        dest = i - before + lo;
    }
    move_particle(kp, in, out, i, dest, pos4, vel4, skip_rv != 0);
    mv.skeys[dest] = key;
}

// The plain sort step: keys and mover flags, the mover plan, the radix passes
// (run only when the plan chose them; not launched at all when the caller
// expects few movers, the plan then sorting any number itself), reorder,
// cell tables and counts of the new order.
hipError_t sort_state(sph_ctx *c, const sph_soa &in, const sph_soa &out, uint32_t n,
                      uint32_t nprev, int expect, bool skip_rv, hipStream_t s) {
    const bool expect_merge = expect == kExpectFew;
    const uint32_t *mode = &c->info->sort_mode;
    const int key_bits = c->cell_bits + 2;
    const int passes = (key_bits + 7) / 8;
    // the movers' tile segments live in (keys_b, vals_b); the sorted movers
    // end in (keys_b, vals_b) after an odd number of passes, else in
    // (perm, vals_a); the other pair holds the stayer splits
    uint32_t *segk = c->keys_b, *segi = (uint32_t *)c->vals_b;
    uint32_t *xk = (uint32_t *)c->perm, *xi = (uint32_t *)c->vals_a;
    uint32_t *outk = (passes & 1) ? segk : xk, *outi = (passes & 1) ? segi : xi;
    uint32_t *tmpk = (passes & 1) ? xk : segk, *tmpi = (passes & 1) ? xi : segi;
    if (n > 0) {
        const uint32_t ntiles = (n + kSortTile - 1) / kSortTile;
        // the first radix pass's digit counts here only when the full passes
        // are likely to run (with a middle number of movers expected, their
        // first pass counts for itself if the plan chooses it after all)
        const bool keys_hist = expect == kExpectAny;
        // with only the merge kernels launched the reorder forms each key
        // again from the particle's data instead of reading it back
        hipLaunchKernelGGL(k_keys_move, dim3(ntiles), dim3(kKeysThreads), 0, s, c->kp, in.x,
                           in.y, in.z, in.type, n, ntiles, expect_merge ? nullptr : c->keys_a,
                           keys_hist ? c->hist : nullptr, c->keys_sorted, nprev, c->mmask,
                           c->mwpre, c->mcnt, segk, segi, c->mtile);
        const uint32_t mid = mid_cap(n) > kIncCap ? mid_cap(n) : 0u;
        hipLaunchKernelGGL(k_move_plan, dim3(1), dim3(kPlanThreads), 0, s, n, ntiles, passes, segk,
                           segi, c->mcnt, c->keys_sorted, nprev, (uint32_t)c->cell_bits, outk,
                           outi, tmpk, tmpi, c->mtile, c->info, expect_merge ? 0 : 1, mid,
                           c->fb_dev);
        if (!expect_merge) {
            if (mid > 0) {
                // kModeMid: the movers to (xk, xi), their radix passes (the
                // count read on the device, the grid sized for mid), ending in
                // (outk, outi) with the other pair as scratch, then the ranges
                // and splits
                const uint32_t cblocks = ntiles < 65535u ? ntiles : 65535u;
                hipLaunchKernelGGL(k_move_compact, dim3(cblocks), dim3(64), 0, s, segk, segi,
                                   c->mcnt, ntiles, xk, xi, mode);
                hipError_t e = radix_sort_bufs(xk, (const int32_t *)xi, outk, (int32_t *)outi, mid,
                                               key_bits, tmpk, (int32_t *)tmpi, c->hist,
                                               c->digit_tot, s, mode, kModeMid, &c->info->movers);
                if (e != hipSuccess) return e;
                // a wave per tile for the ranges, then a thread per mover
                const uint32_t sw = (ntiles + 3u) / 4u, sm = (mid + 255u) / 256u;
                const uint32_t sneed = sw > sm ? sw : sm;
                const uint32_t sblocks = sneed < 4096u ? sneed : 4096u;
                hipLaunchKernelGGL(k_move_split, dim3(sblocks), dim3(256), 0, s, outk, outi, n,
                                   ntiles, c->keys_sorted, nprev, (uint32_t)c->cell_bits, c->mtile,
                                   tmpk, c->info);
            }
            // the first pass takes each key's index as its value
            hipError_t e = radix_sort(c, c->keys_a, nullptr, c->keys_sorted, c->perm, n,
                                      key_bits, s, keys_hist, mode);
            if (e != hipSuccess) return e;
        }
    }
    const MoveArgs mv = {expect_merge ? nullptr : c->keys_a, c->keys_sorted, outk, outi,
                         c->mtile, tmpk, c->mmask, c->mwpre, c->mcnt, c->cell_begin, c->cell_end,
                         nprev};
    hipLaunchKernelGGL(k_gather, dim3(n == 0 ? 1 : (n + 255) / 256), dim3(256), 0, s, c->kp, in,
                       out, c->perm, n, c->pos4, c->vel4, c->info, mv, skip_rv ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_tables(c, n, s, true);
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
