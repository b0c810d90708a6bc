// Learned-surrogate kernels: the per-particle input rows gathered from the
// cell list, bfloat16 matrix-core (MFMA) GEMMs with FP32 accumulation for the
// forward and backward passes of the MLP, the element-wise pieces around them
// (bias, SiLU, loss, column sums, Adam), training targets, the application of
// a prediction to the state, the error of a surrogate state against plain SPH,
// and one fused kernel (rows + network + application) for the advance.
#include "sph_device.h"

namespace sph {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNnSlots = SPH_NN_SLOTS;       // neighbour slots per row
constexpr int kNnIn = SPH_NN_IN;             // 64 * 8 + 32
constexpr int kNnList = 128;                 // in-support neighbours kept before the sort
constexpr uint64_t kNoKey = ~0ull;

struct NnScales {
    float inv_len, inv_vel, rho_ref, inv_rho;
};

// ===================================================== neighbour selection
// LDS of one wave: the in-support neighbours of the current row as
// (FP32 squared-distance bits, sorted index).
struct NnList {
    uint32_t r2[kNnList];
    uint32_t j[kNnList];
};

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// One compare-exchange stage of a bitonic sort over the wave; element e of
// the sequence sits in this register of lane e % 64.
__device__ __forceinline__ uint64_t bitonic_stage(uint64_t key, uint32_t e, uint32_t k,
                                                  uint32_t jj) {
    const uint64_t v = shfl_xor_u64(key, (int)jj);
    const bool asc = (e & k) == 0;
    const bool lower = (e & jj) == 0;
    const uint64_t mn = key < v ? key : v, mx = key < v ? v : key;
    return (lower == asc) ? mn : mx;
}

// Called by a whole wave for one particle i (wave-uniform): finds every j != i
// of the 27 cells around i's cell that passes the FP32 support test (Sec. 2.2,
// cells of Sec. 3.1), keeps the first kNnList in LDS (ballot compaction), and
// sorts them by (r2, j) with a bitonic network over the wave's registers.
// Returns in lane l the l-th smallest key (r2 bits << 32 | j), kNoKey if
// fewer, and the neighbour count before truncation.
// Latency: lanes 0..8 fetch the bounds of the 9 z-runs at once; the runs are
// then walked as one flat candidate range, kNnBatch x 64 candidates (their
// positions loaded together) per round.
constexpr int kNnBatch = 4;

__device__ __forceinline__ uint64_t nn_select(const KParams &kp, const float4 *__restrict__ pos4,
                                              const uint32_t *__restrict__ cbeg,
                                              const uint32_t *__restrict__ cend, uint32_t cell,
                                              uint32_t i, float4 pi, NnList *L,
                                              uint32_t &count) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t ncz = (uint32_t)kp.ncz, ncy = (uint32_t)kp.ncy;
    const int cz = (int)(cell % ncz), cy = (int)((cell / ncz) % ncy), cx = (int)(cell / (ncz * ncy));
    const uint32_t zlo = (uint32_t)(cz > 0 ? cz - 1 : 0);
    const uint32_t zhi = (uint32_t)(cz + 1 < kp.ncz ? cz + 1 : kp.ncz - 1);
    uint32_t rb = 0, re = 0;
    if (lane < 9) {
        const int X = cx + (int)lane / 3 - 1, Y = cy + (int)lane % 3 - 1;
        if (X >= 0 && X < kp.ncx && Y >= 0 && Y < kp.ncy) {
            const uint32_t c0 = ((uint32_t)X * ncy + (uint32_t)Y) * ncz;
            rb = cbeg[c0 + zlo];
            re = cend[c0 + zhi];
        }
    }
    // flat candidate t of run r maps to j = t + delta[r], run r spanning
    // [off[r], off[r+1]) of the flat range (wave-uniform values)
    uint32_t off[10], delta[9];
    off[0] = 0;
#pragma unroll
    for (int r = 0; r < 9; r++) {
        const uint32_t b = __builtin_amdgcn_readlane(rb, r), e = __builtin_amdgcn_readlane(re, r);
        delta[r] = b - off[r];
        off[r + 1] = off[r] + (e - b);
    }
    const uint32_t total = off[9];
    uint32_t cnt = 0;
    for (uint32_t t0 = 0; t0 < total; t0 += 64 * kNnBatch) {
        float4 pj[kNnBatch];
        uint32_t jv[kNnBatch];
#pragma unroll
        for (int u = 0; u < kNnBatch; u++) {
            const uint32_t t = t0 + 64 * u + lane;
            uint32_t j = t + delta[0];
#pragma unroll
            for (int r = 1; r < 9; r++) j = t >= off[r] ? t + delta[r] : j;
            jv[u] = t < total ? j : 0xffffffffu;
            pj[u] = t < total ? pos4[j] : pi;
        }
#pragma unroll
        for (int u = 0; u < kNnBatch; u++) {
            const uint32_t j = jv[u];
            const float dx = pi.x - pj[u].x, dy = pi.y - pj[u].y, dz = pi.z - pj[u].z;
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const bool ok = j != 0xffffffffu && j != i && r2 < kp.r2max;
            const uint64_t m = __ballot(ok);
            const uint32_t pos =
                cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (ok && pos < (uint32_t)kNnList) {
                L->r2[pos] = __float_as_uint(r2);
                L->j[pos] = j;
            }
            cnt += (uint32_t)__popcll(m);
        }
    }
    count = cnt;
    wave_lds_sync();
    const uint32_t m = cnt < (uint32_t)kNnList ? cnt : (uint32_t)kNnList;
    uint64_t k0 = lane < m ? (((uint64_t)L->r2[lane] << 32) | L->j[lane]) : kNoKey;
    if (m <= 64) {
#pragma unroll
        for (uint32_t k = 2; k <= 64; k <<= 1)
#pragma unroll
            for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) k0 = bitonic_stage(k0, lane, k, jj);
    } else {
        uint64_t k1 = lane + 64 < m ? (((uint64_t)L->r2[lane + 64] << 32) | L->j[lane + 64])
                                    : kNoKey;
        // halves in opposite directions, one merge step keeps the smaller 64
        // (a bitonic sequence), which the last six stages sort
#pragma unroll
        for (uint32_t k = 2; k <= 64; k <<= 1)
#pragma unroll
            for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
                k0 = bitonic_stage(k0, lane, k, jj);
                k1 = bitonic_stage(k1, lane + 64, k, jj);
            }
        k0 = k0 < k1 ? k0 : k1;
#pragma unroll
        for (uint32_t jj = 32; jj > 0; jj >>= 1) k0 = bitonic_stage(k0, lane, 128, jj);
    }
    wave_lds_sync();  // the list is rewritten for the next row
    return k0;
}

__device__ __forceinline__ float nn_kind(uint8_t t) { return t == kBoundary ? -1.0f : 1.0f; }

// The 8 features of the neighbour slot held by this lane (zeros if empty).
__device__ __forceinline__ bf16x8 nn_slot(const NnScales &sc, const float4 *__restrict__ pos4,
                                          const float4 *__restrict__ vel4,
                                          const uint8_t *__restrict__ type, uint64_t key,
                                          float4 pi, float4 vi) {
    bf16x8 f;
    if (key == kNoKey) {
#pragma unroll
        for (int q = 0; q < 8; q++) f[q] = (bf16)0.0f;
        return f;
    }
    const uint32_t j = (uint32_t)key;
    const float4 pj = pos4[j], vj = vel4[j];
    f[0] = (bf16)((pj.x - pi.x) * sc.inv_len);
    f[1] = (bf16)((pj.y - pi.y) * sc.inv_len);
    f[2] = (bf16)((pj.z - pi.z) * sc.inv_len);
    f[3] = (bf16)((vj.x - vi.x) * sc.inv_vel);
    f[4] = (bf16)((vj.y - vi.y) * sc.inv_vel);
    f[5] = (bf16)((vj.z - vi.z) * sc.inv_vel);
    f[6] = (bf16)((vj.w - sc.rho_ref) * sc.inv_rho);
    f[7] = (bf16)nn_kind(type[j]);
    return f;
}

// The own block, 8 columns per lane for lanes 0..3 (lane 0 carries the six
// used values, the rest is zero).
__device__ __forceinline__ bf16x8 nn_own(const NnScales &sc, uint32_t lane, float4 vi,
                                         uint32_t count, uint8_t t) {
    bf16x8 f;
#pragma unroll
    for (int q = 0; q < 8; q++) f[q] = (bf16)0.0f;
    if (lane == 0) {
        f[0] = (bf16)((vi.w - sc.rho_ref) * sc.inv_rho);
        f[1] = (bf16)(vi.x * sc.inv_vel);
        f[2] = (bf16)(vi.y * sc.inv_vel);
        f[3] = (bf16)(vi.z * sc.inv_vel);
        f[4] = (bf16)((float)count * (1.0f / 64.0f));
        f[5] = (bf16)nn_kind(t);
    }
    return f;
}

// Builds row `i` (sorted index) into dst (row of kNnIn bfloat16, 16-byte
// aligned; global or LDS). Whole wave, i wave-uniform.
__device__ __forceinline__ void nn_row(const KParams &kp, const NnScales &sc,
                                       const float4 *__restrict__ pos4,
                                       const float4 *__restrict__ vel4,
                                       const uint8_t *__restrict__ type,
                                       const uint32_t *__restrict__ sk,
                                       const uint32_t *__restrict__ cbeg,
                                       const uint32_t *__restrict__ cend, uint32_t i,
                                       uint32_t n0, NnList *L, bf16 *dst, uint32_t *flags) {
    const uint32_t lane = threadIdx.x & 63;
    i = __builtin_amdgcn_readfirstlane(i);
    bf16x8 *d8 = reinterpret_cast<bf16x8 *>(dst);
    if (i >= n0 || type[i] == kGhost) {
        bf16x8 z;
#pragma unroll
        for (int q = 0; q < 8; q++) z[q] = (bf16)0.0f;
        d8[lane] = z;
        if (lane < 4) d8[kNnSlots + lane] = z;
        return;
    }
    const float4 pi = pos4[i], vi = vel4[i];
    uint32_t count;
    const uint64_t key = nn_select(kp, pos4, cbeg, cend, sk[i] & kp.cell_mask, i, pi, L, count);
    if (count > (uint32_t)kNnList && lane == 0) atomicOr(flags, (uint32_t)SPH_S_NN_LIST);
    d8[lane] = nn_slot(sc, pos4, vel4, type, key, pi, vi);
    if (lane < 4) d8[kNnSlots + lane] = nn_own(sc, lane, vi, count, type[i]);
}

__global__ __launch_bounds__(256) void k_nn_features(KParams kp, NnScales sc,
                                                     const float4 *__restrict__ pos4,
                                                     const float4 *__restrict__ vel4,
                                                     const uint8_t *__restrict__ type,
                                                     const uint32_t *__restrict__ sk,
                                                     const uint32_t *__restrict__ cbeg,
                                                     const uint32_t *__restrict__ cend,
                                                     DevInfo *__restrict__ info,
                                                     const int32_t *__restrict__ rows,
                                                     uint32_t nrows, bf16 *__restrict__ X) {
    __shared__ NnList s_list[4];
    const uint32_t w = threadIdx.x >> 6;
    const uint32_t n0 = info->n_label[0];
    for (uint32_t r = blockIdx.x * 4 + w; r < nrows; r += gridDim.x * 4) {
        const uint32_t i = rows ? (uint32_t)rows[r] : r;
        nn_row(kp, sc, pos4, vel4, type, sk, cbeg, cend, i, n0, &s_list[w],
               X + (size_t)r * kNnIn, &info->flags);
    }
}

hipError_t launch_nn_features(sph_ctx *c, const uint8_t *type, const int32_t *rows,
                              uint32_t nrows, const sph_nn_scales &s, void *X, hipStream_t st) {
    if (nrows == 0) return hipSuccess;
    const NnScales sc{s.inv_len, s.inv_vel, s.rho_ref, s.inv_rho};
    const uint32_t blocks = (nrows + 3) / 4 < 65536u ? (nrows + 3) / 4 : 65536u;
    hipLaunchKernelGGL(k_nn_features, dim3(blocks), dim3(256), 0, st, c->kp, sc, c->pos4,
                       c->vel4, type, c->keys_sorted, c->cell_begin, c->cell_end, c->info, rows,
                       nrows, (bf16 *)X);
    return hipGetLastError();
}

// ================================================================== GEMM
// C[m][n] (FP32) = sum_k A[m][k] B[k][n] (+ C if accumulate), A and B
// bfloat16 addressed through element strides (transposed operands need no
// copy). Workgroup tile 64 x 64, 4 waves of 32 x 32 (2 x 2 MFMA tiles of
// 16 x 16), k steps of 32: one v_mfma_f32_16x16x32_bf16 per tile and step.
// Operand tiles are staged in LDS as A[m][k] and B^T[n][k], so each lane
// reads its 8 consecutive k of one row (A) or column (B) with one 16-byte LDS
// load. Staging walks k fastest when that stride is 1, else m (n) fastest,
// so global reads stay contiguous either way. Out-of-range elements are
// staged as zeros. With split-K (gridDim.z > 1) slice z covers
// k in [z kchunk, (z+1) kchunk) and writes its partial product to
// part[z][M][N]; k_gemm_reduce adds the slices in order.
constexpr int kGT = 64;
constexpr int kGK = 32;
constexpr int kGKp = 40;  // padded LDS row (bfloat16)

struct GemmArgs {
    const bf16 *A;
    const bf16 *B;
    float *C;
    int M, N, K;
    long long sam, sak, sbk, sbn, scm, scn;
    int accumulate;
    int kchunk;
    float *part;
};

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) bf16 sA[kGT][kGKp];
    __shared__ __attribute__((aligned(16))) bf16 sB[kGT][kGKp];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int kbeg = blockIdx.z * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);
    const bool a_kfast = g.sak == 1, b_kfast = g.sbk == 1;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16 zero = (bf16)0.0f;
    for (int k0 = kbeg; k0 < kend; k0 += kGK) {
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int idx = e * 256 + tid;
            {
                const int r = a_kfast ? idx >> 5 : idx & 63;
                const int kk = a_kfast ? idx & 31 : idx >> 6;
                const int m = m0 + r, k = k0 + kk;
                sA[r][kk] = (m < g.M && k < kend) ? g.A[m * g.sam + k * g.sak] : zero;
            }
            {
                const int r = b_kfast ? idx >> 5 : idx & 63;
                const int kk = b_kfast ? idx & 31 : idx >> 6;
                const int n = n0 + r, k = k0 + kk;
                sB[r][kk] = (n < g.N && k < kend) ? g.B[k * g.sbk + n * g.sbn] : zero;
            }
        }
        __syncthreads();
        const int row = lane & 15, kb = (lane >> 4) * 8;
        bf16x8 fa[2], fb[2];
#pragma unroll
        for (int t = 0; t < 2; t++) {
            fa[t] = *reinterpret_cast<const bf16x8 *>(&sA[wm + t * 16 + row][kb]);
            fb[t] = *reinterpret_cast<const bf16x8 *>(&sB[wn + t * 16 + row][kb]);
        }
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    // D layout: lane holds rows 4 (lane/16) + r, column lane % 16 of each tile
    const int col = lane & 15, rb = (lane >> 4) * 4;
    const bool split = gridDim.z > 1;
    float *P = split ? g.part + (size_t)blockIdx.z * g.M * g.N : nullptr;
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int m = m0 + wm + a * 16 + rb + r, n = n0 + wn + b * 16 + col;
                if (m < g.M && n < g.N) {
                    if (split) {
                        P[(size_t)m * g.N + n] = acc[a][b][r];
                    } else {
                        float *p = g.C + m * g.scm + n * g.scn;
                        *p = g.accumulate ? *p + acc[a][b][r] : acc[a][b][r];
                    }
                }
            }
}

__global__ __launch_bounds__(256) void k_gemm_reduce(GemmArgs g, int splits) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)g.M * g.N) return;
    const int m = (int)(i / g.N), n = (int)(i % g.N);
    float s = 0.0f;
    for (int z = 0; z < splits; z++) s += g.part[(size_t)z * g.M * g.N + i];
    float *p = g.C + m * g.scm + n * g.scn;
    *p = g.accumulate ? *p + s : s;
}

// Split-K slices for a GEMM: about 1024 k per slice, at most SPH_MLP_SPLITS,
// and only where the M x N tile grid alone would leave the chip idle.
static int gemm_splits(int M, int N, int K) {
    const int tiles = ((M + kGT - 1) / kGT) * ((N + kGT - 1) / kGT);
    if (tiles >= 512 || K <= 2048) return 1;
    const int s = (K + 1023) / 1024;
    return s < kMlpSplits ? s : kMlpSplits;
}

hipError_t launch_gemm_bf16(GemmArgs g, float *part, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.K <= 0) return hipErrorInvalidValue;
    int splits = part ? gemm_splits(g.M, g.N, g.K) : 1;
    int chunk = (g.K + splits - 1) / splits;
    chunk = (chunk + kGK - 1) / kGK * kGK;
    splits = (g.K + chunk - 1) / chunk;
    g.kchunk = chunk;
    g.part = part;
    dim3 grid((g.N + kGT - 1) / kGT, (g.M + kGT - 1) / kGT, splits);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, g);
    if (splits > 1) {
        const long long n = (long long)g.M * g.N;
        hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g,
                           splits);
    }
    return hipGetLastError();
}

hipError_t launch_gemm(const void *A, const void *B, float *C, int M, int N, int K,
                       long long sam, long long sak, long long sbk, long long sbn, long long scm,
                       long long scn, int accumulate, float *part, hipStream_t s) {
    GemmArgs g{(const bf16 *)A, (const bf16 *)B, C, M, N, K, sam, sak, sbk, sbn, scm, scn,
               accumulate, 0, nullptr};
    return launch_gemm_bf16(g, part, s);
}

// ============================================================ element-wise
__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// Z[r][c] += b[c]; Aout = bfloat16(SiLU(Z)) if act, Fout = Z (FP32) if given
__global__ __launch_bounds__(256) void k_bias_act(float *__restrict__ Z, const float *__restrict__ b,
                                                  bf16 *__restrict__ Aout, float *__restrict__ Fout,
                                                  long long rows, int cols, int act) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= rows * cols) return;
    const float z = Z[i] + b[i % cols];
    Z[i] = z;
    if (act && Aout) Aout[i] = (bf16)silu(z);
    if (Fout) Fout[i] = z;
}

// dZ = bfloat16(dA * SiLU'(Z)), or bfloat16(dA) for the linear output layer
__global__ __launch_bounds__(256) void k_act_back(const float *__restrict__ dA,
                                                  const float *__restrict__ Z,
                                                  bf16 *__restrict__ dZ, long long n, int act) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    dZ[i] = (bf16)(act ? dA[i] * silu_grad(Z[i]) : dA[i]);
}

// Weighted mean squared error over rows x cols (cols <= 4): per-block partial
// sums of w_c (Y - T)^2 / (rows cols) and dY = 2 w_c (Y - T) / (rows cols).
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ Y, const float *__restrict__ T,
                                             float w0, float w1, float w2, float w3,
                                             float *__restrict__ dY, long long rows, int cols,
                                             float *__restrict__ part) {
    __shared__ float s[256];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const float inv = 1.0f / (float)(rows * cols);
    float l = 0.0f;
    if (i < rows * cols) {
        const int c = (int)(i % cols);
        const float wc = c == 0 ? w0 : c == 1 ? w1 : c == 2 ? w2 : w3;
        const float d = Y[i] - T[i];
        l = wc * d * d * inv;
        dY[i] = 2.0f * wc * d * inv;
    }
    s[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// out[0] = sum of part[0..n) in a fixed order (one block)
__global__ __launch_bounds__(256) void k_sum_final(const float *__restrict__ part, long long n,
                                                   float *__restrict__ out) {
    __shared__ float s[256];
    float acc = 0.0f;
    for (long long k = threadIdx.x; k < n; k += 256) acc += part[k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

// db[c] = sum_r dZ[r][c] (one block per column, fixed order)
__global__ __launch_bounds__(256) void k_colsum(const bf16 *__restrict__ dZ, long long rows,
                                                int cols, float *__restrict__ db) {
    __shared__ float s[256];
    const int c = blockIdx.x;
    float acc = 0.0f;
    for (long long r = threadIdx.x; r < rows; r += 256) acc += (float)dZ[r * cols + c];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] = s[0];
}

// Adam on FP32 masters (c1 = 1 - b1^t, c2 = 1 - b2^t); refreshes the
// bfloat16 copy when given.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, float *__restrict__ m,
                                              float *__restrict__ v, const float *__restrict__ g,
                                              bf16 *__restrict__ wb, long long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = (bf16)wi;
}

__global__ __launch_bounds__(256) void k_f32_to_bf16(const float *__restrict__ a,
                                                     bf16 *__restrict__ b, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = (bf16)a[i];
}

static inline dim3 grid1(long long n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_bias_act(float *Z, const float *b, void *Aout, float *Fout, long long rows,
                           int cols, int act, hipStream_t s) {
    const long long n = rows * cols;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bias_act, grid1(n), dim3(256), 0, s, Z, b, (bf16 *)Aout, Fout, rows,
                       cols, act);
    return hipGetLastError();
}

hipError_t launch_act_back(const float *dA, const float *Z, void *dZ, long long n, int act,
                           hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_act_back, grid1(n), dim3(256), 0, s, dA, Z, (bf16 *)dZ, n, act);
    return hipGetLastError();
}

hipError_t launch_mse(const float *Y, const float *T, const float *wcol, float *dY,
                      long long rows, int cols, float *part, float *loss, hipStream_t s) {
    const long long n = rows * cols;
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_mse, grid1(n), dim3(256), 0, s, Y, T, wcol[0], wcol[1], wcol[2],
                       wcol[3], dY, rows, cols, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, part, blocks, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const void *dZ, long long rows, int cols, float *db, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3(cols), dim3(256), 0, s, (const bf16 *)dZ, rows, cols, db);
    return hipGetLastError();
}

hipError_t launch_adam(float *w, float *m, float *v, const float *g, void *wb, long long n,
                       float lr, float b1, float b2, float eps, float c1, float c2,
                       hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, grid1(n), dim3(256), 0, s, w, m, v, g, (bf16 *)wb, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float *a, void *b, long long n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_f32_to_bf16, grid1(n), dim3(256), 0, s, a, (bf16 *)b, n);
    return hipGetLastError();
}

// ============================================== targets, application, judge
__global__ __launch_bounds__(256) void k_id_scatter(const int32_t *__restrict__ id, uint32_t n,
                                                    int32_t *__restrict__ where) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) where[id[k]] = (int32_t)k;
}

hipError_t launch_id_scatter(const int32_t *id, uint32_t n, int32_t *where, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_id_scatter, grid1(n), dim3(256), 0, s, id, n, where);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_nn_targets(sph_soa a, sph_soa b,
                                                    const int32_t *__restrict__ where_b,
                                                    const int32_t *__restrict__ rows,
                                                    uint32_t nrows, float inv_dv, float inv_dr,
                                                    float *__restrict__ T) {
    const uint32_t r = blockIdx.x * 256 + threadIdx.x;
    if (r >= nrows) return;
    const uint32_t k = rows ? (uint32_t)rows[r] : r;
    const int32_t q = where_b[a.id[k]];
    T[4 * r + 0] = (b.vx[q] - a.vx[k]) * inv_dv;
    T[4 * r + 1] = (b.vy[q] - a.vy[k]) * inv_dv;
    T[4 * r + 2] = (b.vz[q] - a.vz[k]) * inv_dv;
    T[4 * r + 3] = (b.rho[q] - a.rho[k]) * inv_dr;
}

hipError_t launch_nn_targets(const sph_soa &a, const sph_soa &b, const int32_t *where_b,
                             const int32_t *rows, uint32_t nrows, float inv_dv, float inv_dr,
                             float *T, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_nn_targets, grid1(nrows), dim3(256), 0, s, a, b, where_b, rows, nrows,
                       inv_dv, inv_dr, T);
    return hipGetLastError();
}

struct NnApply {
    float dv_scale, dr_scale, dt4, rho_tol;
};

// Applies output (y0..y3) to sorted particle k: see sph_nn_apply.
__device__ __forceinline__ void nn_apply_one(const KParams &kp, const sph_soa &st, uint32_t k,
                                             float y0, float y1, float y2, float y3,
                                             const NnApply &ap, uint32_t *flags) {
    const uint8_t t = st.type[k];
    if (t == kGhost) return;
    const float dr = y3 * ap.dr_scale;
    const float rn = st.rho[k] + dr;
    st.rho[k] = rn;
    st.rhop[k] = rn - 0.25f * dr;
    bool ok = isfinite(rn) && fabsf(rn * kp.inv_rho0 - 1.0f) <= ap.rho_tol;
    if (t == kFluid) {
        float *pos[3] = {st.x, st.y, st.z};
        float *vel[3] = {st.vx, st.vy, st.vz};
        float *velp[3] = {st.vxp, st.vyp, st.vzp};
        const float y[3] = {y0, y1, y2};
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const float v = vel[d][k];
            const float dv = y[d] * ap.dv_scale;
            const float vn = v + dv;
            const float xn = pos[d][k] + ap.dt4 * 0.5f * (v + vn);
            pos[d][k] = xn;
            vel[d][k] = vn;
            velp[d][k] = vn - 0.25f * dv;
            ok = ok && isfinite(vn) && isfinite(xn);
        }
    }
    if (!ok) atomicOr(flags, (uint32_t)SPH_S_NN_RANGE);
}

__global__ __launch_bounds__(256) void k_nn_apply(KParams kp, sph_soa st,
                                                  const float *__restrict__ Y, uint32_t nrows,
                                                  NnApply ap, DevInfo *__restrict__ info) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= nrows || k >= info->n_label[0]) return;
    nn_apply_one(kp, st, k, Y[4 * k], Y[4 * k + 1], Y[4 * k + 2], Y[4 * k + 3], ap, &info->flags);
}

hipError_t launch_nn_apply(sph_ctx *c, const sph_soa &st, const float *Y, uint32_t nrows,
                           float dv_scale, float dr_scale, float dt4, float rho_tol,
                           hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    const NnApply ap{dv_scale, dr_scale, dt4, rho_tol};
    hipLaunchKernelGGL(k_nn_apply, grid1(nrows), dim3(256), 0, s, c->kp, st, Y, nrows, ap,
                       c->info);
    return hipGetLastError();
}

// Error of surrogate state S against reference R from base B (see
// sph_nn_judge): per-block partials, then one block adds them in order.
constexpr int kJudge = 8;

__global__ __launch_bounds__(256) void k_nn_judge(sph_soa S, sph_soa R, sph_soa B,
                                                  const int32_t *__restrict__ where_r,
                                                  const int32_t *__restrict__ where_b, uint32_t n,
                                                  double *__restrict__ part) {
    __shared__ double sh[kJudge][256];
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    double v[kJudge] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (k < n && S.type[k] == kFluid) {
        const int32_t id = S.id[k];
        const int32_t q = where_r[id], p = where_b[id];
        const double rs = S.rho[k], rr = R.rho[q], rb = B.rho[p];
        v[0] = fabs(rs - rr) / rr;
        v[1] = (rs - rr) * (rs - rr);
        v[2] = (rr - rb) * (rr - rb);
        const double us[3] = {S.vx[k], S.vy[k], S.vz[k]}, ur[3] = {R.vx[q], R.vy[q], R.vz[q]},
                     ub[3] = {B.vx[p], B.vy[p], B.vz[p]};
        const double xs[3] = {S.x[k], S.y[k], S.z[k]}, xr[3] = {R.x[q], R.y[q], R.z[q]},
                     xb[3] = {B.x[p], B.y[p], B.z[p]};
        for (int d = 0; d < 3; d++) {
            v[3] += (us[d] - ur[d]) * (us[d] - ur[d]);
            v[4] += (ur[d] - ub[d]) * (ur[d] - ub[d]);
            v[5] += (xs[d] - xr[d]) * (xs[d] - xr[d]);
            v[6] += (xr[d] - xb[d]) * (xr[d] - xb[d]);
        }
        v[7] = 1.0;
    }
    for (int q = 0; q < kJudge; q++) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + o]);
            for (int q = 1; q < kJudge; q++) sh[q][threadIdx.x] += sh[q][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x < kJudge) part[(size_t)blockIdx.x * kJudge + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_nn_judge_final(const double *__restrict__ part,
                                                        uint32_t blocks, double *__restrict__ out) {
    __shared__ double sh[kJudge][256];
    double v[kJudge] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t b = threadIdx.x; b < blocks; b += 256) {
        v[0] = fmax(v[0], part[(size_t)b * kJudge]);
        for (int q = 1; q < kJudge; q++) v[q] += part[(size_t)b * kJudge + q];
    }
    for (int q = 0; q < kJudge; q++) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + o]);
            for (int q = 1; q < kJudge; q++) sh[q][threadIdx.x] += sh[q][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x < kJudge) out[threadIdx.x] = sh[threadIdx.x][0];
}

hipError_t launch_nn_judge(const sph_soa &S, const sph_soa &R, const sph_soa &B,
                           const int32_t *where_r, const int32_t *where_b, uint32_t n,
                           double *part, double *out, hipStream_t s) {
    const uint32_t blocks = n == 0 ? 1 : (n + 255) / 256;
    hipLaunchKernelGGL(k_nn_judge, dim3(blocks), dim3(256), 0, s, S, R, B, where_r, where_b, n,
                       part);
    hipLaunchKernelGGL(k_nn_judge_final, dim3(1), dim3(256), 0, s, part, blocks, out);
    return hipGetLastError();
}

// ================================================== fused surrogate advance
// One workgroup (14 waves) per tile of 64 sorted particles:
//  1. the waves build the 64 input rows (nn_row, 4 or 5 each) into an LDS
//     tile [64][kXS]; the row being built doubles as that wave's neighbour
//     list;
//  2. layer 1 (544 -> 128): wave w < 8 computes output columns
//     [16w, 16w+16) for all 64 rows, A fragments from the LDS tile, B
//     fragments (16 bytes of a weight row) straight from global memory (the
//     weights stay in L2, each read once per tile);
//  3. bias + SiLU to bfloat16 into LDS (two ping-pong tiles inside the input
//     tile's space), layers 2 and 3 (128 -> 128) likewise;
//  4. layer 4 (128 -> 4) with the output columns padded to 16, one row block
//     per wave w < 4; the 64 x 4 result goes through LDS to one thread per
//     particle, which applies it (nn_apply_one).
// LDS: 64 x 552 bfloat16 (70.6 KB) + 1 KB, two workgroups (28 waves) per CU.
constexpr int kFW = 128;          // hidden width of the fused kernel
constexpr int kXS = kNnIn + 8;    // padded row of the input tile (bfloat16)
constexpr int kHS = kFW + 8;      // padded row of a hidden activation tile
constexpr int kFusedWaves = 14;  // two workgroups per CU at 7 waves per SIMD
constexpr int kMlpWaves = kFW / 16;

struct FusedNet {
    const bf16 *w0, *w1, *w2, *w3;
    const float *b0, *b1, *b2, *b3;
};

// acc[rb] = A(LDS rows 16 rb.., row stride lda) x W^T(cols col0 .. col0+15)
template <int KD>
__device__ __forceinline__ void fused_layer(const bf16 *sA, int lda, const bf16 *__restrict__ W,
                                            int col0, f32x4 (&acc)[4]) {
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kb = (lane >> 4) * 8;
#pragma unroll
    for (int a = 0; a < 4; a++) acc[a] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16 *wrow = W + (size_t)(col0 + row) * KD + kb;
#pragma unroll 2
    for (int k0 = 0; k0 < KD; k0 += 32) {
        const bf16x8 fb = *reinterpret_cast<const bf16x8 *>(wrow + k0);
        bf16x8 fa[4];
#pragma unroll
        for (int a = 0; a < 4; a++)
            fa[a] = *reinterpret_cast<const bf16x8 *>(sA + (a * 16 + row) * lda + k0 + kb);
#pragma unroll
        for (int a = 0; a < 4; a++)
            acc[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb, acc[a], 0, 0, 0);
    }
}

// bias + SiLU of a 64 x 16 column slab (cols col0..) into an LDS tile
__device__ __forceinline__ void fused_store_act(const f32x4 (&acc)[4],
                                                const float *__restrict__ bias, int col0,
                                                bf16 *sH) {
    const int lane = threadIdx.x & 63;
    const int c = col0 + (lane & 15), rb = (lane >> 4) * 4;
    const float bc = bias[c];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int r = 0; r < 4; r++) sH[(a * 16 + rb + r) * kHS + c] = (bf16)silu(acc[a][r] + bc);
}

__global__ __launch_bounds__(64 * 14, 2) void k_nn_fused(KParams kp, NnScales sc, FusedNet net,
                                                      const float4 *__restrict__ pos4,
                                                      const float4 *__restrict__ vel4,
                                                      const uint32_t *__restrict__ sk,
                                                      const uint32_t *__restrict__ cbeg,
                                                      const uint32_t *__restrict__ cend,
                                                      sph_soa st, NnApply ap,
                                                      DevInfo *__restrict__ info) {
    __shared__ __attribute__((aligned(16))) bf16 sX[64 * kXS];
    __shared__ float sY[64][4];
    const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t n0 = info->n_label[0];
    const uint32_t base = xcd_block(blockIdx.x, gridDim.x) * 64;
    // 1. input rows (each row's LDS space is its wave's neighbour list first)
    for (uint32_t rr = w; rr < 64; rr += kFusedWaves)
        nn_row(kp, sc, pos4, vel4, st.type, sk, cbeg, cend, base + rr, n0,
               reinterpret_cast<NnList *>(sX + rr * kXS), sX + rr * kXS, &info->flags);
    __syncthreads();
    // 2-3. hidden layers; activations ping-pong between two tiles in sX
    bf16 *h0 = sX, *h1 = sX + 64 * kHS;
    f32x4 acc[4];
    const int col0 = (int)w * 16;
    const bool mlp = w < (uint32_t)kMlpWaves;
    if (mlp) fused_layer<kNnIn>(sX, kXS, net.w0, col0, acc);
    __syncthreads();  // every wave is done reading the input tile
    if (mlp) fused_store_act(acc, net.b0, col0, h0);
    __syncthreads();
    if (mlp) {
        fused_layer<kFW>(h0, kHS, net.w1, col0, acc);
        fused_store_act(acc, net.b1, col0, h1);
    }
    __syncthreads();
    if (mlp) {
        fused_layer<kFW>(h1, kHS, net.w2, col0, acc);
        fused_store_act(acc, net.b2, col0, h0);  // h0's last reads (layer 2) ended at the sync above
    }
    __syncthreads();
    // 4. output layer: rows [16w, 16w+16), 4 real columns of 16
    if (w < 4) {
        const int row = lane & 15, kb = (lane >> 4) * 8;
        f32x4 o = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < kFW; k0 += 32) {
            const bf16x8 fa = *reinterpret_cast<const bf16x8 *>(h0 + (w * 16 + row) * kHS + k0 + kb);
            bf16x8 fb;
            if (row < SPH_NN_OUT) {
                fb = *reinterpret_cast<const bf16x8 *>(net.w3 + (size_t)row * kFW + k0 + kb);
            } else {
#pragma unroll
                for (int q = 0; q < 8; q++) fb[q] = (bf16)0.0f;
            }
            o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, o, 0, 0, 0);
        }
        const int col = lane & 15, rb = (lane >> 4) * 4;
        if (col < SPH_NN_OUT) {
            const float bc = net.b3[col];
#pragma unroll
            for (int r = 0; r < 4; r++) sY[w * 16 + rb + r][col] = o[r] + bc;
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t k = base + threadIdx.x;
        if (k < n0)
            nn_apply_one(kp, st, k, sY[threadIdx.x][0], sY[threadIdx.x][1], sY[threadIdx.x][2],
                         sY[threadIdx.x][3], ap, &info->flags);
    }
}

hipError_t launch_nn_fused(sph_ctx *c, const sph_mlp &m, const sph_soa &st, uint32_t n,
                           const sph_nn_scales &s, float dv_scale, float dr_scale, float dt4,
                           float rho_tol, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const NnScales sc{s.inv_len, s.inv_vel, s.rho_ref, s.inv_rho};
    const FusedNet net{(const bf16 *)m.wb[0], (const bf16 *)m.wb[1], (const bf16 *)m.wb[2],
                       (const bf16 *)m.wb[3], m.b[0], m.b[1], m.b[2], m.b[3]};
    const NnApply ap{dv_scale, dr_scale, dt4, rho_tol};
    // tiles over all n: rows past the label-0 prefix are zero and not applied
    hipLaunchKernelGGL(k_nn_fused, dim3((n + 63) / 64), dim3(64 * kFusedWaves), 0, stream, c->kp,
                       sc, net,
                       c->pos4, c->vel4, c->keys_sorted, c->cell_begin, c->cell_end, st, ap,
                       c->info);
    return hipGetLastError();
}

}  // namespace sph
