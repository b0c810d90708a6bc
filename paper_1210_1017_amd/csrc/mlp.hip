// Learned-surrogate kernels: the per-particle input rows gathered from the
// cell list, bfloat16 matrix-core (MFMA) GEMMs with FP32 accumulation for the
// forward and backward passes of the MLP, the element-wise pieces around them
// (bias, SiLU, loss, column sums, Adam), training targets, the application of
// a prediction to the state, the error of a surrogate state against plain SPH,
// and the persistent network kernel of the advance (weights in registers).
#include "sph_device.h"

namespace sph {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNnSlots = SPH_NN_SLOTS;       // neighbour slots per row
constexpr int kNnIn = SPH_NN_IN;             // 64 * 8 + 32
constexpr int kNnUnroll = 8;                 // candidates loaded together in the distance test
constexpr int kNnRowThreads = 256;
constexpr uint32_t kNnRsrcWord3 = 0x00020000u;  // buffer resource: 32-bit raw dwords

struct NnScales {
    float inv_len, inv_vel, rho_ref, inv_rho, r2f, inv_acc, inv_drho, inv_dt;
};

// previous-step arrays of the sorted state (the own block's differences)
struct NnPrev {
    const float *vxp, *vyp, *vzp, *rhop;
};

typedef float nv4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float nn_kind(uint8_t t) { return t == kBoundary ? -1.0f : 1.0f; }

// ============================================================ input rows
// One lane per row (the paper's thread-per-particle mapping of Sec. 3.2).
// Row of sorted particle i: the particles j != i of the 27 cells around i's
// cell (Sec. 3.1: 9 contiguous z-runs in the x-major cell order) with FP32
// squared distance fmaf(dz,dz,fmaf(dy,dy,dx*dx)) < r2f, in increasing sorted
// index (runs and their particles are visited in that order); the first 64
// fill the slots (more found: SPH_S_NN_LIST). Pass 1 tests the candidates
// (groups of kNnUnroll buffer loads in flight) and appends (run << 12 |
// offset) entries to the lane's list in LDS; pass 2 walks the list, writes
// each slot's 8 features and sums the pressure and continuity terms of
// Sec. 2.2 for the own block and, if asked, for the FP32 rates of the row
// (pressure acceleration + g for fluid, 0 otherwise; continuity rate).
struct NnRowLds {
    uint16_t list[kNnSlots + 1][kNnRowThreads];  // + a spare row for appends to a full list
    uint32_t base[9][kNnRowThreads];
};

__device__ __forceinline__ void nn_lane_row(const KParams &kp, const NnScales &sc,
                                            const float4 *__restrict__ pos4,
                                            const float4 *__restrict__ vel4,
                                            const uint8_t *__restrict__ type,
                                            const uint32_t *__restrict__ sk,
                                            const uint32_t *__restrict__ cbeg,
                                            const uint32_t *__restrict__ cend, uint32_t n,
                                            uint32_t n0, uint32_t i, const NnPrev &pv,
                                            NnRowLds &L, bf16 *dst, size_t cstride, float4 *rate,
                                            uint32_t *flags) {
    // dst: the row's first 16-byte chunk; chunk q lies cstride chunks further
    // (1: rows are contiguous; the row count: chunk-major, chunk q of every
    // row first, so that a wave's 64 lanes store 1 KB contiguously)
    const int tid = threadIdx.x;
    bf16x8 *d8 = reinterpret_cast<bf16x8 *>(dst);
    bf16x8 zero8;
#pragma unroll
    for (int q = 0; q < 8; q++) zero8[q] = (bf16)0.0f;
    if (i >= n0 || type[i] == kGhost) {
        for (int q = 0; q < kNnIn / 8; q++) d8[q * cstride] = zero8;
        if (rate) *rate = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    const __amdgpu_buffer_rsrc_t rp =
        __builtin_amdgcn_make_buffer_rsrc((void *)pos4, 0, (int)(n * 16u), kNnRsrcWord3);
    const float4 pi = pos4[i], vi = vel4[i];
    const uint32_t cell = sk[i] & kp.cell_mask;
    const uint32_t ncz = (uint32_t)kp.ncz, ncy = (uint32_t)kp.ncy;
    const int cz = (int)(cell % ncz), cy = (int)((cell / ncz) % ncy), cx = (int)(cell / (ncz * ncy));
    const uint32_t zlo = (uint32_t)(cz > 0 ? cz - 1 : 0);
    const uint32_t zhi = (uint32_t)(cz + 1 < kp.ncz ? cz + 1 : kp.ncz - 1);
    // pass 1: distance test, list of the first 64 in sorted-index order. The
    // append has no branch: the entry is always written to the next free slot
    // (the spare row once the list is full) and only a hit advances it.
    uint32_t found = 0;
    uint16_t *const lp0 = &L.list[0][tid];
    uint16_t *const lpend = &L.list[kNnSlots][tid];
    uint16_t *lp = lp0;
    for (int col = 0; col < 9; col++) {
        const int X = cx + col / 3 - 1, Y = cy + col % 3 - 1;
        uint32_t jb = 0, je = 0;
        if (X >= 0 && X < kp.ncx && Y >= 0 && Y < kp.ncy) {
            const uint32_t c0 = ((uint32_t)X * ncy + (uint32_t)Y) * ncz;
            jb = cbeg[c0 + zlo];
            je = cend[c0 + zhi];
        }
        if (je - jb > kRunMax + 1u) {
            atomicOr(flags, (uint32_t)SPH_S_RUN_OVERFLOW);
            je = jb + kRunMax + 1u;
        }
        L.base[col][tid] = jb;
        const uint32_t len = je - jb, voff = jb * 16u;
        for (uint32_t k0 = 0; k0 < len; k0 += kNnUnroll) {
            nv4f q[kNnUnroll];
#pragma unroll
            for (int u = 0; u < kNnUnroll; u++)  // past the run: in-bounds data or 0, masked below
                q[u] = __builtin_amdgcn_raw_buffer_load_b128(rp, voff, (int)(k0 * 16u + 16u * u), 0);
            const uint32_t lim = len - k0;  // candidates left in the run (>= 1)
#pragma unroll
            for (int u = 0; u < kNnUnroll; u++) {
                const float dx = pi.x - q[u].x, dy = pi.y - q[u].y, dz = pi.z - q[u].z;
                const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                const bool hit = (u < (int)lim) & (jb + k0 + u != i) & (r2 < sc.r2f);
                *lp = (uint16_t)(((uint32_t)col << kRunBits) + k0 + u);
                lp += (hit & (lp < lpend)) ? kNnRowThreads : 0;
                found += hit ? 1u : 0u;
            }
        }
    }
    const uint32_t listed = (uint32_t)((lp - lp0) / kNnRowThreads);
    // pass 2: slot features and the pair sums
    float apx = 0.f, apy = 0.f, apz = 0.f, dr = 0.f;
    const float inv_2h = 0.5f * kp.inv_h;
#pragma unroll 4
    for (uint32_t s = 0; s < listed; s++) {
        const uint32_t e = L.list[s][tid];
        const uint32_t j = L.base[e >> kRunBits][tid] + (e & kRunMax);
        const float4 pj = pos4[j], vj = vel4[j];
        const float ddx = pj.x - pi.x, ddy = pj.y - pi.y, ddz = pj.z - pi.z;
        const float dux = vj.x - vi.x, duy = vj.y - vi.y, duz = vj.z - vi.z;
        bf16x8 f;
        f[0] = (bf16)(ddx * sc.inv_len);
        f[1] = (bf16)(ddy * sc.inv_len);
        f[2] = (bf16)(ddz * sc.inv_len);
        f[3] = (bf16)(dux * sc.inv_vel);
        f[4] = (bf16)(duy * sc.inv_vel);
        f[5] = (bf16)(duz * sc.inv_vel);
        f[6] = (bf16)((vj.w - sc.rho_ref) * sc.inv_rho);
        f[7] = (bf16)nn_kind(type[j]);
        d8[s * cstride] = f;
        // r_ij = r_i - r_j = -d, v_ij = -du: grad W = kgrad F r_ij with
        // F = (1 - q/2)^3; the constants m kgrad are applied after the sum
        const float r2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
        const float t = fmaf(-inv_2h, __builtin_amdgcn_sqrtf(r2), 1.0f);
        const float F = t * t * t;
        const float fp = (pi.w + pj.w) * F;
        apx = fmaf(fp, ddx, apx);  // sum (P_i + P_j) F (r_j - r_i)
        apy = fmaf(fp, ddy, apy);
        apz = fmaf(fp, ddz, apz);
        dr = fmaf(F, fmaf(duz, ddz, fmaf(duy, ddy, dux * ddx)), dr);  // sum F v_ij . r_ij
    }
    for (uint32_t s = listed; s < (uint32_t)kNnSlots; s++) d8[s * cstride] = zero8;
    if (found > (uint32_t)kNnSlots) atomicOr(flags, (uint32_t)SPH_S_NN_LIST);
    // ap = -m kgrad sum (P_i + P_j) F r_ij = m kgrad sum (P_i + P_j) F (r_j - r_i);
    // dr = m kgrad sum F v_ij . r_ij = m kgrad sum F (u_j - u_i) . (r_j - r_i)
    const float mk = kp.mass * kp.kgrad;
    if (rate) {
        const bool fl = type[i] == kFluid;
        *rate = make_float4(fl ? fmaf(mk, apx, kp.gx) : 0.f, fl ? fmaf(mk, apy, kp.gy) : 0.f,
                            fl ? fmaf(mk, apz, kp.gz) : 0.f, mk * dr);
    }
    bf16x8 o0 = zero8, o1 = zero8;
    o0[0] = (bf16)((vi.w - sc.rho_ref) * sc.inv_rho);
    o0[1] = (bf16)(vi.x * sc.inv_vel);
    o0[2] = (bf16)(vi.y * sc.inv_vel);
    o0[3] = (bf16)(vi.z * sc.inv_vel);
    o0[4] = (bf16)((float)found * (1.0f / 64.0f));
    o0[5] = (bf16)nn_kind(type[i]);
    o0[6] = (bf16)(mk * apx * sc.inv_acc);
    o0[7] = (bf16)(mk * apy * sc.inv_acc);
    o1[0] = (bf16)(mk * apz * sc.inv_acc);
    o1[1] = (bf16)(mk * dr * sc.inv_drho);
    if (sc.inv_dt != 0.0f) {  // previous-step differences (uniform: a scale of the launch)
#pragma clang fp contract(off)
        o1[2] = (bf16)((vi.x - pv.vxp[i]) * sc.inv_dt * sc.inv_acc);
        o1[3] = (bf16)((vi.y - pv.vyp[i]) * sc.inv_dt * sc.inv_acc);
        o1[4] = (bf16)((vi.z - pv.vzp[i]) * sc.inv_dt * sc.inv_acc);
        o1[5] = (bf16)((vi.w - pv.rhop[i]) * sc.inv_dt * sc.inv_drho);
    }
    d8[(kNnSlots + 0) * cstride] = o0;
    d8[(kNnSlots + 1) * cstride] = o1;
    d8[(kNnSlots + 2) * cstride] = zero8;
    d8[(kNnSlots + 3) * cstride] = zero8;
}

// rows[r] (or r) for r < nrows, one lane each; row-major X (chunk_major = 0)
// or chunk-major X (chunk q of row r at chunk q * nrows + r)
__global__ __launch_bounds__(kNnRowThreads) void k_nn_features(
    KParams kp, NnScales sc, const float4 *__restrict__ pos4, const float4 *__restrict__ vel4,
    const uint8_t *__restrict__ type, const uint32_t *__restrict__ sk,
    const uint32_t *__restrict__ cbeg, const uint32_t *__restrict__ cend, uint32_t n,
    DevInfo *__restrict__ info, const int32_t *__restrict__ rows, uint32_t nrows,
    bf16 *__restrict__ X, int chunk_major, float4 *__restrict__ rates, NnPrev pv) {
    __shared__ NnRowLds L;
    const uint32_t r = xcd_block(blockIdx.x, gridDim.x) * kNnRowThreads + threadIdx.x;
    if (r >= nrows) return;
    const uint32_t i = rows ? (uint32_t)rows[r] : r;
    bf16 *dst = chunk_major ? X + (size_t)r * 8 : X + (size_t)r * kNnIn;
    nn_lane_row(kp, sc, pos4, vel4, type, sk, cbeg, cend, n, info->n_label[0], i, pv, L, dst,
                chunk_major ? (size_t)nrows : 1, rates ? rates + r : nullptr, &info->flags);
}

static NnScales nn_scales(const sph_nn_scales &s) {
    return NnScales{s.inv_len, s.inv_vel, s.rho_ref, s.inv_rho,
                    s.r2f,     s.inv_acc, s.inv_drho, s.inv_dt};
}

hipError_t launch_nn_features(sph_ctx *c, const sph_soa &sorted, const int32_t *rows,
                              uint32_t nrows, const sph_nn_scales &s, void *X, int chunk_major,
                              float *rates, hipStream_t st) {
    if (nrows == 0) return hipSuccess;
    const uint32_t n = c->sorted_n;
    hipLaunchKernelGGL(k_nn_features, dim3((nrows + kNnRowThreads - 1) / kNnRowThreads),
                       dim3(kNnRowThreads), 0, st, c->kp, nn_scales(s), c->pos4, c->vel4,
                       sorted.type, c->keys_sorted, c->cell_begin, c->cell_end, n, c->info, rows,
                       nrows, (bf16 *)X, chunk_major, (float4 *)rates,
                       NnPrev{sorted.vxp, sorted.vyp, sorted.vzp, sorted.rhop});
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
// SiLU z sigma(z) with the hardware exp2 and reciprocal (about 1 ulp each):
// sigma(z) = 1 / (1 + 2^(-z log2 e)); for z -> -inf the reciprocal of inf is
// 0, so SiLU -> -0 as it should.
__device__ __forceinline__ float sigmoid_fast(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.44269504f * z));
}
__device__ __forceinline__ float silu(float z) { return z * sigmoid_fast(z); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = sigmoid_fast(z);
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
                                                    uint32_t nrows,
                                                    const float4 *__restrict__ rates, float span,
                                                    float inv_dv, float inv_dr,
                                                    float *__restrict__ T) {
#pragma clang fp contract(off)
    const uint32_t r = blockIdx.x * 256 + threadIdx.x;
    if (r >= nrows) return;
    const uint32_t k = rows ? (uint32_t)rows[r] : r;
    const int32_t q = where_b[a.id[k]];
    const float4 rt = rates ? rates[r] : make_float4(0.f, 0.f, 0.f, 0.f);
    T[4 * r + 0] = ((b.vx[q] - a.vx[k]) - span * rt.x) * inv_dv;
    T[4 * r + 1] = ((b.vy[q] - a.vy[k]) - span * rt.y) * inv_dv;
    T[4 * r + 2] = ((b.vz[q] - a.vz[k]) - span * rt.z) * inv_dv;
    T[4 * r + 3] = ((b.rho[q] - a.rho[k]) - span * rt.w) * inv_dr;
}

hipError_t launch_nn_targets(const sph_soa &a, const sph_soa &b, const int32_t *where_b,
                             const int32_t *rows, uint32_t nrows, const float *rates, float span,
                             float inv_dv, float inv_dr, float *T, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_nn_targets, grid1(nrows), dim3(256), 0, s, a, b, where_b, rows, nrows,
                       (const float4 *)rates, span, inv_dv, inv_dr, T);
    return hipGetLastError();
}

struct NnApply {
    float dv_scale, dr_scale, dt4, rho_tol;
    int carry;  // SPH_NN_CARRY_PREV: keep each previous-step difference
};

// Applies output (y0..y3) and the row's rates rt (zeros: none) to sorted
// particle k: see sph_nn_apply.
__device__ __forceinline__ void nn_apply_one(const KParams &kp, const sph_soa &st, uint32_t k,
                                             float y0, float y1, float y2, float y3, float4 rt,
                                             const NnApply &ap, uint32_t *flags) {
    const uint8_t t = st.type[k];
    if (t == kGhost) return;
    // rho + dt4 rate + y scale: with no rates (rt = 0) the inner FMA is exact
    // and the result one rounding of rho + y scale
    const float dr = fmaf(ap.dt4, rt.w, y3 * ap.dr_scale);
    const float rho = st.rho[k];
    const float rn = fmaf(y3, ap.dr_scale, fmaf(ap.dt4, rt.w, rho));
    st.rhop[k] = ap.carry ? rn - (rho - st.rhop[k]) : rn - 0.25f * dr;
    st.rho[k] = rn;
    bool ok = isfinite(rn) && fabsf(rn * kp.inv_rho0 - 1.0f) <= ap.rho_tol;
    if (t == kFluid) {
        float *pos[3] = {st.x, st.y, st.z};
        float *vel[3] = {st.vx, st.vy, st.vz};
        float *velp[3] = {st.vxp, st.vyp, st.vzp};
        const float y[3] = {y0, y1, y2};
        const float b[3] = {rt.x, rt.y, rt.z};
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const float v = vel[d][k];
            const float dv = fmaf(ap.dt4, b[d], y[d] * ap.dv_scale);
            const float vn = fmaf(y[d], ap.dv_scale, fmaf(ap.dt4, b[d], v));
            const float xn = pos[d][k] + ap.dt4 * 0.5f * (v + vn);
            pos[d][k] = xn;
            vel[d][k] = vn;
            velp[d][k] = ap.carry ? vn - (v - velp[d][k]) : vn - 0.25f * dv;
            ok = ok && isfinite(vn) && isfinite(xn);
        }
    }
    if (!ok) atomicOr(flags, (uint32_t)SPH_S_NN_RANGE);
}

__global__ __launch_bounds__(256) void k_nn_apply(KParams kp, sph_soa st,
                                                  const float *__restrict__ Y,
                                                  const float4 *__restrict__ rates,
                                                  uint32_t nrows, NnApply ap,
                                                  DevInfo *__restrict__ info) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= nrows || k >= info->n_label[0]) return;
    const float4 rt = rates ? rates[k] : make_float4(0.f, 0.f, 0.f, 0.f);
    nn_apply_one(kp, st, k, Y[4 * k], Y[4 * k + 1], Y[4 * k + 2], Y[4 * k + 3], rt, ap,
                 &info->flags);
}

hipError_t launch_nn_apply(sph_ctx *c, const sph_soa &st, const float *Y, const float *rates,
                           uint32_t nrows, float dv_scale, float dr_scale, float dt4,
                           float rho_tol, int carry, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    const NnApply ap{dv_scale, dr_scale, dt4, rho_tol, carry};
    hipLaunchKernelGGL(k_nn_apply, grid1(nrows), dim3(256), 0, s, c->kp, st, Y,
                       (const float4 *)rates, nrows, ap, c->info);
    return hipGetLastError();
}

// Training noise (see sph_nn_perturb): murmur3's 32-bit finaliser as a
// counter-based generator, one value per (seed, particle, component).
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ float noise_u(uint32_t seed, uint32_t k, uint32_t c) {
    const uint32_t h = fmix32(seed ^ fmix32(4u * k + c + 0x9e3779b9u));
    return (float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f;  // uniform in [-1, 1)
}

__global__ __launch_bounds__(256) void k_nn_perturb(sph_soa st, uint32_t n, uint32_t seed,
                                                    float au, float ar) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n || st.type[k] != kFluid) return;
    float *v[3] = {st.vx, st.vy, st.vz};
    float *vp[3] = {st.vxp, st.vyp, st.vzp};
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const float e = au * noise_u(seed, k, (uint32_t)d);
        v[d][k] += e;
        vp[d][k] += e;
    }
    const float e = ar * noise_u(seed, k, 3u);
    st.rho[k] += e;
    st.rhop[k] += e;
}

hipError_t launch_nn_perturb(const sph_soa &st, uint32_t n, uint32_t seed, float sigma_u,
                             float sigma_rho, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const float k3 = 1.7320508f;  // a uniform on [-a, a) has standard deviation a / sqrt(3)
    hipLaunchKernelGGL(k_nn_perturb, grid1(n), dim3(256), 0, s, st, n, seed, k3 * sigma_u,
                       k3 * sigma_rho);
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

// ============================================ network + application kernel
// Persistent: one workgroup (8 waves) per CU walks the tiles of 64
// consecutive rows of a chunk-major X (rows of sorted particles
// base .. base + 63). Wave w owns output columns [16w, 16w+16) of the three
// hidden layers and keeps its weight fragments (the B operands of
// v_mfma_f32_16x16x32_bf16: 16 bytes of a weight row per lane, k step and
// 16-column block) in registers for the whole kernel, so the layers read
// only LDS. Per tile:
//  1. the tile, prefetched into registers during the previous tile, is
//     stored into LDS [64][kXS] (1 KB contiguous per chunk and tile);
//  2. layer 1 (544 -> 128) for all 64 rows of the wave's columns; bias +
//     SiLU to bfloat16 into LDS (ping-pong tiles inside the input tile's
//     space), layers 2 and 3 (128 -> 128) likewise;
//  3. layer 4 (128 -> 4, output columns padded to 16): one row block per
//     wave w < 4, written to Y (FP32 [nrows][4]); k_nn_apply applies Y to the
//     state afterwards (its loads and stores then overlap freely instead of
//     holding up the tile loop).
constexpr int kFW = 128;          // hidden width of this kernel
constexpr int kXS = kNnIn + 8;    // padded row of the input tile (bfloat16)
constexpr int kHS = kFW + 8;      // padded row of a hidden activation tile
constexpr int kMlpWaves = 8;
constexpr int kMlpCols = kFW / kMlpWaves;   // 16 output columns per wave
constexpr int kMlpCB = kMlpCols / 16;       // 16-column MFMA blocks per wave
constexpr int kMlpThreads = 64 * kMlpWaves;
constexpr int kChunks = kNnIn / 8;                                  // 16-byte chunks per row
constexpr int kPref = (64 * kChunks + kMlpThreads - 1) / kMlpThreads;  // chunks per thread

struct FusedNet {
    const bf16 *w0, *w1, *w2, *w3;
    const float *b0, *b1, *b2, *b3;
};

// acc[rb][cb] = A(LDS rows 16 rb.., row stride lda) x B fragments wb[cb][ks]
template <int KS>
__device__ __forceinline__ void mlp_layer(const bf16 *sA, int lda,
                                          const bf16x8 (&wb)[kMlpCB][KS],
                                          f32x4 (&acc)[4][kMlpCB]) {
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kb = (lane >> 4) * 8;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < kMlpCB; c++) acc[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ks++) {
#pragma unroll
        for (int a = 0; a < 4; a++) {
            const bf16x8 fa =
                *reinterpret_cast<const bf16x8 *>(sA + (a * 16 + row) * lda + ks * 32 + kb);
#pragma unroll
            for (int c = 0; c < kMlpCB; c++)
                acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, wb[c][ks], acc[a][c], 0, 0, 0);
        }
    }
}

// bias + SiLU of the wave's 64 x 32 slab (cols col0..) into an LDS tile
__device__ __forceinline__ void mlp_store_act(const f32x4 (&acc)[4][kMlpCB],
                                              const float (&bias)[kMlpCB], int col0, bf16 *sH) {
    const int lane = threadIdx.x & 63;
    const int rb = (lane >> 4) * 4;
#pragma unroll
    for (int c = 0; c < kMlpCB; c++) {
        const int col = col0 + c * 16 + (lane & 15);
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                sH[(a * 16 + rb + r) * kHS + col] = (bf16)silu(acc[a][c][r] + bias[c]);
    }
}

// Workgroup barrier that waits for this wave's LDS operations only: unlike
// __syncthreads() it leaves the next tile's global prefetch loads in flight.
// The memory clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int KS>
__device__ __forceinline__ void load_frags(const bf16 *__restrict__ W, int ncols_real, int col,
                                           bf16x8 (&wb)[KS]) {
    const int kb = ((threadIdx.x & 63) >> 4) * 8;
#pragma unroll
    for (int ks = 0; ks < KS; ks++) {
        if (col < ncols_real) {
            wb[ks] = *reinterpret_cast<const bf16x8 *>(W + (size_t)col * (KS * 32) + ks * 32 + kb);
        } else {
#pragma unroll
            for (int q = 0; q < 8; q++) wb[ks][q] = (bf16)0.0f;
        }
    }
}

__global__ __launch_bounds__(kMlpThreads, 1) void k_nn_mlp(FusedNet net,
                                                            const bf16 *__restrict__ X,
                                                            uint32_t nrows,
                                                            float *__restrict__ Y) {
    __shared__ __attribute__((aligned(16))) bf16 sX[64 * kXS];
    const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t ntiles = (nrows + 63) / 64;
    const int col0 = (int)w * kMlpCols;
    // weight fragments and biases of this wave, for the whole kernel
    bf16x8 wb0[kMlpCB][kNnIn / 32], wb1[kMlpCB][kFW / 32], wb2[kMlpCB][kFW / 32];
    bf16x8 wb3[1][kFW / 32];
    float bias0[kMlpCB], bias1[kMlpCB], bias2[kMlpCB];
#pragma unroll
    for (int c = 0; c < kMlpCB; c++) {
        const int col = col0 + c * 16 + (int)(lane & 15);
        load_frags<kNnIn / 32>(net.w0, kFW, col, wb0[c]);
        load_frags<kFW / 32>(net.w1, kFW, col, wb1[c]);
        load_frags<kFW / 32>(net.w2, kFW, col, wb2[c]);
        bias0[c] = net.b0[col];
        bias1[c] = net.b1[col];
        bias2[c] = net.b2[col];
    }
    load_frags<kFW / 32>(net.w3, SPH_NN_OUT, (int)(lane & 15), wb3[0]);
    const float bias3 = (lane & 15) < SPH_NN_OUT ? net.b3[lane & 15] : 0.0f;
    bf16x8 pf[kPref];
    auto prefetch = [&](uint32_t tile) {
        const uint32_t base = tile * 64;
#pragma unroll
        for (int e = 0; e < kPref; e++) {
            const int c = e * kMlpThreads + (int)threadIdx.x;  // chunk-major: row = c % 64
            const int q = c / 64, row = c % 64;
            if (c < 64 * kChunks && base + row < nrows) {
                pf[e] = *reinterpret_cast<const bf16x8 *>(X + ((size_t)q * nrows + base + row) * 8);
            } else {
#pragma unroll
                for (int k = 0; k < 8; k++) pf[e][k] = (bf16)0.0f;
            }
        }
    };
    uint32_t tile = blockIdx.x;
    if (tile < ntiles) prefetch(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const uint32_t base = tile * 64;
#pragma unroll
        for (int e = 0; e < kPref; e++) {
            const int c = e * kMlpThreads + (int)threadIdx.x;
            if (c < 64 * kChunks)
                *reinterpret_cast<bf16x8 *>(sX + (c % 64) * kXS + (c / 64) * 8) = pf[e];
        }
        lds_barrier();
        if (tile + gridDim.x < ntiles) prefetch(tile + gridDim.x);
        bf16 *h0 = sX, *h1 = sX + 64 * kHS;
        f32x4 acc[4][kMlpCB];
        mlp_layer<kNnIn / 32>(sX, kXS, wb0, acc);
        lds_barrier();  // every wave is done reading the input tile
        mlp_store_act(acc, bias0, col0, h0);
        lds_barrier();
        mlp_layer<kFW / 32>(h0, kHS, wb1, acc);
        mlp_store_act(acc, bias1, col0, h1);
        lds_barrier();
        mlp_layer<kFW / 32>(h1, kHS, wb2, acc);
        mlp_store_act(acc, bias2, col0, h0);  // h0's last reads (layer 2) ended at the barrier above
        lds_barrier();
        if (w < 4) {
            const int row = lane & 15, kb = (lane >> 4) * 8;
            f32x4 o = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < kFW / 32; ks++) {
                const bf16x8 fa =
                    *reinterpret_cast<const bf16x8 *>(h0 + (w * 16 + row) * kHS + ks * 32 + kb);
                o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, wb3[0][ks], o, 0, 0, 0);
            }
            const int col = lane & 15, rb = (lane >> 4) * 4;
            if (col < SPH_NN_OUT) {
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const uint32_t k = base + w * 16 + rb + r;
                    if (k < nrows) Y[4 * (size_t)k + col] = o[r] + bias3;
                }
            }
        }
        lds_barrier();  // sX is rewritten for the next tile
    }
}

hipError_t launch_nn_mlp_apply(sph_ctx *c, const sph_mlp &m, const sph_soa &st, const void *X,
                               float *Y, const float *rates, uint32_t nrows, float dv_scale,
                               float dr_scale, float dt4, float rho_tol, int carry,
                               hipStream_t stream) {
    if (nrows == 0) return hipSuccess;
    const FusedNet net{(const bf16 *)m.wb[0], (const bf16 *)m.wb[1], (const bf16 *)m.wb[2],
                       (const bf16 *)m.wb[3], m.b[0], m.b[1], m.b[2], m.b[3]};
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const uint32_t ntiles = (nrows + 63) / 64;
    const uint32_t grid = ntiles < (uint32_t)cus ? ntiles : (uint32_t)cus;
    hipLaunchKernelGGL(k_nn_mlp, dim3(grid), dim3(kMlpThreads), 0, stream, net, (const bf16 *)X,
                       nrows, Y);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_nn_apply(c, st, Y, rates, nrows, dv_scale, dr_scale, dt4, rho_tol, carry,
                           stream);
}

}  // namespace sph
