// Internal declarations shared by the HIP translation units of libsph.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "sph.h"

namespace sph {

enum : uint8_t { kFluid = 0, kBoundary = 1, kGhost = 2 };

#ifndef SPH_SORT_ITEMS
#define SPH_SORT_ITEMS 8
#endif
constexpr int kSortThreads = 256;
constexpr int kSortItems = SPH_SORT_ITEMS;  // keys per thread of a radix tile
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per radix tile
constexpr int kInteractThreads = 256;
// Incremental sort: when at most kIncCap particles change their key between
// two sorts, one block sorts them and the merge places every particle; up to
// mid_cap(n) (below), the movers' own radix passes sort them for the merge;
// with more, the radix passes over all keys run (kModeFull).
constexpr uint32_t kIncCap = 8192;
constexpr uint32_t kModeFull = 0u, kModeIncr = 1u, kModeMid = 2u;
constexpr int kRunBits = 12;                          // offset bits of a neighbour entry
constexpr uint32_t kRunMax = (1u << kRunBits) - 1u;

// Constants of the step in the precision the kernels use (converted once).
struct KParams {
    float ox, oy, oz, inv_cs;
    int32_t ncx, ncy, ncz, cell_bits;
    uint32_t ncells, cell_mask;
    int32_t slab_mode;
    float slab_xlo, slab_xhi;
    float h, inv_h, r2max, eta2, mass, alpha;
    float rho0, inv_rho0, B, c0;
    float gx, gy, gz;
    float kgrad;  // -5 aD / h^2, aD = 21 / (16 pi h^3): grad W = kgrad (1 - q/2)^3 r_ij
    float kgrad_cubic;  // -3 aD / (4 h^2), aD = 1 / (pi h^3): cubic spline, see k_interact
    float cfl;
    int32_t euler_every;
    int32_t options;    // SPH_O_* bits
};

// Device-resident results of the last sort / interaction.
struct DevInfo {
    uint32_t lstart[4];   // first sorted index with label >= l
    uint32_t n_label[4];
    uint32_t ranges[14];  // halo_lo, edge_lo, edge_hi, halo_hi, out_lo, out_hi, excluded
    float dt;
    uint32_t flags;
    uint32_t dtmin_bits;  // bits of the smallest per-particle dt limit (positive float)
    uint32_t pad_;
    unsigned long long dtmin64_bits;  // same in FP64 (variant paths)
    unsigned long long pairs;        // neighbour pairs of the last interaction
    unsigned long long pairs_total;  // summed over every interaction since creation
    unsigned long long cand_total;   // candidates tested, summed likewise
    uint32_t sort_mode;  // kModeFull / kModeIncr / kModeMid: the path the last plain sort took
    uint32_t movers;     // particles whose key differs from the previous sort's at their index
    uint32_t pad2_[2];
};

}  // namespace sph

struct sph_ctx {
    sph_params prm;
    sph::KParams kp;
    int device = 0;
    uint32_t capacity = 0;
    int cell_bits = 0;
    uint32_t ncells = 0;
    uint32_t max_tiles = 0;
    // scratch (device)
    uint32_t *keys_a = nullptr, *keys_b = nullptr, *keys_sorted = nullptr;
    int32_t *vals_a = nullptr, *vals_b = nullptr, *perm = nullptr;
    uint32_t *hist = nullptr;       // 256 * max_tiles, digit-major
    // incremental sort: mover bits per 64 particles, movers before each word
    // within its tile, movers per tile (then their exclusive offsets), per
    // tile its key range, then the range of sorted movers below it
    unsigned long long *mmask = nullptr;
    uint32_t *mwpre = nullptr, *mcnt = nullptr;
    uint2 *mtile = nullptr;
    // the mover plan's report to the host (pinned, mapped): movers << 1 |
    // (there was a previous sort); read without waiting to choose the kernels
    // of the next sort
    unsigned long long *fb = nullptr, *fb_dev = nullptr;
    const float *last_out_x = nullptr;  // x array the last plain sort wrote
    uint32_t *digit_tot = nullptr;  // 256
    uint32_t *cell_begin = nullptr, *cell_end = nullptr;
    float4 *pos4 = nullptr, *vel4 = nullptr;  // packed (x,y,z,p/rho^2), (vx,vy,vz,rho)
    float *rate = nullptr;                    // 4 * capacity: ax, ay, az, arho
    sph::DevInfo *info = nullptr;
    // variant paths (allocated when params.features asks for them)
    uint32_t features = 0;
    double cs64 = 0.0;
    double4 *pos8 = nullptr;      // packed (x, y, z, p/rho^2) of the sorted FP64 state
    double4 *vel8 = nullptr;      // packed (vx, vy, vz, rho) of it
    double *drate = nullptr;      // 4 * capacity FP64 rates of sph_dstep
    double *tot_part = nullptr;   // 8 doubles per totals block
    double *nn_part = nullptr;    // 8 doubles per surrogate-judge block
    double *nn_out = nullptr;     // 8 doubles: judge result
    void *nn_x = nullptr;         // surrogate input rows of sph_nn_advance (SPH_F_SURROGATE)
    float *nn_y = nullptr;        // its network outputs, 4 per row
    float *nn_rate = nullptr;     // the rows' pair-sum rates, 4 per row
    uint32_t tot_blocks = 0;
    int last_path = 0;            // 0 plain, 1 cell, 2 FP64: which state the tables describe
    bool dt_in_info = false;      // the last step was symplectic: its dt is info->dt
    // optional per-phase timing of sph_step (events: start, sorted, interacted, updated)
    hipEvent_t *events = nullptr;
    uint32_t ev_slots = 0, ev_used = 0;
    // bookkeeping
    uint32_t sorted_n = 0;
    bool have_sort = false;
    bool have_dt = false;
    std::string err;
};

namespace sph {

// sort.hip
hipError_t launch_keys(const KParams &kp, const sph_soa &in, uint32_t n, uint32_t *keys,
                       int32_t *vals, hipStream_t s);
hipError_t radix_sort(sph_ctx *c, const uint32_t *keys_in, const int32_t *vals_in,
                      uint32_t *keys_out, int32_t *vals_out, uint32_t n, int key_bits,
                      hipStream_t s, bool first_hist_done = false,
                      const uint32_t *skip_mode = nullptr);
// What the host expects of the next sort's movers, from the count of the
// last plan that has run: any number (all kernels launched, the keys kernel
// counting the first radix digit), at most kIncCap (the merge kernels only),
// or between kIncCap and mid_cap(n) (all kernels, no first-digit counts in
// the keys kernel).
enum SortExpect { kExpectAny = 0, kExpectFew = 1, kExpectMid = 2 };
hipError_t sort_state(sph_ctx *c, const sph_soa &in, const sph_soa &out, uint32_t n,
                      uint32_t nprev, int expect, bool skip_rv, hipStream_t s);
// Largest number of movers the merge takes with the movers' own radix passes
// (more: the full radix passes).
inline uint32_t mid_cap(uint32_t n) { return n / 4u; }
hipError_t radix_sort_bufs(const uint32_t *keys_in, const int32_t *vals_in, uint32_t *keys_out,
                           int32_t *vals_out, uint32_t n, int key_bits, uint32_t *ks,
                           int32_t *vs, uint32_t *hist, uint32_t *tot, hipStream_t s,
                           const uint32_t *skip = nullptr, uint32_t run_mode = 0u,
                           const uint32_t *n_dev = nullptr);
hipError_t launch_tables(sph_ctx *c, uint32_t n, hipStream_t s, bool counts = true);
hipError_t launch_pack(sph_ctx *c, const sph_soa &in, uint32_t n, hipStream_t s);
hipError_t launch_clear_flags(sph_ctx *c, hipStream_t s);

// interact.hip
hipError_t launch_interact(sph_ctx *c, const uint8_t *type, uint32_t n, const sph_rates &out,
                           hipStream_t s, hipEvent_t after_kernel = nullptr);

// variants.hip (cell + offset and FP64 paths)
struct GridD {
    double ox, oy, oz, cs;
    int32_t ncx, ncy, ncz;
};
constexpr int kTotThreads = 256;
GridD grid_d(const sph_ctx *c);
hipError_t launch_cell_from_pos(sph_ctx *c, const double *x, const double *y, const double *z,
                                const sph_cstate &out, uint32_t n, hipStream_t s);
hipError_t launch_pos_from_cell(sph_ctx *c, const sph_cstate &st, double *x, double *y,
                                double *z, uint32_t n, hipStream_t s);
hipError_t launch_keys_cell(sph_ctx *c, const sph_cstate &in, uint32_t n, hipStream_t s);
hipError_t launch_gather_cell(sph_ctx *c, const sph_cstate &in, const sph_cstate &out,
                              uint32_t n, hipStream_t s);
hipError_t launch_interact_cell(sph_ctx *c, const sph_cstate &st, uint32_t n,
                                const sph_rates &out, hipStream_t s);
hipError_t launch_update_cell(sph_ctx *c, const sph_cstate &st, const float *ax, const float *ay,
                              const float *az, const float *arho, uint32_t n, uint64_t step,
                              hipStream_t s);
hipError_t launch_totals_cell(sph_ctx *c, const sph_cstate &st, uint32_t n, double *out_host,
                              hipStream_t s);
hipError_t launch_keys_d(sph_ctx *c, const sph_dstate &in, uint32_t n, hipStream_t s);
hipError_t launch_gather_d(sph_ctx *c, const sph_dstate &in, const sph_dstate &out, uint32_t n,
                           hipStream_t s);
hipError_t launch_interact_d(sph_ctx *c, const sph_dstate &st, uint32_t n, const sph_drates &out,
                             hipStream_t s);
hipError_t launch_update_d(sph_ctx *c, const sph_dstate &st, const sph_drates &r, uint32_t n,
                           uint64_t step, hipStream_t s);
hipError_t launch_totals_d(sph_ctx *c, const sph_dstate &st, uint32_t n, double *out_host,
                           hipStream_t s);

// api.hip: record a message for sph_last_error(NULL) and return code
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// mlp.hip (learned surrogate)
constexpr int kMlpSplits = 32;  // split-K slices of a weight-gradient GEMM, at most
hipError_t launch_nn_features(sph_ctx *c, const sph_soa &sorted, const int32_t *rows,
                              uint32_t nrows, const sph_nn_scales &s, void *X, int chunk_major,
                              float *rates, hipStream_t st);
hipError_t launch_gemm(const void *A, const void *B, float *C, int M, int N, int K,
                       long long sam, long long sak, long long sbk, long long sbn, long long scm,
                       long long scn, int accumulate, float *part, hipStream_t s);
hipError_t launch_bias_act(float *Z, const float *b, void *Aout, float *Fout, long long rows,
                           int cols, int act, hipStream_t s);
hipError_t launch_act_back(const float *dA, const float *Z, void *dZ, long long n, int act,
                           hipStream_t s);
hipError_t launch_mse(const float *Y, const float *T, const float *wcol, float *dY,
                      long long rows, int cols, float *part, float *loss, hipStream_t s);
hipError_t launch_colsum(const void *dZ, long long rows, int cols, float *db, hipStream_t s);
hipError_t launch_adam(float *w, float *m, float *v, const float *g, void *wb, long long n,
                       float lr, float b1, float b2, float eps, float c1, float c2,
                       hipStream_t s);
hipError_t launch_f32_to_bf16(const float *a, void *b, long long n, hipStream_t s);
hipError_t launch_id_scatter(const int32_t *id, uint32_t n, int32_t *where, hipStream_t s);
hipError_t launch_nn_targets(const sph_soa &a, const sph_soa &b, const int32_t *where_b,
                             const int32_t *rows, uint32_t nrows, const float *rates, float span,
                             float inv_dv, float inv_dr, float *T, hipStream_t s);
hipError_t launch_nn_apply(sph_ctx *c, const sph_soa &st, const float *Y, const float *rates,
                           uint32_t nrows, float dv_scale, float dr_scale, float dt4,
                           float rho_tol, int carry, hipStream_t s);
hipError_t launch_nn_perturb(const sph_soa &st, uint32_t n, uint32_t seed, float sigma_u,
                             float sigma_rho, hipStream_t s);
hipError_t launch_nn_judge(const sph_soa &S, const sph_soa &R, const sph_soa &B,
                           const int32_t *where_r, const int32_t *where_b, uint32_t n,
                           double *part, double *out, hipStream_t s);
hipError_t launch_nn_mlp_apply(sph_ctx *c, const sph_mlp &m, const sph_soa &st, const void *X,
                               float *Y, const float *rates, uint32_t nrows, float dv_scale,
                               float dr_scale, float dt4, float rho_tol, int carry,
                               hipStream_t stream);

// update.hip
hipError_t launch_sym_half(sph_ctx *c, const sph_soa &st, const float *ax, const float *ay,
                           const float *az, const float *arho, uint32_t n, hipStream_t s);
hipError_t launch_sym_full(sph_ctx *c, const sph_soa &st, const float *ax, const float *ay,
                           const float *az, const float *arho, uint32_t n, hipStream_t s);

// machine probes (probe.hip)
hipError_t launch_probe_fma(float *out, uint32_t blocks, int iters, hipStream_t s);
hipError_t launch_probe_copy(const void *src, void *dst, uint64_t bytes, uint32_t blocks,
                             hipStream_t s);
hipError_t launch_update(sph_ctx *c, const sph_soa &st, const float *ax, const float *ay,
                         const float *az, const float *arho, uint32_t n, uint64_t step,
                         hipStream_t s, bool packed = false);

}  // namespace sph
