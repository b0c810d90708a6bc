/*
 * sph.h - C ABI of libsph.so: one weakly-compressible SPH (WCSPH) time step of
 * free-surface flow on one MI355X (gfx950) GPU, in hand-written HIP.
 *
 * The method is that of Valdez-Balderas, Dominguez, Rogers and Crespo,
 * "Towards accelerating Smoothed Particle Hydrodynamics simulations for
 * free-surface flows on multi-GPU clusters": per sub-domain, particles are
 * binned in cubic cells of side 2h and radix-sorted by cell (Sec. 3.1), the
 * pairwise sums of the SPH continuity and momentum equations are taken over
 * the 27 surrounding cells (Sec. 3.2, Sec. 2.2), and the state is advanced by
 * a second-order Verlet scheme with a CFL-limited time step (Sec. 3.3). The
 * sort key also carries the sub-domain migration label of Sec. 4.2-4.3, so
 * outgoing particles pack contiguously behind the in-domain ones, and the
 * edge and halo strips of width 2h are whole x-layers of cells, hence
 * contiguous index ranges of the sorted arrays.
 *
 * Conventions for every entry point:
 *  - Return 0 on success or a negative SPH_E_* code. Nothing aborts and no
 *    C++ exception crosses the ABI. sph_last_error() gives a message.
 *  - Particle arrays are device pointers owned by the caller (structure of
 *    arrays, FP32 unless noted). The context owns only its scratch memory,
 *    allocated once in sph_create and released in sph_destroy; no entry
 *    point allocates device memory after sph_create.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on that stream except sph_get_* (which
 *    synchronise it). One context serves one stream at a time: calls on a
 *    context must not overlap on different streams.
 *  - Units are SI. Host parameters are FP64 and are converted to FP32 once.
 *
 * Particle types (uint8): 0 fluid, 1 boundary (dynamic boundary particle,
 * Sec. 2.3: same equations, position and velocity held fixed), 2 ghost
 * (halo copy of a neighbouring sub-domain's edge, Sec. 4.2: a neighbour
 * for others, never updated itself).
 */
#ifndef SPH_H
#define SPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_ABI_VERSION 1

enum {
    SPH_OK = 0,
    SPH_E_INVALID_ARG = -1, /* null pointer, bad parameter, n out of range     */
    SPH_E_CAPACITY = -2,    /* n larger than the capacity given to sph_create   */
    SPH_E_KEY_BITS = -3,    /* cell grid needs more than 30 index bits          */
    SPH_E_HIP = -4,         /* a HIP runtime call or kernel launch failed       */
    SPH_E_STATE = -5        /* call order violated (e.g. interact before sort)  */
};

/* Status bits reported by sph_get_status (set on the device, sticky). */
enum {
    SPH_S_NONFINITE = 1u << 0,    /* non-finite position/velocity/density after an update */
    SPH_S_DT = 1u << 1,           /* dt not finite or not positive                        */
    SPH_S_RUN_OVERFLOW = 1u << 2, /* surrogate rows: a 3-cell neighbour run held more
                                     than 4096 particles (their 12-bit run offsets): the
                                     excess was skipped, results of that call invalid.
                                     The plain and the cell + offset interactions
                                     address candidates by full indices and search any
                                     run completely                                       */
    SPH_S_EXCLUDED = 1u << 3,     /* some particles lie outside the cell grid (label 3)   */
    SPH_S_NN_RANGE = 1u << 4,     /* surrogate: a result was non-finite or its density
                                     left the allowed band (sph_nn_apply, sph_nn_advance) */
    SPH_S_NN_LIST = 1u << 5       /* surrogate: a row found more than 64 neighbours within
                                     its radius; its slots and sums kept the first 64 in
                                     sorted-index order (informational)                    */
};

/* Run parameters. */
typedef struct sph_params {
    double dp;          /* lattice spacing (m)                                  */
    double h;           /* smoothing length (m); cell side is 2h (Sec. 3.1)     */
    double rho0;        /* reference density, 1000 kg/m^3 (Sec. 2.2)            */
    double gamma;       /* Tait exponent; must be 7 (Sec. 2.2)                  */
    double c0;          /* speed of sound at rho0 (m/s)                         */
    double alpha;       /* artificial-viscosity coefficient (Sec. 2.2)          */
    double eta_over_h;  /* eta / h in the viscosity denominator, 0.1 (Sec. 2.2) */
    double cfl;         /* CFL number of the time step (Sec. 3.3)               */
    double mass;        /* particle mass (kg), the same for every particle      */
    double g[3];        /* gravity (m/s^2)                                      */
    double origin[3];   /* lower corner of the cell grid (m)                    */
    int32_t ncell[3];   /* cells per axis (grid incl. halo / margin layers)     */
    int32_t euler_every;/* Verlet: an Euler step every this many steps (40)     */
    int32_t slab_mode;  /* 1: sub-domain [slab_xlo, slab_xhi) with migration
                           labels; the grid must then run from slab_xlo - 2h
                           and hold (slab_xhi - slab_xlo)/2h + 2 x-layers       */
    int32_t options;    /* SPH_O_* bits: variants of the plain FP32 step (0 for
                           the Wendland kernel and no density floor)          */
    double slab_xlo, slab_xhi;
    uint32_t capacity;  /* maximum particle count of any call, < 2^28           */
    uint32_t features;  /* SPH_F_* bits: extra scratch for the variant paths    */
} sph_params;

/* Option bits of sph_params.options. They change what sph_interact,
 * sph_update and sph_step compute; the cell, FP64 and surrogate entry points
 * keep the Wendland kernel and reject a context created with options != 0
 * (SPH_E_INVALID_ARG).
 *   SPH_O_CUBIC      the cubic spline kernel of Sec. 2.2 (support 2h):
 *                    W = aD (1 - 3q^2/2 + 3q^3/4) for q < 1, aD (2 - q)^3 / 4
 *                    for 1 <= q < 2, aD = 1/(pi h^3), q = r/h;
 *   SPH_O_RHO_FLOOR  a boundary particle's density is raised to rho0 after
 *                    each update when it falls below (dynamic boundaries of
 *                    Sec. 2.3; a common practice, not in the paper);
 *   SPH_O_SYMPLECTIC sph_step integrates with a symplectic kick-drift
 *                    position-Verlet scheme instead of the Verlet scheme of
 *                    Sec. 3.3: with dt from the rates at n, a half step
 *                    r + dt/2 v, v + dt/2 a, rho + dt/2 D, the rates of that
 *                    half state (same cell tables), then v' = v + dt a_h,
 *                    r' = r + dt (v + v')/2, rho' = rho (2 - e)/(2 + e) with
 *                    e = -(D_h/rho_h) dt. Two interactions per step;
 *                    sph_update is then refused (SPH_E_STATE). */
enum {
    SPH_O_CUBIC = 1u << 0,
    SPH_O_RHO_FLOOR = 1u << 1,
    SPH_O_SYMPLECTIC = 1u << 2
};

/* Feature bits of sph_params.features. */
enum {
    SPH_F_CELL = 1u << 0, /* cell + offset position path (sph_cstate, sph_c*);
                             capacity below 2^27                                */
    SPH_F_FP64 = 1u << 1, /* FP64 reference path (sph_dstate, sph_d*)          */
    SPH_F_SURROGATE = 1u << 2 /* rows, outputs and rates of sph_nn_advance:
                                 capacity x (SPH_NN_IN x 2 + 32) bytes         */
};

/* Structure-of-arrays particle state; every pointer is a device array of
 * at least n elements. v*p / rhop are the Verlet "previous" values. */
typedef struct sph_soa {
    float *x, *y, *z;
    float *vx, *vy, *vz;
    float *rho;
    float *vxp, *vyp, *vzp;
    float *rhop;
    uint8_t *type;
    int32_t *id;
} sph_soa;

/* Time derivatives from the interaction (device arrays of >= n elements).
 * press, nu and npair are optional (NULL: not written). */
typedef struct sph_rates {
    float *ax, *ay, *az; /* dv/dt (fluid; 0 for boundary and ghost)      */
    float *arho;         /* drho/dt (fluid and boundary; 0 for ghost)    */
    float *press;        /* Tait pressure p_i (all in-domain particles)  */
    float *nu;           /* max_j |h v_ij.r_ij / (r_ij^2 + eta^2)|        */
    uint32_t *npair;     /* number of neighbours j of i                  */
} sph_rates;

/* Label counts and packing ranges of the last sort. Ranges are [first, end)
 * indices of the sorted arrays. Layers are x-layers of cells: halo_lo = layer
 * 0, edge_lo = layer 1, edge_hi = layer ncx-2, halo_hi = layer ncx-1 (in slab
 * mode: the incoming ghost strips and the outgoing edge strips, Sec. 4.2). */
typedef struct sph_counts {
    uint32_t n_label[4]; /* 0 in domain, 1 moved left, 2 moved right, 3 outside grid */
    uint32_t halo_lo[2];
    uint32_t edge_lo[2];
    uint32_t edge_hi[2];
    uint32_t halo_hi[2];
    uint32_t out_lo[2];   /* label-1 range */
    uint32_t out_hi[2];   /* label-2 range */
    uint32_t excluded[2]; /* label-3 range */
} sph_counts;

typedef struct sph_ctx sph_ctx;

/* Library ABI version (SPH_ABI_VERSION). */
int sph_abi_version(void);

/* Message for a return code. Never NULL. */
const char *sph_error_string(int code);

/* Last error message recorded on ctx (empty string if none); ctx may be NULL
 * for errors of sph_create and of the machine probes. The pointer stays valid
 * until the next call. */
const char *sph_last_error(const sph_ctx *ctx);

/* Validate params, bind the current HIP device and allocate all scratch for
 * params->capacity particles (keys, values, radix histograms, cell tables,
 * packed interaction inputs, rates, dt partials). On success *out receives
 * the context. Errors: INVALID_ARG (bad params), KEY_BITS (grid needs more
 * than 30 cell bits: label bits would not fit a uint32 key), HIP (allocation). */
int sph_create(const sph_params *params, sph_ctx **out);

/* Free the context and its scratch (waits for the device). NULL is a no-op. */
void sph_destroy(sph_ctx *ctx);

/* Bits of the linear cell index (smallest b with 2^b >= cells); keys are
 * label << bits | cell. */
int sph_cell_bits(const sph_ctx *ctx);

/* Stable key-value LSD radix sort of n (uint32 key, int32 value) pairs on the
 * low key_bits bits (1..32), 8-bit digits (Sec. 3.1 and 4.3: the paper's
 * radix sort; equal keys keep their input order, as in the worked example of
 * Sec. 4.3). Inputs are not modified; outputs must not alias inputs. */
int sph_sort_kv(sph_ctx *ctx, const uint32_t *keys, const int32_t *vals, uint32_t *keys_out,
                int32_t *vals_out, uint32_t n, int key_bits, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * stable sort as sph_sort_kv, bit-identical results, without a context. Its
 * scratch (one key/value ping-pong pair and the radix histograms, about
 * 17 MB) is a fixed device array of the library, which every GPU it runs on
 * holds until the process ends; the call allocates nothing. n is at most
 * SPH_SORT_NOALLOC_MAX: larger n fails with SPH_E_CAPACITY. Every call on one
 * GPU uses that GPU's single array, so calls that overlap on one GPU (on
 * different streams or host threads) race and must be serialised by the
 * caller. Runs on the current HIP device; errors are reported through
 * sph_last_error(NULL). n = 0 does nothing. */
#define SPH_SORT_NOALLOC_MAX (1u << 21)
int sph_sort_kv_noalloc(const uint32_t *keys, const int32_t *vals, uint32_t *keys_out,
                        int32_t *vals_out, uint32_t n, int key_bits, void *stream);

/* Sort step (Sec. 3.1, 4.2-4.3): cell key + migration label per particle,
 * stable sort by key, reorder of every SoA array of `in` into `out`, cell
 * begin/end tables over the label-0 prefix (an empty cell c has
 * begin = end = first index with cell >= c), label counts and packing ranges.
 * `in` and `out` must not share arrays.
 * The stable order is unique, and it is found one of three ways, chosen on
 * the device: when at most n / 4 particles have a key that differs from the
 * key the previous sort on ctx (any path) left at their index (the "movers",
 * e.g. a state that the previous step wrote, moved by one step, with
 * migrants), the movers alone are sorted (by one block up to 8192, by their
 * own radix passes above) and merged with the others, which keep their
 * order; otherwise (a first sort, an unrelated state, many movers) the full
 * radix sort runs. All give the same bits. */
int sph_sort(sph_ctx *ctx, const sph_soa *in, sph_soa *out, uint32_t n, void *stream);

/* Interaction (Sec. 3.2, equations of Sec. 2.2, boundaries of Sec. 2.3) on the
 * state that the last sph_sort on ctx wrote (same n, unmodified since):
 * rates for every in-domain particle, the neighbour-pair count and the CFL
 * time step (Sec. 3.3), which stays on the device (sph_get_dt). */
int sph_interact(sph_ctx *ctx, const sph_soa *sorted, uint32_t n, const sph_rates *out,
                 void *stream);

/* Verlet update (Sec. 3.3) of the in-domain particles of `sorted` in place,
 * with the rates in `rates` and the dt of the last sph_interact. `step` is
 * the step counter (an Euler step when step % euler_every == 0). Refused
 * (SPH_E_STATE) on a context with SPH_O_SYMPLECTIC. */
int sph_update(sph_ctx *ctx, sph_soa *sorted, const sph_rates *rates, uint32_t n,
               uint64_t step, void *stream);

/* One whole time step: sph_sort(cur -> next), interaction into the context's
 * own rate buffers, dt, Verlet update of next (with SPH_O_SYMPLECTIC: the
 * half step, a second interaction and the full step instead). On return
 * `next` holds the new state (sorted); `cur` is left as it was. No host
 * synchronisation. */
int sph_step(sph_ctx *ctx, const sph_soa *cur, sph_soa *next, uint32_t n, uint64_t step,
             void *stream);

/* Readbacks (synchronise `stream`). */
int sph_get_counts(sph_ctx *ctx, sph_counts *out, void *stream);
int sph_get_dt(sph_ctx *ctx, float *dt, void *stream);
int sph_get_pairs(sph_ctx *ctx, uint64_t *pairs, void *stream);
/* The last plain sort (sph_sort, sph_step): its movers (particles whose key
 * differed from the previous sort's at their index) and the path it took:
 * 0 the radix sort of all keys, 1 the mover merge with the movers sorted by
 * one block (at most 8192 of them, or any number when the host expected few),
 * 2 the mover merge with the movers sorted by their own radix passes (more
 * than 8192, at most n / 4). SPH_E_STATE when the last sort was a variant
 * path's. */
int sph_get_sort_stats(sph_ctx *ctx, uint32_t *movers, uint32_t *merged, void *stream);
int sph_get_status(sph_ctx *ctx, uint32_t *flags, void *stream);
/* Clear the status bits (a kernel on the stream; no host synchronisation). */
int sph_clear_status(sph_ctx *ctx, void *stream);
/* Neighbour pairs summed over every interaction since sph_create. */
int sph_get_pair_total(sph_ctx *ctx, uint64_t *pairs, void *stream);
/* Candidates (particles of the 27 cells) given the support test, summed over
 * every interaction since sph_create. */
int sph_get_candidate_total(sph_ctx *ctx, uint64_t *cands, void *stream);

/* Optional phase timing of sph_step with HIP events recorded on the step's
 * stream (no host synchronisation inside the steps). sph_timing_begin creates
 * 4 events for each of the next max_steps (<= 65536) calls of sph_step
 * (0 switches timing off); these are runtime event objects, not device
 * memory. sph_timing_read waits for the recorded steps and writes, per step,
 * 3 durations in ms: sort (keys, radix passes, tables, reorder), interaction
 * kernel, and dt reduction + Verlet update. *count receives the number of
 * steps written. */
int sph_timing_begin(sph_ctx *ctx, uint32_t max_steps);
int sph_timing_read(sph_ctx *ctx, float *ms, uint32_t max_steps, uint32_t *count);

/* Device-to-device copies of the last sort's sorted keys (n of them) and
 * of the cell tables (ncells each) into caller buffers. */
int sph_copy_keys(sph_ctx *ctx, uint32_t *keys_out, uint32_t n, void *stream);
int sph_copy_cell_tables(sph_ctx *ctx, uint32_t *begin_out, uint32_t *end_out, void *stream);

/* ---------------------------------------------------------------------------
 * Machine probes (no context). The published MI355X peaks are what the
 * roofline fractions are quoted against; these two kernels measure what the
 * running GPU reaches with the same build flags, as context for them.
 *
 * sph_probe_fma: `blocks` workgroups of 256 lanes; each lane runs `iters`
 * iterations of 8 independent FP32 fused multiply-adds (non-packed, 16 FLOP
 * per lane per iteration) and writes one float to out[blocks * 256]
 * (device, caller-owned), which keeps the work. Needs 1 <= blocks <= 2^20
 * and iters >= 1.
 * sph_probe_copy: copies `bytes` from src to dst (device, caller-owned,
 * 16-byte aligned, not overlapping; bytes a multiple of 16, at most 2^40)
 * with 16-byte loads and stores in a grid-stride loop over `blocks`
 * workgroups of 256 lanes (1 <= blocks <= 2^20).
 * Both are asynchronous on `stream`; time them with events. Invalid
 * arguments give SPH_E_INVALID_ARG and a launch failure SPH_E_HIP, with the
 * message in sph_last_error(NULL). */
int sph_probe_fma(float *out, uint32_t blocks, int32_t iters, void *stream);
int sph_probe_copy(const void *src, void *dst, uint64_t bytes, uint32_t blocks, void *stream);

/* ---------------------------------------------------------------------------
 * Precision variant. The same step (sort, interaction, dt, Verlet) on a state
 * whose positions are an int32 linear cell index (the x-major cell of the sort
 * key, cells of side cs = 2h, Sec. 3.1) plus an FP32 offset from the cell
 * centre, |offset| <= h per axis: position = origin + (c + 1/2) cs + offset.
 * Offsets keep FP32 resolution at the scale of a cell instead of the domain,
 * so small displacements (dt v) are not rounded away over many steps. Pair
 * separations are formed as (o_i - o_j) + (c_i - c_j) cs; the Verlet update
 * moves a particle to the neighbouring cell when an offset leaves [-h, h).
 * The time-step minimum and the global mass / momentum / energy sums are
 * FP64 on the GPU. Needs SPH_F_CELL in params.features.
 * ------------------------------------------------------------------------- */
typedef struct sph_cstate {
    int32_t *cell;       /* linear cell (x-major); -1 = outside the grid (excluded) */
    float *ox, *oy, *oz; /* offset from the cell centre (m)                          */
    float *vx, *vy, *vz;
    float *rho;
    float *vxp, *vyp, *vzp;
    float *rhop;
    uint8_t *type;
    int32_t *id;
} sph_cstate;

/* Cell and offset of n FP64 device positions (other fields untouched):
 * c = floor((x - o)/cs) in FP64, offset = (float)((x - o)/cs - c - 1/2) * cs;
 * a position outside the grid gets cell -1 and offset 0. */
int sph_cstate_from_positions(sph_ctx *ctx, const double *x, const double *y, const double *z,
                              sph_cstate *out, uint32_t n, void *stream);
/* FP64 positions of a cell state: o + (c + 1/2) cs + offset, per axis
 * (NaN for cell -1). */
int sph_cstate_positions(sph_ctx *ctx, const sph_cstate *s, double *x, double *y, double *z,
                         uint32_t n, void *stream);
/* Sort step (keys from the cells; labels as in sph_sort), reorder into out,
 * cell tables, counts. */
int sph_csort(sph_ctx *ctx, const sph_cstate *in, sph_cstate *out, uint32_t n, void *stream);
/* Interaction on the state of the last sph_csort (rates as in sph_interact);
 * the dt limits are reduced in FP64 (sph_get_dt64). */
int sph_cinteract(sph_ctx *ctx, const sph_cstate *sorted, uint32_t n, const sph_rates *out,
                  void *stream);
/* Whole step on cell states: csort(cur -> next), interaction, FP64 dt,
 * Verlet update with re-celling of next. */
int sph_cstep(sph_ctx *ctx, const sph_cstate *cur, sph_cstate *next, uint32_t n, uint64_t step,
              void *stream);
/* FP64 totals over the in-domain non-ghost particles of a cell state:
 * out[0] mass, out[1..3] momentum, out[4] kinetic energy, out[5] potential
 * energy -m g.r, out[6] internal energy m e(rho) with
 * e(rho) = B[(rho^(g-1) - rho0^(g-1))/((g-1) rho0^g) + 1/rho - 1/rho0]
 * (the work of the Tait pressure), out[7] particle count. Synchronises. */
int sph_ctotals(sph_ctx *ctx, const sph_cstate *s, uint32_t n, double *out, void *stream);

/* FP64 reference path: the same step with every state array, the
 * interaction and the update in FP64 (cell keys from the positions rounded to
 * FP32, which only bins the particles). Needs SPH_F_FP64. */
typedef struct sph_dstate {
    double *x, *y, *z;
    double *vx, *vy, *vz;
    double *rho;
    double *vxp, *vyp, *vzp;
    double *rhop;
    uint8_t *type;
    int32_t *id;
} sph_dstate;

typedef struct sph_drates {
    double *ax, *ay, *az, *arho; /* as sph_rates, FP64 */
} sph_drates;

int sph_dsort(sph_ctx *ctx, const sph_dstate *in, sph_dstate *out, uint32_t n, void *stream);
int sph_dinteract(sph_ctx *ctx, const sph_dstate *sorted, uint32_t n, const sph_drates *out,
                  void *stream);
int sph_dstep(sph_ctx *ctx, const sph_dstate *cur, sph_dstate *next, uint32_t n, uint64_t step,
              void *stream);
int sph_dtotals(sph_ctx *ctx, const sph_dstate *s, uint32_t n, double *out, void *stream);

/* dt of the last sph_cinteract / sph_cstep / sph_dinteract / sph_dstep in
 * FP64 (CFL times the FP64 minimum of the per-particle limits). */
int sph_get_dt64(sph_ctx *ctx, double *dt, void *stream);

/* ---------------------------------------------------------------------------
 * Learned surrogate. An addition to the paper's method: a multilayer
 * perceptron that advances fluid and boundary particles by four time steps
 * at once from their neighbourhoods. Its input row for particle i is built
 * from the cell list of Sec. 3.1 with the FP32 distance expression of the
 * support test of Sec. 2.2: the particles j != i of the 27 cells around i
 * with fmaf(dz,dz,fmaf(dy,dy,dx*dx)) < r2f, in increasing sorted index, the
 * first 64 filling the slots; 8 bfloat16 features per slot and 32 for the
 * particle itself (SPH_NN_IN = 544):
 *   slot s:  (x_j - x_i) inv_len, (y_j - y_i) inv_len, (z_j - z_i) inv_len,
 *            (u_j - u_i) inv_vel (3), (rho_j - rho_ref) inv_rho, kind_j,
 *            zeros for an empty slot;
 *   own:     (rho_i - rho_ref) inv_rho, u_i inv_vel (3), count_i / 64,
 *            kind_i, ap_i inv_acc (3), dr_i inv_drho,
 *            (u_i - u_prev_i) inv_dt inv_acc (3),
 *            (rho_i - rho_prev_i) inv_dt inv_drho, 18 zeros;
 * kind = -1 for boundary particles, +1 otherwise; count_i = neighbours found
 * (before the cut at 64); ap_i = -sum_j m (p_i/rho_i^2 + p_j/rho_j^2)
 * grad_i W_ij and dr_i = sum_j m v_ij . grad_i W_ij over the slots (the
 * pressure part of the momentum equation and the continuity equation of
 * Sec. 2.2, FP32); u_prev, rho_prev are the previous-step values of the
 * Verlet scheme of Sec. 3.3 (the leapfrog's second sequence, which the next
 * steps depend on). Each feature is FP32 arithmetic left to right, rounded
 * to bfloat16 (nearest, ties to even). Ghost rows are zero.
 * Network: 544 -> w -> w -> w -> 4, SiLU after each hidden layer, bfloat16
 * weights and activations with FP32 accumulation on the matrix cores, FP32
 * master weights with Adam. Outputs, scaled: (du_x, du_y, du_z, drho) over
 * the four steps.
 * ------------------------------------------------------------------------- */
#define SPH_NN_SLOTS 64
#define SPH_NN_IN 544
#define SPH_NN_OUT 4
#define SPH_NN_LAYERS 4

typedef struct sph_nn_scales {
    float inv_len;  /* 1 / length scale (1/h)                  */
    float inv_vel;  /* 1 / velocity scale                      */
    float rho_ref;  /* reference density (rho0)                */
    float inv_rho;  /* 1 / density scale                       */
    float r2f;      /* squared radius of the neighbourhood     */
    float inv_acc;  /* 1 / acceleration scale of ap            */
    float inv_drho; /* 1 / density-rate scale of dr            */
    float inv_dt;   /* 1 / time scale of the previous-step
                       differences (0: those features are 0)  */
} sph_nn_scales;

/* Network and training workspace; every buffer is caller-owned device
 * memory (FP32 unless noted). Layer l maps in_l -> out_l with
 * (in, out) = (544, w), (w, w), (w, w), (w, 4); W[l] is row-major out x in.
 * The kernels read the bfloat16 copies wb[l]; sph_mlp_sync and
 * sph_mlp_adam refresh them from the FP32 masters w[l]. */
typedef struct sph_mlp {
    int32_t width;      /* hidden width: multiple of 16, 16..256             */
    uint32_t capacity;  /* rows of the workspace (training batch, <= 2^20)    */
    float *w[4], *b[4]; /* master weights [out][in] and biases [out]          */
    void *wb[4];        /* bfloat16 copies of w[l]                            */
    float *gw[4], *gb[4];                 /* gradients of the last backward   */
    float *mw[4], *vw[4], *mb[4], *vb[4]; /* Adam moments                     */
    float *z[4];        /* pre-activations [capacity][out_l]                 */
    void *a[3];         /* bfloat16 hidden activations [capacity][width]      */
    float *da;          /* [capacity][width]                                  */
    void *dz;           /* bfloat16 [capacity][width]                         */
    float *dy;          /* [capacity][4]                                      */
    float *work;        /* sph_mlp_work_floats(width, capacity) floats        */
    float *loss;        /* [1]: loss of the last sph_mlp_backward             */
} sph_mlp;

/* Size of sph_mlp.work (split-K partial products of the weight gradients
 * and loss partials), in floats. */
uint64_t sph_mlp_work_floats(int32_t width, uint32_t capacity);

/* Refresh the bfloat16 weight copies from the FP32 masters. */
int sph_mlp_sync(sph_ctx *ctx, sph_mlp *net, void *stream);

/* Input rows for particles of the sorted state of the last sph_sort (same
 * n): row r describes sorted particle rows[r] (rows == NULL: particle r).
 * x: bfloat16 [nrows][SPH_NN_IN], device. A row index outside the label-0
 * prefix gives a zero row. Re-packs the sorted arrays first, so the state
 * may have been changed in place since the sort (not reordered).
 * rates (optional, NULL: not written): FP32 [nrows][4], device: the row's
 * pair sums as rates in FP32 before any scaling, (ap + g) for fluid rows and
 * 0 for others (3 components), and dr; zero for ghosts and out-of-prefix rows.
 * They are what sph_nn_targets and sph_nn_apply take as the part of the
 * change that the network need not predict. */
int sph_nn_features(sph_ctx *ctx, const sph_soa *sorted, const int32_t *rows, uint32_t nrows,
                    const sph_nn_scales *scales, void *x, float *rates, void *stream);

/* where[id[k]] = k for k < n (ids must be a permutation of 0..n-1). */
int sph_nn_index(sph_ctx *ctx, const int32_t *id, uint32_t n, int32_t *where, void *stream);

/* Training targets: for r < nrows, particle k = rows[r] (or r) of state a
 * and the particle with the same id in state b (index where_b[id]):
 * t[4r..4r+3] = (((u_b - u_a) - span rates[4r..]) inv_dv (3 components),
 * ((rho_b - rho_a) - span rates[4r+3]) inv_dr), in FP32 in that order
 * without contraction. rates: FP32 [nrows][4] of sph_nn_features for the
 * same rows, or NULL for zeros. */
int sph_nn_targets(sph_ctx *ctx, const sph_soa *a, const sph_soa *b, const int32_t *where_b,
                   const int32_t *rows, uint32_t nrows, const float *rates, float span,
                   float inv_dv, float inv_dr, float *t, void *stream);

/* Forward pass of rows x (bfloat16 [rows][SPH_NN_IN]) into y (FP32
 * [rows][4]); keeps the activations in net for sph_mlp_backward.
 * rows <= net->capacity. */
int sph_mlp_forward(sph_ctx *ctx, sph_mlp *net, const void *x, uint32_t rows, float *y,
                    void *stream);

/* Loss L = sum_{r,c} wcol[c] (y - t)^2 / (4 rows) of the last forward pass
 * (same x and rows) into net->loss, and its gradients into gw, gb.
 * wcol: 4 host floats. */
int sph_mlp_backward(sph_ctx *ctx, sph_mlp *net, const void *x, uint32_t rows, const float *t,
                     const float *wcol, void *stream);

/* One Adam step (step number t >= 1, bias-corrected) on every weight and
 * bias from gw, gb; refreshes the bfloat16 copies. */
int sph_mlp_adam(sph_ctx *ctx, sph_mlp *net, float lr, float beta1, float beta2, float eps,
                 uint32_t t, void *stream);

/* Flags of sph_nn_apply and sph_nn_advance. */
enum {
    SPH_NN_RESIDUAL = 1,   /* advance: add dt4 x the rows' pair-sum rates       */
    SPH_NN_CARRY_PREV = 2  /* previous-step arrays keep their difference to the
                              current values (prev = new - (old - prev_old))
                              instead of being set one step back along the
                              change                                            */
};

/* Apply network outputs y (FP32 [nrows][4], row r = sorted particle r) to
 * the sorted state over a span dt4 of four steps, with rates (FP32
 * [nrows][4] of sph_nn_features, or NULL for zeros): fluid u += dt4
 * rates[0..2] + y[0..2] dv_scale, x += dt4 (u_old + u_new)/2; fluid and
 * boundary rho += dt4 rates[3] + y[3] dr_scale; ghosts untouched. The
 * previous-step arrays are set to one step back along the same change (new -
 * change/4), or with SPH_NN_CARRY_PREV in flags keep their difference to the
 * current values, so a following Verlet step continues the leapfrog. A
 * non-finite result or |rho/rho0 - 1| > rho_tol sets SPH_S_NN_RANGE. */
int sph_nn_apply(sph_ctx *ctx, sph_soa *sorted, const float *y, const float *rates,
                 uint32_t nrows, float dv_scale, float dr_scale, float dt4, float rho_tol,
                 int flags, void *stream);

/* One surrogate advance: sort cur into next (as sph_sort), build every
 * particle's input row (into buffers sph_create allocated for a context with
 * the SPH_F_SURROGATE feature: capacity x SPH_NN_IN bfloat16 rows, 4 FP32
 * rates and 4 FP32 outputs per particle; without the feature the call fails
 * with SPH_E_STATE and allocates nothing), then one kernel runs the network
 * (width 128) on tiles of 64 rows
 * and the result is applied to next as sph_nn_apply does, with the rows'
 * rates if flags has SPH_NN_RESIDUAL (a network trained on targets with
 * rates) and without them otherwise, and with SPH_NN_CARRY_PREV as there. */
int sph_nn_advance(sph_ctx *ctx, const sph_mlp *net, const sph_soa *cur, sph_soa *next,
                   uint32_t n, const sph_nn_scales *scales, float dv_scale, float dr_scale,
                   float dt4, float rho_tol, int flags, void *stream);

/* Training noise: adds to the velocity and density of every fluid particle
 * k < n (and to their previous-step values, so a Verlet step sees the same
 * shift) independent uniform noise of standard deviation sigma_u (m/s, per
 * component) and sigma_rho (kg/m^3), drawn from a counter-based generator
 * (murmur3's 32-bit finaliser of seed, k and the component): the same
 * (seed, n, state) always gives the same result. */
int sph_nn_perturb(sph_ctx *ctx, sph_soa *st, uint32_t n, uint32_t seed, float sigma_u,
                   float sigma_rho, void *stream);

/* Error of a surrogate state s against a reference state r reached from the
 * same base state b by plain SPH steps, over the fluid particles of s
 * (matched by id through where_r and where_b, built by sph_nn_index):
 * out[0] max |rho_s - rho_r| / rho_r, out[1] sum (rho_s - rho_r)^2,
 * out[2] sum (rho_r - rho_b)^2, out[3] sum |u_s - u_r|^2,
 * out[4] sum |u_r - u_b|^2, out[5] sum |x_s - x_r|^2,
 * out[6] sum |x_r - x_b|^2, out[7] fluid count. 8 host doubles;
 * synchronises. */
int sph_nn_judge(sph_ctx *ctx, const sph_soa *s, const sph_soa *r, const sph_soa *b,
                 const int32_t *where_r, const int32_t *where_b, uint32_t n, double *out,
                 void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
