// C ABI of libsph.so (declared in include/sph.h): validation, context and
// scratch management, and the order of kernel launches of each entry point.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "sph_internal.h"

using namespace sph;

namespace {

thread_local std::string g_create_err;

int fail(sph_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(sph_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf; else g_create_err = buf;
    return code;
}

int hip_fail(sph_ctx *c, hipError_t e, const char *what) {
    return fail(c, SPH_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int cell_bits_for(uint64_t ncells) {
    int b = 1;
    while ((1ull << b) < ncells) b++;
    return b;
}

bool soa_ok(const sph_soa *s) {
    return s && s->x && s->y && s->z && s->vx && s->vy && s->vz && s->rho && s->vxp && s->vyp &&
           s->vzp && s->rhop && s->type && s->id;
}

bool rates_ok(const sph_rates *r) { return r && r->ax && r->ay && r->az && r->arho; }

int enter(sph_ctx *c) {
    if (!c) return SPH_E_INVALID_ARG;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    return SPH_OK;
}

void free_events(sph_ctx *c) {
    if (c->events) {
        for (uint32_t k = 0; k < 4 * c->ev_slots; k++) (void)hipEventDestroy(c->events[k]);
        delete[] c->events;
    }
    c->events = nullptr;
    c->ev_slots = c->ev_used = 0;
}

void free_all(sph_ctx *c) {
    free_events(c);
    void *vptrs[] = {c->pos8,   c->vel8,  c->drate, c->tot_part, c->nn_part,
                     c->nn_out, c->nn_x,  c->nn_y,     c->nn_rate};
    for (void *p : vptrs)
        if (p) (void)hipFree(p);
    void *ptrs[] = {c->keys_a, c->keys_b, c->keys_sorted, c->vals_a, c->vals_b, c->perm,
                    c->hist, c->digit_tot, c->cell_begin, c->cell_end, c->pos4, c->vel4,
                    c->rate, c->info, c->mmask, c->mwpre, c->mcnt, c->mtile};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (c->fb) (void)hipHostFree(c->fb);
    c->fb = c->fb_dev = nullptr;
}

}  // namespace

int sph::set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_create_err = buf;
    return code;
}

extern "C" {

int sph_abi_version(void) { return SPH_ABI_VERSION; }

const char *sph_error_string(int code) {
    switch (code) {
        case SPH_OK: return "ok";
        case SPH_E_INVALID_ARG: return "invalid argument";
        case SPH_E_CAPACITY: return "particle count exceeds the context capacity";
        case SPH_E_KEY_BITS: return "cell grid too large for 32-bit keys with 2 label bits";
        case SPH_E_HIP: return "HIP runtime error";
        case SPH_E_STATE: return "entry points called out of order";
        default: return "unknown error";
    }
}

const char *sph_last_error(const sph_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int sph_create(const sph_params *p, sph_ctx **out) {
    g_create_err.clear();
    if (!p || !out) return fail(nullptr, SPH_E_INVALID_ARG, "null params or output pointer");
    *out = nullptr;
    if (!(p->dp > 0 && p->h > 0 && p->rho0 > 0 && p->c0 > 0 && p->alpha >= 0 &&
          p->eta_over_h > 0 && p->cfl > 0 && p->mass > 0))
        return fail(nullptr, SPH_E_INVALID_ARG, "physical parameters must be positive");
    if (p->gamma != 7.0)
        return fail(nullptr, SPH_E_INVALID_ARG, "gamma must be 7 (Tait law of the method)");
    if ((p->options & ~(int32_t)(SPH_O_CUBIC | SPH_O_RHO_FLOOR | SPH_O_SYMPLECTIC)) != 0 ||
        (p->features & ~(uint32_t)(SPH_F_CELL | SPH_F_FP64 | SPH_F_SURROGATE)) != 0)
        return fail(nullptr, SPH_E_INVALID_ARG, "unknown option or feature bits");
    if (p->options != 0 && p->features != 0)
        return fail(nullptr, SPH_E_INVALID_ARG,
                    "the cell, FP64 and surrogate paths keep the Wendland kernel: options must be 0");
    for (int a = 0; a < 3; a++)
        if (p->ncell[a] < 1 || !isfinite(p->origin[a]) || !isfinite(p->g[a]))
            return fail(nullptr, SPH_E_INVALID_ARG, "bad grid or gravity on axis %d", a);
    if (p->capacity < 1 || p->capacity >= (1u << 28))
        return fail(nullptr, SPH_E_INVALID_ARG, "capacity must be in [1, 2^28)");
    if ((p->features & SPH_F_CELL) && p->capacity >= (1u << 27))
        return fail(nullptr, SPH_E_INVALID_ARG,
                    "the cell path lists neighbours as index << 5: capacity must be < 2^27");
    const uint64_t ncells = (uint64_t)p->ncell[0] * p->ncell[1] * p->ncell[2];
    const int bits = cell_bits_for(ncells);
    if (bits > 30)
        return fail(nullptr, SPH_E_KEY_BITS, "grid of %llu cells needs %d bits (max 30)",
                    (unsigned long long)ncells, bits);
    const double cs = 2.0 * p->h;
    if (p->slab_mode != 0 && p->slab_mode != 1)
        return fail(nullptr, SPH_E_INVALID_ARG, "slab_mode must be 0 or 1");
    if (p->slab_mode) {
        const double w = (p->slab_xhi - p->slab_xlo) / cs;
        if (!(w >= 1.0) || fabs(w - nearbyint(w)) > 1e-6 ||
            fabs(p->origin[0] - (p->slab_xlo - cs)) > 1e-6 * cs ||
            p->ncell[0] != (int32_t)nearbyint(w) + 2)
            return fail(nullptr, SPH_E_INVALID_ARG,
                        "slab mode needs origin_x = slab_xlo - 2h and ncell_x = width/2h + 2 "
                        "with an integer width in cells");
    }

    sph_ctx *c = new (std::nothrow) sph_ctx();
    if (!c) return fail(nullptr, SPH_E_HIP, "out of host memory");
    c->prm = *p;
    (void)hipGetDevice(&c->device);
    c->capacity = p->capacity;
    c->cell_bits = bits;
    c->ncells = (uint32_t)ncells;

    KParams &k = c->kp;
    k.ox = (float)p->origin[0];
    k.oy = (float)p->origin[1];
    k.oz = (float)p->origin[2];
    k.inv_cs = (float)(1.0 / cs);
    k.ncx = p->ncell[0];
    k.ncy = p->ncell[1];
    k.ncz = p->ncell[2];
    k.cell_bits = bits;
    k.ncells = (uint32_t)ncells;
    k.cell_mask = (1u << bits) - 1u;
    k.slab_mode = p->slab_mode;
    k.slab_xlo = (float)p->slab_xlo;
    k.slab_xhi = (float)p->slab_xhi;
    k.h = (float)p->h;
    k.inv_h = (float)(1.0 / p->h);
    k.r2max = (float)(4.0 * p->h * p->h);
    const double eta = p->eta_over_h * p->h;
    k.eta2 = (float)(eta * eta);
    k.mass = (float)p->mass;
    k.alpha = (float)p->alpha;
    k.rho0 = (float)p->rho0;
    k.inv_rho0 = (float)(1.0 / p->rho0);
    k.B = (float)(p->c0 * p->c0 * p->rho0 / p->gamma);
    k.c0 = (float)p->c0;
    k.gx = (float)p->g[0];
    k.gy = (float)p->g[1];
    k.gz = (float)p->g[2];
    const double aD = 21.0 / (16.0 * M_PI * p->h * p->h * p->h);
    k.kgrad = (float)(-5.0 * aD / (p->h * p->h));
    k.kgrad_cubic = (float)(-0.75 / (M_PI * p->h * p->h * p->h) / (p->h * p->h));
    k.options = p->options;
    k.cfl = (float)p->cfl;
    k.euler_every = p->euler_every;

    const size_t cap = p->capacity;
    c->max_tiles = (uint32_t)((cap + kSortTile - 1) / kSortTile);
    hipError_t e = hipSuccess;
#define ALLOC(ptr, bytes)                                               \
    do {                                                                \
        if (e == hipSuccess) e = hipMalloc((void **)&(ptr), (bytes));   \
    } while (0)
    ALLOC(c->keys_a, cap * 4);
    // + 64 B: the mover plan reads a tile's first movers in 16-byte pieces,
    // up to 11 entries past the last particle of a partial last tile
    ALLOC(c->keys_b, cap * 4 + 64);
    ALLOC(c->keys_sorted, cap * 4);
    ALLOC(c->vals_a, cap * 4);
    ALLOC(c->vals_b, cap * 4 + 64);
    ALLOC(c->perm, cap * 4);
    ALLOC(c->hist, (size_t)256 * c->max_tiles * 4);
    ALLOC(c->mmask, (cap / 64 + 1) * sizeof(unsigned long long));
    ALLOC(c->mwpre, (cap / 64 + 1) * 4);
    ALLOC(c->mcnt, (size_t)c->max_tiles * 4 + 4);
    ALLOC(c->mtile, (size_t)c->max_tiles * sizeof(uint2) + 8);
    ALLOC(c->digit_tot, 256 * 4);
    ALLOC(c->cell_begin, (size_t)ncells * 4);
    ALLOC(c->cell_end, (size_t)ncells * 4);
    ALLOC(c->pos4, cap * sizeof(float4));
    ALLOC(c->vel4, cap * sizeof(float4));
    ALLOC(c->rate, cap * 4 * sizeof(float));
    ALLOC(c->info, sizeof(DevInfo));
    c->features = p->features;
    c->tot_blocks = (uint32_t)std::min<size_t>(1024, (cap + kTotThreads - 1) / kTotThreads);
    ALLOC(c->tot_part, (size_t)8 * (c->tot_blocks + 1) * sizeof(double));
    ALLOC(c->nn_part, (size_t)8 * (cap / 256 + 2) * sizeof(double));
    ALLOC(c->nn_out, 8 * sizeof(double));
    if (p->features & SPH_F_FP64) {
        ALLOC(c->pos8, cap * sizeof(double4));
        ALLOC(c->vel8, cap * sizeof(double4));
        ALLOC(c->drate, 4 * cap * sizeof(double));
    }
    if (p->features & SPH_F_SURROGATE) {
        // rows, network outputs and pair-sum rates of every particle for sph_nn_advance
        ALLOC(c->nn_x, cap * SPH_NN_IN * 2);
        ALLOC(c->nn_y, cap * SPH_NN_OUT * sizeof(float));
        ALLOC(c->nn_rate, cap * 4 * sizeof(float));
    }
#undef ALLOC
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->fb, sizeof(unsigned long long),
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
        *c->fb = 0ull;
        e = hipHostGetDevicePointer((void **)&c->fb_dev, c->fb, 0);
    }
    if (e == hipSuccess) e = hipMemset(c->info, 0, sizeof(DevInfo));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        fail(nullptr, SPH_E_HIP, "scratch allocation for %zu particles: %s", cap,
             hipGetErrorString(e));
        free_all(c);
        delete c;
        return SPH_E_HIP;
    }
    *out = c;
    return SPH_OK;
}

void sph_destroy(sph_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    free_all(c);
    delete c;
}

int sph_cell_bits(const sph_ctx *c) { return c ? c->cell_bits : SPH_E_INVALID_ARG; }

int sph_sort_kv(sph_ctx *c, const uint32_t *keys, const int32_t *vals, uint32_t *keys_out,
                int32_t *vals_out, uint32_t n, int key_bits, void *stream) {
    int r = enter(c);
    if (r) return r;
    if (n > c->capacity) return fail(c, SPH_E_CAPACITY, "n = %u > capacity %u", n, c->capacity);
    if (key_bits < 1 || key_bits > 32) return fail(c, SPH_E_INVALID_ARG, "key_bits must be 1..32");
    if (n > 0 && (!keys || !vals || !keys_out || !vals_out))
        return fail(c, SPH_E_INVALID_ARG, "null array");
    if (n > 0 && ((const void *)keys == (const void *)keys_out ||
                  (const void *)vals == (const void *)vals_out))
        return fail(c, SPH_E_INVALID_ARG, "outputs must not alias inputs");
    hipError_t e = radix_sort(c, keys, vals, keys_out, vals_out, n, key_bits, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "radix sort");
    return SPH_OK;
}

// skip_rv: the caller (the plain step) takes r, v and rho of the new order
// from the packed arrays; the reorder leaves them out of `out`.
static int do_sort(sph_ctx *c, const sph_soa *in, const sph_soa *out, uint32_t n, hipStream_t s,
                   bool skip_rv = false) {
    // the sorted keys and cell tables of the previous sort (any path) are the
    // reference of the incremental sort; without one every particle moves
    const uint32_t nprev = c->have_sort ? c->sorted_n : 0u;
    // the input is the state the last plain sort wrote (a time loop), and the
    // last mover plan that has run (the host does not wait for it) saw a
    // previous sort and few movers: expect few again and launch only the
    // merge (which still sorts any number of movers, slowly); else launch
    // the radix passes too and let the plan choose
    const unsigned long long fb = __atomic_load_n(c->fb, __ATOMIC_RELAXED);
    const bool loop = nprev > 0 && c->last_path == 0 && in->x == c->last_out_x && (fb & 1ull);
    const unsigned long long last_m = fb >> 1;
    const int expect = !loop ? kExpectAny
                             : (last_m <= kIncCap ? kExpectFew
                                                  : (last_m <= mid_cap(n) ? kExpectMid : kExpectAny));
    hipError_t e = sort_state(c, *in, *out, n, nprev, expect, skip_rv, s);
    if (e != hipSuccess) return hip_fail(c, e, "sort step");
    c->last_out_x = out->x;
    c->sorted_n = n;
    c->have_sort = true;
    c->have_dt = false;
    c->last_path = 0;
    return SPH_OK;
}

int sph_sort(sph_ctx *c, const sph_soa *in, sph_soa *out, uint32_t n, void *stream) {
    int r = enter(c);
    if (r) return r;
    if (n > c->capacity) return fail(c, SPH_E_CAPACITY, "n = %u > capacity %u", n, c->capacity);
    if (!soa_ok(in) || !soa_ok(out)) return fail(c, SPH_E_INVALID_ARG, "null state array");
    if (in->x == out->x || in->rho == out->rho || in->type == out->type || in->id == out->id)
        return fail(c, SPH_E_INVALID_ARG, "in and out must not share arrays");
    return do_sort(c, in, out, n, (hipStream_t)stream);
}

int sph_interact(sph_ctx *c, const sph_soa *sorted, uint32_t n, const sph_rates *out,
                 void *stream) {
    int r = enter(c);
    if (r) return r;
    if (!soa_ok(sorted) || !rates_ok(out)) return fail(c, SPH_E_INVALID_ARG, "null array");
    if (!c->have_sort || n != c->sorted_n || c->last_path != 0)
        return fail(c, SPH_E_STATE, "sph_interact needs a preceding sph_sort of the same n");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_pack(c, *sorted, n, s);
    if (e == hipSuccess) e = launch_interact(c, sorted->type, n, *out, s);
    if (e != hipSuccess) return hip_fail(c, e, "interaction");
    c->have_dt = true;
    c->dt_in_info = false;
    return SPH_OK;
}

int sph_update(sph_ctx *c, sph_soa *sorted, const sph_rates *rates, uint32_t n, uint64_t step,
               void *stream) {
    int r = enter(c);
    if (r) return r;
    if (!soa_ok(sorted) || !rates_ok(rates)) return fail(c, SPH_E_INVALID_ARG, "null array");
    if (!c->have_dt || n != c->sorted_n || c->last_path != 0)
        return fail(c, SPH_E_STATE, "sph_update needs a preceding sph_interact of the same n");
    if (c->kp.options & SPH_O_SYMPLECTIC)
        return fail(c, SPH_E_STATE, "the symplectic step needs two interactions: use sph_step");
    hipError_t e = launch_update(c, *sorted, rates->ax, rates->ay, rates->az, rates->arho, n, step,
                                 (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "update");
    return SPH_OK;
}

int sph_step(sph_ctx *c, const sph_soa *cur, sph_soa *next, uint32_t n, uint64_t step,
             void *stream) {
    int r = enter(c);
    if (r) return r;
    if (n > c->capacity) return fail(c, SPH_E_CAPACITY, "n = %u > capacity %u", n, c->capacity);
    if (!soa_ok(cur) || !soa_ok(next)) return fail(c, SPH_E_INVALID_ARG, "null state array");
    if (cur->x == next->x || cur->rho == next->rho || cur->type == next->type || cur->id == next->id)
        return fail(c, SPH_E_INVALID_ARG, "cur and next must not share arrays");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t *ev = (c->events && c->ev_used < c->ev_slots) ? c->events + 4 * c->ev_used : nullptr;
    if (ev) {
        c->ev_used++;
        (void)hipEventRecord(ev[0], s);
    }
    // the plain update writes r, v and rho of every particle from the packed
    // arrays; the symplectic half step overwrites those, so it needs them in
    // the state
    const bool sym = (c->kp.options & SPH_O_SYMPLECTIC) != 0;
    r = do_sort(c, cur, next, n, s, !sym);
    if (r) return r;
    if (ev) (void)hipEventRecord(ev[1], s);
    const size_t cap = c->capacity;
    sph_rates rt = {c->rate, c->rate + cap, c->rate + 2 * cap, c->rate + 3 * cap,
                    nullptr, nullptr, nullptr};
    hipError_t e;
    if (c->kp.options & SPH_O_SYMPLECTIC) {
        // rates at n (and the CFL limits), half state into the packed inputs,
        // rates of the half state on the same cell tables, full step
        e = launch_interact(c, next->type, n, rt, s);
        if (e == hipSuccess) e = launch_sym_half(c, *next, rt.ax, rt.ay, rt.az, rt.arho, n, s);
        if (e == hipSuccess) e = launch_interact(c, next->type, n, rt, s, ev ? ev[2] : nullptr);
        if (e == hipSuccess) e = launch_sym_full(c, *next, rt.ax, rt.ay, rt.az, rt.arho, n, s);
    } else {
        e = launch_interact(c, next->type, n, rt, s, ev ? ev[2] : nullptr);
        if (e == hipSuccess)
            e = launch_update(c, *next, rt.ax, rt.ay, rt.az, rt.arho, n, step, s, true);
    }
    if (ev) (void)hipEventRecord(ev[3], s);
    if (e != hipSuccess) return hip_fail(c, e, "step");
    c->have_dt = true;
    c->dt_in_info = (c->kp.options & SPH_O_SYMPLECTIC) != 0;
    return SPH_OK;
}

static int read_info(sph_ctx *c, DevInfo *h, void *stream) {
    int r = enter(c);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(h, c->info, sizeof(DevInfo), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "readback");
    return SPH_OK;
}

int sph_get_counts(sph_ctx *c, sph_counts *out, void *stream) {
    if (!out) return c ? fail(c, SPH_E_INVALID_ARG, "null output") : SPH_E_INVALID_ARG;
    DevInfo h;
    int r = read_info(c, &h, stream);
    if (r) return r;
    memcpy(out->n_label, h.n_label, sizeof h.n_label);
    memcpy(out->halo_lo, h.ranges + 0, 8);
    memcpy(out->edge_lo, h.ranges + 2, 8);
    memcpy(out->edge_hi, h.ranges + 4, 8);
    memcpy(out->halo_hi, h.ranges + 6, 8);
    memcpy(out->out_lo, h.ranges + 8, 8);
    memcpy(out->out_hi, h.ranges + 10, 8);
    memcpy(out->excluded, h.ranges + 12, 8);
    return SPH_OK;
}

int sph_get_dt(sph_ctx *c, float *dt, void *stream) {
    if (!dt) return c ? fail(c, SPH_E_INVALID_ARG, "null output") : SPH_E_INVALID_ARG;
    DevInfo h;
    int r = read_info(c, &h, stream);
    if (r) return r;
    if (!c->have_dt) return fail(c, SPH_E_STATE, "no interaction yet");
    if (c->last_path != 0) {  // variant paths: the FP32 rounding of CFL * FP64 minimum
        double m64;
        memcpy(&m64, &h.dtmin64_bits, sizeof m64);
        *dt = (float)((double)c->kp.cfl * m64);
        return SPH_OK;
    }
    if (c->dt_in_info) {  // symplectic step: the dt its half step formed and used
        *dt = h.dt;
        return SPH_OK;
    }
    // the same FP32 product as the update kernel forms: CFL * min limit
    float m;
    memcpy(&m, &h.dtmin_bits, sizeof m);
    *dt = c->kp.cfl * m;
    return SPH_OK;
}

int sph_get_sort_stats(sph_ctx *c, uint32_t *movers, uint32_t *merged, void *stream) {
    if (!movers || !merged) return c ? fail(c, SPH_E_INVALID_ARG, "null output") : SPH_E_INVALID_ARG;
    DevInfo h;
    int r = read_info(c, &h, stream);
    if (r) return r;
    if (!c->have_sort || c->last_path != 0) return fail(c, SPH_E_STATE, "no plain sort yet");
    *movers = h.movers;
    *merged = h.sort_mode;  // kModeFull 0, kModeIncr 1, kModeMid 2
    return SPH_OK;
}

int sph_get_pairs(sph_ctx *c, uint64_t *pairs, void *stream) {
    if (!pairs) return c ? fail(c, SPH_E_INVALID_ARG, "null output") : SPH_E_INVALID_ARG;
    DevInfo h;
    int r = read_info(c, &h, stream);
    if (r) return r;
    *pairs = h.pairs;
    return SPH_OK;
}

int sph_get_pair_total(sph_ctx *c, uint64_t *pairs, void *stream) {
    if (!pairs) return c ? fail(c, SPH_E_INVALID_ARG, "null output") : SPH_E_INVALID_ARG;
    DevInfo h;
    int r = read_info(c, &h, stream);
    if (r) return r;
    *pairs = h.pairs_total;
    return SPH_OK;
}

int sph_get_candidate_total(sph_ctx *c, uint64_t *cands, void *stream) {
    if (!cands) return c ? fail(c, SPH_E_INVALID_ARG, "null output") : SPH_E_INVALID_ARG;
    DevInfo h;
    int r = read_info(c, &h, stream);
    if (r) return r;
    *cands = h.cand_total;
    return SPH_OK;
}

int sph_timing_begin(sph_ctx *c, uint32_t max_steps) {
    int r = enter(c);
    if (r) return r;
    if (max_steps > 65536) return fail(c, SPH_E_INVALID_ARG, "max_steps must be <= 65536");
    free_events(c);
    if (max_steps == 0) return SPH_OK;
    c->events = new (std::nothrow) hipEvent_t[4 * (size_t)max_steps];
    if (!c->events) return fail(c, SPH_E_HIP, "out of host memory");
    for (uint32_t k = 0; k < 4 * max_steps; k++) {
        hipError_t e = hipEventCreate(&c->events[k]);
        if (e != hipSuccess) {
            for (uint32_t q = 0; q < k; q++) (void)hipEventDestroy(c->events[q]);
            delete[] c->events;
            c->events = nullptr;
            return hip_fail(c, e, "hipEventCreate");
        }
    }
    c->ev_slots = max_steps;
    c->ev_used = 0;
    return SPH_OK;
}

int sph_timing_read(sph_ctx *c, float *ms, uint32_t max_steps, uint32_t *count) {
    int r = enter(c);
    if (r) return r;
    if (!count || (!ms && max_steps)) return fail(c, SPH_E_INVALID_ARG, "null output");
    const uint32_t m = c->ev_used < max_steps ? c->ev_used : max_steps;
    for (uint32_t k = 0; k < m; k++) {
        hipEvent_t *ev = c->events + 4 * k;
        hipError_t e = hipEventSynchronize(ev[3]);
        for (int q = 0; q < 3 && e == hipSuccess; q++) e = hipEventElapsedTime(&ms[3 * k + q], ev[q], ev[q + 1]);
        if (e != hipSuccess) return hip_fail(c, e, "event timing");
    }
    *count = m;
    return SPH_OK;
}

int sph_get_status(sph_ctx *c, uint32_t *flags, void *stream) {
    if (!flags) return c ? fail(c, SPH_E_INVALID_ARG, "null output") : SPH_E_INVALID_ARG;
    DevInfo h;
    int r = read_info(c, &h, stream);
    if (r) return r;
    *flags = h.flags;
    return SPH_OK;
}

int sph_clear_status(sph_ctx *c, void *stream) {
    int r = enter(c);
    if (r) return r;
    hipError_t e = launch_clear_flags(c, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "clear status");
    return SPH_OK;
}

int sph_copy_keys(sph_ctx *c, uint32_t *keys_out, uint32_t n, void *stream) {
    int r = enter(c);
    if (r) return r;
    if (!keys_out && n) return fail(c, SPH_E_INVALID_ARG, "null output");
    if (!c->have_sort || n > c->sorted_n) return fail(c, SPH_E_STATE, "no sort of that size yet");
    if (n == 0) return SPH_OK;
    hipError_t e = hipMemcpyAsync(keys_out, c->keys_sorted, (size_t)n * 4,
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? SPH_OK : hip_fail(c, e, "copy keys");
}

int sph_copy_cell_tables(sph_ctx *c, uint32_t *begin_out, uint32_t *end_out, void *stream) {
    int r = enter(c);
    if (r) return r;
    if (!begin_out || !end_out) return fail(c, SPH_E_INVALID_ARG, "null output");
    if (!c->have_sort) return fail(c, SPH_E_STATE, "no sort yet");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(begin_out, c->cell_begin, (size_t)c->ncells * 4,
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(end_out, c->cell_end, (size_t)c->ncells * 4, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? SPH_OK : hip_fail(c, e, "copy cell tables");
}

// ------------------------------------------------------------ machine probes

int sph_probe_fma(float *out, uint32_t blocks, int32_t iters, void *stream) {
    g_create_err.clear();
    if (!out || blocks == 0 || blocks > (1u << 20) || iters < 1)
        return fail(nullptr, SPH_E_INVALID_ARG,
                    "probe_fma: needs out, 1 <= blocks <= 2^20 and iters >= 1");
    hipError_t e = launch_probe_fma(out, blocks, iters, (hipStream_t)stream);
    return e == hipSuccess ? SPH_OK : hip_fail(nullptr, e, "probe_fma");
}

int sph_probe_copy(const void *src, void *dst, uint64_t bytes, uint32_t blocks, void *stream) {
    g_create_err.clear();
    if (!src || !dst || bytes % 16 != 0 || bytes > (1ull << 40) || blocks == 0 ||
        blocks > (1u << 20) || ((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
        return fail(nullptr, SPH_E_INVALID_ARG,
                    "probe_copy: needs 16-byte aligned buffers, bytes a multiple of 16 "
                    "(at most 2^40) and 1 <= blocks <= 2^20");
    const uintptr_t a = (uintptr_t)src, d = (uintptr_t)dst;
    if (bytes && a < d + bytes && d < a + bytes)
        return fail(nullptr, SPH_E_INVALID_ARG, "probe_copy: source and destination overlap");
    hipError_t e = launch_probe_copy(src, dst, bytes, blocks, (hipStream_t)stream);
    return e == hipSuccess ? SPH_OK : hip_fail(nullptr, e, "probe_copy");
}

// ------------------------------------------------------------ variants

static bool cstate_ok(const sph_cstate *s) {
    return s && s->cell && s->ox && s->oy && s->oz && s->vx && s->vy && s->vz && s->rho && s->vxp &&
           s->vyp && s->vzp && s->rhop && s->type && s->id;
}

static bool dstate_ok(const sph_dstate *s) {
    return s && s->x && s->y && s->z && s->vx && s->vy && s->vz && s->rho && s->vxp && s->vyp &&
           s->vzp && s->rhop && s->type && s->id;
}

static int need(sph_ctx *c, uint32_t feature, uint32_t n) {
    int r = enter(c);
    if (r) return r;
    if (!(c->features & feature))
        return fail(c, SPH_E_STATE, "this path needs feature bit %u in sph_params.features", feature);
    if (n > c->capacity) return fail(c, SPH_E_CAPACITY, "n = %u > capacity %u", n, c->capacity);
    return SPH_OK;
}

int sph_cstate_from_positions(sph_ctx *c, const double *x, const double *y, const double *z,
                              sph_cstate *out, uint32_t n, void *stream) {
    int r = need(c, SPH_F_CELL, n);
    if (r) return r;
    if (n && (!x || !y || !z || !out || !out->cell || !out->ox || !out->oy || !out->oz))
        return fail(c, SPH_E_INVALID_ARG, "null array");
    hipError_t e = launch_cell_from_pos(c, x, y, z, *out, n, (hipStream_t)stream);
    return e == hipSuccess ? SPH_OK : hip_fail(c, e, "cells from positions");
}

int sph_cstate_positions(sph_ctx *c, const sph_cstate *st, double *x, double *y, double *z,
                         uint32_t n, void *stream) {
    int r = need(c, SPH_F_CELL, n);
    if (r) return r;
    if (n && (!x || !y || !z || !st || !st->cell || !st->ox || !st->oy || !st->oz))
        return fail(c, SPH_E_INVALID_ARG, "null array");
    hipError_t e = launch_pos_from_cell(c, *st, x, y, z, n, (hipStream_t)stream);
    return e == hipSuccess ? SPH_OK : hip_fail(c, e, "positions from cells");
}

static int do_csort(sph_ctx *c, const sph_cstate *in, const sph_cstate *out, uint32_t n,
                    hipStream_t s) {
    hipError_t e = launch_keys_cell(c, *in, n, s);
    if (e == hipSuccess) e = radix_sort(c, c->keys_a, c->vals_a, c->keys_sorted, c->perm, n,
                                        c->cell_bits + 2, s);
    if (e == hipSuccess) e = launch_tables(c, n, s);
    if (e == hipSuccess) e = launch_gather_cell(c, *in, *out, n, s);
    if (e != hipSuccess) return hip_fail(c, e, "cell sort step");
    c->sorted_n = n;
    c->have_sort = true;
    c->have_dt = false;
    c->last_path = 1;
    return SPH_OK;
}

int sph_csort(sph_ctx *c, const sph_cstate *in, sph_cstate *out, uint32_t n, void *stream) {
    int r = need(c, SPH_F_CELL, n);
    if (r) return r;
    if (!cstate_ok(in) || !cstate_ok(out)) return fail(c, SPH_E_INVALID_ARG, "null state array");
    if (in->cell == out->cell || in->ox == out->ox || in->type == out->type)
        return fail(c, SPH_E_INVALID_ARG, "in and out must not share arrays");
    return do_csort(c, in, out, n, (hipStream_t)stream);
}

int sph_cinteract(sph_ctx *c, const sph_cstate *sorted, uint32_t n, const sph_rates *out,
                  void *stream) {
    int r = need(c, SPH_F_CELL, n);
    if (r) return r;
    if (!cstate_ok(sorted) || !rates_ok(out)) return fail(c, SPH_E_INVALID_ARG, "null array");
    if (!c->have_sort || n != c->sorted_n || c->last_path != 1)
        return fail(c, SPH_E_STATE, "sph_cinteract needs a preceding sph_csort of the same n");
    hipError_t e = launch_interact_cell(c, *sorted, n, *out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "cell interaction");
    c->have_dt = true;
    return SPH_OK;
}

int sph_cstep(sph_ctx *c, const sph_cstate *cur, sph_cstate *next, uint32_t n, uint64_t step,
              void *stream) {
    int r = need(c, SPH_F_CELL, n);
    if (r) return r;
    if (!cstate_ok(cur) || !cstate_ok(next)) return fail(c, SPH_E_INVALID_ARG, "null state array");
    if (cur->cell == next->cell || cur->ox == next->ox || cur->type == next->type)
        return fail(c, SPH_E_INVALID_ARG, "cur and next must not share arrays");
    hipStream_t s = (hipStream_t)stream;
    r = do_csort(c, cur, next, n, s);
    if (r) return r;
    const size_t cap = c->capacity;
    sph_rates rt = {c->rate, c->rate + cap, c->rate + 2 * cap, c->rate + 3 * cap,
                    nullptr, nullptr, nullptr};
    hipError_t e = launch_interact_cell(c, *next, n, rt, s);
    if (e == hipSuccess) e = launch_update_cell(c, *next, rt.ax, rt.ay, rt.az, rt.arho, n, step, s);
    if (e != hipSuccess) return hip_fail(c, e, "cell step");
    c->have_dt = true;
    return SPH_OK;
}

int sph_ctotals(sph_ctx *c, const sph_cstate *st, uint32_t n, double *out, void *stream) {
    int r = need(c, SPH_F_CELL, n);
    if (r) return r;
    if (!cstate_ok(st) || !out) return fail(c, SPH_E_INVALID_ARG, "null array");
    hipError_t e = launch_totals_cell(c, *st, n, out, (hipStream_t)stream);
    return e == hipSuccess ? SPH_OK : hip_fail(c, e, "cell totals");
}

static int do_dsort(sph_ctx *c, const sph_dstate *in, const sph_dstate *out, uint32_t n,
                    hipStream_t s) {
    hipError_t e = launch_keys_d(c, *in, n, s);
    if (e == hipSuccess) e = radix_sort(c, c->keys_a, c->vals_a, c->keys_sorted, c->perm, n,
                                        c->cell_bits + 2, s);
    if (e == hipSuccess) e = launch_tables(c, n, s);
    if (e == hipSuccess) e = launch_gather_d(c, *in, *out, n, s);
    if (e != hipSuccess) return hip_fail(c, e, "FP64 sort step");
    c->sorted_n = n;
    c->have_sort = true;
    c->have_dt = false;
    c->last_path = 2;
    return SPH_OK;
}

int sph_dsort(sph_ctx *c, const sph_dstate *in, sph_dstate *out, uint32_t n, void *stream) {
    int r = need(c, SPH_F_FP64, n);
    if (r) return r;
    if (!dstate_ok(in) || !dstate_ok(out)) return fail(c, SPH_E_INVALID_ARG, "null state array");
    if (in->x == out->x || in->rho == out->rho || in->type == out->type)
        return fail(c, SPH_E_INVALID_ARG, "in and out must not share arrays");
    return do_dsort(c, in, out, n, (hipStream_t)stream);
}

int sph_dinteract(sph_ctx *c, const sph_dstate *sorted, uint32_t n, const sph_drates *out,
                  void *stream) {
    int r = need(c, SPH_F_FP64, n);
    if (r) return r;
    if (!dstate_ok(sorted) || !out || !out->ax || !out->ay || !out->az || !out->arho)
        return fail(c, SPH_E_INVALID_ARG, "null array");
    if (!c->have_sort || n != c->sorted_n || c->last_path != 2)
        return fail(c, SPH_E_STATE, "sph_dinteract needs a preceding sph_dsort of the same n");
    hipError_t e = launch_interact_d(c, *sorted, n, *out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "FP64 interaction");
    c->have_dt = true;
    return SPH_OK;
}

int sph_dstep(sph_ctx *c, const sph_dstate *cur, sph_dstate *next, uint32_t n, uint64_t step,
              void *stream) {
    int r = need(c, SPH_F_FP64, n);
    if (r) return r;
    if (!dstate_ok(cur) || !dstate_ok(next)) return fail(c, SPH_E_INVALID_ARG, "null state array");
    if (cur->x == next->x || cur->rho == next->rho || cur->type == next->type)
        return fail(c, SPH_E_INVALID_ARG, "cur and next must not share arrays");
    hipStream_t s = (hipStream_t)stream;
    r = do_dsort(c, cur, next, n, s);
    if (r) return r;
    const size_t cap = c->capacity;
    sph_drates rt = {c->drate, c->drate + cap, c->drate + 2 * cap, c->drate + 3 * cap};
    hipError_t e = launch_interact_d(c, *next, n, rt, s);
    if (e == hipSuccess) e = launch_update_d(c, *next, rt, n, step, s);
    if (e != hipSuccess) return hip_fail(c, e, "FP64 step");
    c->have_dt = true;
    return SPH_OK;
}

int sph_dtotals(sph_ctx *c, const sph_dstate *st, uint32_t n, double *out, void *stream) {
    int r = need(c, SPH_F_FP64, n);
    if (r) return r;
    if (!dstate_ok(st) || !out) return fail(c, SPH_E_INVALID_ARG, "null array");
    hipError_t e = launch_totals_d(c, *st, n, out, (hipStream_t)stream);
    return e == hipSuccess ? SPH_OK : hip_fail(c, e, "FP64 totals");
}

int sph_get_dt64(sph_ctx *c, double *dt, void *stream) {
    if (!dt) return c ? fail(c, SPH_E_INVALID_ARG, "null output") : SPH_E_INVALID_ARG;
    DevInfo h;
    int r = read_info(c, &h, stream);
    if (r) return r;
    if (!c->have_dt || c->last_path == 0)
        return fail(c, SPH_E_STATE, "no cell or FP64 interaction yet");
    double m;
    memcpy(&m, &h.dtmin64_bits, sizeof m);
    *dt = c->prm.cfl * m;
    return SPH_OK;
}

}  // extern "C"

/* ------------------------------------------------------------ surrogate */

static void layer_dims(int width, int l, int *in, int *out) {
    *in = l == 0 ? SPH_NN_IN : width;
    *out = l == SPH_NN_LAYERS - 1 ? SPH_NN_OUT : width;
}

static uint64_t split_floats(int32_t width) {
    return (uint64_t)kMlpSplits * (uint64_t)width * SPH_NN_IN;
}

uint64_t sph_mlp_work_floats(int32_t width, uint32_t capacity) {
    if (width <= 0) return 0;
    return split_floats(width) + ((uint64_t)capacity * SPH_NN_OUT + 255) / 256 + 64;
}

static int mlp_check(sph_ctx *c, const sph_mlp *m, bool train) {
    if (!m) return fail(c, SPH_E_INVALID_ARG, "null network");
    if (m->width < 16 || m->width > 256 || m->width % 16)
        return fail(c, SPH_E_INVALID_ARG, "width %d: must be a multiple of 16 in [16, 256]",
                    (int)m->width);
    for (int l = 0; l < SPH_NN_LAYERS; l++)
        if (!m->w[l] || !m->b[l] || !m->wb[l])
            return fail(c, SPH_E_INVALID_ARG, "null weight array of layer %d", l);
    if (!train) return SPH_OK;
    if (m->capacity == 0 || m->capacity > (1u << 20))
        return fail(c, SPH_E_INVALID_ARG, "workspace capacity %u not in [1, 2^20]", m->capacity);
    for (int l = 0; l < SPH_NN_LAYERS; l++)
        if (!m->gw[l] || !m->gb[l] || !m->mw[l] || !m->vw[l] || !m->mb[l] || !m->vb[l] ||
            !m->z[l])
            return fail(c, SPH_E_INVALID_ARG, "null training array of layer %d", l);
    for (int l = 0; l < SPH_NN_LAYERS - 1; l++)
        if (!m->a[l]) return fail(c, SPH_E_INVALID_ARG, "null activation array %d", l);
    if (!m->da || !m->dz || !m->dy || !m->work || !m->loss)
        return fail(c, SPH_E_INVALID_ARG, "null training workspace");
    return SPH_OK;
}

int sph_mlp_sync(sph_ctx *c, sph_mlp *m, void *stream) {
    int r = enter(c);
    if (r) return r;
    if ((r = mlp_check(c, m, false))) return r;
    hipError_t e = hipSuccess;
    for (int l = 0; l < SPH_NN_LAYERS && e == hipSuccess; l++) {
        int in, out;
        layer_dims(m->width, l, &in, &out);
        e = launch_f32_to_bf16(m->w[l], m->wb[l], (long long)in * out, (hipStream_t)stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "mlp sync");
    return SPH_OK;
}

int sph_nn_features(sph_ctx *c, const sph_soa *sorted, const int32_t *rows, uint32_t nrows,
                    const sph_nn_scales *scales, void *x, float *rates, void *stream) {
    int r = enter(c);
    if (r) return r;
    if (!soa_ok(sorted) || !scales || (nrows && !x))
        return fail(c, SPH_E_INVALID_ARG, "null argument");
    if (c->prm.options != 0)
        return fail(c, SPH_E_INVALID_ARG, "surrogate rows use the Wendland kernel: options must be 0");
    if (!c->have_sort || c->last_path != 0)
        return fail(c, SPH_E_STATE, "sph_nn_features needs a preceding sph_sort");
    if (!rows && nrows > c->sorted_n)
        return fail(c, SPH_E_INVALID_ARG, "nrows = %u > n = %u of the sort", nrows, c->sorted_n);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_pack(c, *sorted, c->sorted_n, s);
    if (e == hipSuccess)
        e = launch_nn_features(c, *sorted, rows, nrows, *scales, x, 0, rates, s);
    if (e != hipSuccess) return hip_fail(c, e, "features");
    return SPH_OK;
}

int sph_nn_index(sph_ctx *c, const int32_t *id, uint32_t n, int32_t *where, void *stream) {
    int r = enter(c);
    if (r) return r;
    if (n && (!id || !where)) return fail(c, SPH_E_INVALID_ARG, "null argument");
    if (n > c->capacity) return fail(c, SPH_E_CAPACITY, "n = %u > capacity %u", n, c->capacity);
    hipError_t e = launch_id_scatter(id, n, where, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "index");
    return SPH_OK;
}

int sph_nn_targets(sph_ctx *c, const sph_soa *a, const sph_soa *b, const int32_t *where_b,
                   const int32_t *rows, uint32_t nrows, const float *rates, float span,
                   float inv_dv, float inv_dr, float *t, void *stream) {
    int r = enter(c);
    if (r) return r;
    if (!soa_ok(a) || !soa_ok(b) || (nrows && (!where_b || !t)))
        return fail(c, SPH_E_INVALID_ARG, "null argument");
    hipError_t e = launch_nn_targets(*a, *b, where_b, rows, nrows, rates, span, inv_dv, inv_dr,
                                     t, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "targets");
    return SPH_OK;
}

int sph_mlp_forward(sph_ctx *c, sph_mlp *m, const void *x, uint32_t rows, float *y,
                    void *stream) {
    int r = enter(c);
    if (r) return r;
    if ((r = mlp_check(c, m, true))) return r;
    if (rows > m->capacity)
        return fail(c, SPH_E_CAPACITY, "rows = %u > workspace capacity %u", rows, m->capacity);
    if (rows == 0) return SPH_OK;
    if (!x || !y) return fail(c, SPH_E_INVALID_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    const void *A = x;
    for (int l = 0; l < SPH_NN_LAYERS && e == hipSuccess; l++) {
        int in, out;
        layer_dims(m->width, l, &in, &out);
        // Z = A W^T: B[k][n] = W[n][k]
        e = launch_gemm(A, m->wb[l], m->z[l], (int)rows, out, in, in, 1, 1, in, out, 1, 0,
                        nullptr, s);
        if (e != hipSuccess) break;
        if (l < SPH_NN_LAYERS - 1) {
            e = launch_bias_act(m->z[l], m->b[l], m->a[l], nullptr, rows, out, 1, s);
            A = m->a[l];
        } else {
            e = launch_bias_act(m->z[l], m->b[l], nullptr, y, rows, out, 0, s);
        }
    }
    if (e != hipSuccess) return hip_fail(c, e, "mlp forward");
    return SPH_OK;
}

int sph_mlp_backward(sph_ctx *c, sph_mlp *m, const void *x, uint32_t rows, const float *t,
                     const float *wcol, void *stream) {
    int r = enter(c);
    if (r) return r;
    if ((r = mlp_check(c, m, true))) return r;
    if (rows == 0 || rows > m->capacity)
        return fail(c, SPH_E_CAPACITY, "rows = %u not in [1, %u]", rows, m->capacity);
    if (!x || !t || !wcol) return fail(c, SPH_E_INVALID_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    float *part = m->work, *lpart = m->work + split_floats(m->width);
    hipError_t e = launch_mse(m->z[SPH_NN_LAYERS - 1], t, wcol, m->dy, rows, SPH_NN_OUT, lpart,
                              m->loss, s);
    if (e == hipSuccess) e = launch_act_back(m->dy, nullptr, m->dz, (long long)rows * SPH_NN_OUT, 0, s);
    for (int l = SPH_NN_LAYERS - 1; l >= 0 && e == hipSuccess; l--) {
        int in, out;
        layer_dims(m->width, l, &in, &out);
        const void *Ap = l == 0 ? x : m->a[l - 1];
        // dW (out x in) = dZ^T (out x rows) . A_prev (rows x in)
        e = launch_gemm(m->dz, Ap, m->gw[l], out, in, (int)rows, 1, out, in, 1, in, 1, 0, part, s);
        if (e == hipSuccess) e = launch_colsum(m->dz, rows, out, m->gb[l], s);
        if (l == 0 || e != hipSuccess) continue;
        // dA (rows x in) = dZ (rows x out) . W (out x in); dZ_prev = dA * SiLU'(Z_prev)
        e = launch_gemm(m->dz, m->wb[l], m->da, (int)rows, in, out, out, 1, in, 1, in, 1, 0,
                        nullptr, s);
        if (e == hipSuccess)
            e = launch_act_back(m->da, m->z[l - 1], m->dz, (long long)rows * in, 1, s);
    }
    if (e != hipSuccess) return hip_fail(c, e, "mlp backward");
    return SPH_OK;
}

int sph_mlp_adam(sph_ctx *c, sph_mlp *m, float lr, float beta1, float beta2, float eps,
                 uint32_t t, void *stream) {
    int r = enter(c);
    if (r) return r;
    if ((r = mlp_check(c, m, true))) return r;
    if (t == 0 || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
        return fail(c, SPH_E_INVALID_ARG, "Adam: t >= 1 and betas in [0, 1) required");
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)t));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)t));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    for (int l = 0; l < SPH_NN_LAYERS && e == hipSuccess; l++) {
        int in, out;
        layer_dims(m->width, l, &in, &out);
        e = launch_adam(m->w[l], m->mw[l], m->vw[l], m->gw[l], m->wb[l], (long long)in * out, lr,
                        beta1, beta2, eps, c1, c2, s);
        if (e == hipSuccess)
            e = launch_adam(m->b[l], m->mb[l], m->vb[l], m->gb[l], nullptr, out, lr, beta1, beta2,
                            eps, c1, c2, s);
    }
    if (e != hipSuccess) return hip_fail(c, e, "adam");
    return SPH_OK;
}

int sph_nn_apply(sph_ctx *c, sph_soa *sorted, const float *y, const float *rates, uint32_t nrows,
                 float dv_scale, float dr_scale, float dt4, float rho_tol, int flags,
                 void *stream) {
    int r = enter(c);
    if (r) return r;
    if (!soa_ok(sorted) || (nrows && !y)) return fail(c, SPH_E_INVALID_ARG, "null argument");
    if (!c->have_sort || c->last_path != 0 || nrows > c->sorted_n)
        return fail(c, SPH_E_STATE, "sph_nn_apply needs a preceding sph_sort of >= nrows");
    if (flags & ~(int)(SPH_NN_RESIDUAL | SPH_NN_CARRY_PREV))
        return fail(c, SPH_E_INVALID_ARG, "unknown surrogate flag bits");
    hipError_t e = launch_nn_apply(c, *sorted, y, rates, nrows, dv_scale, dr_scale, dt4, rho_tol,
                                   (flags & SPH_NN_CARRY_PREV) ? 1 : 0, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "apply");
    c->have_dt = false;
    return SPH_OK;
}

int sph_nn_advance(sph_ctx *c, const sph_mlp *m, const sph_soa *cur, sph_soa *next, uint32_t n,
                   const sph_nn_scales *scales, float dv_scale, float dr_scale, float dt4,
                   float rho_tol, int flags, void *stream) {
    int r = enter(c);
    if (r) return r;
    if ((r = mlp_check(c, m, false))) return r;
    if (m->width != 128) return fail(c, SPH_E_INVALID_ARG, "the advance kernel needs width 128");
    if (c->prm.options != 0)
        return fail(c, SPH_E_INVALID_ARG, "surrogate rows use the Wendland kernel: options must be 0");
    if (n > c->capacity) return fail(c, SPH_E_CAPACITY, "n = %u > capacity %u", n, c->capacity);
    if (!soa_ok(cur) || !soa_ok(next) || !scales)
        return fail(c, SPH_E_INVALID_ARG, "null argument");
    if (flags & ~(int)(SPH_NN_RESIDUAL | SPH_NN_CARRY_PREV))
        return fail(c, SPH_E_INVALID_ARG, "unknown surrogate flag bits");
    if (cur->x == next->x || cur->rho == next->rho || cur->type == next->type || cur->id == next->id)
        return fail(c, SPH_E_INVALID_ARG, "cur and next must not share arrays");
    hipStream_t s = (hipStream_t)stream;
    if (!(c->features & SPH_F_SURROGATE))
        return fail(c, SPH_E_STATE,
                    "sph_nn_advance needs a context created with the SPH_F_SURROGATE feature");
    if ((r = do_sort(c, cur, next, n, s))) return r;
    float *rates = (flags & SPH_NN_RESIDUAL) ? c->nn_rate : nullptr;
    hipError_t e = launch_nn_features(c, *next, nullptr, n, *scales, c->nn_x, 1, rates, s);
    if (e == hipSuccess)
        e = launch_nn_mlp_apply(c, *m, *next, c->nn_x, c->nn_y, rates, n, dv_scale, dr_scale,
                                dt4, rho_tol, (flags & SPH_NN_CARRY_PREV) ? 1 : 0, s);
    if (e != hipSuccess) return hip_fail(c, e, "surrogate advance");
    c->have_dt = false;
    return SPH_OK;
}

int sph_nn_perturb(sph_ctx *c, sph_soa *st, uint32_t n, uint32_t seed, float sigma_u,
                   float sigma_rho, void *stream) {
    int r = enter(c);
    if (r) return r;
    if (!soa_ok(st)) return fail(c, SPH_E_INVALID_ARG, "null state array");
    if (n > c->capacity) return fail(c, SPH_E_CAPACITY, "n = %u > capacity %u", n, c->capacity);
    if (!(sigma_u >= 0.0f) || !(sigma_rho >= 0.0f))
        return fail(c, SPH_E_INVALID_ARG, "noise levels must be >= 0");
    hipError_t e = launch_nn_perturb(*st, n, seed, sigma_u, sigma_rho, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "perturb");
    return SPH_OK;
}

int sph_nn_judge(sph_ctx *c, const sph_soa *sv, const sph_soa *rv, const sph_soa *bv,
                 const int32_t *where_r, const int32_t *where_b, uint32_t n, double *out,
                 void *stream) {
    int r = enter(c);
    if (r) return r;
    if (!soa_ok(sv) || !soa_ok(rv) || !soa_ok(bv) || !out || (n && (!where_r || !where_b)))
        return fail(c, SPH_E_INVALID_ARG, "null argument");
    if (n > c->capacity) return fail(c, SPH_E_CAPACITY, "n = %u > capacity %u", n, c->capacity);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_nn_judge(*sv, *rv, *bv, where_r, where_b, n, c->nn_part, c->nn_out, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, c->nn_out, 8 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "judge");
    return SPH_OK;
}
