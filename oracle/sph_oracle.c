/*
 * Plain FP64 CPU reference for one weakly-compressible SPH (WCSPH) time step.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library. It shares no code, header, table or
 * constant with the HIP path; both are written independently from the paper
 * (Valdez-Balderas et al., "Towards accelerating SPH simulations for
 * free-surface flows on multi-GPU clusters") and from the readings listed in
 * the design notes.
 *
 * Precision: every physical quantity is FP64. Two integer decisions are taken
 * in FP32 on purpose, in the same precision as the GPU kernels that the oracle
 * checks, so that both sides make the same decision:
 *   - the cell coordinate floorf((x - o) * (1/cs)) of Sec. 3.1 (cells of 2h);
 *   - the neighbour test |r_i - r_j|^2 < (2h)^2 of Sec. 2.2 (compact support,
 *     kappa = 2), evaluated as fmaf(dz,dz, fmaf(dy,dy, fmaf(dx,dx, -r2))) < 0
 *     with r2 = (float)(4h^2): the difference r^2 - 4h^2 as one chain of
 *     fused multiply-adds.
 * Build with -ffp-contract=off so that no other expression is contracted.
 *
 * Particle types: 0 fluid, 1 boundary (dynamic boundary, Sec. 2.3),
 * 2 ghost (halo copy of a neighbouring sub-domain, Sec. 4.2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { T_FLUID = 0, T_BOUNDARY = 1, T_GHOST = 2 };

typedef struct {
    double dp, h, rho0, gamma, c0, alpha, eta_over_h, cfl, mass;
    double g[3];
    double origin[3];
    int32_t ncell[3];
    int32_t euler_every;
    int32_t slab_mode;
    int32_t options;   /* OPT_* bits below */
    double slab_xlo, slab_xhi;
} orc_params;

/* Variants of the plain step: the cubic spline kernel of Sec. 2.2 in place of
 * Wendland C2, a density floor rho >= rho0 for boundary particles after each
 * update (a common practice with dynamic boundaries, not in the paper), and a
 * symplectic integrator in place of the Verlet scheme of Sec. 3.3. */
enum { OPT_CUBIC = 1, OPT_RHO_FLOOR = 2, OPT_SYMPLECTIC = 4 };

int orc_abi_version(void) { return 1; }

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (for timing the oracle at one
 * thread and at all host cores; no effect on any result). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------- keys (a1) */

/* Bits of a linear cell index: smallest b with 2^b >= number of cells. */
int orc_cell_bits(const orc_params *p)
{
    int64_t nc = (int64_t)p->ncell[0] * p->ncell[1] * p->ncell[2];
    int b = 1;
    while (((int64_t)1 << b) < nc) b++;
    return b;
}

/*
 * Sec. 3.1: one label per particle naming its cubic cell of side 2h; Sec. 4.2
 * (migration): 0 stays, 1 moved out to the left, 2 moved out to the right.
 * Label 3 marks a particle outside the cell grid (excluded, never lost
 * silently). Ghosts inside the grid are always label 0.
 * key = label << Bc | ((cx*ncy + cy)*ncz + cz); label-3 keys carry cell 0.
 */
void orc_keys(const orc_params *p, int64_t n, const double *x, const double *y,
              const double *z, const uint8_t *type, uint32_t *key)
{
    const int bc = orc_cell_bits(p);
    const double cs = 2.0 * p->h;
    const float inv = (float)(1.0 / cs);
    const float o[3] = {(float)p->origin[0], (float)p->origin[1], (float)p->origin[2]};
    const float xlo = (float)p->slab_xlo, xhi = (float)p->slab_xhi;
    for (int64_t i = 0; i < n; i++) {
        const float r[3] = {(float)x[i], (float)y[i], (float)z[i]};
        int c[3];
        int inside = 1;
        for (int a = 0; a < 3; a++) {
            const float t = (r[a] - o[a]) * inv;
            if (!(t >= 0.0f && t < (float)p->ncell[a])) { inside = 0; c[a] = 0; }
            else c[a] = (int)floorf(t);
            if (inside && c[a] >= p->ncell[a]) inside = 0;
        }
        uint32_t label = 0, cell = 0;
        if (!inside) {
            label = 3;
        } else {
            cell = (uint32_t)(((int64_t)c[0] * p->ncell[1] + c[1]) * p->ncell[2] + c[2]);
            if (p->slab_mode && type[i] != T_GHOST) {
                if (r[0] < xlo) label = 1;
                else if (r[0] >= xhi) label = 2;
            }
        }
        key[i] = (label << bc) | cell;
    }
}

/* --------------------------------------------------------- stable sort (a2) */

typedef struct { uint32_t k; int32_t i; } kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *u = (const kv_t *)a, *v = (const kv_t *)b;
    if (u->k != v->k) return u->k < v->k ? -1 : 1;
    return (u->i > v->i) - (u->i < v->i);  /* ties keep input order (stable) */
}

/* Sort (key, original index) by key; equal keys keep their input order, as in
 * the radix-sort example of Sec. 4.3. perm[k] = input position of output k. */
void orc_stable_sort(int64_t n, const uint32_t *key, uint32_t *key_out, int32_t *perm)
{
    kv_t *t = (kv_t *)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) { t[i].k = key[i]; t[i].i = (int32_t)i; }
    qsort(t, (size_t)n, sizeof(kv_t), kv_cmp);
    for (int64_t i = 0; i < n; i++) { key_out[i] = t[i].k; perm[i] = t[i].i; }
    free(t);
}

/* Sort arbitrary (key, value) pairs stably by key (values travel with keys). */
void orc_stable_sort_kv(int64_t n, const uint32_t *key, const int32_t *val,
                        uint32_t *key_out, int32_t *val_out)
{
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    orc_stable_sort(n, key, key_out, perm);
    for (int64_t i = 0; i < n; i++) val_out[i] = val[perm[i]];
    free(perm);
}

/* ------------------------------------------------------- cell tables (a4/a5) */

static int64_t lower_bound_u32(const uint32_t *a, int64_t n, uint32_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/*
 * Sec. 3.1 (index of the first particle of each cell) and Sec. 4.4 (first and
 * last particle of a region). Over the label-0 prefix of the sorted keys:
 * begin[c] = lower_bound(c), end[c] = upper_bound(c); an empty cell has
 * begin = end = lower_bound(c). counts[l] = particles with label l.
 */
void orc_cell_tables(const orc_params *p, int64_t n, const uint32_t *skey,
                     uint32_t *begin, uint32_t *end, uint32_t *counts)
{
    const int bc = orc_cell_bits(p);
    const int64_t nc = (int64_t)p->ncell[0] * p->ncell[1] * p->ncell[2];
    int64_t start[5];
    for (uint32_t l = 0; l < 4; l++) start[l] = lower_bound_u32(skey, n, l << bc);
    start[4] = n;
    for (int l = 0; l < 4; l++) counts[l] = (uint32_t)(start[l + 1] - start[l]);
    const int64_t n0 = start[1];
    for (int64_t c = 0; c < nc; c++) {
        begin[c] = (uint32_t)lower_bound_u32(skey, n0, (uint32_t)c);
        end[c] = (uint32_t)lower_bound_u32(skey, n0, (uint32_t)c + 1u);
    }
}

/*
 * Packing ranges of Sec. 4.2-4.3 read off the x-major cell order: every
 * x-layer of cells is one contiguous index range. out[0..1] left halo (layer
 * 0), out[2..3] left edge (layer 1), out[4..5] right edge (layer ncx-2),
 * out[6..7] right halo (layer ncx-1), out[8..9] moved-left range,
 * out[10..11] moved-right range, out[12..13] excluded range.
 */
void orc_ranges(const orc_params *p, const uint32_t *begin, const uint32_t *end,
                const uint32_t *counts, uint32_t *out)
{
    const int64_t layer = (int64_t)p->ncell[1] * p->ncell[2];
    const int ncx = p->ncell[0];
    const int lay[4] = {0, 1, ncx - 2, ncx - 1};
    for (int k = 0; k < 4; k++) {
        int L = lay[k] < 0 ? 0 : lay[k];
        out[2 * k] = begin[L * layer];
        out[2 * k + 1] = end[(L + 1) * layer - 1];
    }
    uint32_t n0 = counts[0], n1 = counts[1], n2 = counts[2], n3 = counts[3];
    out[8] = n0; out[9] = n0 + n1;
    out[10] = n0 + n1; out[11] = n0 + n1 + n2;
    out[12] = n0 + n1 + n2; out[13] = n0 + n1 + n2 + n3;
}

/* ------------------------------------------------------------ kernel, EOS */

/* Wendland C2 kernel in 3-D (the workload's choice in place of the cubic
 * spline of Sec. 2.2): W(q) = aD (1 - q/2)^4 (2q + 1), q = r/h <= 2,
 * aD = 21 / (16 pi h^3). */
double orc_kernel_w(double r, double h)
{
    const double q = r / h;
    if (q >= 2.0) return 0.0;
    const double aD = 21.0 / (16.0 * M_PI * h * h * h);
    const double t = 1.0 - 0.5 * q;
    return aD * t * t * t * t * (2.0 * q + 1.0);
}

/* grad_i W_ij = F(r) * (r_i - r_j): dW/dq = -5 aD q (1 - q/2)^3, so
 * F = (dW/dr) / r = -5 aD (1 - q/2)^3 / h^2. */
double orc_kernel_f(double r, double h)
{
    const double q = r / h;
    if (q >= 2.0) return 0.0;
    const double aD = 21.0 / (16.0 * M_PI * h * h * h);
    const double t = 1.0 - 0.5 * q;
    return -5.0 * aD * t * t * t / (h * h);
}

/* Cubic spline kernel in 3-D (the kernel of Sec. 2.2, support 2h), in the
 * textbook form with q = r/h and aD = 1/(pi h^3):
 *   W = aD (1 - 3q^2/2 + 3q^3/4)   for 0 <= q < 1,
 *   W = aD (2 - q)^3 / 4           for 1 <= q < 2,   0 beyond. */
double orc_cubic_w(double r, double h)
{
    const double q = r / h;
    const double aD = 1.0 / (M_PI * h * h * h);
    if (q >= 2.0) return 0.0;
    if (q < 1.0) return aD * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
    const double t = 2.0 - q;
    return aD * 0.25 * t * t * t;
}

/* grad_i W_ij = F(r) (r_i - r_j) for the cubic spline: dW/dq = aD (-3q +
 * 9q^2/4) below q = 1 and -3 aD (2 - q)^2 / 4 above, and F = (dW/dq)/(h r)
 * = (dW/dq) / (h^2 q). */
double orc_cubic_f(double r, double h)
{
    const double q = r / h;
    const double aD = 1.0 / (M_PI * h * h * h);
    if (q >= 2.0) return 0.0;
    if (q < 1.0) return aD * (-3.0 + 2.25 * q) / (h * h);
    const double t = 2.0 - q;
    return -0.75 * aD * t * t / (q * h * h);
}

/* F of the kernel that the parameters select. */
static double kernel_f(const orc_params *p, double r)
{
    return (p->options & OPT_CUBIC) ? orc_cubic_f(r, p->h) : orc_kernel_f(r, p->h);
}

/* Tait equation of state, Sec. 2.2: p = B[(rho/rho0)^gamma - 1],
 * B = c0^2 rho0 / gamma; sound speed c = sqrt(dp/drho) =
 * c0 (rho/rho0)^((gamma-1)/2). */
void orc_eos(const orc_params *p, double rho, double *press, double *c)
{
    const double B = p->c0 * p->c0 * p->rho0 / p->gamma;
    const double r = rho / p->rho0;
    *press = B * (pow(r, p->gamma) - 1.0);
    *c = p->c0 * pow(r, 0.5 * (p->gamma - 1.0));
}

/* ----------------------------------------------------------- pair terms (b) */

typedef struct { double ax, ay, az, drho, nu; } acc_t;

/*
 * Contribution of neighbour j to particle i, Sec. 2.2:
 *   continuity  drho_i/dt += m v_ij . grad_i W_ij
 *   momentum    dv_i/dt   -= m (p_i/rho_i^2 + p_j/rho_j^2 + Pi_ij) grad_i W_ij
 *   Pi_ij = -alpha cbar_ij mu_ij / rhobar_ij if r_ij . v_ij < 0, else 0,
 *   mu_ij = h v_ij . r_ij / (r_ij^2 + eta^2), eta = 0.1 h,
 *   cbar = (c_i + c_j)/2, rhobar = (rho_i + rho_j)/2,
 * and nu_i = max_j |mu_ij| for the CFL limit.
 * (rx, ry, rz) = r_i - r_j and (ux, uy, uz) = v_i - v_j, in FP64.
 */
static void pair_terms(const orc_params *p, double rx, double ry, double rz,
                       double ux, double uy, double uz, double rho_i, double rho_j,
                       double P_i, double P_j, double c_i, double c_j, acc_t *a)
{
    const double h = p->h, m = p->mass;
    const double r2 = rx * rx + ry * ry + rz * rz;
    const double F = kernel_f(p, sqrt(r2));
    const double vr = ux * rx + uy * ry + uz * rz;
    const double eta = p->eta_over_h * h;
    const double mu = h * vr / (r2 + eta * eta);
    double Pi = 0.0;
    if (vr < 0.0)
        Pi = -p->alpha * 0.5 * (c_i + c_j) * mu / (0.5 * (rho_i + rho_j));
    const double s = P_i + P_j + Pi;
    a->ax -= m * s * F * rx;
    a->ay -= m * s * F * ry;
    a->az -= m * s * F * rz;
    a->drho += m * vr * F;
    if (fabs(mu) > a->nu) a->nu = fabs(mu);
}

/* r^2 - 4h^2 in FP32, one fused chain (see header). */
static float support_excess(float dx, float dy, float dz, float r2max)
{
    return fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, -r2max)));
}

/* Neighbour decision in FP32 (see header). */
static int within_support(float xi, float yi, float zi, float xj, float yj, float zj,
                          float r2max)
{
    const float dx = xi - xj, dy = yi - yj, dz = zi - zj;
    return support_excess(dx, dy, dz, r2max) < 0.0f;
}

static float support_r2(const orc_params *p)
{
    return (float)(4.0 * p->h * p->h);
}

/*
 * Interaction (Sec. 3.2): for each selected non-ghost particle i of the
 * label-0 prefix, neighbours j != i are searched in i's cell and the 26 cells
 * around it (cells of 2h, Sec. 3.1). Outputs per selected particle k:
 *   a = -sum_j m(P_i+P_j+Pi_ij) grad W + g for fluid i, 0 otherwise;
 *   D = drho/dt for fluid and boundary i (boundary i: same equations,
 *       Sec. 2.3);
 *   nu = max_j |mu_ij|; p, c from the equation of state; npair = |N(i)|.
 * sel == NULL selects every index in [0, n0); ghosts get zeros.
 */
void orc_interact(const orc_params *p, int64_t n, const double *x, const double *y,
                  const double *z, const double *vx, const double *vy,
                  const double *vz, const double *rho, const uint8_t *type,
                  const uint32_t *skey, const uint32_t *begin, const uint32_t *end,
                  int64_t n0, int64_t nsel, const int64_t *sel, double *ax, double *ay,
                  double *az, double *drho, double *nu, double *press, double *csound,
                  int64_t *npair)
{
    (void)n;
    const int bc = orc_cell_bits(p);
    const uint32_t cmask = (bc >= 32) ? 0xffffffffu : ((1u << bc) - 1u);
    const int ncx = p->ncell[0], ncy = p->ncell[1], ncz = p->ncell[2];
    const float r2max = support_r2(p);
    const int64_t cnt = sel ? nsel : n0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; k++) {
        const int64_t i = sel ? sel[k] : k;
        acc_t a = {0, 0, 0, 0, 0};
        double Pi_, ci, pi;
        orc_eos(p, rho[i], &pi, &ci);
        Pi_ = pi / (rho[i] * rho[i]);
        int64_t np_ = 0;
        if (type[i] != T_GHOST && i < n0) {
            const uint32_t cell = skey[i] & cmask;
            const int cz = (int)(cell % (uint32_t)ncz);
            const int cy = (int)((cell / (uint32_t)ncz) % (uint32_t)ncy);
            const int cx = (int)(cell / ((uint32_t)ncz * (uint32_t)ncy));
            const float xi = (float)x[i], yi = (float)y[i], zi = (float)z[i];
            for (int ox = -1; ox <= 1; ox++)
            for (int oy = -1; oy <= 1; oy++)
            for (int oz = -1; oz <= 1; oz++) {
                const int X = cx + ox, Y = cy + oy, Z = cz + oz;
                if (X < 0 || X >= ncx || Y < 0 || Y >= ncy || Z < 0 || Z >= ncz) continue;
                const int64_t c = ((int64_t)X * ncy + Y) * ncz + Z;
                for (int64_t j = begin[c]; j < (int64_t)end[c]; j++) {
                    if (j == i) continue;
                    if (!within_support(xi, yi, zi, (float)x[j], (float)y[j], (float)z[j], r2max))
                        continue;
                    double pj, cj;
                    orc_eos(p, rho[j], &pj, &cj);
                    pair_terms(p, x[i] - x[j], y[i] - y[j], z[i] - z[j], vx[i] - vx[j],
                               vy[i] - vy[j], vz[i] - vz[j], rho[i], rho[j], Pi_,
                               pj / (rho[j] * rho[j]), ci, cj, &a);
                    np_++;
                }
            }
        }
        if (type[i] == T_FLUID && i < n0) {
            ax[k] = a.ax + p->g[0];
            ay[k] = a.ay + p->g[1];
            az[k] = a.az + p->g[2];
        } else {
            ax[k] = ay[k] = az[k] = 0.0;
        }
        drho[k] = (type[i] != T_GHOST && i < n0) ? a.drho : 0.0;
        nu[k] = a.nu;
        if (press) press[k] = pi;
        if (csound) csound[k] = ci;
        if (npair) npair[k] = np_;
    }
}

/*
 * Brute-force O(N^2) version of the same sums over every pair (for tests):
 * no cells, every non-ghost i against every j != i. With box != NULL the
 * domain is periodic with those side lengths (minimum image), which gives a
 * closed system for momentum-conservation checks.
 */
void orc_interact_brute(const orc_params *p, int64_t n, const double *x, const double *y,
                        const double *z, const double *vx, const double *vy,
                        const double *vz, const double *rho, const uint8_t *type,
                        const double *box, double *ax, double *ay, double *az,
                        double *drho, double *nu, int64_t *npair)
{
    const float r2max = support_r2(p);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        acc_t a = {0, 0, 0, 0, 0};
        double pi, ci;
        orc_eos(p, rho[i], &pi, &ci);
        const double Pi_ = pi / (rho[i] * rho[i]);
        int64_t np_ = 0;
        if (type[i] != T_GHOST) {
            for (int64_t j = 0; j < n; j++) {
                if (j == i) continue;
                double r[3] = {x[i] - x[j], y[i] - y[j], z[i] - z[j]};
                if (box)
                    for (int d = 0; d < 3; d++) r[d] -= box[d] * nearbyint(r[d] / box[d]);
                /* same FP32 test on the (minimum-image) separation */
                const float dx = (float)r[0], dy = (float)r[1], dz = (float)r[2];
                if (box) {
                    if (!(support_excess(dx, dy, dz, r2max) < 0.0f)) continue;
                } else if (!within_support((float)x[i], (float)y[i], (float)z[i], (float)x[j],
                                           (float)y[j], (float)z[j], r2max)) {
                    continue;
                }
                double pj, cj;
                orc_eos(p, rho[j], &pj, &cj);
                pair_terms(p, r[0], r[1], r[2], vx[i] - vx[j], vy[i] - vy[j], vz[i] - vz[j],
                           rho[i], rho[j], Pi_, pj / (rho[j] * rho[j]), ci, cj, &a);
                np_++;
            }
        }
        if (type[i] == T_FLUID) {
            ax[i] = a.ax + p->g[0]; ay[i] = a.ay + p->g[1]; az[i] = a.az + p->g[2];
        } else {
            ax[i] = ay[i] = az[i] = 0.0;
        }
        drho[i] = type[i] != T_GHOST ? a.drho : 0.0;
        nu[i] = a.nu;
        if (npair) npair[i] = np_;
    }
}

/* Neighbour lists by brute force (CSR, j ascending) for sets-equality tests. */
int64_t orc_neighbours_brute(const orc_params *p, int64_t n, const double *x,
                             const double *y, const double *z, int64_t *rowptr,
                             int32_t *cols, int64_t cap)
{
    const float r2max = support_r2(p);
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        rowptr[i] = m;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            if (!within_support((float)x[i], (float)y[i], (float)z[i], (float)x[j],
                                (float)y[j], (float)z[j], r2max))
                continue;
            if (m < cap) cols[m] = (int32_t)j;
            m++;
        }
    }
    rowptr[n] = m;
    return m;
}

/* The same lists through the cell tables (27 cells), in input order of i. */
int64_t orc_neighbours_cells(const orc_params *p, int64_t n0, const double *x,
                             const double *y, const double *z, const uint32_t *skey,
                             const uint32_t *begin, const uint32_t *end, int64_t *rowptr,
                             int32_t *cols, int64_t cap)
{
    const int bc = orc_cell_bits(p);
    const uint32_t cmask = (bc >= 32) ? 0xffffffffu : ((1u << bc) - 1u);
    const int ncx = p->ncell[0], ncy = p->ncell[1], ncz = p->ncell[2];
    const float r2max = support_r2(p);
    int64_t m = 0;
    for (int64_t i = 0; i < n0; i++) {
        rowptr[i] = m;
        const uint32_t cell = skey[i] & cmask;
        const int cz = (int)(cell % (uint32_t)ncz);
        const int cy = (int)((cell / (uint32_t)ncz) % (uint32_t)ncy);
        const int cx = (int)(cell / ((uint32_t)ncz * (uint32_t)ncy));
        for (int ox = -1; ox <= 1; ox++)
        for (int oy = -1; oy <= 1; oy++)
        for (int oz = -1; oz <= 1; oz++) {
            const int X = cx + ox, Y = cy + oy, Z = cz + oz;
            if (X < 0 || X >= ncx || Y < 0 || Y >= ncy || Z < 0 || Z >= ncz) continue;
            const int64_t c = ((int64_t)X * ncy + Y) * ncz + Z;
            for (int64_t j = begin[c]; j < (int64_t)end[c]; j++) {
                if (j == i) continue;
                if (!within_support((float)x[i], (float)y[i], (float)z[i], (float)x[j],
                                    (float)y[j], (float)z[j], r2max))
                    continue;
                if (m < cap) cols[m] = (int32_t)j;
                m++;
            }
        }
    }
    rowptr[n0] = m;
    return m;
}

/* ------------------------------------------------------------- dt (c1) */

/*
 * Variable time step (Sec. 3.3: CFL condition and magnitude of the
 * interactions; Monaghan-Kos form of the cited SPHysics formulation):
 *   dt = CFL * min( min_fluid sqrt(h/|a_i|), min_nonghost h/(c_i + nu_i) ),
 * over the first n0 particles. A particle with |a| = 0 imposes no force limit.
 */
double orc_dt(const orc_params *p, int64_t n0, const uint8_t *type, const double *ax,
              const double *ay, const double *az, const double *rho, const double *nu)
{
    double dtf = INFINITY, dtcv = INFINITY;
    for (int64_t i = 0; i < n0; i++) {
        if (type[i] == T_GHOST) continue;
        double pr, c;
        orc_eos(p, rho[i], &pr, &c);
        const double v = p->h / (c + nu[i]);
        if (v < dtcv) dtcv = v;
        if (type[i] == T_FLUID) {
            const double amag = sqrt(ax[i] * ax[i] + ay[i] * ay[i] + az[i] * az[i]);
            if (amag > 0.0) {
                const double f = sqrt(p->h / amag);
                if (f < dtf) dtf = f;
            }
        }
    }
    return p->cfl * (dtf < dtcv ? dtf : dtcv);
}

/* ---------------------------------------------------------- Verlet (c2) */

/*
 * Second-order Verlet update (Sec. 3.3) in leapfrog form, with an Euler step
 * every euler_every steps (step 0 included):
 *   Euler:    v' = v + dt a,        rho' = rho + dt D
 *   leapfrog: v' = v_prev + 2dt a,  rho' = rho_prev + 2dt D
 *   always    r' = r + dt v + dt^2 a / 2,  then (v_prev, rho_prev) <- (v, rho).
 * Fluid updates r, v, rho. Boundary particles update rho only (position and
 * velocity fixed, Sec. 2.3). Ghosts are not updated. Applies to [0, n0).
 * With OPT_RHO_FLOOR a boundary particle's new density is raised to rho0 when
 * it falls below.
 */
void orc_verlet(const orc_params *p, int64_t n0, int64_t step, double dt,
                const uint8_t *type, double *x, double *y, double *z, double *vx,
                double *vy, double *vz, double *rho, double *vxp, double *vyp, double *vzp,
                double *rhop, const double *ax, const double *ay, const double *az,
                const double *drho)
{
    const int euler = p->euler_every > 0 ? (step % p->euler_every == 0) : (step == 0);
    for (int64_t i = 0; i < n0; i++) {
        if (type[i] == T_GHOST) continue;
        double r_new = euler ? rho[i] + dt * drho[i] : rhop[i] + 2.0 * dt * drho[i];
        if ((p->options & OPT_RHO_FLOOR) && type[i] == T_BOUNDARY && r_new < p->rho0)
            r_new = p->rho0;
        rhop[i] = rho[i];
        rho[i] = r_new;
        if (type[i] != T_FLUID) continue;
        double v[3] = {vx[i], vy[i], vz[i]};
        double vp[3] = {vxp[i], vyp[i], vzp[i]};
        double a[3] = {ax[i], ay[i], az[i]};
        double vn[3];
        for (int d = 0; d < 3; d++) vn[d] = euler ? v[d] + dt * a[d] : vp[d] + 2.0 * dt * a[d];
        x[i] += dt * v[0] + 0.5 * dt * dt * a[0];
        y[i] += dt * v[1] + 0.5 * dt * dt * a[1];
        z[i] += dt * v[2] + 0.5 * dt * dt * a[2];
        vxp[i] = v[0]; vyp[i] = v[1]; vzp[i] = v[2];
        vx[i] = vn[0]; vy[i] = vn[1]; vz[i] = vn[2];
    }
}

/* ----------------------------------------------- symplectic variant (c2) */

/*
 * Symplectic position-Verlet step (kick-drift form of Leimkuhler, Reich and
 * Skeel, as used in SPH codes of the paper's family; an alternative to the
 * Verlet scheme of Sec. 3.3, not in the paper), with dt from the rates at n:
 *   half step:  rho_h = rho + dt/2 D,  and for fluid
 *               r_h = r + dt/2 v,  v_h = v + dt/2 a;
 *   rates a_h, D_h of the half state (orc_interact on it);
 *   full step:  for fluid  v' = v + dt a_h,  r' = r + dt (v + v')/2;
 *               rho' = rho (2 - e) / (2 + e) with e = -(D_h / rho_h) dt
 *               (the exact integral of drho/rho = (D_h/rho_h) dt over a step,
 *               to second order, which keeps rho positive);
 *   then (v_prev, rho_prev) <- (v, rho) at n.
 * Boundary particles move nothing and update rho (Sec. 2.3); ghosts are not
 * updated. OPT_RHO_FLOOR applies to the full step's boundary density.
 */
void orc_symplectic_half(const orc_params *p, int64_t n0, double dt, const uint8_t *type,
                         const double *x, const double *y, const double *z, const double *vx,
                         const double *vy, const double *vz, const double *rho,
                         const double *ax, const double *ay, const double *az,
                         const double *drho, double *xh, double *yh, double *zh, double *vxh,
                         double *vyh, double *vzh, double *rhoh)
{
    (void)p;
    const double hdt = 0.5 * dt;
    for (int64_t i = 0; i < n0; i++) {
        xh[i] = x[i]; yh[i] = y[i]; zh[i] = z[i];
        vxh[i] = vx[i]; vyh[i] = vy[i]; vzh[i] = vz[i];
        rhoh[i] = rho[i];
        if (type[i] == T_GHOST) continue;
        rhoh[i] = rho[i] + hdt * drho[i];
        if (type[i] != T_FLUID) continue;
        xh[i] = x[i] + hdt * vx[i];
        yh[i] = y[i] + hdt * vy[i];
        zh[i] = z[i] + hdt * vz[i];
        vxh[i] = vx[i] + hdt * ax[i];
        vyh[i] = vy[i] + hdt * ay[i];
        vzh[i] = vz[i] + hdt * az[i];
    }
}

void orc_symplectic_full(const orc_params *p, int64_t n0, double dt, const uint8_t *type,
                         double *x, double *y, double *z, double *vx, double *vy, double *vz,
                         double *rho, double *vxp, double *vyp, double *vzp, double *rhop,
                         const double *rhoh, const double *axh, const double *ayh,
                         const double *azh, const double *drhoh)
{
    for (int64_t i = 0; i < n0; i++) {
        if (type[i] == T_GHOST) continue;
        const double e = -(drhoh[i] / rhoh[i]) * dt;
        double r_new = rho[i] * (2.0 - e) / (2.0 + e);
        if ((p->options & OPT_RHO_FLOOR) && type[i] == T_BOUNDARY && r_new < p->rho0)
            r_new = p->rho0;
        rhop[i] = rho[i];
        rho[i] = r_new;
        if (type[i] != T_FLUID) continue;
        double *v[3] = {&vx[i], &vy[i], &vz[i]};
        double *r[3] = {&x[i], &y[i], &z[i]};
        double *vp[3] = {&vxp[i], &vyp[i], &vzp[i]};
        const double a[3] = {axh[i], ayh[i], azh[i]};
        for (int d = 0; d < 3; d++) {
            const double v0 = *v[d];
            const double v1 = v0 + dt * a[d];
            *r[d] += dt * 0.5 * (v0 + v1);
            *vp[d] = v0;
            *v[d] = v1;
        }
    }
}

/* ------------------------------------------------------ global totals */

/* Internal energy per unit mass of the barotropic Tait fluid, the work of
 * the pressure from rho0: e(rho) = int_{rho0}^{rho} p(r)/r^2 dr
 *   = B [ (rho^(g-1) - rho0^(g-1)) / ((g-1) rho0^g) + 1/rho - 1/rho0 ]. */
double orc_internal_energy(const orc_params *p, double rho)
{
    const double B = p->c0 * p->c0 * p->rho0 / p->gamma;
    const double g = p->gamma;
    return B * ((pow(rho, g - 1.0) - pow(p->rho0, g - 1.0)) / ((g - 1.0) * pow(p->rho0, g)) +
                1.0 / rho - 1.0 / p->rho0);
}

/* Totals over the non-ghost particles with finite positions: out[0] mass,
 * out[1..3] momentum, out[4] kinetic energy, out[5] potential energy
 * -m g.r, out[6] internal energy m e(rho), out[7] count. */
void orc_totals(const orc_params *p, int64_t n, const double *x, const double *y,
                const double *z, const double *vx, const double *vy, const double *vz,
                const double *rho, const uint8_t *type, double *out)
{
    for (int q = 0; q < 8; q++) out[q] = 0.0;
    const double m = p->mass;
    for (int64_t i = 0; i < n; i++) {
        if (type[i] == T_GHOST || !isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i])) continue;
        out[0] += m;
        out[1] += m * vx[i];
        out[2] += m * vy[i];
        out[3] += m * vz[i];
        out[4] += 0.5 * m * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
        out[5] += -m * (p->g[0] * x[i] + p->g[1] * y[i] + p->g[2] * z[i]);
        out[6] += m * orc_internal_energy(p, rho[i]);
        out[7] += 1.0;
    }
}

/* ------------------------------------- neighbour rows of the surrogate */

/*
 * Input neighbourhood of the learned surrogate (an addition to the paper's
 * method, built on its cell list of Sec. 3.1): for each selected particle
 * i = sel[s] of the label-0 prefix, the particles j != i of the 27 cells
 * around i's cell with FP32 squared distance
 * fmaf(dz,dz,fmaf(dy,dy,dx*dx)) < r2f (the support test of Sec. 2.2 with a
 * smaller radius), in increasing sorted index (the order in which the cells
 * and the particles within a cell follow each other); the first k go to
 * nbr[s*k ...] (-1 where fewer), the number found to count[s].
 */
void orc_nn_rows(const orc_params *p, const double *x, const double *y, const double *z,
                 const uint32_t *skey, const uint32_t *begin, const uint32_t *end,
                 int64_t nsel, const int64_t *sel, float r2f, int32_t k, int32_t *nbr,
                 int32_t *count)
{
    const int bc = orc_cell_bits(p);
    const uint32_t cmask = (bc >= 32) ? 0xffffffffu : ((1u << bc) - 1u);
    const int ncx = p->ncell[0], ncy = p->ncell[1], ncz = p->ncell[2];
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < nsel; s++) {
        const int64_t i = sel[s];
        const uint32_t cell = skey[i] & cmask;
        const int cz = (int)(cell % (uint32_t)ncz);
        const int cy = (int)((cell / (uint32_t)ncz) % (uint32_t)ncy);
        const int cx = (int)(cell / ((uint32_t)ncz * (uint32_t)ncy));
        int32_t m = 0;
        for (int q = 0; q < k; q++) nbr[s * k + q] = -1;
        for (int ox = -1; ox <= 1; ox++)
        for (int oy = -1; oy <= 1; oy++)
        for (int oz = -1; oz <= 1; oz++) {
            const int X = cx + ox, Y = cy + oy, Z = cz + oz;
            if (X < 0 || X >= ncx || Y < 0 || Y >= ncy || Z < 0 || Z >= ncz) continue;
            const int64_t c = ((int64_t)X * ncy + Y) * ncz + Z;
            for (int64_t j = begin[c]; j < (int64_t)end[c]; j++) {
                if (j == i) continue;
                if (!within_support((float)x[i], (float)y[i], (float)z[i], (float)x[j],
                                    (float)y[j], (float)z[j], r2f))
                    continue;
                if (m < k) nbr[s * k + m] = (int32_t)j;
                m++;
            }
        }
        count[s] = m;
    }
}

/*
 * Pair sums of a surrogate input row over its listed neighbours nbr[s*k ..]
 * (-1 = none), in FP64 with the kernel gradient and equation of state of
 * Sec. 2.2: the pressure part of the momentum equation
 *   ap_i = - sum_j m (p_i/rho_i^2 + p_j/rho_j^2) grad_i W_ij
 * and the continuity rate
 *   dr_i = sum_j m (v_i - v_j) . grad_i W_ij,
 * grad_i W_ij = F(r_ij) (r_i - r_j) with the Wendland kernel whatever the
 * options select (the surrogate's inputs are defined with it).
 * out[4 s ..] = (ap_x, ap_y, ap_z, dr).
 */
void orc_nn_sums(const orc_params *p, const double *x, const double *y, const double *z,
                 const double *vx, const double *vy, const double *vz, const double *rho,
                 int64_t nsel, const int64_t *sel, const int32_t *nbr, int32_t k, double *out)
{
    const double m = p->mass, h = p->h;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < nsel; s++) {
        const int64_t i = sel[s];
        double pi, ci;
        orc_eos(p, rho[i], &pi, &ci);
        const double Pi = pi / (rho[i] * rho[i]);
        double ax = 0.0, ay = 0.0, az = 0.0, dr = 0.0;
        for (int q = 0; q < k; q++) {
            const int32_t j = nbr[s * k + q];
            if (j < 0) continue;
            double pj, cj;
            orc_eos(p, rho[j], &pj, &cj);
            const double Pj = pj / (rho[j] * rho[j]);
            const double rx = x[i] - x[j], ry = y[i] - y[j], rz = z[i] - z[j];
            const double F = orc_kernel_f(sqrt(rx * rx + ry * ry + rz * rz), h);
            const double f = m * (Pi + Pj) * F;
            ax -= f * rx;
            ay -= f * ry;
            az -= f * rz;
            dr += m * F * ((vx[i] - vx[j]) * rx + (vy[i] - vy[j]) * ry + (vz[i] - vz[j]) * rz);
        }
        out[4 * s + 0] = ax;
        out[4 * s + 1] = ay;
        out[4 * s + 2] = az;
        out[4 * s + 3] = dr;
    }
}
