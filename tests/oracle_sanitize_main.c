/*
 * Driver for the sanitizer build of the FP64 oracle (test infrastructure).
 *
 * Compiled together with oracle/sph_oracle.c (included below, one translation
 * unit) with AddressSanitizer and UndefinedBehaviorSanitizer, it runs every
 * entry point of the oracle on a small state that has fluid, boundary and
 * ghost particles, particles outside the grid, a non-finite position and
 * slab migration labels, then checks a few invariants (cell-list sums equal
 * brute-force sums, counts add up). Any memory error or undefined behaviour
 * aborts with a sanitizer report; a failed invariant exits with status 2.
 */
#include "../oracle/sph_oracle.c"

#include <stdio.h>

static uint32_t lcg = 12345u;
static double urand(void) /* uniform in [0, 1), a fixed linear congruential sequence */
{
    lcg = lcg * 1664525u + 1013904223u;
    return (double)(lcg >> 8) / 16777216.0;
}

#define NMAX 4096

static double x[NMAX], y[NMAX], z[NMAX], vx[NMAX], vy[NMAX], vz[NMAX], rho[NMAX];
static double vxp[NMAX], vyp[NMAX], vzp[NMAX], rhop[NMAX];
static uint8_t type[NMAX];
static uint32_t key[NMAX], skey[NMAX];
static int32_t perm[NMAX];
static double sx[NMAX], sy[NMAX], sz[NMAX], svx[NMAX], svy[NMAX], svz[NMAX], srho[NMAX];
static double svxp[NMAX], svyp[NMAX], svzp[NMAX], srhop[NMAX];
static uint8_t stype[NMAX];
static double ax[NMAX], ay[NMAX], az[NMAX], drho[NMAX], nu[NMAX], pr[NMAX], cs[NMAX];
static double bx[NMAX], by[NMAX], bz[NMAX], bdrho[NMAX], bnu[NMAX];
static int64_t npair[NMAX], bnpair[NMAX];
static double hx[NMAX], hy[NMAX], hz[NMAX], hvx[NMAX], hvy[NMAX], hvz[NMAX], hrho[NMAX];

static int fail(const char *what)
{
    fprintf(stderr, "invariant failed: %s\n", what);
    return 2;
}

static int run(int slab)
{
    const double dp = 0.02, h = 1.3 * dp;
    orc_params p;
    memset(&p, 0, sizeof p);
    p.dp = dp; p.h = h; p.rho0 = 1000; p.gamma = 7; p.c0 = 17.155174; p.alpha = 0.01;
    p.eta_over_h = 0.1; p.cfl = 0.2; p.mass = 1000 * dp * dp * dp;
    p.g[2] = -9.81;
    p.euler_every = 40;
    const double c2h = 2 * h;
    if (slab) {
        p.slab_mode = 1; p.slab_xlo = 0.0; p.slab_xhi = 6 * c2h;
        p.origin[0] = -c2h; p.ncell[0] = 8;
    } else {
        p.origin[0] = -c2h; p.ncell[0] = 9;
    }
    p.origin[1] = -c2h; p.origin[2] = -c2h; p.ncell[1] = 7; p.ncell[2] = 7;

    int64_t n = 0;
    for (int i = 0; i < 10; i++)
        for (int j = 0; j < 9; j++)
            for (int k = 0; k < 8; k++) {
                x[n] = (i + 0.5) * dp + 1e-4 * dp * (urand() - 0.5);
                y[n] = (j + 0.5) * dp + 1e-4 * dp * (urand() - 0.5);
                z[n] = (k + 0.5) * dp + 1e-4 * dp * (urand() - 0.5);
                vx[n] = urand() - 0.5; vy[n] = urand() - 0.5; vz[n] = urand() - 0.5;
                rho[n] = 1000 * (1 + 0.01 * (urand() - 0.5));
                type[n] = (k == 0) ? T_BOUNDARY : (i == 0 && slab ? T_GHOST : T_FLUID);
                n++;
            }
    /* outside the grid, a non-finite position, migrants on both sides */
    x[n] = 50; y[n] = 0.05; z[n] = 0.05; type[n] = T_FLUID; rho[n] = 1000; n++;
    x[n] = NAN; y[n] = 0.05; z[n] = 0.05; type[n] = T_FLUID; rho[n] = 1000; n++;
    x[n] = -0.3 * dp; y[n] = 0.05; z[n] = 0.05; type[n] = T_FLUID; rho[n] = 1000; n++;
    x[n] = 6 * c2h + 0.2 * dp; y[n] = 0.05; z[n] = 0.05; type[n] = T_FLUID; rho[n] = 1000; n++;
    for (int64_t i = 0; i < n; i++) {
        vxp[i] = vx[i]; vyp[i] = vy[i]; vzp[i] = vz[i]; rhop[i] = rho[i];
    }

    const int bc = orc_cell_bits(&p);
    orc_keys(&p, n, x, y, z, type, key);
    orc_stable_sort(n, key, skey, perm);
    for (int64_t k = 0; k < n; k++) {
        const int32_t s = perm[k];
        sx[k] = x[s]; sy[k] = y[s]; sz[k] = z[s]; svx[k] = vx[s]; svy[k] = vy[s]; svz[k] = vz[s];
        srho[k] = rho[s]; svxp[k] = vxp[s]; svyp[k] = vyp[s]; svzp[k] = vzp[s];
        srhop[k] = rhop[s]; stype[k] = type[s];
    }
    const int64_t nc = (int64_t)p.ncell[0] * p.ncell[1] * p.ncell[2];
    uint32_t *begin = malloc(sizeof(uint32_t) * nc), *end = malloc(sizeof(uint32_t) * nc);
    uint32_t counts[4], ranges[14];
    orc_cell_tables(&p, n, skey, begin, end, counts);
    orc_ranges(&p, begin, end, counts, ranges);
    if ((int64_t)counts[0] + counts[1] + counts[2] + counts[3] != n) return fail("label counts");
    if (counts[3] != 2) return fail("two particles outside the grid");
    if (slab && (counts[1] != 1 || counts[2] != 1)) return fail("one migrant per face");
    (void)bc;
    const int64_t n0 = counts[0];
    orc_interact(&p, n, sx, sy, sz, svx, svy, svz, srho, stype, skey, begin, end, n0, 0, NULL,
                 ax, ay, az, drho, nu, pr, cs, npair);
    orc_interact_brute(&p, n0, sx, sy, sz, svx, svy, svz, srho, stype, NULL, bx, by, bz, bdrho,
                       bnu, bnpair);
    for (int64_t i = 0; i < n0; i++) {
        if (npair[i] != bnpair[i]) return fail("pair counts: cells vs brute force");
        if (fabs(ax[i] - bx[i]) > 1e-9 * (1 + fabs(bx[i])) ||
            fabs(drho[i] - bdrho[i]) > 1e-9 * (1 + fabs(bdrho[i])))
            return fail("sums: cells vs brute force");
    }
    int64_t rowptr[NMAX + 1];
    static int32_t cols[NMAX * 128];
    const int64_t m1 = orc_neighbours_brute(&p, n0, sx, sy, sz, rowptr, cols, NMAX * 128);
    const int64_t m2 = orc_neighbours_cells(&p, n0, sx, sy, sz, skey, begin, end, rowptr, cols,
                                            NMAX * 128);
    if (m1 != m2) return fail("neighbour list lengths");
    const double dt = orc_dt(&p, n0, stype, ax, ay, az, srho, nu);
    if (!(dt > 0 && isfinite(dt))) return fail("dt");
    orc_symplectic_half(&p, n0, dt, stype, sx, sy, sz, svx, svy, svz, srho, ax, ay, az, drho, hx,
                        hy, hz, hvx, hvy, hvz, hrho);
    orc_symplectic_full(&p, n0, dt, stype, hx, hy, hz, hvx, hvy, hvz, hrho, svxp, svyp, svzp,
                        srhop, hrho, ax, ay, az, drho);
    orc_verlet(&p, n0, 1, dt, stype, sx, sy, sz, svx, svy, svz, srho, svxp, svyp, svzp, srhop, ax,
               ay, az, drho);
    double tot[8];
    orc_totals(&p, n, sx, sy, sz, svx, svy, svz, srho, stype, tot);
    if (!(tot[0] > 0)) return fail("totals");
    int64_t sel[16];
    for (int s = 0; s < 16; s++) sel[s] = (s * 37) % n0;
    int32_t nbr[16 * 64], cnt[16];
    orc_nn_rows(&p, sx, sy, sz, skey, begin, end, 16, sel, (float)(4 * h * h), 64, nbr, cnt);
    double sums[16 * 4];
    orc_nn_sums(&p, sx, sy, sz, svx, svy, svz, srho, 16, sel, nbr, 64, sums);
    for (double r = 0; r < 2.5 * h; r += 0.1 * h) {
        if (!isfinite(orc_kernel_w(r, h) + orc_kernel_f(r, h) + orc_cubic_w(r, h) +
                      orc_cubic_f(r + 1e-3 * h, h) + orc_internal_energy(&p, 990 + 10 * r / h)))
            return fail("kernel values");
    }
    uint32_t kv_k[64], kv_ko[64];
    int32_t kv_v[64], kv_vo[64];
    for (int i = 0; i < 64; i++) { kv_k[i] = (uint32_t)(urand() * 8); kv_v[i] = i; }
    orc_stable_sort_kv(64, kv_k, kv_v, kv_ko, kv_vo);
    for (int i = 1; i < 64; i++)
        if (kv_ko[i - 1] > kv_ko[i] || (kv_ko[i - 1] == kv_ko[i] && kv_vo[i - 1] > kv_vo[i]))
            return fail("stable sort order");
    free(begin);
    free(end);
    return 0;
}

int main(void)
{
    int r = run(0);
    if (!r) r = run(1);
    if (!r) printf("oracle sanitizer run: ok\n");
    return r;
}
