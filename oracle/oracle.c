/*
 * FP64 CPU oracle for the Lennard-Jones molecular-dynamics step of tinyMD
 * (arXiv 2009.07400).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP path is checked against.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * What it computes, and where the paper defines it:
 *   - LJ 12-6 pair force (Sec. 3.2, Eq. 2): with s = |x_ij|^2 and
 *     q = (sigma^2 / s)^3, f = 24 eps q (2 q - 1) / s and F_ij = f x_ij.
 *   - LJ pair energy (the potential written beside Eq. 2): 4 eps (sr6^2 - sr6),
 *     unshifted; virial W = 1/2 sum_i sum_j s f(s).
 *   - Periodic boundaries in all directions (Sec. 3.2): minimum image per
 *     axis, positions wrapped into [0, L) after each drift.
 *   - Cell lists of side >= r = cutoff + skin and the Verlet list of all atoms
 *     within r (Sec. 3.2, Fig. 1 and its caption), full list (each pair stored
 *     for both atoms; Sec. 4.2 and the evaluation setup in Sec. 6); the half
 *     list (each pair once) and its forces by Newton's third law (Sec. 3.2,
 *     the half_nb variant of Sec. 4.2).
 *   - Time integration of Newton's law (Sec. 3.2, Eq. 1) read as
 *     velocity Verlet; lists rebuilt every `rebuild_every` steps (Sec. 6).
 *   - The exact derivative of that discrete map with lists and cutoff
 *     indicators held fixed (adjoint and tangent-linear), for gradients with
 *     respect to epsilon, sigma and the initial state.
 *   - The Spring-Dashpot contact force between spheres (Sec. 3.2, Eq. 3)
 *     with the same lists and integrator (the damping takes the half-step
 *     velocities).
 *
 * Readings where the paper is silent: strict '<' for both the cutoff and the
 * list radius; canonical minimum image `d = a - b; if d > L/2: d -= L; else if
 * d < -L/2: d += L`; s summed left to right as dx*dx + dy*dy + dz*dz; cell
 * count per axis floor(L / r) and the deduplicated 27-cell stencil; each
 * atom's list sorted by atom index; forces summed in list order.
 *
 * Compiled with -ffp-contract=off: no fused multiply-add anywhere here.
 * Parity pins: see tests/test_oracle_*.py (brute force, closed forms,
 * invariants, dot-product and finite-difference checks).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from here on (timing runs only). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Wall-clock seconds, for the per-phase times of orc_run. */
static double wall(void)
{
#ifdef _OPENMP
    return omp_get_wtime();
#else
    return 0.0;
#endif
}

/* ------------------------------------------------------------------ */
/* Pair terms                                                          */
/* ------------------------------------------------------------------ */

/* Scalar LJ force factor f(s) with F_ij = f(s) * x_ij, s = |x_ij|^2, as
 * Sec. 3.2 Eq. 2 writes it: 24 eps (sigma/r)^6 [2 (sigma/r)^6 - 1] / r^2. */
double orc_pair_force(double s, double eps, double sigma)
{
    double t = sigma * sigma / s; /* (sigma/r)^2 */
    double q = t * t * t;         /* (sigma/r)^6 */
    return 24.0 * eps * q * (2.0 * q - 1.0) / s;
}

/* LJ pair energy 4 eps [(sigma/r)^12 - (sigma/r)^6] (beside Eq. 2). */
double orc_pair_energy(double s, double eps, double sigma)
{
    double t = sigma * sigma / s;
    double q = t * t * t;
    return 4.0 * eps * (q * q - q);
}

/* d f / d s = -336 eps sigma^12 s^-8 + 96 eps sigma^6 s^-5 */
static double pair_dforce_ds(double s, double eps, double sigma)
{
    return -336.0 * eps * pow(sigma, 12.0) * pow(s, -8.0) + 96.0 * eps * pow(sigma, 6.0) * pow(s, -5.0);
}

/* d f / d eps = f / eps; d f / d sigma = 576 eps sigma^11 s^-7 - 144 eps sigma^5 s^-4 */
static double pair_dforce_deps(double s, double eps, double sigma)
{
    return orc_pair_force(s, eps, sigma) / eps;
}

static double pair_dforce_dsigma(double s, double eps, double sigma)
{
    return 576.0 * eps * pow(sigma, 11.0) * pow(s, -7.0) - 144.0 * eps * pow(sigma, 5.0) * pow(s, -4.0);
}

/* Canonical minimum-image difference along one axis. */
static double mic(double a, double b, double L)
{
    double d = a - b;
    double h = 0.5 * L;
    if (d > h)
        d -= L;
    else if (d < -h)
        d += L;
    return d;
}

static double dist2(const double *x, const double *y, const double *z, int i, int j, double L,
                    double *dx, double *dy, double *dz)
{
    *dx = mic(x[i], x[j], L);
    *dy = mic(y[i], y[j], L);
    *dz = mic(z[i], z[j], L);
    return *dx * *dx + *dy * *dy + *dz * *dz;
}

/* ------------------------------------------------------------------ */
/* Cells and neighbor lists                                            */
/* ------------------------------------------------------------------ */

int orc_cells_per_axis(double L, double r)
{
    int nc = (int)floor(L / r);
    return nc < 1 ? 1 : nc;
}

static int cell_coord(double p, double side, int nc)
{
    int c = (int)floor(p / side);
    if (c < 0)
        c = 0;
    if (c > nc - 1)
        c = nc - 1;
    return c;
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/*
 * Verlet list of every atom via cell lists: N(i) = { j != i in the
 * deduplicated 27-cell stencil of i's cell : s_ij < r^2 }.  Output is
 * particle-major, nbr[i*maxnb + k], each list sorted ascending.  Entries past
 * maxnb are dropped; the return value is the largest list length seen, so a
 * caller detects overflow by comparing it with maxnb.
 */
long orc_build_list(int n, const double *x, const double *y, const double *z, double L, double r,
                    int maxnb, int *count, int *nbr)
{
    int nc = orc_cells_per_axis(L, r);
    double side = L / nc;
    long ncell = (long)nc * nc * nc;
    int *cell_of = (int *)malloc(sizeof(int) * (size_t)n);
    long *start = (long *)calloc((size_t)ncell + 1, sizeof(long));
    int *sorted = (int *)malloc(sizeof(int) * (size_t)n);
    long *fill = (long *)malloc(sizeof(long) * (size_t)ncell);
    double r2 = r * r;
    long maxc = 0;

    for (int i = 0; i < n; ++i) {
        int cx = cell_coord(x[i], side, nc), cy = cell_coord(y[i], side, nc), cz = cell_coord(z[i], side, nc);
        cell_of[i] = (cz * nc + cy) * nc + cx;
        start[cell_of[i] + 1]++;
    }
    for (long c = 0; c < ncell; ++c)
        start[c + 1] += start[c];
    memcpy(fill, start, sizeof(long) * (size_t)ncell);
    for (int i = 0; i < n; ++i) /* stable: cells hold ascending atom ids */
        sorted[fill[cell_of[i]]++] = i;

#pragma omp parallel for schedule(dynamic, 64) reduction(max : maxc)
    for (int i = 0; i < n; ++i) {
        int c = cell_of[i];
        int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
        int stencil[27];
        int ns = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int sx = (cx + dx + nc) % nc, sy = (cy + dy + nc) % nc, sz = (cz + dz + nc) % nc;
                    int s = (sz * nc + sy) * nc + sx;
                    int dup = 0;
                    for (int q = 0; q < ns; ++q)
                        if (stencil[q] == s)
                            dup = 1;
                    if (!dup)
                        stencil[ns++] = s;
                }
        long cnt = 0;
        int *mine = nbr + (size_t)i * (size_t)maxnb;
        for (int q = 0; q < ns; ++q) {
            for (long p = start[stencil[q]]; p < start[stencil[q] + 1]; ++p) {
                int j = sorted[p];
                double dx, dy, dz;
                if (j == i)
                    continue;
                if (dist2(x, y, z, i, j, L, &dx, &dy, &dz) < r2) {
                    if (cnt < maxnb)
                        mine[cnt] = j;
                    cnt++;
                }
            }
        }
        count[i] = (int)(cnt < maxnb ? cnt : maxnb);
        qsort(mine, (size_t)count[i], sizeof(int), cmp_int);
        if (cnt > maxc)
            maxc = cnt;
    }
    free(cell_of);
    free(start);
    free(sorted);
    free(fill);
    return maxc;
}

/* The same list by the naive all-pairs definition (Sec. 3.2, first
 * paragraph on Verlet lists): every j != i with s_ij < r^2. */
long orc_build_list_brute(int n, const double *x, const double *y, const double *z, double L, double r,
                          int maxnb, int *count, int *nbr)
{
    double r2 = r * r;
    long maxc = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : maxc)
    for (int i = 0; i < n; ++i) {
        long cnt = 0;
        for (int j = 0; j < n; ++j) {
            double dx, dy, dz;
            if (j == i)
                continue;
            if (dist2(x, y, z, i, j, L, &dx, &dy, &dz) < r2) {
                if (cnt < maxnb)
                    nbr[(size_t)i * maxnb + cnt] = j;
                cnt++;
            }
        }
        count[i] = (int)(cnt < maxnb ? cnt : maxnb);
        if (cnt > maxc)
            maxc = cnt;
    }
    return maxc;
}

/* Sorted neighbor ids of one atom by brute force; returns the count (entries
 * beyond cap are counted but not stored). */
long orc_atom_neighbors(int n, const double *x, const double *y, const double *z, double L, double r, int i,
                        int *out, long cap)
{
    double r2 = r * r;
    long cnt = 0;
    for (int j = 0; j < n; ++j) {
        double dx, dy, dz;
        if (j == i)
            continue;
        if (dist2(x, y, z, i, j, L, &dx, &dy, &dz) < r2) {
            if (cnt < cap)
                out[cnt] = j;
            cnt++;
        }
    }
    return cnt;
}

/* ------------------------------------------------------------------ */
/* Forces, energy, virial                                              */
/* ------------------------------------------------------------------ */

/*
 * Totals over atoms (energy, virial, kinetic energy) are compensated sums
 * (Neumaier's variant of Kahan summation): the quantities are exact sums
 * over pairs or atoms, and adding 10^5 to 10^7 similar per-atom terms left
 * to right drifts from that sum by ~1e-12 relative (on a perfect lattice
 * every term is the same and the rounding errors add up).
 */
typedef struct {
    double sum, comp;
} ksum_t;

static void ksum_add(ksum_t *k, double v)
{
    double t = k->sum + v;
    if (fabs(k->sum) >= fabs(v))
        k->comp += (k->sum - t) + v;
    else
        k->comp += (v - t) + k->sum;
    k->sum = t;
}

static double ksum_value(const ksum_t *k)
{
    return k->sum + k->comp;
}

/*
 * F_i = sum over j in list(i) (list order) with s < rc^2 of f(s) d_ij.
 * Optionally per-atom scale[i] = sum_j |f(s) d_ij| (the conditioning scale of
 * the sum), total energy and virial (each pair counted once: 1/2 of the
 * double sum over the full list).
 */
static uint64_t pair_hash(const double *x, const double *y, const double *z, double L, const int *count,
                          const int *nbr, int maxnb, double rc, int n)
{
    /* XOR over interacting pairs (i < j, s < rc^2) of a multiplicative hash of i*n + j:
     * changes whenever a pair crosses the cutoff. */
    uint64_t hsh = 0;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < count[i]; ++k) {
            int j = nbr[(size_t)i * maxnb + k];
            double dx, dy, dz;
            if (j > i && dist2(x, y, z, i, j, L, &dx, &dy, &dz) < rc * rc)
                hsh ^= ((uint64_t)i * (uint64_t)n + (uint64_t)j + 1u) * 0x9E3779B97F4A7C15ull;
        }
    return hsh;
}

void orc_forces(int n, const double *x, const double *y, const double *z, double L, const int *count,
                const int *nbr, int maxnb, double eps, double sigma, double rc, double *fx, double *fy,
                double *fz, double *scale, double *energy, double *virial)
{
    double rc2 = rc * rc;
    double *ui = (double *)calloc((size_t)n, sizeof(double));
    double *wi = (double *)calloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0, sc = 0.0, u = 0.0, w = 0.0;
        for (int k = 0; k < count[i]; ++k) {
            int j = nbr[(size_t)i * maxnb + k];
            double dx, dy, dz;
            double s = dist2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (s < rc2) {
                double f = orc_pair_force(s, eps, sigma);
                ax += f * dx;
                ay += f * dy;
                az += f * dz;
                sc += fabs(f) * sqrt(s);
                u += orc_pair_energy(s, eps, sigma);
                w += s * f;
            }
        }
        fx[i] = ax;
        fy[i] = ay;
        fz[i] = az;
        if (scale)
            scale[i] = sc;
        ui[i] = u;
        wi[i] = w;
    }
    ksum_t U = {0.0, 0.0}, W = {0.0, 0.0};
    for (int i = 0; i < n; ++i) {
        ksum_add(&U, ui[i]);
        ksum_add(&W, wi[i]);
    }
    if (energy)
        *energy = 0.5 * ksum_value(&U);
    if (virial)
        *virial = 0.5 * ksum_value(&W);
    free(ui);
    free(wi);
}

/*
 * Half neighbor list (Sec. 3.2, the paragraph on half lists): every pair of
 * the full list stored once, by the atom of lower index - hlist(i) = { j in
 * list(i) : j > i }, in list order.
 */
void orc_half_list(int n, const int *count, const int *nbr, int maxnb, int *hcount, int *hnbr)
{
    for (int i = 0; i < n; ++i) {
        int c = 0;
        for (int k = 0; k < count[i]; ++k) {
            int j = nbr[(size_t)i * maxnb + k];
            if (j > i)
                hnbr[(size_t)i * maxnb + c++] = j;
        }
        hcount[i] = c;
    }
}

/*
 * Forces from a half list with Newton's third law (Sec. 3.2: the force of a
 * pair is added to i and subtracted from j; the half_nb variant of
 * compute_potential in Sec. 4.2): for i in ascending order and j in hlist(i)
 * with s < rc^2, F_i += f d_ij and F_j -= f d_ij.  One thread, so the order
 * of every sum is the loop order.  Energy and virial count each listed pair
 * once.
 */
void orc_forces_half(int n, const double *x, const double *y, const double *z, double L, const int *hcount,
                     const int *hnbr, int maxnb, double eps, double sigma, double rc, double *fx, double *fy,
                     double *fz, double *energy, double *virial)
{
    double rc2 = rc * rc;
    ksum_t U = {0.0, 0.0}, W = {0.0, 0.0};
    for (int i = 0; i < n; ++i)
        fx[i] = fy[i] = fz[i] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < hcount[i]; ++k) {
            int j = hnbr[(size_t)i * maxnb + k];
            double dx, dy, dz;
            double s = dist2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (s < rc2) {
                double f = orc_pair_force(s, eps, sigma);
                fx[i] += f * dx;
                fy[i] += f * dy;
                fz[i] += f * dz;
                fx[j] -= f * dx;
                fy[j] -= f * dy;
                fz[j] -= f * dz;
                ksum_add(&U, orc_pair_energy(s, eps, sigma));
                ksum_add(&W, s * f);
            }
        }
    if (energy)
        *energy = ksum_value(&U);
    if (virial)
        *virial = ksum_value(&W);
}

/* Force on atom i from every atom j within rc (no list): the all-pairs
 * definition, summed in ascending j.  scale = sum_j |f d_ij|. */
void orc_atom_force(int n, const double *x, const double *y, const double *z, double L, int i, double eps,
                    double sigma, double rc, double *out3, double *scale)
{
    double rc2 = rc * rc, ax = 0.0, ay = 0.0, az = 0.0, sc = 0.0;
    for (int j = 0; j < n; ++j) {
        double dx, dy, dz;
        if (j == i)
            continue;
        double s = dist2(x, y, z, i, j, L, &dx, &dy, &dz);
        if (s < rc2) {
            double f = orc_pair_force(s, eps, sigma);
            ax += f * dx;
            ay += f * dy;
            az += f * dz;
            sc += fabs(f) * sqrt(s);
        }
    }
    out3[0] = ax;
    out3[1] = ay;
    out3[2] = az;
    if (scale)
        *scale = sc;
}

/* ------------------------------------------------------------------ */
/* Velocity Verlet with a fixed rebuild schedule                       */
/* ------------------------------------------------------------------ */

static double wrap1(double p, double L)
{
    if (p >= L)
        p -= L;
    if (p < 0.0)
        p += L;
    return p;
}

static double kinetic(int n, const double *vx, const double *vy, const double *vz, double mass)
{
    ksum_t s = {0.0, 0.0};
    for (int i = 0; i < n; ++i)
        ksum_add(&s, vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
    return 0.5 * mass * ksum_value(&s);
}

/* thermo row: KE, T (3N-3 degrees of freedom), U, W, E = KE + U */
static void thermo_row(double *row, int n, double ke, double u, double w)
{
    row[0] = ke;
    row[1] = 2.0 * ke / (3.0 * n - 3.0);
    row[2] = u;
    row[3] = w;
    row[4] = ke + u;
}

/*
 * Advance (x, v) by nsteps velocity-Verlet steps in place:
 *   v += (dt/2m) F;  x += dt v;  wrap;  [rebuild list if step % rebuild_every == 0];
 *   F = F(x);  v += (dt/2m) F
 * with the initial list and forces computed from the input positions.
 * thermo (nullable) receives nsteps+1 rows of 5 values (row 0 = input state);
 * hashes (nullable) receives nsteps+1 hashes of the set of interacting pairs.
 * Returns the largest list length seen (> maxnb means lists overflowed).
 */
long orc_run(int n, double *x, double *y, double *z, double *vx, double *vy, double *vz, double L, double eps,
             double sigma, double mass, double rc, double skin, double dt, int rebuild_every, int maxnb,
             int nsteps, double *thermo, double *fx, double *fy, double *fz, uint64_t *hashes, double *times)
{
    /* times (nullable): seconds spent in the force sums, the list builds
     * and everything else of the loop (the Force / Neigh / Other split of
     * the paper's Sec. 6 figures) */
    int *count = (int *)malloc(sizeof(int) * (size_t)n);
    int *nbr = (int *)malloc(sizeof(int) * (size_t)n * (size_t)maxnb);
    double h = 0.5 * dt / mass;
    double U, W;
    double t_force = 0.0, t_neigh = 0.0, t_all = wall(), t0;
    t0 = wall();
    long maxc = orc_build_list(n, x, y, z, L, rc + skin, maxnb, count, nbr);
    t_neigh += wall() - t0;
    t0 = wall();
    orc_forces(n, x, y, z, L, count, nbr, maxnb, eps, sigma, rc, fx, fy, fz, NULL, &U, &W);
    t_force += wall() - t0;
    if (thermo)
        thermo_row(thermo, n, kinetic(n, vx, vy, vz, mass), U, W);
    if (hashes)
        hashes[0] = pair_hash(x, y, z, L, count, nbr, maxnb, rc, n);
    for (int step = 1; step <= nsteps; ++step) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            vx[i] = vx[i] + h * fx[i];
            vy[i] = vy[i] + h * fy[i];
            vz[i] = vz[i] + h * fz[i];
            x[i] = wrap1(x[i] + dt * vx[i], L);
            y[i] = wrap1(y[i] + dt * vy[i], L);
            z[i] = wrap1(z[i] + dt * vz[i], L);
        }
        if (rebuild_every > 0 && step % rebuild_every == 0) {
            t0 = wall();
            long m = orc_build_list(n, x, y, z, L, rc + skin, maxnb, count, nbr);
            t_neigh += wall() - t0;
            if (m > maxc)
                maxc = m;
        }
        t0 = wall();
        orc_forces(n, x, y, z, L, count, nbr, maxnb, eps, sigma, rc, fx, fy, fz, NULL, &U, &W);
        t_force += wall() - t0;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            vx[i] = vx[i] + h * fx[i];
            vy[i] = vy[i] + h * fy[i];
            vz[i] = vz[i] + h * fz[i];
        }
        if (thermo)
            thermo_row(thermo + 5 * (size_t)step, n, kinetic(n, vx, vy, vz, mass), U, W);
        if (hashes)
            hashes[step] = pair_hash(x, y, z, L, count, nbr, maxnb, rc, n);
    }
    if (times) {
        times[0] = t_force;
        times[1] = t_neigh;
        times[2] = wall() - t_all - t_force - t_neigh;
    }
    free(count);
    free(nbr);
    return maxc;
}

/* ------------------------------------------------------------------ */
/* Derivatives of the discrete map                                     */
/* ------------------------------------------------------------------ */

/*
 * Jacobian-vector product of the force field, J = dF/dx (symmetric for a
 * symmetric full list), with the list and cutoff indicators held fixed:
 *   (J w)_i = sum_{j in list(i), s < rc^2} [ f(s) (w_i - w_j) + 2 f'(s) (d_ij . (w_i - w_j)) d_ij ].
 * Also accumulates, when gpar is non-null, the force-parameter sensitivities
 * against a vector a:  gpar[0] += sum_i a_i . dF_i/deps,  gpar[1] += sum_i a_i . dF_i/dsigma.
 */
void orc_jvp(int n, const double *x, const double *y, const double *z, double L, const int *count,
             const int *nbr, int maxnb, double eps, double sigma, double rc, const double *wx, const double *wy,
             const double *wz, double *ox, double *oy, double *oz, const double *ax_, const double *ay_,
             const double *az_, double *gpar)
{
    double rc2 = rc * rc;
    double *pe = (double *)calloc((size_t)n, sizeof(double));
    double *ps = (double *)calloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double gx = 0.0, gy = 0.0, gz = 0.0, de = 0.0, ds = 0.0;
        for (int k = 0; k < count[i]; ++k) {
            int j = nbr[(size_t)i * maxnb + k];
            double dx, dy, dz;
            double s = dist2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (!(s < rc2))
                continue;
            double f = orc_pair_force(s, eps, sigma);
            double fp = pair_dforce_ds(s, eps, sigma);
            double ux = wx[i] - wx[j], uy = wy[i] - wy[j], uz = wz[i] - wz[j];
            double dot = dx * ux + dy * uy + dz * uz;
            gx += f * ux + 2.0 * fp * dot * dx;
            gy += f * uy + 2.0 * fp * dot * dy;
            gz += f * uz + 2.0 * fp * dot * dz;
            if (gpar) {
                double adot = ax_[i] * dx + ay_[i] * dy + az_[i] * dz;
                de += pair_dforce_deps(s, eps, sigma) * adot;
                ds += pair_dforce_dsigma(s, eps, sigma) * adot;
            }
        }
        ox[i] = gx;
        oy[i] = gy;
        oz[i] = gz;
        pe[i] = de;
        ps[i] = ds;
    }
    if (gpar) {
        for (int i = 0; i < n; ++i) {
            gpar[0] += pe[i];
            gpar[1] += ps[i];
        }
    }
    free(pe);
    free(ps);
}

/* dF_i/deps and dF_i/dsigma as vectors (for the tangent-linear model). */
static void force_param_derivs(int n, const double *x, const double *y, const double *z, double L,
                               const int *count, const int *nbr, int maxnb, double eps, double sigma, double rc,
                               double *ex, double *ey, double *ez, double *sx, double *sy, double *sz)
{
    double rc2 = rc * rc;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0;
        for (int k = 0; k < count[i]; ++k) {
            int j = nbr[(size_t)i * maxnb + k];
            double dx, dy, dz;
            double s = dist2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (!(s < rc2))
                continue;
            double ge = pair_dforce_deps(s, eps, sigma), gs = pair_dforce_dsigma(s, eps, sigma);
            a0 += ge * dx;
            a1 += ge * dy;
            a2 += ge * dz;
            b0 += gs * dx;
            b1 += gs * dy;
            b2 += gs * dz;
        }
        ex[i] = a0;
        ey[i] = a1;
        ez[i] = a2;
        sx[i] = b0;
        sy[i] = b1;
        sz[i] = b2;
    }
}

/* Forward trajectory with every position and every list kept (plain, no
 * checkpointing).  xs holds (nsteps+1) blocks of 3n doubles. */
typedef struct {
    int n, maxnb, nsteps, rebuild_every, nlists;
    double *xs;  /* [(nsteps+1)][3][n] */
    int *counts; /* [nlists][n] */
    int *nbrs;   /* [nlists][n*maxnb] */
    long maxc;
} traj_t;

static int list_index(const traj_t *t, int step)
{
    return t->rebuild_every > 0 ? step / t->rebuild_every : 0;
}

static void record_forward(traj_t *t, int n, const double *x0, const double *y0, const double *z0,
                           const double *vx0, const double *vy0, const double *vz0, double L, double eps,
                           double sigma, double mass, double rc, double skin, double dt, int rebuild_every,
                           int maxnb, int nsteps, double *vxT, double *vyT, double *vzT)
{
    t->n = n;
    t->maxnb = maxnb;
    t->nsteps = nsteps;
    t->rebuild_every = rebuild_every;
    t->nlists = (rebuild_every > 0 ? nsteps / rebuild_every : 0) + 1;
    t->xs = (double *)malloc(sizeof(double) * 3 * (size_t)n * (size_t)(nsteps + 1));
    t->counts = (int *)malloc(sizeof(int) * (size_t)n * (size_t)t->nlists);
    t->nbrs = (int *)malloc(sizeof(int) * (size_t)n * (size_t)maxnb * (size_t)t->nlists);
    double *x = t->xs, *y = x + n, *z = y + n;
    memcpy(x, x0, sizeof(double) * n);
    memcpy(y, y0, sizeof(double) * n);
    memcpy(z, z0, sizeof(double) * n);
    double *vx = vxT, *vy = vyT, *vz = vzT;
    memcpy(vx, vx0, sizeof(double) * n);
    memcpy(vy, vy0, sizeof(double) * n);
    memcpy(vz, vz0, sizeof(double) * n);
    double *fx = (double *)malloc(sizeof(double) * 3 * (size_t)n), *fy = fx + n, *fz = fy + n;
    double h = 0.5 * dt / mass;
    t->maxc = orc_build_list(n, x, y, z, L, rc + skin, maxnb, t->counts, t->nbrs);
    orc_forces(n, x, y, z, L, t->counts, t->nbrs, maxnb, eps, sigma, rc, fx, fy, fz, NULL, NULL, NULL);
    for (int step = 1; step <= nsteps; ++step) {
        double *px = t->xs + (size_t)(step - 1) * 3 * n, *py = px + n, *pz = py + n;
        x = t->xs + (size_t)step * 3 * n;
        y = x + n;
        z = y + n;
        for (int i = 0; i < n; ++i) {
            vx[i] = vx[i] + h * fx[i];
            vy[i] = vy[i] + h * fy[i];
            vz[i] = vz[i] + h * fz[i];
            x[i] = wrap1(px[i] + dt * vx[i], L);
            y[i] = wrap1(py[i] + dt * vy[i], L);
            z[i] = wrap1(pz[i] + dt * vz[i], L);
        }
        int li = list_index(t, step);
        if (rebuild_every > 0 && step % rebuild_every == 0) {
            long m = orc_build_list(n, x, y, z, L, rc + skin, maxnb, t->counts + (size_t)li * n,
                                    t->nbrs + (size_t)li * n * maxnb);
            if (m > t->maxc)
                t->maxc = m;
        }
        orc_forces(n, x, y, z, L, t->counts + (size_t)li * n, t->nbrs + (size_t)li * n * maxnb, maxnb, eps,
                   sigma, rc, fx, fy, fz, NULL, NULL, NULL);
        for (int i = 0; i < n; ++i) {
            vx[i] = vx[i] + h * fx[i];
            vy[i] = vy[i] + h * fy[i];
            vz[i] = vz[i] + h * fz[i];
        }
    }
    free(fx);
}

static void free_traj(traj_t *t)
{
    free(t->xs);
    free(t->counts);
    free(t->nbrs);
}

/*
 * Reverse-mode derivative of the nsteps velocity-Verlet map.  Given the
 * cotangents (lx, lv) of the final state, returns in place the cotangents of
 * the initial state, and gpar[0..1] = dL/deps, dL/dsigma.  Per step k,
 * going backward with h = dt/(2m):
 *   lx~ = lx_{k+1} + h J(x_{k+1}) lv_{k+1}
 *   lv' = lv_{k+1} + dt lx~
 *   lx_k = lx~ + h J(x_k) lv'
 *   lv_k = lv'
 * and each force evaluation F_m used in a kick adds h (lv after that kick) .
 * dF_m/dtheta to the parameter gradient.  Returns the largest list length.
 */
long orc_adjoint(int n, const double *x0, const double *y0, const double *z0, const double *vx0,
                 const double *vy0, const double *vz0, double L, double eps, double sigma, double mass, double rc,
                 double skin, double dt, int rebuild_every, int maxnb, int nsteps, double *lx, double *ly,
                 double *lz, double *lvx, double *lvy, double *lvz, double *gpar)
{
    traj_t t;
    double *vT = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    record_forward(&t, n, x0, y0, z0, vx0, vy0, vz0, L, eps, sigma, mass, rc, skin, dt, rebuild_every, maxnb,
                   nsteps, vT, vT + n, vT + 2 * n);
    double h = 0.5 * dt / mass;
    double *g = (double *)malloc(sizeof(double) * 3 * (size_t)n), *gy = g + n, *gz = gy + n;
    gpar[0] = 0.0;
    gpar[1] = 0.0;
    for (int k = nsteps - 1; k >= 0; --k) {
        const double *xk1 = t.xs + (size_t)(k + 1) * 3 * n;
        const double *xk = t.xs + (size_t)k * 3 * n;
        int l1 = list_index(&t, k + 1), l0 = list_index(&t, k);
        /* second kick of step k: v_{k+1} = v' + h F(x_{k+1}) */
        double pe[2] = {0.0, 0.0};
        orc_jvp(n, xk1, xk1 + n, xk1 + 2 * n, L, t.counts + (size_t)l1 * n, t.nbrs + (size_t)l1 * n * maxnb,
                maxnb, eps, sigma, rc, lvx, lvy, lvz, g, gy, gz, lvx, lvy, lvz, pe);
        gpar[0] += h * pe[0];
        gpar[1] += h * pe[1];
        for (int i = 0; i < n; ++i) {
            lx[i] = lx[i] + h * g[i];
            ly[i] = ly[i] + h * gy[i];
            lz[i] = lz[i] + h * gz[i];
            lvx[i] = lvx[i] + dt * lx[i];
            lvy[i] = lvy[i] + dt * ly[i];
            lvz[i] = lvz[i] + dt * lz[i];
        }
        /* first kick of step k: v' = v_k + h F(x_k) */
        pe[0] = pe[1] = 0.0;
        orc_jvp(n, xk, xk + n, xk + 2 * n, L, t.counts + (size_t)l0 * n, t.nbrs + (size_t)l0 * n * maxnb, maxnb,
                eps, sigma, rc, lvx, lvy, lvz, g, gy, gz, lvx, lvy, lvz, pe);
        gpar[0] += h * pe[0];
        gpar[1] += h * pe[1];
        for (int i = 0; i < n; ++i) {
            lx[i] = lx[i] + h * g[i];
            ly[i] = ly[i] + h * gy[i];
            lz[i] = lz[i] + h * gz[i];
        }
    }
    long maxc = t.maxc;
    free(g);
    free(vT);
    free_traj(&t);
    return maxc;
}

/*
 * Tangent-linear (forward-mode) derivative of the same map: pushes
 * (dx, dv, deps, dsigma) through nsteps steps, in place on dx, dv:
 *   dF_k = J(x_k) dx_k + dF/deps deps + dF/dsigma dsigma
 *   dv' = dv_k + h dF_k;  dx_{k+1} = dx_k + dt dv';  dv_{k+1} = dv' + h dF_{k+1}
 */
long orc_tangent(int n, const double *x0, const double *y0, const double *z0, const double *vx0,
                 const double *vy0, const double *vz0, double L, double eps, double sigma, double mass, double rc,
                 double skin, double dt, int rebuild_every, int maxnb, int nsteps, double *dx, double *dy,
                 double *dz, double *dvx, double *dvy, double *dvz, double deps, double dsigma)
{
    traj_t t;
    double *vT = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    record_forward(&t, n, x0, y0, z0, vx0, vy0, vz0, L, eps, sigma, mass, rc, skin, dt, rebuild_every, maxnb,
                   nsteps, vT, vT + n, vT + 2 * n);
    double h = 0.5 * dt / mass;
    double *g = (double *)malloc(sizeof(double) * 9 * (size_t)n);
    double *gy = g + n, *gz = gy + n, *ex = gz + n, *ey = ex + n, *ez = ey + n, *sx = ez + n, *sy = sx + n,
           *sz = sy + n;
    for (int k = 0; k < nsteps; ++k) {
        for (int half = 0; half < 2; ++half) {
            int m = k + half; /* force evaluation at x_m */
            const double *xm = t.xs + (size_t)m * 3 * n;
            int li = list_index(&t, m);
            const int *cnt = t.counts + (size_t)li * n;
            const int *nb = t.nbrs + (size_t)li * n * maxnb;
            if (half == 1) {
                for (int i = 0; i < n; ++i) {
                    dx[i] = dx[i] + dt * dvx[i];
                    dy[i] = dy[i] + dt * dvy[i];
                    dz[i] = dz[i] + dt * dvz[i];
                }
            }
            orc_jvp(n, xm, xm + n, xm + 2 * n, L, cnt, nb, maxnb, eps, sigma, rc, dx, dy, dz, g, gy, gz, NULL, NULL,
                    NULL, NULL);
            force_param_derivs(n, xm, xm + n, xm + 2 * n, L, cnt, nb, maxnb, eps, sigma, rc, ex, ey, ez, sx, sy, sz);
            for (int i = 0; i < n; ++i) {
                dvx[i] = dvx[i] + h * (g[i] + ex[i] * deps + sx[i] * dsigma);
                dvy[i] = dvy[i] + h * (gy[i] + ey[i] * deps + sy[i] * dsigma);
                dvz[i] = dvz[i] + h * (gz[i] + ez[i] * deps + sz[i] * dsigma);
            }
        }
    }
    long maxc = t.maxc;
    free(g);
    free(vT);
    free_traj(&t);
    return maxc;
}

/* ------------------------------------------------------------------ */
/* Spring-Dashpot contact model (Sec. 3.2, Eq. 3)                      */
/* ------------------------------------------------------------------ */

/*
 * Spheres of diameter sigma.  For a pair with separation vector x_ij =
 * x_i - x_j (minimum image), distance r = |x_ij|, unit vector u = x_ij / r and
 * relative velocity v_ij = v_i - v_j, Eq. 3 gives the force on i
 *     F_ij = K xi + gamma xi_dot,
 *     xi     = u (sigma - r) Theta(sigma - r),
 *     xi_dot = -u (u . v_ij) Theta(sigma - r),
 * i.e. F_ij = [K (sigma - r) - gamma (u . v_ij)] u while the spheres overlap
 * (r < sigma: Theta(0) read as 0, the contact starts at strict overlap) and
 * zero otherwise.  K is the spring constant, gamma the dissipation constant.
 *
 * Only overlapping pairs interact, so the Verlet list is built at
 * cutoff + skin with cutoff >= sigma and the contact test is r < sigma.
 * The force depends on velocities: in velocity Verlet the force at step
 * k + 1 takes the half-step velocities v_{k+1/2} (the full-step ones need
 * that very force); the first force takes the initial velocities.
 */

/* Force on i from one pair, added to out3; returns the pair force magnitude
 * K (sigma - r) - gamma (u . v_ij) (0 without contact). */
double orc_sd_pair(double dx, double dy, double dz, double dvx, double dvy, double dvz, double k, double gamma,
                   double sigma, double *out3)
{
    double s = dx * dx + dy * dy + dz * dz;
    if (!(s < sigma * sigma))
        return 0.0;
    double r = sqrt(s);
    double ux = dx / r, uy = dy / r, uz = dz / r;
    double un = ux * dvx + uy * dvy + uz * dvz;
    double fm = k * (sigma - r) - gamma * un;
    out3[0] += fm * ux;
    out3[1] += fm * uy;
    out3[2] += fm * uz;
    return fm;
}

/*
 * F_i = sum over j in list(i) (list order) of F_ij.  scale[i] (nullable) =
 * sum_j |F_ij| (the conditioning scale).  energy = the springs' elastic
 * energy 1/2 K (sigma - r)^2 per overlapping pair; virial = sum over pairs
 * of x_ij . F_ij (each pair once: 1/2 of the double sums).
 */
void orc_sd_forces(int n, const double *x, const double *y, const double *z, const double *vx, const double *vy,
                   const double *vz, double L, const int *count, const int *nbr, int maxnb, double k, double gamma,
                   double sigma, double *fx, double *fy, double *fz, double *scale, double *energy, double *virial)
{
    double *ui = (double *)calloc((size_t)n, sizeof(double));
    double *wi = (double *)calloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double a[3] = {0.0, 0.0, 0.0}, sc = 0.0, u = 0.0, w = 0.0;
        for (int q = 0; q < count[i]; ++q) {
            int j = nbr[(size_t)i * maxnb + q];
            double dx, dy, dz;
            double s = dist2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (s < sigma * sigma) {
                double fm = orc_sd_pair(dx, dy, dz, vx[i] - vx[j], vy[i] - vy[j], vz[i] - vz[j], k, gamma, sigma, a);
                double r = sqrt(s);
                sc += fabs(fm);
                u += 0.5 * k * (sigma - r) * (sigma - r);
                w += fm * r;
            }
        }
        fx[i] = a[0];
        fy[i] = a[1];
        fz[i] = a[2];
        if (scale)
            scale[i] = sc;
        ui[i] = u;
        wi[i] = w;
    }
    ksum_t U = {0.0, 0.0}, W = {0.0, 0.0};
    for (int i = 0; i < n; ++i) {
        ksum_add(&U, ui[i]);
        ksum_add(&W, wi[i]);
    }
    if (energy)
        *energy = 0.5 * ksum_value(&U);
    if (virial)
        *virial = 0.5 * ksum_value(&W);
    free(ui);
    free(wi);
}

/* Force on atom i from every atom j (no list), ascending j: the all-pairs
 * definition of Eq. 3. */
void orc_sd_atom_force(int n, const double *x, const double *y, const double *z, const double *vx,
                       const double *vy, const double *vz, double L, int i, double k, double gamma, double sigma,
                       double *out3)
{
    double a[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < n; ++j) {
        double dx, dy, dz;
        if (j == i)
            continue;
        dist2(x, y, z, i, j, L, &dx, &dy, &dz);
        orc_sd_pair(dx, dy, dz, vx[i] - vx[j], vy[i] - vy[j], vz[i] - vz[j], k, gamma, sigma, a);
    }
    out3[0] = a[0];
    out3[1] = a[1];
    out3[2] = a[2];
}

/*
 * Velocity Verlet of Spring-Dashpot spheres, in place:
 *   v += (dt/2m) F;  x += dt v;  wrap;  [rebuild list if step % rebuild_every == 0];
 *   F = F(x, v);  v += (dt/2m) F
 * where the force takes the half-step velocities of the line before it; the
 * initial list and forces come from the input state.  thermo (nullable):
 * nsteps+1 rows (KE, T, U elastic, W, E = KE + U).  Returns the largest list
 * length seen.
 */
long orc_sd_run(int n, double *x, double *y, double *z, double *vx, double *vy, double *vz, double L, double k,
                double gamma, double sigma, double mass, double cutoff, double skin, double dt, int rebuild_every,
                int maxnb, int nsteps, double *thermo, double *fx, double *fy, double *fz)
{
    int *count = (int *)malloc(sizeof(int) * (size_t)n);
    int *nbr = (int *)malloc(sizeof(int) * (size_t)n * (size_t)maxnb);
    double h = 0.5 * dt / mass;
    double U, W;
    long maxc = orc_build_list(n, x, y, z, L, cutoff + skin, maxnb, count, nbr);
    orc_sd_forces(n, x, y, z, vx, vy, vz, L, count, nbr, maxnb, k, gamma, sigma, fx, fy, fz, NULL, &U, &W);
    if (thermo)
        thermo_row(thermo, n, kinetic(n, vx, vy, vz, mass), U, W);
    for (int step = 1; step <= nsteps; ++step) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            vx[i] = vx[i] + h * fx[i];
            vy[i] = vy[i] + h * fy[i];
            vz[i] = vz[i] + h * fz[i];
            x[i] = wrap1(x[i] + dt * vx[i], L);
            y[i] = wrap1(y[i] + dt * vy[i], L);
            z[i] = wrap1(z[i] + dt * vz[i], L);
        }
        if (rebuild_every > 0 && step % rebuild_every == 0) {
            long m = orc_build_list(n, x, y, z, L, cutoff + skin, maxnb, count, nbr);
            if (m > maxc)
                maxc = m;
        }
        orc_sd_forces(n, x, y, z, vx, vy, vz, L, count, nbr, maxnb, k, gamma, sigma, fx, fy, fz, NULL, &U, &W);
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            vx[i] = vx[i] + h * fx[i];
            vy[i] = vy[i] + h * fy[i];
            vz[i] = vz[i] + h * fz[i];
        }
        if (thermo)
            thermo_row(thermo + 5 * (size_t)step, n, kinetic(n, vx, vy, vz, mass), U, W);
    }
    free(count);
    free(nbr);
    return maxc;
}
