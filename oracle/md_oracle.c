/*
 * md_oracle.c -- TEST INFRASTRUCTURE ONLY (see md_oracle.h).
 *
 * Plain FP64 reference for the per-step short-range MD work of Rapaport,
 * arXiv:2003.14061, section 2.3.  Written for a reader to check against the
 * paper by eye: single loops, no blocking, no fusion.  The only parallelism
 * is an OpenMP "parallel for" over atoms in loops whose iterations are
 * independent; every per-atom sum runs serially in a fixed order, and every
 * global sum runs serially in id order, so results do not depend on the
 * thread count.
 *
 * Floating-point conventions (shared with the GPU path by specification,
 * not by code; both follow the same written reading of the method):
 *   - minimum image: d - L*rint(d/L) with rint rounding half to even and
 *     1/L formed once;
 *   - squared distance: dx*dx, then two fused multiply-adds (C99 fma);
 *   - list membership r2 < (r_cut+skin)^2 and interaction r2 < r_cut^2,
 *     both strict;
 *   - cell of a coordinate: floor(x * (nc/L)), clamped to nc-1;
 *   - kick v + (dt/(2m))*f and drift x + dt*v as a multiply then an add.
 * The file is compiled with -ffp-contract=off so that no other fusion
 * happens.
 */
#include "md_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int32_t or_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Potential.  The paper names soft spheres (SP, cutoff 2^(1/6)) and
 * Lennard-Jones (cutoff 2.5) but leaves the formulae to its references; the
 * standard 12-6 form is used:
 *   u(r) = 4 eps [ (sigma/r)^12 - (sigma/r)^6 ] - u_shift,   r < r_cut
 *   F_i  = 48 eps / r^2 [ (sigma/r)^12 - (sigma/r)^6 / 2 ] (r_i - r_j)
 * Soft spheres are this potential cut and shifted at r_cut = 2^(1/6) sigma. */

double or_shift(const or_sys* s)
{
    if (s->potential != OR_LJ_SHIFTED) return 0.0;
    double sr2 = (s->sigma * s->sigma) / (s->r_cut * s->r_cut);
    double sr6 = sr2 * sr2 * sr2;
    return 4.0 * s->eps * (sr6 * sr6 - sr6);
}

double or_pair(const or_sys* s, double r2, double* fr)
{
    double rc2 = s->r_cut * s->r_cut;
    if (!(r2 < rc2)) {
        *fr = 0.0;
        return 0.0;
    }
    double sr2 = (s->sigma * s->sigma) / r2;
    double sr6 = sr2 * sr2 * sr2;
    double sr12 = sr6 * sr6;
    *fr = 48.0 * s->eps * (sr12 - 0.5 * sr6) / r2;
    return 4.0 * s->eps * (sr12 - sr6) - or_shift(s);
}

/* ------------------------------------------------------------------ */
/* Periodic box. */

double or_wrap(double x, double L)
{
    /* An atom moves far less than L per step, so x is in (-L, 2L).
     * x - L is exact for x in [L, 2L); x + L may round up to L, which is
     * mapped to 0 so that the result always lies in [0, L). */
    if (x >= L) {
        x -= L;
    } else if (x < 0.0) {
        x += L;
        if (x >= L) x = 0.0;
    }
    return x;
}

double or_minimg(double d, double L, double invL)
{
    return d - L * rint(d * invL);
}

double or_dist2(double dx, double dy, double dz)
{
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

/* ------------------------------------------------------------------ */
/* N1-N4: cells of width w = L/nc >= r_cell; nc = floor(L/r_cell). */

int32_t or_cells_per_side(double L, double r_cell)
{
    return (int32_t)floor(L / r_cell);
}

static int32_t cell_1d(double x, double inv_w, int32_t nc)
{
    int32_t c = (int32_t)floor(x * inv_w);
    if (c < 0) c = 0;
    if (c > nc - 1) c = nc - 1;
    return c;
}

static int32_t wrap_cell(int32_t c, int32_t nc)
{
    if (c < 0) return c + nc;
    if (c >= nc) return c - nc;
    return c;
}

void or_build_cells(const or_sys* s, int32_t nc,
                    const double* x, const double* y, const double* z,
                    int32_t* cell_of, int32_t* cell_start, int32_t* cell_atoms)
{
    int32_t n = s->n;
    int64_t ncell = (int64_t)nc * nc * nc;
    double inv_w = (double)nc / s->L;

    /* N1: cell of every atom */
    for (int32_t i = 0; i < n; ++i) {
        int32_t cx = cell_1d(x[i], inv_w, nc);
        int32_t cy = cell_1d(y[i], inv_w, nc);
        int32_t cz = cell_1d(z[i], inv_w, nc);
        cell_of[i] = (cz * nc + cy) * nc + cx;
    }
    /* N2/N3: occupancy counts, then offsets (exclusive prefix sum) */
    for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = 0;
    for (int32_t i = 0; i < n; ++i) cell_start[cell_of[i] + 1] += 1;
    for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
    /* N4: fill each cell; visiting atoms in id order leaves every cell's
     * members in ascending id */
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)ncell);
    for (int64_t c = 0; c < ncell; ++c) fill[c] = cell_start[c];
    for (int32_t i = 0; i < n; ++i) cell_atoms[fill[cell_of[i]]++] = i;
    free(fill);
}

/* ------------------------------------------------------------------ */
/* N5: neighbor list.  Neighbor cells are visited with dz, dy, dx each
 * running -1, 0, +1 (dz slowest), periodic; within a cell in ascending id. */

int32_t or_build_nl(const or_sys* s, int32_t nc,
                    const double* x, const double* y, const double* z,
                    const int32_t* cell_of, const int32_t* cell_start,
                    const int32_t* cell_atoms,
                    int32_t* nl_count, int32_t* nl)
{
    int32_t n = s->n, cap = s->nl_cap;
    double L = s->L, invL = 1.0 / s->L;
    double r_list = s->r_cut + s->skin;
    double rl2 = r_list * r_list;
    int32_t longest = 0;

#pragma omp parallel for schedule(static) reduction(max : longest)
    for (int32_t i = 0; i < n; ++i) {
        int32_t c = cell_of[i];
        int32_t cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
        int32_t m = 0;
        for (int32_t dz = -1; dz <= 1; ++dz)
            for (int32_t dy = -1; dy <= 1; ++dy)
                for (int32_t dx = -1; dx <= 1; ++dx) {
                    int32_t c2 = (wrap_cell(cz + dz, nc) * nc + wrap_cell(cy + dy, nc)) * nc
                                 + wrap_cell(cx + dx, nc);
                    for (int32_t k = cell_start[c2]; k < cell_start[c2 + 1]; ++k) {
                        int32_t j = cell_atoms[k];
                        if (j == i) continue;
                        double ddx = or_minimg(x[i] - x[j], L, invL);
                        double ddy = or_minimg(y[i] - y[j], L, invL);
                        double ddz = or_minimg(z[i] - z[j], L, invL);
                        if (or_dist2(ddx, ddy, ddz) < rl2) {
                            if (m < cap) nl[(int64_t)i * cap + m] = j;
                            ++m;
                        }
                    }
                }
        nl_count[i] = m < cap ? m : cap;
        if (m > longest) longest = m;
    }
    return longest;
}

/* The half list: the entries of the full list whose partner comes later in
 * the cell order (cell index, then permanent id), in the same order; every
 * pair appears once, in the list of its earlier atom. */
int32_t or_build_nl_half(const or_sys* s, int32_t nc,
                         const double* x, const double* y, const double* z,
                         const int32_t* cell_of, const int32_t* cell_start,
                         const int32_t* cell_atoms,
                         int32_t* nl_count, int32_t* nl)
{
    int32_t n = s->n, cap = s->nl_cap;
    double L = s->L, invL = 1.0 / s->L;
    double r_list = s->r_cut + s->skin;
    double rl2 = r_list * r_list;
    int32_t longest = 0;

#pragma omp parallel for schedule(static) reduction(max : longest)
    for (int32_t i = 0; i < n; ++i) {
        int32_t c = cell_of[i];
        int32_t cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
        int32_t m = 0;
        for (int32_t dz = -1; dz <= 1; ++dz)
            for (int32_t dy = -1; dy <= 1; ++dy)
                for (int32_t dx = -1; dx <= 1; ++dx) {
                    int32_t c2 = (wrap_cell(cz + dz, nc) * nc + wrap_cell(cy + dy, nc)) * nc
                                 + wrap_cell(cx + dx, nc);
                    for (int32_t k = cell_start[c2]; k < cell_start[c2 + 1]; ++k) {
                        int32_t j = cell_atoms[k];
                        if (j == i) continue;
                        if (cell_of[j] < c || (cell_of[j] == c && j < i)) continue;
                        double ddx = or_minimg(x[i] - x[j], L, invL);
                        double ddy = or_minimg(y[i] - y[j], L, invL);
                        double ddz = or_minimg(z[i] - z[j], L, invL);
                        if (or_dist2(ddx, ddy, ddz) < rl2) {
                            if (m < cap) nl[(int64_t)i * cap + m] = j;
                            ++m;
                        }
                    }
                }
        nl_count[i] = m < cap ? m : cap;
        if (m > longest) longest = m;
    }
    return longest;
}

/* ------------------------------------------------------------------ */
/* F1: forces.  Each pair (i, j) contributes to atom i only; it is met again
 * from atom j (full list, section 2.3). */

/* Scale of the rounding error of one pair force: the magnitudes of its
 * repulsive and attractive parts added, 48 eps (sr^12 + sr^6/2) / r.  Where
 * the two parts cancel (near the minimum at 2^(1/6) sigma) this stays of the
 * order of the parts while the force itself goes to zero. */
double or_pair_scale(const or_sys* s, double r2)
{
    if (!(r2 < s->r_cut * s->r_cut)) return 0.0;
    double sr2 = (s->sigma * s->sigma) / r2;
    double sr6 = sr2 * sr2 * sr2;
    return 48.0 * s->eps * (sr6 * sr6 + 0.5 * sr6) / sqrt(r2);
}

static void pair_into(const or_sys* s, double dx, double dy, double dz,
                      double* f3, double* u, double* w, double* sm)
{
    double r2 = or_dist2(dx, dy, dz);
    if (!(r2 < s->r_cut * s->r_cut)) return;
    double fr;
    double up = or_pair(s, r2, &fr);
    f3[0] += fr * dx;
    f3[1] += fr * dy;
    f3[2] += fr * dz;
    *u += 0.5 * up;
    *w += 0.5 * (fr * r2);
    *sm += or_pair_scale(s, r2);
}

static void store_atom(int32_t i, const double* f3, double u, double w, double sm,
                       double* fx, double* fy, double* fz,
                       double* u_i, double* w_i, double* s_i)
{
    fx[i] = f3[0];
    fy[i] = f3[1];
    fz[i] = f3[2];
    if (u_i) u_i[i] = u;
    if (w_i) w_i[i] = w;
    if (s_i) s_i[i] = sm;
}

void or_forces_nl(const or_sys* s,
                  const double* x, const double* y, const double* z,
                  const int32_t* nl_count, const int32_t* nl,
                  double* fx, double* fy, double* fz,
                  double* u_i, double* w_i, double* s_i)
{
    int32_t n = s->n, cap = s->nl_cap;
    double L = s->L, invL = 1.0 / s->L;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double f3[3] = {0.0, 0.0, 0.0}, u = 0.0, w = 0.0, sm = 0.0;
        for (int32_t m = 0; m < nl_count[i]; ++m) {
            int32_t j = nl[(int64_t)i * cap + m];
            pair_into(s, or_minimg(x[i] - x[j], L, invL), or_minimg(y[i] - y[j], L, invL),
                      or_minimg(z[i] - z[j], L, invL), f3, &u, &w, &sm);
        }
        store_atom(i, f3, u, w, sm, fx, fy, fz, u_i, w_i, s_i);
    }
}

/* Forces from a half list (Newton's third law): each listed pair adds F_ij
 * to atom i and -F_ij to atom j, and half of its energy, virial and error
 * scale to each.  Serial, in list order. */
void or_forces_half(const or_sys* s,
                    const double* x, const double* y, const double* z,
                    const int32_t* nl_count, const int32_t* nl,
                    double* fx, double* fy, double* fz,
                    double* u_i, double* w_i, double* s_i)
{
    const int32_t n = s->n;
    const double L = s->L, invL = 1.0 / s->L, rc2 = s->r_cut * s->r_cut;
    for (int32_t i = 0; i < n; ++i) {
        fx[i] = fy[i] = fz[i] = 0.0;
        if (u_i) u_i[i] = 0.0;
        if (w_i) w_i[i] = 0.0;
        if (s_i) s_i[i] = 0.0;
    }
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t m = 0; m < nl_count[i]; ++m) {
            const int32_t j = nl[(int64_t)i * s->nl_cap + m];
            const double dx = or_minimg(x[i] - x[j], L, invL);
            const double dy = or_minimg(y[i] - y[j], L, invL);
            const double dz = or_minimg(z[i] - z[j], L, invL);
            const double r2 = or_dist2(dx, dy, dz);
            if (!(r2 < rc2)) continue;
            double fr;
            const double u = or_pair(s, r2, &fr);  /* shifted pair energy */
            fx[i] += fr * dx;
            fy[i] += fr * dy;
            fz[i] += fr * dz;
            fx[j] -= fr * dx;
            fy[j] -= fr * dy;
            fz[j] -= fr * dz;
            if (u_i) {
                u_i[i] += 0.5 * u;
                u_i[j] += 0.5 * u;
            }
            if (w_i) {
                w_i[i] += 0.5 * fr * r2;
                w_i[j] += 0.5 * fr * r2;
            }
            if (s_i) {
                const double sc = or_pair_scale(s, r2);
                s_i[i] += sc;
                s_i[j] += sc;
            }
        }
    }
}

void or_forces_cells(const or_sys* s, int32_t nc,
                     const double* x, const double* y, const double* z,
                     const int32_t* cell_of, const int32_t* cell_start,
                     const int32_t* cell_atoms,
                     double* fx, double* fy, double* fz,
                     double* u_i, double* w_i, double* s_i)
{
    int32_t n = s->n;
    double L = s->L, invL = 1.0 / s->L;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double f3[3] = {0.0, 0.0, 0.0}, u = 0.0, w = 0.0, sm = 0.0;
        int32_t c = cell_of[i];
        int32_t cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
        for (int32_t dz = -1; dz <= 1; ++dz)
            for (int32_t dy = -1; dy <= 1; ++dy)
                for (int32_t dx = -1; dx <= 1; ++dx) {
                    int32_t c2 = (wrap_cell(cz + dz, nc) * nc + wrap_cell(cy + dy, nc)) * nc
                                 + wrap_cell(cx + dx, nc);
                    for (int32_t k = cell_start[c2]; k < cell_start[c2 + 1]; ++k) {
                        int32_t j = cell_atoms[k];
                        if (j == i) continue;
                        pair_into(s, or_minimg(x[i] - x[j], L, invL),
                                  or_minimg(y[i] - y[j], L, invL),
                                  or_minimg(z[i] - z[j], L, invL), f3, &u, &w, &sm);
                    }
                }
        store_atom(i, f3, u, w, sm, fx, fy, fz, u_i, w_i, s_i);
    }
}

static void brute_one(const or_sys* s, const double* x, const double* y, const double* z,
                      int32_t i, double* f3, double* u, double* w, double* sm)
{
    double L = s->L, invL = 1.0 / s->L;
    for (int32_t j = 0; j < s->n; ++j) {
        if (j == i) continue;
        pair_into(s, or_minimg(x[i] - x[j], L, invL), or_minimg(y[i] - y[j], L, invL),
                  or_minimg(z[i] - z[j], L, invL), f3, u, w, sm);
    }
}

void or_forces_allpairs(const or_sys* s,
                        const double* x, const double* y, const double* z,
                        double* fx, double* fy, double* fz,
                        double* u_i, double* w_i, double* s_i)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < s->n; ++i) {
        double f3[3] = {0.0, 0.0, 0.0}, u = 0.0, w = 0.0, sm = 0.0;
        brute_one(s, x, y, z, i, f3, &u, &w, &sm);
        store_atom(i, f3, u, w, sm, fx, fy, fz, u_i, w_i, s_i);
    }
}

void or_forces_sample(const or_sys* s,
                      const double* x, const double* y, const double* z,
                      const int32_t* idx, int32_t k,
                      double* fx, double* fy, double* fz,
                      double* u_i, double* w_i, double* s_i)
{
#pragma omp parallel for schedule(dynamic)
    for (int32_t q = 0; q < k; ++q) {
        double f3[3] = {0.0, 0.0, 0.0}, u = 0.0, w = 0.0, sm = 0.0;
        brute_one(s, x, y, z, idx[q], f3, &u, &w, &sm);
        store_atom(q, f3, u, w, sm, fx, fy, fz, u_i, w_i, s_i);
    }
}

/* ------------------------------------------------------------------ */
/* F2: reductions (serial, id order). */

double or_sum(const double* a, int32_t n)
{
    double t = 0.0;
    for (int32_t i = 0; i < n; ++i) t += a[i];
    return t;
}

double or_kinetic(const or_sys* s, const double* vx, const double* vy, const double* vz)
{
    double t = 0.0;
    for (int32_t i = 0; i < s->n; ++i) t += (vx[i] * vx[i] + vy[i] * vy[i]) + vz[i] * vz[i];
    return 0.5 * s->mass * t;
}

void or_momentum(const or_sys* s, const double* vx, const double* vy, const double* vz,
                 double* p3)
{
    double px = 0.0, py = 0.0, pz = 0.0;
    for (int32_t i = 0; i < s->n; ++i) {
        px += vx[i];
        py += vy[i];
        pz += vz[i];
    }
    p3[0] = s->mass * px;
    p3[1] = s->mass * py;
    p3[2] = s->mass * pz;
}

double or_max_disp2(const or_sys* s,
                    const double* x, const double* y, const double* z,
                    const double* xr, const double* yr, const double* zr)
{
    double L = s->L, invL = 1.0 / s->L, m = 0.0;
    for (int32_t i = 0; i < s->n; ++i) {
        double d2 = or_dist2(or_minimg(x[i] - xr[i], L, invL), or_minimg(y[i] - yr[i], L, invL),
                             or_minimg(z[i] - zr[i], L, invL));
        if (d2 > m) m = d2;
    }
    return m;
}

/* ------------------------------------------------------------------ */
/* Leapfrog, kick-drift-kick. */

void or_kick(const or_sys* s, double* vx, double* vy, double* vz,
             const double* fx, const double* fy, const double* fz)
{
    double h = (0.5 * s->dt) / s->mass;
    for (int32_t i = 0; i < s->n; ++i) {
        vx[i] = vx[i] + h * fx[i];
        vy[i] = vy[i] + h * fy[i];
        vz[i] = vz[i] + h * fz[i];
    }
}

void or_drift(const or_sys* s, double* x, double* y, double* z,
              const double* vx, const double* vy, const double* vz)
{
    for (int32_t i = 0; i < s->n; ++i) {
        x[i] = or_wrap(x[i] + s->dt * vx[i], s->L);
        y[i] = or_wrap(y[i] + s->dt * vy[i], s->L);
        z[i] = or_wrap(z[i] + s->dt * vz[i], s->L);
    }
}

/* ------------------------------------------------------------------ */
/* A whole run. */

typedef struct {
    int32_t nc;
    int32_t *cell_of, *cell_start, *cell_atoms, *nl_count, *nl;
    double *xr, *yr, *zr, *u_i, *w_i;
} run_ws;

static int32_t rebuild(const or_sys* s, run_ws* ws,
                       const double* x, const double* y, const double* z)
{
    or_build_cells(s, ws->nc, x, y, z, ws->cell_of, ws->cell_start, ws->cell_atoms);
    if (!s->use_nl) return 0;
    int32_t longest = or_build_nl(s, ws->nc, x, y, z, ws->cell_of, ws->cell_start,
                                  ws->cell_atoms, ws->nl_count, ws->nl);
    memcpy(ws->xr, x, sizeof(double) * (size_t)s->n);
    memcpy(ws->yr, y, sizeof(double) * (size_t)s->n);
    memcpy(ws->zr, z, sizeof(double) * (size_t)s->n);
    return longest;
}

static void forces(const or_sys* s, run_ws* ws,
                   const double* x, const double* y, const double* z,
                   double* fx, double* fy, double* fz)
{
    if (s->use_nl)
        or_forces_nl(s, x, y, z, ws->nl_count, ws->nl, fx, fy, fz, ws->u_i, ws->w_i, NULL);
    else
        or_forces_cells(s, ws->nc, x, y, z, ws->cell_of, ws->cell_start, ws->cell_atoms,
                        fx, fy, fz, ws->u_i, ws->w_i, NULL);
}

int32_t or_run(const or_sys* s, int32_t n_steps,
               double* x, double* y, double* z,
               double* vx, double* vy, double* vz,
               double* fx, double* fy, double* fz,
               or_obs* obs)
{
    return or_run_hooked(s, NULL, NULL, n_steps, x, y, z, vx, vy, vz, fx, fy, fz, obs);
}

int32_t or_run_hooked(const or_sys* s, or_force_hook hook, const void* hook_ctx,
                      int32_t n_steps,
                      double* x, double* y, double* z,
                      double* vx, double* vy, double* vz,
                      double* fx, double* fy, double* fz,
                      or_obs* obs)
{
    if (s->n <= 0 || n_steps < 0 || s->L <= 0.0) return -1;
    double r_cell = s->use_nl ? s->r_cut + s->skin : s->r_cut;
    run_ws ws;
    ws.nc = or_cells_per_side(s->L, r_cell);
    if (ws.nc < 3) return -2;
    int64_t ncell = (int64_t)ws.nc * ws.nc * ws.nc;
    size_t n = (size_t)s->n;
    ws.cell_of = (int32_t*)malloc(sizeof(int32_t) * n);
    ws.cell_start = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
    ws.cell_atoms = (int32_t*)malloc(sizeof(int32_t) * n);
    ws.nl_count = (int32_t*)malloc(sizeof(int32_t) * n);
    ws.nl = s->use_nl ? (int32_t*)malloc(sizeof(int32_t) * n * (size_t)s->nl_cap) : NULL;
    ws.xr = (double*)malloc(sizeof(double) * n);
    ws.yr = (double*)malloc(sizeof(double) * n);
    ws.zr = (double*)malloc(sizeof(double) * n);
    ws.u_i = (double*)malloc(sizeof(double) * n);
    ws.w_i = (double*)malloc(sizeof(double) * n);

    double thr = (0.5 * s->skin) * (0.5 * s->skin);
    int32_t n_rebuild = 0, err = 0;
    int32_t longest = rebuild(s, &ws, x, y, z);
    if (longest > s->nl_cap) err = -3;
    if (!err) forces(s, &ws, x, y, z, fx, fy, fz);
    if (!err && hook) err = hook(hook_ctx, s, x, y, z, fx, fy, fz, ws.u_i, ws.w_i);

    for (int32_t step = 0; step < n_steps && !err; ++step) {
        or_kick(s, vx, vy, vz, fx, fy, fz);
        or_drift(s, x, y, z, vx, vy, vz);
        int32_t rebuilt = 0;
        double dmax2 = 0.0;
        longest = 0;
        if (s->use_nl) {
            dmax2 = or_max_disp2(s, x, y, z, ws.xr, ws.yr, ws.zr);
            if (dmax2 > thr) rebuilt = 1;
        } else {
            rebuilt = 1; /* cell-only mode: cells must follow every step */
        }
        if (rebuilt) {
            longest = rebuild(s, &ws, x, y, z);
            if (longest > s->nl_cap) {
                err = -3;
                break;
            }
            if (s->use_nl) ++n_rebuild;
        }
        forces(s, &ws, x, y, z, fx, fy, fz);
        if (hook) {
            err = hook(hook_ctx, s, x, y, z, fx, fy, fz, ws.u_i, ws.w_i);
            if (err) break;
        }
        or_kick(s, vx, vy, vz, fx, fy, fz);
        if (obs) {
            or_obs* o = &obs[step];
            o->U = or_sum(ws.u_i, s->n);
            o->W = or_sum(ws.w_i, s->n);
            o->K = or_kinetic(s, vx, vy, vz);
            or_momentum(s, vx, vy, vz, o->P);
            o->dmax2 = dmax2;
            o->rebuilt = rebuilt;
            o->max_nl = longest;
        }
    }

    free(ws.cell_of);
    free(ws.cell_start);
    free(ws.cell_atoms);
    free(ws.nl_count);
    free(ws.nl);
    free(ws.xr);
    free(ws.yr);
    free(ws.zr);
    free(ws.u_i);
    free(ws.w_i);
    return err ? err : n_rebuild;
}
