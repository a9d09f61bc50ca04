/*
 * md_oracle_adjoint.c -- TEST INFRASTRUCTURE ONLY.  See md_oracle_adjoint.h.
 *
 * Plain FP64 loops.  The forward trajectory is stored whole (every
 * position of every step); the reverse pass walks it backwards, rebuilding
 * the cells and the neighbor list at every point it visits.
 */
#include "md_oracle_adjoint.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Pair derivatives.  With s = sigma / r the pair energy is
 *   u(r) = 4 eps (s^12 - s^6)  (minus a constant shift),
 * so, written out in powers of r:
 *   u'(r)      = 4 eps (-12 sigma^12 r^-13 + 6 sigma^6 r^-7)
 *   fr = -u'/r = 4 eps (12 sigma^12 r^-14 - 6 sigma^6 r^-8)
 *   d fr / dr  = 4 eps (-168 sigma^12 r^-15 + 48 sigma^6 r^-9)
 *   d fr / dsigma = 4 eps (144 sigma^11 r^-14 - 36 sigma^5 r^-8)           */

void or_pair_deriv(const or_sys* s, double r2, double* fr, double* gr, double* fs)
{
    *fr = 0.0;
    *gr = 0.0;
    *fs = 0.0;
    if (!(r2 < s->r_cut * s->r_cut)) return;
    const double r = sqrt(r2);
    const double sg = s->sigma;
    const double sg6 = pow(sg, 6.0), sg12 = sg6 * sg6;
    const double e4 = 4.0 * s->eps;
    *fr = e4 * (12.0 * sg12 * pow(r, -14.0) - 6.0 * sg6 * pow(r, -8.0));
    const double dfr_dr = e4 * (-168.0 * sg12 * pow(r, -15.0) + 48.0 * sg6 * pow(r, -9.0));
    *gr = dfr_dr / r;
    *fs = e4 * (144.0 * pow(sg, 11.0) * pow(r, -14.0) - 36.0 * pow(sg, 5.0) * pow(r, -8.0));
}

static void sep(const or_sys* s, const double* x, const double* y, const double* z, int32_t i,
                int32_t j, double* dx, double* dy, double* dz)
{
    const double invL = 1.0 / s->L;
    *dx = or_minimg(x[i] - x[j], s->L, invL);
    *dy = or_minimg(y[i] - y[j], s->L, invL);
    *dz = or_minimg(z[i] - z[j], s->L, invL);
}

void or_hvp(const or_sys* s, const double* x, const double* y, const double* z,
            const int32_t* nl_count, const int32_t* nl,
            const double* lx, const double* ly, const double* lz,
            double* jx, double* jy, double* jz, double* dfde, double* dfds)
{
    const int32_t n = s->n;
    double* pe = (double*)malloc(sizeof(double) * (size_t)n);
    double* ps = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0;     /* (dF/dx) lambda, row i */
        double fx = 0.0, fy = 0.0, fz = 0.0;     /* F_i */
        double sx = 0.0, sy = 0.0, sz = 0.0;     /* dF_i / dsigma */
        for (int32_t m = 0; m < nl_count[i]; ++m) {
            const int32_t j = nl[(size_t)i * (size_t)s->nl_cap + (size_t)m];
            double dx, dy, dz;
            sep(s, x, y, z, i, j, &dx, &dy, &dz);
            const double r2 = or_dist2(dx, dy, dz);
            double fr, gr, fs;
            or_pair_deriv(s, r2, &fr, &gr, &fs);
            if (fr == 0.0 && gr == 0.0) continue;
            const double ex = lx[i] - lx[j], ey = ly[i] - ly[j], ez = lz[i] - lz[j];
            const double de = dx * ex + dy * ey + dz * ez;
            ax += fr * ex + gr * de * dx;
            ay += fr * ey + gr * de * dy;
            az += fr * ez + gr * de * dz;
            fx += fr * dx;
            fy += fr * dy;
            fz += fr * dz;
            sx += fs * dx;
            sy += fs * dy;
            sz += fs * dz;
        }
        jx[i] = ax;
        jy[i] = ay;
        jz[i] = az;
        /* F is linear in eps, so dF/deps = F / eps */
        pe[i] = (lx[i] * fx + ly[i] * fy + lz[i] * fz) / s->eps;
        ps[i] = lx[i] * sx + ly[i] * sy + lz[i] * sz;
    }
    *dfde = or_sum(pe, n);
    *dfds = or_sum(ps, n);
    free(pe);
    free(ps);
}

/* ------------------------------------------------------------------ */
/* Soft radial distribution. */

/* Gaussian of standard deviation w, lowered by its value at 3w and cut
 * there, so that the kernel (and every g_b) is continuous in the positions */
static double gauss(double t, double w)
{
    if (fabs(t) >= 3.0 * w) return 0.0;
    return (exp(-0.5 * (t / w) * (t / w)) - exp(-4.5)) / (w * sqrt(2.0 * acos(-1.0)));
}

static double gr_norm(const or_sys* s, const or_gr_spec* g, int32_t b)
{
    const double rho = (double)s->n / (s->L * s->L * s->L);
    const double rb = (b + 0.5) * g->rmax / g->n_bins;
    return (double)s->n * rho * 4.0 * acos(-1.0) * rb * rb;
}

/* pair (i, j) at distance r adds K(r - r_b) to every bin */
static void gr_pair(const or_gr_spec* g, double r, double* acc)
{
    for (int32_t b = 0; b < g->n_bins; ++b) {
        const double rb = (b + 0.5) * g->rmax / g->n_bins;
        acc[b] += gauss(r - rb, g->width);
    }
}

int32_t or_gr(const or_sys* s, const or_gr_spec* g,
              const double* x, const double* y, const double* z,
              const int32_t* nl_count, const int32_t* nl, double* out)
{
    if (g->rmax + 3.0 * g->width > s->r_cut + s->skin) return -1;
    const int32_t B = g->n_bins;
    double* acc = (double*)calloc((size_t)B, sizeof(double));
    for (int32_t i = 0; i < s->n; ++i) {
        for (int32_t m = 0; m < nl_count[i]; ++m) {
            const int32_t j = nl[(size_t)i * (size_t)s->nl_cap + (size_t)m];
            double dx, dy, dz;
            sep(s, x, y, z, i, j, &dx, &dy, &dz);
            gr_pair(g, sqrt(or_dist2(dx, dy, dz)), acc);
        }
    }
    for (int32_t b = 0; b < B; ++b) out[b] = acc[b] / gr_norm(s, g, b);
    free(acc);
    return 0;
}

void or_gr_allpairs(const or_sys* s, const or_gr_spec* g,
                    const double* x, const double* y, const double* z, double* out)
{
    const int32_t B = g->n_bins;
    double* acc = (double*)calloc((size_t)B, sizeof(double));
    for (int32_t i = 0; i < s->n; ++i)
        for (int32_t j = 0; j < s->n; ++j) {
            if (j == i) continue;
            double dx, dy, dz;
            sep(s, x, y, z, i, j, &dx, &dy, &dz);
            gr_pair(g, sqrt(or_dist2(dx, dy, dz)), acc);
        }
    for (int32_t b = 0; b < B; ++b) out[b] = acc[b] / gr_norm(s, g, b);
    free(acc);
}

/* d/dx_i of sum_b wgt_b g_b: the ordered pairs (i, j) and (j, i) both hold
 * r_ij, so each list partner j adds 2 sum_b (wgt_b / norm_b) K'(r - r_b) d / r,
 * with K'(t) = -(t / w^2) exp(-t^2 / 2w^2) / (w sqrt(2 pi)) inside 3w. */
void or_gr_grad(const or_sys* s, const or_gr_spec* g,
                const double* x, const double* y, const double* z,
                const int32_t* nl_count, const int32_t* nl, const double* wgt,
                double* gx, double* gy, double* gz)
{
    const int32_t B = g->n_bins;
    double* wn = (double*)malloc(sizeof(double) * (size_t)(B > 0 ? B : 1));
    for (int32_t b = 0; b < B; ++b) wn[b] = wgt[b] / gr_norm(s, g, b);
    const double w = g->width;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < s->n; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int32_t m = 0; m < nl_count[i]; ++m) {
            const int32_t j = nl[(size_t)i * (size_t)s->nl_cap + (size_t)m];
            double dx, dy, dz;
            sep(s, x, y, z, i, j, &dx, &dy, &dz);
            const double r = sqrt(or_dist2(dx, dy, dz));
            double c = 0.0;
            for (int32_t b = 0; b < B; ++b) {
                const double t = r - (b + 0.5) * g->rmax / B;
                if (fabs(t) < 3.0 * w)
                    c += wn[b] * (-(t / (w * w)) * exp(-0.5 * (t / w) * (t / w)) /
                                  (w * sqrt(2.0 * acos(-1.0))));
            }
            ax += 2.0 * c * dx / r;
            ay += 2.0 * c * dy / r;
            az += 2.0 * c * dz / r;
        }
        gx[i] = ax;
        gy[i] = ay;
        gz[i] = az;
    }
    free(wn);
}

/* ------------------------------------------------------------------ */
/* Trajectories. */

typedef struct {
    int32_t nc;
    int32_t *cell_of, *cell_start, *cell_atoms, *nl_count, *nl;
    double *fx, *fy, *fz, *u_i, *w_i;
} pt_ws;

static int32_t ws_init(const or_sys* s, pt_ws* w)
{
    memset(w, 0, sizeof(*w));
    if (s->n <= 0 || !s->use_nl) return -1;
    w->nc = or_cells_per_side(s->L, s->r_cut + s->skin);
    if (w->nc < 3) return -2;
    const size_t n = (size_t)s->n, ncell = (size_t)w->nc * w->nc * w->nc;
    w->cell_of = (int32_t*)malloc(sizeof(int32_t) * n);
    w->cell_start = (int32_t*)malloc(sizeof(int32_t) * (ncell + 1));
    w->cell_atoms = (int32_t*)malloc(sizeof(int32_t) * n);
    w->nl_count = (int32_t*)malloc(sizeof(int32_t) * n);
    w->nl = (int32_t*)malloc(sizeof(int32_t) * n * (size_t)s->nl_cap);
    w->fx = (double*)malloc(sizeof(double) * n);
    w->fy = (double*)malloc(sizeof(double) * n);
    w->fz = (double*)malloc(sizeof(double) * n);
    w->u_i = (double*)malloc(sizeof(double) * n);
    w->w_i = (double*)malloc(sizeof(double) * n);
    return 0;
}

static void ws_free(pt_ws* w)
{
    free(w->cell_of);
    free(w->cell_start);
    free(w->cell_atoms);
    free(w->nl_count);
    free(w->nl);
    free(w->fx);
    free(w->fy);
    free(w->fz);
    free(w->u_i);
    free(w->w_i);
}

/* cells, list and forces at one point; U and W of the point */
static int32_t at_point(const or_sys* s, pt_ws* w, const double* x, const double* y,
                        const double* z, double* U, double* W)
{
    or_build_cells(s, w->nc, x, y, z, w->cell_of, w->cell_start, w->cell_atoms);
    const int32_t longest = or_build_nl(s, w->nc, x, y, z, w->cell_of, w->cell_start,
                                        w->cell_atoms, w->nl_count, w->nl);
    if (longest > s->nl_cap) return -3;
    or_forces_nl(s, x, y, z, w->nl_count, w->nl, w->fx, w->fy, w->fz, w->u_i, w->w_i, NULL);
    *U = or_sum(w->u_i, s->n);
    *W = or_sum(w->w_i, s->n);
    return 0;
}

/* Forward: positions of every step into traj[(s * 3 + k) * n]. */
static int32_t forward(const or_sys* s, const or_gr_spec* g, int32_t S, pt_ws* w,
                       const double* x0, const double* y0, const double* z0,
                       const double* vx0, const double* vy0, const double* vz0,
                       double* traj, double* ubar)
{
    const size_t n = (size_t)s->n;
    if (g && g->n_bins > 0 && g->rmax + 3.0 * g->width > s->r_cut + s->skin) return -4;
    double* x = traj;
    double* y = traj + n;
    double* z = traj + 2 * n;
    memcpy(x, x0, sizeof(double) * n);
    memcpy(y, y0, sizeof(double) * n);
    memcpy(z, z0, sizeof(double) * n);
    double* vx = (double*)malloc(sizeof(double) * n);
    double* vy = (double*)malloc(sizeof(double) * n);
    double* vz = (double*)malloc(sizeof(double) * n);
    memcpy(vx, vx0, sizeof(double) * n);
    memcpy(vy, vy0, sizeof(double) * n);
    memcpy(vz, vz0, sizeof(double) * n);
    double U, W, usum = 0.0;
    int32_t err = at_point(s, w, x, y, z, &U, &W);
    for (int32_t st = 0; st < S && !err; ++st) {
        double* xn = traj + (size_t)(st + 1) * 3 * n;
        double* yn = xn + n;
        double* zn = yn + n;
        or_kick(s, vx, vy, vz, w->fx, w->fy, w->fz);
        memcpy(xn, traj + (size_t)st * 3 * n, sizeof(double) * 3 * n);
        or_drift(s, xn, yn, zn, vx, vy, vz);
        err = at_point(s, w, xn, yn, zn, &U, &W);
        if (err) break;
        or_kick(s, vx, vy, vz, w->fx, w->fy, w->fz);
        usum += U;
    }
    *ubar = usum / ((double)S * (double)s->n);
    free(vx);
    free(vy);
    free(vz);
    return err;
}

int32_t or_traj_obs(const or_sys* s, const or_gr_spec* g, int32_t S,
                    const double* x0, const double* y0, const double* z0,
                    const double* vx0, const double* vy0, const double* vz0,
                    double* ubar, double* gout)
{
    if (S < 1) return -1;
    pt_ws w;
    int32_t err = ws_init(s, &w);
    if (err) return err;
    const size_t n = (size_t)s->n;
    double* traj = (double*)malloc(sizeof(double) * 3 * n * (size_t)(S + 1));
    err = forward(s, g, S, &w, x0, y0, z0, vx0, vy0, vz0, traj, ubar);
    if (!err && g && g->n_bins > 0) {
        /* the list built at the last step is the list at x_S */
        const double* xs = traj + (size_t)S * 3 * n;
        err = or_gr(s, g, xs, xs + n, xs + 2 * n, w.nl_count, w.nl, gout) ? -4 : 0;
    }
    free(traj);
    ws_free(&w);
    return err;
}

int32_t or_traj_adjoint(const or_sys* s, const or_gr_spec* g, int32_t S,
                        const double* x0, const double* y0, const double* z0,
                        const double* vx0, const double* vy0, const double* vz0,
                        double gU, const double* gG, double* ubar, double* gout,
                        double* gx0, double* gy0, double* gz0,
                        double* gvx0, double* gvy0, double* gvz0, double* gtheta)
{
    if (S < 1) return -1;
    pt_ws w;
    int32_t err = ws_init(s, &w);
    if (err) return err;
    const size_t n = (size_t)s->n;
    const int32_t B = g ? g->n_bins : 0;
    double* traj = (double*)malloc(sizeof(double) * 3 * n * (size_t)(S + 1));
    double* jx = (double*)malloc(sizeof(double) * n);
    double* jy = (double*)malloc(sizeof(double) * n);
    double* jz = (double*)malloc(sizeof(double) * n);
    /* lambda_x = dL/dx (current point), lambda_v = dL/dv (after the kick
       of the current point, before it going backwards) */
    double* lx = gx0;
    double* ly = gy0;
    double* lz = gz0;
    double* mx = gvx0;
    double* my = gvy0;
    double* mz = gvz0;
    double ge = 0.0, gs = 0.0;
    const double c = (0.5 * s->dt) / s->mass;       /* one half kick: v += c f */
    const double lu = gU / ((double)S * (double)s->n); /* dL/dU(x_s), s >= 1 */
    err = forward(s, g, S, &w, x0, y0, z0, vx0, vy0, vz0, traj, ubar);
    if (err) goto done;
    for (size_t i = 0; i < n; ++i) mx[i] = my[i] = mz[i] = 0.0;
    for (int32_t st = S; st >= 0; --st) {
        const double* x = traj + (size_t)st * 3 * n;
        const double* y = x + n;
        const double* z = y + n;
        double U, W;
        err = at_point(s, &w, x, y, z, &U, &W);
        if (err) goto done;
        if (st == S) {
            /* the observables' direct dependence on x_S */
            if (B > 0) {
                if (or_gr(s, g, x, y, z, w.nl_count, w.nl, gout)) {
                    err = -4;
                    goto done;
                }
                or_gr_grad(s, g, x, y, z, w.nl_count, w.nl, gG, lx, ly, lz);
            } else {
                for (size_t i = 0; i < n; ++i) lx[i] = ly[i] = lz[i] = 0.0;
            }
        } else {
            /* the kicks that use F(x_st): the first half kick of step st and
               the second half kick of step st-1 (none before step 0); both
               see the same lambda_v, so they act together */
            const double k = st == 0 ? c : 2.0 * c;
            double de, ds;
            or_hvp(s, x, y, z, w.nl_count, w.nl, mx, my, mz, jx, jy, jz, &de, &ds);
            for (size_t i = 0; i < n; ++i) {
                lx[i] += k * jx[i];
                ly[i] += k * jy[i];
                lz[i] += k * jz[i];
            }
            ge += k * de;
            gs += k * ds;
        }
        if (st >= 1) {
            /* ubar holds U(x_st) / (S N): dU/dx = -F, dU/deps = U / eps and,
               with the cutoff moving with sigma, dU/dsigma = W / sigma */
            for (size_t i = 0; i < n; ++i) {
                lx[i] -= lu * w.fx[i];
                ly[i] -= lu * w.fy[i];
                lz[i] -= lu * w.fz[i];
            }
            ge += lu * U / s->eps;
            gs += lu * W / s->sigma;
            /* the drift of step st-1: x_st = x_{st-1} + dt v */
            for (size_t i = 0; i < n; ++i) {
                mx[i] += s->dt * lx[i];
                my[i] += s->dt * ly[i];
                mz[i] += s->dt * lz[i];
            }
        }
    }
    gtheta[0] = ge;
    gtheta[1] = gs;
done:
    free(traj);
    free(jx);
    free(jy);
    free(jz);
    ws_free(&w);
    return err;
}
