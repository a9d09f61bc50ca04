/*
 * md_oracle_bonded.c -- TEST INFRASTRUCTURE ONLY.  Bonded chain forces
 * (section 4.3, item (2)); the readings are stated in md_oracle_bonded.h.
 * Every term is evaluated once, in chain order, and its forces are applied
 * to all of its atoms.
 */
#include "md_oracle_bonded.h"

#include <math.h>
#include <stddef.h>

typedef struct {
    double x, y, z;
} v3;

static v3 vsub(v3 a, v3 b) { return (v3){a.x - b.x, a.y - b.y, a.z - b.z}; }
static v3 vscale(v3 a, double k) { return (v3){k * a.x, k * a.y, k * a.z}; }
static double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static double vnorm(v3 a) { return sqrt(vdot(a, a)); }
static v3 vcross(v3 a, v3 b)
{
    return (v3){a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

/* Bond vector from atom i to atom j under the minimum image. */
static v3 bond(const or_sys* s, const double* x, const double* y, const double* z,
               int32_t i, int32_t j)
{
    double L = s->L, invL = 1.0 / s->L;
    return (v3){or_minimg(x[j] - x[i], L, invL), or_minimg(y[j] - y[i], L, invL),
                or_minimg(z[j] - z[i], L, invL)};
}

typedef struct {
    double *fx, *fy, *fz, *u, *w, *sm;
} sink;

static void push(const sink* o, int32_t i, v3 f, double scale)
{
    o->fx[i] += f.x;
    o->fy[i] += f.y;
    o->fz[i] += f.z;
    if (o->sm) o->sm[i] += scale;
}

static int valid(const or_sys* s, const or_bonded* b)
{
    return b && b->chain_length >= 2 && s->n % b->chain_length == 0 && b->fene_r0 > 0.0;
}

/* FENE bond i -> j with d = r_j - r_i: energy, and the force on i (the force
 * on j is its negative).  Returns -1 when |d| >= R0. */
static int fene(const or_bonded* b, v3 d, double* U, double* W, v3* f_i)
{
    double r2 = vdot(d, d), R2 = b->fene_r0 * b->fene_r0;
    if (!(r2 < R2)) return -1;
    double q = 1.0 - r2 / R2;
    *U = -0.5 * b->fene_k * R2 * log(q);
    /* dU/dr = k r / q, pulling i toward j */
    double g = b->fene_k / q;
    *f_i = vscale(d, g);
    *W = -g * r2; /* (r_i - r_j) . F_i */
    return 0;
}

/* cos of the angle between b1 and b2, and its gradients with respect to
 * both vectors. */
static double cos_and_grad(v3 b1, v3 b2, v3* g1, v3* g2)
{
    double n1 = vnorm(b1), n2 = vnorm(b2);
    double c = vdot(b1, b2) / (n1 * n2);
    *g1 = vsub(vscale(b2, 1.0 / (n1 * n2)), vscale(b1, c / (n1 * n1)));
    *g2 = vsub(vscale(b1, 1.0 / (n1 * n2)), vscale(b2, c / (n2 * n2)));
    return c;
}

static double tors_energy(const or_bonded* b, double c)
{
    return b->tors_c[0] + c * (b->tors_c[1] + c * (b->tors_c[2] + c * b->tors_c[3]));
}

static double tors_slope(const or_bonded* b, double c)
{
    return b->tors_c[1] + c * (2.0 * b->tors_c[2] + c * 3.0 * b->tors_c[3]);
}

static int has_tors(const or_bonded* b)
{
    return b->tors_c[0] != 0.0 || b->tors_c[1] != 0.0 || b->tors_c[2] != 0.0 ||
           b->tors_c[3] != 0.0;
}

/* One pass over all terms.  With o == NULL only the energy is summed. */
static int32_t terms(const or_sys* s, const or_bonded* b,
                     const double* x, const double* y, const double* z,
                     const sink* o, double* U_total)
{
    int32_t M = b->chain_length;
    double Ut = 0.0;
    for (int32_t c0 = 0; c0 < s->n; c0 += M) {
        /* bonds */
        if (b->fene_k != 0.0) {
            for (int32_t p = 0; p + 1 < M; ++p) {
                int32_t i = c0 + p, j = i + 1;
                double U, W;
                v3 f;
                if (fene(b, bond(s, x, y, z, i, j), &U, &W, &f)) return -1;
                Ut += U;
                if (o) {
                    double m = vnorm(f);
                    push(o, i, f, m);
                    push(o, j, vscale(f, -1.0), m);
                    if (o->u) o->u[i] += U;
                    if (o->w) o->w[i] += W;
                }
            }
        }
        /* angles i, j, k: U = k_b (1 - cos theta), F = k_b grad cos theta */
        if (b->bend_k != 0.0) {
            for (int32_t p = 0; p + 2 < M; ++p) {
                int32_t i = c0 + p, j = i + 1, k = i + 2;
                v3 g1, g2;
                double c = cos_and_grad(bond(s, x, y, z, i, j), bond(s, x, y, z, j, k), &g1, &g2);
                double kb = b->bend_k;
                Ut += kb * (1.0 - c);
                if (o) {
                    double m1 = kb * vnorm(g1), m2 = kb * vnorm(g2);
                    push(o, i, vscale(g1, -kb), m1);
                    push(o, j, vscale(vsub(g1, g2), kb), m1 + m2);
                    push(o, k, vscale(g2, kb), m2);
                    if (o->u) o->u[i] += kb * (1.0 - c);
                }
            }
        }
        /* dihedrals i, j, k, l over bonds b1, b2, b3 */
        if (has_tors(b)) {
            for (int32_t p = 0; p + 3 < M; ++p) {
                int32_t i = c0 + p, j = i + 1, k = i + 2, l = i + 3;
                v3 b1 = bond(s, x, y, z, i, j), b2 = bond(s, x, y, z, j, k);
                v3 b3 = bond(s, x, y, z, k, l);
                v3 A = vcross(b1, b2), B = vcross(b2, b3), gA, gB;
                double c = cos_and_grad(A, B, &gA, &gB);
                Ut += tors_energy(b, c);
                if (o) {
                    /* dc/db through A = b1 x b2 and B = b2 x b3 */
                    v3 d1 = vcross(b2, gA);
                    v3 d2a = vcross(gA, b1), d2b = vcross(b3, gB);
                    v3 d2 = (v3){d2a.x + d2b.x, d2a.y + d2b.y, d2a.z + d2b.z};
                    v3 d3 = vcross(gB, b2);
                    double e = tors_slope(b, c), ae = fabs(e);
                    double m1 = ae * vnorm(d1), m2 = ae * vnorm(d2), m3 = ae * vnorm(d3);
                    /* F_a = -dU/dc * dc/dr_a; b1 = r_j - r_i, b2 = r_k - r_j, b3 = r_l - r_k */
                    push(o, i, vscale(d1, e), m1);
                    push(o, j, vscale(vsub(d1, d2), -e), m1 + m2);
                    push(o, k, vscale(vsub(d2, d3), -e), m2 + m3);
                    push(o, l, vscale(d3, -e), m3);
                    if (o->u) o->u[i] += tors_energy(b, c);
                }
            }
        }
    }
    if (U_total) *U_total = Ut;
    return 0;
}

int32_t or_forces_bonded(const or_sys* s, const or_bonded* b,
                         const double* x, const double* y, const double* z,
                         double* fx, double* fy, double* fz,
                         double* u_i, double* w_i, double* s_i)
{
    if (!valid(s, b)) return -1;
    sink o = {fx, fy, fz, u_i, w_i, s_i};
    return terms(s, b, x, y, z, &o, NULL);
}

double or_energy_bonded(const or_sys* s, const or_bonded* b,
                        const double* x, const double* y, const double* z)
{
    double U = 0.0;
    if (!valid(s, b) || terms(s, b, x, y, z, NULL, &U)) return NAN;
    return U;
}

static int32_t bonded_hook(const void* ctx, const or_sys* s,
                           const double* x, const double* y, const double* z,
                           double* fx, double* fy, double* fz,
                           double* u_i, double* w_i)
{
    return or_forces_bonded(s, (const or_bonded*)ctx, x, y, z, fx, fy, fz, u_i, w_i, NULL)
               ? -4
               : 0;
}

int32_t or_run_bonded(const or_sys* s, const or_bonded* b, int32_t n_steps,
                      double* x, double* y, double* z,
                      double* vx, double* vy, double* vz,
                      double* fx, double* fy, double* fz,
                      or_obs* obs)
{
    if (b && !valid(s, b)) return -1;
    return or_run_hooked(s, b ? bonded_hook : NULL, b, n_steps, x, y, z, vx, vy, vz,
                         fx, fy, fz, obs);
}
