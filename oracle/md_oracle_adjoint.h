/*
 * md_oracle_adjoint.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Reverse-mode (adjoint) reference for trajectories of the MD step in
 * md_oracle.h.  The paper (Rapaport, arXiv:2003.14061) has no gradients;
 * what is differentiated is its method: the pair forces of section 2.3 and
 * the kick-drift-kick leapfrog mentioned in section 4.3.  Plain FP64, one
 * loop per formula, sharing nothing with the GPU library.
 *
 * Readings (none of this is fixed by the paper):
 *   - parameters theta = (eps, sigma); the cutoff moves with sigma
 *     (r_cut / sigma fixed), so the energy shift u_LJ(r_cut) does not depend
 *     on sigma.  Pairs crossing the cutoff contribute nothing (the pathwise
 *     derivative of a truncated potential).
 *   - observables of a trajectory x_0 .. x_S (S kick-drift-kick steps):
 *       ubar  = (1/S) sum_{s=1..S} U(x_s) / N
 *       g_b   = soft radial distribution at x_S:
 *               g_b = sum_i sum_{j != i} K(r_ij - r_b) / (N rho 4 pi r_b^2)
 *               r_b = (b + 1/2) rmax / B, K(t) a unit-area Gaussian of
 *               standard deviation w = `width` minus its value at 3w, zero
 *               beyond 3w (continuous, so the loss is continuous too).
 *     A loss L(ubar, g) enters only through its gradient (gU = dL/dubar,
 *     gG[b] = dL/dg_b).
 *
 * Arrays are structure-of-arrays in atom-id order, owned by the caller.
 */
#ifndef MD_ORACLE_ADJOINT_H
#define MD_ORACLE_ADJOINT_H

#include <stdint.h>

#include "md_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_bins;  /* B (0: no g(r) observable) */
    double  rmax;    /* bins cover [0, rmax) */
    double  width;   /* Gaussian standard deviation */
} or_gr_spec;

/* Pair derivatives at squared separation r2 (zero at r2 >= r_cut^2):
 *   fr = -u'(r) / r               force on i is fr * d, d = x_i - x_j
 *   gr = (1/r) d fr / dr          so dF_i/dx_i (one pair) = fr I + gr d d^T
 *   fs = d fr / d sigma           at fixed r                                  */
void or_pair_deriv(const or_sys* s, double r2, double* fr, double* gr, double* fs);

/* Jacobian of the forces applied to lambda over the list:
 *   j_i = sum_k (dF_i/dx_k) lambda_k
 *       = sum_{j in NL(i), r < r_cut} fr (lambda_i - lambda_j)
 *                                   + gr (d . (lambda_i - lambda_j)) d
 * and the parameter contractions
 *   dfde = sum_i lambda_i . dF_i/deps,  dfds = sum_i lambda_i . dF_i/dsigma. */
void or_hvp(const or_sys* s, const double* x, const double* y, const double* z,
            const int32_t* nl_count, const int32_t* nl,
            const double* lx, const double* ly, const double* lz,
            double* jx, double* jy, double* jz, double* dfde, double* dfds);

/* Soft g(r) over the list pairs (needs rmax + 3 width <= r_cut + skin);
 * returns 0, or -1 when the list radius is too short. */
int32_t or_gr(const or_sys* s, const or_gr_spec* g,
              const double* x, const double* y, const double* z,
              const int32_t* nl_count, const int32_t* nl, double* out);

/* The same sum over every pair of atoms (minimum image), no list. */
void or_gr_allpairs(const or_sys* s, const or_gr_spec* g,
                    const double* x, const double* y, const double* z, double* out);

/* Gradient with respect to every position of sum_b wgt_b g_b. */
void or_gr_grad(const or_sys* s, const or_gr_spec* g,
                const double* x, const double* y, const double* z,
                const int32_t* nl_count, const int32_t* nl, const double* wgt,
                double* gx, double* gy, double* gz);

/* Observables of the S-step trajectory from (x0, v0): ubar and g (length
 * n_bins, may be NULL when n_bins is 0).  The list is rebuilt at every step.
 * Returns 0, or a negative value on error (-1 arguments, -2 box too small,
 * -3 list overflow, -4 list radius too short for the g(r) range). */
int32_t or_traj_obs(const or_sys* s, const or_gr_spec* g, int32_t S,
                    const double* x0, const double* y0, const double* z0,
                    const double* vx0, const double* vy0, const double* vz0,
                    double* ubar, double* gout);

/* Reverse mode over the stored trajectory: given gU = dL/dubar and gG[b] =
 * dL/dg_b, the gradients of L with respect to x_0, v_0 and (eps, sigma)
 * (gtheta[0], gtheta[1]).  Also returns the observables.  Same errors as
 * or_traj_obs. */
int32_t or_traj_adjoint(const or_sys* s, const or_gr_spec* g, int32_t S,
                        const double* x0, const double* y0, const double* z0,
                        const double* vx0, const double* vy0, const double* vz0,
                        double gU, const double* gG, double* ubar, double* gout,
                        double* gx0, double* gy0, double* gz0,
                        double* gvx0, double* gvy0, double* gvz0, double* gtheta);

#ifdef __cplusplus
}
#endif
#endif
