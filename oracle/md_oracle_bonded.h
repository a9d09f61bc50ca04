/*
 * md_oracle_bonded.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Bonded forces of linear polymer chains, the extension the paper outlines
 * among its further MD studies (section 4.3, item (2)): atoms linked by
 * elastic bonds, a bond-angle interaction between adjacent bonds, and an
 * optional dihedral (twist) interaction over three consecutive bonds, on top
 * of the non-bonded pair forces between all atoms.  The paper gives no
 * functional forms; the readings used here are
 *
 *   bond      FENE  U = -(k R0^2 / 2) ln(1 - r^2 / R0^2),  r < R0
 *   angle     U = k_b (1 - cos theta),  theta the angle between consecutive
 *             bond vectors b1 = r_j - r_i, b2 = r_k - r_j (0 for a straight
 *             chain)
 *   dihedral  U = sum_{m=0..3} c_m cos^m phi, cos phi = n1.n2 / (|n1||n2|),
 *             n1 = b1 x b2, n2 = b2 x b3 (phi = 0 cis, pi trans)
 *
 * Chains: atom ids c*M .. c*M + M - 1 form chain c in that order (M >= 2,
 * N a multiple of M).  Bond vectors take the minimum image, so chains may
 * cross the periodic boundary.  Each term is evaluated once and its forces
 * applied to all its atoms; its energy and virial are booked to its first
 * atom.  The virial of a term that depends only on bond vectors is
 * -sum_b b . dU/db: zero for the angle and dihedral terms (they depend on
 * directions only), -k r^2 / (1 - r^2/R0^2) for a bond.
 *
 * Plain FP64, one loop per formula, sharing nothing with the GPU library.
 * Arrays are structure-of-arrays in atom-id order, owned by the caller.
 */
#ifndef MD_ORACLE_BONDED_H
#define MD_ORACLE_BONDED_H

#include <stdint.h>

#include "md_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t chain_length; /* M >= 2 */
    int32_t pad;
    double  fene_k;       /* k > 0 (0: no bond force) */
    double  fene_r0;      /* R0 > 0 */
    double  bend_k;       /* k_b (0: no angle term) */
    double  tors_c[4];    /* c_0 .. c_3 (all 0: no dihedral term) */
} or_bonded;

/* Adds the bonded forces to fx, fy, fz and the bonded energy, virial and
 * rounding-error scale (sum over terms of the magnitudes of the parts of
 * each atom's force) to u_i, w_i, s_i (any of the three may be NULL).
 * Returns 0, or -1 if a bond reached R0 (no force is then defined). */
int32_t or_forces_bonded(const or_sys* s, const or_bonded* b,
                         const double* x, const double* y, const double* z,
                         double* fx, double* fy, double* fz,
                         double* u_i, double* w_i, double* s_i);

/* Total bonded energy (for finite-difference checks); NaN if a bond
 * reached R0. */
double or_energy_bonded(const or_sys* s, const or_bonded* b,
                        const double* x, const double* y, const double* z);

/* or_run with the bonded forces added to the pair forces at every force
 * evaluation (b may be NULL: then exactly or_run). */
int32_t or_run_bonded(const or_sys* s, const or_bonded* b, int32_t n_steps,
                      double* x, double* y, double* z,
                      double* vx, double* vy, double* vz,
                      double* fx, double* fy, double* fz,
                      or_obs* obs);

#ifdef __cplusplus
}
#endif

#endif
