/*
 * md_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference for the short-range molecular dynamics
 * step of Rapaport, "GPU molecular dynamics: Algorithms and performance"
 * (arXiv:2003.14061).  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library and includes nothing from it.
 *
 * What it computes (section 2.3 of the paper):
 *   N1      cell of every atom from its position
 *   N2-N4   cell occupancy; here as cell_start / cell_atoms, atoms of a cell
 *           in ascending id (the paper leaves the in-cell order open)
 *   N5      neighbor list: for each atom, every other atom of the 27
 *           surrounding cells closer than r_cut + skin
 *   F1      per-atom force and energy over the list, full list, no
 *           Newton's-third-law sharing
 *   F2      total energy, kinetic energy, virial and momentum, summed
 *           serially in id order
 * and the symplectic leapfrog integrator mentioned in section 4.3, taken as
 * kick-drift-kick, with the list refreshed "at intervals of several time
 * steps" (section 2.3), here when the largest displacement since the last
 * build exceeds half the skin.
 *
 * Arrays are structure-of-arrays in atom-id order; every array is owned by
 * the caller.  Nothing here allocates memory that outlives a call.
 */
#ifndef MD_ORACLE_H
#define MD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_LJ_SHIFTED = 0, OR_LJ_TRUNC = 1 };

typedef struct {
    int32_t n;          /* number of atoms */
    int32_t potential;  /* OR_LJ_SHIFTED or OR_LJ_TRUNC */
    double  L;          /* edge of the periodic cube; positions in [0, L) */
    double  eps, sigma, mass;
    double  r_cut;      /* interaction cutoff, absolute length */
    double  skin;       /* neighbor shell thickness (the paper's delta) */
    double  dt;         /* time step */
    int32_t use_nl;     /* 1: neighbor list from cells of width >= r_cut+skin;
                           0: forces straight from cells of width >= r_cut */
    int32_t nl_cap;     /* entries reserved per atom in the oracle's list */
} or_sys;

typedef struct {
    double  U;          /* potential energy */
    double  K;          /* kinetic energy */
    double  W;          /* pair virial, sum over pairs i<j of r_ij . F_ij */
    double  P[3];       /* total momentum */
    double  dmax2;      /* largest squared displacement since the last
                           build, taken before the rebuild decision */
    int32_t rebuilt;    /* 1 if cells (and list) were rebuilt this step */
    int32_t max_nl;     /* longest list after this step's build (0 if none) */
} or_obs;

/* ---- potential (the paper defers the form to its references; the reading
 *      used is Lennard-Jones, cut at r_cut, optionally energy-shifted) ---- */
double or_pair(const or_sys* s, double r2, double* fr);
double or_shift(const or_sys* s);

/* ---- periodic box ---- */
double or_wrap(double x, double L);
double or_minimg(double d, double L, double invL);
double or_dist2(double dx, double dy, double dz);

/* ---- N1-N4: cells ---- */
int32_t or_cells_per_side(double L, double r_cell);
void or_build_cells(const or_sys* s, int32_t nc,
                    const double* x, const double* y, const double* z,
                    int32_t* cell_of, int32_t* cell_start, int32_t* cell_atoms);

/* ---- N5: neighbor list; nl is [n][nl_cap] row-major.  Returns the
 *      longest list; a value above nl_cap means entries were dropped. ---- */
int32_t or_build_nl(const or_sys* s, int32_t nc,
                    const double* x, const double* y, const double* z,
                    const int32_t* cell_of, const int32_t* cell_start,
                    const int32_t* cell_atoms,
                    int32_t* nl_count, int32_t* nl);

/* The half list (for Newton's-third-law force passes): the entries of the
 * full list whose partner comes later in the cell order (cell index, then
 * permanent id), same order and layout as or_build_nl. */
int32_t or_build_nl_half(const or_sys* s, int32_t nc,
                         const double* x, const double* y, const double* z,
                         const int32_t* cell_of, const int32_t* cell_start,
                         const int32_t* cell_atoms,
                         int32_t* nl_count, int32_t* nl);

/* ---- F1: forces.  u_i gets half of each pair energy, w_i half of each
 *      pair virial, s_i the sum over pairs of or_pair_scale (the scale of
 *      the rounding error of the force sum, used for tolerances).  Any of
 *      u_i, w_i, s_i may be NULL. ---- */
double or_pair_scale(const or_sys* s, double r2);
void or_forces_nl(const or_sys* s,
                  const double* x, const double* y, const double* z,
                  const int32_t* nl_count, const int32_t* nl,
                  double* fx, double* fy, double* fz,
                  double* u_i, double* w_i, double* s_i);
/* Forces from a half list: each pair adds F_ij to i and -F_ij to j (and
 * half its energy, virial and scale to each); serial, in list order. */
void or_forces_half(const or_sys* s,
                    const double* x, const double* y, const double* z,
                    const int32_t* nl_count, const int32_t* nl,
                    double* fx, double* fy, double* fz,
                    double* u_i, double* w_i, double* s_i);
void or_forces_cells(const or_sys* s, int32_t nc,
                     const double* x, const double* y, const double* z,
                     const int32_t* cell_of, const int32_t* cell_start,
                     const int32_t* cell_atoms,
                     double* fx, double* fy, double* fz,
                     double* u_i, double* w_i, double* s_i);
void or_forces_allpairs(const or_sys* s,
                        const double* x, const double* y, const double* z,
                        double* fx, double* fy, double* fz,
                        double* u_i, double* w_i, double* s_i);
/* brute force over all atoms for the k atoms listed in idx (outputs length k) */
void or_forces_sample(const or_sys* s,
                      const double* x, const double* y, const double* z,
                      const int32_t* idx, int32_t k,
                      double* fx, double* fy, double* fz,
                      double* u_i, double* w_i, double* s_i);

/* ---- F2: reductions, serial in id order ---- */
double or_sum(const double* a, int32_t n);
double or_kinetic(const or_sys* s, const double* vx, const double* vy, const double* vz);
void   or_momentum(const or_sys* s, const double* vx, const double* vy, const double* vz,
                   double* p3);
double or_max_disp2(const or_sys* s,
                    const double* x, const double* y, const double* z,
                    const double* xr, const double* yr, const double* zr);

/* ---- leapfrog pieces ---- */
void or_kick(const or_sys* s, double* vx, double* vy, double* vz,
             const double* fx, const double* fy, const double* fz);
void or_drift(const or_sys* s, double* x, double* y, double* z,
              const double* vx, const double* vy, const double* vz);

/* ---- a whole run: n_steps of kick-drift-[rebuild]-force-kick.  On entry
 *      x,v hold the state; f is ignored and recomputed.  obs receives one
 *      record per step (may be NULL).  Returns the number of rebuilds, or a
 *      negative value on error (-1 bad arguments, -2 box too small for 3
 *      cells per side, -3 list overflow). ---- */
int32_t or_run(const or_sys* s, int32_t n_steps,
               double* x, double* y, double* z,
               double* vx, double* vy, double* vz,
               double* fx, double* fy, double* fz,
               or_obs* obs);

/* Extra forces added after every pair-force evaluation of a run: the hook
 * adds to the forces and to the per-atom energy and virial (id order) and
 * returns 0, or a negative code that ends the run with that code. */
typedef int32_t (*or_force_hook)(const void* ctx, const or_sys* s,
                                 const double* x, const double* y, const double* z,
                                 double* fx, double* fy, double* fz,
                                 double* u_i, double* w_i);

/* or_run with a force hook (hook NULL: exactly or_run). */
int32_t or_run_hooked(const or_sys* s, or_force_hook hook, const void* hook_ctx,
                      int32_t n_steps,
                      double* x, double* y, double* z,
                      double* vx, double* vy, double* vz,
                      double* fx, double* fy, double* fz,
                      or_obs* obs);

/* number of OpenMP threads the per-atom loops use (1 without OpenMP) */
int32_t or_threads(void);

#ifdef __cplusplus
}
#endif
#endif
