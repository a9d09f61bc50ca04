/*
 * md.h -- C ABI of libmd, a short-range molecular dynamics engine for AMD
 * MI355X (gfx950), after Rapaport, "GPU molecular dynamics: Algorithms and
 * performance", arXiv:2003.14061.
 *
 * The calls follow the paper's statement of the problem (section 2.3): atoms
 * are assigned to cells (steps N1-N4), a neighbor list is built from the 27
 * surrounding cells (N5), forces are accumulated per atom over the list
 * without Newton's-third-law sharing (F1), and energies are reduced (F2); the
 * list is refreshed only every several steps.  Integration is the symplectic
 * leapfrog (section 4.3) in kick-drift-kick form.
 *
 * Memory.  The caller owns every byte of device memory: the per-atom state
 * arrays and one workspace block whose size md_workspace_bytes() reports.
 * The library never allocates or frees device memory.  All per-atom arrays
 * are structure-of-arrays (one array per component), length n_atoms, stored
 * in the library's current storage order; id[k] is the permanent id of the
 * atom held in slot k (section 4.1, factor (1)).  With reorder enabled the
 * slots are permuted into cell order at every rebuild.
 *
 * Streams.  Every call except md_init, md_workspace_bytes, md_layout,
 * md_geometry, md_reduce, md_history and md_destroy only enqueues work on
 * the stream given to md_bind and returns at once.  md_reduce and md_history
 * synchronize that stream.  A context is not thread-safe; distinct contexts
 * on distinct streams are independent.
 *
 * Errors.  Calls return md_status.  Argument errors are detected on the host
 * before anything is enqueued.  Conditions found on the device (list
 * overflow, non-finite force) are latched in a device flag word and reported
 * by the next md_reduce; they stay latched until md_bind is called again.
 * No C++ exception crosses this interface.
 */
#ifndef MD_H
#define MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct md_ctx md_ctx;

typedef enum {
    MD_OK = 0,
    MD_ERR_ARG = -1,            /* invalid argument or parameter */
    MD_ERR_BOX_TOO_SMALL = -2,  /* fewer than 3 cells per side */
    MD_ERR_NL_OVERFLOW = -3,    /* an atom had more list entries than nl_capacity */
    MD_ERR_NONFINITE = -4,      /* a force or energy was not finite */
    MD_ERR_HIP = -5,            /* a HIP runtime call failed */
    MD_ERR_NOT_BOUND = -6,      /* md_bind has not been called */
    MD_ERR_STATE = -7,          /* call out of order (e.g. step before forces) */
    MD_ERR_LAYER_OVERFLOW = -8, /* a cell held more atoms than the layer matrix has layers
                                   (MD_PIPE_LAYERS) */
    MD_ERR_BOND_BROKEN = -9,    /* a bonded pair reached the FENE limit R0 (md_set_bonded) */
    MD_ERR_TOPOLOGY = -10,      /* the permanent ids are not a permutation of 0 .. N-1, so
                                   the chains of md_set_bonded are undefined */
    MD_ERR_WORKSPACE_TOO_LARGE = -11 /* md_bind_static: the context needs more workspace than
                                        MD_STATIC_WORKSPACE_BYTES */
} md_status;

/* Size of the library's own device workspace array used by md_bind_static
 * (one per GPU, held until the process ends). */
#define MD_STATIC_WORKSPACE_BYTES (64u << 20)

enum { MD_LJ_SHIFTED = 0, MD_LJ_TRUNC = 1 };      /* potential */
enum { MD_FP64 = 0, MD_FP32_MIXED = 1 };          /* precision */
enum { MD_CELLS_ONLY = 0, MD_NEIGHBOR_LIST = 1 }; /* mode */
enum { MD_PIPE_TILED = 0, MD_PIPE_LAYERS = 1, MD_PIPE_ALLPAIRS = 2 }; /* pipeline */
enum { MD_NL_AUTO = 0, MD_NL_LANES = 1, MD_NL_CELL_WAVES = 2 }; /* md_tuning.nl_method */

/* Device flag bits (md_observables.flags). */
enum { MD_FLAG_NL_OVERFLOW = 1, MD_FLAG_NONFINITE = 2, MD_FLAG_LAYER_OVERFLOW = 4,
       MD_FLAG_BOND_BROKEN = 8, MD_FLAG_TOPOLOGY = 16 };

/* System and method parameters, copied by md_init.  Lengths in the units of
 * sigma's length, energies in eps's units. */
typedef struct {
    int32_t n_atoms;     /* N >= 1 */
    int32_t potential;   /* MD_LJ_SHIFTED: 12-6 potential cut at r_cut and shifted to
                            vanish there (soft spheres: r_cut = 2^(1/6) sigma);
                            MD_LJ_TRUNC: cut, not shifted (forces identical) */
    double  L;           /* edge of the periodic cube; positions must lie in [0, L) */
    double  eps, sigma, mass;
    double  r_cut;       /* cutoff, absolute */
    double  skin;        /* neighbor shell thickness (the paper's delta); list radius
                            r_cut + skin; the list is rebuilt when some atom has moved
                            more than skin/2 since the last build */
    double  dt;          /* time step */
    int32_t precision;   /* MD_FP64, or MD_FP32_MIXED: pair forces formed and summed in
                            FP32 from FP64 separations, cutoff test in FP64; positions,
                            velocities, integration and energy sums stay FP64 */
    int32_t mode;        /* MD_NEIGHBOR_LIST (cells of width >= r_cut+skin, list) or
                            MD_CELLS_ONLY (cells of width >= r_cut, rebuilt every step,
                            forces straight from the 27 cells) */
    int32_t newton3;     /* 0: full list, no atomics (the paper's choice, section 2.3);
                            1: half list, the partner's force added with atomics */
    int32_t nl_capacity; /* list entries reserved per atom; 0 picks a bound from the
                            density */
    int32_t reorder;     /* 1: permute the atom slots into cell order at every rebuild
                            (section 4.1, factor (1)); 0: never permute.  MD_PIPE_LAYERS:
                            k > 0 permutes them into the layer matrix's cell order every
                            k-th step of md_step, counted from md_bind (section 2.4 item
                            (4); the paper's runs use k = 100, section 3), then rebuilds
                            both matrices; md_step launches directly then (no graph) */
    int32_t block;       /* threads per workgroup for per-atom kernels, a multiple of 64
                            in [64, 1024]; 0 = 256 */
    int32_t pipeline;    /* MD_PIPE_TILED (default): LDS-staged tiles, 16-bit list entries;
                            MD_PIPE_LAYERS: the paper's own steps as it lays them out
                            (section 2.3), one thread per atom throughout: an atomic layer
                            index per atom (N2), the dense cell-by-layer matrix (N3-N4),
                            the neighbor matrix W of 32-bit atom indices read in rows
                            (N5) and the force pass gathering partners from memory (F1);
                            within a cell the atoms follow the order of the atomics, so
                            the list order is not reproducible, its content is.
                            Requires MD_NEIGHBOR_LIST, newton3 = 0, reorder = 0; not in
                            batches or trajectory mode.
                            MD_PIPE_ALLPAIRS: the all-pairs force evaluation the paper
                            compares against (section 4.2, alternative (2)): every atom
                            against every other under the minimum image, partner
                            positions staged through LDS in tiles, no cells and no list;
                            md_build_cells only folds the positions into [0, L) and the
                            drift of md_step keeps them there.  Work grows as N^2.
                            Requires MD_CELLS_ONLY (whose box rule, L >= 3 r_cut, makes
                            the minimum image unique) and reorder = 0; not in batches or
                            trajectory mode */
} md_params;

/* Device buffers supplied by the caller (all device pointers). */
typedef struct {
    double*  x;  double* y;  double* z;    /* positions, in [0, L) */
    double*  vx; double* vy; double* vz;   /* velocities */
    void*    fx; void*   fy; void*   fz;   /* forces: double (MD_FP64) or float (MD_FP32_MIXED) */
    int32_t* id;                           /* permanent atom ids */
    void*    workspace;                    /* md_workspace_bytes() bytes, 256-byte aligned */
} md_buffers;

/* Derived geometry (host side, filled by md_geometry). */
typedef struct {
    int32_t nc;          /* cells per side */
    int32_t n_cells;     /* nc^3 */
    int32_t nl_capacity; /* list rows */
    int32_t n_pad;       /* row pitch of the list, n rounded up to 64 */
    double  cell_width;  /* L / nc */
    int32_t n_layers;    /* layers per cell of the layer matrix (MD_PIPE_LAYERS; else 0) */
    int32_t pad;
} md_grid;

/* Results of md_reduce.  Energies are totals over the system. */
typedef struct {
    double  U;           /* potential energy */
    double  K;           /* kinetic energy, (m/2) sum v^2 */
    double  W;           /* pair virial, sum over pairs i<j of r_ij . F_ij */
    double  P[3];        /* total momentum */
    double  T;           /* 2K / (3(N-1)) */
    double  pressure;    /* (2K + W) / (3 L^3) */
    double  dmax;        /* largest displacement since the last list build, as of the
                            last drift */
    int64_t step;        /* steps completed since md_bind */
    int64_t n_rebuilds;  /* list (or cell) rebuilds triggered by md_step */
    int32_t max_occupancy; /* largest cell occupancy at the last cell build */
    int32_t max_nl;        /* longest list at the last list build */
    int32_t flags;         /* latched MD_FLAG_* bits */
    int32_t pad;
} md_observables;

/* One record of the step history (md_history). */
typedef struct {
    int64_t step;
    double  U, K, W, P[3], dmax;
    int32_t rebuilt;     /* 1 if this step rebuilt the cells/list */
    int32_t pad;
} md_record;

/* Array identifiers for md_layout (each lives inside the workspace). */
enum {
    MD_ARR_CELL_OF = 0,    /* int32[n]     cell of the atom in slot k (N1); the three cell
                              arrays do not exist under MD_PIPE_ALLPAIRS (MD_ERR_ARG) */
    MD_ARR_CELL_START = 1, /* int32[nc^3+1] first entry of each cell in CELL_ATOMS (N2-N4) */
    MD_ARR_CELL_ATOMS = 2, /* int32[n]     slots grouped by cell, ascending id in a cell */
    MD_ARR_NL = 3,         /* uint16[cap][n_pad] in 4-entry chunks: the m-th neighbor of slot k
                              is 16-bit word m%4 of 8-byte chunk (m/4)*n_pad + k; the word holds
                              the neighbor's index among its tile's staged atoms (13 bits) and
                              its periodic wrap bits (3 bits); md_export_neighbors decodes it.
                              MD_PIPE_LAYERS: int32[cap][n_pad], entry m*n_pad + k the m-th
                              neighbor of atom k */
    MD_ARR_NL_COUNT = 4,   /* int32[n]     list length per slot */
    MD_ARR_XREF = 5,       /* double[3][n] positions at the last list build */
    MD_ARR_LAYERS = 6,     /* int32[nc^3][n_layers] layer matrix: the atom in each layer of
                              each cell (MD_PIPE_LAYERS only) */
    MD_ARR_LAYER_COUNT = 7,/* int32[nc^3] atoms per cell, i.e. layers in use (MD_PIPE_LAYERS) */
    MD_ARR_COUNT_ = 8
};

/* md_init: validate parameters, derive the cell grid and list capacity.
 * No device work.  *out receives a new context on MD_OK.  Returns
 * MD_ERR_ARG for bad values, MD_ERR_BOX_TOO_SMALL when floor(L / cell
 * width) < 3. */
md_status md_init(const md_params* params, md_ctx** out);

/* Bonded chains (section 4.3, item (2): polymers as atoms linked by elastic
 * bonds, with a bond-angle and an optional dihedral interaction, on top of
 * the pair forces between all atoms).  The paper gives no functional forms;
 * these are used:
 *   bond      FENE  U = -(fene_k fene_r0^2 / 2) ln(1 - r^2 / fene_r0^2)
 *   angle     U = bend_k (1 - cos theta), theta the angle between the bond
 *             vectors b1 = r_j - r_i and b2 = r_k - r_j of consecutive bonds
 *             (zero for a straight chain)
 *   dihedral  U = sum_{m=0..3} tors_c[m] cos^m phi over three consecutive
 *             bonds, cos phi = n1.n2 / (|n1||n2|), n1 = b1 x b2, n2 = b2 x b3
 *             (phi = 0 cis, pi trans)
 * Chains are linear: the atoms with permanent ids c*M .. c*M + M - 1 form
 * chain c in that order (M = chain_length).  Bond vectors take the minimum
 * image.  A term whose coefficient is zero is skipped. */
typedef struct {
    int32_t chain_length;  /* M >= 2; n_atoms must be a multiple of M */
    int32_t pad;
    double  fene_k;        /* >= 0 */
    double  fene_r0;       /* > 0; a bond reaching it latches MD_FLAG_BOND_BROKEN */
    double  bend_k;
    double  tors_c[4];
} md_bonded;

/* md_set_bonded: add the bonded forces of `b` to every force evaluation
 * (md_forces, md_step), their energy to U and the bonds' virial to W.  NULL
 * removes them.  Call before md_bind (the workspace grows by an id-to-slot
 * map and the bonded partials: query md_workspace_bytes afterwards);
 * MD_ERR_STATE once bound, MD_ERR_ARG for bad values.  Each atom's thread
 * evaluates the bonded terms it takes part in (no atomics).  Not available in
 * batches or trajectory mode.  The permanent ids must be a permutation of
 * 0 .. N-1, else md_reduce reports MD_ERR_TOPOLOGY. */
md_status md_set_bonded(md_ctx* ctx, const md_bonded* b);

/* Bytes of workspace the context needs (0 for a NULL context). */
size_t md_workspace_bytes(const md_ctx* ctx);

/* Geometry derived by md_init. */
md_status md_geometry(const md_ctx* ctx, md_grid* out);

/* Byte offset and element count of a workspace array (MD_ARR_*). */
md_status md_layout(const md_ctx* ctx, int32_t which, size_t* offset, size_t* count);

/* md_bind: borrow the caller's buffers and stream (a hipStream_t; NULL means
 * the null stream).  Clears the device counters and flags (enqueued).  The
 * buffers must stay valid until the context is destroyed or bound again. */
md_status md_bind(md_ctx* ctx, const md_buffers* bufs, void* hip_stream);

/* md_bind_static: md_bind for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The caller still passes the state arrays; bufs->workspace must
 * be NULL.  The workspace is taken from a static device array of
 * MD_STATIC_WORKSPACE_BYTES (64 MiB; about 130 000 atoms of the dense LJ
 * state, 250 000 of soft spheres) that the library holds on each GPU until
 * the process ends; its used part is cleared on the stream (a fill kernel),
 * then the device counters, as md_bind does.  Returns
 * MD_ERR_WORKSPACE_TOO_LARGE, enqueuing nothing, when md_workspace_bytes(ctx)
 * exceeds the array.  Neither this call nor any later call on the context
 * allocates device memory (md_set_timing's events aside).  Every context
 * bound this way on one GPU shares that GPU's array, which keeps the last
 * call's contents: binding another context there overwrites the earlier
 * one's cells, list and counters (rebind it before using it again), and
 * calls of two such contexts that overlap in time race.  md_layout offsets
 * are relative to the array, which the caller cannot address. */
md_status md_bind_static(md_ctx* ctx, const md_buffers* bufs, void* hip_stream);

/* md_build_cells (N1-N4, and the reorder): assign every atom to its cell,
 * group the slots by cell with ascending id inside a cell, and, with reorder
 * on, permute positions, velocities, forces and ids into that order.
 * MD_PIPE_ALLPAIRS: fold the positions into [0, L) only.  Enqueued. */
md_status md_build_cells(md_ctx* ctx);

/* md_build_neighbors (N5): for every atom, the other atoms of the 27
 * surrounding cells (visited with dz, dy, dx each -1, 0, +1, dz slowest;
 * inside a cell in ascending id) whose minimum-image separation is below
 * r_cut + skin, squared separation formed as dx*dx + dy*dy + dz*dz with two
 * fused multiply-adds.  Records the positions as the displacement
 * reference.  Requires md_build_cells.  MD_NEIGHBOR_LIST mode only.
 * Enqueued; overflow is latched. */
md_status md_build_neighbors(md_ctx* ctx);

/* md_export_neighbors: decode the list into global slots, dst[m * n_pad +
 * k] = slot of the m-th neighbor of slot k for m < count, -1 for the
 * remaining rows; dst is a device buffer of nl_capacity * n_pad int32
 * owned by the caller.  Requires md_build_neighbors.  Enqueued. */
md_status md_export_neighbors(md_ctx* ctx, int32_t* dst);

/* md_forces (F1): per-atom force over the list (or the 27 cells in
 * MD_CELLS_ONLY mode, or every other atom under MD_PIPE_ALLPAIRS), pairs
 * closer than r_cut, plus per-workgroup partial sums of the potential energy
 * and the virial.  Requires the cells (and list).  Enqueued. */
md_status md_forces(md_ctx* ctx);

/* md_step: n_steps leapfrog steps, kick-drift-kick: v += dt/(2m) f; x += dt v;
 * rebuild cells (and list) when needed; forces; v += dt/(2m) f.  Positions
 * are folded into [0, L) at every cell build and may lie outside the box by
 * less than skin/2 in between (the list's periodic wrap bits stay valid);
 * separations always use the minimum image.  Requires md_forces to have
 * run on the current state.
 * When record_every > 0, every step whose index is a multiple of
 * record_every is appended to the history (capacity 4096 records, oldest
 * overwritten).  Enqueued. */
md_status md_step(md_ctx* ctx, int32_t n_steps, int32_t record_every);

/* md_set_graph: with enable != 0 md_step replays runs of 32 steps from a HIP
 * graph captured at its first use (recaptured after md_bind, md_set_tuning or
 * a different record_every); the first step of a call and the remainder are
 * launched directly.  A call of 10 to 32 steps replays one graph of all its
 * steps but the first (recaptured when that length changes), and calls of up
 * to 9 steps launch directly.  The default is off: direct launches measured
 * 9-20% faster per step on MI355X for 4000 to 131 072 atoms, so the graph is
 * for callers that want the steps as a graph.  When the bound stream is the
 * null stream the graph runs on a stream of the context's own, ordered after
 * the bound stream's earlier work and before its later work by events.
 * enable = 0 launches every kernel directly.  Results are identical either
 * way; md_set_timing also selects the direct launches. */
md_status md_set_graph(md_ctx* ctx, int32_t enable);

/* md_reduce (F2): finish the reductions on the device (kinetic energy,
 * momentum, the potential energy and virial of the last force pass) and
 * copy them to *out.  Synchronizes the stream.  Returns the latched device
 * condition, if any, as its status (MD_ERR_NL_OVERFLOW, MD_ERR_NONFINITE). */
md_status md_reduce(md_ctx* ctx, md_observables* out);

/* md_history: copy up to max_records history records, oldest first, to the
 * host array out; *n_out receives the count.  Synchronizes the stream. */
md_status md_history(md_ctx* ctx, md_record* out, int32_t max_records, int32_t* n_out);

/* Launch shape of the hot kernels.  Every setting gives results within the
 * parity tolerances; the force pass's summation order depends on
 * force_lanes, so bitwise reproducibility holds for a fixed tuning. */
typedef struct {
    int32_t force_lanes;    /* lanes sharing one atom's list in the force pass: 1, 2, 4, 8
                               (2 after md_init) */
    int32_t force_block;    /* threads per workgroup of the force pass: 64..1024, multiple of 64
                               (512 after md_init) */
    int32_t nl_block;       /* threads per workgroup of the list build: 64..1024, multiple of 64;
                               0 = automatic (a lane per home atom of a mean tile, or a wave
                               per home cell of the widest tile, at most 16 waves) */
    int32_t tile_cells;     /* neighbor-list mode: cells per tile (a block of cells) along x;
                               0 = automatic: the block with the fewest staged cells per home
                               cell whose staged atoms fit three force workgroups per CU and
                               whose home atoms fill at most three force passes */
    int32_t stage_cap;      /* atoms a workgroup stages in LDS (0 = 1.15x the mean need plus
                               64); tiles that hold more read positions from global memory
                               instead */
    int32_t integrate_grid; /* 1024-thread workgroups of the per-atom kernels (integration,
                               observables): 1..4096; 0 = 256 */
    int32_t nl_method;      /* list build: MD_NL_LANES (one lane per home atom, for sparse
                               cells), MD_NL_CELL_WAVES (one wave per home cell, for dense
                               ones) or MD_NL_AUTO (lanes below 8 atoms per cell); the list
                               is the same either way.  md_get_tuning reports the method
                               in use */
    int32_t tile_y;         /* cells per tile along y (0 = automatic, as tile_cells) */
    int32_t tile_z;         /* cells per tile along z (0 = automatic, as tile_cells) */
} md_tuning;

/* md_set_tuning: change the launch shape (host only; takes effect at the
 * next launch).  The forces must be recomputed (md_forces) before md_step,
 * and a change of the tile size also needs md_build_neighbors, since list
 * entries index the tile's staged atoms.  md_get_tuning: the current shape
 * (tile_cells, tile_y, tile_z as resolved: the largest block in use). */
md_status md_set_tuning(md_ctx* ctx, const md_tuning* tuning);
md_status md_get_tuning(const md_ctx* ctx, md_tuning* tuning);

/* md_autotune: the autotuner of md_batch_autotune for one system (tiled
 * pipeline, neighbor-list mode): each candidate builds the cells once, then
 * `reps` lists and force passes on the current state are timed; the cost is
 * the mean force pass plus a tenth of the mean list build.  Leaves the
 * cheapest shape set, with cells, list and forces rebuilt for it (md_step
 * may follow).  ms_out[n], *best and cache_path (keyed by the system, the
 * candidate list and the device) as for md_batch_autotune.  Synchronizes the
 * stream. */
md_status md_autotune(md_ctx* ctx, const md_tuning* candidates, int32_t n, int32_t reps,
                      const char* cache_path, double* ms_out, int32_t* best);

/* md_set_timing: when enable != 0, bracket every force-pass launch with HIP
 * events on the bound stream; md_get_timing returns the summed elapsed time
 * (ms) and the number of timed launches since timing was enabled, and
 * synchronizes the stream.  While timing is on, md_step also brackets every
 * other part of each step and launches each kernel directly;
 * md_get_timing_parts returns, per part (MD_PART_*, the rows of the paper's
 * breakdown of a step's time, section 3.2 Table 2), the summed time (ms)
 * in ms[MD_PART_COUNT] and the number of timed launch groups in
 * launches[MD_PART_COUNT].  The energy and virial are summed inside the
 * force pass and the kinetic sums inside the integration pass; MD_PART_ENERGY
 * is the per-system pass that completes these reductions (with the step
 * record and the rebuild decision).  MD_PART_CELLS is the cell build (the
 * counting sort with its reorder, or the layer matrix), MD_PART_NEIGHBORS
 * the list or neighbor-matrix build, MD_PART_REORDER the layer pipeline's
 * periodic reorder.  The rebuild-gated parts are timed on every step, idle
 * or not.  Synchronizes the stream. */
enum { MD_PART_NEIGHBORS = 0, MD_PART_FORCES = 1, MD_PART_INTEGRATE = 2, MD_PART_ENERGY = 3,
       MD_PART_CELLS = 4, MD_PART_REORDER = 5, MD_PART_COUNT = 6 };
md_status md_set_timing(md_ctx* ctx, int32_t enable);
md_status md_get_timing(md_ctx* ctx, double* total_ms, int64_t* launches);
md_status md_get_timing_parts(md_ctx* ctx, double* ms, int64_t* launches);

/* ---- Reverse mode: gradients of trajectory observables ----
 *
 * Not part of the paper, which has no gradients: the derivative of its
 * method (pair forces F1 over the neighbor list, section 2.3, inside the
 * kick-drift-kick leapfrog of section 4.3) with respect to the initial
 * positions and velocities and the potential parameters (eps, sigma).  The
 * cutoff is taken to move with sigma (r_cut / sigma fixed); pairs crossing
 * the cutoff contribute nothing (the pathwise derivative).
 *
 * Observables of an S-step trajectory x_0 .. x_S, as a device array obs of
 * 1 + n_bins doubles:
 *   obs[0]     = (1/S) sum_{s=1..S} U(x_s) / N
 *   obs[1 + b] = g_b(x_S) = sum_i sum_{j != i} K(r_ij - r_b) / (N rho 4 pi r_b^2),
 *                r_b = (b + 1/2) gr_rmax / n_bins, K a unit-area Gaussian of
 *                standard deviation gr_width, lowered by its value at 3
 *                widths and zero beyond (continuous in the positions).
 * The pairs of g come from the neighbor list, so gr_rmax + 3 gr_width must
 * not exceed r_cut + skin.
 *
 * Checkpointing: md_traj_forward keeps (x, v) every checkpoint_every steps
 * and at the end; md_traj_backward recomputes each segment forward from its
 * checkpoint, keeping its positions, then walks it backwards.  Both need a
 * neighbor-list context with reorder = 0 (gradients then come out in the
 * bound storage order, which never changes), bound buffers, and a
 * caller-owned device block of md_traj_workspace_bytes() bytes (256-byte
 * aligned) that md_traj_backward reads as md_traj_forward left it.  n_steps
 * may not exceed 4096 (the history the mean energy is read from). */
typedef struct {
    int32_t n_steps;           /* S >= 1 */
    int32_t checkpoint_every;  /* >= 1 */
    int32_t n_bins;            /* 0..1024 (0: obs holds the mean energy only) */
    int32_t pad;
    double  gr_rmax;           /* > 0 when n_bins > 0 */
    double  gr_width;          /* > 0 when n_bins > 0 */
} md_traj_params;

/* Bytes of the trajectory workspace; 0 on invalid arguments. */
size_t md_traj_workspace_bytes(const md_ctx* ctx, const md_traj_params* tp);

/* Run n_steps leapfrog steps from the bound state (computing the forces
 * first if needed), keeping the checkpoints in traj_ws and writing the
 * observables to obs (device, 1 + n_bins doubles).  Leaves the state at step
 * n_steps.  Enqueued. */
md_status md_traj_forward(md_ctx* ctx, const md_traj_params* tp, void* traj_ws, double* obs);

/* Given grad_obs = dL/dobs (device, 1 + n_bins doubles), write dL/dx_0 and
 * dL/dv_0 (device, 3 * n_atoms doubles each: all x, then all y, then all z)
 * and dL/d(eps, sigma) (device, 2 doubles).  Uses the checkpoints of the
 * last md_traj_forward on traj_ws; restores the state at step n_steps before
 * returning (the step counter also counts the recomputed steps).  Enqueued. */
md_status md_traj_backward(md_ctx* ctx, const md_traj_params* tp, void* traj_ws,
                           const double* grad_obs, double* grad_x0, double* grad_v0,
                           double* grad_theta);

void md_destroy(md_ctx* ctx);

/* ---- Batched replicas ----
 *
 * Many independent systems advanced together: section 4.3 runs a set of
 * mutually invisible realizations in one program so that systems too small
 * for the GPU still fill it (the single-system kernels are those of section
 * 2.3).  Every kernel of a step is one launch over all
 * replicas: each workgroup finds its replica in a table and works on that
 * replica's data, so replicas of very different sizes share the machine
 * without one launch per replica.  md_batch_run captures a whole run in one
 * HIP graph and launches it once (the graph is kept and relaunched while the
 * step count, record interval and tuning stay the same).
 *
 * Every replica is an ordinary context (md_init parameters; its results are
 * read with md_reduce, md_history and md_layout on md_batch_replica()), owned
 * by the batch: do not md_destroy it or md_bind it yourself.  All replicas
 * must share precision, mode, reorder and block; the launch shape (md_tuning)
 * applies to all of them, with tile_cells = 0 resolved per replica from its
 * density. */
typedef struct md_batch md_batch;

/* Validates params[0 .. n_replicas-1] (each as md_init would) and plans the
 * shared workspace; 1 <= n_replicas <= 32768.  MD_ERR_ARG if the replicas
 * disagree on precision, mode, reorder or block. */
md_status md_batch_init(const md_params* params, int32_t n_replicas, md_batch** out);

/* Bytes of the one workspace block of the whole batch (256-byte aligned). */
size_t md_batch_workspace_bytes(const md_batch* b);

/* The context of replica r (owned by the batch). */
md_status md_batch_replica(md_batch* b, int32_t r, md_ctx** ctx);

/* buffers[r]: the state arrays of replica r (its workspace field is
 * ignored); workspace: md_batch_workspace_bytes() bytes, 256-byte aligned.
 * The stream must be a created stream (not the legacy null stream), since
 * md_batch_run captures graphs on it.  Clears every replica's device state;
 * copies the launch tables to the device (synchronously). */
md_status md_batch_bind(md_batch* b, const md_buffers* buffers, void* workspace, void* stream);

/* Cells, lists and forces of every replica from scratch.  Enqueued. */
md_status md_batch_prepare(md_batch* b);

/* The force pass (F1, section 2.3) of every replica, one launch, on the
 * current lists.  Enqueued. */
md_status md_batch_forces(md_batch* b);

/* md_layout of replica r, with the offset counted from the start of the
 * batch workspace. */
md_status md_batch_layout(const md_batch* b, int32_t r, int32_t which, size_t* offset,
                          size_t* count);

/* n_steps leapfrog steps of every replica (as md_step).  use_graph != 0:
 * the run is captured once into a HIP graph and launched as one graph
 * (relaunched on later calls with the same n_steps and record_every);
 * 0: the kernels are launched one by one.  Needs md_batch_prepare after
 * binding or retuning.  Enqueued. */
md_status md_batch_run(md_batch* b, int32_t n_steps, int32_t record_every, int32_t use_graph);

/* Launch shape of every replica (see md_tuning); lists and forces must be
 * rebuilt afterwards (md_batch_prepare). */
md_status md_batch_set_tuning(md_batch* b, const md_tuning* tuning);
md_status md_batch_get_tuning(const md_batch* b, md_tuning* tuning);

/* Autotuner (the best workgroup size depends on the GPU and the model,
 * section 4.1 factor (2)): for each of the n candidate shapes, rebuild the replicas'
 * cells and lists with it and time `reps` list builds and force passes (HIP
 * events on the bound stream); the cost of a candidate is the mean force
 * pass plus a tenth of the mean list build (a rebuild every ~10 steps).
 * Writes the costs (ms) to ms_out[n] and the index of the cheapest to *best,
 * and leaves the batch set to it and prepared.  Synchronizes the stream.
 * Positions are only folded into the box and, with reorder, permuted.
 * cache_path (NULL: none) names a JSON file of earlier results, keyed by
 * the replicas' sizes and geometry, the candidate list and the device: on a
 * hit the cached shape is applied without timing (ms_out all -1, *best its
 * index among the candidates); otherwise the winner is added to the file. */
md_status md_batch_autotune(md_batch* b, const md_tuning* candidates, int32_t n, int32_t reps,
                            const char* cache_path, double* ms_out, int32_t* best);

void md_batch_destroy(md_batch* b);

/* Static string for a status code. */
const char* md_status_str(int32_t status);

#ifdef __cplusplus
}
#endif
#endif
