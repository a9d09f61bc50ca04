// md_internal.h -- shared definitions of libmd (not part of the public ABI).
//
// Kernel parameters travel by value as one kernarg block (the paper keeps
// its unvarying pointers and constants in one small structure in constant
// memory, section 2.4 item (2); a kernarg block is the gfx950 equivalent).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/md.h"

namespace md {

constexpr int kWave = 64;
constexpr int kHistCap = 4096;     // history records kept on the device
constexpr int kIntegrateGridMax = 4096;  // largest grid of the grid-stride per-atom kernels
constexpr int kIntegrateGridDefault = 256;
constexpr int kIntThreads = 1024;        // workgroup of the integration and observables
constexpr int kFinishThreads = 256;      // workgroup of the per-system end of a pass
constexpr int kGateGridDefault = 2048;   // per system; a batch divides it among its replicas

// Device-resident control block (first bytes of the workspace).
struct DevState {
    int64_t  step;         // steps completed since bind
    int64_t  n_rebuilds;   // rebuilds triggered by the displacement rule
    int64_t  hist_count;   // records appended to the history
    double   dmax2;        // largest squared displacement at the last drift
    int32_t  rebuild;      // 1: the chain after this drift must rebuild
    uint32_t blocks_done;  // last-workgroup-done counter
    int32_t  flags;        // MD_FLAG_* latched bits
    int32_t  max_occ;      // largest cell occupancy at the last build
    int32_t  max_nl;       // longest list at the last build
    int32_t  pad[3];
    double   obs[8];       // U, K, W, Px, Py, Pz, dmax2, spare (md_reduce)
};

// Everything a kernel needs.
struct KParams {
    // sizes
    int32_t n, npad, nc, ncell, cap, potential, precision, mode, reorder, newton3;
    int32_t pipeline, n_layers;  // MD_PIPE_*; layers per cell of the layer matrix
    // constants (all formed once on the host)
    double L, invL, inv_w, rc2, rl2, sig2, eps2, eps48, half_shift, hdt, dt, disp_thr2, mass;
    double ushift;          // half_shift / eps2: the shift in the units of the u sums
    double ushift2;         // 2 ushift = shift / (2 eps): the constant of the lean sums
    double eps, sigma;
    double inner_lo, inner_hi;  // atoms with every coordinate in [lo, hi] need no minimum image
    // state (caller-owned)
    double *x, *y, *z, *vx, *vy, *vz;
    void *fx, *fy, *fz;
    int32_t* id;
    // workspace arrays
    DevState* dev;
    // a batch replica's entries of the batch's workgroup -> replica table in
    // the grid rules of the rebuild-gated kernels (kGatedRules), whose bit 15
    // the integration finish sets to the rebuild flag; null for a system alone
    uint16_t* gate_tab[3] = {nullptr, nullptr, nullptr};
    int32_t gate_n[3] = {0, 0, 0};
    int32_t rep = 0;  // the replica's index in its batch
    int32_t *cell_count, *cell_start, *cell_of, *slot, *order, *tmp;
    uint64_t* nl64;       // list chunks: 4 x 16-bit entries, chunk c of slot k at c*npad + k
    int32_t* nl_count;
    double *xr, *yr, *zr;
    double *sx, *sy, *sz, *svx, *svy, *svz, *sfx, *sfy, *sfz;  // permutation scratch
    int32_t *sid, *scell;
    int32_t *layers;  // layer matrix [ncell][n_layers] (MD_PIPE_LAYERS)
    int32_t *w32;     // neighbor matrix, 32-bit atom indices [cap][npad] (MD_PIPE_LAYERS)
    void *apart;      // all-pairs per-chunk force partials [ap_split][3][npad] (MD_PIPE_ALLPAIRS)
    double *fpart;    // force-pass partials [nblk_force][2]: U, W
    double *ipart;    // per-atom kernel partials [int_grid][8]
    md_record* hist;
    int32_t nblk_force;     // workgroups of the last-configured force pass
    int32_t block;
    int32_t force_lanes;    // lanes per home atom in the tiled force pass (1, 2, 4, 8)
    int32_t force_block;    // threads per workgroup of the tiled force pass
    int32_t nl_block;       // threads per workgroup of the list build
    int32_t int_grid;       // workgroups of the grid-stride per-atom kernels
    int32_t gate_grid;      // most workgroups of a rebuild-gated per-atom or per-cell kernel
    int32_t nl_method;      // MD_NL_LANES or MD_NL_CELL_WAVES
    // tiling of the neighbor-list mode: blocks of cells, the grid cut into
    // tiles_x x tiles_y x tiles_z near-equal blocks of at most kx_max x ky_max x
    // kz_max cells
    int32_t tiles_x, tiles_y, tiles_z, kx_max, ky_max, kz_max, n_tiles;
    int32_t scap;           // staged atoms a workgroup's LDS holds
    int32_t scap_aux;       // the same with a second 3-vector staged per atom
    int32_t ap_split, ap_chunk;  // all-pairs: partner chunks per home block, atoms per chunk
    // bonded chains (md_set_bonded): chain of id i is i / chain_len
    int32_t bonded_on, chain_len, nblk_bonded, tors_on;
    double fene_k, fene_r02, bend_k, tors_c[4];
    int32_t *slot_of;  // [n] current slot of each permanent id
    double *bpart;     // [nblk_bonded][2] bonded energy and virial partials
};

// Arguments of one reverse-mode point (md_adjoint.hip).  lambda_x is the
// adjoint of the positions, lambda_v that of the velocities; the point reads
// vx/vy/vz (lambda_v of this point) and writes nx/ny/nz (lambda_v after the
// drift of the step before it).
struct AdjArgs {
    double *lx, *ly, *lz;
    const double *vx, *vy, *vz;
    double *nx, *ny, *nz;
    double* theta;         // [2] accumulated dL/deps, dL/dsigma
    double* tpart;         // [workgroups][2] partials of this launch
    const double* gobs;    // dL/d(observables); gobs[0] = dL/dubar
    double coef;           // (dt/2m) times the number of half kicks that use F here
    double loss_scale;     // 1/(S N) when the mean energy depends on this point, else 0
    double drift;          // dt when a drift precedes this point, else 0
    int32_t cap;           // staged atoms with positions and lambda_v
};

// Soft g(r) (md_adjoint.hip): n_bins bins on [0, rmax), Gaussian kernel of
// standard deviation width lowered by its value at 3 widths and cut there.
struct GrArgs {
    unsigned long long* hist;  // [n_bins] fixed-point sums
    double* out;               // [n_bins] g_b
    const double* gobs;        // dL/d(observables); gobs[1 + b] = dL/dg_b (gradient only)
    double* lx;                // gradient output (x); ly, lz follow
    double *ly, *lz;
    int32_t n_bins;
    double rmax, width, scale;  // scale: fixed-point units per unit of kernel value
};

// ---- where a workgroup's parameters come from ----

struct Wg {
    int id, n;  // workgroup index and count within its system's share of the launch
};

// The grid rules of the launches; a batched launch concatenates, per rule,
// the workgroups of every replica.
enum GridKind { G_ATOMS, G_ONE, G_INTEGRATE, G_TILES, G_NL, G_KINDS };
// The grid rules of the rebuild-gated kernels (cell chain, list build).
constexpr GridKind kGatedRules[3] = {G_ATOMS, G_ONE, G_NL};

constexpr int kScanThreads = 1024;  // the one workgroup of the cell-offset scan
constexpr int kCellLanes = 32;      // lanes per atom of the cells-only force pass
constexpr int kScanPer = 4;

__host__ __device__ inline int grid_of(const KParams& p, GridKind k)
{
    auto up = [](int64_t n, int64_t b) { return (int)((n + b - 1) / b); };
    switch (k) {
        case G_ATOMS: {
            const int g = up(p.n, p.block);
            return g < p.gate_grid ? (g > 0 ? g : 1) : p.gate_grid;
        }
        case G_ONE: return 1;
        case G_INTEGRATE: {
            const int g = up(p.n, kIntThreads);
            return g < p.int_grid ? (g > 0 ? g : 1) : p.int_grid;
        }
        case G_TILES:
            return p.mode == MD_NEIGHBOR_LIST ? p.n_tiles : up((int64_t)kCellLanes * p.n, p.block);
        case G_NL:  // the list build: one workgroup per tile
            return p.mode == MD_NEIGHBOR_LIST ? p.n_tiles : 1;
        default: return 1;
    }
}

// A pointer the caller knows to address global memory (so the compiler
// emits global, not flat, accesses through it).  A plain cast to the global
// address space and back is folded away as a no-op pair, losing the fact;
// the empty asm makes the global-space value opaque, so the generic pointer
// is visibly derived from a global one and its accesses are rewritten.  The
// asm operand is a scalar register: q must be the same in every lane of the
// wave (a parameter-block pointer, chosen per workgroup).
template <class T>
__device__ __forceinline__ T* as_global(T* q)
{
    auto g = (__attribute__((address_space(1))) T*)q;
    asm("" : "+s"(g));
    return (T*)g;
}

// A register copy of a parameter block read from device memory, with every
// pointer marked global: stores through those pointers cannot alias the
// copy, so nothing is reloaded inside loops.
__device__ __forceinline__ KParams global_view(const KParams& q)
{
    KParams p = q;
    p.x = as_global(q.x); p.y = as_global(q.y); p.z = as_global(q.z);
    p.vx = as_global(q.vx); p.vy = as_global(q.vy); p.vz = as_global(q.vz);
    p.fx = as_global(q.fx); p.fy = as_global(q.fy); p.fz = as_global(q.fz);
    p.id = as_global(q.id);
    p.dev = as_global(q.dev);
    p.cell_count = as_global(q.cell_count); p.cell_start = as_global(q.cell_start);
    p.cell_of = as_global(q.cell_of); p.slot = as_global(q.slot);
    p.order = as_global(q.order); p.tmp = as_global(q.tmp);
    p.nl64 = as_global(q.nl64); p.nl_count = as_global(q.nl_count);
    p.xr = as_global(q.xr); p.yr = as_global(q.yr); p.zr = as_global(q.zr);
    p.sx = as_global(q.sx); p.sy = as_global(q.sy); p.sz = as_global(q.sz);
    p.svx = as_global(q.svx); p.svy = as_global(q.svy); p.svz = as_global(q.svz);
    p.sfx = as_global(q.sfx); p.sfy = as_global(q.sfy); p.sfz = as_global(q.sfz);
    p.sid = as_global(q.sid); p.scell = as_global(q.scell);
    p.fpart = as_global(q.fpart); p.ipart = as_global(q.ipart);
    p.hist = as_global(q.hist);
    p.layers = as_global(q.layers); p.w32 = as_global(q.w32);
    p.apart = as_global(q.apart);
    p.slot_of = as_global(q.slot_of); p.bpart = as_global(q.bpart);
    return p;
}

// A single system: the parameters are the kernel argument.
struct Single {
    KParams p;
    __device__ __forceinline__ bool fetch(GridKind, Wg& w, KParams& out) const
    {
        w.id = (int)blockIdx.x;
        w.n = (int)gridDim.x;
        out = p;
        return true;
    }
    // fetch for a rebuild-gated kernel: also false when the system does not
    // rebuild this step (and the call does not force it)
    __device__ __forceinline__ bool fetch_gated(GridKind k, int force, Wg& w, KParams& out) const
    {
        fetch(k, w, out);
        return force || p.dev->rebuild;
    }
};

// Independent replicas in one launch.  For grid rule k, replica r owns
// workgroups [first[k][r], first[k][r] + count[k][r]); for the tile rules
// first is rounded up to a multiple of 8 so that the XCD-aware tile order
// (workgroup b runs on XCD b mod 8) holds inside every replica.  rep_of maps
// every workgroup of a
// launch of rule k (from rep_base[k]) to its replica in one load; workgroups
// in the gaps map to the replica before them and return.
constexpr int kGateBit = 1 << 15, kRepMask = kGateBit - 1;  // at most 32768 replicas

struct Batch {
    const KParams* __restrict__ kp;      // [R] per-replica parameters (device)
    const int32_t* __restrict__ first;   // [G_KINDS][R + 1]
    const int32_t* __restrict__ count;   // [G_KINDS][R]
    // workgroup -> replica (bits 0-14), all rules back to back; in the gated
    // rules bit 15 holds the replica's rebuild flag of the current step
    const uint16_t* __restrict__ rep_of;
    int32_t rep_base[G_KINDS];
    int32_t R;
    __device__ __forceinline__ bool fetch(GridKind k, Wg& w, KParams& out) const
    {
        const int blk = (int)blockIdx.x;
        const int r = rep_of[rep_base[(int)k] + blk] & kRepMask;
        return fetch_rep(k, r, w, out);
    }
    // fetch for a rebuild-gated kernel: a workgroup of a replica that does not
    // rebuild this step (unless forced) returns after one load (its table
    // entry) instead of three (its replica, the replica's parameters, the
    // flag they point to)
    __device__ __forceinline__ bool fetch_gated(GridKind k, int force, Wg& w, KParams& out) const
    {
        const int blk = (int)blockIdx.x;
        const int v = rep_of[rep_base[(int)k] + blk];
        if (!force && !(v & kGateBit)) return false;
        return fetch_rep(k, v & kRepMask, w, out);
    }
    __device__ __forceinline__ bool fetch_rep(GridKind k, int r, Wg& w, KParams& out) const
    {
        w.id = (int)blockIdx.x - first[(int)k * (R + 1) + r];
        w.n = count[(int)k * R + r];
        if (w.id >= w.n) return false;
        out = global_view(kp[r]);
        return true;
    }
};

// Uniform launch shape: workgroups per grid rule, block sizes, dynamic LDS.
struct LaunchShape {
    int grid[G_KINDS];
    int block, force_block, force_lanes, nl_block, nl_method, newton3;
    size_t nl_lds, force_lds;
    int precision, reorder, mode;
    // the list build's full kernel: some system has fewer than 5 cells per side
    // (image mode 2) or a list beyond the buffer stores' reach (nl_small)
    int nl_full;
};

// The cell-wave list build stores hits through 32-bit byte offsets, row
// products in 24 bits: 8 n_pad < 2^24 and the whole list (its spare chunk row
// included) below 4 GiB.
__host__ __device__ inline bool nl_small(const KParams& p)
{
    return 8ull * (uint64_t)p.npad < (1ull << 24) &&
           (uint64_t)(p.cap / 4 + 1) * 8ull * (uint64_t)p.npad < (1ull << 32);
}

LaunchShape shape_of(const KParams& p);

// Largest number of force-pass workgroups any tuning can ask for (the
// cells-only pass takes kCellLanes lanes per atom, workgroups of at least 64).
inline int64_t max_force_blocks(int64_t n, int64_t ncell)
{
    const int64_t a = (kCellLanes * n + 63) / 64 + 1;
    return a > ncell + 1 ? a : ncell + 1;
}

// Host-side launchers (one translation unit per stage).
void launch_adj_reimage(const KParams& p, const double* px, const double* py, const double* pz,
                        hipStream_t s);
void launch_adj_point(const KParams& p, const AdjArgs& a, hipStream_t s);
void launch_gr(const KParams& p, const GrArgs& g, hipStream_t s);
void launch_gr_grad(const KParams& p, const GrArgs& g, hipStream_t s);
void launch_traj_ubar(const KParams& p, int32_t n_steps, double* out, hipStream_t s);
void launch_fill(double* a, size_t n, double v, hipStream_t s);
void launch_layer_cells(const KParams& p, int force, hipStream_t s);
void launch_layer_nl(const KParams& p, int force, hipStream_t s);
void launch_layer_forces(const KParams& p, hipStream_t s);
void launch_layer_export(const KParams& p, int32_t* out, hipStream_t s);
void launch_layer_reorder(const KParams& p, hipStream_t s);
void launch_cell_scan(const KParams& p, hipStream_t s);
void launch_sort_small_finish(const KParams& p, int phase, int record_every, hipStream_t s);
int allpairs_home_blocks(int n);
void allpairs_split(int n, int* split, int* chunk);
void launch_allpairs_forces(const KParams& p, hipStream_t s);
void launch_allpairs_fold(const KParams& p, hipStream_t s);
int bonded_blocks(int n);
void launch_bond_map(const KParams& p, int force, hipStream_t s);
void launch_bonded(const KParams& p, hipStream_t s);

void launch_clear(const KParams& p, hipStream_t s);
// launch_cells / launch_neighbors flags: bit 0 forces the build (else it is
// gated by the rebuild flag); kFoldCopy (tiled pipeline with reorder, list
// mode) leaves the cell-sorted data in the scratch arrays, and the list
// build copies each tile's home atoms into the state arrays (saving the
// separate copy-back pass and its launch).
constexpr int kFoldCopy = 2;
// Further launch_cells flags of md_step's cells-only sequence: kFoldBin --
// the integration pass has already binned the atoms (k_bin is left out);
// kSortSmallOk -- a system of at most kSortSmall atoms scans, scatters and
// sorts in one workgroup (k_sort_small).  launch_forces takes kFoldCopy:
// the cells-only force pass then copies each atom back from the scratch
// arrays.
constexpr int kFoldBin = 4;
constexpr int kSortSmallOk = 8;
constexpr int kSortSmall = 16384;
void launch_cells(const KParams& p, int force, hipStream_t s);
void launch_neighbors(const KParams& p, int force, hipStream_t s);
void launch_nl_export(const KParams& p, int32_t* out, hipStream_t s);
void launch_forces(const KParams& p, hipStream_t s, int flags = 0);
// the same over a batch of replicas
void launch_clear(const Batch& b, const LaunchShape& sh, hipStream_t s);
void launch_cells(const Batch& b, const LaunchShape& sh, int force, hipStream_t s);
void launch_neighbors(const Batch& b, const LaunchShape& sh, int force, hipStream_t s);
void launch_forces(const Batch& b, const LaunchShape& sh, hipStream_t s);
void launch_integrate(const Batch& b, const LaunchShape& sh, int phase, int record_every,
                      hipStream_t s);
size_t nl_lds_bytes(const KParams& p);
size_t force_lds_bytes(const KParams& p);
int force_blocks(const KParams& p);  // workgroups of the force pass for the current tuning
// phase 0: kick + drift; 1: kick, record, kick + drift; 2: kick, record
void launch_integrate(const KParams& p, int phase, int record_every, hipStream_t s);
// The two halves of launch_integrate: the per-atom pass, then the per-system
// finish (reductions, step count and record, rebuild decision).
// bin: the pass also bins the atoms (cells-only steps; with phase <= 1 only).
void launch_integrate_pass(const KParams& p, int phase, int record_every, hipStream_t s,
                           bool bin = false);
void launch_integrate_finish(const KParams& p, int phase, int record_every, hipStream_t s);
void launch_observe(const KParams& p, hipStream_t s);

}  // namespace md
