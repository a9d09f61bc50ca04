// md_forces.hip -- step F1 of section 2.3 (and the per-workgroup part of F2).
//
// Neighbor-list mode: one workgroup per tile (md_tiles.h).  After the
// tile's cell tables are known, one round of loads brings the tile's 27-cell
// neighborhoods into LDS; `lanes` lanes per home atom then walk the atom's
// list straight from the neighbor matrix (lane s takes chunks s, s+lanes,
// ...; a chunk is 4 entries, and each lane loads its next chunk before it
// works on the current one), gather the partners from LDS and accumulate the
// force on the home atom alone.  Every pair is met twice,
// once from each side, so no atomics are needed (the paper's choice).
// Pairs at r^2 >= r_cut^2 are skipped.  Separations take the minimum image
// from the wrap bits carried by each entry (section 4.1, factor (4)); tiles
// with no periodic wrap skip even that.
//
// With a half list (Newton's third law, the optional atomic variant the
// paper sets aside in section 2.3) every pair is met once, from the atom
// earlier in cell order; the partner's reaction force is added with LDS
// atomics into a per-staged-atom accumulator beside the staged positions,
// the home atom's own total goes there too, and at the end of the tile every
// accumulator that was touched is added into the force arrays with global
// atomics (which were cleared before the pass).  Tiles whose atoms do not
// fit in LDS add straight into the force arrays.  The order of the atomic
// adds is not fixed, so the forces are reproducible to rounding only.
//
// Cells-only mode: one lane per atom walks the 27 surrounding cells.
//
// Precision: FP64 forms everything in double.  FP32-mixed forms the pair
// separation and the cutoff test in double, then the pair force, energy and
// virial and the per-atom sums in float.
//
// The energy and virial are reduced per workgroup (wave64 shuffles, then
// LDS) and written as partials for the reduction kernels.
#include "md_pair.h"
#include "md_tiles.h"

namespace md {

// Pair operation of the force pass: the pair force, energy and virial of
// partners inside the cutoff.
template <typename Acc>
struct ForceOp {
    const KParams& p;
    Acc& a;
    __device__ __forceinline__ void operator()(double dx, double dy, double dz, double r2, int,
                                               int)
    {
        if (r2 < p.rc2) pair_acc(p, dx, dy, dz, r2, a);
    }
};

// Pair operation of the third-law pass: as ForceOp, and the reaction
// -F into the partner's LDS accumulator (staged index e), or straight into
// the force arrays at slot j when the tile is not staged.
template <typename F, typename Acc>
struct HalfOp {
    const KParams& p;
    Acc& a;
    MD_LDS F* r;  // [cap][3] reaction accumulators
    __device__ __forceinline__ void operator()(double dx, double dy, double dz, double r2, int e,
                                               int j)
    {
        if (r2 >= p.rc2) return;
        F g[3];
        pair_acc(p, dx, dy, dz, r2, a, g);
        if (j < 0) {
            lds_add(r + 3 * e, -g[0]);
            lds_add(r + 3 * e + 1, -g[1]);
            lds_add(r + 3 * e + 2, -g[2]);
        } else {
            global_add(static_cast<F*>(p.fx) + j, -g[0]);
            global_add(static_cast<F*>(p.fy) + j, -g[1]);
            global_add(static_cast<F*>(p.fz) + j, -g[2]);
        }
    }
};

template <typename F, typename Acc, int LANES, class B>
__global__ void k_forces_half(B b)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_TILES, wg, p)) return;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ double red[(1024 / kWave) * 2];
    const Tile g = tile_of(p, xcd_tile(wg.id, wg.n));
    Stage s = stage_layout(p, smem, p.scap_aux, true);
    stage_tables(p, g, s);
    const int nh = home_count(s);
    const int mode = staged_image_mode(p, s, tile_interior(p, g));
    stage_positions_imaged(p, s);
    // the accumulators, in the aux region (F-typed, interleaved)
    MD_LDS F* r = reinterpret_cast<MD_LDS F*>(s.a3);
    if (s.fits) {
        for (int k = threadIdx.x; k < 3 * s.total; k += blockDim.x) r[k] = F(0);
    }
    __syncthreads();
    const int per_pass = blockDim.x / LANES;
    const int sub = threadIdx.x % LANES;
    double e[2] = {0.0, 0.0};
    for (int hb = 0; hb < nh; hb += per_pass) {
        const int h = hb + threadIdx.x / LANES;
        Acc a;
        int slot_i = 0, eh = 0;
        if (h < nh) {
            int pos;
            home_atom(s, h, eh, pos);
            slot_i = atom_at(p, pos);
            double xi, yi, zi;
            home_position(p, s, eh, slot_i, xi, yi, zi);
            HalfOp<F, Acc> op{p, a, r};
            walk_home<LANES>(p, s, mode, slot_i, sub, p.nl_count[slot_i], xi, yi, zi, op);
        }
        if (LANES > 1) {
            a.fx = lane_group_sum<LANES>(a.fx);
            a.fy = lane_group_sum<LANES>(a.fy);
            a.fz = lane_group_sum<LANES>(a.fz);
            a.u = lane_group_sum<LANES>(a.u);
            a.w = lane_group_sum<LANES>(a.w);
        }
        if (h < nh && sub == 0) {
            if (s.fits) {
                lds_add(r + 3 * eh, a.fx);
                lds_add(r + 3 * eh + 1, a.fy);
                lds_add(r + 3 * eh + 2, a.fz);
            } else {
                global_add(static_cast<F*>(p.fx) + slot_i, a.fx);
                global_add(static_cast<F*>(p.fy) + slot_i, a.fy);
                global_add(static_cast<F*>(p.fz) + slot_i, a.fz);
            }
            // each pair once: its whole energy 4 eps (sr12 - sr6) - shift, and virial
            const double ui = 2.0 * p.eps2 * (double)a.u;
            e[0] += ui;
            e[1] += (double)a.w;
            if (!isfinite(ui + (double)a.fx + (double)a.fy + (double)a.fz))
                atomicOr(&p.dev->flags, (int)MD_FLAG_NONFINITE);
        }
    }
    __syncthreads();
    if (s.fits) {
        // flush every touched accumulator (home atoms always; partners in
        // the cells behind the home row in cell order never)
        for (int k = threadIdx.x; k < s.total; k += blockDim.x) {
            const F ax = r[3 * k], ay = r[3 * k + 1], az = r[3 * k + 2];
            if (ax != F(0) || ay != F(0) || az != F(0)) {
                const int j = staged_slot(p, s, k);
                global_add(static_cast<F*>(p.fx) + j, ax);
                global_add(static_cast<F*>(p.fy) + j, ay);
                global_add(static_cast<F*>(p.fz) + j, az);
            }
        }
    }
    block_sum<2>(e, red);
    if (threadIdx.x == 0) {
        p.fpart[2 * wg.id] = e[0];
        p.fpart[2 * wg.id + 1] = e[1];
    }
}

// Clears the force arrays before a third-law pass.
template <typename F, class B>
__global__ void k_zero_forces(B b)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_ATOMS, wg, p)) return;
    for (int i = wg.id * blockDim.x + threadIdx.x; i < p.n; i += wg.n * blockDim.x) {
        static_cast<F*>(p.fx)[i] = F(0);
        static_cast<F*>(p.fy)[i] = F(0);
        static_cast<F*>(p.fz)[i] = F(0);
    }
}

// Six waves per SIMD (at most 80 VGPRs): three workgroups of the default
// shape fit a CU by LDS, and the compiler's own allocation otherwise crosses
// the five-wave line.
template <typename F, typename Acc, int LANES, class B>
__global__ __attribute__((amdgpu_waves_per_eu(6))) void k_forces_tiles(B b)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_TILES, wg, p)) return;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ double red[(1024 / kWave) * 2];
    const Tile g = tile_of(p, xcd_tile(wg.id, wg.n));
    Stage s = stage_layout(p, smem);
    stage_tables(p, g, s);
    const int nh = home_count(s);
    const int mode = staged_image_mode(p, s, tile_interior(p, g));
    stage_positions_imaged(p, s);
    __syncthreads();
    const int per_pass = blockDim.x / LANES;
    const int sub = threadIdx.x % LANES;
    double e[2] = {0.0, 0.0};
    for (int hb = 0; hb < nh; hb += per_pass) {
        const int h = hb + threadIdx.x / LANES;
        LeanOf<F> a;
        int slot_i = 0;
        if (h < nh) {
            int eh, pos;
            home_atom(s, h, eh, pos);
            slot_i = atom_at(p, pos);
            double xi, yi, zi;
            home_position(p, s, eh, slot_i, xi, yi, zi);
            ForceOp<LeanOf<F>> op{p, a};
            // the lane's list-row offset is formed here for each pass: hoisted out
            // of the pass loop it is a 64-bit value live across the whole kernel
            // (the empty asm hides that sub is the same in every pass)
            int sub_p = sub;
            asm volatile("" : "+v"(sub_p));
            walk_home<LANES>(p, s, mode, slot_i, sub_p, p.nl_count[slot_i], xi, yi, zi, op);
        }
        if (LANES > 1) {
            a.fx = lane_group_sum<LANES>(a.fx);
            a.fy = lane_group_sum<LANES>(a.fy);
            a.fz = lane_group_sum<LANES>(a.fz);
            a.q = lane_group_sum<LANES>(a.q);
            a.s6 = lane_group_sum<LANES>(a.s6);
        }
        if (h < nh && sub == 0) {
            F fx, fy, fz;
            double ui, wi;
            lean_finish(p, a, fx, fy, fz, ui, wi);
            static_cast<F*>(p.fx)[slot_i] = fx;
            static_cast<F*>(p.fy)[slot_i] = fy;
            static_cast<F*>(p.fz)[slot_i] = fz;
            e[0] += ui;
            e[1] += wi;
            if (!isfinite(ui + (double)fx + (double)fy + (double)fz))
                atomicOr(&p.dev->flags, (int)MD_FLAG_NONFINITE);
        }
    }
    block_sum<2>(e, red);
    if (threadIdx.x == 0) {
        p.fpart[2 * wg.id] = e[0];
        p.fpart[2 * wg.id + 1] = e[1];
    }
}

// ---- cells-only mode ----
//
// kCellLanes lanes per atom: lane c < 27 walks neighbor cell c of the atom's
// 27 (dz, dy, dx each -1, 0, +1, dz slowest) straight from the cell arrays,
// with the full minimum image; the lanes' sums are then added across the
// group.  At about one atom per cell a lane has one or two partners, so the
// pass is as deep as a few dependent loads rather than the 27 cells in turn.

template <typename Acc>
__device__ __forceinline__ void walk_cell(const KParams& p, int i, double xi, double yi,
                                          double zi, int c2, Acc& a)
{
    const int k1 = p.cell_start[c2 + 1];
    for (int k = p.cell_start[c2]; k < k1; ++k) {
        const int j = atom_at(p, k);
        if (j == i) continue;
        const double dx = minimg(xi - p.x[j], p.L, p.invL);
        const double dy = minimg(yi - p.y[j], p.L, p.invL);
        const double dz = minimg(zi - p.z[j], p.L, p.invL);
        const double r2 = dist2(dx, dy, dz);
        if (r2 < p.rc2) pair_acc(p, dx, dy, dz, r2, a);
    }
}

// kCopy (md_step with reorder): the cell build left the sorted data in the
// scratch arrays; the pass reads them there and each atom's lane 0 copies its
// atom into the state arrays, forces written straight into the state.
template <typename F, typename Acc, class B, bool kCopy>
__global__ void k_forces_cells(B b)
{
    Wg wg;
    KParams pw;
    if (!b.fetch(G_TILES, wg, pw)) return;
    const KParams p = kCopy ? scratch_view(pw) : pw;
    F* const fout[3] = {static_cast<F*>(pw.fx), static_cast<F*>(pw.fy),
                        static_cast<F*>(pw.fz)};
    __shared__ double red[(1024 / kWave) * 2];
    const int64_t t = (int64_t)xcd_tile(wg.id, wg.n) * blockDim.x + threadIdx.x;
    const int i = (int)(t / kCellLanes), sub = (int)(t % kCellLanes);
    LeanOf<F> a;
    if (i < p.n && sub < 27) {
        const int c = p.cell_of[i], nc = p.nc;
        const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
        const int dz = sub / 9 - 1, dy = (sub / 3) % 3 - 1, dx = sub % 3 - 1;
        const int c2 = (wrap_cell(cz + dz, nc) * nc + wrap_cell(cy + dy, nc)) * nc +
                       wrap_cell(cx + dx, nc);
        walk_cell(p, i, p.x[i], p.y[i], p.z[i], c2, a);
    }
    a.fx = lane_group_sum<kCellLanes>(a.fx);
    a.fy = lane_group_sum<kCellLanes>(a.fy);
    a.fz = lane_group_sum<kCellLanes>(a.fz);
    a.q = lane_group_sum<kCellLanes>(a.q);
    a.s6 = lane_group_sum<kCellLanes>(a.s6);
    double e[2] = {0.0, 0.0};
    if (i < p.n && sub == 0) {
        F fx, fy, fz;
        lean_finish(p, a, fx, fy, fz, e[0], e[1]);
        copy_home<kCopy, false>(p, i);
        fout[0][i] = fx;
        fout[1][i] = fy;
        fout[2][i] = fz;
        if (!isfinite(e[0] + (double)fx + (double)fy + (double)fz))
            atomicOr(&p.dev->flags, (int)MD_FLAG_NONFINITE);
    }
    block_sum<2>(e, red);
    if (threadIdx.x == 0) {
        p.fpart[2 * wg.id] = e[0];
        p.fpart[2 * wg.id + 1] = e[1];
    }
}

template <typename F, typename Acc, class B>
static void half_seq(const B& b, const LaunchShape& sh, hipStream_t s)
{
    hipLaunchKernelGGL((k_zero_forces<F, B>), dim3(sh.grid[G_ATOMS]), dim3(sh.block), 0, s, b);
    const dim3 g(sh.grid[G_TILES]), t(sh.force_block);
    const size_t lds = sh.force_lds;
    switch (sh.force_lanes) {
        case 8: hipLaunchKernelGGL((k_forces_half<F, Acc, 8, B>), g, t, lds, s, b); break;
        case 2: hipLaunchKernelGGL((k_forces_half<F, Acc, 2, B>), g, t, lds, s, b); break;
        case 4: hipLaunchKernelGGL((k_forces_half<F, Acc, 4, B>), g, t, lds, s, b); break;
        default: hipLaunchKernelGGL((k_forces_half<F, Acc, 1, B>), g, t, lds, s, b); break;
    }
}

template <typename F, typename Acc, class B>
static void tiles_seq(const B& b, const LaunchShape& sh, hipStream_t s)
{
    if (sh.newton3) {
        half_seq<F, Acc>(b, sh, s);
        return;
    }
    const dim3 g(sh.grid[G_TILES]), t(sh.force_block);
    const size_t lds = sh.force_lds;
    switch (sh.force_lanes) {
        case 8: hipLaunchKernelGGL((k_forces_tiles<F, Acc, 8, B>), g, t, lds, s, b); break;
        case 2: hipLaunchKernelGGL((k_forces_tiles<F, Acc, 2, B>), g, t, lds, s, b); break;
        case 4: hipLaunchKernelGGL((k_forces_tiles<F, Acc, 4, B>), g, t, lds, s, b); break;
        default: hipLaunchKernelGGL((k_forces_tiles<F, Acc, 1, B>), g, t, lds, s, b); break;
    }
}

template <class B>
static void forces_seq(const B& b, const LaunchShape& sh, hipStream_t s, int flags = 0)
{
    if (sh.mode == MD_CELLS_ONLY) {
        const dim3 g(sh.grid[G_TILES]), t(sh.block);
        const bool copy = (flags & kFoldCopy) && sh.reorder;
        if (sh.precision == MD_FP64 && copy)
            hipLaunchKernelGGL((k_forces_cells<double, AccD, B, true>), g, t, 0, s, b);
        else if (sh.precision == MD_FP64)
            hipLaunchKernelGGL((k_forces_cells<double, AccD, B, false>), g, t, 0, s, b);
        else if (copy)
            hipLaunchKernelGGL((k_forces_cells<float, AccF, B, true>), g, t, 0, s, b);
        else
            hipLaunchKernelGGL((k_forces_cells<float, AccF, B, false>), g, t, 0, s, b);
        return;
    }
    if (sh.precision == MD_FP64)
        tiles_seq<double, AccD>(b, sh, s);
    else
        tiles_seq<float, AccF>(b, sh, s);
}

int force_blocks(const KParams& p) { return grid_of(p, G_TILES); }

size_t force_lds_bytes(const KParams& p)
{
    if (p.mode != MD_NEIGHBOR_LIST) return 0;
    return p.newton3 ? stage_bytes(p, p.scap_aux, true) : stage_bytes(p, p.scap);
}

LaunchShape shape_of(const KParams& p)
{
    LaunchShape sh;
    for (int k = 0; k < G_KINDS; ++k) sh.grid[k] = grid_of(p, (GridKind)k);
    sh.block = p.block;
    sh.force_block = p.force_block;
    sh.force_lanes = p.force_lanes;
    sh.nl_block = p.nl_block;
    sh.nl_method = p.nl_method;
    sh.nl_lds = p.mode == MD_NEIGHBOR_LIST ? nl_lds_bytes(p) : 0;
    sh.force_lds = force_lds_bytes(p);
    sh.precision = p.precision;
    sh.reorder = p.reorder;
    sh.mode = p.mode;
    sh.newton3 = p.newton3;
    sh.nl_full = p.nc < 5 || !nl_small(p);
    return sh;
}

void launch_forces(const KParams& p, hipStream_t s, int flags)
{
    forces_seq(Single{p}, shape_of(p), s, flags);
}

void launch_forces(const Batch& b, const LaunchShape& sh, hipStream_t s) { forces_seq(b, sh, s); }

}  // namespace md
