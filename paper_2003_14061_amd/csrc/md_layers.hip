// md_layers.hip -- the paper's own pipeline, kept beside the tiled one as an
// A/B alternative (md_params.pipeline = MD_PIPE_LAYERS).  Section 2.3, as
// the paper lays the steps out, one thread per atom throughout:
//
//   N1      cell of each atom from its position (folded into [0, L) first)
//   N2      layer of the atom in its cell: an atomic increment of the cell's
//           occupancy (the order of atoms within a cell is the order the
//           atomics happened in, which the paper notes is indeterminate)
//   N3-N4   the layer matrix: entry (cell, layer) holds the atom
//   N5      the neighbor matrix W: for each atom, the 27 surrounding cells in
//           (dz, dy, dx) order, each cell's layers in order; entry m of atom
//           i at row m, column i (32-bit atom indices), so the threads of a
//           wave read one row at consecutive addresses
//   F1      forces: each thread walks its atom's column of W and gathers the
//           partners' positions from global memory
//
// The energy and virial of F1 go to per-workgroup partials, reduced like
// those of the tiled pass.  Separations take the minimum image d - L
// rint(d/L) in every coordinate (no wrap bits).
//
// Reorder (section 2.4, item (4); every 100 steps in the paper's runs,
// section 3): with md_params.reorder = k > 0, every k-th step packs the
// layer matrix of the last build into the atom sequence s (cells in order,
// each cell's layers in order) and permutes the atoms' coordinates,
// velocities and permanent ids to it through scratch arrays, after which the
// layer and neighbor matrices are rebuilt.  The paper builds s on the host
// and names the GPU alternative, a prefix scan of the cell occupancies that
// tells each cell where its atoms go; that is what is done here (k_scan of
// the tiled cell build, then one thread per cell).  The forces are not
// permuted: the force pass that follows rewrites all of them.
#include "md_pair.h"

namespace md {

__global__ void k_layer_clear(KParams p, int force)
{
    if (!force && !p.dev->rebuild) return;
    const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
    for (int c = i0; c < p.ncell; c += gridDim.x * blockDim.x) p.cell_count[c] = 0;
    if (i0 == 0) {
        p.dev->max_occ = 0;
        p.dev->max_nl = 0;
    }
}

// N1, N2, N3: fold, cell, layer, layer-matrix entry.
__global__ void k_layer_assign(KParams p, int force)
{
    if (!force && !p.dev->rebuild) return;
    int occ = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += gridDim.x * blockDim.x) {
        const double x = wrap(p.x[i], p.L), y = wrap(p.y[i], p.L), z = wrap(p.z[i], p.L);
        p.x[i] = x;
        p.y[i] = y;
        p.z[i] = z;
        const int c = cell_of_pos(x, y, z, p);
        p.cell_of[i] = c;
        const int l = atomicAdd(&p.cell_count[c], 1);
        if (l < p.n_layers)
            p.layers[(int64_t)c * p.n_layers + l] = i;
        else
            atomicOr(&p.dev->flags, (int)MD_FLAG_LAYER_OVERFLOW);
        occ = l + 1 > occ ? l + 1 : occ;
    }
    occ = workgroup_max(occ);
    if (threadIdx.x == 0 && occ > 0) atomicMax(&p.dev->max_occ, occ);
}

// N5: the neighbor matrix, and the displacement references.
__global__ void k_layer_nl(KParams p, int force)
{
    if (!force && !p.dev->rebuild) return;
    int longest = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += gridDim.x * blockDim.x) {
        const double xi = p.x[i], yi = p.y[i], zi = p.z[i];
        const int nc = p.nc, c = p.cell_of[i];
        const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
        int m = 0;
        for (int dz = -1; dz <= 1; ++dz) {
            const int zz = wrap_cell(cz + dz, nc);
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = wrap_cell(cy + dy, nc);
                for (int dx = -1; dx <= 1; ++dx) {
                    const int c2 = (zz * nc + yy) * nc + wrap_cell(cx + dx, nc);
                    const int occ = p.cell_count[c2];
                    const int nl = occ < p.n_layers ? occ : p.n_layers;
                    const int* col = p.layers + (int64_t)c2 * p.n_layers;
                    for (int l = 0; l < nl; ++l) {
                        const int j = col[l];
                        if (j == i) continue;
                        const double ex = minimg(xi - p.x[j], p.L, p.invL);
                        const double ey = minimg(yi - p.y[j], p.L, p.invL);
                        const double ez = minimg(zi - p.z[j], p.L, p.invL);
                        if (dist2(ex, ey, ez) < p.rl2) {
                            if (m < p.cap) p.w32[(int64_t)m * p.npad + i] = j;
                            ++m;
                        }
                    }
                }
            }
        }
        p.nl_count[i] = m < p.cap ? m : p.cap;
        p.xr[i] = xi;
        p.yr[i] = yi;
        p.zr[i] = zi;
        longest = m > longest ? m : longest;
    }
    longest = workgroup_max(longest);
    if (threadIdx.x == 0 && longest > 0) {
        atomicMax(&p.dev->max_nl, longest);
        if (longest > p.cap) atomicOr(&p.dev->flags, (int)MD_FLAG_NL_OVERFLOW);
    }
}

// F1: a thread per atom over its column of W; partners gathered from HBM.
template <typename F, typename Acc>
__global__ void k_layer_forces(KParams p)
{
    __shared__ double red[(1024 / kWave) * 2];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    Acc a;
    if (i < p.n) {
        const double xi = p.x[i], yi = p.y[i], zi = p.z[i];
        const int cnt = p.nl_count[i];
        for (int m = 0; m < cnt; ++m) {
            const int j = p.w32[(int64_t)m * p.npad + i];
            const double ex = minimg(xi - p.x[j], p.L, p.invL);
            const double ey = minimg(yi - p.y[j], p.L, p.invL);
            const double ez = minimg(zi - p.z[j], p.L, p.invL);
            const double r2 = dist2(ex, ey, ez);
            if (r2 < p.rc2) pair_acc(p, ex, ey, ez, r2, a);
        }
        static_cast<F*>(p.fx)[i] = a.fx;
        static_cast<F*>(p.fy)[i] = a.fy;
        static_cast<F*>(p.fz)[i] = a.fz;
    }
    double e[2];
    e[0] = i < p.n ? p.eps2 * (double)a.u : 0.0;
    e[1] = i < p.n ? 0.5 * (double)a.w : 0.0;
    if (i < p.n && !isfinite(e[0] + (double)a.fx + (double)a.fy + (double)a.fz))
        atomicOr(&p.dev->flags, (int)MD_FLAG_NONFINITE);
    block_sum<2>(e, red);
    if (threadIdx.x == 0) {
        p.fpart[2 * blockIdx.x] = e[0];
        p.fpart[2 * blockIdx.x + 1] = e[1];
    }
}

// ---- reorder ----
// Every kernel leaves the state alone when a layer overflow is latched (the
// layer matrix then lacks atoms, so s would not be a permutation).

__device__ __forceinline__ bool layers_whole(const KParams& p)
{
    return (p.dev->flags & MD_FLAG_LAYER_OVERFLOW) == 0;
}

// s: the atoms of cell c at cell_start[c] .. in layer order.
__global__ void k_layer_pack(KParams p)
{
    if (!layers_whole(p)) return;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < p.ncell;
         c += gridDim.x * blockDim.x) {
        const int a = p.cell_start[c], cnt = p.cell_start[c + 1] - a;
        const int* col = p.layers + (int64_t)c * p.n_layers;
        for (int l = 0; l < cnt && l < p.n_layers; ++l) p.tmp[a + l] = col[l];
    }
}

// New slot d takes atom s[d]: coordinates, velocities and id into scratch.
__global__ void k_layer_permute(KParams p)
{
    if (!layers_whole(p)) return;
    for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < p.n; d += gridDim.x * blockDim.x) {
        const int a = p.tmp[d];
        p.sx[d] = p.x[a];
        p.sy[d] = p.y[a];
        p.sz[d] = p.z[a];
        p.svx[d] = p.vx[a];
        p.svy[d] = p.vy[a];
        p.svz[d] = p.vz[a];
        p.sid[d] = p.id[a];
    }
}

__global__ void k_layer_copyback(KParams p)
{
    if (!layers_whole(p)) return;
    for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < p.n; d += gridDim.x * blockDim.x) {
        p.x[d] = p.sx[d];
        p.y[d] = p.sy[d];
        p.z[d] = p.sz[d];
        p.vx[d] = p.svx[d];
        p.vy[d] = p.svy[d];
        p.vz[d] = p.svz[d];
        p.id[d] = p.sid[d];
    }
}

// W with -1 past each atom's length (the layout of md_export_neighbors).
__global__ void k_layer_export(KParams p, int32_t* out)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
         q < (int64_t)p.cap * p.npad; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q % p.npad), m = (int)(q / p.npad);
        out[q] = i < p.n && m < p.nl_count[i] ? p.w32[q] : -1;
    }
}

static dim3 atom_grid(const KParams& p)
{
    const int g = (p.n + p.block - 1) / p.block;
    return dim3(g < p.gate_grid ? g : p.gate_grid);
}

void launch_layer_cells(const KParams& p, int force, hipStream_t s)
{
    int gc = (p.ncell + p.block - 1) / p.block;
    gc = gc < p.gate_grid ? gc : p.gate_grid;
    hipLaunchKernelGGL(k_layer_clear, dim3(gc), dim3(p.block), 0, s, p, force);
    hipLaunchKernelGGL(k_layer_assign, atom_grid(p), dim3(p.block), 0, s, p, force);
}

void launch_layer_nl(const KParams& p, int force, hipStream_t s)
{
    hipLaunchKernelGGL(k_layer_nl, atom_grid(p), dim3(p.block), 0, s, p, force);
}

void launch_layer_forces(const KParams& p, hipStream_t s)
{
    const dim3 g((p.n + p.block - 1) / p.block);
    if (p.precision == MD_FP64)
        hipLaunchKernelGGL((k_layer_forces<double, AccD>), g, dim3(p.block), 0, s, p);
    else
        hipLaunchKernelGGL((k_layer_forces<float, AccF>), g, dim3(p.block), 0, s, p);
}

void launch_layer_reorder(const KParams& p, hipStream_t s)
{
    launch_cell_scan(p, s);
    int gc = (p.ncell + p.block - 1) / p.block;
    gc = gc < p.gate_grid ? gc : p.gate_grid;
    hipLaunchKernelGGL(k_layer_pack, dim3(gc), dim3(p.block), 0, s, p);
    hipLaunchKernelGGL(k_layer_permute, atom_grid(p), dim3(p.block), 0, s, p);
    hipLaunchKernelGGL(k_layer_copyback, atom_grid(p), dim3(p.block), 0, s, p);
}

void launch_layer_export(const KParams& p, int32_t* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_layer_export, dim3(1024), dim3(256), 0, s, p, out);
}

}  // namespace md
