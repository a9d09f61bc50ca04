// md_neighbors.hip -- step N5 of section 2.3: the neighbor matrix.
//
// One lane per atom.  The 27 surrounding cells are visited with dz, dy, dx
// each -1, 0, +1 (dz slowest) and each cell's atoms in the order the cell
// build left them (ascending permanent id), so the list comes out in one
// canonical order.  The list is stored the way the paper stores W: row m
// holds the m-th neighbor of every atom, so the force pass reads it with
// consecutive lanes at consecutive addresses.
//
// A workgroup whose atoms all sit in interior cells (no periodic wrap among
// the 27 cells, at least 5 cells per side) skips the minimum-image step:
// there every separation is below 2L/5, so rint(d/L) = 0 and the image
// correction leaves d unchanged bit for bit.
#include "md_device.h"

namespace md {

template <bool kInterior>
__device__ __forceinline__ int nl_scan_atom(const KParams& p, int i, int c)
{
    const double xi = p.x[i], yi = p.y[i], zi = p.z[i];
    const int nc = p.nc;
    const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
    int m = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        const int zz = wrap_cell(cz + dz, nc);
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = wrap_cell(cy + dy, nc);
            for (int dx = -1; dx <= 1; ++dx) {
                const int c2 = (zz * nc + yy) * nc + wrap_cell(cx + dx, nc);
                const int a = p.cell_start[c2], b = p.cell_start[c2 + 1];
                for (int k = a; k < b; ++k) {
                    const int j = p.order[k];
                    double ddx = xi - p.x[j], ddy = yi - p.y[j], ddz = zi - p.z[j];
                    if (!kInterior) {
                        ddx = minimg(ddx, p.L, p.invL);
                        ddy = minimg(ddy, p.L, p.invL);
                        ddz = minimg(ddz, p.L, p.invL);
                    }
                    if (dist2(ddx, ddy, ddz) < p.rl2 && j != i) {
                        if (m < p.cap) p.nl[(int64_t)m * p.npad + i] = j;
                        ++m;
                    }
                }
            }
        }
    }
    return m;
}

__global__ void k_nl_build(KParams p, int force)
{
    if (!force && !p.dev->rebuild) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int m = 0;
    if (i < p.n) {
        const int c = p.cell_of[i];
        const int nc = p.nc;
        const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
        const bool inner = nc >= 5 && cx >= 1 && cx <= nc - 2 && cy >= 1 && cy <= nc - 2 &&
                           cz >= 1 && cz <= nc - 2;
        if (__all(inner))
            m = nl_scan_atom<true>(p, i, c);
        else
            m = nl_scan_atom<false>(p, i, c);
        p.nl_count[i] = m < p.cap ? m : p.cap;
        p.xr[i] = p.x[i];
        p.yr[i] = p.y[i];
        p.zr[i] = p.z[i];
    }
    const int wm = wave_max(m);
    if ((threadIdx.x & (kWave - 1)) == 0 && wm > 0) {
        atomicMax(&p.dev->max_nl, wm);
        if (wm > p.cap) atomicOr(&p.dev->flags, (int)MD_FLAG_NL_OVERFLOW);
    }
}

void launch_neighbors(const KParams& p, int force, hipStream_t s)
{
    const int b = p.block;
    hipLaunchKernelGGL(k_nl_build, dim3((p.n + b - 1) / b), dim3(b), 0, s, p, force);
}

}  // namespace md
