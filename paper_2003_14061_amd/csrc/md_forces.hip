// md_forces.hip -- step F1 of section 2.3 (and the per-workgroup part of F2).
//
// One lane per atom walks its row of the neighbor matrix (or, in cells-only
// mode, the 27 surrounding cells) and accumulates the force on that atom
// alone: every pair is met twice, once from each side, so no atomics are
// needed (the paper's choice).  Pairs at r^2 >= r_cut^2 are skipped.  The
// potential energy and virial are reduced per workgroup (wave64 shuffles,
// then LDS) and written as partials for the reduction kernels.
//
// Precision: FP64 forms everything in double.  FP32-mixed forms the pair
// separation and the cutoff test in double, then the pair force, energy and
// virial and the per-atom sums in float.
//
// Atoms whose coordinates all lie at least r_cut + skin from every face
// (and whose partners therefore cannot straddle the periodic boundary)
// skip the minimum-image step when the whole wave qualifies; there the
// image correction is exactly zero.
#include "md_device.h"

namespace md {

struct AccD {
    double fx = 0, fy = 0, fz = 0, u = 0, w = 0;
    int np = 0;
};

struct AccF {
    float fx = 0, fy = 0, fz = 0, u = 0, w = 0;
    int np = 0;
};

__device__ __forceinline__ void pair_acc(const KParams& p, double dx, double dy, double dz,
                                         double r2, AccD& a)
{
    const double inv = recip(r2);
    const double sr2 = p.sig2 * inv;
    const double sr6 = sr2 * sr2 * sr2;
    const double fr = p.eps48 * sr6 * (sr6 - 0.5) * inv;
    a.fx += fr * dx;
    a.fy += fr * dy;
    a.fz += fr * dz;
    a.u += sr6 * (sr6 - 1.0);
    a.w += fr * r2;
    a.np += 1;
}

__device__ __forceinline__ float recipf(float a)
{
    float y = __builtin_amdgcn_rcpf(a);
    return __builtin_fmaf(y, __builtin_fmaf(-a, y, 1.0f), y);
}

__device__ __forceinline__ void pair_acc(const KParams& p, double dx, double dy, double dz,
                                         double r2, AccF& a)
{
    const float r2f = (float)r2;
    const float inv = recipf(r2f);
    const float sr2 = (float)p.sig2 * inv;
    const float sr6 = sr2 * sr2 * sr2;
    const float fr = (float)p.eps48 * sr6 * (sr6 - 0.5f) * inv;
    a.fx += fr * (float)dx;
    a.fy += fr * (float)dy;
    a.fz += fr * (float)dz;
    a.u += sr6 * (sr6 - 1.0f);
    a.w += fr * r2f;
    a.np += 1;
}

template <bool kInterior, typename Acc>
__device__ __forceinline__ void visit(const KParams& p, double xi, double yi, double zi, int j,
                                      Acc& a)
{
    double dx = xi - p.x[j], dy = yi - p.y[j], dz = zi - p.z[j];
    if (!kInterior) {
        dx = minimg(dx, p.L, p.invL);
        dy = minimg(dy, p.L, p.invL);
        dz = minimg(dz, p.L, p.invL);
    }
    const double r2 = dist2(dx, dy, dz);
    if (r2 < p.rc2) pair_acc(p, dx, dy, dz, r2, a);
}

template <bool kInterior, typename Acc>
__device__ __forceinline__ void walk_list(const KParams& p, int i, Acc& a)
{
    const double xi = p.x[i], yi = p.y[i], zi = p.z[i];
    const int cnt = p.nl_count[i];
    const int* row = p.nl + i;
    for (int m = 0; m < cnt; ++m) visit<kInterior>(p, xi, yi, zi, row[(int64_t)m * p.npad], a);
}

template <bool kInterior, typename Acc>
__device__ __forceinline__ void walk_cells(const KParams& p, int i, Acc& a)
{
    const double xi = p.x[i], yi = p.y[i], zi = p.z[i];
    const int nc = p.nc, c = p.cell_of[i];
    const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
    for (int dz = -1; dz <= 1; ++dz) {
        const int zz = wrap_cell(cz + dz, nc);
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = wrap_cell(cy + dy, nc);
            for (int dx = -1; dx <= 1; ++dx) {
                const int c2 = (zz * nc + yy) * nc + wrap_cell(cx + dx, nc);
                for (int k = p.cell_start[c2]; k < p.cell_start[c2 + 1]; ++k) {
                    const int j = p.order[k];
                    if (j != i) visit<kInterior>(p, xi, yi, zi, j, a);
                }
            }
        }
    }
}

template <typename F, typename Acc, bool kCells>
__global__ void k_forces(KParams p)
{
    __shared__ double red[(1024 / kWave) * 2];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    Acc a;
    if (i < p.n) {
        bool inner;
        if (kCells) {
            const int c = p.cell_of[i], nc = p.nc;
            const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
            inner = nc >= 5 && cx >= 1 && cx <= nc - 2 && cy >= 1 && cy <= nc - 2 && cz >= 1 &&
                    cz <= nc - 2;
        } else {
            const double xi = p.x[i], yi = p.y[i], zi = p.z[i];
            inner = xi >= p.inner_lo && xi <= p.inner_hi && yi >= p.inner_lo &&
                    yi <= p.inner_hi && zi >= p.inner_lo && zi <= p.inner_hi;
        }
        if (__all(inner)) {
            if (kCells) walk_cells<true>(p, i, a); else walk_list<true>(p, i, a);
        } else {
            if (kCells) walk_cells<false>(p, i, a); else walk_list<false>(p, i, a);
        }
        static_cast<F*>(p.fx)[i] = a.fx;
        static_cast<F*>(p.fy)[i] = a.fy;
        static_cast<F*>(p.fz)[i] = a.fz;
    }
    // per-atom energy: half of each pair's 4 eps (sr12 - sr6) - shift
    double e[2];
    e[0] = i < p.n ? p.eps2 * (double)a.u - p.half_shift * (double)a.np : 0.0;
    e[1] = i < p.n ? 0.5 * (double)a.w : 0.0;
    if (i < p.n && !isfinite(e[0] + (double)a.fx + (double)a.fy + (double)a.fz))
        atomicOr(&p.dev->flags, (int)MD_FLAG_NONFINITE);
    block_sum<2>(e, red);
    if (threadIdx.x == 0) {
        p.fpart[2 * blockIdx.x] = e[0];
        p.fpart[2 * blockIdx.x + 1] = e[1];
    }
}

void launch_forces(const KParams& p, hipStream_t s)
{
    const int b = p.block;
    const dim3 g(p.nblk_force), t(b);
    const bool cells = p.mode == MD_CELLS_ONLY;
    if (p.precision == MD_FP64) {
        if (cells) hipLaunchKernelGGL((k_forces<double, AccD, true>), g, t, 0, s, p);
        else hipLaunchKernelGGL((k_forces<double, AccD, false>), g, t, 0, s, p);
    } else {
        if (cells) hipLaunchKernelGGL((k_forces<float, AccF, true>), g, t, 0, s, p);
        else hipLaunchKernelGGL((k_forces<float, AccF, false>), g, t, 0, s, p);
    }
}

}  // namespace md
