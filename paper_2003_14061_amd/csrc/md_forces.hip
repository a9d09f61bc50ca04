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
// Cells-only mode: one lane per atom walks the 27 surrounding cells.
//
// Precision: FP64 forms everything in double.  FP32-mixed forms the pair
// separation and the cutoff test in double, then the pair force, energy and
// virial and the per-atom sums in float.
//
// The energy and virial are reduced per workgroup (wave64 shuffles, then
// LDS) and written as partials for the reduction kernels.
#include "md_tiles.h"

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

template <int LANES, typename T>
__device__ __forceinline__ T lane_group_sum(T v)
{
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// The 4 entries of one chunk.  kMask = false: partners from LDS, padded
// entries point at the sentinel atom, nothing needs masking (wrap-bit image
// modes only).  kMask = true: entries past the list are masked; with
// kFits = false the partners come from global memory.
template <int kImage, bool kFits, bool kMask, typename Acc>
__device__ __forceinline__ void chunk_pairs(const KParams& p, const Stage& s, uint64_t ch,
                                            int mbase, int cnt, double xi, double yi, double zi,
                                            Acc& a)
{
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
        const uint32_t v = (uint32_t)(ch >> (16 * k)) & 0xffffu;
        const bool valid = !kMask || mbase + k < cnt;
        int e = (int)(v & kEntryMask);
        double xj, yj, zj;
        if (kFits) {
            if (kMask) e = valid ? e : 0;
            xj = s.xs[e];
            yj = s.ys[e];
            zj = s.zs[e];
        } else {
            const int j = staged_slot(p, s, valid && e < s.total ? e : 0);
            xj = p.x[j];
            yj = p.y[j];
            zj = p.z[j];
        }
        double dx = xi - xj, dy = yi - yj, dz = zi - zj;
        image<kImage>(p, (int)(v >> kEntryBits), dx, dy, dz);
        const double r2 = dist2(dx, dy, dz);
        if (valid && r2 < p.rc2) pair_acc(p, dx, dy, dz, r2, a);
    }
}

// Chunks c = sub, sub+LANES, ... of one home atom's list, each loaded one
// step ahead of its use.
template <int LANES, int kImage, bool kFits, bool kMask, typename Acc>
__device__ __forceinline__ void walk_list(const KParams& p, const Stage& s, int slot_i, int sub,
                                          int cnt, double xi, double yi, double zi, Acc& a)
{
    const int nchunk = (cnt + kChunk - 1) / kChunk;
    const uint64_t* col = p.nl64 + slot_i;
    int c = sub;
    uint64_t next = c < nchunk ? col[(int64_t)c * p.npad] : 0;
    while (c < nchunk) {
        const uint64_t ch = next;
        const int cn = c + LANES;
        if (cn < nchunk) next = col[(int64_t)cn * p.npad];
        chunk_pairs<kImage, kFits, kMask>(p, s, ch, c * kChunk, cnt, xi, yi, zi, a);
        c = cn;
    }
}

template <typename F, typename Acc, int LANES>
__global__ void k_forces_tiles(KParams p)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ double red[(1024 / kWave) * 2];
    const Tile g = tile_of(p, xcd_tile(blockIdx.x, gridDim.x));
    Stage s = stage_layout(p, smem);
    stage_tables(p, g, s);
    const int nh = home_count(s), h0 = home_first_lds(s), slot0 = home_first_slot(s);
    const int mode = image_mode(p, tile_interior(p, g));
    stage_positions(p, s);
    __syncthreads();
    const int per_pass = blockDim.x / LANES;
    const int sub = threadIdx.x % LANES;
    double e[2] = {0.0, 0.0};
    for (int hb = 0; hb < nh; hb += per_pass) {
        const int h = hb + threadIdx.x / LANES;
        Acc a;
        int slot_i = 0;
        if (h < nh) {
            slot_i = atom_at(p, slot0 + h);
            const int cnt = p.nl_count[slot_i];
            double xi, yi, zi;
            if (s.fits) {
                xi = s.xs[h0 + h];
                yi = s.ys[h0 + h];
                zi = s.zs[h0 + h];
            } else {
                xi = p.x[slot_i];
                yi = p.y[slot_i];
                zi = p.z[slot_i];
            }
            if (!s.fits) {
                if (mode == 2)
                    walk_list<LANES, 2, false, true>(p, s, slot_i, sub, cnt, xi, yi, zi, a);
                else
                    walk_list<LANES, 1, false, true>(p, s, slot_i, sub, cnt, xi, yi, zi, a);
            } else if (mode == 0) {
                walk_list<LANES, 0, true, false>(p, s, slot_i, sub, cnt, xi, yi, zi, a);
            } else if (mode == 1) {
                walk_list<LANES, 1, true, false>(p, s, slot_i, sub, cnt, xi, yi, zi, a);
            } else {
                walk_list<LANES, 2, true, true>(p, s, slot_i, sub, cnt, xi, yi, zi, a);
            }
        }
        if (LANES > 1) {
            a.fx = lane_group_sum<LANES>(a.fx);
            a.fy = lane_group_sum<LANES>(a.fy);
            a.fz = lane_group_sum<LANES>(a.fz);
            a.u = lane_group_sum<LANES>(a.u);
            a.w = lane_group_sum<LANES>(a.w);
            a.np = lane_group_sum<LANES>(a.np);
        }
        if (h < nh && sub == 0) {
            static_cast<F*>(p.fx)[slot_i] = a.fx;
            static_cast<F*>(p.fy)[slot_i] = a.fy;
            static_cast<F*>(p.fz)[slot_i] = a.fz;
            // per-atom energy: half of each pair's 4 eps (sr12 - sr6) - shift
            const double ui = p.eps2 * (double)a.u - p.half_shift * (double)a.np;
            e[0] += ui;
            e[1] += 0.5 * (double)a.w;
            if (!isfinite(ui + (double)a.fx + (double)a.fy + (double)a.fz))
                atomicOr(&p.dev->flags, (int)MD_FLAG_NONFINITE);
        }
    }
    block_sum<2>(e, red);
    if (threadIdx.x == 0) {
        p.fpart[2 * blockIdx.x] = e[0];
        p.fpart[2 * blockIdx.x + 1] = e[1];
    }
}

// ---- cells-only mode ----

template <bool kInterior, typename Acc>
__device__ __forceinline__ void visit(const KParams& p, double xi, double yi, double zi,
                                      double xj, double yj, double zj, bool valid, Acc& a)
{
    double dx = xi - xj, dy = yi - yj, dz = zi - zj;
    if (!kInterior) {
        dx = minimg(dx, p.L, p.invL);
        dy = minimg(dy, p.L, p.invL);
        dz = minimg(dz, p.L, p.invL);
    }
    const double r2 = dist2(dx, dy, dz);
    if (valid && r2 < p.rc2) pair_acc(p, dx, dy, dz, r2, a);
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
                    visit<kInterior>(p, xi, yi, zi, p.x[j], p.y[j], p.z[j], j != i, a);
                }
            }
        }
    }
}

template <typename F, typename Acc>
__global__ void k_forces_cells(KParams p)
{
    __shared__ double red[(1024 / kWave) * 2];
    const int i = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    Acc a;
    if (i < p.n) {
        const int c = p.cell_of[i], nc = p.nc;
        const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
        const bool inner = nc >= 5 && cx >= 1 && cx <= nc - 2 && cy >= 1 && cy <= nc - 2 &&
                           cz >= 1 && cz <= nc - 2;
        if (__all(inner))
            walk_cells<true>(p, i, a);
        else
            walk_cells<false>(p, i, a);
        static_cast<F*>(p.fx)[i] = a.fx;
        static_cast<F*>(p.fy)[i] = a.fy;
        static_cast<F*>(p.fz)[i] = a.fz;
    }
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

template <typename F, typename Acc>
static void launch_tiles(const KParams& p, hipStream_t s)
{
    const dim3 g(p.n_tiles), t(p.force_block);
    const size_t lds = stage_bytes(p.scap, p.kx_max);
    switch (p.force_lanes) {
        case 8: hipLaunchKernelGGL((k_forces_tiles<F, Acc, 8>), g, t, lds, s, p); break;
        case 2: hipLaunchKernelGGL((k_forces_tiles<F, Acc, 2>), g, t, lds, s, p); break;
        case 4: hipLaunchKernelGGL((k_forces_tiles<F, Acc, 4>), g, t, lds, s, p); break;
        default: hipLaunchKernelGGL((k_forces_tiles<F, Acc, 1>), g, t, lds, s, p); break;
    }
}

int force_blocks(const KParams& p)
{
    if (p.mode == MD_CELLS_ONLY) return (p.n + p.block - 1) / p.block;
    return p.n_tiles;
}

void launch_forces(const KParams& p, hipStream_t s)
{
    if (p.mode == MD_CELLS_ONLY) {
        const dim3 g(p.nblk_force), t(p.block);
        if (p.precision == MD_FP64)
            hipLaunchKernelGGL((k_forces_cells<double, AccD>), g, t, 0, s, p);
        else
            hipLaunchKernelGGL((k_forces_cells<float, AccF>), g, t, 0, s, p);
        return;
    }
    if (p.precision == MD_FP64)
        launch_tiles<double, AccD>(p, s);
    else
        launch_tiles<float, AccF>(p, s);
}

}  // namespace md
