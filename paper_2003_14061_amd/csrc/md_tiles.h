// md_tiles.h -- LDS-staged cell tiles shared by the list build and the
// force pass.
//
// A tile is a run of `kx` consecutive cells along x in one (cy, cz) row of
// cells.  Its workgroup stages, for each of the 9 rows (cz+dz, cy+dy),
// dz, dy in {-1, 0, 1} (dz slowest), the kx+2 cells cx0-1 .. cx0+kx in that
// order, taken modulo nc (a cell can appear twice when kx+2 > nc).  Staged
// cell (s, q), s = 3(dz+1) + (dy+1), q = 0..kx+1, occupies LDS entries
// [off[s(kx+2)+q], off[s(kx+2)+q+1]), in the cell's slot order (ascending
// permanent id).  So for a home cell at q the three cells dx = -1, 0, +1 are
// q-1, q, q+1 of every staged row: the paper's 27-cell neighborhood, walked
// in the canonical order (section 2.3, step N5).
//
// Each staged cell carries wrap bits (1: x, 2: y, 4: z) telling which
// coordinates of a pair that reaches it cross the periodic boundary, the
// flag bits of section 4.1, factor (4).  With at least 5 cells per side a
// non-wrapped separation is below 2L/5 and a wrapped one lies between 3L/5
// and L, so the minimum image is the raw difference, minus L*sign(d) in
// each flagged coordinate: the same two roundings as d - L*rint(d/L).
//
// List entries are 16 bits: the LDS index of the neighbor (13 bits) and its
// wrap bits (3 bits).  Tiles whose staged atoms exceed the LDS capacity
// still get a list (indices into the same virtual layout) and read the
// positions from global memory through the cell tables.
#pragma once

#include "md_device.h"

namespace md {

#define MD_LDS __attribute__((address_space(3)))

constexpr int kEntryBits = 13;
constexpr int kEntryMask = (1 << kEntryBits) - 1;
constexpr int kMaxStaged = 1 << kEntryBits;  // virtual layout limit
constexpr int kChunk = 4;                    // entries per 8-byte list chunk

struct Tile {
    int cz, cy, cx0, kx;
};

// Atom stored at position k of the cell-ordered list (the identity once the
// atoms have been reordered by cell).
__device__ __forceinline__ int atom_at(const KParams& p, int k)
{
    return p.reorder ? k : p.order[k];
}

__device__ __forceinline__ Tile tile_of(const KParams& p, int t)
{
    const int row = t / p.tiles_per_row, seg = t % p.tiles_per_row;
    const int base = p.nc / p.tiles_per_row, rem = p.nc % p.tiles_per_row;
    Tile g;
    g.cz = row / p.nc;
    g.cy = row % p.nc;
    g.cx0 = seg * base + (seg < rem ? seg : rem);
    g.kx = base + (seg < rem ? 1 : 0);
    return g;
}

// LDS view of one staged tile.  Entry `total` of xs, ys, zs holds a sentinel
// atom far outside the box; list chunks are padded with its index, so a
// padded entry never falls inside the cutoff.
struct Stage {
    MD_LDS double *xs, *ys, *zs;  // [scap]
    MD_LDS int* off;              // [ntab + 1] LDS offset of each staged cell
    MD_LDS int* slot;             // [ntab] global slot of each staged cell's first atom
    MD_LDS int* flag;             // [ntab] wrap bits
    MD_LDS int* scan;             // [kWave] scratch
    int ntab, stride, total;
    bool fits;                    // total + 1 <= scap: positions (and sentinel) staged
};

constexpr double kSentinel = 1.0e30;

// Ints of the table region, rounded up to 16 bytes.
__host__ __device__ __forceinline__ int stage_table_ints(int kx_max)
{
    const int ntab = 9 * (kx_max + 2);
    return (3 * ntab + 1 + kWave + 3) / 4 * 4;
}

// Dynamic LDS bytes of the staged tile.
inline size_t stage_bytes(int scap, int kx_max)
{
    return sizeof(double) * 3 * (size_t)scap + sizeof(int) * (size_t)stage_table_ints(kx_max);
}

__device__ __forceinline__ Stage stage_layout(const KParams& p, char* smem)
{
    Stage s;
    s.xs = (MD_LDS double*)smem;
    s.ys = s.xs + p.scap;
    s.zs = s.ys + p.scap;
    const int ntab_max = 9 * (p.kx_max + 2);
    s.off = (MD_LDS int*)(s.zs + p.scap);
    s.slot = s.off + ntab_max + 1;
    s.flag = s.slot + ntab_max;
    s.scan = s.flag + ntab_max;
    return s;
}

// Cell tables of tile g: slots, wrap bits and LDS offsets of the staged
// cells (one round of global loads, then a workgroup scan).  Every thread of
// the workgroup must call it.
__device__ __forceinline__ void stage_tables(const KParams& p, const Tile& g, Stage& s)
{
    const int nc = p.nc;
    s.stride = g.kx + 2;
    s.ntab = 9 * s.stride;
    int carry = 0;
    for (int base = 0; base < s.ntab; base += blockDim.x) {
        const int t = base + threadIdx.x;
        int cnt = 0;
        if (t < s.ntab) {
            const int sg = t / s.stride, q = t % s.stride;
            const int zz = g.cz + sg / 3 - 1, yy = g.cy + sg % 3 - 1, xx = g.cx0 - 1 + q;
            const int fl = ((xx < 0 || xx >= nc) ? 1 : 0) | ((yy < 0 || yy >= nc) ? 2 : 0) |
                           ((zz < 0 || zz >= nc) ? 4 : 0);
            const int c = (wrap_cell(zz, nc) * nc + wrap_cell(yy, nc)) * nc + wrap_cell(xx, nc);
            const int a = p.cell_start[c];
            cnt = p.cell_start[c + 1] - a;
            s.slot[t] = a;
            s.flag[t] = fl;
        }
        // workgroup exclusive scan of cnt
        const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
        int inc = cnt;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int v = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += v;
        }
        if (lane == kWave - 1) s.scan[wid] = inc;
        __syncthreads();
        int before = 0, tot = 0;
        for (int w = 0; w < (int)blockDim.x / kWave; ++w) {
            before += w < wid ? s.scan[w] : 0;
            tot += s.scan[w];
        }
        if (t < s.ntab) s.off[t] = carry + before + inc - cnt;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) s.off[s.ntab] = carry;
    s.total = carry;
    s.fits = carry < p.scap;
    __syncthreads();
}

// Last staged cell t with off[t] <= k (k < total), i.e. the cell holding
// staged entry k (empty cells are skipped by taking the last match).
__device__ __forceinline__ int staged_cell(const Stage& s, int k)
{
    int lo = 0, hi = s.ntab - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.off[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Positions of the staged atoms into LDS (when they fit), plus the sentinel.
// Each thread takes entries tid, tid + blockDim, ... four at a time, so that
// several loads are in flight per thread.  No barrier: the caller syncs.
__device__ __forceinline__ void stage_positions(const KParams& p, const Stage& s)
{
    if (!s.fits) return;
    constexpr int U = 4;
    for (int k0 = threadIdx.x; k0 < s.total; k0 += U * blockDim.x) {
        double vx[U], vy[U], vz[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * blockDim.x;
            if (k < s.total) {
                const int t = staged_cell(s, k);
                const int j = atom_at(p, s.slot[t] + (k - s.off[t]));
                vx[u] = p.x[j];
                vy[u] = p.y[j];
                vz[u] = p.z[j];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * blockDim.x;
            if (k < s.total) {
                s.xs[k] = vx[u];
                s.ys[k] = vy[u];
                s.zs[k] = vz[u];
            }
        }
    }
    if (threadIdx.x == 0) {
        s.xs[s.total] = kSentinel;
        s.ys[s.total] = kSentinel;
        s.zs[s.total] = kSentinel;
    }
}

// Atom (storage slot) of staged entry e.
__device__ __forceinline__ int staged_slot(const KParams& p, const Stage& s, int e)
{
    const int t = staged_cell(s, e);
    return atom_at(p, s.slot[t] + (e - s.off[t]));
}

// Minimum image of a staged pair.  kImage: 0 -- no wrap anywhere in the
// tile, the raw difference is exact; 1 -- at least 5 cells per side: the raw
// difference, minus L*sign(d) in each flagged coordinate; 2 -- fewer than 5
// cells per side: d - L*rint(d/L) in every coordinate.
template <int kImage>
__device__ __forceinline__ void image(const KParams& p, int fl, double& dx, double& dy,
                                      double& dz)
{
#pragma clang fp contract(off)
    if (kImage == 2) {
        dx = minimg(dx, p.L, p.invL);
        dy = minimg(dy, p.L, p.invL);
        dz = minimg(dz, p.L, p.invL);
    } else if (kImage == 1) {
        if (fl) {
            if (fl & 1) dx = dx > 0.0 ? dx - p.L : dx + p.L;
            if (fl & 2) dy = dy > 0.0 ? dy - p.L : dy + p.L;
            if (fl & 4) dz = dz > 0.0 ? dz - p.L : dz + p.L;
        }
    }
}

// Which image rule a tile needs (see image()).
__device__ __forceinline__ int image_mode(const KParams& p, bool interior)
{
    return p.nc < 5 ? 2 : (interior ? 0 : 1);
}

// Home atoms of a tile: the kx cells q = 1..kx of the middle row (s = 4),
// contiguous in LDS and in the cell-ordered list (home atom h is
// atom_at(home_first_slot + h)).
__device__ __forceinline__ int home_first_lds(const Stage& s) { return s.off[4 * s.stride + 1]; }
__device__ __forceinline__ int home_count(const Stage& s)
{
    return s.off[4 * s.stride + s.stride - 1] - s.off[4 * s.stride + 1];
}
__device__ __forceinline__ int home_first_slot(const Stage& s) { return s.slot[4 * s.stride + 1]; }

// True when no staged cell of the tile wraps (and the grid has >= 5 cells).
__device__ __forceinline__ bool tile_interior(const KParams& p, const Tile& g)
{
    return p.nc >= 5 && g.cx0 >= 1 && g.cx0 + g.kx <= p.nc - 1 && g.cy >= 1 &&
           g.cy <= p.nc - 2 && g.cz >= 1 && g.cz <= p.nc - 2;
}

}  // namespace md
