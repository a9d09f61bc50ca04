// md_tiles.h -- LDS-staged cell tiles shared by the list build and the
// force pass.
//
// A tile is a block of kx x ky x kz home cells, x fastest: cells
// cx0 .. cx0+kx-1, cy0 .. cy0+ky-1, cz0 .. cz0+kz-1.  Its workgroup stages
// the (kx+2)(ky+2)(kz+2) cells around the block, taken modulo nc (a cell
// can appear twice on small grids): staged row (b, c), b = 0..ky+1,
// c = 0..kz+1, is the line of cells y = cy0-1+b, z = cz0-1+c; row index
// s = c (ky+2) + b; along a row, column q = 0..kx+1 is the cell
// x = cx0-1+q.  Staged cell t = s (kx+2) + q occupies LDS entries
// [off[t], off[t+1]) in the cell's slot order (ascending permanent id).  For
// home cell (a, b, c) (1 <= a <= kx, 1 <= b <= ky, 1 <= c <= kz) the 27-cell
// neighborhood in the canonical order (dz, dy, dx each -1, 0, +1, dz
// slowest; section 2.3, step N5) is, for each (dz, dy), the three
// consecutive staged cells q = a-1, a, a+1 of row (c+dz)(ky+2) + (b+dy).
// A block stages fewer cells per home cell than a single row of cells
// (9 (kx+2) / kx): at 3 x 2 x 2 cells it is 6.7 against 11.25 at 8 x 1 x 1.
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

// Floating-point adds for the third-law force pass: workgroup-scope on LDS,
// device-scope on global memory (the force arrays are ordinary device
// allocations, where the hardware's float and double atomic adds apply).
template <typename T>
__device__ __forceinline__ void lds_add(MD_LDS T* a, T v)
{
    __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <typename T>
__device__ __forceinline__ void global_add(T* a, T v)
{
    unsafeAtomicAdd(a, v);
}

constexpr int kEntryBits = 13;
constexpr int kEntryMask = (1 << kEntryBits) - 1;
constexpr int kMaxStaged = 1 << kEntryBits;  // virtual layout limit
constexpr int kChunk = 4;                    // entries per 8-byte list chunk
// Fourth word of a raw buffer resource on the gfx9 family (CDNA): 32-bit
// data, no swizzle, the range check on the byte offset alone.
constexpr int kBufferWord3 = 0x00020000;

struct Tile {
    int cx0, cy0, cz0, kx, ky, kz;
};

// Atom stored at position k of the cell-ordered list (the identity once the
// atoms have been reordered by cell).
__device__ __forceinline__ int atom_at(const KParams& p, int k)
{
    return p.reorder ? k : p.order[k];
}

// Cells c0 .. c0+k-1 of part i of nc cells cut into `parts` near-equal parts.
__device__ __forceinline__ void split_cells(int nc, int parts, int i, int& c0, int& k)
{
    const int base = nc / parts, rem = nc % parts;
    c0 = i * base + (i < rem ? i : rem);
    k = base + (i < rem ? 1 : 0);
}

// Tile t, x fastest, then y, then z: consecutive tiles are neighbors, so the
// contiguous tile ranges of the XCD-aware order are compact slabs.
__device__ __forceinline__ Tile tile_of(const KParams& p, int t)
{
    const int tx = t % p.tiles_x, r = t / p.tiles_x;
    const int ty = r % p.tiles_y, tz = r / p.tiles_y;
    Tile g;
    split_cells(p.nc, p.tiles_x, tx, g.cx0, g.kx);
    split_cells(p.nc, p.tiles_y, ty, g.cy0, g.ky);
    split_cells(p.nc, p.tiles_z, tz, g.cz0, g.kz);
    return g;
}

// LDS view of one staged tile.  Positions are interleaved, x y z of staged
// atom e at p3[3e .. 3e+2], so that one address serves a paired 16-byte read
// of (x, y) and an 8-byte read of z.  Entry `total` holds a sentinel atom
// far outside the box; list chunks are padded with its index, so a padded
// entry never falls inside the cutoff.  Kernels that also need a per-atom
// vector of each partner (the adjoint's lambda, the third-law reactions)
// keep it in a3, interleaved the same way.
struct Stage {
    MD_LDS double* p3;            // [cap][3]
    MD_LDS double* a3;            // [cap][3] when staged with an auxiliary vector
    MD_LDS int* off;              // [ntab + 1] LDS offset of each staged cell
    MD_LDS int* slot;             // [ntab] global slot of each staged cell's first atom
    MD_LDS int* flag;             // [ntab] wrap bits
    MD_LDS int* scan;             // [kWave] scratch of the scan; afterwards [0], [1]: the
                                  // columns where the staged x index wraps to 0 (or stride)
    MD_LDS int* hp;               // [nhr + 1] home atoms before each home row (prefix)
    int ntab, stride, rows_y, nrows, kx, ky, nhr, total, cap;
    bool fits;                    // total + 1 <= cap: positions (and sentinel) staged
};

constexpr double kSentinel = 1.0e30;

// The 3-vector of staged atom e from an interleaved [cap][3] LDS array.
__device__ __forceinline__ void lds_xyz(const MD_LDS double* a, int e, double& x, double& y,
                                        double& z)
{
    const MD_LDS double* q = a + 3 * e;
    x = q[0];
    y = q[1];
    z = q[2];
}

// Staged cells of the largest tile.
__host__ __device__ __forceinline__ int stage_cells_max(const KParams& p)
{
    return (p.kx_max + 2) * (p.ky_max + 2) * (p.kz_max + 2);
}

// Ints of the table region, rounded up to 16 bytes.
__host__ __device__ __forceinline__ int stage_table_ints(const KParams& p)
{
    const int ntab = stage_cells_max(p), nhr = p.ky_max * p.kz_max;
    return (3 * ntab + 1 + kWave + nhr + 1 + 3) / 4 * 4;
}

// Dynamic LDS bytes of the staged tile: positions (and with `aux` a second
// 3-vector) of cap atoms, then the cell tables.
inline size_t stage_bytes(const KParams& p, int cap, bool aux = false)
{
    return sizeof(double) * (aux ? 6 : 3) * (size_t)cap +
           sizeof(int) * (size_t)stage_table_ints(p);
}

// Candidate rounds (of 64) held in registers by the cell-wave list build
// (blocks of 192: the 533 candidates of the dense LJ state take three blocks
// either way, and three rounds hold fewer registers than four).
constexpr int kNlRounds = 3;

__device__ __forceinline__ Stage stage_layout(const KParams& p, char* smem, int cap, bool aux)
{
    Stage s;
    s.cap = cap;
    s.p3 = (MD_LDS double*)smem;
    s.a3 = aux ? s.p3 + 3 * cap : nullptr;
    const int ntab_max = stage_cells_max(p);
    s.off = (MD_LDS int*)(s.p3 + (aux ? 6 : 3) * cap);
    s.slot = s.off + ntab_max + 1;
    s.flag = s.slot + ntab_max;
    s.scan = s.flag + ntab_max;
    s.hp = s.scan + kWave;
    return s;
}

__device__ __forceinline__ Stage stage_layout(const KParams& p, char* smem)
{
    return stage_layout(p, smem, p.scap, false);
}

// Cell tables of tile g: slots, wrap bits and LDS offsets of the staged
// cells (one round of global loads, then a workgroup scan), and the prefix
// of home atoms over the home rows.  Every thread of the workgroup must call
// it.
__device__ __forceinline__ void stage_tables(const KParams& p, const Tile& g, Stage& s)
{
    const int nc = p.nc;
    s.kx = g.kx;
    s.ky = g.ky;
    s.stride = g.kx + 2;
    s.rows_y = g.ky + 2;
    s.nrows = s.rows_y * (g.kz + 2);
    s.ntab = s.nrows * s.stride;
    s.nhr = g.ky * g.kz;
    int carry = 0;
    for (int base = 0; base < s.ntab; base += blockDim.x) {
        const int t = base + threadIdx.x;
        int cnt = 0;
        if (t < s.ntab) {
            const int row = t / s.stride, q = t - row * s.stride;
            const int c = row / s.rows_y, b = row - c * s.rows_y;
            const int zz = g.cz0 - 1 + c, yy = g.cy0 - 1 + b, xx = g.cx0 - 1 + q;
            const int fl = ((xx < 0 || xx >= nc) ? 1 : 0) | ((yy < 0 || yy >= nc) ? 2 : 0) |
                           ((zz < 0 || zz >= nc) ? 4 : 0);
            const int cell = (wrap_cell(zz, nc) * nc + wrap_cell(yy, nc)) * nc + wrap_cell(xx, nc);
            const int a = p.cell_start[cell];
            cnt = p.cell_start[cell + 1] - a;
            s.slot[t] = a;
            s.flag[t] = fl;
        }
        // workgroup exclusive scan of cnt
        const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
        const int inc = wave_scan_incl(cnt);
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
    if (threadIdx.x == 0) {
        s.off[s.ntab] = carry;
        // staged column q holds cell x = cx0 - 1 + q (mod nc); along a staged row
        // the slots run on from cell to cell except where x wraps from nc - 1 to
        // 0, at q = 1 - cx0 (mod nc), at most twice in the kx + 2 columns
        int q1 = (1 - g.cx0) % nc;
        q1 = q1 <= 0 ? q1 + nc : q1;
        s.scan[0] = q1 <= g.kx + 1 ? q1 : s.stride;
        s.scan[1] = q1 + nc <= g.kx + 1 ? q1 + nc : s.stride;
    }
    s.total = carry;
    s.fits = carry < s.cap;
    __syncthreads();
    // home rows r = (c - 1) ky + (b - 1): the prefix of their home atoms (one wave,
    // a row per lane, at most 64 rows)
    if (threadIdx.x < kWave) {
        const int r = threadIdx.x;
        int cnt = 0;
        if (r < s.nhr) {
            const int b = 1 + r % g.ky, c = 1 + r / g.ky;
            const int t0 = (c * s.rows_y + b) * s.stride;
            cnt = s.off[t0 + g.kx + 1] - s.off[t0 + 1];
        }
        const int inc = wave_scan_incl(cnt);
        if (r < s.nhr) s.hp[r + 1] = inc;
        if (r == 0) s.hp[0] = 0;
    }
    __syncthreads();
}

// First staged cell t of the run of slot-contiguous cells holding staged
// entry k (k < total): its staged row by a binary search over the row starts
// (off of each row's first cell, monotone; an empty row shares its start with
// the next one and is passed over), then the wrap break(s) of that row.  The
// slot of entry k is then s.slot[t] + (k - s.off[t]).
__device__ __forceinline__ int staged_run(const Stage& s, int k)
{
    int lo = 0, hi = s.nrows - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (k >= s.off[mid * s.stride])
            lo = mid;
        else
            hi = mid - 1;
    }
    const int t0 = lo * s.stride, qb0 = s.scan[0], qb1 = s.scan[1];
    int t = t0;
    if (k >= s.off[t0 + qb0]) t = t0 + qb0;
    if (k >= s.off[t0 + qb1]) t = t0 + qb1;
    return t;
}

// Positions of the staged atoms into LDS (when they fit), plus the sentinel;
// with kAux also the vector (vx, vy, vz) of each staged atom (zero for the
// sentinel).  Each thread takes entries tid, tid + blockDim, ... four at a
// time, so that several loads are in flight per thread.  No barrier: the
// caller syncs.
//
// kShift (grids of at least 5 cells per side): every staged cell that wraps
// is staged as its periodic image next to the tile, shifted by -L on the low
// side of an axis (staged column 0, row b = 0 or c = 0) and +L on the high
// side, so that the raw difference of a home atom and any staged partner is
// already the minimum image and the pair loop needs no image rule.
template <bool kAux, bool kShift = false>
__device__ __forceinline__ void stage_atoms(const KParams& p, const Stage& s, const double* vx,
                                            const double* vy, const double* vz)
{
    if (!s.fits) return;
    constexpr int U = 4;
    const bool shift = kShift && p.nc >= 5;
    for (int k0 = threadIdx.x; k0 < s.total; k0 += U * blockDim.x) {
        double px[U], py[U], pz[U], qx[U], qy[U], qz[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * blockDim.x;
            if (k < s.total) {
                const int t = staged_run(s, k);
                const int j = atom_at(p, s.slot[t] + (k - s.off[t]));
                px[u] = p.x[j];
                py[u] = p.y[j];
                pz[u] = p.z[j];
                const int fl = shift ? s.flag[t] : 0;
                if (fl) {
                    const int row = t / s.stride, q = t - row * s.stride;
                    const int c = row / s.rows_y, b = row - c * s.rows_y;
                    if (fl & 1) px[u] += q == 0 ? -p.L : p.L;
                    if (fl & 2) py[u] += b == 0 ? -p.L : p.L;
                    if (fl & 4) pz[u] += c == 0 ? -p.L : p.L;
                }
                if (kAux) {
                    qx[u] = vx[j];
                    qy[u] = vy[j];
                    qz[u] = vz[j];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * blockDim.x;
            if (k < s.total) {
                s.p3[3 * k] = px[u];
                s.p3[3 * k + 1] = py[u];
                s.p3[3 * k + 2] = pz[u];
                if (kAux) {
                    s.a3[3 * k] = qx[u];
                    s.a3[3 * k + 1] = qy[u];
                    s.a3[3 * k + 2] = qz[u];
                }
            }
        }
    }
    if (threadIdx.x == 0) {
        s.p3[3 * s.total] = kSentinel;
        s.p3[3 * s.total + 1] = kSentinel;
        s.p3[3 * s.total + 2] = kSentinel;
        if (kAux) {
            s.a3[3 * s.total] = 0.0;
            s.a3[3 * s.total + 1] = 0.0;
            s.a3[3 * s.total + 2] = 0.0;
        }
    }
}

__device__ __forceinline__ void stage_positions(const KParams& p, const Stage& s)
{
    stage_atoms<false>(p, s, nullptr, nullptr, nullptr);
}

// Staged positions as periodic images next to the tile (see stage_atoms);
// pair loops over them take image mode staged_image_mode.
__device__ __forceinline__ void stage_positions_imaged(const KParams& p, const Stage& s)
{
    stage_atoms<false, true>(p, s, nullptr, nullptr, nullptr);
}

// Atom (storage slot) of staged entry e.
__device__ __forceinline__ int staged_slot(const KParams& p, const Stage& s, int e)
{
    const int t = staged_run(s, e);
    return atom_at(p, s.slot[t] + (e - s.off[t]));
}

// Minimum image of a staged pair.  kImage: 0 -- no wrap anywhere in the
// tile, or the wrapped cells staged as shifted images: the raw difference is
// the minimum image; 1 -- at least 5 cells per side: the raw
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

// The image rule over positions staged by stage_positions_imaged: none when
// they are in LDS (wrapped cells are already shifted), the list's wrap bits
// when the partners are read from global memory.
__device__ __forceinline__ int staged_image_mode(const KParams& p, const Stage& s, bool interior)
{
    return image_mode(p, interior || s.fits);
}

// Home atoms of a tile: the kx cells a = 1..kx of every home row (b, c),
// 1 <= b <= ky, 1 <= c <= kz, numbered h = 0 .. home_count - 1 row by row
// (home row r = (c - 1) ky + (b - 1)); each row's atoms are contiguous in LDS
// and in the cell-ordered slots.
__device__ __forceinline__ int home_count(const Stage& s) { return s.hp[s.nhr]; }

// Staged cell (column 1) of home row r.
__device__ __forceinline__ int home_row_cell(const Stage& s, int r)
{
    const int b = 1 + r % s.ky, c = 1 + r / s.ky;
    return (c * s.rows_y + b) * s.stride + 1;
}

// Home atom h: its LDS entry e, its cell-ordered slot position pos (the
// atom is atom_at(p, pos)) and the staged cell of column 1 of its row.
__device__ __forceinline__ void home_atom(const Stage& s, int h, int& e, int& pos, int& t1)
{
    int lo = 0, hi = s.nhr - 1;
    while (lo < hi) {  // the last row whose prefix is <= h (empty rows passed over)
        const int mid = (lo + hi + 1) >> 1;
        if (h >= s.hp[mid])
            lo = mid;
        else
            hi = mid - 1;
    }
    t1 = home_row_cell(s, lo);
    const int d = h - s.hp[lo];
    e = s.off[t1] + d;
    pos = s.slot[t1] + d;
}

__device__ __forceinline__ void home_atom(const Stage& s, int h, int& e, int& pos)
{
    int t1;
    home_atom(s, h, e, pos, t1);
}

// True when no staged cell of the tile wraps (and the grid has >= 5 cells).
__device__ __forceinline__ bool tile_interior(const KParams& p, const Tile& g)
{
    return p.nc >= 5 && g.cx0 >= 1 && g.cx0 + g.kx <= p.nc - 1 && g.cy0 >= 1 &&
           g.cy0 + g.ky <= p.nc - 1 && g.cz0 >= 1 && g.cz0 + g.kz <= p.nc - 1;
}

// ---- walking one home atom's list ----
//
// The pair operation `op(dx, dy, dz, r2, e, j)` gets the minimum-image
// separation home - partner, its squared length, the partner's staged
// index e and, when the tile's atoms did not fit in LDS, its storage slot j
// (-1 otherwise).  It applies its own cutoff.

// The 4 entries of one chunk.  kMask = false: partners from LDS, padded
// entries point at the sentinel atom, nothing needs masking (wrap-bit image
// modes only).  kMask = true: entries past the list are masked; with
// kFits = false the partners come from global memory.
template <int kImage, bool kFits, bool kMask, class Op>
__device__ __forceinline__ void chunk_pairs(const KParams& p, const Stage& s, uint64_t ch,
                                            int mbase, int cnt, double xi, double yi, double zi,
                                            Op& op)
{
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
        const uint32_t v = (uint32_t)(ch >> (16 * k)) & 0xffffu;
        const bool valid = !kMask || mbase + k < cnt;
        int e = (int)(v & kEntryMask);
        double xj, yj, zj;
        int j = -1;
        if (kFits) {
            if (kMask) e = valid ? e : 0;
            lds_xyz(s.p3, e, xj, yj, zj);
        } else {
            j = staged_slot(p, s, valid && e < s.total ? e : 0);
            xj = p.x[j];
            yj = p.y[j];
            zj = p.z[j];
        }
        double dx = xi - xj, dy = yi - yj, dz = zi - zj;
        image<kImage>(p, (int)(v >> kEntryBits), dx, dy, dz);
        const double r2 = dist2(dx, dy, dz);
        if (valid) op(dx, dy, dz, r2, e, j);
    }
}

// Chunks c = sub, sub+LANES, ... of one home atom's list, each loaded one
// step ahead of its use.  The first one is loaded whether or not the list
// reaches it (row sub exists when it is inside the cap / 4 + 1 allocated
// rows), so that its load does not wait for the count.
template <int LANES, int kImage, bool kFits, bool kMask, class Op>
__device__ __forceinline__ void walk_list(const KParams& p, const Stage& s, int slot_i, int sub,
                                          int cnt, double xi, double yi, double zi, Op& op)
{
    const uint64_t* col = p.nl64 + slot_i;
    int c = sub;
    uint64_t next = c <= p.cap / kChunk ? col[(int64_t)c * p.npad] : 0;
    const int nchunk = (cnt + kChunk - 1) / kChunk;
    while (c < nchunk) {
        const uint64_t ch = next;
        const int cn = c + LANES;
        if (cn < nchunk) next = col[(int64_t)cn * p.npad];
        chunk_pairs<kImage, kFits, kMask>(p, s, ch, c * kChunk, cnt, xi, yi, zi, op);
        c = cn;
    }
}

// The list of one home atom, with the image rule of its tile (mode, see
// image_mode) and the LDS or global partner path.
template <int LANES, class Op>
__device__ __forceinline__ void walk_home(const KParams& p, const Stage& s, int mode, int slot_i,
                                          int sub, int cnt, double xi, double yi, double zi,
                                          Op& op)
{
    if (!s.fits) {
        if (mode == 2)
            walk_list<LANES, 2, false, true>(p, s, slot_i, sub, cnt, xi, yi, zi, op);
        else
            walk_list<LANES, 1, false, true>(p, s, slot_i, sub, cnt, xi, yi, zi, op);
    } else if (mode == 0) {
        walk_list<LANES, 0, true, false>(p, s, slot_i, sub, cnt, xi, yi, zi, op);
    } else if (mode == 1) {
        walk_list<LANES, 1, true, false>(p, s, slot_i, sub, cnt, xi, yi, zi, op);
    } else {
        walk_list<LANES, 2, true, true>(p, s, slot_i, sub, cnt, xi, yi, zi, op);
    }
}

// Position of the home atom at LDS entry e and storage slot slot_i (LDS when
// staged).
__device__ __forceinline__ void home_position(const KParams& p, const Stage& s, int e,
                                              int slot_i, double& xi, double& yi, double& zi)
{
    if (s.fits) {
        lds_xyz(s.p3, e, xi, yi, zi);
    } else {
        xi = p.x[slot_i];
        yi = p.y[slot_i];
        zi = p.z[slot_i];
    }
}

// DPP lane moves: lane i of each quad takes lane i ^ 1 or i ^ 2 of the quad;
// the half-row mirror gives lane i of each group of 8 lane 7 - i.
constexpr int kDppQuadXor1 = 0xB1;   // quad_perm(1, 0, 3, 2)
constexpr int kDppQuadXor2 = 0x4E;   // quad_perm(2, 3, 0, 1)
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;  // lane i of each row of 16 takes lane 15 - i

template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move(T v)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        const int b = __builtin_bit_cast(int, v);
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, b, CTRL, 0xF, 0xF, false));
    } else {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo =
            (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32),
                                                                  CTRL, 0xF, 0xF, false);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

// Sum over aligned groups of LANES lanes (1, 2, 4, 8, 16 or 32); every lane
// of a group gets the group's sum.  The lane exchanges are DPP moves on the VALU
// (a shuffle would go through LDS, which the pair loops keep busy).  Every
// lane of the wave must be active.
template <int LANES, typename T>
__device__ __forceinline__ T lane_group_sum(T v)
{
    static_assert(LANES == 1 || LANES == 2 || LANES == 4 || LANES == 8 || LANES == 16 ||
                      LANES == 32,
                  "lanes per atom");
    if constexpr (LANES == 32) v += __shfl_xor(v, 16, kWave);  // across the two rows
    if constexpr (LANES >= 16) v += dpp_move<kDppRowMirror>(v);
    if constexpr (LANES >= 8) v += dpp_move<kDppHalfMirror>(v);
    if constexpr (LANES >= 4) v += dpp_move<kDppQuadXor2>(v);
    if constexpr (LANES >= 2) v += dpp_move<kDppQuadXor1>(v);
    return v;
}

}  // namespace md
