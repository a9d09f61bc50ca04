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
    int ntab, stride, total, cap;
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

// Ints of the table region, rounded up to 16 bytes.
__host__ __device__ __forceinline__ int stage_table_ints(int kx_max)
{
    const int ntab = 9 * (kx_max + 2);
    return (3 * ntab + 1 + kWave + 3) / 4 * 4;
}

// Dynamic LDS bytes of the staged tile: positions (and with `aux` a second
// 3-vector) of cap atoms, then the cell tables.
inline size_t stage_bytes(int cap, int kx_max, bool aux = false)
{
    return sizeof(double) * (aux ? 6 : 3) * (size_t)cap +
           sizeof(int) * (size_t)stage_table_ints(kx_max);
}

// Candidate rounds (of 64) held in registers by the cell-wave list build.
constexpr int kNlRounds = 4;

__device__ __forceinline__ Stage stage_layout(const KParams& p, char* smem, int cap, bool aux)
{
    Stage s;
    s.cap = cap;
    s.p3 = (MD_LDS double*)smem;
    s.a3 = aux ? s.p3 + 3 * cap : nullptr;
    const int ntab_max = 9 * (p.kx_max + 2);
    s.off = (MD_LDS int*)(s.p3 + (aux ? 6 : 3) * cap);
    s.slot = s.off + ntab_max + 1;
    s.flag = s.slot + ntab_max;
    s.scan = s.flag + ntab_max;
    return s;
}

__device__ __forceinline__ Stage stage_layout(const KParams& p, char* smem)
{
    return stage_layout(p, smem, p.scap, false);
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
}

// First staged cell t of the run of slot-contiguous cells holding staged
// entry k (k < total): its staged row from the 9 row starts (off of each
// row's first cell; independent LDS reads, the same address in every lane),
// then the wrap break(s) of that row.  The slot of entry k is then
// s.slot[t] + (k - s.off[t]).
__device__ __forceinline__ int staged_run(const Stage& s, int k)
{
    int sg = 0;
#pragma unroll
    for (int r = 1; r < 9; ++r) sg += k >= s.off[r * s.stride] ? 1 : 0;
    const int t0 = sg * s.stride, qb0 = s.scan[0], qb1 = s.scan[1];
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
// side of an axis (staged column 0, row y or z index -1) and +L on the high
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
                    const int sg = t / s.stride, q = t - sg * s.stride;
                    if (fl & 1) px[u] += q == 0 ? -p.L : p.L;
                    if (fl & 2) py[u] += sg % 3 == 0 ? -p.L : p.L;
                    if (fl & 4) pz[u] += sg / 3 == 0 ? -p.L : p.L;
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
// step ahead of its use.
template <int LANES, int kImage, bool kFits, bool kMask, class Op>
__device__ __forceinline__ void walk_list(const KParams& p, const Stage& s, int slot_i, int sub,
                                          int cnt, double xi, double yi, double zi, Op& op)
{
    const int nchunk = (cnt + kChunk - 1) / kChunk;
    const uint64_t* col = p.nl64 + slot_i;
    int c = sub;
    uint64_t next = c < nchunk ? col[(int64_t)c * p.npad] : 0;
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

// Position of home atom h (LDS when staged).
__device__ __forceinline__ void home_position(const KParams& p, const Stage& s, int h0, int h,
                                              int slot_i, double& xi, double& yi, double& zi)
{
    if (s.fits) {
        lds_xyz(s.p3, h0 + h, xi, yi, zi);
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
