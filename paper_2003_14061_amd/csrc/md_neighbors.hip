// md_neighbors.hip -- step N5 of section 2.3: the neighbor matrix.
//
// One workgroup per tile (md_tiles.h) stages the tile's 27-cell
// neighborhoods in LDS.  A home atom's candidates are the three cells
// dx = -1, 0, +1 of each of the 9 staged rows next to its cell (dz, dy each
// -1, 0, +1, dz slowest), every cell in ascending permanent id; its list
// keeps them in that canonical order.  An entry is kept when the minimum-image squared
// separation is below (r_cut + skin)^2 (dx*dx, then two fused
// multiply-adds) and it is not the atom itself.  Two ways to walk them:
//
//   lanes (default)  one lane per home atom walks its 27 cells; entries are
//                    packed four to a chunk in a register and stored a
//                    chunk at a time
//   cell waves       one wave per home cell spreads the cell's candidates
//                    over its 64 lanes, 64 per round; for each home atom a
//                    ballot and a prefix count place the hits
//
// The half list (for the Newton's-third-law force pass) keeps a candidate
// only if it comes after the home atom in cell order (cell index, then
// permanent id).  That order is the order of the cell-ordered slots:
// candidate e of staged cell t sits at slot[t] + (e - off[t]), and so does the
// home atom, so the test is one integer comparison, and a
// staged cell whose last slot is not past the home atom's is skipped whole.
//
// Storage follows the paper's W (section 2.3): row m holds the m-th
// neighbor of every atom, so a wave of the force pass reads consecutive
// atoms' entries at consecutive addresses.  Entries are 16 bits (staged
// index + wrap bits), four to an 8-byte chunk: chunk c of slot k sits at
// 8-byte index c * n_pad + k.
#include "md_tiles.h"

namespace md {

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// LDS bytes of the list build: the staged tile.
size_t nl_lds_bytes(const KParams& p) { return stage_bytes(p, p.scap); }

// Staged cell of column a - 1 in the row (dz, dy) = (sg / 3 - 1, sg % 3 - 1)
// next to home cell home_t (at column a): the first cell of window sg.
__device__ __forceinline__ int window_cell(const Stage& s, int home_t, int sg)
{
    const int dz = (sg >= 3 ? 1 : 0) + (sg >= 6 ? 1 : 0) - 1, dy = sg - 3 * (dz + 1) - 1;
    return home_t - 1 + (dz * s.rows_y + dy) * s.stride;
}

// Staged cell of home cell hc (0 .. kx ky kz - 1, x fastest).
__device__ __forceinline__ int home_cell(const Stage& s, int hc)
{
    const int a = 1 + hc % s.kx, r = hc / s.kx;
    return home_row_cell(s, r) + (a - 1);
}

// The lists of home cell hc's atoms, by one wave; wmax: the longest list of
// this lane's home atoms so far.  The candidates (the 9 windows of three cells
// next to it, concatenated, in canonical order) are taken kRounds x 64 at a
// time: lane l holds candidate k0 + 64 r + l (position, wrap bits, encoded
// entry) in registers.  Each home atom hh in turn is broadcast from lane hh
// (readlane) and tested against the block; for round r the hit ballot places
// the hits: a hit lane's entry goes to list position m_hh + (hits of lower
// lanes), m_hh being hh's running list length, kept in a scalar register while
// hh is tested and in lane hh of a vector register between blocks.  Lanes past
// the candidates read the home cell's first atom (e = hb) and never hit.
template <int kImage, bool kHalf, bool kFits, bool kCopy, int kRounds, bool kFull>
__device__ __forceinline__ void nl_home_cell(const KParams& p, const Stage& s, int hc, bool small,
                                             int& wmax)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int home_t = home_cell(s, hc);
    // table values are the same in every lane: keep them in scalar registers
    const int hb = uniform(s.off[home_t]), he = uniform(s.off[home_t + 1]);
    const int hslot0 = uniform(s.slot[home_t]);
    int wp[10];  // candidates before each window (the windows' own cells follow per lane)
    wp[0] = 0;
#pragma unroll
    for (int sg = 0; sg < 9; ++sg) {
        const int tw = window_cell(s, home_t, sg);
        wp[sg + 1] = wp[sg] + (uniform(s.off[tw + 3]) - uniform(s.off[tw]));
    }
    const int ncand = wp[9];
    const uint32_t cap = (uint32_t)p.cap;  // a multiple of 4
    uint16_t* nl16 = reinterpret_cast<uint16_t*>(p.nl64);
    const uint32_t npad4 = 4u * (uint32_t)p.npad;  // 16-bit entries per chunk row
    // small (the list within 32-bit byte offsets, rows within 24-bit products,
    // always so without kFull): hits go out as buffer stores, the list's base
    // in a resource, the home atom's chunk column as the scalar offset and row
    // and column of the entry as the 32-bit lane offset (no 64-bit address
    // arithmetic per hit).  With kFull the choice is a uniform branch at the
    // store (a second copy of the loop would raise the register count).
    const uint32_t rowb = 8u * (uint32_t)p.npad;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(p.nl64, 0, -1, kBufferWord3);
    for (int h0 = hb; h0 < he; h0 += kWave) {
        const int nhs = he - h0 < kWave ? he - h0 : kWave;
        const bool home_lane = lane < nhs;
        const int hl = h0 + (home_lane ? lane : 0);
        const int slot_l = atom_at(p, hslot0 + (hl - hb));
        double hx, hy, hz;
        if (kFits) {
            lds_xyz(s.p3, hl, hx, hy, hz);
        } else {
            hx = p.x[slot_l];
            hy = p.y[slot_l];
            hz = p.z[slot_l];
        }
        int mreg = 0;  // lane hh: home atom hh's list length so far
        for (int k0 = 0; k0 < ncand; k0 += kRounds * kWave) {
            double cx[kRounds], cy[kRounds], cz[kRounds];
            int ce[kRounds], cfl[kRounds], cpos[kRounds];
            uint16_t cenc[kRounds];
#pragma unroll
            for (int r = 0; r < kRounds; ++r) {
                const int k = k0 + r * kWave + lane;
                const bool valid = k < ncand;
                int sg = 0, pre = 0;
#pragma unroll
                for (int j = 1; j < 9; ++j) {
                    sg += k >= wp[j] ? 1 : 0;
                    pre = k >= wp[j] ? wp[j] : pre;
                }
                const int t0 = window_cell(s, home_t, sg);
                const int e = valid ? s.off[t0] + (k - pre) : hb;
                const int w = (e >= s.off[t0 + 1] ? 1 : 0) + (e >= s.off[t0 + 2] ? 1 : 0);
                const int t = valid ? t0 + w : home_t;
                // lanes past the candidates: index -1 (never the home atom) and a
                // NaN position (never near, under any image rule)
                ce[r] = valid ? e : -1;
                cfl[r] = s.flag[t];
                cpos[r] = s.slot[t] + (e - s.off[t]);
                cenc[r] = (uint16_t)((uint32_t)e | ((uint32_t)cfl[r] << kEntryBits));
                if (kFits) {
                    lds_xyz(s.p3, e, cx[r], cy[r], cz[r]);
                } else {
                    const int j = atom_at(p, cpos[r]);
                    cx[r] = p.x[j];
                    cy[r] = p.y[j];
                    cz[r] = p.z[j];
                }
                if (!valid) cx[r] = __builtin_nan("");
            }
            for (int hh = 0; hh < nhs; ++hh) {
                const int eh = h0 + hh;
                const int pos_i = hslot0 + (eh - hb);
                // the home atom's position: with the tile staged, one LDS read that
                // the whole wave shares (its address is the same in every lane), which
                // measured 11% faster per build than six readlanes
                double xi, yi, zi;
                if (kFits) {
                    lds_xyz(s.p3, eh, xi, yi, zi);
                } else {
                    xi = readlane_f64(hx, hh);
                    yi = readlane_f64(hy, hh);
                    zi = readlane_f64(hz, hh);
                }
                const uint32_t slot4 = 4u * (uint32_t)__builtin_amdgcn_readlane(slot_l, hh);
                uint32_t m_h = (uint32_t)__builtin_amdgcn_readlane(mreg, hh);
                // the tests of all rounds first (independent), then the stores
                bool hit[kRounds];
                uint64_t mk[kRounds];
#pragma unroll
                for (int r = 0; r < kRounds; ++r) {
                    double dx = xi - cx[r], dy = yi - cy[r], dz = zi - cz[r];
                    image<kImage>(p, cfl[r], dx, dy, dz);
                    // each condition balloted on its own (the compare results are
                    // the lane masks; a ballot of their conjunction would turn
                    // them into a vector and back)
                    const bool near = dist2(dx, dy, dz) < p.rl2;
                    const bool other = ce[r] != eh;
                    const bool later = !kHalf || cpos[r] > pos_i;
                    mk[r] = __builtin_amdgcn_ballot_w64(near) & __builtin_amdgcn_ballot_w64(other);
                    if (kHalf) mk[r] &= __builtin_amdgcn_ballot_w64(later);
                    hit[r] = near & other & later;
                }
#pragma unroll
                for (int r = 0; r < kRounds; ++r) {
                    if (hit[r]) {
                        // position m_h plus the hits of lower lanes; past the
                        // capacity into the spare chunk row (counted, not kept)
                        uint32_t m = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(mk[r] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk[r], m_h));
                        m = m < cap ? m : cap;
                        if (!kFull || small) {
                            // row (m >> 2) of rowb bytes, entry m & 3 of the chunk:
                            // 2 m + (m >> 2) (rowb - 8), one 24-bit multiply-add
                            uint32_t off;
                            asm("v_mad_u32_u24 %0, %1, %2, %3"
                                : "=v"(off)
                                : "v"(m >> 2), "s"(rowb - 8u), "v"(2u * m));
                            __builtin_amdgcn_raw_buffer_store_b16(cenc[r], rsrc, (int)off,
                                                                  (int)(2u * slot4), 0);
                        } else {
                            nl16[(size_t)(m >> 2) * npad4 + ((m & 3u) | slot4)] = cenc[r];
                        }
                    }
                    m_h += (uint32_t)__popcll(mk[r]);
                }
                mreg = lane == hh ? (int)m_h : mreg;
            }
        }
        // lengths, sentinel padding of the last chunk, displacement references
        if (home_lane) {
            const int stored = mreg < (int)cap ? mreg : (int)cap;
            p.nl_count[slot_l] = stored;
            uint16_t* base = nl16 + (int64_t)slot_l * kChunk;
            for (int mm = stored; mm % kChunk != 0; ++mm)
                base[(int64_t)(mm / kChunk) * npad4 + mm % kChunk] = (uint16_t)s.total;
            p.xr[slot_l] = hx;
            p.yr[slot_l] = hy;
            p.zr[slot_l] = hz;
            copy_home<kCopy>(p, slot_l);
        }
        wmax = home_lane && mreg > wmax ? mreg : wmax;
    }
}

// True when home cell hc (0 .. kx ky kz - 1, x fastest) of tile g lies on a
// periodic boundary: some of its 26 neighbor cells wrap.
__device__ __forceinline__ bool home_wraps(const KParams& p, const Tile& g, int hc)
{
    const int a = hc % g.kx, r = hc / g.kx, b = r % g.ky, c = r / g.ky;
    const int xx = g.cx0 + a, yy = g.cy0 + b, zz = g.cz0 + c, e = p.nc - 1;
    return xx == 0 || xx == e || yy == 0 || yy == e || zz == 0 || zz == e;
}

// Home cell of row cell t1 (column 1 of its home row) holding staged entry e.
__device__ __forceinline__ int home_column_cell(const Stage& s, int t1, int e)
{
    int lo = 0, hi = s.kx - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.off[t1 + mid] <= e)
            lo = mid;
        else
            hi = mid - 1;
    }
    return t1 + lo;
}

// The list of home atom h, by one lane.  Returns the number of entries found
// (beyond the capacity: overflow).
template <int kImage, bool kFits, bool kHalf, bool kCopy>
__device__ __forceinline__ int nl_home_atom(const KParams& p, const Stage& s, int h)
{
    int e_self, pos_i, t1;
    home_atom(s, h, e_self, pos_i, t1);
    const int home_t = home_column_cell(s, t1, e_self);
    const int slot_i = atom_at(p, pos_i);
    double xi, yi, zi;
    if (kFits) {
        lds_xyz(s.p3, e_self, xi, yi, zi);
    } else {
        xi = p.x[slot_i];
        yi = p.y[slot_i];
        zi = p.z[slot_i];
    }
    const uint32_t cap = (uint32_t)p.cap;  // a multiple of 4
    uint64_t* col = p.nl64 + slot_i;
    uint64_t chunk = 0;
    uint32_t m = 0;
    // An interior tile (kImage 0) has no wrapped cell: the three cells of a
    // window are consecutive cells of one row, contiguous both among the staged
    // atoms and in the cell-ordered slots, with no wrap bits, so each window is
    // walked as one run (9 loops instead of 27).
    constexpr int kRuns = kImage == 0 ? 1 : 3;
    for (int sg = 0; sg < 9; ++sg) {
        const int tw = window_cell(s, home_t, sg);
#pragma unroll
        for (int w = 0; w < kRuns; ++w) {
            const int t = tw + w;
            const int eb = s.off[t], ee = s.off[t + (kImage == 0 ? 3 : 1)];
            const int fl = kImage == 0 ? 0 : s.flag[t];
            const int tslot = kFits && !kHalf ? 0 : s.slot[t];
            const uint64_t tag = (uint64_t)fl << kEntryBits;
            if (kHalf && tslot + (ee - eb) <= pos_i) continue;
            for (int e = eb; e < ee; ++e) {
                double xj, yj, zj;
                if (kFits) {
                    lds_xyz(s.p3, e, xj, yj, zj);
                } else {
                    const int j = atom_at(p, tslot + (e - eb));
                    xj = p.x[j];
                    yj = p.y[j];
                    zj = p.z[j];
                }
                double dx = xi - xj, dy = yi - yj, dz = zi - zj;
                image<kImage>(p, fl, dx, dy, dz);
                const bool later = !kHalf || tslot + (e - eb) > pos_i;
                if (later && dist2(dx, dy, dz) < p.rl2 && e != e_self) {
                    if (m < cap) {
                        chunk |= ((uint64_t)e | tag) << (16 * (m % kChunk));
                        if (m % kChunk == kChunk - 1) {
                            col[(int64_t)(m / kChunk) * p.npad] = chunk;
                            chunk = 0;
                        }
                    }
                    ++m;
                }
            }
        }
    }
    const uint32_t stored = m < cap ? m : cap;
    if (stored % kChunk != 0) {  // pad the last chunk with the sentinel
        for (uint32_t mm = stored % kChunk; mm < kChunk; ++mm)
            chunk |= (uint64_t)s.total << (16 * mm);
        col[(int64_t)(stored / kChunk) * p.npad] = chunk;
    }
    p.nl_count[slot_i] = (int)stored;
    p.xr[slot_i] = xi;
    p.yr[slot_i] = yi;
    p.zr[slot_i] = zi;
    copy_home<kCopy>(p, slot_i);
    return (int)m;
}

template <int kImage, bool kFits, bool kHalf, bool kCopy>
__device__ __forceinline__ void nl_lanes(const KParams& p, const Stage& s, int& wmax)
{
    const int nh = home_count(s);
    for (int h = threadIdx.x; h < nh; h += blockDim.x) {
        const int m = nl_home_atom<kImage, kFits, kHalf, kCopy>(p, s, h);
        wmax = m > wmax ? m : wmax;
    }
}

// One tile's lists (every thread of the workgroup calls it); wmax: the longest
// list this thread has seen (its wave's, in the cell-wave build).  kFull: the
// image rule of grids under 5 cells per side (mode 2) and list stores beyond
// 32-bit offsets are compiled in; a kernel without them serves only grids of 5
// cells per side or more whose lists fit the buffer stores, and holds fewer
// registers.
template <int kMethod, bool kHalf, bool kCopy, bool kFull>
__device__ __forceinline__ void nl_tile(const KParams& p, int t, char* smem, int& wmax)
{
    const Tile g = tile_of(p, t);
    Stage s = stage_layout(p, smem);
    stage_tables(p, g, s);
    if (s.total >= kMaxStaged) {
        // the 13-bit entry cannot address this tile (and its sentinel): report it
        // as an overflow
        const int nh = home_count(s);
        for (int h = threadIdx.x; h < nh; h += blockDim.x) {
            int e, pos;
            home_atom(s, h, e, pos);
            p.nl_count[atom_at(p, pos)] = 0;
            copy_home<kCopy>(p, atom_at(p, pos));
        }
        if (threadIdx.x == 0) atomicOr(&p.dev->flags, (int)MD_FLAG_NL_OVERFLOW);
        return;
    }
    stage_positions(p, s);
    __syncthreads();
    const int mode = image_mode(p, tile_interior(p, g));
    if (kMethod == MD_NL_LANES) {
        if (kFull && mode == 2) {
            if (s.fits)
                nl_lanes<2, true, kHalf, kCopy>(p, s, wmax);
            else
                nl_lanes<2, false, kHalf, kCopy>(p, s, wmax);
        } else if (!s.fits) {
            nl_lanes<1, false, kHalf, kCopy>(p, s, wmax);
        } else if (mode == 0) {
            nl_lanes<0, true, kHalf, kCopy>(p, s, wmax);
        } else {
            nl_lanes<1, true, kHalf, kCopy>(p, s, wmax);
        }
        return;
    }
    const int wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int ncells = g.kx * g.ky * g.kz;
    const bool small = nl_small(p);
    // Home cells next to a periodic boundary (real index 0 or nc - 1 on some
    // axis) have wrapped candidates and take the image rule; the other home
    // cells of a boundary tile have none and take the interior path.  The rare
    // tiles that do not fit in LDS, and grids under 5 cells per side, take one
    // round of 64 candidates at a time: those paths then hold fewer registers
    // than the common ones (the kernel's register count is that of its largest
    // path), which keeps six waves per SIMD.
    for (int hc = wid; hc < ncells; hc += nw) {
        if (kFull && mode == 2) {
            if (s.fits)
                nl_home_cell<2, kHalf, true, kCopy, 1, kFull>(p, s, hc, small, wmax);
            else
                nl_home_cell<2, kHalf, false, kCopy, 1, kFull>(p, s, hc, small, wmax);
        } else if (!s.fits) {
            nl_home_cell<1, kHalf, false, kCopy, 1, kFull>(p, s, hc, small, wmax);
        } else if (mode == 0 || !home_wraps(p, g, hc)) {
            nl_home_cell<0, kHalf, true, kCopy, kNlRounds, kFull>(p, s, hc, small, wmax);
        } else {
            nl_home_cell<1, kHalf, true, kCopy, kNlRounds, kFull>(p, s, hc, small, wmax);
        }
    }
}

// The list build, gated by the rebuild flag.  Workgroups take tiles
// v = id, id + n, ... (grid rule G_NL, one tile each at present: a capped grid
// looping over tiles idles less per launch but measured slower per rebuild,
// from the uneven tile counts of the last wave of workgroups); tile v keeps
// the XCD-aware order (v mod 8 is the workgroup's XCD when n is a multiple
// of 8).
// At most 80 VGPRs: six waves per SIMD, which the LDS of the dense LJ tiles
// (three workgroups of eight waves per CU) allows.
template <class B, int kMethod, bool kHalf, bool kCopy, bool kFull>
__global__ __attribute__((amdgpu_waves_per_eu(6))) void k_nl_tiles(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch_gated(G_NL, force, wg, p)) return;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const KParams q = kCopy ? scratch_view(p) : p;
    int wmax = 0;
    for (int v = wg.id; v < q.n_tiles; v += wg.n) {
        nl_tile<kMethod, kHalf, kCopy, kFull>(q, xcd_tile(v, q.n_tiles), smem, wmax);
        __syncthreads();  // the next tile reuses the LDS
    }
    // the longest list: one global atomic per workgroup
    const int mmax = workgroup_max(wmax);
    if (threadIdx.x == 0 && mmax > 0) {
        atomicMax(&q.dev->max_nl, mmax);
        if (mmax > q.cap) atomicOr(&q.dev->flags, (int)MD_FLAG_NL_OVERFLOW);
    }
}

// Decode the list into global slots: out[m * n_pad + k] for m < count[k],
// -1 elsewhere.
__global__ void k_nl_export(KParams p, int32_t* out)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const Tile g = tile_of(p, xcd_tile(blockIdx.x, gridDim.x));
    Stage s = stage_layout(p, smem);
    stage_tables(p, g, s);
    const int nh = home_count(s);
    for (int h = threadIdx.x; h < nh; h += blockDim.x) {
        int e, pos;
        home_atom(s, h, e, pos);
        const int k = atom_at(p, pos), cnt = p.nl_count[k];
        for (int m = 0; m < p.cap; ++m) {
            int v = -1;
            if (m < cnt) {
                const uint64_t ch = p.nl64[(int64_t)(m / kChunk) * p.npad + k];
                const int e = (int)((ch >> (16 * (m % kChunk))) & kEntryMask);
                v = e < s.total ? staged_slot(p, s, e) : -2;
            }
            out[(int64_t)m * p.npad + k] = v;
        }
    }
}

template <class B, bool kHalf, bool kCopy, bool kFull>
static void neighbors_seq(const B& b, const LaunchShape& sh, int force, hipStream_t s)
{
    const dim3 g(sh.grid[G_NL]), t(sh.nl_block);
    if (sh.nl_method == MD_NL_CELL_WAVES)
        hipLaunchKernelGGL((k_nl_tiles<B, MD_NL_CELL_WAVES, kHalf, kCopy, kFull>), g, t, sh.nl_lds,
                           s, b, force);
    else
        hipLaunchKernelGGL((k_nl_tiles<B, MD_NL_LANES, kHalf, kCopy, kFull>), g, t, sh.nl_lds, s,
                           b, force);
}

template <class B, bool kHalf, bool kCopy>
static void neighbors_seq(const B& b, const LaunchShape& sh, int force, hipStream_t s)
{
    if (sh.nl_full)
        neighbors_seq<B, kHalf, kCopy, true>(b, sh, force, s);
    else
        neighbors_seq<B, kHalf, kCopy, false>(b, sh, force, s);
}

template <class B>
static void neighbors_seq(const B& b, const LaunchShape& sh, int flags, hipStream_t s)
{
    const int force = flags & 1;
    const bool copy = (flags & kFoldCopy) && sh.reorder;
    if (sh.newton3)
        copy ? neighbors_seq<B, true, true>(b, sh, force, s)
             : neighbors_seq<B, true, false>(b, sh, force, s);
    else
        copy ? neighbors_seq<B, false, true>(b, sh, force, s)
             : neighbors_seq<B, false, false>(b, sh, force, s);
}

void launch_neighbors(const KParams& p, int force, hipStream_t s)
{
    neighbors_seq(Single{p}, shape_of(p), force, s);
}

void launch_neighbors(const Batch& b, const LaunchShape& sh, int force, hipStream_t s)
{
    neighbors_seq(b, sh, force, s);
}

void launch_nl_export(const KParams& p, int32_t* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_nl_export, dim3(p.n_tiles), dim3(p.nl_block),
                       nl_lds_bytes(p), s, p, out);
}

}  // namespace md
