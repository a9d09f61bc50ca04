// md_neighbors.hip -- step N5 of section 2.3: the neighbor matrix.
//
// One workgroup per tile (md_tiles.h) stages the tile's 27-cell
// neighborhoods in LDS.  Each wave then takes one home cell at a time and
// spreads that cell's candidates -- the three cells dx = -1, 0, +1 of each
// of the 9 staged rows (dz, dy each -1, 0, +1, dz slowest), every cell in
// ascending permanent id -- across its 64 lanes, 64 candidates per round.
// For each home atom of the cell in turn, every lane tests its candidate;
// a wave ballot and a prefix count give each hit its position in the home
// atom's list, so the list comes out in the canonical candidate order.  An
// entry is kept when the minimum-image squared separation is below
// (r_cut + skin)^2 (dx*dx, then two fused multiply-adds) and it is not the
// atom itself.
//
// Storage follows the paper's W (section 2.3): row m holds the m-th
// neighbor of every atom, so a wave of the force pass reads consecutive
// atoms' entries at consecutive addresses.  Entries are 16 bits (staged
// index + wrap bits), four to an 8-byte chunk: chunk c of slot k sits at
// 8-byte index c * n_pad + k.
#include "md_tiles.h"

namespace md {

// LDS bytes of the list build: the staged tile plus per-wave list counters.
inline size_t nl_lds_bytes(const KParams& p)
{
    return stage_bytes(p.scap, p.kx_max) + sizeof(int) * (p.nl_block / kWave) * kMaxHomeSweep;
}

template <bool kFlags>
__device__ void nl_home_cell(const KParams& p, const Stage& s, int q, int* mh)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int home_t = 4 * s.stride + q;
    const int hb = s.off[home_t], he = s.off[home_t + 1];
    const int hslot0 = s.slot[home_t];
    // the 9 candidate windows (cells q-1..q+1 of every staged row), concatenated
    int wa[9], wp[10];
    wp[0] = 0;
#pragma unroll
    for (int sg = 0; sg < 9; ++sg) {
        wa[sg] = s.off[sg * s.stride + q - 1];
        wp[sg + 1] = wp[sg] + (s.off[sg * s.stride + q + 2] - wa[sg]);
    }
    const int total = wp[9];
    const uint32_t cap = (uint32_t)p.cap;
    uint16_t* nl16 = reinterpret_cast<uint16_t*>(p.nl64);
    for (int h0 = hb; h0 < he; h0 += kMaxHomeSweep) {
        const int h1 = he < h0 + kMaxHomeSweep ? he : h0 + kMaxHomeSweep;
        for (int h = h0 + lane; h < h1; h += kWave) mh[h - h0] = 0;
        for (int k0 = 0; k0 < total; k0 += kWave) {
            const int k = k0 + lane;
            const bool valid = k < total;
            int sg = 0;
#pragma unroll
            for (int j = 1; j < 9; ++j) sg += k >= wp[j] ? 1 : 0;
            int a = wa[0], pre = wp[0];
#pragma unroll
            for (int j = 1; j < 9; ++j) {
                a = sg == j ? wa[j] : a;
                pre = sg == j ? wp[j] : pre;
            }
            const int e = valid ? a + (k - pre) : hb;
            // which of the window's three cells holds e, and its wrap bits
            const int t0 = sg * s.stride + q - 1;
            const int w = (e >= s.off[t0 + 1] ? 1 : 0) + (e >= s.off[t0 + 2] ? 1 : 0);
            const int fl = s.flag[t0 + w];
            double xj, yj, zj;
            if (s.fits) {
                xj = s.xs[e];
                yj = s.ys[e];
                zj = s.zs[e];
            } else {
                // lanes past the candidates read the home cell's first atom (e is
                // not inside window cell t0 + w for them)
                const int j = atom_at(p, valid ? s.slot[t0 + w] + (e - s.off[t0 + w]) : hslot0);
                xj = p.x[j];
                yj = p.y[j];
                zj = p.z[j];
            }
            const uint32_t enc = (uint32_t)e | ((uint32_t)fl << kEntryBits);
            for (int h = h0; h < h1; ++h) {
                double xi, yi, zi;
                if (s.fits) {
                    xi = s.xs[h];
                    yi = s.ys[h];
                    zi = s.zs[h];
                } else {
                    const int i = atom_at(p, hslot0 + (h - hb));
                    xi = p.x[i];
                    yi = p.y[i];
                    zi = p.z[i];
                }
                double dx = xi - xj, dy = yi - yj, dz = zi - zj;
                image<kFlags>(p, fl, dx, dy, dz);
                const bool hit = valid && dist2(dx, dy, dz) < p.rl2 && e != h;
                const uint64_t mask = __ballot(hit);
                if (mask) {
                    const int base = mh[h - h0];
                    if (hit) {
                        const uint32_t m = (uint32_t)base + __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                        if (m < cap) {
                            const int slot_i = atom_at(p, hslot0 + (h - hb));
                            nl16[((int64_t)(m / kChunk) * p.npad + slot_i) * kChunk + m % kChunk] =
                                (uint16_t)enc;
                        }
                    }
                    if (lane == 0) mh[h - h0] = base + __popcll(mask);
                }
            }
        }
        // lengths, displacement references, overflow
        int mmax = 0;
        for (int h = h0 + lane; h < h1; h += kWave) {
            const int m = mh[h - h0];
            const int slot_i = atom_at(p, hslot0 + (h - hb));
            p.nl_count[slot_i] = m < p.cap ? m : p.cap;
            double xi, yi, zi;
            if (s.fits) {
                xi = s.xs[h];
                yi = s.ys[h];
                zi = s.zs[h];
            } else {
                xi = p.x[slot_i];
                yi = p.y[slot_i];
                zi = p.z[slot_i];
            }
            p.xr[slot_i] = xi;
            p.yr[slot_i] = yi;
            p.zr[slot_i] = zi;
            mmax = m > mmax ? m : mmax;
        }
        mmax = wave_max(mmax);
        if (lane == 0 && mmax > 0) {
            atomicMax(&p.dev->max_nl, mmax);
            if (mmax > p.cap) atomicOr(&p.dev->flags, (int)MD_FLAG_NL_OVERFLOW);
        }
    }
}

__global__ void k_nl_tiles(KParams p, int force)
{
    if (!force && !p.dev->rebuild) return;
    extern __shared__ char smem[];
    const Tile g = tile_of(p, xcd_tile(blockIdx.x, gridDim.x));
    Stage s = stage_layout(p, smem);
    int* mh_all = s.scan + kWave;
    stage_tables(p, g, s);
    if (s.total > kMaxStaged) {
        // the 13-bit entry cannot address this tile: report it as an overflow
        const int nh = home_count(s);
        for (int h = threadIdx.x; h < nh; h += blockDim.x)
            p.nl_count[atom_at(p, home_first_slot(s) + h)] = 0;
        if (threadIdx.x == 0) atomicOr(&p.dev->flags, (int)MD_FLAG_NL_OVERFLOW);
        return;
    }
    stage_positions(p, s);
    const int wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
    int* mh = mh_all + wid * kMaxHomeSweep;
    const bool flags = !tile_interior(p, g);
    for (int q = 1 + wid; q <= g.kx; q += nw) {
        if (flags)
            nl_home_cell<true>(p, s, q, mh);
        else
            nl_home_cell<false>(p, s, q, mh);
    }
}

// Decode the list into global slots: out[m * n_pad + k] for m < count[k],
// -1 elsewhere.
__global__ void k_nl_export(KParams p, int32_t* out)
{
    extern __shared__ char smem[];
    const Tile g = tile_of(p, xcd_tile(blockIdx.x, gridDim.x));
    Stage s = stage_layout(p, smem);
    stage_tables(p, g, s);
    const int nh = home_count(s), slot0 = home_first_slot(s);
    for (int h = threadIdx.x; h < nh; h += blockDim.x) {
        const int k = atom_at(p, slot0 + h), cnt = p.nl_count[k];
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

void launch_neighbors(const KParams& p, int force, hipStream_t s)
{
    hipLaunchKernelGGL(k_nl_tiles, dim3(p.n_tiles), dim3(p.nl_block), nl_lds_bytes(p), s, p,
                       force);
}

void launch_nl_export(const KParams& p, int32_t* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_nl_export, dim3(p.n_tiles), dim3(p.nl_block),
                       stage_bytes(p.scap, p.kx_max), s, p, out);
}

}  // namespace md
