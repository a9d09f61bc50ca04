// md_device.h -- device helpers shared by the libmd kernels.
//
// The arithmetic that decides membership (cells, neighbor list, cutoff,
// rebuild) is written so that it rounds exactly as specified in md.h:
//   minimum image   d - L*rint(d/L), with 1/L formed on the host
//   squared length  dx*dx then two fused multiply-adds
//   cell index      floor(x * (nc/L)) clamped to nc-1
//   kick / drift    v + (dt/2m)*f and x + dt*v, multiply then add
// Contraction is switched off inside those helpers so the compiler cannot
// fuse them differently.
#pragma once

#include <hip/hip_runtime.h>

#include "md_internal.h"

namespace md {

__device__ __forceinline__ double minimg(double d, double L, double invL)
{
#pragma clang fp contract(off)
    return d - L * rint(d * invL);
}

__device__ __forceinline__ double dist2(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
}

__device__ __forceinline__ double wrap(double x, double L)
{
#pragma clang fp contract(off)
    if (x >= L) {
        x -= L;
    } else if (x < 0.0) {
        x += L;
        if (x >= L) x = 0.0;
    }
    return x;
}

__device__ __forceinline__ int cell_1d(double x, double inv_w, int nc)
{
#pragma clang fp contract(off)
    int c = (int)floor(x * inv_w);
    c = c < 0 ? 0 : c;
    return c > nc - 1 ? nc - 1 : c;
}

__device__ __forceinline__ int cell_of_pos(double x, double y, double z, const KParams& p)
{
    int cx = cell_1d(x, p.inv_w, p.nc);
    int cy = cell_1d(y, p.inv_w, p.nc);
    int cz = cell_1d(z, p.inv_w, p.nc);
    return (cz * p.nc + cy) * p.nc + cx;
}

__device__ __forceinline__ int wrap_cell(int c, int nc)
{
    return c < 0 ? c + nc : (c >= nc ? c - nc : c);
}

__device__ __forceinline__ double kick(double v, double hdt, double f)
{
#pragma clang fp contract(off)
    return v + hdt * f;
}

__device__ __forceinline__ double drift(double x, double dt, double v)
{
#pragma clang fp contract(off)
    return x + dt * v;
}

// Reciprocal: hardware estimate refined by two Newton-Raphson steps
// y <- y + y(1 - a y), each roughly squaring the relative error.
__device__ __forceinline__ double recip(double a)
{
    double y = __builtin_amdgcn_rcp(a);
    double e = __builtin_fma(-a, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-a, y, 1.0);
    return __builtin_fma(y, e, y);
}

// Single-precision reciprocal: estimate plus one Newton-Raphson step.
__device__ __forceinline__ float recipf(float a)
{
    float y = __builtin_amdgcn_rcpf(a);
    return __builtin_fmaf(y, __builtin_fmaf(-a, y, 1.0f), y);
}

// ---- XCD-aware tile order ----
// MI355X deals workgroup b to XCD (b mod 8).  Atoms are stored in cell
// order, so giving each XCD one contiguous range of tiles keeps the
// neighborhoods its workgroups gather from inside its own L2.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    const int per = nblocks / kXcds, rem = nblocks % kXcds;
    const int x = b % kXcds, k = b / kXcds;
    return x * per + (x < rem ? x : rem) + k;
}

// ---- wave64 and workgroup reductions (fixed order: deterministic) ----

// v as read from another lane by DPP control kCtrl under row mask kRows;
// lanes with no source lane (shifted in from outside their row with kBound,
// or in a row outside kRows) get old.  32- or 64-bit values (a 64-bit one
// moves as its two halves).
template <int kCtrl, int kRows, bool kBound, typename T>
__device__ __forceinline__ T dpp_read(T old, T v)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(
            T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v),
                                           kCtrl, kRows, 0xf, kBound));
    } else {
        const uint64_t o = __builtin_bit_cast(uint64_t, old), b = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(
            (int)(uint32_t)o, (int)(uint32_t)b, kCtrl, kRows, 0xf, kBound);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(
            (int)(uint32_t)(o >> 32), (int)(uint32_t)(b >> 32), kCtrl, kRows, 0xf, kBound);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

// Lane 63's v, in every lane (scalar registers).
template <typename T>
__device__ __forceinline__ T from_lane63(T v)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
    } else {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

// Sum and maximum over the 64 lanes of a wave, in every lane, by DPP lane
// moves on the VALU (no LDS round trips): the combining pattern of
// wave_scan_incl (shifts by 1, 2, 4, 8 lanes inside each row of 16, then the
// lane-15 and lane-31 broadcasts into the rows above), after which lane 63
// holds the result; the sum adds in that fixed order.  Every lane of the wave
// must be active.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    const T z = T(0);
    v += dpp_read<0x111, 0xf, true>(z, v);   // row_shr:1
    v += dpp_read<0x112, 0xf, true>(z, v);   // row_shr:2
    v += dpp_read<0x114, 0xf, true>(z, v);   // row_shr:4
    v += dpp_read<0x118, 0xf, true>(z, v);   // row_shr:8
    v += dpp_read<0x142, 0xa, false>(z, v);  // row_bcast:15 into rows 1, 3
    v += dpp_read<0x143, 0xc, false>(z, v);  // row_bcast:31 into rows 2, 3
    return from_lane63(v);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
    // lanes with no source read their own value, which leaves them unchanged
    T w;
    w = dpp_read<0x111, 0xf, false>(v, v);
    v = w > v ? w : v;
    w = dpp_read<0x112, 0xf, false>(v, v);
    v = w > v ? w : v;
    w = dpp_read<0x114, 0xf, false>(v, v);
    v = w > v ? w : v;
    w = dpp_read<0x118, 0xf, false>(v, v);
    v = w > v ? w : v;
    w = dpp_read<0x142, 0xa, false>(v, v);
    v = w > v ? w : v;
    w = dpp_read<0x143, 0xc, false>(v, v);
    v = w > v ? w : v;
    return from_lane63(v);
}

// Inclusive prefix sum of v over the 64 lanes of a wave by DPP lane moves on
// the VALU (no LDS round trip): shifts by 1, 2, 4 and 8 lanes inside each row
// of 16 lanes (lanes shifted in from outside the row read 0) give each row's
// own prefix; then each row's last lane is added to the rows above it (lane
// 15 into rows 1 and 3, lane 31 into rows 2 and 3).  Every lane of the wave
// must be active.
__device__ __forceinline__ int wave_scan_incl(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// The maximum of v over the workgroup, valid in thread 0 (0 elsewhere).  Every
// thread of the workgroup calls it.  Kernels fold a per-thread maximum into a
// device-wide one with this and a single global atomic per workgroup: atomics
// from every wave on one word serialize in L2 (one per wave of a 2 M-atom list
// build cost about a millisecond).
__device__ __forceinline__ int workgroup_max(int v)
{
    __shared__ int m;
    if (threadIdx.x == 0) m = 0;
    __syncthreads();
    v = wave_max(v);
    if ((threadIdx.x & (kWave - 1)) == 0 && v > 0) atomicMax(&m, v);
    __syncthreads();
    return threadIdx.x == 0 ? m : 0;
}

// Sum K values across the workgroup; the result is valid in thread 0.
// red must hold (blockDim.x / 64) * K doubles of LDS.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[wid * K + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = 0.0;
            for (int w = 0; w < nw; ++w) t += red[w * K + k];
            v[k] = t;
        }
    }
    __syncthreads();
}

// A value another workgroup of the running kernel published before its
// release in last_block: an agent-scope atomic load, which reads the
// coherence point past this XCD's L2 without invalidating it.
__device__ __forceinline__ double load_coherent(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int load_coherent(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last-workgroup-done (the paper's completion scheme, section 2.3): every
// workgroup publishes its partial, bumps a counter, and the one that sees
// the final count finishes the reduction.  n_wg is the number of
// workgroups of this system's share of the launch.  Returns true in every
// thread of that last workgroup.
//
// The partial must have been stored by thread 0: its counter increment is a
// release at agent scope, which orders thread 0's own earlier stores before
// it (on gfx950 it writes back the XCD's L2).  The last workgroup reads the
// partials with load_coherent, which sees them without the L2 invalidation
// an agent-scope acquire fence would cost on every XCD that holds a last
// workgroup (one per replica in a batch); its own ordering is a
// workgroup-scope acquire after the counter.  Data of earlier kernels is
// visible through the kernel boundary.
__device__ __forceinline__ bool last_block(DevState* dev, int n_wg)
{
    __shared__ int is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = __hip_atomic_fetch_add(&dev->blocks_done, 1u, __ATOMIC_RELEASE,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        is_last = (t == (unsigned)n_wg - 1);
    }
    __syncthreads();
    const bool last = is_last != 0;
    if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return last;
}

// Slot of atom i inside its cell c (every lane of the wave calls it; act:
// lane i holds an atom).  Atoms stored in cell order put a wave's lanes into
// runs of one cell: the first lane of each run takes one atomic for the whole
// run (all runs of the wave at once) and the others rank themselves by their
// distance from it.  A cell met in two runs takes two atomics; the in-cell
// order is fixed later, so only distinct slots matter.
__device__ __forceinline__ void rank_in_cell(const KParams& p, bool act, int c, int i)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int prev = __shfl_up(c, 1, kWave);
    const bool head = act && (lane == 0 || prev != c);
    const uint64_t heads = __ballot(head);
    const int n_act = (int)__popcll(__ballot(act));  // active lanes are a prefix
    const uint64_t upto = (2ull << lane) - 1ull;     // lanes 0..lane
    const int h = act ? 63 - (int)__clzll(heads & upto) : lane;
    int base = 0;
    if (head) {
        const uint64_t later = heads & ~upto;
        int end = later ? (int)__ffsll((unsigned long long)later) - 1 : kWave;
        end = end < n_act ? end : n_act;
        base = atomicAdd(&p.cell_count[c], end - lane);
    }
    base = __shfl(base, h, kWave);
    if (act) p.slot[i] = base + (lane - h);
}

// The copy-back of the reorder folded into the pass that follows the cell
// build (kFoldCopy: the list build, or the cells-only force pass): the cell
// build left the atoms' data in cell order in the scratch arrays, so that
// pass runs over the view of p with state and scratch arrays exchanged
// (positions read from the sorted copy), and every atom's data is copied
// from there into the state arrays by the one thread that owns it (its
// tile's, or its own); no thread reads another atom's data from the state
// arrays during the pass.
__device__ __forceinline__ KParams scratch_view(const KParams& p)
{
    KParams q = p;
    q.x = p.sx; q.sx = p.x;
    q.y = p.sy; q.sy = p.y;
    q.z = p.sz; q.sz = p.z;
    q.vx = p.svx; q.svx = p.vx;
    q.vy = p.svy; q.svy = p.vy;
    q.vz = p.svz; q.svz = p.vz;
    // the force scratch arrays are typed double but hold the force type
    q.fx = p.sfx; q.sfx = static_cast<double*>(p.fx);
    q.fy = p.sfy; q.sfy = static_cast<double*>(p.fy);
    q.fz = p.sfz; q.sfz = static_cast<double*>(p.fz);
    q.id = p.sid; q.sid = p.id;
    q.cell_of = p.scell; q.scell = p.cell_of;
    return q;
}

// Atom at slot k, over scratch_view: its sorted data into the state (the
// forces too unless kForces is false, for a pass that writes them anew).
template <bool kCopy, bool kForces = true>
__device__ __forceinline__ void copy_home(const KParams& q, int k)
{
    if (!kCopy) return;
    q.sx[k] = q.x[k];
    q.sy[k] = q.y[k];
    q.sz[k] = q.z[k];
    q.svx[k] = q.vx[k];
    q.svy[k] = q.vy[k];
    q.svz[k] = q.vz[k];
    if (!kForces) {
    } else if (q.precision == MD_FP64) {
        q.sfx[k] = static_cast<const double*>(q.fx)[k];
        q.sfy[k] = static_cast<const double*>(q.fy)[k];
        q.sfz[k] = static_cast<const double*>(q.fz)[k];
    } else {
        reinterpret_cast<float*>(q.sfx)[k] = static_cast<const float*>(q.fx)[k];
        reinterpret_cast<float*>(q.sfy)[k] = static_cast<const float*>(q.fy)[k];
        reinterpret_cast<float*>(q.sfz)[k] = static_cast<const float*>(q.fz)[k];
    }
    q.sid[k] = q.id[k];
    q.scell[k] = q.cell_of[k];
    q.order[k] = k;
}

}  // namespace md
