// md_cells.hip -- steps N1-N4 of section 2.3 as a counting sort, plus the
// reorder of section 2.4 item (4) done on the GPU with the prefix-scan the
// paper names as the alternative to its CPU pass.
//
//   k_bin        N1/N2: cell of every atom; atomic occupancy count gives the
//                atom's (unordered) rank in its cell
//   k_scan_*     N3/N4: exclusive scan of the counts -> cell_start, and the
//                largest occupancy; clears the counts for the next build
//   k_scatter    slots grouped by cell (in the order the atomics gave), with
//                each slot's permanent id beside it
//   k_cellsort   inside each cell, ascending permanent id (the paper leaves
//                the order open; a fixed order makes the list reproducible):
//                each atom's place is the number of its cell's members with
//                a smaller id; with reorder on it also writes the atom's data
//                to that place in the scratch arrays
//   k_copyback   with reorder on: the scratch arrays back into the state
//
// Every kernel returns at once unless the rebuild flag is set (or the call
// forces the build), so a step's launch sequence is fixed.  Each kernel is a
// template over where its parameters come from (one system, or one replica
// of a batch: md_internal.h).
#include "md_finish.h"

namespace md {

__device__ __forceinline__ bool rebuild_on(const KParams& p, int force)
{
    return force || p.dev->rebuild;
}

template <class B>
__global__ void k_clear(B b)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_ATOMS, wg, p)) return;
    const int i0 = wg.id * blockDim.x + threadIdx.x;
    for (int i = i0; i < p.ncell; i += wg.n * blockDim.x) p.cell_count[i] = 0;
    if (i0 == 0) {
        DevState* d = p.dev;
        d->step = 0;
        d->n_rebuilds = 0;
        d->hist_count = 0;
        d->dmax2 = 0.0;
        d->rebuild = 0;
        d->blocks_done = 0;
        d->flags = 0;
        d->max_occ = 0;
        d->max_nl = 0;
        for (int k = 0; k < 8; ++k) d->obs[k] = 0.0;
    }
}

template <class B>
__global__ void k_bin(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch_gated(G_ATOMS, force, wg, p)) return;
    for (int i0 = wg.id * blockDim.x; i0 < p.n; i0 += wg.n * blockDim.x) {
        const int i = i0 + threadIdx.x;
        const bool act = i < p.n;
        int c = -1;
        if (act) {
            // positions are folded into [0, L) here, at each cell build, and
            // drift freely in between (by less than skin/2), so the wrap bits
            // of the list stay valid until the next build
            const double x = wrap(p.x[i], p.L), y = wrap(p.y[i], p.L), z = wrap(p.z[i], p.L);
            p.x[i] = x;
            p.y[i] = y;
            p.z[i] = z;
            c = cell_of_pos(x, y, z, p);
            p.cell_of[i] = c;
        }
        rank_in_cell(p, act, c, i);
    }
}

// The cell offsets: one workgroup of kScanThreads threads scans the counts
// kScanPer cells per thread at a time (one 16-byte load each), in chunks of
// kScanThreads * kScanPer cells carried over in order; writes cell_start,
// clears the counts for the next binning and records the largest
// occupancy.  A single launch, so that a step with no rebuild pays for one
// idle kernel here rather than three.
// The scan itself, by one workgroup of kScanThreads threads (wsum: LDS, one
// int per wave).
__device__ __forceinline__ void scan_cells(const KParams& p, int* wsum, int* lds_start = nullptr)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int carry = 0, m = 0;
    for (int c0 = 0; c0 < p.ncell; c0 += kScanThreads * kScanPer) {
        const int c = c0 + threadIdx.x * kScanPer;
        int v[kScanPer];
        if (c + kScanPer <= p.ncell) {
            const int4 q = *reinterpret_cast<const int4*>(p.cell_count + c);
            v[0] = q.x;
            v[1] = q.y;
            v[2] = q.z;
            v[3] = q.w;
        } else {
#pragma unroll
            for (int k = 0; k < kScanPer; ++k) v[k] = c + k < p.ncell ? p.cell_count[c + k] : 0;
        }
        int sum = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            sum += v[k];
            m = v[k] > m ? v[k] : m;
        }
        // exclusive scan of the thread sums: wave64 DPP scan, then the wave totals
        const int inc = wave_scan_incl(sum);
        if (lane == kWave - 1) wsum[wid] = inc;
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kScanThreads / kWave; ++w) {
            before += w < wid ? wsum[w] : 0;
            total += wsum[w];
        }
        __syncthreads();
        int ex = carry + before + inc - sum;
        if (c + kScanPer <= p.ncell) {
            const int4 st = make_int4(ex, ex + v[0], ex + v[0] + v[1], ex + v[0] + v[1] + v[2]);
            *reinterpret_cast<int4*>(p.cell_start + c) = st;
            *reinterpret_cast<int4*>(p.cell_count + c) = make_int4(0, 0, 0, 0);
            if (lds_start) {
                lds_start[c] = st.x;
                lds_start[c + 1] = st.y;
                lds_start[c + 2] = st.z;
                lds_start[c + 3] = st.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < kScanPer; ++k) {
                if (c + k < p.ncell) {
                    p.cell_start[c + k] = ex;
                    p.cell_count[c + k] = 0;
                    if (lds_start) lds_start[c + k] = ex;
                }
                ex += v[k];
            }
        }
        carry += total;
    }
    m = wave_max(m);
    if (lane == 0) wsum[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tm = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) tm = wsum[w] > tm ? wsum[w] : tm;
        p.dev->max_occ = tm;
        p.dev->max_nl = 0;
        p.cell_start[p.ncell] = carry;
        if (lds_start) lds_start[p.ncell] = carry;
    }
}

template <class B>
__global__ __launch_bounds__(kScanThreads) void k_scan(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch_gated(G_ONE, force, wg, p)) return;
    __shared__ int wsum[kScanThreads / kWave];
    scan_cells(p, wsum);
}

// Slot q of atom i in cell order (in the order the atomics gave), with its
// permanent id beside it for the in-cell rank.
__device__ __forceinline__ void scatter_atom(const KParams& p, int i)
{
    const int q = p.cell_start[p.cell_of[i]] + p.slot[i];
    p.tmp[q] = i;
    p.tmp[p.n + q] = p.id[i];  // the ids of a cell side by side
}

// Canonical order inside each cell: ascending permanent id.  The atom at
// slot-order position q counts the members of its cell with a smaller id
// (ids are distinct); that count is its place.  With kPermute the atom's
// data go to that place in the scratch arrays (the permutation into cell
// order, scattered from the atom rather than gathered by a second pass).
template <typename F, bool kPermute>
__device__ __forceinline__ void sort_slot(const KParams& p, int q)
{
    const int32_t* ids = p.tmp + p.n;  // ids in slot order (scatter_atom)
    const int s = p.tmp[q];
    const int c = p.cell_of[s];
    const int a = p.cell_start[c], cnt = p.cell_start[c + 1] - a;
    const int key = ids[q];
    int rank = 0;
#pragma unroll 4
    for (int j = 0; j < cnt; ++j) rank += ids[a + j] < key ? 1 : 0;
    const int d = a + rank;
    p.order[d] = s;
    if (kPermute) {
        p.sx[d] = p.x[s];
        p.sy[d] = p.y[s];
        p.sz[d] = p.z[s];
        p.svx[d] = p.vx[s];
        p.svy[d] = p.vy[s];
        p.svz[d] = p.vz[s];
        reinterpret_cast<F*>(p.sfx)[d] = static_cast<const F*>(p.fx)[s];
        reinterpret_cast<F*>(p.sfy)[d] = static_cast<const F*>(p.fy)[s];
        reinterpret_cast<F*>(p.sfz)[d] = static_cast<const F*>(p.fz)[s];
        p.sid[d] = key;
        p.scell[d] = c;
    }
}

template <class B>
__global__ void k_scatter(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch_gated(G_ATOMS, force, wg, p)) return;
    for (int i = wg.id * blockDim.x + threadIdx.x; i < p.n; i += wg.n * blockDim.x)
        scatter_atom(p, i);
}

template <typename F, class B, bool kPermute>
__global__ void k_cellsort(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch_gated(G_ATOMS, force, wg, p)) return;
    for (int q = wg.id * blockDim.x + threadIdx.x; q < p.n; q += wg.n * blockDim.x)
        sort_slot<F, kPermute>(p, q);
}

// Small systems (at most kSortSmall atoms): the scan, the scatter and the
// in-cell sort by one workgroup, one launch instead of three (their
// barriers order the global writes of one phase before the reads of the
// next inside the workgroup).  kFinish (cells-only steps, which rebuild
// every step): the workgroup first finishes the integration pass before it
// (finish_step), in place of k_int_finish.
template <typename F, class B, bool kPermute, bool kFinish>
__global__ __launch_bounds__(kScanThreads) void k_sort_small(B b, int force, int phase,
                                                             int record_every)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_ONE, wg, p)) return;
    if (kFinish) {
        __shared__ double red[(kScanThreads / kWave) * 5];
        finish_step(p, phase, record_every, red);
        __syncthreads();
    } else if (!rebuild_on(p, force)) {
        return;
    }
    __shared__ int wsum[kScanThreads / kWave];
    scan_cells(p, wsum);
    __syncthreads();
    for (int i = threadIdx.x; i < p.n; i += blockDim.x) scatter_atom(p, i);
    __syncthreads();
    for (int q = threadIdx.x; q < p.n; q += blockDim.x) sort_slot<F, kPermute>(p, q);
}

// k_sort_small's cells-only form (kFinish) with its tables in LDS: the cell
// starts (ncell + 1), and per slot-order position q the atom with its cell
// (atom | cell << kSortAtomBits) and its id (2 n), so that the scatter and the
// in-cell sort read global memory only for the binning of the integration
// pass and the atom data they permute.  Same results as k_sort_small; for
// systems whose tables fit (sort_lds_bytes).
constexpr int kSortAtomBits = 14;  // atoms of a small system: at most kSortSmall = 2^14

template <typename F, bool kPermute>
__global__ __launch_bounds__(kScanThreads) void k_sort_lds(Single b, int phase, int record_every)
{
    const KParams& p = b.p;
    {
        __shared__ double red[(kScanThreads / kWave) * 5];
        finish_step(p, phase, record_every, red);
        __syncthreads();
    }
    extern __shared__ int lds[];
    int* cs = lds;                      // [ncell + 1]
    int* slot_ac = cs + p.ncell + 1;    // [n] atom | cell << kSortAtomBits
    int* slot_id = slot_ac + p.n;       // [n]
    __shared__ int wsum[kScanThreads / kWave];
    scan_cells(p, wsum, cs);
    __syncthreads();
    for (int i = threadIdx.x; i < p.n; i += blockDim.x) {
        const int c = p.cell_of[i], sl = p.slot[i], key = p.id[i];
        const int q = cs[c] + sl;
        slot_ac[q] = i | (c << kSortAtomBits);
        slot_id[q] = key;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < p.n; q += blockDim.x) {
        const int ac = slot_ac[q], s = ac & ((1 << kSortAtomBits) - 1), c = ac >> kSortAtomBits;
        const int a = cs[c], cnt = cs[c + 1] - a, key = slot_id[q];
        int rank = 0;
        for (int j = 0; j < cnt; ++j) rank += slot_id[a + j] < key ? 1 : 0;
        const int d = a + rank;
        p.order[d] = s;
        if (kPermute) {
            p.sx[d] = p.x[s];
            p.sy[d] = p.y[s];
            p.sz[d] = p.z[s];
            p.svx[d] = p.vx[s];
            p.svy[d] = p.vy[s];
            p.svz[d] = p.vz[s];
            reinterpret_cast<F*>(p.sfx)[d] = static_cast<const F*>(p.fx)[s];
            reinterpret_cast<F*>(p.sfy)[d] = static_cast<const F*>(p.fy)[s];
            reinterpret_cast<F*>(p.sfz)[d] = static_cast<const F*>(p.fz)[s];
            p.sid[d] = key;
            p.scell[d] = c;
        }
    }
}

// LDS bytes of k_sort_lds for p, or 0 when its tables do not fit (60 KiB) or
// a cell index does not fit beside the atom.
static size_t sort_lds_bytes(const KParams& p)
{
    if (p.n > (1 << kSortAtomBits) || p.ncell >= (1 << (31 - kSortAtomBits))) return 0;
    const size_t b = sizeof(int) * ((size_t)p.ncell + 1 + 2 * (size_t)p.n);
    return b <= 61440 ? b : 0;
}

template <typename F, class B>
__global__ void k_copyback(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch_gated(G_ATOMS, force, wg, p)) return;
    for (int q = wg.id * blockDim.x + threadIdx.x; q < p.n; q += wg.n * blockDim.x) {
        p.x[q] = p.sx[q];
        p.y[q] = p.sy[q];
        p.z[q] = p.sz[q];
        p.vx[q] = p.svx[q];
        p.vy[q] = p.svy[q];
        p.vz[q] = p.svz[q];
        static_cast<F*>(p.fx)[q] = reinterpret_cast<const F*>(p.sfx)[q];
        static_cast<F*>(p.fy)[q] = reinterpret_cast<const F*>(p.sfy)[q];
        static_cast<F*>(p.fz)[q] = reinterpret_cast<const F*>(p.sfz)[q];
        p.id[q] = p.sid[q];
        p.cell_of[q] = p.scell[q];
        p.order[q] = q;
    }
}

template <class B>
static void clear_seq(const B& b, const LaunchShape& sh, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear<B>, dim3(sh.grid[G_ATOMS]), dim3(sh.block), 0, s, b);
}

template <class B>
static void cells_seq(const B& b, const LaunchShape& sh, int flags, hipStream_t s, int n_small)
{
    const int force = flags & 1;
    const bool copy = !(flags & kFoldCopy);  // else the list or force pass copies back
    const dim3 atoms(sh.grid[G_ATOMS]), blk(sh.block);
    if (!(flags & kFoldBin)) hipLaunchKernelGGL(k_bin<B>, atoms, blk, 0, s, b, force);
    if (n_small) {  // one system of at most kSortSmall atoms
        const dim3 one(1), t(kScanThreads);
        if (!sh.reorder)
            hipLaunchKernelGGL((k_sort_small<double, B, false, false>), one, t, 0, s, b, force,
                               0, 0);
        else if (sh.precision == MD_FP64)
            hipLaunchKernelGGL((k_sort_small<double, B, true, false>), one, t, 0, s, b, force, 0,
                               0);
        else
            hipLaunchKernelGGL((k_sort_small<float, B, true, false>), one, t, 0, s, b, force, 0,
                               0);
    } else {
        hipLaunchKernelGGL(k_scan<B>, dim3(sh.grid[G_ONE]), dim3(kScanThreads), 0, s, b, force);
        hipLaunchKernelGGL(k_scatter<B>, atoms, blk, 0, s, b, force);
        if (!sh.reorder)
            hipLaunchKernelGGL((k_cellsort<double, B, false>), atoms, blk, 0, s, b, force);
        else if (sh.precision == MD_FP64)
            hipLaunchKernelGGL((k_cellsort<double, B, true>), atoms, blk, 0, s, b, force);
        else
            hipLaunchKernelGGL((k_cellsort<float, B, true>), atoms, blk, 0, s, b, force);
    }
    if (sh.reorder && copy) {
        if (sh.precision == MD_FP64)
            hipLaunchKernelGGL((k_copyback<double, B>), atoms, blk, 0, s, b, force);
        else
            hipLaunchKernelGGL((k_copyback<float, B>), atoms, blk, 0, s, b, force);
    }
}

void launch_clear(const KParams& p, hipStream_t s) { clear_seq(Single{p}, shape_of(p), s); }

void launch_cells(const KParams& p, int force, hipStream_t s)
{
    const bool small = (force & kSortSmallOk) && p.n <= kSortSmall;
    cells_seq(Single{p}, shape_of(p), force, s, small ? p.n : 0);
}

// The cell offsets from the occupancy counts alone (forced), for the layer
// pipeline's reorder.
void launch_cell_scan(const KParams& p, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan<Single>, dim3(1), dim3(kScanThreads), 0, s, Single{p}, 1);
}

// The cells-only step's cell build of a small system (atoms binned by the
// integration pass) with the finish of that pass in front (see k_sort_small).
void launch_sort_small_finish(const KParams& p, int phase, int record_every, hipStream_t s)
{
    const dim3 one(1), t(kScanThreads);
    const Single b{p};
    const size_t lds = sort_lds_bytes(p);
    if (lds) {
        if (!p.reorder)
            hipLaunchKernelGGL((k_sort_lds<double, false>), one, t, lds, s, b, phase,
                               record_every);
        else if (p.precision == MD_FP64)
            hipLaunchKernelGGL((k_sort_lds<double, true>), one, t, lds, s, b, phase, record_every);
        else
            hipLaunchKernelGGL((k_sort_lds<float, true>), one, t, lds, s, b, phase, record_every);
        return;
    }
    if (!p.reorder)
        hipLaunchKernelGGL((k_sort_small<double, Single, false, true>), one, t, 0, s, b, 1, phase,
                           record_every);
    else if (p.precision == MD_FP64)
        hipLaunchKernelGGL((k_sort_small<double, Single, true, true>), one, t, 0, s, b, 1, phase,
                           record_every);
    else
        hipLaunchKernelGGL((k_sort_small<float, Single, true, true>), one, t, 0, s, b, 1, phase,
                           record_every);
}

void launch_clear(const Batch& b, const LaunchShape& sh, hipStream_t s) { clear_seq(b, sh, s); }

void launch_cells(const Batch& b, const LaunchShape& sh, int force, hipStream_t s)
{
    cells_seq(b, sh, force, s, 0);
}

}  // namespace md
