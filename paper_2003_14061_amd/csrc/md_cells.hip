// md_cells.hip -- steps N1-N4 of section 2.3 as a counting sort, plus the
// reorder of section 2.4 item (4) done on the GPU with the prefix-scan the
// paper names as the alternative to its CPU pass.
//
//   k_bin        N1/N2: cell of every atom; atomic occupancy count gives the
//                atom's (unordered) rank in its cell
//   k_scan_*     N3/N4: exclusive scan of the counts -> cell_start, and the
//                largest occupancy; clears the counts for the next build
//   k_scatter    slots grouped by cell (in the order the atomics gave)
//   k_cellsort   inside each cell, ascending permanent id (the paper leaves
//                the order open; a fixed order makes the list reproducible):
//                each atom's place is the number of its cell's members with
//                a smaller id
//   k_permute /  with reorder on: atom data permuted into cell order
//   k_copyback
//
// Every kernel returns at once unless the rebuild flag is set (or the call
// forces the build), so a step's launch sequence is fixed.  Each kernel is a
// template over where its parameters come from (one system, or one replica
// of a batch: md_internal.h).
#include "md_device.h"

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
    if (!b.fetch(G_ATOMS, wg, p)) return;
    if (!rebuild_on(p, force)) return;
    const int lane = threadIdx.x & (kWave - 1);
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
        // Atoms stored in cell order put a wave's 64 atoms into a few cells:
        // the lanes of one cell take one atomic together and rank themselves
        // by their position in the wave (the in-cell order is fixed later).
        uint64_t todo = __ballot(act);
        while (todo) {
            const int leader = __ffsll((unsigned long long)todo) - 1;
            const int cl = __shfl(c, leader, kWave);
            const uint64_t same = __ballot(act && c == cl);
            int base = 0;
            if (lane == leader) base = atomicAdd(&p.cell_count[cl], (int)__popcll(same));
            base = __shfl(base, leader, kWave);
            if (act && c == cl)
                p.slot[i] = base + (int)__popcll(same & ((1ull << lane) - 1ull));
            todo &= ~same;
        }
    }
}

// Inclusive scan across a wave64.
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread across the workgroup (kScanThreads).
__device__ __forceinline__ int block_excl_scan(int v, int* total)
{
    __shared__ int wsum[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Per tile: sum and max of the counts.
template <class B>
__global__ __launch_bounds__(kScanThreads) void k_scan_partial(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_SCAN, wg, p)) return;
    if (!rebuild_on(p, force)) return;
    const int base = wg.id * kScanTile + threadIdx.x * kScanPer;
    int s = 0, m = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        int c = base + k;
        int v = c < p.ncell ? p.cell_count[c] : 0;
        s += v;
        m = v > m ? v : m;
    }
    s = wave_sum(s);
    m = wave_max(m);
    __shared__ int ss[kScanThreads / kWave], sm[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) {
        ss[wid] = s;
        sm[wid] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int ts = 0, tm = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) {
            ts += ss[w];
            tm = sm[w] > tm ? sm[w] : tm;
        }
        p.scanpart[2 * wg.id] = ts;
        p.scanpart[2 * wg.id + 1] = tm;
    }
}

// One workgroup: exclusive scan of the tile sums (in place), largest occupancy.
template <class B>
__global__ __launch_bounds__(kScanThreads) void k_scan_top(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_ONE, wg, p)) return;
    if (!rebuild_on(p, force)) return;
    const int ntile = grid_of(p, G_SCAN);
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    int m = 0;
    for (int base = 0; base < ntile; base += kScanThreads) {
        int t = base + threadIdx.x;
        int v = t < ntile ? p.scanpart[2 * t] : 0;
        int mv = t < ntile ? p.scanpart[2 * t + 1] : 0;
        m = mv > m ? mv : m;
        int total;
        int ex = block_excl_scan(v, &total);
        if (t < ntile) p.scanpart[2 * t] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
    m = wave_max(m);
    __shared__ int sm[kScanThreads / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) sm[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tm = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) tm = sm[w] > tm ? sm[w] : tm;
        p.dev->max_occ = tm;
        p.dev->max_nl = 0;
        p.cell_start[p.ncell] = carry;
    }
}

// Per tile: local exclusive scan plus the tile offset -> cell_start; clear counts.
template <class B>
__global__ __launch_bounds__(kScanThreads) void k_scan_final(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_SCAN, wg, p)) return;
    if (!rebuild_on(p, force)) return;
    const int base = wg.id * kScanTile + threadIdx.x * kScanPer;
    int v[kScanPer], s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        int c = base + k;
        v[k] = c < p.ncell ? p.cell_count[c] : 0;
        s += v[k];
    }
    int total;
    int ex = block_excl_scan(s, &total) + p.scanpart[2 * wg.id];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        int c = base + k;
        if (c < p.ncell) {
            p.cell_start[c] = ex;
            p.cell_count[c] = 0;
        }
        ex += v[k];
    }
}

template <class B>
__global__ void k_scatter(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_ATOMS, wg, p)) return;
    if (!rebuild_on(p, force)) return;
    for (int i = wg.id * blockDim.x + threadIdx.x; i < p.n; i += wg.n * blockDim.x)
        p.tmp[p.cell_start[p.cell_of[i]] + p.slot[i]] = i;
}

// Canonical order inside each cell: ascending permanent id.  One lane per
// atom counts the members of its cell with a smaller id (ids are distinct);
// that count is its place.
template <class B>
__global__ void k_cellsort(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_ATOMS, wg, p)) return;
    if (!rebuild_on(p, force)) return;
    for (int q = wg.id * blockDim.x + threadIdx.x; q < p.n; q += wg.n * blockDim.x) {
        const int s = p.tmp[q];
        const int c = p.cell_of[s];
        const int a = p.cell_start[c], cnt = p.cell_start[c + 1] - a;
        const int key = p.id[s];
        int rank = 0;
        for (int j = 0; j < cnt; ++j) rank += p.id[p.tmp[a + j]] < key ? 1 : 0;
        p.order[a + rank] = s;
    }
}

template <typename F, class B>
__global__ void k_permute(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_ATOMS, wg, p)) return;
    if (!rebuild_on(p, force)) return;
    for (int q = wg.id * blockDim.x + threadIdx.x; q < p.n; q += wg.n * blockDim.x) {
        const int o = p.order[q];
        p.sx[q] = p.x[o];
        p.sy[q] = p.y[o];
        p.sz[q] = p.z[o];
        p.svx[q] = p.vx[o];
        p.svy[q] = p.vy[o];
        p.svz[q] = p.vz[o];
        reinterpret_cast<F*>(p.sfx)[q] = static_cast<const F*>(p.fx)[o];
        reinterpret_cast<F*>(p.sfy)[q] = static_cast<const F*>(p.fy)[o];
        reinterpret_cast<F*>(p.sfz)[q] = static_cast<const F*>(p.fz)[o];
        p.sid[q] = p.id[o];
        p.scell[q] = p.cell_of[o];
    }
}

template <typename F, class B>
__global__ void k_copyback(B b, int force)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_ATOMS, wg, p)) return;
    if (!rebuild_on(p, force)) return;
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
static void cells_seq(const B& b, const LaunchShape& sh, int force, hipStream_t s)
{
    const dim3 atoms(sh.grid[G_ATOMS]), blk(sh.block);
    hipLaunchKernelGGL(k_bin<B>, atoms, blk, 0, s, b, force);
    hipLaunchKernelGGL(k_scan_partial<B>, dim3(sh.grid[G_SCAN]), dim3(kScanThreads), 0, s, b,
                       force);
    hipLaunchKernelGGL(k_scan_top<B>, dim3(sh.grid[G_ONE]), dim3(kScanThreads), 0, s, b, force);
    hipLaunchKernelGGL(k_scan_final<B>, dim3(sh.grid[G_SCAN]), dim3(kScanThreads), 0, s, b,
                       force);
    hipLaunchKernelGGL(k_scatter<B>, atoms, blk, 0, s, b, force);
    hipLaunchKernelGGL(k_cellsort<B>, atoms, blk, 0, s, b, force);
    if (sh.reorder) {
        if (sh.precision == MD_FP64) {
            hipLaunchKernelGGL((k_permute<double, B>), atoms, blk, 0, s, b, force);
            hipLaunchKernelGGL((k_copyback<double, B>), atoms, blk, 0, s, b, force);
        } else {
            hipLaunchKernelGGL((k_permute<float, B>), atoms, blk, 0, s, b, force);
            hipLaunchKernelGGL((k_copyback<float, B>), atoms, blk, 0, s, b, force);
        }
    }
}

void launch_clear(const KParams& p, hipStream_t s) { clear_seq(Single{p}, shape_of(p), s); }

void launch_cells(const KParams& p, int force, hipStream_t s)
{
    cells_seq(Single{p}, shape_of(p), force, s);
}

void launch_clear(const Batch& b, const LaunchShape& sh, hipStream_t s) { clear_seq(b, sh, s); }

void launch_cells(const Batch& b, const LaunchShape& sh, int force, hipStream_t s)
{
    cells_seq(b, sh, force, s);
}

}  // namespace md
