// md_allpairs.hip -- the all-pairs force evaluation the paper sets beside the
// cell and list methods for comparison (section 4.2, alternative (2)):
// every atom is tested against every other, the partner positions passing
// through on-chip memory in tiles so that each global load serves many
// pairs, as in a dense matrix product.  md_params.pipeline = MD_PIPE_ALLPAIRS.
//
// Work split.  A workgroup of kApThreads threads (four waves) owns a block of
// 64 home atoms, one per lane, held by all four waves, and one contiguous
// chunk of partners.  The chunk passes through LDS in tiles of kApThreads
// positions (each thread loads one; the next tile is fetched into registers
// while the current one is used); wave w takes entries [64w, 64w + 64) of
// every tile, every lane reading the same entry (an LDS broadcast).  The
// four waves' sums are added in LDS in wave order.  When the partners are
// split into S > 1 chunks (so that a small system still fills the chip),
// each workgroup stores its per-atom sums as partials and a second kernel
// adds them in chunk order, so the forces are the same from run to run.
// (A last-chunk-done combine inside the kernel needs an agent-scope release
// by every workgroup, a write-back of its XCD's L2, which cost more than the
// second launch.)
//
// Pairs: minimum image d - L rint(d/L) in every coordinate, self excluded,
// pairs at r^2 >= r_cut^2 skipped; the pair terms and the precision rule
// are those of the list-based pass (md_pair.h).  Energy and virial partials
// per workgroup go to the same reduction as the other force passes.
#include "md_pair.h"

namespace md {

constexpr int kApThreads = 256;            // threads per workgroup; also the tile size
constexpr int kApWaves = kApThreads / kWave;

struct alignas(32) Pos4 {
    double x, y, z, w;
};

// One wave's share of one tile: cnt partners from q, global index of q[0] j.
template <typename Acc>
__device__ __forceinline__ void ap_pass(const KParams& p, const Pos4* q, int cnt, int j,
                                        int i, double xi, double yi, double zi, Acc& a)
{
#pragma unroll 8
    for (int t = 0; t < cnt; ++t) {
        const Pos4 r = q[t];
        const double dx = minimg(xi - r.x, p.L, p.invL);
        const double dy = minimg(yi - r.y, p.L, p.invL);
        const double dz = minimg(zi - r.z, p.L, p.invL);
        const double r2 = dist2(dx, dy, dz);
        if (r2 < p.rc2 && j + t != i) pair_acc(p, dx, dy, dz, r2, a);
    }
}

template <typename F, typename Acc>
__global__ __launch_bounds__(kApThreads) void k_forces_allpairs(KParams p)
{
    __shared__ Pos4 tile[2][kApThreads];
    __shared__ F sums[kApWaves - 1][5][kWave];
    const int S = p.ap_split;
    const int ib = (int)blockIdx.x / S, s = (int)blockIdx.x % S;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int i = ib * kWave + lane;
    const bool home = i < p.n;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    if (home) {
        xi = p.x[i];
        yi = p.y[i];
        zi = p.z[i];
    }
    const int j0 = s * p.ap_chunk;
    const int j1 = p.n - j0 < p.ap_chunk ? p.n : j0 + p.ap_chunk;
    // first tile
    double qx = 0.0, qy = 0.0, qz = 0.0;
    {
        const int j = j0 + (int)threadIdx.x;
        if (j < j1) {
            qx = p.x[j];
            qy = p.y[j];
            qz = p.z[j];
        }
        tile[0][threadIdx.x] = Pos4{qx, qy, qz, 0.0};
    }
    __syncthreads();
    Acc a;
    int buf = 0;
    for (int t0 = j0; t0 < j1; t0 += kApThreads) {
        const int tn = t0 + kApThreads;
        if (tn < j1) {  // next tile into registers while this one is used
            const int j = tn + (int)threadIdx.x;
            if (j < j1) {
                qx = p.x[j];
                qy = p.y[j];
                qz = p.z[j];
            }
        }
        const int e0 = wv * kWave;
        int cnt = j1 - t0 - e0;
        cnt = cnt > kWave ? kWave : cnt;
        if (home && cnt > 0) {
            if (cnt == kWave)
                ap_pass(p, &tile[buf][e0], kWave, t0 + e0, i, xi, yi, zi, a);
            else
                ap_pass(p, &tile[buf][e0], cnt, t0 + e0, i, xi, yi, zi, a);
        }
        if (tn < j1) tile[buf ^ 1][threadIdx.x] = Pos4{qx, qy, qz, 0.0};
        __syncthreads();
        buf ^= 1;
    }
    // the four waves' sums, added in wave order by wave 0
    if (wv > 0) {
        sums[wv - 1][0][lane] = a.fx;
        sums[wv - 1][1][lane] = a.fy;
        sums[wv - 1][2][lane] = a.fz;
        sums[wv - 1][3][lane] = a.u;
        sums[wv - 1][4][lane] = a.w;
    }
    __syncthreads();
    if (wv != 0) return;  // wave 0 alone from here; no workgroup barrier follows
    for (int w = 0; w < kApWaves - 1; ++w) {
        a.fx += sums[w][0][lane];
        a.fy += sums[w][1][lane];
        a.fz += sums[w][2][lane];
        a.u += sums[w][3][lane];
        a.w += sums[w][4][lane];
    }
    double eu = home ? p.eps2 * (double)a.u : 0.0;
    double ew = home ? 0.5 * (double)a.w : 0.0;
    if (home && !isfinite(eu + (double)a.fx + (double)a.fy + (double)a.fz))
        atomicOr(&p.dev->flags, (int)MD_FLAG_NONFINITE);
    eu = wave_sum(eu);
    ew = wave_sum(ew);
    if (lane == 0) {
        p.fpart[2 * blockIdx.x] = eu;
        p.fpart[2 * blockIdx.x + 1] = ew;
    }
    F* fx = static_cast<F*>(p.fx);
    F* fy = static_cast<F*>(p.fy);
    F* fz = static_cast<F*>(p.fz);
    if (S == 1) {
        if (home) {
            fx[i] = a.fx;
            fy[i] = a.fy;
            fz[i] = a.fz;
        }
        return;
    }
    // partials of this chunk; k_ap_combine adds them up after the launch
    F* part = static_cast<F*>(p.apart);
    if (home) {
        part[(3 * (int64_t)s + 0) * p.npad + i] = a.fx;
        part[(3 * (int64_t)s + 1) * p.npad + i] = a.fy;
        part[(3 * (int64_t)s + 2) * p.npad + i] = a.fz;
    }
}

// The force on each atom: its S chunk partials added in chunk order, a
// thread per atom and component, sixteen chunks' loads issued at a time.
template <typename F>
__global__ void k_ap_combine(KParams p)
{
    constexpr int kBatch = 16;
    const F* part = static_cast<const F*>(p.apart);
    const int S = p.ap_split;
    const int64_t total = 3 * (int64_t)p.n;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(q / p.n), i = (int)(q % p.n);
        const F* src = part + (int64_t)k * p.npad + i;  // chunk c at src + 3c npad
        F g = F(0);
        for (int c0 = 0; c0 < S; c0 += kBatch) {
            F v[kBatch];
#pragma unroll
            for (int c = 0; c < kBatch; ++c)
                v[c] = c0 + c < S ? src[3 * (int64_t)(c0 + c) * p.npad] : F(0);
#pragma unroll
            for (int c = 0; c < kBatch; ++c)
                if (c0 + c < S) g += v[c];
        }
        F* out = static_cast<F*>(k == 0 ? p.fx : (k == 1 ? p.fy : p.fz));
        out[i] = g;
        if (!isfinite((double)g)) atomicOr(&p.dev->flags, (int)MD_FLAG_NONFINITE);
    }
}

// Folds the positions into [0, L) (the all-pairs pipeline's stand-in for the
// cell build; during a run the drift folds them).
__global__ void k_ap_fold(KParams p)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += gridDim.x * blockDim.x) {
        p.x[i] = wrap(p.x[i], p.L);
        p.y[i] = wrap(p.y[i], p.L);
        p.z[i] = wrap(p.z[i], p.L);
    }
}

int allpairs_home_blocks(int n) { return (n + kWave - 1) / kWave; }

// Chunks per home block: enough workgroups to give every SIMD several waves
// (2048 workgroups of four waves), each chunk at least one whole tile.
void allpairs_split(int n, int* split, int* chunk)
{
    const int nb = allpairs_home_blocks(n);
    const int tiles = (n + kApThreads - 1) / kApThreads;
    int s = (2048 + nb - 1) / nb;
    s = s < tiles ? s : tiles;
    s = s < 1 ? 1 : s;
    const int per = (n + s - 1) / s;
    int c = (per + kApThreads - 1) / kApThreads * kApThreads;
    c = c < kApThreads ? kApThreads : c;
    *chunk = c;
    *split = (n + c - 1) / c;
}

void launch_allpairs_forces(const KParams& p, hipStream_t s)
{
    const dim3 g(allpairs_home_blocks(p.n) * p.ap_split);
    const int64_t need = (3 * (int64_t)p.n + 255) / 256;
    const dim3 gc((unsigned)(need < 4096 ? need : 4096));
    if (p.precision == MD_FP64) {
        hipLaunchKernelGGL((k_forces_allpairs<double, AccD>), g, dim3(kApThreads), 0, s, p);
        if (p.ap_split > 1) hipLaunchKernelGGL(k_ap_combine<double>, gc, dim3(256), 0, s, p);
    } else {
        hipLaunchKernelGGL((k_forces_allpairs<float, AccF>), g, dim3(kApThreads), 0, s, p);
        if (p.ap_split > 1) hipLaunchKernelGGL(k_ap_combine<float>, gc, dim3(256), 0, s, p);
    }
}

void launch_allpairs_fold(const KParams& p, hipStream_t s)
{
    int g = (p.n + p.block - 1) / p.block;
    g = g < p.gate_grid ? g : p.gate_grid;
    hipLaunchKernelGGL(k_ap_fold, dim3(g), dim3(p.block), 0, s, p);
}

}  // namespace md
