// md_integrate.hip -- leapfrog integration and the global reductions.
//
// The leapfrog (section 4.3) is kick-drift-kick with two separate half
// kicks.  The second half kick of step s and the first of step s+1 use the
// same force, so one pass over the atoms does both (in that order, each
// rounded on its own) and measures the kinetic energy and momentum at the
// full step in between.  The drift measures each atom's displacement from
// the list reference (minimum image; positions are folded back into [0, L)
// only when the cells are rebuilt, see k_bin); the largest one decides
// whether the cells and list are rebuilt before the next force pass (the
// paper refreshes "at intervals of several time steps", section 2.3, from a
// bound on the maximal velocity; here the bound is the displacement itself).
//
// Reductions (section 2.3, F2): each integration workgroup writes its
// partial sums, and k_int_finish, one workgroup per system launched right
// after, sums them in workgroup order and publishes the result on the
// device (the rebuild decision, the step count, the history record).  The
// paper's completion scheme, where the last workgroup to finish does this,
// is used by the one-off observables pass (k_observe); per step it would
// cost every workgroup an agent-scope release, which on this GPU writes
// back its XCD's L2 and measured several microseconds per launch, more
// than the extra launch.
#include "md_finish.h"

namespace md {

// kBin (cells-only steps, which rebuild the cells every step): the drift also
// folds the positions into [0, L) and bins them (cell and slot, as k_bin), so
// that the cell build that follows starts at the scan.
template <typename F, class B, bool kBin>
__global__ __launch_bounds__(kIntThreads) void k_integrate(B b, int phase, int record_every)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_INTEGRATE, wg, p)) return;
    __shared__ double red[(kIntThreads / kWave) * 5];
    const F* fx = static_cast<const F*>(p.fx);
    const F* fy = static_cast<const F*>(p.fy);
    const F* fz = static_cast<const F*>(p.fz);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // v^2, Px, Py, Pz, (unused)
    double dmax2 = 0.0;
    const int stride = wg.n * blockDim.x;
    const bool drift_now = phase <= 1, track = phase <= 1 && p.mode == MD_NEIGHBOR_LIST;
    const bool fold = p.pipeline == MD_PIPE_ALLPAIRS || kBin;
    for (int i0 = wg.id * blockDim.x; i0 < p.n; i0 += stride) {
        const int i = i0 + threadIdx.x;
        int c = -1;
        if (i < p.n) {
            // every input first, so that one round of loads serves the iteration
            const double gx = (double)fx[i], gy = (double)fy[i], gz = (double)fz[i];
            double vx = p.vx[i], vy = p.vy[i], vz = p.vz[i];
            double x = 0.0, y = 0.0, z = 0.0, rx = 0.0, ry = 0.0, rz = 0.0;
            if (drift_now) {
                x = p.x[i];
                y = p.y[i];
                z = p.z[i];
            }
            if (track) {
                rx = p.xr[i];
                ry = p.yr[i];
                rz = p.zr[i];
            }
            if (phase >= 1) {  // second half kick of the finished step
                vx = kick(vx, p.hdt, gx);
                vy = kick(vy, p.hdt, gy);
                vz = kick(vz, p.hdt, gz);
                acc[0] += (vx * vx + vy * vy) + vz * vz;
                acc[1] += vx;
                acc[2] += vy;
                acc[3] += vz;
            }
            if (drift_now) {  // first half kick and drift of the next step
                vx = kick(vx, p.hdt, gx);
                vy = kick(vy, p.hdt, gy);
                vz = kick(vz, p.hdt, gz);
                x = drift(x, p.dt, vx);
                y = drift(y, p.dt, vy);
                z = drift(z, p.dt, vz);
                if (fold) {  // no cell build follows to fold them (or it starts here)
                    x = wrap(x, p.L);
                    y = wrap(y, p.L);
                    z = wrap(z, p.L);
                }
                if (kBin) {
                    c = cell_of_pos(x, y, z, p);
                    p.cell_of[i] = c;
                }
                p.x[i] = x;
                p.y[i] = y;
                p.z[i] = z;
                if (track) {
                    const double d2 =
                        dist2(minimg(x - rx, p.L, p.invL), minimg(y - ry, p.L, p.invL),
                              minimg(z - rz, p.L, p.invL));
                    dmax2 = d2 > dmax2 ? d2 : dmax2;
                }
            }
            p.vx[i] = vx;
            p.vy[i] = vy;
            p.vz[i] = vz;
        }
        if (kBin && drift_now) rank_in_cell(p, i < p.n, c, i);
    }
    block_sum<5>(acc, red);
    dmax2 = wave_max(dmax2);
    {
        const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
        if (lane == 0) red[wid] = dmax2;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < (int)blockDim.x / kWave; ++w) t = red[w] > t ? red[w] : t;
            dmax2 = t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = p.ipart + 8 * wg.id;
        o[0] = acc[0];
        o[1] = acc[1];
        o[2] = acc[2];
        o[3] = acc[3];
        o[4] = dmax2;
    }
}

// The end of an integration pass (one workgroup per system, see finish_step).
template <class B>
__global__ __launch_bounds__(kFinishThreads) void k_int_finish(B b, int phase, int record_every)
{
    Wg wg;
    KParams p;
    if (!b.fetch(G_ONE, wg, p)) return;
    __shared__ double red[(kFinishThreads / kWave) * 5];
    finish_step(p, phase, record_every, red);
}

// Observables of the current state: K and P from the velocities, U and W
// from the partials of the last force pass.
__global__ __launch_bounds__(kIntThreads) void k_observe(KParams p)
{
    __shared__ double red[(kIntThreads / kWave) * 4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += stride) {
        const double vx = p.vx[i], vy = p.vy[i], vz = p.vz[i];
        acc[0] += (vx * vx + vy * vy) + vz * vz;
        acc[1] += vx;
        acc[2] += vy;
        acc[3] += vz;
    }
    block_sum<4>(acc, red);
    if (threadIdx.x == 0) {
        double* o = p.ipart + 8 * blockIdx.x;
        for (int k = 0; k < 4; ++k) o[k] = acc[k];
    }
    if (!last_block(p.dev, gridDim.x)) return;
    double U = finish_sum<kIntThreads>(p.fpart, p.nblk_force, 2, 0, red);
    double W = finish_sum<kIntThreads>(p.fpart, p.nblk_force, 2, 1, red);
    if (p.bonded_on) {
        U += finish_sum<kIntThreads>(p.bpart, p.nblk_bonded, 2, 0, red);
        W += finish_sum<kIntThreads>(p.bpart, p.nblk_bonded, 2, 1, red);
    }
    double s[4];
    for (int k = 0; k < 4; ++k) s[k] = finish_sum<kIntThreads>(p.ipart, gridDim.x, 8, k, red);
    if (threadIdx.x == 0) {
        DevState* d = p.dev;
        d->obs[0] = U;
        d->obs[1] = 0.5 * p.mass * s[0];
        d->obs[2] = W;
        d->obs[3] = p.mass * s[1];
        d->obs[4] = p.mass * s[2];
        d->obs[5] = p.mass * s[3];
        d->obs[6] = d->dmax2;
        d->blocks_done = 0;
    }
}

template <class B>
static void integrate_pass(const B& b, const LaunchShape& sh, int phase, int record_every,
                           hipStream_t s, bool bin = false)
{
    const dim3 g(sh.grid[G_INTEGRATE]), t(kIntThreads);
    if (bin && phase <= 1) {
        if (sh.precision == MD_FP64)
            hipLaunchKernelGGL((k_integrate<double, B, true>), g, t, 0, s, b, phase, record_every);
        else
            hipLaunchKernelGGL((k_integrate<float, B, true>), g, t, 0, s, b, phase, record_every);
    } else if (sh.precision == MD_FP64) {
        hipLaunchKernelGGL((k_integrate<double, B, false>), g, t, 0, s, b, phase, record_every);
    } else {
        hipLaunchKernelGGL((k_integrate<float, B, false>), g, t, 0, s, b, phase, record_every);
    }
}

template <class B>
static void integrate_finish(const B& b, const LaunchShape& sh, int phase, int record_every,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_int_finish<B>, dim3(sh.grid[G_ONE]), dim3(kFinishThreads), 0, s, b,
                       phase, record_every);
}

template <class B>
static void integrate_seq(const B& b, const LaunchShape& sh, int phase, int record_every,
                          hipStream_t s)
{
    integrate_pass(b, sh, phase, record_every, s);
    integrate_finish(b, sh, phase, record_every, s);
}

void launch_integrate(const KParams& p, int phase, int record_every, hipStream_t s)
{
    integrate_seq(Single{p}, shape_of(p), phase, record_every, s);
}

void launch_integrate_pass(const KParams& p, int phase, int record_every, hipStream_t s,
                           bool bin)
{
    integrate_pass(Single{p}, shape_of(p), phase, record_every, s, bin);
}

void launch_integrate_finish(const KParams& p, int phase, int record_every, hipStream_t s)
{
    integrate_finish(Single{p}, shape_of(p), phase, record_every, s);
}

void launch_integrate(const Batch& b, const LaunchShape& sh, int phase, int record_every,
                      hipStream_t s)
{
    integrate_seq(b, sh, phase, record_every, s);
}

void launch_observe(const KParams& p, hipStream_t s)
{
    hipLaunchKernelGGL(k_observe, dim3(grid_of(p, G_INTEGRATE)), dim3(kIntThreads), 0, s, p);
}

}  // namespace md
