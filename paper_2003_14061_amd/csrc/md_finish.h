// md_finish.h -- the per-system finish of an integration pass (reductions of
// section 2.3 F2, step count and history, rebuild decision), shared by the
// finish kernel and the small-system cell sort that takes it over in
// cells-only steps.
#pragma once
#include "md_device.h"

namespace md {

// Sum partials [nb][stride] (component k) over workgroups in a fixed order,
// by one workgroup (the step's finish, or the last workgroup of k_observe,
// see last_block), reading the partials with coherent loads.  The first kT
// threads of the workgroup take the partials (strided by kT); any further
// threads add zeros, so a larger workgroup sums in the same order.
template <int kT>
__device__ __forceinline__ double finish_sum(const double* part, int nb, int stride, int k,
                                             double* red)
{
    double v[1] = {0.0};
    if ((int)threadIdx.x < kT)
        for (int b = threadIdx.x; b < nb; b += kT) v[0] += load_coherent(part + b * stride + k);
    block_sum<1>(v, red);
    return v[0];
}

template <int kT>
__device__ __forceinline__ double finish_max(const double* part, int nb, int stride, int k,
                                             double* red)
{
    double m = 0.0;
    if ((int)threadIdx.x < kT)
        for (int b = threadIdx.x; b < nb; b += kT) {
            double t = load_coherent(part + b * stride + k);
            m = t > m ? t : m;
        }
    m = wave_max(m);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) red[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)blockDim.x / kWave; ++w) t = red[w] > t ? red[w] : t;
        m = t;
    }
    __syncthreads();
    return m;
}

// Finish a completed step: count it, and on steps the history asks for, sum
// U, W (last force pass) and K, P (this kernel's n_wg partials) and append
// them.
__device__ __forceinline__ void record_step(const KParams& p, int n_wg, int record_every,
                                            double* red)
{
    DevState* dd = p.dev;
    const int64_t step = dd->step + 1;
    __syncthreads();
    if (threadIdx.x == 0) dd->step = step;
    if (!(record_every > 0 && step % record_every == 0)) return;
    double U = finish_sum<kFinishThreads>(p.fpart, p.nblk_force, 2, 0, red);
    double W = finish_sum<kFinishThreads>(p.fpart, p.nblk_force, 2, 1, red);
    if (p.bonded_on) {
        U += finish_sum<kFinishThreads>(p.bpart, p.nblk_bonded, 2, 0, red);
        W += finish_sum<kFinishThreads>(p.bpart, p.nblk_bonded, 2, 1, red);
    }
    const double K = finish_sum<kFinishThreads>(p.ipart, n_wg, 8, 0, red);
    const double Px = finish_sum<kFinishThreads>(p.ipart, n_wg, 8, 1, red);
    const double Py = finish_sum<kFinishThreads>(p.ipart, n_wg, 8, 2, red);
    const double Pz = finish_sum<kFinishThreads>(p.ipart, n_wg, 8, 3, red);
    if (threadIdx.x == 0) {
        md_record* r = p.hist + (dd->hist_count % kHistCap);
        r->step = step;
        r->U = U;
        r->K = 0.5 * p.mass * K;
        r->W = W;
        r->P[0] = p.mass * Px;
        r->P[1] = p.mass * Py;
        r->P[2] = p.mass * Pz;
        r->dmax = sqrt(dd->dmax2);
        r->rebuilt = dd->rebuild;
        r->pad = 0;
        dd->hist_count += 1;
    }
}

// The end of an integration pass: count the step and record it (phase >= 1),
// and from the largest displacement decide whether the cells and list are
// rebuilt before the next force pass (phase <= 1).  By one workgroup of at
// least kFinishThreads threads (red: LDS, (blockDim / 64) * 5 doubles).
__device__ __forceinline__ void finish_step(const KParams& p, int phase, int record_every,
                                            double* red)
{
    const int n_wg = grid_of(p, G_INTEGRATE);
    if (phase >= 1) record_step(p, n_wg, record_every, red);
    if (phase <= 1) {
        __shared__ int rb_all;
        const double m = finish_max<kFinishThreads>(p.ipart, n_wg, 8, 4, red);
        if (threadIdx.x == 0) {
            DevState* d = p.dev;
            d->dmax2 = m;
            const int rb = p.mode == MD_CELLS_ONLY ? 1 : (m > p.disp_thr2 ? 1 : 0);
            d->rebuild = rb;
            if (rb) d->n_rebuilds += 1;
            rb_all = rb;
        }
        if (p.gate_tab[0]) {  // a batch replica: its gate bits in the workgroup table
            __syncthreads();
            const uint16_t v = (uint16_t)(p.rep | (rb_all ? kGateBit : 0));
            for (int j = 0; j < 3; ++j)
                for (int i = threadIdx.x; i < p.gate_n[j]; i += blockDim.x) p.gate_tab[j][i] = v;
        }
    }
}

}  // namespace md
