// md_pair.h -- the pair terms of the force pass (step F1 of section 2.3),
// shared by the tiled kernels and the layer-matrix pipeline.
//
// Precision: FP64 forms everything in double.  FP32-mixed forms the pair
// separation and the cutoff test in double (the callers do), then the pair
// force, energy and virial and the per-atom sums in float.
#pragma once

#include "md_device.h"

namespace md {

// Per-atom sums: force, u = sum over pairs of sr^12 - sr^6 - shift/(4 eps)
// (the pair energy is 4 eps u_pair, half of it the atom's), virial.
struct AccD {
    double fx = 0, fy = 0, fz = 0, u = 0, w = 0;
};

struct AccF {
    float fx = 0, fy = 0, fz = 0, u = 0, w = 0;
};

// 1/r^2 of the pair terms: the hardware estimate and one Newton-Raphson step,
// y + y(1 - a y).  The estimate's relative error of about 2^-24 becomes about
// 2e-15 (10 ulp), three orders inside the FP64 force tolerance; the second
// step of recip() cost 2.5% of the force pass.
__device__ __forceinline__ double recip_pair(double a)
{
    const double y = __builtin_amdgcn_rcp(a);
    return __builtin_fma(y, __builtin_fma(-a, y, 1.0), y);
}

// Adds the pair's force on the home atom, energy and virial to a, and
// returns the force in g (for the partner's reaction under the third law).
__device__ __forceinline__ void pair_acc(const KParams& p, double dx, double dy, double dz,
                                         double r2, AccD& a, double g[3])
{
    const double inv = recip_pair(r2);
    const double sr2 = p.sig2 * inv;
    const double sr6 = sr2 * sr2 * sr2;
    const double fr = p.eps48 * sr6 * (sr6 - 0.5) * inv;
    g[0] = fr * dx;
    g[1] = fr * dy;
    g[2] = fr * dz;
    a.fx += g[0];
    a.fy += g[1];
    a.fz += g[2];
    a.u += sr6 * (sr6 - 1.0) - p.ushift;
    a.w += fr * r2;
}

__device__ __forceinline__ void pair_acc(const KParams& p, double dx, double dy, double dz,
                                         double r2, AccF& a, float g[3])
{
    const float r2f = (float)r2;
    const float inv = recipf(r2f);
    const float sr2 = (float)p.sig2 * inv;
    const float sr6 = sr2 * sr2 * sr2;
    const float fr = (float)p.eps48 * sr6 * (sr6 - 0.5f) * inv;
    g[0] = fr * (float)dx;
    g[1] = fr * (float)dy;
    g[2] = fr * (float)dz;
    a.fx += g[0];
    a.fy += g[1];
    a.fz += g[2];
    a.u += sr6 * (sr6 - 1.0f) - (float)p.ushift;
    a.w += fr * r2f;
}

template <typename Acc>
__device__ __forceinline__ void pair_acc(const KParams& p, double dx, double dy, double dz,
                                         double r2, Acc& a)
{
    decltype(a.fx) g[3];
    pair_acc(p, dx, dy, dz, r2, a, g);
}

}  // namespace md
