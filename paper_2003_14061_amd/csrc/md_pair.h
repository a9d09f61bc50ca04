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

// Per-atom sums of the full-list passes in a leaner form.  With
// q = sr6 (sr6 - 1/2) the pair force on the home atom is 48 eps (q / r^2) d
// and the pair's r.F is 48 eps q, so the sums are f' = sum (q / r^2) d,
// Q = sum q and S = sum (sr6 + 2 c), c = shift / (4 eps); the constant
// factors are applied once per atom (lean_finish), and the pair energy sum
// sum (sr12 - sr6 - c) equals Q - S / 2.  Fifteen operations per pair
// against seventeen for the form above.
template <typename T>
struct Lean {
    T fx = 0, fy = 0, fz = 0, q = 0, s6 = 0;
};
using LeanD = Lean<double>;
using LeanF = Lean<float>;

__device__ __forceinline__ void pair_acc(const KParams& p, double dx, double dy, double dz,
                                         double r2, LeanD& a)
{
    const double inv = recip_pair(r2);
    const double sr2 = p.sig2 * inv;
    const double sr4 = sr2 * sr2;
    const double sr6 = sr4 * sr2;
    const double q = sr6 * (sr6 - 0.5);
    const double g = q * inv;
    a.fx = __builtin_fma(g, dx, a.fx);
    a.fy = __builtin_fma(g, dy, a.fy);
    a.fz = __builtin_fma(g, dz, a.fz);
    a.q += q;
    a.s6 += sr6 + p.ushift2;
}

__device__ __forceinline__ void pair_acc(const KParams& p, double dx, double dy, double dz,
                                         double r2, LeanF& a)
{
    const float inv = recipf((float)r2);
    const float sr2 = (float)p.sig2 * inv;
    const float sr4 = sr2 * sr2;
    const float sr6 = sr4 * sr2;
    const float q = sr6 * (sr6 - 0.5f);
    const float g = q * inv;
    a.fx = __builtin_fmaf(g, (float)dx, a.fx);
    a.fy = __builtin_fmaf(g, (float)dy, a.fy);
    a.fz = __builtin_fmaf(g, (float)dz, a.fz);
    a.q += q;
    a.s6 += sr6 + (float)p.ushift2;
}

// The home atom's force, its energy u_i (half of each pair's) and its half
// of each pair's virial, from its lean sums.
template <typename T>
__device__ __forceinline__ void lean_finish(const KParams& p, const Lean<T>& a, T& fx, T& fy,
                                            T& fz, double& ui, double& wi)
{
    const T k = (T)p.eps48;
    fx = k * a.fx;
    fy = k * a.fy;
    fz = k * a.fz;
    ui = p.eps2 * ((double)a.q - 0.5 * (double)a.s6);
    wi = 0.5 * p.eps48 * (double)a.q;
}

// Accumulator type of the full-list passes for force type F.
template <typename F>
using LeanOf = Lean<F>;

template <typename Acc>
__device__ __forceinline__ void pair_acc(const KParams& p, double dx, double dy, double dz,
                                         double r2, Acc& a)
{
    decltype(a.fx) g[3];
    pair_acc(p, dx, dy, dz, r2, a, g);
}

}  // namespace md
