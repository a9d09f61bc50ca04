// md_bonded.hip -- bonded forces of linear polymer chains (section 4.3,
// item (2)): elastic bonds, a bond-angle term between adjacent bonds and a
// dihedral term over three consecutive bonds, added to the pair forces.
//
// As the paper suggests, each thread deals with one atom and every bonded
// interaction it takes part in: the thread of the atom at chain position p
// gathers the positions of chain positions p-3 .. p+3, forms the bond
// vectors between them (minimum image), and adds to its own force the share
// of the two bonds, three angles and four dihedrals that contain it.  Each
// term is thus evaluated by every thread it touches; no atomics are needed
// and the forces are reproducible.  A term's energy (and a bond's virial) is
// booked once, by the thread of its first atom, into per-workgroup partials.
//
// Forms (md_bonded in md.h): FENE bonds U = -(k R0^2/2) ln(1 - r^2/R0^2);
// angles U = k_b (1 - cos theta), theta between consecutive bond vectors;
// dihedrals U = sum_m c_m cos^m phi, cos phi = n1.n2/(|n1||n2|) with
// n1 = b1 x b2, n2 = b2 x b3.  The chain of permanent id i is i / M, its
// position i mod M; slot_of maps an id to its current slot and is rebuilt
// whenever the slots are permuted.  Everything is FP64; in FP32-mixed mode
// the bonded force is added to the FP32 force arrays.
#include "md_device.h"

namespace md {

constexpr int kBondThreads = 256;

struct V3 {
    double x, y, z;
};

__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(double k, V3 a) { return {k * a.x, k * a.y, k * a.z}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// cos of the angle between u and v, and its gradients with respect to both.
__device__ __forceinline__ double cos_grad(V3 u, V3 v, V3& gu, V3& gv)
{
    const double uu = dot(u, u), vv = dot(v, v);
    const double inv = 1.0 / sqrt(uu * vv);
    const double c = dot(u, v) * inv;
    gu = inv * v - (c / uu) * u;
    gv = inv * u - (c / vv) * v;
    return c;
}

// slot_of[id[k]] = k for every slot (after each permutation of the slots).
// Ids outside [0, n) are flagged; duplicate ids leave the map inconsistent,
// which k_bonded detects.
__global__ void k_bond_map(KParams p, int force)
{
    if (!force && !p.dev->rebuild) return;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < p.n; k += gridDim.x * blockDim.x) {
        const int i = p.id[k];
        if (i >= 0 && i < p.n)
            p.slot_of[i] = k;
        else
            atomicOr(&p.dev->flags, (int)MD_FLAG_TOPOLOGY);
    }
}

template <typename F>
__global__ __launch_bounds__(kBondThreads) void k_bonded(KParams p)
{
    __shared__ double red[(kBondThreads / kWave) * 2];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double e[2] = {0.0, 0.0};  // energy and virial of the terms this atom owns
    if (k < p.n) {
        const int M = p.chain_len;
        const int id = p.id[k];
        const int pos = id % M, base = id - pos;
        // positions of chain positions pos-3 .. pos+3 (r[d + 3])
        V3 r[7];
        bool ok = id >= 0 && id < p.n, have[7];
#pragma unroll
        for (int d = -3; d <= 3; ++d) {
            const int q = pos + d;
            have[d + 3] = q >= 0 && q < M;
            r[d + 3] = {0.0, 0.0, 0.0};
            if (have[d + 3] && ok) {
                int s = k;
                if (d != 0) {
                    s = p.slot_of[base + q];
                    if (s < 0 || s >= p.n || p.id[s] != base + q) {
                        ok = false;
                        continue;
                    }
                }
                r[d + 3] = {p.x[s], p.y[s], p.z[s]};
            }
        }
        if (!ok) {
            atomicOr(&p.dev->flags, (int)MD_FLAG_TOPOLOGY);
        } else {
            // bond vectors b[j + 3] from chain position pos+j to pos+j+1, j = -3 .. 2
            V3 b[6];
#pragma unroll
            for (int j = -3; j <= 2; ++j) {
                const V3 d = r[j + 4] - r[j + 3];
                b[j + 3] = {minimg(d.x, p.L, p.invL), minimg(d.y, p.L, p.invL),
                            minimg(d.z, p.L, p.invL)};
            }
            V3 f = {0.0, 0.0, 0.0};
            // bonds (pos-1, pos) and (pos, pos+1)
            if (p.fene_k != 0.0) {
#pragma unroll
                for (int j = -1; j <= 0; ++j) {
                    if (!have[j + 3] || !have[j + 4]) continue;
                    const V3 d = b[j + 3];
                    const double r2 = dot(d, d);
                    if (!(r2 < p.fene_r02)) {
                        atomicOr(&p.dev->flags, (int)MD_FLAG_BOND_BROKEN);
                        continue;
                    }
                    const double q = 1.0 - r2 / p.fene_r02;
                    const double g = p.fene_k / q;
                    f = f + (j == 0 ? g : -g) * d;  // pulls the atom toward its partner
                    if (j == 0) {
                        e[0] += -0.5 * p.fene_k * p.fene_r02 * log(q);
                        e[1] += -g * r2;
                    }
                }
            }
            // angles with first atom at pos+a: bonds b[a], b[a+1]
            if (p.bend_k != 0.0) {
#pragma unroll
                for (int a = -2; a <= 0; ++a) {
                    if (!have[a + 3] || !have[a + 5]) continue;
                    V3 g1, g2;
                    const double c = cos_grad(b[a + 3], b[a + 4], g1, g2);
                    const double kb = p.bend_k;
                    if (a == 0) {
                        f = f - kb * g1;
                        e[0] += kb * (1.0 - c);
                    } else if (a == -1) {
                        f = f + kb * (g1 - g2);
                    } else {
                        f = f + kb * g2;
                    }
                }
            }
            // dihedrals with first atom at pos+a: bonds b[a], b[a+1], b[a+2]
            if (p.tors_on) {
#pragma unroll
                for (int a = -3; a <= 0; ++a) {
                    if (!have[a + 3] || !have[a + 6]) continue;
                    const V3 b1 = b[a + 3], b2 = b[a + 4], b3 = b[a + 5];
                    V3 gA, gB;
                    const double c = cos_grad(cross(b1, b2), cross(b2, b3), gA, gB);
                    const double slope =
                        p.tors_c[1] + c * (2.0 * p.tors_c[2] + c * 3.0 * p.tors_c[3]);
                    // d cos(phi) / d b1, b2, b3
                    const V3 d1 = cross(b2, gA);
                    const V3 d2 = cross(gA, b1) + cross(b3, gB);
                    const V3 d3 = cross(gB, b2);
                    V3 dc;  // d cos(phi) / d r of this atom
                    if (a == 0)
                        dc = -1.0 * d1;
                    else if (a == -1)
                        dc = d1 - d2;
                    else if (a == -2)
                        dc = d2 - d3;
                    else
                        dc = d3;
                    f = f - slope * dc;
                    if (a == 0)
                        e[0] += p.tors_c[0] + c * (p.tors_c[1] + c * (p.tors_c[2] + c * p.tors_c[3]));
                }
            }
            if (!isfinite(f.x + f.y + f.z + e[0]))
                atomicOr(&p.dev->flags, (int)MD_FLAG_NONFINITE);
            F* fx = static_cast<F*>(p.fx);
            F* fy = static_cast<F*>(p.fy);
            F* fz = static_cast<F*>(p.fz);
            fx[k] = (F)((double)fx[k] + f.x);
            fy[k] = (F)((double)fy[k] + f.y);
            fz[k] = (F)((double)fz[k] + f.z);
        }
    }
    block_sum<2>(e, red);
    if (threadIdx.x == 0) {
        p.bpart[2 * blockIdx.x] = e[0];
        p.bpart[2 * blockIdx.x + 1] = e[1];
    }
}

int bonded_blocks(int n) { return (n + kBondThreads - 1) / kBondThreads; }

void launch_bond_map(const KParams& p, int force, hipStream_t s)
{
    int g = (p.n + p.block - 1) / p.block;
    g = g < p.gate_grid ? g : p.gate_grid;
    hipLaunchKernelGGL(k_bond_map, dim3(g), dim3(p.block), 0, s, p, force);
}

void launch_bonded(const KParams& p, hipStream_t s)
{
    const dim3 g(bonded_blocks(p.n));
    if (p.precision == MD_FP64)
        hipLaunchKernelGGL(k_bonded<double>, g, dim3(kBondThreads), 0, s, p);
    else
        hipLaunchKernelGGL(k_bonded<float>, g, dim3(kBondThreads), 0, s, p);
}

}  // namespace md
