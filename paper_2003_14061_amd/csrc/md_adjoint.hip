// md_adjoint.hip -- reverse mode of a trajectory of the leapfrog.
//
// What is differentiated is the method of section 2.3 (pair forces F1 over
// the neighbor list) inside the kick-drift-kick leapfrog of section 4.3.
// Going backwards through the steps, every point x_s of the trajectory is
// visited once.  Both half kicks that use F(x_s) (the first of step s and
// the second of step s-1) see the same velocity adjoint lambda_v, so one
// pass over the list per point applies them together:
//
//   lambda_x += coef * J(x_s) lambda_v          J = dF/dx (symmetric)
//   theta    += coef * lambda_v . dF/d(eps, sigma)
//   lambda_x -= (dL/dubar) / (S N) * F(x_s)     the mean-energy observable
//   theta    += (dL/dubar) / (S N) * (U/eps, W/sigma)
//   lambda_v' = lambda_v + dt * lambda_x        the drift of step s-1
//
// For one pair with separation d = x_i - x_j, r = |d| and s = sigma/r,
//   F_i   = fr d,  fr = 48 eps (s^12 - s^6/2) / r^2
//   J     : (J lambda)_i = sum_j fr (l_i - l_j) + gr (d . (l_i - l_j)) d,
//           gr = (1/r) dfr/dr = -96 eps (7 s^12 - 2 s^6) / r^4
//   dF/deps = F / eps,  dfr/dsigma = 144 eps (4 s^12 - s^6) / (sigma r^2)
// and with the cutoff moving with sigma (r_cut / sigma fixed) the energy
// shift does not depend on sigma, so dU/dsigma = W / sigma and dU/deps =
// U / eps.  Pairs crossing the cutoff add nothing (pathwise derivative).
//
// The soft radial distribution g_b (a Gaussian of standard deviation w per
// pair, lowered by its value at 3w and cut there) is summed per bin in
// 64-bit fixed point: integer sums do not depend on the order of the
// atomic adds, so g is reproducible bit for bit.
#include "md_tiles.h"

namespace md {

constexpr double kPi = 3.141592653589793;
constexpr double kSqrt2Pi = 2.5066282746310002;  // sqrt(2 pi)
constexpr int kMaxBins = 1024;

// ---- positions of a stored point, re-imaged onto the current list ----

// x_i <- p_i - L * rint((p_i - xr_i) / L) per coordinate: the stored position
// moved by whole box lengths next to the list's reference, so that the wrap
// bits of the list stay valid.  The largest squared displacement from the
// reference decides (last workgroup) whether the cells and list are rebuilt.
__global__ __launch_bounds__(256) void k_adj_reimage(KParams p, const double* px,
                                                     const double* py, const double* pz)
{
    __shared__ double red[256 / kWave];
    double m = 0.0;
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += stride) {
        const double ex = px[i] - p.xr[i], ey = py[i] - p.yr[i], ez = pz[i] - p.zr[i];
        p.x[i] = px[i] - p.L * rint(ex * p.invL);
        p.y[i] = py[i] - p.L * rint(ey * p.invL);
        p.z[i] = pz[i] - p.L * rint(ez * p.invL);
        const double d2 = dist2(minimg(ex, p.L, p.invL), minimg(ey, p.L, p.invL),
                                minimg(ez, p.L, p.invL));
        m = d2 > m ? d2 : m;
    }
    m = wave_max(m);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) red[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)blockDim.x / kWave; ++w) t = red[w] > t ? red[w] : t;
        p.ipart[8 * blockIdx.x + 4] = t;
    }
    if (!last_block(p.dev, gridDim.x)) return;
    // the last workgroup: maximum over the partials, spread over its threads
    double t = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) {
        const double v = load_coherent(p.ipart + 8 * b + 4);
        t = v > t ? v : t;
    }
    t = wave_max(t);
    __syncthreads();
    if (lane == 0) red[wid] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)blockDim.x / kWave; ++w) t = red[w] > t ? red[w] : t;
        p.dev->dmax2 = t;
        p.dev->rebuild = t > p.disp_thr2 ? 1 : 0;
        p.dev->blocks_done = 0;
    }
}

// ---- one reverse point ----

__device__ __forceinline__ double rcp_t(double a) { return recip(a); }
__device__ __forceinline__ float rcp_t(float a) { return recipf(a); }

template <typename T>
struct AdjAcc {
    T jx = 0, jy = 0, jz = 0;  // (J lambda_v)_i
    T fx = 0, fy = 0, fz = 0;  // F_i
    T gx = 0, gy = 0, gz = 0;  // dF_i / dsigma
    T u = 0, w = 0;
    int np = 0;
};

template <typename T>
struct AdjOp {
    const KParams& p;
    const Stage& s;
    const AdjArgs& q;
    double lix, liy, liz;  // lambda_v of the home atom
    AdjAcc<T>& a;
    __device__ __forceinline__ void operator()(double dx, double dy, double dz, double r2, int e,
                                               int j)
    {
        if (!(r2 < p.rc2)) return;
        double ljx, ljy, ljz;
        if (j < 0) {
            lds_xyz(s.a3, e, ljx, ljy, ljz);
        } else {
            ljx = q.vx[j];
            ljy = q.vy[j];
            ljz = q.vz[j];
        }
        const T inv = rcp_t((T)r2);
        const T sr2 = (T)p.sig2 * inv;
        const T sr6 = sr2 * sr2 * sr2;
        const T sr12 = sr6 * sr6;
        const T e48 = (T)p.eps48;
        const T fr = e48 * sr6 * (sr6 - (T)0.5) * inv;
        const T gr = -(T)2 * e48 * inv * inv * ((T)7 * sr12 - (T)2 * sr6);
        const T fs = (T)(3.0 * p.eps48 / p.sigma) * inv * ((T)4 * sr12 - sr6);
        const T tx = (T)dx, ty = (T)dy, tz = (T)dz;
        const T ex = (T)(lix - ljx), ey = (T)(liy - ljy), ez = (T)(liz - ljz);
        const T gde = gr * (tx * ex + ty * ey + tz * ez);
        a.jx += fr * ex + gde * tx;
        a.jy += fr * ey + gde * ty;
        a.jz += fr * ez + gde * tz;
        a.fx += fr * tx;
        a.fy += fr * ty;
        a.fz += fr * tz;
        a.gx += fs * tx;
        a.gy += fs * ty;
        a.gz += fs * tz;
        a.u += sr6 * (sr6 - (T)1);
        a.w += fr * (T)r2;
        a.np += 1;
    }
};

template <typename T, int LANES>
__global__ void k_adj_point(KParams p, AdjArgs q)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ double red[(1024 / kWave) * 2];
    const Tile g = tile_of(p, xcd_tile(blockIdx.x, gridDim.x));
    Stage s = stage_layout(p, smem, q.cap, true);
    stage_tables(p, g, s);
    const int nh = home_count(s);
    const int mode = staged_image_mode(p, s, tile_interior(p, g));
    stage_atoms<true, true>(p, s, q.vx, q.vy, q.vz);
    __syncthreads();
    const double lu = q.loss_scale != 0.0 ? q.gobs[0] * q.loss_scale : 0.0;
    const int per_pass = blockDim.x / LANES;
    const int sub = threadIdx.x % LANES;
    double th[2] = {0.0, 0.0};
    for (int hb = 0; hb < nh; hb += per_pass) {
        const int h = hb + threadIdx.x / LANES;
        AdjAcc<T> a;
        int i = 0;
        double vix = 0.0, viy = 0.0, viz = 0.0;
        if (h < nh) {
            int eh, pos;
            home_atom(s, h, eh, pos);
            i = atom_at(p, pos);
            double xi, yi, zi;
            home_position(p, s, eh, i, xi, yi, zi);
            if (s.fits) {
                lds_xyz(s.a3, eh, vix, viy, viz);
            } else {
                vix = q.vx[i];
                viy = q.vy[i];
                viz = q.vz[i];
            }
            AdjOp<T> op{p, s, q, vix, viy, viz, a};
            walk_home<LANES>(p, s, mode, i, sub, p.nl_count[i], xi, yi, zi, op);
        }
        if (LANES > 1) {
            a.jx = lane_group_sum<LANES>(a.jx);
            a.jy = lane_group_sum<LANES>(a.jy);
            a.jz = lane_group_sum<LANES>(a.jz);
            a.fx = lane_group_sum<LANES>(a.fx);
            a.fy = lane_group_sum<LANES>(a.fy);
            a.fz = lane_group_sum<LANES>(a.fz);
            a.gx = lane_group_sum<LANES>(a.gx);
            a.gy = lane_group_sum<LANES>(a.gy);
            a.gz = lane_group_sum<LANES>(a.gz);
            a.u = lane_group_sum<LANES>(a.u);
            a.w = lane_group_sum<LANES>(a.w);
            a.np = lane_group_sum<LANES>(a.np);
        }
        if (h < nh && sub == 0) {
            const double Fx = a.fx, Fy = a.fy, Fz = a.fz;
            const double lx = q.lx[i] + q.coef * (double)a.jx - lu * Fx;
            const double ly = q.ly[i] + q.coef * (double)a.jy - lu * Fy;
            const double lz = q.lz[i] + q.coef * (double)a.jz - lu * Fz;
            q.lx[i] = lx;
            q.ly[i] = ly;
            q.lz[i] = lz;
            q.nx[i] = vix + q.drift * lx;
            q.ny[i] = viy + q.drift * ly;
            q.nz[i] = viz + q.drift * lz;
            const double ui = p.eps2 * (double)a.u - p.half_shift * (double)a.np;
            const double wi = 0.5 * (double)a.w;
            th[0] += q.coef * (vix * Fx + viy * Fy + viz * Fz) / p.eps + lu * ui / p.eps;
            th[1] += q.coef * (vix * (double)a.gx + viy * (double)a.gy + viz * (double)a.gz) +
                     lu * wi / p.sigma;
            if (!isfinite(lx + ly + lz)) atomicOr(&p.dev->flags, (int)MD_FLAG_NONFINITE);
        }
    }
    block_sum<2>(th, red);
    if (threadIdx.x == 0) {
        q.tpart[2 * blockIdx.x] = th[0];
        q.tpart[2 * blockIdx.x + 1] = th[1];
    }
    if (!last_block(p.dev, gridDim.x)) return;
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) {
        v[0] += load_coherent(q.tpart + 2 * b);
        v[1] += load_coherent(q.tpart + 2 * b + 1);
    }
    block_sum<2>(v, red);
    if (threadIdx.x == 0) {
        q.theta[0] += v[0];
        q.theta[1] += v[1];
        p.dev->blocks_done = 0;
    }
}

// ---- soft g(r) ----

__device__ __forceinline__ double bin_center(const GrArgs& g, int b)
{
    return (b + 0.5) * g.rmax / g.n_bins;
}

__device__ __forceinline__ double gr_norm(const KParams& p, const GrArgs& g, int b)
{
    const double rho = (double)p.n / (p.L * p.L * p.L);
    const double rb = bin_center(g, b);
    return (double)p.n * rho * 4.0 * kPi * rb * rb;
}

// Bins whose kernel reaches distance r: |r - r_b| < 3w.
__device__ __forceinline__ void bin_range(const GrArgs& g, double r, int& b0, int& b1)
{
    const double delta = g.rmax / g.n_bins;
    b0 = (int)floor((r - 3.0 * g.width) / delta - 0.5);
    b1 = (int)ceil((r + 3.0 * g.width) / delta - 0.5);
    b0 = b0 < 0 ? 0 : b0;
    b1 = b1 > g.n_bins - 1 ? g.n_bins - 1 : b1;
}

struct GrOp {
    const GrArgs& g;
    unsigned long long* lh;  // LDS histogram
    double reach2;
    __device__ __forceinline__ void operator()(double, double, double, double r2, int, int)
    {
        if (!(r2 < reach2)) return;
        const double r = sqrt(r2), w = g.width;
        int b0, b1;
        bin_range(g, r, b0, b1);
        for (int b = b0; b <= b1; ++b) {
            const double t = r - bin_center(g, b);
            if (fabs(t) < 3.0 * w) {
                const double k = (exp(-0.5 * (t / w) * (t / w)) - exp(-4.5)) / (w * kSqrt2Pi);
                atomicAdd(&lh[b], (unsigned long long)llrint(k * g.scale));
            }
        }
    }
};

__global__ void k_gr_clear(GrArgs g)
{
    for (int b = threadIdx.x; b < g.n_bins; b += blockDim.x) g.hist[b] = 0ull;
}

__global__ void k_gr_hist(KParams p, GrArgs g, int cap)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ unsigned long long lh[kMaxBins];
    for (int b = threadIdx.x; b < g.n_bins; b += blockDim.x) lh[b] = 0ull;
    const Tile t = tile_of(p, xcd_tile(blockIdx.x, gridDim.x));
    Stage s = stage_layout(p, smem, cap, false);
    stage_tables(p, t, s);
    const int nh = home_count(s);
    const int mode = staged_image_mode(p, s, tile_interior(p, t));
    stage_positions_imaged(p, s);
    __syncthreads();
    const double reach = g.rmax + 3.0 * g.width;
    GrOp op{g, lh, reach * reach};
    for (int h = threadIdx.x; h < nh; h += blockDim.x) {
        int eh, pos;
        home_atom(s, h, eh, pos);
        const int i = atom_at(p, pos);
        double xi, yi, zi;
        home_position(p, s, eh, i, xi, yi, zi);
        walk_home<1>(p, s, mode, i, 0, p.nl_count[i], xi, yi, zi, op);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < g.n_bins; b += blockDim.x)
        if (lh[b]) atomicAdd(&g.hist[b], lh[b]);
}

__global__ void k_gr_finish(KParams p, GrArgs g)
{
    for (int b = threadIdx.x; b < g.n_bins; b += blockDim.x)
        g.out[b] = (double)g.hist[b] / g.scale / gr_norm(p, g, b);
}

// Gradient of sum_b (dL/dg_b) g_b: each list partner j of atom i adds
// 2 sum_b (dL/dg_b / norm_b) K'(r - r_b) d / r (the ordered pairs (i, j) and
// (j, i) both hold r_ij).  Written into lambda_x (the observables' direct
// dependence on the last positions).
struct GrGradOp {
    const GrArgs& g;
    const double* wn;  // LDS: dL/dg_b / norm_b
    double reach2;
    double ax = 0.0, ay = 0.0, az = 0.0;
    __device__ __forceinline__ void operator()(double dx, double dy, double dz, double r2, int,
                                               int)
    {
        if (!(r2 < reach2)) return;
        const double r = sqrt(r2), w = g.width;
        int b0, b1;
        bin_range(g, r, b0, b1);
        double c = 0.0;
        for (int b = b0; b <= b1; ++b) {
            const double t = r - bin_center(g, b);
            if (fabs(t) < 3.0 * w)
                c += wn[b] * (-(t / (w * w)) * exp(-0.5 * (t / w) * (t / w)) / (w * kSqrt2Pi));
        }
        const double f = 2.0 * c / r;
        ax += f * dx;
        ay += f * dy;
        az += f * dz;
    }
};

__global__ void k_gr_grad(KParams p, GrArgs g, int cap)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ double wn[kMaxBins];
    for (int b = threadIdx.x; b < g.n_bins; b += blockDim.x)
        wn[b] = g.gobs[1 + b] / gr_norm(p, g, b);
    const Tile t = tile_of(p, xcd_tile(blockIdx.x, gridDim.x));
    Stage s = stage_layout(p, smem, cap, false);
    stage_tables(p, t, s);
    const int nh = home_count(s);
    const int mode = staged_image_mode(p, s, tile_interior(p, t));
    stage_positions_imaged(p, s);
    __syncthreads();
    const double reach = g.rmax + 3.0 * g.width;
    for (int h = threadIdx.x; h < nh; h += blockDim.x) {
        int eh, pos;
        home_atom(s, h, eh, pos);
        const int i = atom_at(p, pos);
        double xi, yi, zi;
        home_position(p, s, eh, i, xi, yi, zi);
        GrGradOp op{g, wn, reach * reach};
        walk_home<1>(p, s, mode, i, 0, p.nl_count[i], xi, yi, zi, op);
        g.lx[i] = op.ax;
        g.ly[i] = op.ay;
        g.lz[i] = op.az;
    }
}

// ---- small kernels of the trajectory driver ----

// Mean over the last n_steps history records of U, divided by N.
__global__ __launch_bounds__(256) void k_traj_ubar(KParams p, int32_t n_steps, double* out)
{
    __shared__ double red[256 / kWave];
    const int64_t count = p.dev->hist_count;
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < n_steps; t += blockDim.x)
        v[0] += p.hist[(count - n_steps + t) % kHistCap].U;
    block_sum<1>(v, red);
    if (threadIdx.x == 0) out[0] = v[0] / ((double)n_steps * (double)p.n);
}

__global__ void k_fill(double* a, size_t n, double v)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = v;
}

// ---- launchers ----

static int gr_stage_cap(const KParams& p)
{
    // the static LDS of the g(r) kernels (kMaxBins 8-byte words) comes out of
    // the planned room
    const int less = (int)(kMaxBins * sizeof(double) / (3 * sizeof(double)));
    int cap = p.scap - (less + 63) / 64 * 64;
    return cap < 64 ? 64 : cap;
}

void launch_adj_reimage(const KParams& p, const double* px, const double* py, const double* pz,
                        hipStream_t s)
{
    int g = (p.n + 255) / 256;
    g = g < p.int_grid ? (g > 0 ? g : 1) : p.int_grid;
    hipLaunchKernelGGL(k_adj_reimage, dim3(g), dim3(256), 0, s, p, px, py, pz);
}

template <typename T>
static void launch_adj_t(const KParams& p, const AdjArgs& a, hipStream_t s)
{
    const dim3 g(p.n_tiles), t(p.force_block);
    const size_t lds = stage_bytes(p, a.cap, true);
    switch (p.force_lanes) {
        case 8: hipLaunchKernelGGL((k_adj_point<T, 8>), g, t, lds, s, p, a); break;
        case 4: hipLaunchKernelGGL((k_adj_point<T, 4>), g, t, lds, s, p, a); break;
        case 2: hipLaunchKernelGGL((k_adj_point<T, 2>), g, t, lds, s, p, a); break;
        default: hipLaunchKernelGGL((k_adj_point<T, 1>), g, t, lds, s, p, a); break;
    }
}

void launch_adj_point(const KParams& p, const AdjArgs& a, hipStream_t s)
{
    if (p.precision == MD_FP64)
        launch_adj_t<double>(p, a, s);
    else
        launch_adj_t<float>(p, a, s);
}

void launch_gr(const KParams& p, const GrArgs& g, hipStream_t s)
{
    const int cap = gr_stage_cap(p);
    hipLaunchKernelGGL(k_gr_clear, dim3(1), dim3(256), 0, s, g);
    hipLaunchKernelGGL(k_gr_hist, dim3(p.n_tiles), dim3(p.force_block),
                       stage_bytes(p, cap), s, p, g, cap);
    hipLaunchKernelGGL(k_gr_finish, dim3(1), dim3(256), 0, s, p, g);
}

void launch_gr_grad(const KParams& p, const GrArgs& g, hipStream_t s)
{
    const int cap = gr_stage_cap(p);
    hipLaunchKernelGGL(k_gr_grad, dim3(p.n_tiles), dim3(p.force_block),
                       stage_bytes(p, cap), s, p, g, cap);
}

void launch_traj_ubar(const KParams& p, int32_t n_steps, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_traj_ubar, dim3(1), dim3(256), 0, s, p, n_steps, out);
}

void launch_fill(double* a, size_t n, double v, hipStream_t s)
{
    size_t g = (n + 255) / 256;
    g = g < 1024 ? (g > 0 ? g : 1) : 1024;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)g), dim3(256), 0, s, a, n, v);
}

}  // namespace md
