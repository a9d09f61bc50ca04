// md_api.hip -- the C ABI of libmd (declared in include/md.h).
//
// Host side only: validation, derived geometry, workspace layout, the
// kernel-parameter block and the order of launches.  All arithmetic on atoms
// happens in the kernels of the other translation units.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <initializer_list>
#include <mutex>
#include <new>
#include <vector>

#include "md_internal.h"
#include "md_tiles.h"

using namespace md;

#include "md_ctx.h"

using md::align_up;
using md::kAlign;

extern "C" const char* md_status_str(int32_t st)
{
    switch (st) {
        case MD_OK: return "ok";
        case MD_ERR_ARG: return "invalid argument";
        case MD_ERR_BOX_TOO_SMALL: return "box too small: fewer than 3 cells per side";
        case MD_ERR_NL_OVERFLOW: return "neighbor list overflow: raise nl_capacity";
        case MD_ERR_NONFINITE: return "non-finite force or energy";
        case MD_ERR_HIP: return "HIP runtime error";
        case MD_ERR_NOT_BOUND: return "buffers not bound (call md_bind)";
        case MD_ERR_STATE: return "call out of order";
        case MD_ERR_LAYER_OVERFLOW: return "layer matrix overflow: a cell held more atoms than layers";
        case MD_ERR_BOND_BROKEN: return "a bond reached the FENE limit R0";
        case MD_ERR_TOPOLOGY: return "atom ids are not a permutation of 0..N-1 (chains undefined)";
        case MD_ERR_WORKSPACE_TOO_LARGE:
            return "workspace larger than the library's static array (md_bind_static)";
        default: return "unknown status";
    }
}

// Tiling of the neighbor-list mode: the grid is cut into near-equal blocks of
// about kx x ky x kz cells (a requested size of 0 is chosen here).  The
// choice minimizes the staged cells per home cell, (kx+2)(ky+2)(kz+2) over
// kx ky kz, among blocks whose expected staged atoms (1.15x the mean plus 64)
// fit the LDS share that lets three force workgroups share a CU, whose
// expected home atoms fill at most three passes of the force workgroup and,
// for a system alone, that give at least one tile per CU (ties: the longer
// block along x, whose slot runs are longer).  The LDS
// capacity then allows 1.15x the mean staged count plus 64 of the largest
// block; a tile that does not fit takes its partners from global memory.
static void plan_tiles(md_ctx* c)
{
    KParams& k = c->kp;
    const int nc = k.nc;
    const double occ = (double)k.n / ((double)nc * nc * nc);
    const double lds_share = 160.0 * 1024.0 / 3.0 - 2048.0;  // bytes, three per CU
    const double home_max = 3.0 * k.force_block / k.force_lanes;
    // a system alone keeps a workgroup per CU at least (replicas of a batch share
    // the machine)
    const int64_t ncell = (int64_t)nc * nc * nc;
    const int64_t min_tiles = c->min_tiles < ncell ? c->min_tiles : ncell;
    auto maxsize = [nc](int req) {
        const int parts = (nc + req - 1) / req;
        return (nc + parts - 1) / parts;
    };
    int best[3] = {1, 1, 1};
    double best_ratio = 1e300;
    const int kx_hi = nc < 64 ? nc : 64, kyz_hi = nc < 4 ? nc : 4;
    for (int kz = 1; kz <= kyz_hi; ++kz)
        for (int ky = kz; ky <= kyz_hi; ++ky)
            for (int kx = 1; kx <= kx_hi; ++kx) {
                const int ax = c->tile_cells > 0 ? c->tile_cells : kx;
                const int ay = c->tile_y > 0 ? c->tile_y : ky;
                const int az = c->tile_z > 0 ? c->tile_z : kz;
                const int mx = maxsize(ax), my = maxsize(ay), mz = maxsize(az);
                const double staged = (double)(mx + 2) * (my + 2) * (mz + 2) * occ;
                const double home = (double)mx * my * mz * occ;
                const int64_t tiles = (int64_t)((nc + ax - 1) / ax) * ((nc + ay - 1) / ay) *
                                      ((nc + az - 1) / az);
                const bool ok = (1.15 * staged + 64.0) * 3.0 * sizeof(double) <= lds_share &&
                                home <= home_max && tiles >= min_tiles;
                const double ratio = (double)(mx + 2) * (my + 2) * (mz + 2) / ((double)mx * my * mz);
                // a block that breaks the limits is taken only while nothing fits
                const double score = ok ? ratio : 1e200 + ratio;
                if (score < best_ratio - 1e-9 ||
                    (fabs(score - best_ratio) <= 1e-9 && mx > best[0])) {
                    best_ratio = score;
                    best[0] = ax;
                    best[1] = ay;
                    best[2] = az;
                }
            }
    k.tiles_x = (nc + best[0] - 1) / best[0];
    k.tiles_y = (nc + best[1] - 1) / best[1];
    k.tiles_z = (nc + best[2] - 1) / best[2];
    k.kx_max = (nc + k.tiles_x - 1) / k.tiles_x;
    k.ky_max = (nc + k.tiles_y - 1) / k.tiles_y;
    k.kz_max = (nc + k.tiles_z - 1) / k.tiles_z;
    k.n_tiles = k.tiles_x * k.tiles_y * k.tiles_z;
    c->tile_cells_res = k.kx_max;
    c->tile_y_res = k.ky_max;
    c->tile_z_res = k.kz_max;
    const double s_mean = (double)(k.kx_max + 2) * (k.ky_max + 2) * (k.kz_max + 2) * occ;
    // tables and static LDS
    const size_t tables = stage_bytes(k, 0) + 2048;
    const size_t room = c->lds_limit > tables ? c->lds_limit - tables : 0;
    int scap = c->stage_cap > 0 ? c->stage_cap : (int)(1.15 * s_mean + 64.0);
    const int scap_max = (int)(room / (3 * sizeof(double)));
    if (scap > scap_max) scap = scap_max;
    scap = scap / 64 * 64;
    k.scap = scap < 64 ? 64 : scap;
    // with a second 3-vector per staged atom (adjoint, third-law forces)
    int aux = (int)(room / (6 * sizeof(double)));
    aux = (aux < k.scap ? aux : k.scap) / 64 * 64;
    k.scap_aux = aux < 64 ? 64 : aux;
    if (k.pipeline == MD_PIPE_LAYERS)
        k.nblk_force = (k.n + k.block - 1) / k.block;
    else if (k.pipeline == MD_PIPE_ALLPAIRS)
        k.nblk_force = allpairs_home_blocks(k.n) * k.ap_split;
    else
        k.nblk_force = force_blocks(k);
    // list build: a lane per home atom of a mean tile (25% spare), or waves
    // taking the home cells in turn: 8 waves from 8 home cells on, else 4 (a
    // multiple of the CU's four SIMDs measured best: 6 or 12 waves for 12
    // cells were 28-35% slower than 8 or 4)
    k.nl_method = c->nl_method_req != MD_NL_AUTO ? c->nl_method_req
                                                 : (occ < 8.0 ? MD_NL_LANES : MD_NL_CELL_WAVES);
    const int home_cells = k.kx_max * k.ky_max * k.kz_max;
    int waves;
    if (k.nl_method == MD_NL_LANES) {
        waves = (int)ceil(1.25 * home_cells * occ / kWave);
        waves = waves > 16 ? 16 : waves;
    } else {
        waves = home_cells >= 8 ? 8 : (home_cells >= 4 ? 4 : home_cells);
    }
    waves = waves < 1 ? 1 : waves;
    const int nlb = c->nl_block_req > 0 ? c->nl_block_req : kWave * waves;
    k.nl_block = nlb < kWave ? kWave : (nlb > 1024 ? 1024 : nlb);
}

void replan_tiles(md_ctx* c) { plan_tiles(c); }

static md_status hip_ok(hipError_t e) { return e == hipSuccess ? MD_OK : MD_ERR_HIP; }

// Offsets of the workspace regions from their sizes.
static void relayout(md_ctx* c)
{
    size_t o = 0;
    for (int r = 0; r < R_COUNT; ++r) {
        c->off[r] = o;
        o += align_up(c->bytes[r]);
    }
    c->ws_bytes = o;
}

static md_status launched() { return hip_ok(hipGetLastError()); }

static void drop_graph(md_ctx* c);  // md_step's captured graph (below)

extern "C" md_status md_init(const md_params* in, md_ctx** out)
{
    if (!in || !out) return MD_ERR_ARG;
    *out = nullptr;
    md_params p = *in;
    if (p.block == 0) p.block = 256;
    const bool finite = isfinite(p.L) && isfinite(p.eps) && isfinite(p.sigma) &&
                        isfinite(p.mass) && isfinite(p.r_cut) && isfinite(p.skin) &&
                        isfinite(p.dt);
    if (!finite || p.n_atoms < 1 || p.L <= 0 || p.eps <= 0 || p.sigma <= 0 || p.mass <= 0 ||
        p.r_cut <= 0 || p.skin < 0 || p.dt <= 0)
        return MD_ERR_ARG;
    if ((p.potential != MD_LJ_SHIFTED && p.potential != MD_LJ_TRUNC) ||
        (p.precision != MD_FP64 && p.precision != MD_FP32_MIXED) ||
        (p.mode != MD_CELLS_ONLY && p.mode != MD_NEIGHBOR_LIST) ||
        (p.newton3 != 0 && p.newton3 != 1) || (p.newton3 && p.mode != MD_NEIGHBOR_LIST) ||
        (p.pipeline != MD_PIPE_TILED && p.pipeline != MD_PIPE_LAYERS &&
         p.pipeline != MD_PIPE_ALLPAIRS) ||
        (p.pipeline == MD_PIPE_LAYERS && (p.mode != MD_NEIGHBOR_LIST || p.newton3 != 0)) ||
        (p.pipeline == MD_PIPE_ALLPAIRS && (p.mode != MD_CELLS_ONLY || p.reorder != 0)) ||
        p.nl_capacity < 0 || p.reorder < 0 ||
        (p.pipeline != MD_PIPE_LAYERS && p.reorder > 1) || p.block % 64 != 0 ||
        p.block < 64 || p.block > 1024)
        return MD_ERR_ARG;

    const bool nl = p.mode == MD_NEIGHBOR_LIST;
    const double r_list = p.r_cut + p.skin;
    const double r_cell = nl ? r_list : p.r_cut;
    double ncd = floor(p.L / r_cell);
    if (ncd > 1290) ncd = 1290;  // keeps nc^3 within int32
    int nc = (int)ncd;
    if (nc >= 1 && p.L / nc < r_cell) --nc;
    if (nc < 3) return MD_ERR_BOX_TOO_SMALL;

    md_ctx* c = new (std::nothrow) md_ctx();
    if (!c) return MD_ERR_ARG;
    c->prm = p;
    c->graph_on = false;  // md_set_graph
    const int64_t n = p.n_atoms;
    const int npad = (int)((n + 63) / 64 * 64);
    int cap = 0;
    if (nl) {
        if (p.nl_capacity > 0) {
            cap = p.nl_capacity;
        } else {
            const double rho = (double)n / (p.L * p.L * p.L);
            const double mean = 4.0 / 3.0 * M_PI * r_list * r_list * r_list * rho;
            cap = (int)ceil(mean + 10.0 * sqrt(mean) + 16.0);
            cap = (cap + 7) / 8 * 8;
        }
        if (cap > n - 1) cap = (int)(n - 1 > 0 ? n - 1 : 1);
        cap = (cap + 3) / 4 * 4;  // whole 4-entry chunks
    }
    c->geo.nc = nc;
    c->geo.n_cells = nc * nc * nc;
    c->geo.nl_capacity = cap;
    c->geo.n_pad = npad;
    c->geo.cell_width = p.L / nc;
    // layers per cell of the layer matrix: the mean occupancy plus six of its
    // Poisson standard deviations plus 8 (overflow is latched, not silent)
    int n_layers = 0;
    if (p.pipeline == MD_PIPE_LAYERS) {
        const double occ = (double)p.n_atoms / ((double)nc * nc * nc);
        n_layers = (int)ceil(occ + 6.0 * sqrt(occ) + 8.0);
    }
    c->geo.n_layers = n_layers;
    // all-pairs: partner chunks per 64-atom home block
    int ap_split = 0, ap_chunk = 0;
    if (p.pipeline == MD_PIPE_ALLPAIRS) allpairs_split(p.n_atoms, &ap_split, &ap_chunk);
    const int64_t ap_blocks = ap_split > 0 ? (int64_t)allpairs_home_blocks(p.n_atoms) * ap_split : 0;

    // workspace layout
    const int64_t ncell = (int64_t)nc * nc * nc;
    const size_t fsz = p.precision == MD_FP64 ? sizeof(double) : sizeof(float);
    size_t* b = c->bytes;
    b[R_DEV] = sizeof(DevState);
    b[R_CELL_COUNT] = sizeof(int32_t) * ncell;
    b[R_CELL_START] = sizeof(int32_t) * (ncell + 1);
    b[R_CELL_OF] = b[R_SLOT] = b[R_ORDER] = sizeof(int32_t) * n;
    b[R_TMP] = 2 * sizeof(int32_t) * n;  // slot -> atom, then slot -> permanent id
    const bool layers = p.pipeline == MD_PIPE_LAYERS;
    // plus one chunk row past the list: the cell-wave build writes entries
    // beyond the capacity there instead of testing each store (overflow is
    // counted and latched all the same)
    b[R_NL] = layers ? 0 : sizeof(uint16_t) * (size_t)(cap + kChunk) * npad;
    b[R_LAYERS] = sizeof(int32_t) * (size_t)ncell * n_layers;
    b[R_W32] = layers ? sizeof(int32_t) * (size_t)cap * npad : 0;
    b[R_NL_COUNT] = sizeof(int32_t) * npad;
    b[R_XR] = b[R_YR] = b[R_ZR] = nl ? sizeof(double) * n : 0;
    const size_t perm = p.reorder ? 1 : 0;
    b[R_SX] = b[R_SY] = b[R_SZ] = b[R_SVX] = b[R_SVY] = b[R_SVZ] = perm * sizeof(double) * n;
    b[R_SFX] = b[R_SFY] = b[R_SFZ] = perm * fsz * n;
    b[R_SID] = b[R_SCELL] = perm * sizeof(int32_t) * n;
    b[R_APART] = ap_split > 1 ? fsz * 3 * (size_t)ap_split * npad : 0;
    const int64_t fblocks = max_force_blocks(n, ncell);
    b[R_FPART] = sizeof(double) * 2 * (size_t)(ap_blocks > fblocks ? ap_blocks : fblocks);
    b[R_IPART] = sizeof(double) * 8 * kIntegrateGridMax;
    b[R_HIST] = sizeof(md_record) * kHistCap;
    relayout(c);

    KParams& k = c->kp;
    memset(&k, 0, sizeof(k));
    k.n = (int)n;
    k.npad = npad;
    k.nc = nc;
    k.ncell = (int)ncell;
    k.cap = cap;
    k.potential = p.potential;
    k.precision = p.precision;
    k.mode = p.mode;
    k.reorder = p.reorder;
    k.newton3 = p.newton3;
    k.pipeline = p.pipeline;
    k.n_layers = n_layers;
    k.ap_split = ap_split;
    k.ap_chunk = ap_chunk;
    k.L = p.L;
    k.invL = 1.0 / p.L;
    k.inv_w = (double)nc / p.L;
    k.rc2 = p.r_cut * p.r_cut;
    k.rl2 = r_list * r_list;
    k.sig2 = p.sigma * p.sigma;
    k.eps2 = 2.0 * p.eps;
    k.eps48 = 48.0 * p.eps;
    k.eps = p.eps;
    k.sigma = p.sigma;
    double shift = 0.0;
    if (p.potential == MD_LJ_SHIFTED) {
        const double sr2 = k.sig2 / k.rc2, sr6 = sr2 * sr2 * sr2;
        shift = 4.0 * p.eps * (sr6 * sr6 - sr6);
    }
    k.half_shift = 0.5 * shift;
    k.ushift = k.half_shift / k.eps2;
    k.ushift2 = 2.0 * k.ushift;
    k.hdt = (0.5 * p.dt) / p.mass;
    k.dt = p.dt;
    k.disp_thr2 = (0.5 * p.skin) * (0.5 * p.skin);
    k.mass = p.mass;
    // the minimum-image shortcut of the force pass needs partners closer than L/2
    const double reach = r_list + p.skin;
    if (nl && 2.0 * reach < 0.999 * p.L) {
        k.inner_lo = reach;
        k.inner_hi = p.L - reach;
    } else {
        k.inner_lo = 1.0;
        k.inner_hi = 0.0;  // empty range: always take the minimum image
    }
    k.block = p.block;
    // 2 lanes per atom (2.048 M-atom LJ, 512-thread workgroups: FP64 force pass
    // 255 us at 2 lanes, 267 at 4, 356 at 8; FP32-mixed 228, 244, 324)
    k.force_lanes = 2;
    k.force_block = 512;
    c->nl_block_req = 0;
    k.int_grid = kIntegrateGridDefault;
    k.gate_grid = kGateGridDefault;
    plan_tiles(c);
    *out = c;
    return MD_OK;
}

extern "C" size_t md_workspace_bytes(const md_ctx* c) { return c ? c->ws_bytes : 0; }

extern "C" md_status md_set_bonded(md_ctx* c, const md_bonded* b)
{
    if (!c) return MD_ERR_ARG;
    if (c->bound) return MD_ERR_STATE;
    KParams& k = c->kp;
    if (!b) {
        k.bonded_on = 0;
        c->bytes[R_SLOT_OF] = c->bytes[R_BPART] = 0;
        relayout(c);
        return MD_OK;
    }
    const bool finite = isfinite(b->fene_k) && isfinite(b->fene_r0) && isfinite(b->bend_k) &&
                        isfinite(b->tors_c[0]) && isfinite(b->tors_c[1]) &&
                        isfinite(b->tors_c[2]) && isfinite(b->tors_c[3]);
    if (!finite || b->chain_length < 2 || c->prm.n_atoms % b->chain_length != 0 ||
        !(b->fene_r0 > 0.0) || b->fene_k < 0.0)
        return MD_ERR_ARG;
    k.bonded_on = 1;
    k.chain_len = b->chain_length;
    k.fene_k = b->fene_k;
    k.fene_r02 = b->fene_r0 * b->fene_r0;
    k.bend_k = b->bend_k;
    for (int m = 0; m < 4; ++m) k.tors_c[m] = b->tors_c[m];
    k.tors_on = b->tors_c[0] != 0.0 || b->tors_c[1] != 0.0 || b->tors_c[2] != 0.0 ||
                b->tors_c[3] != 0.0;
    k.nblk_bonded = bonded_blocks(k.n);
    c->bytes[R_SLOT_OF] = sizeof(int32_t) * (size_t)k.n;
    c->bytes[R_BPART] = sizeof(double) * 2 * (size_t)k.nblk_bonded;
    relayout(c);
    return MD_OK;
}

extern "C" md_status md_geometry(const md_ctx* c, md_grid* out)
{
    if (!c || !out) return MD_ERR_ARG;
    *out = c->geo;
    return MD_OK;
}

extern "C" md_status md_layout(const md_ctx* c, int32_t which, size_t* offset, size_t* count)
{
    if (!c || !offset || !count) return MD_ERR_ARG;
    const int64_t n = c->prm.n_atoms;
    const bool layers = c->prm.pipeline == MD_PIPE_LAYERS;
    const bool allpairs = c->prm.pipeline == MD_PIPE_ALLPAIRS;
    switch (which) {
        case MD_ARR_CELL_OF:
            if (allpairs) return MD_ERR_ARG;
            *offset = c->off[R_CELL_OF];
            *count = n;
            break;
        case MD_ARR_CELL_START:
            if (layers || allpairs) return MD_ERR_ARG;
            *offset = c->off[R_CELL_START];
            *count = c->geo.n_cells + 1;
            break;
        case MD_ARR_CELL_ATOMS:
            if (layers || allpairs) return MD_ERR_ARG;
            *offset = c->off[R_ORDER];
            *count = n;
            break;
        case MD_ARR_NL:
            *offset = c->off[layers ? R_W32 : R_NL];
            *count = (size_t)c->geo.nl_capacity * c->geo.n_pad;
            break;
        case MD_ARR_LAYERS:
            if (!layers) return MD_ERR_ARG;
            *offset = c->off[R_LAYERS];
            *count = (size_t)c->geo.n_cells * c->geo.n_layers;
            break;
        case MD_ARR_LAYER_COUNT:
            if (!layers) return MD_ERR_ARG;
            *offset = c->off[R_CELL_COUNT];
            *count = c->geo.n_cells;
            break;
        case MD_ARR_NL_COUNT: *offset = c->off[R_NL_COUNT]; *count = n; break;
        case MD_ARR_XREF:
            if (c->prm.mode != MD_NEIGHBOR_LIST) return MD_ERR_ARG;
            *offset = c->off[R_XR];  // x, y, z references follow at 256-byte-aligned pitch
            *count = n;
            break;
        default: return MD_ERR_ARG;
    }
    return MD_OK;
}

static bool state_buffers_ok(const md_buffers* bf)
{
    return bf->x && bf->y && bf->z && bf->vx && bf->vy && bf->vz && bf->fx && bf->fy &&
           bf->fz && bf->id;
}

// Points the kernel parameters at the caller's state arrays and at the
// workspace regions inside ws, binds the stream, plans the tiles and
// enqueues the clearing of the device counters.
static md_status bind_to(md_ctx* c, const md_buffers* bf, char* ws, void* stream)
{
    KParams& k = c->kp;
    drop_graph(c);  // the pointers are baked into it
    auto at = [&](int r) -> void* { return c->bytes[r] ? ws + c->off[r] : nullptr; };
    k.x = bf->x; k.y = bf->y; k.z = bf->z;
    k.vx = bf->vx; k.vy = bf->vy; k.vz = bf->vz;
    k.fx = bf->fx; k.fy = bf->fy; k.fz = bf->fz;
    k.id = bf->id;
    k.dev = static_cast<DevState*>(at(R_DEV));
    k.cell_count = static_cast<int32_t*>(at(R_CELL_COUNT));
    k.cell_start = static_cast<int32_t*>(at(R_CELL_START));
    k.cell_of = static_cast<int32_t*>(at(R_CELL_OF));
    k.slot = static_cast<int32_t*>(at(R_SLOT));
    k.order = static_cast<int32_t*>(at(R_ORDER));
    k.tmp = static_cast<int32_t*>(at(R_TMP));
    k.nl64 = static_cast<uint64_t*>(at(R_NL));
    k.nl_count = static_cast<int32_t*>(at(R_NL_COUNT));
    k.xr = static_cast<double*>(at(R_XR));
    k.yr = static_cast<double*>(at(R_YR));
    k.zr = static_cast<double*>(at(R_ZR));
    k.sx = static_cast<double*>(at(R_SX));
    k.sy = static_cast<double*>(at(R_SY));
    k.sz = static_cast<double*>(at(R_SZ));
    k.svx = static_cast<double*>(at(R_SVX));
    k.svy = static_cast<double*>(at(R_SVY));
    k.svz = static_cast<double*>(at(R_SVZ));
    k.sfx = static_cast<double*>(at(R_SFX));
    k.sfy = static_cast<double*>(at(R_SFY));
    k.sfz = static_cast<double*>(at(R_SFZ));
    k.sid = static_cast<int32_t*>(at(R_SID));
    k.layers = static_cast<int32_t*>(at(R_LAYERS));
    k.w32 = static_cast<int32_t*>(at(R_W32));
    k.apart = at(R_APART);
    k.slot_of = static_cast<int32_t*>(at(R_SLOT_OF));
    k.bpart = static_cast<double*>(at(R_BPART));
    k.scell = static_cast<int32_t*>(at(R_SCELL));
    k.fpart = static_cast<double*>(at(R_FPART));
    k.ipart = static_cast<double*>(at(R_IPART));
    k.hist = static_cast<md_record*>(at(R_HIST));
    c->stream = static_cast<hipStream_t>(stream);
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return MD_ERR_HIP;
    c->lds_limit = (size_t)lds;
    plan_tiles(c);
    c->bound = true;
    c->host_steps = 0;
    c->cells_ok = c->nl_ok = c->forces_ok = false;
    launch_clear(k, c->stream);
    return launched();
}

extern "C" md_status md_bind(md_ctx* c, const md_buffers* bf, void* stream)
{
    if (!c || !bf) return MD_ERR_ARG;
    if (!state_buffers_ok(bf) || !bf->workspace) return MD_ERR_ARG;
    if (((uintptr_t)bf->workspace) % kAlign != 0) return MD_ERR_ARG;
    return bind_to(c, bf, static_cast<char*>(bf->workspace), stream);
}

// ---- binding to the library's own workspace (no allocation) ----
//
// One static device array per GPU holds the workspace of contexts bound
// with md_bind_static.  In host code the array's name stands for a host
// shadow, not for device memory, so its device address is looked up once
// per device (with that device current) and only that address is used.

static __device__ __align__(256) unsigned char scratch[MD_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of scratch on each device
}  // namespace

static md_status static_workspace(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MD_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return MD_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return MD_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MD_OK;
}

extern "C" md_status md_bind_static(md_ctx* c, const md_buffers* bf, void* stream)
{
    if (!c || !bf) return MD_ERR_ARG;
    if (!state_buffers_ok(bf) || bf->workspace) return MD_ERR_ARG;
    if (c->ws_bytes > (size_t)MD_STATIC_WORKSPACE_BYTES) return MD_ERR_WORKSPACE_TOO_LARGE;
    void* ws = nullptr;
    md_status st = static_workspace(&ws);
    if (st != MD_OK) return st;
    // a caller-supplied workspace starts zeroed; so does this one, whatever
    // an earlier binding left in it (a fill kernel, not a memset node, so the
    // call may sit in a captured graph)
    launch_fill(static_cast<double*>(ws), c->ws_bytes / sizeof(double), 0.0,
                static_cast<hipStream_t>(stream));
    st = launched();
    if (st != MD_OK) return st;
    return bind_to(c, bf, static_cast<char*>(ws), stream);
}

// The stages of either pipeline.
// flags: bit 0 forces the build; the tiled cell build also takes kFoldCopy,
// kFoldBin and kSortSmallOk (md_internal.h).
static void cells_any(const KParams& k, int flags, hipStream_t s)
{
    const int force = flags & 1;
    if (k.pipeline == MD_PIPE_LAYERS)
        launch_layer_cells(k, force, s);
    else if (k.pipeline == MD_PIPE_ALLPAIRS) {
        if (force) launch_allpairs_fold(k, s);  // in a step the drift folds
    } else
        launch_cells(k, flags, s);
    if (k.bonded_on) launch_bond_map(k, force, s);  // after any permutation of the slots
}

static void neighbors_any(const KParams& k, int force, hipStream_t s)
{
    if (k.pipeline == MD_PIPE_LAYERS)
        launch_layer_nl(k, force, s);
    else
        launch_neighbors(k, force, s);
}

// flags: kFoldCopy for the tiled cells-only pass (md_internal.h).
static void forces_any(const KParams& k, hipStream_t s, int flags = 0)
{
    if (k.pipeline == MD_PIPE_LAYERS)
        launch_layer_forces(k, s);
    else if (k.pipeline == MD_PIPE_ALLPAIRS)
        launch_allpairs_forces(k, s);
    else
        launch_forces(k, s, flags);
    if (k.bonded_on) launch_bonded(k, s);  // adds to the pair forces
}

extern "C" md_status md_build_cells(md_ctx* c)
{
    if (!c) return MD_ERR_ARG;
    if (!c->bound) return MD_ERR_NOT_BOUND;
    cells_any(c->kp, 1, c->stream);
    c->cells_ok = true;
    c->nl_ok = false;
    c->forces_ok = false;
    return launched();
}

extern "C" md_status md_build_neighbors(md_ctx* c)
{
    if (!c) return MD_ERR_ARG;
    if (!c->bound) return MD_ERR_NOT_BOUND;
    if (c->prm.mode != MD_NEIGHBOR_LIST) return MD_ERR_ARG;
    if (!c->cells_ok) return MD_ERR_STATE;
    neighbors_any(c->kp, 1, c->stream);
    c->nl_ok = true;
    return launched();
}

// Launches fn on the bound stream; with timing on, between two events
// counted toward part (MD_PART_*).
template <class Fn>
static void timed(md_ctx* c, int part, Fn&& fn)
{
    if (!c->timing) {
        fn();
        return;
    }
    hipEvent_t ev[2];
    for (int k = 0; k < 2; ++k) {
        if (!c->ev_free.empty()) {
            ev[k] = c->ev_free.back();
            c->ev_free.pop_back();
        } else {
            (void)hipEventCreate(&ev[k]);
        }
    }
    (void)hipEventRecord(ev[0], c->stream);
    fn();
    (void)hipEventRecord(ev[1], c->stream);
    c->ev_pending.push_back(ev[0]);
    c->ev_pending.push_back(ev[1]);
    c->ev_part.push_back(part);
}

static void timed_forces(md_ctx* c, int flags = 0)
{
    timed(c, MD_PART_FORCES, [&] { forces_any(c->kp, c->stream, flags); });
}

static md_status fold_timing(md_ctx* c)
{
    if (c->ev_pending.empty()) return MD_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MD_ERR_HIP;
    for (size_t k = 0; k + 1 < c->ev_pending.size(); k += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev_pending[k], c->ev_pending[k + 1]) != hipSuccess)
            return MD_ERR_HIP;
        const int part = c->ev_part[k / 2];
        if (part == MD_PART_FORCES) {
            c->timed_ms += ms;
            c->timed_launches += 1;
        }
        c->part_ms[part] += ms;
        c->part_launches[part] += 1;
        c->ev_free.push_back(c->ev_pending[k]);
        c->ev_free.push_back(c->ev_pending[k + 1]);
    }
    c->ev_pending.clear();
    c->ev_part.clear();
    return MD_OK;
}

extern "C" md_status md_export_neighbors(md_ctx* c, int32_t* dst)
{
    if (!c || !dst) return MD_ERR_ARG;
    if (!c->bound) return MD_ERR_NOT_BOUND;
    if (c->prm.mode != MD_NEIGHBOR_LIST) return MD_ERR_ARG;
    if (!c->nl_ok) return MD_ERR_STATE;
    if (c->kp.pipeline == MD_PIPE_LAYERS)
        launch_layer_export(c->kp, dst, c->stream);
    else
        launch_nl_export(c->kp, dst, c->stream);
    return launched();
}

extern "C" md_status md_forces(md_ctx* c)
{
    if (!c) return MD_ERR_ARG;
    if (!c->bound) return MD_ERR_NOT_BOUND;
    if (!c->cells_ok || (c->prm.mode == MD_NEIGHBOR_LIST && !c->nl_ok)) return MD_ERR_STATE;
    timed_forces(c);
    c->forces_ok = true;
    return launched();
}

// ---- md_step ----
//
// A step is a fixed launch sequence (integrate, the rebuild-gated cell and
// list kernels, forces), so runs of kGraphSteps steps can be captured once
// into a HIP graph and replayed (md_set_graph), for callers that need the
// step as a graph.  It is off by default: with the present launch sequence
// (an integration pass and its one-workgroup finish, the gated cell and list
// kernels, the force pass) direct launches measured faster on MI355X at
// every size tried, 9-20% per step for 4000 to 131 072 atoms (4000-atom WCA
// cells-only 29.7 against 32.4 us, 32 000-atom LJ 38.2 against 45.9 us).
// The first step of a call (its integrate kernel
// only kicks and drifts) and the remainder are launched directly.  A call of
// fewer than kGraphSteps + 1 steps (but at least kGraphMin + 1) replays one
// graph of its own length instead, so that repeated short calls (the
// adjoint's forward segments) are captured too; the graph is recaptured when
// the length changes.  Timing (md_set_timing) brackets each force launch with
// events and uses the direct path throughout.

constexpr int kGraphSteps = 32;
constexpr int kGraphMin = 8;

static void drop_graph(md_ctx* c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->g_record = -1;
    c->g_len = 0;
    c->g_run = nullptr;
}

// The layer pipeline's periodic reorder (md_params.reorder = k > 0): due
// before the force pass of every k-th step.
static bool layer_reorder_on(const md_ctx* c)
{
    return c->kp.pipeline == MD_PIPE_LAYERS && c->kp.reorder > 0;
}

// Launches of n steps, the first of them step step0 + 1 since md_bind;
// first: it is the first step of the run.
static md_status step_launches(md_ctx* c, hipStream_t s, bool first, int32_t n,
                               int32_t record_every, int64_t step0)
{
    const KParams& k = c->kp;
    const bool nl = c->prm.mode == MD_NEIGHBOR_LIST;
    const bool tiled = k.pipeline == MD_PIPE_TILED;
    // the reorder's copy-back folded into the pass after the cell build (the
    // list build, or the cells-only force pass)
    const int fold = tiled && k.reorder && !k.bonded_on ? kFoldCopy : 0;
    // cells only: the cells are rebuilt every step, so the integration pass
    // bins the atoms and a small system sorts them in one workgroup
    const bool cells = tiled && !nl;
    const int cflags = fold | (cells ? kFoldBin | kSortSmallOk : 0);
    const int fflags = cells ? fold : 0;
    // a small cells-only system finishes the integration pass inside its one
    // cell-sort workgroup (one launch less)
    const bool small = cells && k.n <= kSortSmall && !k.bonded_on;
    auto finish_and_cells = [&](int phase) {
        if (small) {
            launch_sort_small_finish(k, phase, record_every, s);
        } else {
            launch_integrate_finish(k, phase, record_every, s);
            cells_any(k, cflags, s);
        }
    };
    if (s != c->stream) {  // captured into a graph: never timed, never reordered
        for (int32_t i = 0; i < n; ++i) {
            const int phase = first && i == 0 ? 0 : 1;
            launch_integrate_pass(k, phase, record_every, s, cells);
            finish_and_cells(phase);
            if (nl) neighbors_any(k, fold, s);
            forces_any(k, s, fflags);
        }
        return MD_OK;
    }
    for (int32_t i = 0; i < n; ++i) {
        const int phase = first && i == 0 ? 0 : 1;
        timed(c, MD_PART_INTEGRATE,
              [&] { launch_integrate_pass(k, phase, record_every, s, cells); });
        const bool reorder = layer_reorder_on(c) && (step0 + i + 1) % k.reorder == 0;
        if (small) {  // the finish and the cell build in one launch (counted as cells)
            timed(c, MD_PART_CELLS, [&] { finish_and_cells(phase); });
        } else {
            timed(c, MD_PART_ENERGY, [&] { launch_integrate_finish(k, phase, record_every, s); });
            if (reorder) timed(c, MD_PART_REORDER, [&] { launch_layer_reorder(k, s); });
            timed(c, MD_PART_CELLS, [&] { cells_any(k, reorder ? 1 : cflags, s); });
        }
        if (nl) timed(c, MD_PART_NEIGHBORS, [&] { neighbors_any(k, reorder ? 1 : fold, s); });
        timed_forces(c, fflags);
        if (c->timing && c->ev_pending.size() >= 8192) {
            md_status st = fold_timing(c);
            if (st != MD_OK) return st;
        }
    }
    return MD_OK;
}

// n_graphs replays of the graph of len steps, captured first if needed.
// The null stream cannot be captured: then the graph runs on the context's own
// stream, ordered after and before the bound stream's work by events.
static md_status step_graphs(md_ctx* c, int32_t len, int32_t n_graphs, int32_t record_every)
{
    hipStream_t run = c->stream;
    const bool own = run == nullptr;
    if (own) {
        if (!c->gstream &&
            hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess)
            return MD_ERR_HIP;
        for (int e = 0; e < 2; ++e)
            if (!c->gev[e] &&
                hipEventCreateWithFlags(&c->gev[e], hipEventDisableTiming) != hipSuccess)
                return MD_ERR_HIP;
        run = c->gstream;
    }
    if (!(c->gexec && c->g_record == record_every && c->g_run == run && c->g_len == len)) {
        drop_graph(c);
        if (hipStreamBeginCapture(run, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return MD_ERR_HIP;
        const md_status st = step_launches(c, run, false, len, record_every, 0);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(run, &g);
        if (st != MD_OK) return st;
        if (ec != hipSuccess || !g) return MD_ERR_HIP;
        c->graph = g;
        if (hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(c);
            return MD_ERR_HIP;
        }
        c->g_record = record_every;
        c->g_len = len;
        c->g_run = run;
    }
    if (own && (hipEventRecord(c->gev[0], c->stream) != hipSuccess ||
                hipStreamWaitEvent(run, c->gev[0], 0) != hipSuccess))
        return MD_ERR_HIP;
    for (int32_t g = 0; g < n_graphs; ++g)
        if (hipGraphLaunch(c->gexec, run) != hipSuccess) return MD_ERR_HIP;
    if (own && (hipEventRecord(c->gev[1], run) != hipSuccess ||
                hipStreamWaitEvent(c->stream, c->gev[1], 0) != hipSuccess))
        return MD_ERR_HIP;
    return MD_OK;
}

extern "C" md_status md_step(md_ctx* c, int32_t n_steps, int32_t record_every)
{
    if (!c || n_steps < 0 || record_every < 0) return MD_ERR_ARG;
    if (!c->bound) return MD_ERR_NOT_BOUND;
    if (!c->forces_ok) return MD_ERR_STATE;
    if (n_steps == 0) return MD_OK;
    md_status st;
    const int64_t step0 = c->host_steps;
    if (c->timing || !c->graph_on || layer_reorder_on(c) || n_steps <= kGraphMin) {
        st = step_launches(c, c->stream, true, n_steps, record_every, step0);
    } else {
        const int32_t rest = n_steps - 1;
        const int32_t len = rest < kGraphSteps ? rest : kGraphSteps, n_graphs = rest / len;
        st = step_launches(c, c->stream, true, 1, record_every, step0);
        if (st == MD_OK) st = step_graphs(c, len, n_graphs, record_every);
        if (st == MD_OK)
            st = step_launches(c, c->stream, false, rest - n_graphs * len, record_every,
                               step0 + 1 + (int64_t)n_graphs * len);
    }
    c->host_steps = step0 + n_steps;
    if (st != MD_OK) return st;
    launch_integrate(c->kp, 2, record_every, c->stream);
    return launched();
}

extern "C" md_status md_set_graph(md_ctx* c, int32_t enable)
{
    if (!c) return MD_ERR_ARG;
    c->graph_on = enable != 0;
    if (!c->graph_on) drop_graph(c);
    return MD_OK;
}

extern "C" md_status md_reduce(md_ctx* c, md_observables* out)
{
    if (!c || !out) return MD_ERR_ARG;
    if (!c->bound) return MD_ERR_NOT_BOUND;
    launch_observe(c->kp, c->stream);
    md_status st = launched();
    if (st != MD_OK) return st;
    DevState d;
    if (hipMemcpyAsync(&d, c->kp.dev, sizeof(d), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return MD_ERR_HIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MD_ERR_HIP;
    const double n = c->prm.n_atoms;
    const double V = c->prm.L * c->prm.L * c->prm.L;
    memset(out, 0, sizeof(*out));
    out->U = d.obs[0];
    out->K = d.obs[1];
    out->W = d.obs[2];
    out->P[0] = d.obs[3];
    out->P[1] = d.obs[4];
    out->P[2] = d.obs[5];
    out->T = n > 1 ? 2.0 * out->K / (3.0 * (n - 1)) : 0.0;
    out->pressure = (2.0 * out->K + out->W) / (3.0 * V);
    out->dmax = sqrt(d.dmax2);
    out->step = d.step;
    out->n_rebuilds = d.n_rebuilds;
    out->max_occupancy = d.max_occ;
    out->max_nl = d.max_nl;
    out->flags = d.flags;
    if (d.flags & MD_FLAG_TOPOLOGY) return MD_ERR_TOPOLOGY;
    if (d.flags & MD_FLAG_BOND_BROKEN) return MD_ERR_BOND_BROKEN;
    if (d.flags & MD_FLAG_LAYER_OVERFLOW) return MD_ERR_LAYER_OVERFLOW;
    if (d.flags & MD_FLAG_NL_OVERFLOW) return MD_ERR_NL_OVERFLOW;
    if (d.flags & MD_FLAG_NONFINITE) return MD_ERR_NONFINITE;
    return MD_OK;
}

// ---- reverse mode ----

namespace {

constexpr int kTrajMaxBins = 1024;

// Byte offsets inside the trajectory workspace.  Every per-atom array has
// the same 256-byte-aligned pitch.
struct TrajLayout {
    int k;         // steps per segment
    int nseg;      // segments (one checkpoint each, plus the final state)
    size_t pitch;  // bytes of one per-atom double array
    size_t ck, snap, lam, theta, tpart, hist, total;
};

bool traj_layout(const md_ctx* c, const md_traj_params* tp, TrajLayout* L)
{
    if (!c || !tp) return false;
    if (tp->n_steps < 1 || tp->n_steps > kHistCap || tp->checkpoint_every < 1 ||
        tp->n_bins < 0 || tp->n_bins > kTrajMaxBins)
        return false;
    if (tp->n_bins > 0 && !(tp->gr_rmax > 0.0 && tp->gr_width > 0.0 && isfinite(tp->gr_rmax) &&
                            isfinite(tp->gr_width)))
        return false;
    const size_t n = (size_t)c->prm.n_atoms;
    L->k = tp->checkpoint_every < tp->n_steps ? tp->checkpoint_every : tp->n_steps;
    L->nseg = (tp->n_steps + L->k - 1) / L->k;
    L->pitch = align_up(sizeof(double) * n);
    size_t o = 0;
    L->ck = o;  // (x, y, z, vx, vy, vz) at the start of every segment and at the end
    o += (size_t)(L->nseg + 1) * 6 * L->pitch;
    L->snap = o;  // positions of the recomputed steps inside one segment
    o += (size_t)(L->k - 1) * 3 * L->pitch;
    L->lam = o;  // lambda_x, lambda_v (two buffers)
    o += 9 * L->pitch;
    L->theta = o;
    o += align_up(2 * sizeof(double));
    L->tpart = o;
    o += align_up(2 * sizeof(double) * (size_t)max_force_blocks(n, c->geo.n_cells));
    L->hist = o;
    o += align_up(sizeof(unsigned long long) * (size_t)(tp->n_bins > 0 ? tp->n_bins : 1));
    L->total = o;
    return true;
}

double* arr(void* ws, const TrajLayout& L, size_t off, size_t idx)
{
    return reinterpret_cast<double*>(static_cast<char*>(ws) + off + idx * L.pitch);
}

}  // namespace

static md_status traj_check(md_ctx* c, const md_traj_params* tp, void* ws, TrajLayout* L)
{
    if (!c || !tp || !ws || !traj_layout(c, tp, L)) return MD_ERR_ARG;
    if (!c->bound) return MD_ERR_NOT_BOUND;
    if (c->prm.mode != MD_NEIGHBOR_LIST || c->prm.reorder != 0 || c->prm.newton3 != 0 ||
        c->prm.pipeline != MD_PIPE_TILED || c->kp.bonded_on)
        return MD_ERR_ARG;
    if (((uintptr_t)ws) % kAlign != 0) return MD_ERR_ARG;
    if (tp->n_bins > 0 && tp->gr_rmax + 3.0 * tp->gr_width > c->prm.r_cut + c->prm.skin)
        return MD_ERR_ARG;
    return MD_OK;
}

static GrArgs gr_args(const md_ctx* c, const md_traj_params* tp, void* ws, const TrajLayout& L)
{
    GrArgs g;
    memset(&g, 0, sizeof(g));
    g.hist = reinterpret_cast<unsigned long long*>(static_cast<char*>(ws) + L.hist);
    g.n_bins = tp->n_bins;
    g.rmax = tp->gr_rmax;
    g.width = tp->gr_width;
    // fixed-point units: the largest possible bin sum (every atom, a full
    // list, each pair at the kernel's peak) stays below 2^62
    const double kmax = 1.0 / (tp->gr_width * sqrt(2.0 * M_PI));
    const double bound = (double)c->prm.n_atoms * (double)c->geo.nl_capacity * kmax;
    int e = (int)floor(log2(ldexp(1.0, 62) / (bound > 1.0 ? bound : 1.0)));
    g.scale = ldexp(1.0, e < 40 ? e : 40);
    return g;
}

// Copy the state (x, y, z, vx, vy, vz) to or from a checkpoint.
static md_status checkpoint(md_ctx* c, double* const* ck, bool save)
{
    const KParams& k = c->kp;
    double* st[6] = {k.x, k.y, k.z, k.vx, k.vy, k.vz};
    const size_t bytes = sizeof(double) * (size_t)c->prm.n_atoms;
    for (int a = 0; a < 6; ++a)
        if (hipMemcpyAsync(save ? ck[a] : st[a], save ? st[a] : ck[a], bytes,
                           hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
            return MD_ERR_HIP;
    return MD_OK;
}

static void checkpoint_arrays(void* ws, const TrajLayout& L, int seg, double** out)
{
    for (int a = 0; a < 6; ++a) out[a] = arr(ws, L, L.ck, (size_t)seg * 6 + a);
}

// Cells, list and forces from scratch at the current positions.
static void rebuild_all(md_ctx* c)
{
    launch_cells(c->kp, 1, c->stream);
    launch_neighbors(c->kp, 1, c->stream);
    launch_forces(c->kp, c->stream);
    c->cells_ok = c->nl_ok = c->forces_ok = true;
}

extern "C" size_t md_traj_workspace_bytes(const md_ctx* c, const md_traj_params* tp)
{
    TrajLayout L;
    return traj_layout(c, tp, &L) ? L.total : 0;
}

extern "C" md_status md_traj_forward(md_ctx* c, const md_traj_params* tp, void* ws, double* obs)
{
    TrajLayout L;
    md_status st = traj_check(c, tp, ws, &L);
    if (st != MD_OK) return st;
    if (!obs) return MD_ERR_ARG;
    if (!c->forces_ok) rebuild_all(c);
    double* ck[6];
    // the segments launch directly: on a system made for one trajectory (the
    // usual case, since eps and sigma are fixed at md_init) capturing a graph
    // of the segment cost more than its replays saved (measured on MI355X at
    // 32 000 atoms and 20-step segments: 59 against 49 us per step)
    const bool graph_on = c->graph_on;
    c->graph_on = false;
    for (int seg = 0; seg < L.nseg && st == MD_OK; ++seg) {
        checkpoint_arrays(ws, L, seg, ck);
        if ((st = checkpoint(c, ck, true)) != MD_OK) break;
        const int m = tp->n_steps - seg * L.k < L.k ? tp->n_steps - seg * L.k : L.k;
        st = md_step(c, m, 1);
    }
    c->graph_on = graph_on;
    if (st != MD_OK) return st;
    checkpoint_arrays(ws, L, L.nseg, ck);
    if ((st = checkpoint(c, ck, true)) != MD_OK) return st;
    launch_traj_ubar(c->kp, tp->n_steps, obs, c->stream);
    if (tp->n_bins > 0) {
        // a list built steps ago holds every pair only out to r_cut; the g(r)
        // range may reach r_cut + skin, so build it afresh at x_S
        rebuild_all(c);
        GrArgs g = gr_args(c, tp, ws, L);
        g.out = obs + 1;
        launch_gr(c->kp, g, c->stream);
    }
    return launched();
}

extern "C" md_status md_traj_backward(md_ctx* c, const md_traj_params* tp, void* ws,
                                      const double* grad_obs, double* grad_x0, double* grad_v0,
                                      double* grad_theta)
{
    TrajLayout L;
    md_status st = traj_check(c, tp, ws, &L);
    if (st != MD_OK) return st;
    if (!grad_obs || !grad_x0 || !grad_v0 || !grad_theta) return MD_ERR_ARG;
    const KParams& k = c->kp;
    hipStream_t sm = c->stream;
    const int S = tp->n_steps;
    const size_t n = (size_t)c->prm.n_atoms;
    double* lam[3] = {arr(ws, L, L.lam, 0), arr(ws, L, L.lam, 1), arr(ws, L, L.lam, 2)};
    double* vbuf[2][3] = {{arr(ws, L, L.lam, 3), arr(ws, L, L.lam, 4), arr(ws, L, L.lam, 5)},
                          {arr(ws, L, L.lam, 6), arr(ws, L, L.lam, 7), arr(ws, L, L.lam, 8)}};
    double* theta = reinterpret_cast<double*>(static_cast<char*>(ws) + L.theta);
    AdjArgs a;
    memset(&a, 0, sizeof(a));
    a.lx = lam[0];
    a.ly = lam[1];
    a.lz = lam[2];
    a.theta = theta;
    a.tpart = reinterpret_cast<double*>(static_cast<char*>(ws) + L.tpart);
    a.gobs = grad_obs;
    a.cap = k.scap_aux;
    int cur = 0;
    // one point: lambda_v of buffer cur in, of the other buffer out
    auto point = [&](double coef, double loss_scale, double drift) {
        a.vx = vbuf[cur][0];
        a.vy = vbuf[cur][1];
        a.vz = vbuf[cur][2];
        a.nx = vbuf[1 - cur][0];
        a.ny = vbuf[1 - cur][1];
        a.nz = vbuf[1 - cur][2];
        a.coef = coef;
        a.loss_scale = loss_scale;
        a.drift = drift;
        launch_adj_point(k, a, sm);
        cur = 1 - cur;
    };
    const double half = k.hdt;  // dt / 2m: one half kick
    const double lscale = 1.0 / ((double)S * (double)n);
    launch_fill(theta, 2, 0.0, sm);
    for (int d = 0; d < 3; ++d) launch_fill(vbuf[0][d], n, 0.0, sm);

    // the last point: the observables' direct dependence on x_S
    double* ck[6];
    checkpoint_arrays(ws, L, L.nseg, ck);
    launch_adj_reimage(k, ck[0], ck[1], ck[2], sm);
    launch_cells(k, 1, sm);
    launch_neighbors(k, 1, sm);
    if (tp->n_bins > 0) {
        GrArgs g = gr_args(c, tp, ws, L);
        g.gobs = grad_obs;
        g.lx = lam[0];
        g.ly = lam[1];
        g.lz = lam[2];
        launch_gr_grad(k, g, sm);
    } else {
        for (int d = 0; d < 3; ++d) launch_fill(lam[d], n, 0.0, sm);
    }
    point(0.0, lscale, k.dt);

    for (int seg = L.nseg - 1; seg >= 0; --seg) {
        const int s0 = seg * L.k;
        const int s1 = s0 + L.k < S ? s0 + L.k : S;
        // recompute the segment, keeping the positions of its inner points
        checkpoint_arrays(ws, L, seg, ck);
        if ((st = checkpoint(c, ck, false)) != MD_OK) return st;
        rebuild_all(c);
        for (int j = 1; j < s1 - s0; ++j) {
            launch_integrate(k, j == 1 ? 0 : 1, 0, sm);
            launch_cells(k, 0, sm);
            launch_neighbors(k, 0, sm);
            launch_forces(k, sm);
            for (int d = 0; d < 3; ++d)
                if (hipMemcpyAsync(arr(ws, L, L.snap, (size_t)(j - 1) * 3 + d),
                                   d == 0 ? k.x : (d == 1 ? k.y : k.z), sizeof(double) * n,
                                   hipMemcpyDeviceToDevice, sm) != hipSuccess)
                    return MD_ERR_HIP;
        }
        // walk it backwards
        for (int s = s1 - 1; s >= s0; --s) {
            const double* px[3];
            for (int d = 0; d < 3; ++d)
                px[d] = s == s0 ? ck[d] : arr(ws, L, L.snap, (size_t)(s - s0 - 1) * 3 + d);
            launch_adj_reimage(k, px[0], px[1], px[2], sm);
            launch_cells(k, 0, sm);
            launch_neighbors(k, 0, sm);
            // the first half kick of step s and the second of step s-1 (none
            // before step 0) act together; the mean energy counts x_1 .. x_S
            point(s == 0 ? half : 2.0 * half, s >= 1 ? lscale : 0.0, s >= 1 ? k.dt : 0.0);
        }
    }
    for (int d = 0; d < 3; ++d) {
        if (hipMemcpyAsync(grad_x0 + d * n, lam[d], sizeof(double) * n, hipMemcpyDeviceToDevice,
                           sm) != hipSuccess ||
            hipMemcpyAsync(grad_v0 + d * n, vbuf[cur][d], sizeof(double) * n,
                           hipMemcpyDeviceToDevice, sm) != hipSuccess)
            return MD_ERR_HIP;
    }
    if (hipMemcpyAsync(grad_theta, theta, 2 * sizeof(double), hipMemcpyDeviceToDevice, sm) !=
        hipSuccess)
        return MD_ERR_HIP;
    // back to the state at step S
    checkpoint_arrays(ws, L, L.nseg, ck);
    if ((st = checkpoint(c, ck, false)) != MD_OK) return st;
    rebuild_all(c);
    return launched();
}

extern "C" md_status md_history(md_ctx* c, md_record* out, int32_t max_records, int32_t* n_out)
{
    if (!c || !n_out || max_records < 0 || (max_records > 0 && !out)) return MD_ERR_ARG;
    if (!c->bound) return MD_ERR_NOT_BOUND;
    DevState d;
    if (hipMemcpyAsync(&d, c->kp.dev, sizeof(d), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return MD_ERR_HIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MD_ERR_HIP;
    std::vector<md_record> ring(kHistCap);
    if (hipMemcpy(ring.data(), c->kp.hist, sizeof(md_record) * kHistCap,
                  hipMemcpyDeviceToHost) != hipSuccess)
        return MD_ERR_HIP;
    const int64_t total = d.hist_count;
    const int64_t avail = total < kHistCap ? total : kHistCap;
    const int64_t take = avail < max_records ? avail : max_records;
    const int64_t first = total - avail;  // oldest record still held
    for (int64_t r = 0; r < take; ++r) out[r] = ring[(first + r) % kHistCap];
    *n_out = (int32_t)take;
    return MD_OK;
}

static bool one_of(int v, std::initializer_list<int> set)
{
    for (int s : set)
        if (v == s) return true;
    return false;
}

extern "C" md_status md_set_tuning(md_ctx* c, const md_tuning* t)
{
    if (!c || !t) return MD_ERR_ARG;
    if (!one_of(t->force_lanes, {1, 2, 4, 8}) || t->force_block % 64 != 0 ||
        t->force_block < 64 || t->force_block > 1024 || t->nl_block % 64 != 0 ||
        t->nl_block < 0 || t->nl_block > 1024 || t->tile_cells < 0 || t->tile_y < 0 ||
        t->tile_z < 0 || t->stage_cap < 0 ||
        t->integrate_grid < 0 || t->integrate_grid > kIntegrateGridMax ||
        !one_of(t->nl_method, {MD_NL_AUTO, MD_NL_LANES, MD_NL_CELL_WAVES}))
        return MD_ERR_ARG;
    KParams& k = c->kp;
    drop_graph(c);  // launch shapes and parameters are baked into it
    const int old[4] = {k.n_tiles, k.kx_max, k.ky_max, k.kz_max};
    k.force_lanes = t->force_lanes;
    k.force_block = t->force_block;
    c->nl_block_req = t->nl_block;
    c->nl_method_req = t->nl_method;
    k.int_grid = t->integrate_grid > 0 ? t->integrate_grid : kIntegrateGridDefault;
    c->stage_cap = t->stage_cap;
    c->tile_cells = t->tile_cells;
    c->tile_y = t->tile_y;
    c->tile_z = t->tile_z;
    plan_tiles(c);
    // the list encoding depends on the tiling
    if (k.n_tiles != old[0] || k.kx_max != old[1] || k.ky_max != old[2] || k.kz_max != old[3])
        c->nl_ok = false;
    // the partials of the last force pass are laid out for the old grid
    c->forces_ok = false;
    return MD_OK;
}

extern "C" md_status md_get_tuning(const md_ctx* c, md_tuning* t)
{
    if (!c || !t) return MD_ERR_ARG;
    t->force_lanes = c->kp.force_lanes;
    t->force_block = c->kp.force_block;
    t->nl_block = c->kp.nl_block;
    t->integrate_grid = c->kp.int_grid;
    t->nl_method = c->kp.nl_method;
    t->tile_cells = c->tile_cells_res;
    t->tile_y = c->tile_y_res;
    t->tile_z = c->tile_z_res;
    t->stage_cap = c->kp.scap;
    return MD_OK;
}

extern "C" md_status md_set_timing(md_ctx* c, int32_t enable)
{
    if (!c) return MD_ERR_ARG;
    md_status st = fold_timing(c);
    c->timing = enable != 0;
    c->timed_ms = 0.0;
    c->timed_launches = 0;
    for (int k = 0; k < MD_PART_COUNT; ++k) {
        c->part_ms[k] = 0.0;
        c->part_launches[k] = 0;
    }
    return st;
}

extern "C" md_status md_get_timing_parts(md_ctx* c, double* ms, int64_t* launches)
{
    if (!c || !ms || !launches) return MD_ERR_ARG;
    md_status st = fold_timing(c);
    for (int k = 0; k < MD_PART_COUNT; ++k) {
        ms[k] = c->part_ms[k];
        launches[k] = c->part_launches[k];
    }
    return st;
}

extern "C" md_status md_get_timing(md_ctx* c, double* total_ms, int64_t* launches)
{
    if (!c || !total_ms || !launches) return MD_ERR_ARG;
    md_status st = fold_timing(c);
    *total_ms = c->timed_ms;
    *launches = c->timed_launches;
    return st;
}

extern "C" void md_destroy(md_ctx* c)
{
    if (!c) return;
    if (!c->ev_pending.empty() || c->gexec) (void)hipStreamSynchronize(c->stream);
    if (c->gstream) (void)hipStreamSynchronize(c->gstream);
    drop_graph(c);
    for (int e = 0; e < 2; ++e)
        if (c->gev[e]) (void)hipEventDestroy(c->gev[e]);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_pending) (void)hipEventDestroy(e);
    delete c;
}
