// md_batch.hip -- many independent replicas advanced by shared launches.
//
// Host side only.  Each replica is an ordinary context (md_api.hip); the
// batch lays their workspaces out in one block, copies every replica's
// kernel parameters and a per-grid-rule table of workgroup ranges to the
// device, and launches each kernel of the step once over all replicas
// (md_internal.h: Batch).  A run is captured into a HIP graph and launched
// as one graph.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "md_ctx.h"

using namespace md;

struct md_batch {
    std::vector<md_ctx*> rep;
    std::vector<size_t> rep_off;  // workspace offset of each replica
    size_t tab_off = 0;           // parameters and tables
    size_t ws_bytes = 0;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false, prepared = false;
    Batch dev{};
    LaunchShape sh{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int g_steps = -1, g_record = -1;
};

namespace {

// Workgroups per replica of the rebuild-gated grid-stride kernels in a
// batch of R.
int gate_share(int R)
{
    const int g = 4 * kGateGridDefault / R;
    return g > 64 ? g : 64;
}

// A replica's integration workgroups: one per 8192 atoms (eight per lane),
// so that large and small replicas finish together; fewer, longer
// workgroups measured faster than one lane per atom.
int integrate_share(int64_t n)
{
    const int64_t g = (n + 8 * kIntThreads - 1) / (8 * kIntThreads);
    return (int)(g < 1 ? 1 : g > kIntegrateGridDefault ? kIntegrateGridDefault : g);
}

// Most workgroups replica c can ask of any grid rule, for any tuning.
int64_t max_workgroups(const md_ctx* c)
{
    const int64_t n = c->prm.n_atoms, ncell = c->geo.n_cells, b = c->kp.block;
    return (n + b - 1) / b + 1 + kIntegrateGridMax + 2 * max_force_blocks(n, ncell) +
           8 * G_KINDS;
}

size_t table_bytes(const md_batch* b)
{
    const size_t R = b->rep.size();
    int64_t wg = 0;
    for (const md_ctx* c : b->rep) wg += max_workgroups(c);
    return align_up(sizeof(KParams) * R) + align_up(sizeof(int32_t) * G_KINDS * (R + 1)) +
           align_up(sizeof(int32_t) * G_KINDS * R) + align_up(sizeof(uint16_t) * (size_t)wg);
}

void drop_graph(md_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->g_steps = b->g_record = -1;
}

// Parameters and workgroup tables to the device; the uniform launch shape.
// Work already queued on the stream may read the old tables: it finishes
// first.
md_status upload(md_batch* b)
{
    if (b->stream && hipStreamSynchronize(b->stream) != hipSuccess) return MD_ERR_HIP;
    const int R = (int)b->rep.size();
    std::vector<KParams> kp(R);
    std::vector<int32_t> first((size_t)G_KINDS * (R + 1)), count((size_t)G_KINDS * R);
    std::vector<uint16_t> rep_of;
    int32_t rep_base[G_KINDS];
    LaunchShape sh;
    memset(&sh, 0, sizeof(sh));
    for (int r = 0; r < R; ++r) kp[r] = b->rep[r]->kp;
    for (int k = 0; k < G_KINDS; ++k) {
        int64_t off = 0;
        for (int r = 0; r < R; ++r) {
            const int n = grid_of(kp[r], (GridKind)k);
            first[(size_t)k * (R + 1) + r] = (int32_t)off;
            count[(size_t)k * R + r] = n;
            off += n;
            // the tile grids start each replica on XCD 0
            if (r + 1 < R && (k == G_TILES || k == G_NL)) off = (off + 7) / 8 * 8;
        }
        if (off > 0x7fffffff) return MD_ERR_ARG;
        first[(size_t)k * (R + 1) + R] = (int32_t)off;
        sh.grid[k] = (int)off;
        rep_base[k] = (int32_t)rep_of.size();
        for (int r = 0; r < R; ++r) {
            const int32_t end = first[(size_t)k * (R + 1) + r + 1];
            for (int32_t w = first[(size_t)k * (R + 1) + r]; w < end; ++w)
                rep_of.push_back((uint16_t)r);
        }
    }
    const KParams& p0 = kp[0];
    sh.block = p0.block;
    sh.force_block = p0.force_block;
    sh.force_lanes = p0.force_lanes;
    sh.nl_method = p0.nl_method;
    sh.precision = p0.precision;
    sh.reorder = p0.reorder;
    sh.mode = p0.mode;
    sh.newton3 = p0.newton3;
    for (int r = 0; r < R; ++r) {
        sh.nl_full |= kp[r].nc < 5 || !nl_small(kp[r]);
        const int nlb = kp[r].nl_block;
        sh.nl_block = nlb > sh.nl_block ? nlb : sh.nl_block;
        if (p0.mode == MD_NEIGHBOR_LIST) {
            const size_t a = nl_lds_bytes(kp[r]), f = force_lds_bytes(kp[r]);
            sh.nl_lds = a > sh.nl_lds ? a : sh.nl_lds;
            sh.force_lds = f > sh.force_lds ? f : sh.force_lds;
        }
    }
    char* t = b->ws + b->tab_off;
    KParams* d_kp = reinterpret_cast<KParams*>(t);
    int32_t* d_first = reinterpret_cast<int32_t*>(t + align_up(sizeof(KParams) * (size_t)R));
    int32_t* d_count = reinterpret_cast<int32_t*>(
        t + align_up(sizeof(KParams) * (size_t)R) +
        align_up(sizeof(int32_t) * (size_t)G_KINDS * (size_t)(R + 1)));
    uint16_t* d_rep = reinterpret_cast<uint16_t*>(
        reinterpret_cast<char*>(d_count) + align_up(sizeof(int32_t) * (size_t)G_KINDS * R));
    if ((char*)(d_rep + rep_of.size()) > b->ws + b->ws_bytes) return MD_ERR_ARG;
    // each replica's entries of the gated rules (their gate bits start clear;
    // every step's integration finish sets them before a gated kernel runs)
    for (int r = 0; r < R; ++r) {
        kp[r].rep = r;
        for (int j = 0; j < 3; ++j) {
            const int k = (int)kGatedRules[j];
            kp[r].gate_tab[j] = d_rep + rep_base[k] + first[(size_t)k * (R + 1) + r];
            kp[r].gate_n[j] = count[(size_t)k * R + r];
        }
    }
    if (hipMemcpy(d_kp, kp.data(), sizeof(KParams) * (size_t)R, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(d_first, first.data(), sizeof(int32_t) * first.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(d_count, count.data(), sizeof(int32_t) * count.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(d_rep, rep_of.data(), sizeof(uint16_t) * rep_of.size(),
                  hipMemcpyHostToDevice) != hipSuccess)
        return MD_ERR_HIP;
    b->dev.kp = d_kp;
    b->dev.first = d_first;
    b->dev.count = d_count;
    b->dev.rep_of = d_rep;
    for (int k = 0; k < G_KINDS; ++k) b->dev.rep_base[k] = rep_base[k];
    b->dev.R = R;
    b->sh = sh;
    drop_graph(b);
    return MD_OK;
}

void step_sequence(md_batch* b, int32_t n_steps, int32_t record_every)
{
    const bool nl = b->sh.mode == MD_NEIGHBOR_LIST;
    for (int32_t s = 0; s < n_steps; ++s) {
        launch_integrate(b->dev, b->sh, s == 0 ? 0 : 1, record_every, b->stream);
        // the reorder's copy-back folded into the list build
        const int fold = nl && b->sh.reorder ? kFoldCopy : 0;
        launch_cells(b->dev, b->sh, fold, b->stream);
        if (nl) launch_neighbors(b->dev, b->sh, fold, b->stream);
        launch_forces(b->dev, b->sh, b->stream);
    }
    launch_integrate(b->dev, b->sh, 2, record_every, b->stream);
}

void set_flags(md_batch* b, bool ok)
{
    for (md_ctx* c : b->rep) c->cells_ok = c->nl_ok = c->forces_ok = ok;
}

md_status prepare(md_batch* b)
{
    launch_cells(b->dev, b->sh, 1, b->stream);
    if (b->sh.mode == MD_NEIGHBOR_LIST) launch_neighbors(b->dev, b->sh, 1, b->stream);
    launch_forces(b->dev, b->sh, b->stream);
    if (hipGetLastError() != hipSuccess) return MD_ERR_HIP;
    set_flags(b, true);
    b->prepared = true;
    return MD_OK;
}

}  // namespace

extern "C" md_status md_batch_init(const md_params* params, int32_t n_replicas, md_batch** out)
{
    if (!params || !out || n_replicas < 1 || n_replicas > kRepMask + 1) return MD_ERR_ARG;
    *out = nullptr;
    md_batch* b = new (std::nothrow) md_batch;
    if (!b) return MD_ERR_ARG;
    size_t off = 0;
    for (int32_t r = 0; r < n_replicas; ++r) {
        const md_params& p = params[r];
        const md_params& p0 = params[0];
        if (p.precision != p0.precision || p.mode != p0.mode || p.reorder != p0.reorder ||
            p.newton3 != p0.newton3 || p.block != p0.block || p.pipeline != MD_PIPE_TILED) {
            md_batch_destroy(b);
            return MD_ERR_ARG;
        }
        md_ctx* c = nullptr;
        md_status st = md_init(&p, &c);
        if (st != MD_OK) {
            md_batch_destroy(b);
            return st;
        }
        // the gated per-atom and per-cell kernels and the integration share
        // the machine among the replicas
        c->kp.gate_grid = gate_share(n_replicas);
        c->kp.int_grid = integrate_share(p.n_atoms);
        c->min_tiles = 0;  // the replicas together fill the machine
        replan_tiles(c);
        b->rep.push_back(c);
        b->rep_off.push_back(off);
        off += align_up(c->ws_bytes);
    }
    b->tab_off = off;
    b->ws_bytes = off + table_bytes(b);
    *out = b;
    return MD_OK;
}

extern "C" size_t md_batch_workspace_bytes(const md_batch* b) { return b ? b->ws_bytes : 0; }

extern "C" md_status md_batch_replica(md_batch* b, int32_t r, md_ctx** ctx)
{
    if (!b || !ctx || r < 0 || r >= (int32_t)b->rep.size()) return MD_ERR_ARG;
    *ctx = b->rep[r];
    return MD_OK;
}

extern "C" md_status md_batch_bind(md_batch* b, const md_buffers* buffers, void* workspace,
                                   void* stream)
{
    if (!b || !buffers || !workspace || !stream) return MD_ERR_ARG;
    if (((uintptr_t)workspace) % kAlign != 0) return MD_ERR_ARG;
    b->ws = static_cast<char*>(workspace);
    b->stream = static_cast<hipStream_t>(stream);
    for (size_t r = 0; r < b->rep.size(); ++r) {
        md_buffers bf = buffers[r];
        bf.workspace = b->ws + b->rep_off[r];
        md_status st = md_bind(b->rep[r], &bf, stream);
        if (st != MD_OK) return st;
    }
    md_status st = upload(b);
    if (st != MD_OK) return st;
    b->bound = true;
    b->prepared = false;
    return MD_OK;
}

extern "C" md_status md_batch_prepare(md_batch* b)
{
    if (!b) return MD_ERR_ARG;
    if (!b->bound) return MD_ERR_NOT_BOUND;
    return prepare(b);
}

extern "C" md_status md_batch_forces(md_batch* b)
{
    if (!b) return MD_ERR_ARG;
    if (!b->bound) return MD_ERR_NOT_BOUND;
    if (!b->prepared) return MD_ERR_STATE;
    launch_forces(b->dev, b->sh, b->stream);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

extern "C" md_status md_batch_layout(const md_batch* b, int32_t r, int32_t which, size_t* offset,
                                     size_t* count)
{
    if (!b || r < 0 || r >= (int32_t)b->rep.size()) return MD_ERR_ARG;
    md_status st = md_layout(b->rep[r], which, offset, count);
    if (st == MD_OK) *offset += b->rep_off[r];
    return st;
}

extern "C" md_status md_batch_run(md_batch* b, int32_t n_steps, int32_t record_every,
                                  int32_t use_graph)
{
    if (!b || n_steps < 0 || record_every < 0) return MD_ERR_ARG;
    if (!b->bound) return MD_ERR_NOT_BOUND;
    for (md_ctx* c : b->rep)
        if (!c->forces_ok) return MD_ERR_STATE;
    if (n_steps == 0) return MD_OK;
    if (!use_graph) {
        step_sequence(b, n_steps, record_every);
        return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
    }
    if (!(b->exec && b->g_steps == n_steps && b->g_record == record_every)) {
        drop_graph(b);
        if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return MD_ERR_HIP;
        step_sequence(b, n_steps, record_every);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(b->stream, &g);
        if (ec != hipSuccess || !g) return MD_ERR_HIP;
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(b);
            return MD_ERR_HIP;
        }
        b->g_steps = n_steps;
        b->g_record = record_every;
    }
    return hipGraphLaunch(b->exec, b->stream) == hipSuccess ? MD_OK : MD_ERR_HIP;
}

extern "C" md_status md_batch_set_tuning(md_batch* b, const md_tuning* t)
{
    if (!b || !t) return MD_ERR_ARG;
    const int R = (int)b->rep.size();
    for (md_ctx* c : b->rep) {
        md_status st = md_set_tuning(c, t);
        if (st != MD_OK) return st;
        if (t->integrate_grid == 0) c->kp.int_grid = integrate_share(c->prm.n_atoms);
    }
    b->prepared = false;
    set_flags(b, false);
    if (!b->bound) return MD_OK;
    return upload(b);
}

extern "C" md_status md_batch_get_tuning(const md_batch* b, md_tuning* t)
{
    if (!b || !t) return MD_ERR_ARG;
    return md_get_tuning(b->rep[0], t);
}

extern "C" md_status md_batch_autotune(md_batch* b, const md_tuning* cand, int32_t n, int32_t reps,
                                       const char* cache_path, double* ms_out, int32_t* best)
{
    if (!b || !cand || n < 1 || reps < 1 || !ms_out || !best) return MD_ERR_ARG;
    if (!b->bound) return MD_ERR_NOT_BOUND;
    const uint64_t key = tuning_key_batch(b->rep.data(), (int32_t)b->rep.size(), cand, n);
    md_tuning hit;
    if (tuning_cache_get(cache_path, key, &hit)) {
        for (int32_t i = 0; i < n; ++i) ms_out[i] = -1.0;
        *best = -1;
        for (int32_t i = 0; i < n; ++i)
            if (memcmp(&cand[i], &hit, sizeof hit) == 0) *best = i;
        md_status st = md_batch_set_tuning(b, &hit);
        return st == MD_OK ? prepare(b) : st;
    }
    hipEvent_t ev[3];
    for (int k = 0; k < 3; ++k)
        if (hipEventCreate(&ev[k]) != hipSuccess) return MD_ERR_HIP;
    md_status st = MD_OK;
    int32_t arg = -1;
    for (int32_t i = 0; i < n && st == MD_OK; ++i) {
        if ((st = md_batch_set_tuning(b, &cand[i])) != MD_OK) break;
        if ((st = prepare(b)) != MD_OK) break;
        (void)hipEventRecord(ev[0], b->stream);
        for (int32_t k = 0; k < reps; ++k) launch_neighbors(b->dev, b->sh, 1, b->stream);
        (void)hipEventRecord(ev[1], b->stream);
        for (int32_t k = 0; k < reps; ++k) launch_forces(b->dev, b->sh, b->stream);
        (void)hipEventRecord(ev[2], b->stream);
        float t_nl = 0.f, t_f = 0.f;
        if (hipEventSynchronize(ev[2]) != hipSuccess ||
            hipEventElapsedTime(&t_nl, ev[0], ev[1]) != hipSuccess ||
            hipEventElapsedTime(&t_f, ev[1], ev[2]) != hipSuccess) {
            st = MD_ERR_HIP;
            break;
        }
        ms_out[i] = (double)t_f / reps + 0.1 * (double)t_nl / reps;
        if (arg < 0 || ms_out[i] < ms_out[arg]) arg = i;
    }
    for (int k = 0; k < 3; ++k) (void)hipEventDestroy(ev[k]);
    if (st != MD_OK) return st;
    *best = arg;
    if ((st = md_batch_set_tuning(b, &cand[arg])) != MD_OK) return st;
    if ((st = prepare(b)) != MD_OK) return st;
    tuning_cache_put(cache_path, key, cand[arg], ms_out[arg]);
    return MD_OK;
}

extern "C" void md_batch_destroy(md_batch* b)
{
    if (!b) return;
    drop_graph(b);
    for (md_ctx* c : b->rep) md_destroy(c);
    delete b;
}
