// md_ctx.h -- the host-side context of one system (private to libmd).
#pragma once

#include <stddef.h>

#include <vector>

#include "md_internal.h"

namespace md {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Regions of the workspace block, in order.
enum Region {
    R_DEV, R_CELL_COUNT, R_CELL_START, R_CELL_OF, R_SLOT, R_ORDER, R_TMP, R_NL, R_NL_COUNT,
    R_XR, R_YR, R_ZR, R_SX, R_SY, R_SZ, R_SVX, R_SVY, R_SVZ, R_SFX, R_SFY, R_SFZ, R_SID,
    R_SCELL, R_LAYERS, R_W32, R_APART, R_SLOT_OF, R_BPART, R_FPART, R_IPART, R_HIST, R_COUNT
};

}  // namespace md

struct md_ctx;
void replan_tiles(md_ctx* c);  // the tiling again, after a change of min_tiles

// Tuning cache (md_tune.hip): keys of a system or a batch with a candidate
// list on this device, and the cached tuning of a key in a cache file.
uint64_t tuning_key_ctx(const md_ctx* c, const md_tuning* cand, int32_t n);
uint64_t tuning_key_batch(const md_ctx* const* reps, int32_t r, const md_tuning* cand, int32_t n);
bool tuning_cache_get(const char* path, uint64_t key, md_tuning* out);
bool tuning_cache_put(const char* path, uint64_t key, const md_tuning& t, double ms);

struct md_ctx {
    md_params prm;
    md_grid geo;
    md::KParams kp;
    size_t off[md::R_COUNT];
    size_t bytes[md::R_COUNT];
    size_t ws_bytes;
    hipStream_t stream = nullptr;
    bool bound = false, cells_ok = false, nl_ok = false, forces_ok = false;
    int nl_block_req = 0;   // requested list-build workgroup size (0: automatic)
    int nl_method_req = 0;  // requested list-build method (MD_NL_AUTO: by density)
    bool timing = false;
    std::vector<hipEvent_t> ev_free, ev_pending;  // pending holds start/stop pairs
    double timed_ms = 0.0;                 // force passes (md_get_timing)
    int64_t timed_launches = 0;
    std::vector<int> ev_part;              // MD_PART_* of each pending pair
    double part_ms[MD_PART_COUNT] = {};    // md_get_timing_parts
    int64_t part_launches[MD_PART_COUNT] = {};
    int64_t host_steps = 0;                // md_step steps since md_bind (the layer reorder
                                           // schedule)
    size_t lds_limit = 160 * 1024;  // per-workgroup LDS; refreshed from the device at bind
    int tile_cells = 0, tile_y = 0, tile_z = 0;  // requested block size (0: automatic)
    int tile_cells_res = 0, tile_y_res = 0, tile_z_res = 0;  // largest block in use
    int stage_cap = 0;              // requested staged-atom capacity (0: from density)
    int min_tiles = 256;            // automatic tiling: at least this many tiles (one per CU)
    // md_step's graph of kGraphSteps steps (see md_api.hip)
    bool graph_on = false;  // set by md_init from the system size
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int g_record = -1;                     // record_every the graph was captured with
    int g_len = 0;                         // steps in the graph
    hipStream_t g_run = nullptr;           // stream it was captured on
    hipStream_t gstream = nullptr;         // own stream, when the bound one is the null stream
    hipEvent_t gev[2] = {nullptr, nullptr};
};
