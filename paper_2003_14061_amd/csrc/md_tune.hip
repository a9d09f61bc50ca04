// md_tune.hip -- the autotuner of the launch shape (single systems) and the
// tuning cache shared with the batched autotuner.
//
// Host side only.  The block-size sensitivity of the kernels is hardware
// dependent (section 4.1, factor (2)), so the launch shape is chosen by
// timing candidates on the device: each candidate builds the list and
// evaluates the forces `reps` times on the current state, and its cost is
// the force time plus a tenth of the list time (a rebuild every ten steps or
// so).  The winner can be kept in a cache file, keyed by a hash of the
// system (sizes, geometry, precision, modes), of the candidate list and of
// the device name, so that a later run of the same workload on the same
// kind of GPU takes the tuning without timing again.
//
// The cache file is a JSON object, one entry per line:
//   {
//   "<key>": {"force_lanes": 4, "force_block": 512, ..., "ms": 0.2761},
//   ...
//   }
// Lines this code did not write are kept as they are; the file is replaced
// atomically (written beside it, then renamed).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "md_ctx.h"

using namespace md;

namespace {

struct Field {
    const char* name;
    int32_t md_tuning::*member;
};

const Field kFields[] = {
    {"force_lanes", &md_tuning::force_lanes},   {"force_block", &md_tuning::force_block},
    {"nl_block", &md_tuning::nl_block},         {"tile_cells", &md_tuning::tile_cells},
    {"stage_cap", &md_tuning::stage_cap},       {"integrate_grid", &md_tuning::integrate_grid},
    {"nl_method", &md_tuning::nl_method},       {"tile_y", &md_tuning::tile_y},
    {"tile_z", &md_tuning::tile_z},
};

// FNV-1a over bytes.
struct Hash {
    uint64_t h = 1469598103934665603ull;
    void add(const void* p, size_t n)
    {
        const unsigned char* c = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
    }
    template <class T>
    void add(const T& v)
    {
        add(&v, sizeof(v));
    }
};

void add_system(Hash& h, const md_ctx* c)
{
    const md_params& p = c->prm;
    h.add(p.n_atoms);
    h.add(p.L);
    h.add(p.r_cut);
    h.add(p.skin);
    h.add(p.sigma);
    h.add(p.precision);
    h.add(p.mode);
    h.add(p.newton3);
    h.add(p.reorder);
    h.add(p.pipeline);
    h.add(c->geo.nc);
    h.add(c->geo.nl_capacity);
}

void add_candidates(Hash& h, const md_tuning* cand, int32_t n)
{
    for (int32_t i = 0; i < n; ++i)
        for (const Field& f : kFields) h.add(cand[i].*(f.member));
}

void add_device(Hash& h)
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        h.add(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
        h.add(prop.multiProcessorCount);
    }
}

std::string hex(uint64_t v)
{
    char b[17];
    snprintf(b, sizeof b, "%016llx", (unsigned long long)v);
    return b;
}

bool read_lines(const char* path, std::vector<std::string>& lines)
{
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char buf[4096];
    std::string cur;
    while (fgets(buf, sizeof buf, f)) {
        cur += buf;
        if (!cur.empty() && cur.back() == '\n') {
            cur.pop_back();
            lines.push_back(cur);
            cur.clear();
        }
    }
    if (!cur.empty()) lines.push_back(cur);
    fclose(f);
    return true;
}

// The integer after "name": in s, if present.
bool field_value(const std::string& s, const char* name, int32_t* out)
{
    const std::string tag = std::string("\"") + name + "\":";
    const size_t at = s.find(tag);
    if (at == std::string::npos) return false;
    char* end = nullptr;
    const long v = strtol(s.c_str() + at + tag.size(), &end, 10);
    if (end == s.c_str() + at + tag.size()) return false;
    *out = (int32_t)v;
    return true;
}

}  // namespace

uint64_t tuning_key_ctx(const md_ctx* c, const md_tuning* cand, int32_t n)
{
    Hash h;
    add_system(h, c);
    add_candidates(h, cand, n);
    add_device(h);
    return h.h;
}

uint64_t tuning_key_batch(const md_ctx* const* reps, int32_t r, const md_tuning* cand, int32_t n)
{
    Hash h;
    h.add(r);
    for (int32_t i = 0; i < r; ++i) add_system(h, reps[i]);
    add_candidates(h, cand, n);
    add_device(h);
    return h.h;
}

bool tuning_cache_get(const char* path, uint64_t key, md_tuning* out)
{
    if (!path) return false;
    std::vector<std::string> lines;
    if (!read_lines(path, lines)) return false;
    const std::string tag = "\"" + hex(key) + "\":";
    for (const std::string& s : lines) {
        if (s.find(tag) == std::string::npos) continue;
        md_tuning t;
        memset(&t, 0, sizeof t);
        for (const Field& f : kFields)
            if (!field_value(s, f.name, &(t.*(f.member)))) return false;
        *out = t;
        return true;
    }
    return false;
}

bool tuning_cache_put(const char* path, uint64_t key, const md_tuning& t, double ms)
{
    if (!path) return false;
    std::vector<std::string> lines, keep;
    read_lines(path, lines);
    const std::string tag = "\"" + hex(key) + "\":";
    for (const std::string& s : lines) {
        if (s == "{" || s == "}" || s.empty()) continue;
        if (s.find(tag) != std::string::npos) continue;
        std::string e = s;
        if (!e.empty() && e.back() == ',') e.pop_back();
        keep.push_back(e);
    }
    std::string mine = tag + " {";
    for (size_t i = 0; i < sizeof kFields / sizeof kFields[0]; ++i) {
        char b[64];
        snprintf(b, sizeof b, "\"%s\": %d, ", kFields[i].name, (int)(t.*(kFields[i].member)));
        mine += b;
    }
    char b[64];
    snprintf(b, sizeof b, "\"ms\": %.6g}", ms);
    mine += b;
    keep.push_back(mine);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fputs("{\n", f);
    for (size_t i = 0; i < keep.size(); ++i)
        fprintf(f, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
    fputs("}\n", f);
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

extern "C" md_status md_autotune(md_ctx* c, const md_tuning* cand, int32_t n, int32_t reps,
                                 const char* cache_path, double* ms_out, int32_t* best)
{
    if (!c || !cand || n < 1 || reps < 1 || !ms_out || !best) return MD_ERR_ARG;
    if (!c->bound) return MD_ERR_NOT_BOUND;
    if (c->prm.mode != MD_NEIGHBOR_LIST || c->prm.pipeline != MD_PIPE_TILED) return MD_ERR_ARG;
    const uint64_t key = tuning_key_ctx(c, cand, n);
    md_tuning hit;
    if (tuning_cache_get(cache_path, key, &hit)) {
        for (int32_t i = 0; i < n; ++i) ms_out[i] = -1.0;
        *best = -1;
        for (int32_t i = 0; i < n; ++i)
            if (memcmp(&cand[i], &hit, sizeof hit) == 0) *best = i;
        md_status st = md_set_tuning(c, &hit);
        if (st == MD_OK) st = md_build_cells(c);
        if (st == MD_OK) st = md_build_neighbors(c);
        if (st == MD_OK) st = md_forces(c);
        return st;
    }
    hipEvent_t ev[3];
    for (int k = 0; k < 3; ++k)
        if (hipEventCreate(&ev[k]) != hipSuccess) return MD_ERR_HIP;
    md_status st = MD_OK;
    int32_t arg = -1;
    for (int32_t i = 0; i < n && st == MD_OK; ++i) {
        if ((st = md_set_tuning(c, &cand[i])) != MD_OK) break;
        if ((st = md_build_cells(c)) != MD_OK) break;
        (void)hipEventRecord(ev[0], c->stream);
        for (int32_t k = 0; k < reps && st == MD_OK; ++k) st = md_build_neighbors(c);
        (void)hipEventRecord(ev[1], c->stream);
        for (int32_t k = 0; k < reps && st == MD_OK; ++k) st = md_forces(c);
        (void)hipEventRecord(ev[2], c->stream);
        float t_nl = 0.f, t_f = 0.f;
        if (st == MD_OK && (hipEventSynchronize(ev[2]) != hipSuccess ||
                            hipEventElapsedTime(&t_nl, ev[0], ev[1]) != hipSuccess ||
                            hipEventElapsedTime(&t_f, ev[1], ev[2]) != hipSuccess))
            st = MD_ERR_HIP;
        if (st != MD_OK) break;
        ms_out[i] = (double)t_f / reps + 0.1 * (double)t_nl / reps;
        if (arg < 0 || ms_out[i] < ms_out[arg]) arg = i;
    }
    for (int k = 0; k < 3; ++k) (void)hipEventDestroy(ev[k]);
    if (st != MD_OK) return st;
    *best = arg;
    if ((st = md_set_tuning(c, &cand[arg])) != MD_OK) return st;
    if ((st = md_build_cells(c)) != MD_OK) return st;
    if ((st = md_build_neighbors(c)) != MD_OK) return st;
    if ((st = md_forces(c)) != MD_OK) return st;
    tuning_cache_put(cache_path, key, cand[arg], ms_out[arg]);
    return MD_OK;
}
