// Launch-shape search shared by single plans and batches: the candidate
// list, the timing loop and the on-disk cache of winners.
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <cstdio>
#include <functional>
#include <string>
#include <utility>
#include <vector>

#include "internal.hpp"

namespace fdtd {

namespace {

// Candidates: tile rows x z-chunk x tile order (automatic, which follows
// each launch's state size, or runs of 16); for plans with two-level steps
// then the two-level tile rows x z-chunk, and single steps.
const int TUNE_ROWS[] = {2, 4, 8, 12, 16};
const int TUNE_Z[] = {4, 8, 16, 32, 64};
const int TUNE_ORDER[] = {-1, 16};
const int TUNE_TB_ROWS[] = {8, 10, 13};
const int TUNE_TB_Z[] = {8, 16, 32, 64};
constexpr int TUNE_STAGE1 = 5 * 5 * 2;   // per schedule

// The cache is a JSON object written one entry per line:
//   {
//   "gfx950:...|400x120x80;": [4, 32, 0.0312, 0, 2, 13, 16, 0],
//   ...
//   }
// (rows, z-chunk, milliseconds per step, tile order, two-level depth, tile
// rows and z-chunk, lockstep; an entry without the order leaves it
// automatic, one without the two-level fields the two-level defaults, one
// without the last field the configured schedule).  Unknown lines are
// ignored.
std::vector<std::pair<std::string, std::string>> cache_read(const char *path)
{
    std::vector<std::pair<std::string, std::string>> out;
    FILE *f = std::fopen(path, "r");
    if (!f) return out;
    char line[4096];
    while (std::fgets(line, sizeof line, f)) {
        std::string s(line);
        const size_t q0 = s.find('"'), q1 = s.find("\": [");
        const size_t b1 = s.find(']');
        if (q0 == std::string::npos || q1 == std::string::npos || b1 == std::string::npos ||
            q1 <= q0 || b1 < q1 + 4)
            continue;
        out.emplace_back(s.substr(q0 + 1, q1 - q0 - 1), s.substr(q1 + 4, b1 - q1 - 4));
    }
    std::fclose(f);
    return out;
}

bool cache_lookup(const char *path, const std::string &key, LaunchCfg &cfg)
{
    for (const auto &e : cache_read(path)) {
        if (e.first != key) continue;
        int rows = 0, z = 0, order = -1, depth = 2, tbr = 13, tbz = 32, lock = 0;
        double ms = 0;
        const int n = std::sscanf(e.second.c_str(), "%d , %d , %lf , %d , %d , %d , %d , %d", &rows,
                                  &z, &ms, &order, &depth, &tbr, &tbz, &lock);
        if (n >= 2 && valid_rows(rows) && z >= 1 && z <= 64 && valid_order(order) &&
            (depth == 1 || depth == 2) && valid_tb_rows(tbr) && tbz >= 4 && tbz <= 256 &&
            (lock == 0 || lock == 1)) {
            cfg.rows = rows;
            cfg.zchunk = z;
            cfg.order = order;
            cfg.tb_depth = depth;
            cfg.tb_rows = tbr;
            cfg.tb_zchunk = tbz;
            cfg.lockstep = lock;
            return true;
        }
        return false;
    }
    return false;
}

void cache_store(const char *path, const std::string &key, const LaunchCfg &cfg, double ms)
{
    auto entries = cache_read(path);
    char val[128];
    std::snprintf(val, sizeof val, "%d, %d, %.6g, %d, %d, %d, %d, %d", cfg.rows, cfg.zchunk, ms,
                  cfg.order, cfg.tb_depth, cfg.tb_rows, cfg.tb_zchunk, cfg.lockstep);
    bool found = false;
    for (auto &e : entries)
        if (e.first == key) { e.second = val; found = true; }
    if (!found) entries.emplace_back(key, val);
    // written under a per-process name, then renamed over the cache: a
    // reader sees the old file or the new one, never a partial write
    const std::string tmp = std::string(path) + "." + std::to_string((long)getpid()) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    for (size_t q = 0; q < entries.size(); ++q)
        std::fprintf(f, "\"%s\": [%s]%s\n", entries[q].first.c_str(), entries[q].second.c_str(),
                     q + 1 < entries.size() ? "," : "");
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), path);
    else std::remove(tmp.c_str());
}

// Two events, destroyed on every exit path.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t create()
    {
        hipError_t e = hipEventCreate(&a);
        return e != hipSuccess ? e : hipEventCreate(&b);
    }
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

std::string tune_device_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    return prop.gcnArchName;
}

std::string tune_shape_key(const Plan *const *plans, size_t n)
{
    std::string k;
    for (size_t q = 0; q < n; ++q) {
        char buf[64];
        std::snprintf(buf, sizeof buf, "%dx%dx%d;", plans[q]->g.nx, plans[q]->g.ny, plans[q]->g.nz);
        k += buf;
    }
    return k;
}

hipError_t tune_search(const TuneHooks &h, int32_t trial_steps, const char *cache_path,
                       const std::string &key, hipStream_t s, LaunchCfg &best_cfg, int32_t &best_index)
{
    if (cache_path && cache_lookup(cache_path, key, best_cfg)) {
        best_index = -1;
        h.apply(best_cfg);
        return hipSuccess;
    }
    EventPair ev;
    hipError_t e = ev.create();
    if (e != hipSuccess) return e;
    // time one candidate: its milliseconds for trial_steps steps
    auto time_one = [&](const LaunchCfg &c, float &ms) -> hipError_t {
        h.apply(c);
        h.run(1);   // warm-up
        hipError_t r;
        if ((r = hipEventRecord(ev.a, s)) != hipSuccess) return r;
        h.run(trial_steps);
        if ((r = hipEventRecord(ev.b, s)) != hipSuccess) return r;
        if ((r = hipEventSynchronize(ev.b)) != hipSuccess) return r;
        return hipEventElapsedTime(&ms, ev.a, ev.b);
    };
    float best = 1e30f;
    int idx = 0;
    best_index = -1;
    for (int sch = 0; sch < h.schedules; ++sch)
        for (int r : TUNE_ROWS)
            for (int z : TUNE_Z)
                for (int o : TUNE_ORDER) {
                    LaunchCfg c;
                    c.rows = r;
                    c.zchunk = z;
                    c.order = o;
                    c.lockstep = sch;
                    float ms = 0;
                    if ((e = time_one(c, ms)) != hipSuccess) return e;
                    if (ms < best) { best = ms; best_index = idx; best_cfg = c; }
                    ++idx;
                }
    if (h.two_level) {
        // the winner's launch shape with each two-level tile shape, then
        // with single steps; all timed afresh, so the stage compares like
        // with like
        const LaunchCfg base = best_cfg;
        const int i1 = best_index;
        float best2 = 1e30f;
        int j = 0;
        auto consider = [&](const LaunchCfg &c) -> hipError_t {
            float ms = 0;
            const hipError_t r = time_one(c, ms);
            if (r != hipSuccess) return r;
            if (ms < best2) { best2 = ms; best_index = i1 + TUNE_STAGE1 * j; best_cfg = c; }
            ++j;
            return hipSuccess;
        };
        for (int r : TUNE_TB_ROWS)
            for (int z : TUNE_TB_Z) {
                LaunchCfg c = base;
                c.tb_depth = 2;
                c.tb_rows = r;
                c.tb_zchunk = z;
                if ((e = consider(c)) != hipSuccess) return e;
            }
        LaunchCfg c = base;
        c.tb_depth = 1;
        if ((e = consider(c)) != hipSuccess) return e;
        best = best2;
    }
    h.apply(best_cfg);
    if (cache_path) cache_store(cache_path, key, best_cfg, best / trial_steps);
    return hipSuccess;
}

}  // namespace fdtd
