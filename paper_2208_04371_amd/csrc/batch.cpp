// Batches: several FP32 fused plans (uneven shapes allowed) advanced
// together.  One step of all members (or of one group of consecutive
// members, when the members' state exceeds the group budget) is one fused
// launch pair over an instance table, with probe sampling inside the
// boundary launch; one DFT launch per history ring folds every member's
// samples.  This is how the per-port runs of one S-matrix (Sec. II-A: one
// incident and one total run per driving port) and the variants of a
// geometry sweep share the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "internal.hpp"



namespace fdtd {

// shared with plan.cpp
void plan_bind_slice(Plan &P, char *base, size_t bytes, hipStream_t s);
void plan_reset(Plan &P, hipStream_t s);
void plan_finalize(Plan &P);
DevProbes plan_dev_probes(const Plan &P);
DevDft plan_dev_dft(const Plan &P);

namespace {

struct BatchError : std::runtime_error {
    fdtd_status code;
    BatchError(fdtd_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define BREQUIRE(cond, code, msg)                          \
    do {                                                   \
        if (!(cond)) throw BatchError((code), (msg));      \
    } while (0)

void hcheck(hipError_t e, const char *what)
{
    if (e != hipSuccess) throw BatchError(FDTD_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

template <class F>
fdtd_status bguard(Batch *b, F &&f)
{
    try {
        f();
        if (b) b->err.clear();
        return FDTD_OK;
    } catch (const BatchError &e) {
        if (b) b->err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        if (b) b->err = "host allocation failed";
        return FDTD_E_NOMEM;
    } catch (const std::exception &e) {
        if (b) b->err = e.what();
        return FDTD_E_INVALID_ARG;
    }
}

// Device tables of a bound batch (offsets inside its workspace):
// [grids parity 0][grids parity 1][tile sets][group tile sets][probes][dft]
struct Tables {
    size_t grids[2], sets, gsets, probes, dft, bytes;
};

Tables table_layout(int n)
{
    Tables t{};
    size_t cur = 0;
    t.grids[0] = cur; cur = al256(cur + sizeof(DevGrid<float>) * n);
    t.grids[1] = cur; cur = al256(cur + sizeof(DevGrid<float>) * n);
    t.sets = cur; cur = al256(cur + sizeof(TileSet) * n);
    t.gsets = cur; cur = al256(cur + sizeof(TileSet) * n);
    t.probes = cur; cur = al256(cur + sizeof(DevProbes) * n);
    t.dft = cur; cur = al256(cur + sizeof(DevDft) * n);
    t.bytes = cur;
    return t;
}

void compute_blocks(Batch &B)
{
    B.sets.assign(B.plans.size(), TileSet{});
    int32_t nb = 0, ni = 0;
    for (size_t q = 0; q < B.plans.size(); ++q) {
        TileSet &t = B.sets[q];
        t = make_tileset(*B.plans[q], B.cfg);
        t.sb = nb;
        t.si = ni;
        nb += t.nb;
        ni += t.ni;
    }
    B.nb_total = nb;
    B.ni_total = ni;
    // groups: consecutive members packed greedily under group_bytes (one
    // group of all in lockstep)
    B.groups.clear();
    B.gsets = B.sets;
    const size_t budget = B.cfg.lockstep ? 0 : B.group_bytes;
    size_t total = 0;
    for (const Plan *P : B.plans) total += P->ws_bytes;
    for (size_t q = 0; q < B.plans.size(); ++q) {
        const size_t w = B.plans[q]->ws_bytes;
        const bool fresh = B.groups.empty() ||
                           (budget > 0 && total > budget && B.groups.back().bytes + w > budget);
        if (fresh) B.groups.push_back({(int32_t)q, 0, 0, 0, 0});
        Batch::Group &g = B.groups.back();
        TileSet &t = B.gsets[q];
        t.sb = g.nb;
        t.si = g.ni;
        g.count += 1;
        g.nb += t.nb;
        g.ni += t.ni;
        g.bytes += w;
    }
    B.lut_cap = 1;
    B.id_bits = 5;
    for (const Plan *P : B.plans) {
        B.lut_cap = std::max<int32_t>(B.lut_cap, (int32_t)(P->lut[0].size() / 4));
        if (P->id_bits != 5) B.id_bits = 8;
    }
}

// Default launch shape, sized for the largest group (the launches of a
// grouped schedule cover one group each).
void default_config(Batch &B)
{
    size_t big = 0;
    for (size_t q = 1; q < B.groups.size(); ++q)
        if (B.groups[q].bytes > B.groups[big].bytes) big = q;
    const LaunchCfg keep = B.cfg;
    B.cfg = default_launch(B.plans.data() + B.groups[big].first, (size_t)B.groups[big].count);
    B.cfg.order = keep.order;
    compute_blocks(B);
}

// Upload the instance tables for the current parity of the member plans.
void upload_tables(Batch &B, hipStream_t s)
{
    const int n = (int)B.plans.size();
    const Tables t = table_layout(n);
    std::vector<DevGrid<float>> g0(n), g1(n);
    std::vector<DevProbes> pr(n);
    std::vector<DevDft> df(n);
    for (int q = 0; q < n; ++q) {
        Plan &P = *B.plans[q];
        const int keep = P.parity;
        P.parity = 0;
        g0[q] = P.dev_grid<float>();
        P.parity = 1;
        g1[q] = P.dev_grid<float>();
        P.parity = keep;
        pr[q] = plan_dev_probes(P);
        df[q] = plan_dev_dft(P);
    }
    compute_blocks(B);
    char *base = B.base + B.r_table.off;
    hcheck(hipMemcpyAsync(base + t.grids[0], g0.data(), sizeof(DevGrid<float>) * n, hipMemcpyHostToDevice, s), "table");
    hcheck(hipMemcpyAsync(base + t.grids[1], g1.data(), sizeof(DevGrid<float>) * n, hipMemcpyHostToDevice, s), "table");
    hcheck(hipMemcpyAsync(base + t.sets, B.sets.data(), sizeof(TileSet) * n, hipMemcpyHostToDevice, s), "table");
    hcheck(hipMemcpyAsync(base + t.gsets, B.gsets.data(), sizeof(TileSet) * n, hipMemcpyHostToDevice, s), "table");
    hcheck(hipMemcpyAsync(base + t.probes, pr.data(), sizeof(DevProbes) * n, hipMemcpyHostToDevice, s), "table");
    hcheck(hipMemcpyAsync(base + t.dft, df.data(), sizeof(DevDft) * n, hipMemcpyHostToDevice, s), "table");
    hcheck(hipStreamSynchronize(s), "table sync");
}

// Fold the pending history samples of members [a, a + m) into their DFTs
// (the members of one span step, sample and fold in lockstep).
void span_flush(Batch &B, int a, int m, hipStream_t s)
{
    Plan &P0 = *B.plans[a];
    if (P0.sampled > P0.dft_n) {
        const Tables t = table_layout((int)B.plans.size());
        hcheck(launch_dft_batch(reinterpret_cast<const DevDft *>(B.base + B.r_table.off + t.dft) + a,
                                m, B.max_probes, B.max_nf, P0.dft_n + 1, P0.sampled - P0.dft_n, s),
               "batch dft");
        for (int q = a; q < a + m; ++q) B.plans[q]->dft_n = P0.sampled;
    }
}

// Advance members [a, a + m) by nsteps steps in lockstep, one fused launch
// pair per step.  sets_dev holds their tile sets with first blocks counted
// from member a; nb, ni are their tile totals; state is their workspace.
void run_span(Batch &B, int a, int m, const TileSet *sets_dev, int32_t nb, int32_t ni,
              size_t state, int64_t nsteps, hipStream_t s)
{
    const Tables t = table_layout((int)B.plans.size());
    char *tb = B.base + B.r_table.off;
    const DevProbes *probes = reinterpret_cast<const DevProbes *>(tb + t.probes) + a;
    Plan &P0 = *B.plans[a];
    const bool sample = B.max_probes > 0;
    LaunchCfg cfg = B.cfg;
    cfg.order = tile_order(B.cfg, state);
    cfg.stream = stream_stores(B.cfg, state);
    for (int64_t q = 0; q < nsteps; ++q) {
        const DevGrid<float> *g = reinterpret_cast<const DevGrid<float> *>(tb + t.grids[P0.parity]) + a;
        hipEvent_t e0, e1;
        hcheck(B.timer.step(e0, e1, q == 0, q + 1 == nsteps), "timer");
        // every member's step, plus sampling of its input level
        hcheck(launch_fused(g, sets_dev, m, nb, ni, cfg, B.lut_cap, B.id_bits, P0.step, probes,
                            B.max_probes, sample, s, e0, e1),
               "batch step");
        const int64_t sampled = (sample && P0.step >= 1) ? std::max(P0.sampled, P0.step) : P0.sampled;
        for (int r = a; r < a + m; ++r) {
            Plan *P = B.plans[r];
            P->parity = 1 - P->parity;
            P->step += 1;
            P->sampled = sampled;
        }
        if (P0.sampled - P0.dft_n >= P0.K - 1) span_flush(B, a, m, s);
    }
    if (sample && P0.sampled < P0.step) {
        const DevGrid<float> *gc = reinterpret_cast<const DevGrid<float> *>(tb + t.grids[P0.parity]) + a;
        hcheck(launch_probe_batch(gc, probes, m, B.max_probes, P0.step, s), "batch probe");
        for (int r = a; r < a + m; ++r) B.plans[r]->sampled = P0.step;
    }
    span_flush(B, a, m, s);
}

// All members advance by nsteps.  With one group, in lockstep; with
// several, group after group (each group's state stays in the memory-side
// cache for its whole span).  Members are independent, so both give the
// same results.
void batch_run(Batch &B, int64_t nsteps, hipStream_t s)
{
    BREQUIRE(B.bound, FDTD_E_STATE, "batch not bound");
    BREQUIRE(nsteps >= 0, FDTD_E_INVALID_ARG, "negative step count");
    const int n = (int)B.plans.size();
    const Tables t = table_layout(n);
    const char *tb = B.base + B.r_table.off;
    if (B.groups.size() <= 1) {
        run_span(B, 0, n, reinterpret_cast<const TileSet *>(tb + t.sets), B.nb_total, B.ni_total,
                 B.ws_bytes, nsteps, s);
        return;
    }
    for (const Batch::Group &g : B.groups)
        run_span(B, g.first, g.count, reinterpret_cast<const TileSet *>(tb + t.gsets) + g.first, g.nb,
                 g.ni, g.bytes, nsteps, s);
}

}  // namespace
}  // namespace fdtd

using namespace fdtd;

extern "C" {

// Message of the last failed fdtd_batch_create on this thread.
static std::string &create_error()
{
    static thread_local std::string msg;
    return msg;
}

fdtd_status fdtd_batch_create(fdtd_plan *const *plans, int32_t n, fdtd_batch **out)
{
    if (!plans || n < 1 || !out) return FDTD_E_INVALID_ARG;
    *out = nullptr;
    fdtd_batch *b = new (std::nothrow) fdtd_batch();
    if (!b) return FDTD_E_NOMEM;
    const fdtd_status st = bguard(b, [&]() {
        for (int q = 0; q < n; ++q) {
            Plan *P = plans[q];
            BREQUIRE(P, FDTD_E_INVALID_ARG, "null plan");
            BREQUIRE(P->g.kernel == FDTD_KERNEL_FUSED && P->g.precision == FDTD_FP32,
                     FDTD_E_UNSUPPORTED, "batches take FP32 fused plans");
            BREQUIRE(!P->bound && !P->in_batch, FDTD_E_STATE, "plan already bound");
            BREQUIRE(P->tb_mode != 1 && !P->tb, FDTD_E_UNSUPPORTED,
                     "plans with two-level steps run alone, not in a batch");
            if (!P->finalized) P->tb_mode = 0;
            plan_finalize(*P);
            b->plans.push_back(P);
            b->max_probes = std::max(b->max_probes, P->nprobe());
            b->max_nf = std::max(b->max_nf, P->nf());
        }
        for (int q = 0; q < n; ++q)
            for (int r = q + 1; r < n; ++r)
                BREQUIRE(plans[q] != plans[r], FDTD_E_INVALID_ARG, "plan listed twice");
        // one launch reads one id format: if any member needs 32-bit id
        // words, the others are laid out with them too
        bool wide = false;
        for (const Plan *P : b->plans) wide = wide || P->id_bits != 5;
        if (wide)
            for (Plan *P : b->plans)
                if (P->id_bits == 5) {
                    P->wide_ids = true;
                    P->finalized = false;
                    plan_finalize(*P);
                }
        compute_blocks(*b);
        default_config(*b);
    });
    if (st != FDTD_OK) {
        create_error() = b->err;
        delete b;
        return st;
    }
    create_error().clear();
    *out = b;
    return FDTD_OK;
}

fdtd_status fdtd_batch_workspace_size(fdtd_batch *batch, size_t *bytes)
{
    if (!batch || !bytes) return FDTD_E_INVALID_ARG;
    size_t cur = 0;
    for (Plan *P : batch->plans) cur = al256(cur + P->ws_bytes);
    batch->r_table.off = cur;
    batch->r_table.bytes = table_layout((int)batch->plans.size()).bytes;
    batch->ws_bytes = cur + batch->r_table.bytes;
    *bytes = batch->ws_bytes;
    return FDTD_OK;
}

fdtd_status fdtd_batch_bind(fdtd_batch *batch, void *dptr, size_t bytes, void *stream)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    return bguard(batch, [&]() {
        Batch &B = *batch;
        size_t need = 0;
        BREQUIRE(fdtd_batch_workspace_size(batch, &need) == FDTD_OK, FDTD_E_INVALID_ARG, "size");
        BREQUIRE(dptr && ((uintptr_t)dptr & 255) == 0, FDTD_E_INVALID_ARG, "workspace null or misaligned");
        BREQUIRE(bytes >= need, FDTD_E_NOMEM, "workspace smaller than fdtd_batch_workspace_size");
        hipStream_t s = static_cast<hipStream_t>(stream);
        B.base = static_cast<char *>(dptr);
        size_t cur = 0;
        for (Plan *P : B.plans) {
            try {
                plan_bind_slice(*P, B.base + cur, P->ws_bytes, s);
            } catch (const std::exception &e) {
                throw BatchError(FDTD_E_HIP, std::string("binding a member plan: ") + e.what());
            }
            P->in_batch = true;
            cur = al256(cur + P->ws_bytes);
        }
        upload_tables(B, s);
        B.bound = true;
    });
}

fdtd_status fdtd_batch_reset(fdtd_batch *batch, void *stream)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    return bguard(batch, [&]() {
        BREQUIRE(batch->bound, FDTD_E_STATE, "batch not bound");
        for (Plan *P : batch->plans) plan_reset(*P, static_cast<hipStream_t>(stream));
    });
}

fdtd_status fdtd_batch_run(fdtd_batch *batch, int64_t nsteps, void *stream)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    return bguard(batch, [&]() { batch_run(*batch, nsteps, static_cast<hipStream_t>(stream)); });
}

fdtd_status fdtd_batch_get_config(const fdtd_batch *batch, int32_t *rows, int32_t *zchunk)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    if (rows) *rows = batch->cfg.rows;
    if (zchunk) *zchunk = batch->cfg.zchunk;
    return FDTD_OK;
}

fdtd_status fdtd_batch_set_config(fdtd_batch *batch, int32_t rows, int32_t zchunk)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    return bguard(batch, [&]() {
        BREQUIRE(valid_rows(rows), FDTD_E_INVALID_ARG, "tile rows must be 2, 4, 8, 12 or 16");
        BREQUIRE(zchunk >= 1 && zchunk <= 64, FDTD_E_INVALID_ARG, "z-chunk must be in [1, 64]");
        batch->cfg.rows = rows;
        batch->cfg.zchunk = zchunk;
        batch->cfg_auto = false;
        compute_blocks(*batch);
        if (batch->bound) upload_tables(*batch, nullptr);
    });
}

fdtd_status fdtd_batch_set_group_bytes(fdtd_batch *batch, uint64_t bytes)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    return bguard(batch, [&]() {
        batch->group_bytes = (size_t)bytes;
        batch->cfg.lockstep = 0;
        compute_blocks(*batch);
        if (batch->cfg_auto) default_config(*batch);
        if (batch->bound) upload_tables(*batch, nullptr);
    });
}

fdtd_status fdtd_batch_get_groups(const fdtd_batch *batch, int32_t *ngroups)
{
    if (!batch || !ngroups) return FDTD_E_INVALID_ARG;
    *ngroups = (int32_t)batch->groups.size();
    return FDTD_OK;
}

fdtd_status fdtd_batch_set_stream_stores(fdtd_batch *batch, int32_t mode)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    return bguard(batch, [&]() {
        BREQUIRE(mode >= -1 && mode <= 1, FDTD_E_INVALID_ARG, "stream-store mode must be -1, 0 or 1");
        batch->cfg.stream = mode;
    });
}

fdtd_status fdtd_batch_set_tile_order(fdtd_batch *batch, int32_t order)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    return bguard(batch, [&]() {
        BREQUIRE(valid_order(order), FDTD_E_INVALID_ARG, "tile order must be -1 or in [0, 4096]");
        batch->cfg.order = order;
    });
}

fdtd_status fdtd_batch_get_tile_order(const fdtd_batch *batch, int32_t *order, int32_t *used)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    if (order) *order = batch->cfg.order;
    if (used) *used = tile_order(batch->cfg, batch->ws_bytes);
    return FDTD_OK;
}

fdtd_status fdtd_batch_autotune(fdtd_batch *batch, int32_t trial_steps, const char *cache_path,
                                void *stream, int32_t *best_index)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    return bguard(batch, [&]() {
        Batch &B = *batch;
        BREQUIRE(B.bound, FDTD_E_STATE, "batch not bound");
        BREQUIRE(trial_steps >= 1, FDTD_E_INVALID_ARG, "trial_steps must be >= 1");
        hipStream_t s = static_cast<hipStream_t>(stream);
        // groups under the configured budget (a lockstep choice set aside)
        const LaunchCfg keep = B.cfg;
        B.cfg.lockstep = 0;
        compute_blocks(B);
        const size_t ngroups = B.groups.size();
        B.cfg = keep;
        compute_blocks(B);
        // the grouped schedule launches per group: its best shape differs,
        // and lockstep is searched beside it
        std::string key = tune_device_name() + "|" + tune_shape_key(B.plans.data(), B.plans.size());
        if (ngroups > 1) key += "groups=" + std::to_string(ngroups) + ";";
        TimerPause pause(B.timer);   // trial launches are not the caller's
        TuneHooks h;
        h.apply = [&](const LaunchCfg &c) {
            B.cfg = c;
            upload_tables(B, s);
        };
        h.run = [&](int32_t n) { batch_run(B, n, s); };
        h.schedules = ngroups > 1 ? 2 : 1;
        LaunchCfg best = B.cfg;
        int32_t best_i = -1;
        hcheck(tune_search(h, trial_steps, cache_path, key, s, best, best_i), "autotune");
        B.cfg_auto = false;
        if (best_i >= 0) {
            for (Plan *P : B.plans) plan_reset(*P, s);
            hcheck(hipStreamSynchronize(s), "sync");
        }
        if (best_index) *best_index = best_i;
    });
}

fdtd_status fdtd_batch_set_timing(fdtd_batch *batch, int32_t enable)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    return bguard(batch, [&]() {
        BREQUIRE(enable >= 0, FDTD_E_INVALID_ARG, "negative timing stride");
        hcheck(batch->timer.drain(), "timer drain");
        batch->timer.reset();
        batch->timer.on = enable != 0;
        batch->timer.every = enable > 1 ? enable : 1;
    });
}

fdtd_status fdtd_batch_get_kernel_time(fdtd_batch *batch, double *ms, int64_t *launches)
{
    if (!batch) return FDTD_E_INVALID_ARG;
    return bguard(batch, [&]() {
        hcheck(batch->timer.drain(), "timer drain");
        if (ms) *ms = batch->timer.ms;
        if (launches) *launches = batch->timer.launches;
    });
}

const char *fdtd_batch_last_error(const fdtd_batch *batch)
{
    return batch ? batch->err.c_str() : create_error().c_str();
}

void fdtd_batch_destroy(fdtd_batch *batch)
{
    if (!batch) return;
    for (Plan *P : batch->plans) {
        P->in_batch = false;
        P->bound = false;
    }
    batch->timer.destroy();
    delete batch;
}

}  // extern "C"
