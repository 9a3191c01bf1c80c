// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/fdtd.h"

namespace fdtd {

// Auxiliary (convolutional PML) arrays, one per (field component,
// derivative axis) pair.
enum PsiId {
    PSI_HXY, PSI_HXZ, PSI_HYZ, PSI_HYX, PSI_HZX, PSI_HZY,
    PSI_EXY, PSI_EXZ, PSI_EYZ, PSI_EYX, PSI_EZX, PSI_EZY, PSI_COUNT
};

// Per-axis profile tables, each n_axis long: E entries sit on integer
// positions, H entries half a cell further along the axis.
enum ProfId { PR_BE, PR_CE, PR_KE, PR_BH, PR_CH, PR_KH, PR_COUNT };

// Everything a field-update kernel needs about one grid.  Plain data so it
// can be passed by value or stored in a device table.
//
// Field storage: element (i, j, k), i in [-1, nx], j in [-1, ny],
// k in [-1, nz], sits at  off + i + px*j + px*py*k  with py = ny + 2; the
// guard layer stays zero.  After the last plane: a zero guard of 18 rows
// (read past by tile halos) and the 64-element sink.  Only i < nx, j < ny, k < nz is ever written: on
// the upper faces every component is either absent or tangential-PEC zero.
// Material ids: i + nx*(j + ny*k).
// Auxiliary arrays live only inside the layers:
//   x-layers  xs + Lx*(j + ny*k)   xs = i (i < lo) or i - nx + Lx
//   y-layers  i + nx*(ys + Ly*k)
//   z-layers  i + nx*(j + ny*zs)
// Fused plans ping-pong the H auxiliaries; E auxiliaries (read and written
// only by the thread that owns the cell) are updated in place.
template <typename T>
struct DevGrid {
    T *E[3], *H[3];          // fields read this step
    T *Eo[3], *Ho[3];        // fields written this step (== E/H in place)
    T *Em[3], *Hm[3];        // two-level launches: where the intermediate level
                             // of the rim and probe tiles goes (else unused)
    const uint8_t *tbflag;   // two-level launches: per tile, 1 = write the
                             // intermediate level of every own cell
    const void *ids[3];      // uint8 or uint16 per edge; fused plans: ids[0] holds
                             // all three packed in one word per cell (5 bits
                             // each in a uint16 if at most 32 coefficient
                             // sets, else 8 bits each in a uint32)
    const T *lut[3];         // per component [id][4] = Ca, Cb/d_first, Cb/d_second, 0
    T *psi[PSI_COUNT];       // auxiliaries read this step
    T *psi_o[PSI_COUNT];     // auxiliaries written this step (== psi in place)
    const T *prof[3];        // per axis: PR_COUNT tables of n_axis entries
    int64_t off;
    int64_t cstride;         // bytes from component c to c+1 of E, H, Eo and Ho
    int64_t sink;            // first of 64 elements per field array that are
                             // written by lanes without a cell and never read
    int32_t nx, ny, nz, px, py;
    int32_t id16;
    int32_t nlut;            // entries per LUT
    int32_t lo[3], hi[3];    // layer cells on the low / high face of each axis
    T ch[3];                 // dt / (mu0 d_axis)
    // soft source on Ez
    int32_t src_kind;
    int32_t src_box[6];
    double src_t0, src_w, src_fc, src_tau, src_amp, dt;
    const double *src_samples;   // SAMPLED: value for level m + 1 at [m]
    int64_t src_nsamp;
};

// Probe tables: every probe is a weighted sum of field samples.
struct DevProbes {
    const int64_t *toff;     // element offsets into a field array
    const int32_t *tcomp;    // 0..5 = Ex..Hz
    const double *tw;        // weights
    const int32_t *range;    // per probe: V terms [r0, r1), I terms [r2, r3)
    double *hist;            // [probe][2][K]
    int32_t K;
    int32_t nprobe;
};

struct LaunchCfg {
    int32_t rows = 4;        // tile rows (y) per block of the fused kernel
    int32_t zchunk = 32;     // planes marched per block
    int32_t tb_rows = 13;    // two-level kernel: tile rows (8, 10 or 13)
    int32_t tb_zchunk = 32;  // two-level kernel: planes marched per block (4..256)
    int32_t tb_depth = 2;    // levels per pass of the two-level tiles of a plan
                             // with the third buffer: 2, or 1 (single steps)
    int32_t lockstep = 0;    // batches: 1 = every member in one group whatever
                             // the group budget (set by the autotuner)
    int32_t order = -1;      // block-to-tile order (see tile_order), -1 = automatic
    int32_t stream = -1;     // streaming field stores (see stream_stores), -1 = automatic
};

// Blocks are dispatched to the 8 XCDs in turn.  Order 0 hands each XCD one
// contiguous run of tiles (neighbours share its L2: best while the state
// stays in the 256 MB memory-side cache); order k >= 1 deals runs of k
// tiles to the XCDs in turn (all XCDs work on one region of the grid at a
// time: better once the state streams from HBM).  Automatic: 0 up to that
// cache size, else 16.
constexpr size_t MALL_BYTES = (size_t)256 << 20;
// Static probe history ring of fdtd_run_noalloc: 32 probes x 2 signals x
// 512 samples x 8 bytes.
constexpr size_t NOALLOC_RING_BYTES = (size_t)256 << 10;
inline int32_t tile_order(const LaunchCfg &c, size_t state_bytes)
{
    return c.order >= 0 ? c.order : (state_bytes <= MALL_BYTES ? 0 : 16);
}
inline bool valid_order(int32_t order) { return order >= -1 && order <= 4096; }

// Streaming (non-temporal) stores of the output fields pay once the state
// clearly exceeds the memory-side cache (the outputs are next read a step
// later); for a state inside it, or not far above it (where much of it
// still hits), they push next step's inputs out of the cache.  Measured: a
// 400 x ny x 80 microstrip series turns faster from 296 MiB up, but sweep
// grids of 289 and 308 MiB turn much slower; 5-6 % faster from 365 MiB up
// in the series, 3.5 % on a 7 GiB line.  Automatic switches at 512 MiB.
constexpr size_t STREAM_BYTES = 2 * MALL_BYTES;
inline int32_t stream_stores(const LaunchCfg &c, size_t state_bytes)
{
    return c.stream >= 0 ? c.stream : (state_bytes > STREAM_BYTES ? 1 : 0);
}

// Tile heights the fused kernel is instantiated for.
inline bool valid_rows(int32_t rows)
{
    return rows == 2 || rows == 4 || rows == 8 || rows == 12 || rows == 16;
}

// Tile decomposition of one grid for the fused kernels.  A tile is 64 cells
// in x, `rows` in y and `zchunk` planes in z.  The tiles whose cells, halo
// cells (x0-1, y0-1) and first input plane (z0-1) all lie outside every
// absorbing layer form a box [ix0, ix1) x [iy0, iy1) x [iz0, iz1) of tile
// indices (the condition is separable per axis); they run through the
// interior kernel, the others through the boundary kernel.
// A ragged last x column of at most 32 cells is covered by nxw narrow
// tiles of 16 x 4R cells per (row of narrow tiles, z-chunk) instead of one
// mostly empty 64-wide tile; they run in the boundary launch, interleaved
// with the 64-wide boundary tiles.
struct TileSet {
    int32_t tx, ty, tz;               // 64-wide tiles per axis
    int32_t ix0, ix1, iy0, iy1, iz0, iz1;
    int32_t nb, ni;                   // boundary (incl. narrow) / interior tiles
    int32_t sb, si;                   // first block of this grid in each launch
    int32_t nxw, nty;                 // narrow sub-columns (0..2), narrow tile rows
};

// Two-level (temporally blocked) tiles: the cells [x0, x1) x [y0, y1) x
// [z0, z1) of the interior box, whose cells lie at least two cells away
// from every absorbing layer (and from the grid's x and y faces), cut into
// tiles of TB_W x rows x zc cells (ragged last tiles).  They advance two
// levels per pass; every other tile takes two single-level passes.
constexpr int TB_W = 60;
inline bool valid_tb_rows(int32_t r) { return r == 8 || r == 10 || r == 13; }
struct TBSet {
    int32_t x0, x1, y0, y1, z0, z1;
    int32_t rows, zc;
    int32_t ntx, nty, ntz, n;         // tiles per axis and in all (0: no two-level tiles)
};
// Most two-level tiles a grid can have (smallest tile shape), for the
// per-tile flags.
inline size_t tb_max_tiles(int nx, int ny, int nz)
{
    return (size_t)((nx + TB_W - 1) / TB_W) * ((ny + 7) / 8) * ((nz + 3) / 4);
}

// ---------------------------------------------------------------------------
// host-side plan
// ---------------------------------------------------------------------------
struct Region {
    size_t off = 0, bytes = 0;
};

// Pool of HIP event pairs that time the steps of a run in windows of
// `every` consecutive steps (one pair per window; a run's last window may
// be shorter).  A pair is read back only when it is about to be reused (or
// on drain), so timing never stalls the launch queue.
struct KernelTimer {
    static constexpr size_t SLOTS = 512;
    bool on = false;
    int32_t every = 1;            // steps per window
    double ms = 0;
    int64_t launches = 0;         // steps of the windows read back
    std::vector<hipEvent_t> ev;   // 2 per slot
    std::vector<int64_t> used;    // steps of the slot's closed window, 0 = free
    size_t next = 0;
    long open = -1;               // slot of the open window
    int32_t in_window = 0;        // steps in the open window
    // Events to record around the next step: a opens a window, b closes it
    // (full, or `last` step of the run); either may be null.  A window left
    // open by a run that failed is dropped at the `first` step of the next.
    // (count: steps the bracketed launches advance, 2 for a two-level pass)
    hipError_t step(hipEvent_t &a, hipEvent_t &b, bool first, bool last, int32_t count = 1);
    hipError_t drain();
    void reset();
    void destroy();
};

// Keeps launches out of a timer for a scope (restored also when it unwinds).
struct TimerPause {
    KernelTimer &t;
    bool keep;
    explicit TimerPause(KernelTimer &k) : t(k), keep(k.on) { t.on = false; }
    ~TimerPause() { t.on = keep; }
    TimerPause(const TimerPause &) = delete;
    TimerPause &operator=(const TimerPause &) = delete;
};

struct Plan {
    fdtd_grid g{};
    std::vector<uint8_t> cells;
    std::vector<fdtd_material> mats;
    fdtd_boundary bnd{};
    std::vector<fdtd_port> ports;
    struct Point { int32_t comp, i, j, k; };
    std::vector<Point> points;
    fdtd_source src{};
    std::vector<double> src_samples;     // SAMPLED source values (level m + 1 at [m])
    std::vector<double> freqs;

    // derived at finalize
    bool finalized = false;
    double dt = 0, eps0 = 0, mu0 = 0, c0 = 0;
    int32_t px = 0, py = 0, pz = 0;
    size_t field_elems = 0, id_elems = 0;
    size_t cstride = 0;                  // bytes between field components
    size_t sink = 0;                     // first of 64 write-only elements per field array
    int32_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    int32_t id16 = 0;
    int32_t id_bits = 8;                 // fused plans: bits per packed id (5 or 8)
    bool wide_ids = false;               // set by a batch: pack ids in 32 bits regardless
    std::vector<uint16_t> ids[3];
    std::vector<double> lut[3];          // [id][4]
    std::vector<double> prof[3];         // [PR_COUNT][n_axis]
    size_t psi_elems[PSI_COUNT] = {};
    std::vector<int64_t> toff;
    std::vector<int32_t> tcomp;
    std::vector<double> tw;
    std::vector<int32_t> prange;
    int32_t K = 512;                     // probe history ring length
    int32_t nbuf = 1;                    // field buffers (2 for ping-pong, 3 with
                                         // two-level steps)
    int32_t tb_mode = -1;                // two-level steps: 1 on, 0 off, -1 automatic
    bool tb = false;                     // finalized with the third buffer
    TBSet tbset{};                       // two-level tiles of the current launch shape
    std::vector<uint8_t> tbflags;        // per two-level tile: holds a probe term
    size_t elt = 4;                      // bytes per field value

    // workspace layout (offsets relative to the bound pointer)
    Region r_ids[3], r_lut[3], r_prof[3], r_toff, r_tcomp, r_tw, r_range, r_freq, r_src;
    Region r_E[3][3], r_H[3][3], r_psi[2][PSI_COUNT], r_hist, r_acc;
    Region r_grid;                       // fused plans: launch table (DevGrids, tile sets, probes)
    Region r_tbflag;                     // two-level plans: per-tile flags
    Region r_static, r_mut;
    size_t ws_bytes = 0;

    // bound state
    char *base = nullptr;
    bool bound = false;
    bool in_batch = false;
    int64_t step = 0;                    // completed steps
    int64_t dft_n = 0;                   // last sample folded into the DFT
    int64_t sampled = 0;                 // last sample written to the history ring
    int32_t parity = 0;                  // which field buffer holds the current level
                                         // (0..nbuf-1); the H auxiliaries of the
                                         // current level are in copy (step & 1)
    int32_t ring_dev = -1;               // device the plan is bound on
    double *ring = nullptr;              // its static history ring (fdtd_run_noalloc)
    LaunchCfg cfg;
    TileSet tiles{};                     // fused plans: decomposition on the device
    LaunchCfg tiles_cfg{0, 0};           // the launch shape `tiles` was made for

    KernelTimer timer;

    std::string err;

    int nprobe() const { return (int)(ports.size() + points.size()); }
    int nf() const { return (int)freqs.size(); }
    template <typename T> DevGrid<T> dev_grid() const;
    // Single-level step from field buffer `cur` (into the next one) with
    // the H auxiliaries of copy pp; two-level pass from buffer cur.
    DevGrid<float> dev_grid_at(int cur, int pp) const;
    DevGrid<float> dev_grid_tb(int cur) const;
};

struct Batch {
    std::vector<Plan *> plans;
    LaunchCfg cfg;
    Region r_table;
    size_t ws_bytes = 0;
    char *base = nullptr;
    bool bound = false;
    std::vector<TileSet> sets;          // per plan: tile decomposition and first blocks
    int32_t nb_total = 0, ni_total = 0; // boundary / interior tiles of all plans
    // Groups of consecutive members whose state fits group_bytes (0: one
    // group of all); with several, a run advances one group at a time.
    size_t group_bytes = MALL_BYTES;
    bool cfg_auto = true;               // launch shape not set by the caller
    struct Group { int32_t first, count, nb, ni; size_t bytes; };
    std::vector<Group> groups;
    std::vector<TileSet> gsets;         // as sets, first blocks counted per group
    int32_t lut_cap = 1;                // largest coefficient table of the plans
    int32_t id_bits = 8;                // 5 if every plan packs its ids in 16 bits
    int32_t max_probes = 0;
    int32_t max_nf = 0;
    KernelTimer timer;
    std::string err;
};

// DFT accumulation for one grid's probes.
struct DevDft {
    const double *hist;      // [probe][2][K]
    double *acc;             // [probe][2][nf][2]
    const double *freqs;
    int32_t nf, nprobe, K;
    double dt;
};

// kernel launchers (kernels.hip / fused.hip)
template <typename T>
hipError_t launch_plain_step(const DevGrid<T> &d, int64_t level, hipStream_t s,
                             hipEvent_t e0, hipEvent_t e1);
template <typename T>
hipError_t launch_probe(const DevGrid<T> &d, const DevProbes &p, int64_t sample, hipStream_t s);
hipError_t launch_dft(const DevDft &d, int64_t n_first, int64_t count, hipStream_t s);
// One fused step of ninst grids (device tables grids_dev and sets_dev;
// nb boundary and ni interior tiles in all): a boundary launch then an
// interior launch.  With sample_input the boundary launch also samples every
// probe of the input level `level` (if level >= 1).
// lut_cap: LUT entries per component the launch reserves in LDS (at least
// the largest nlut of the instances, at most 256).  id_bits: 5 when every
// instance packs its ids into 16-bit words (at most 32 coefficient sets),
// else 8 (32-bit words).
hipError_t launch_fused(const DevGrid<float> *grids_dev, const TileSet *sets_dev, int32_t ninst,
                        int32_t nb, int32_t ni, const LaunchCfg &cfg, int32_t lut_cap,
                        int32_t id_bits, int64_t level, const DevProbes *probes_dev,
                        int32_t max_probes, bool sample_input, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1);
// Two-level pass over the tiles of `set`: reads levels n (`level`) from
// g.E/g.H, writes level n+2 to g.Eo/g.Ho and level n+1 of the rim and probe
// tiles to g.Em/g.Hm.
hipError_t launch_tb(const DevGrid<float> *g_dev, const TBSet *set_dev, int32_t ntiles,
                     const LaunchCfg &cfg, int32_t lut_cap, int32_t id_bits, int64_t level,
                     hipStream_t s);
hipError_t launch_probe_batch(const DevGrid<float> *grids_dev, const DevProbes *probes_dev,
                              int32_t ninst, int32_t max_probes, int64_t sample, hipStream_t s);
hipError_t launch_dft_batch(const DevDft *dft_dev, int32_t ninst, int32_t max_probes,
                            int32_t max_nf, int64_t n_first, int64_t count, hipStream_t s);
// Tile decomposition of grid P under cfg (sb, si left zero).
TileSet make_tileset(const Plan &P, const LaunchCfg &cfg);
// Two-level tiles of P under cfg; shrinks the interior box of t (made by
// make_tileset with cfg) to the tiles whose two-cell margin avoids the layers.
TBSet make_tbset(const Plan &P, const LaunchCfg &cfg, TileSet &t);
// Default launch shape for one step of the given grids.
LaunchCfg default_launch(const Plan *const *plans, size_t n);

// Launch-shape search.  apply() installs a shape, run(n) enqueues n steps on
// the stream being timed; both throw on failure.
struct TuneHooks {
    std::function<void(const LaunchCfg &)> apply;
    std::function<void(int32_t)> run;
    bool two_level = false;  // a plan with the third buffer: also search the
                             // depth and tile shape of its two-level passes
    int32_t schedules = 1;   // 2: a grouped batch, searched grouped and in lockstep
};
// GPU architecture name of the current device (the cache key's first part).
std::string tune_device_name();
// "NXxNYxNZ;" per grid, in order (the cache key's second part).
std::string tune_shape_key(const Plan *const *plans, size_t n);
// Times every candidate shape for trial_steps steps after one warm-up step
// and applies the fastest; with cache_path, a stored shape for key is applied
// instead (best_index = -1) and a timed winner is stored.  The first stage
// searches (schedule, rows, z-chunk, order) in lexicographic order (index
// i1 < 50 * schedules; schedule 0 is the configured one, 1 lockstep);
// with two_level, a second stage keeps that winner and searches two-level
// passes over (tile rows, z-chunk) in lexicographic order, then single
// steps (index i2 < 13).  best_index = i1 (+ 50 * i2 with two_level).
hipError_t tune_search(const TuneHooks &h, int32_t trial_steps, const char *cache_path,
                       const std::string &key, hipStream_t s, LaunchCfg &best_cfg, int32_t &best_index);

}  // namespace fdtd

// The opaque handles of the C interface are the host-side objects.
struct fdtd_plan : fdtd::Plan {};
struct fdtd_batch : fdtd::Batch {};
