// Host side of the library: plan construction (per-edge coefficients,
// absorbing-layer profiles, probe tables), workspace layout, binding, the
// step loop and the C interface declared in include/fdtd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <new>
#include <stdexcept>
#include <utility>

#include "internal.hpp"



namespace fdtd {

struct ApiError : std::runtime_error {
    fdtd_status code;
    ApiError(fdtd_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define REQUIRE(cond, code, msg)                                   \
    do {                                                           \
        if (!(cond)) throw ::fdtd::ApiError((code), (msg));        \
    } while (0)

static void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess)
        throw ApiError(FDTD_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
static fdtd_status guarded(Plan *p, F &&f)
{
    try {
        f();
        if (p) p->err.clear();
        return FDTD_OK;
    } catch (const ApiError &e) {
        if (p) p->err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        if (p) p->err = "host allocation failed";
        return FDTD_E_NOMEM;
    } catch (const std::exception &e) {
        if (p) p->err = e.what();
        return FDTD_E_INVALID_ARG;
    }
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Layout of a fused plan's launch table (region r_grid): the descriptors of
// a single-level step from each field buffer with each copy of the H
// auxiliaries (index 2 * buffer + copy), those of a two-level pass from each
// buffer, the tile decomposition, the two-level tiles, the probes.
static constexpr size_t GRID_TB_OFF = 6 * sizeof(DevGrid<float>);
static constexpr size_t GRID_SET_OFF = 9 * sizeof(DevGrid<float>);
static constexpr size_t GRID_TBSET_OFF = (GRID_SET_OFF + sizeof(TileSet) + 63) & ~size_t(63);
static constexpr size_t GRID_PROBES_OFF = (GRID_TBSET_OFF + sizeof(TBSet) + 63) & ~size_t(63);
// the probe table again, pointing at the static history ring of
// fdtd_run_noalloc instead of the workspace's
static constexpr size_t GRID_PROBES2_OFF = (GRID_PROBES_OFF + sizeof(DevProbes) + 63) & ~size_t(63);

// ---------------------------------------------------------------------------
// static history ring of the allocation-free run
// ---------------------------------------------------------------------------
// fdtd_run_noalloc keeps the probe history ring (the FP64 staging between
// each step's port sums and the DFT fold) in this file-scope device array
// instead of the caller's workspace.  Every GPU holds its own copy until the
// process ends; in host code the name is only a stand-in, so kernels get the
// address hipGetSymbolAddress returns for the current device (looked up
// once per device when a plan is bound there).  No slot needs clearing: a run
// folds every sample it writes before it returns, and writes each slot
// before reading it.
static __device__ __align__(256) double scratch[NOALLOC_RING_BYTES / sizeof(double)];

static std::mutex g_scratch_mu;
static std::unordered_map<int, double *> g_scratch;   // device -> address of `scratch`

// Address of `scratch` on the current device (looked up once per device).
static hipError_t scratch_ring(int &dev, double *&ptr)
{
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        ptr = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr = static_cast<double *>(p);
    g_scratch[dev] = ptr;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// finalize: everything derived from the description
// ---------------------------------------------------------------------------

// Per-edge Ca, Cb.  An edge is PEC when it lies on a domain face it is
// tangential to (every face is PEC or PEC-backed) or when a cell sharing it
// is PEC; otherwise eps and sigma are averaged over the (four) cells that
// share it.
static void build_coefficients(Plan &P)
{
    const int nx = P.g.nx, ny = P.g.ny, nz = P.g.nz;
    std::map<std::pair<double, double>, int> uniq;
    std::vector<std::pair<double, double>> table;
    auto lookup = [&](double ca, double cb) {
        auto key = std::make_pair(ca, cb);
        auto it = uniq.find(key);
        if (it != uniq.end()) return it->second;
        int id = (int)table.size();
        uniq.emplace(key, id);
        table.push_back(key);
        return id;
    };
    auto cell = [&](int i, int j, int k) -> uint32_t {
        return P.cells[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)];
    };
    // coefficient id of an edge from the ids of its four cells (memoized:
    // neighbouring edges almost always share their materials)
    std::unordered_map<uint32_t, int> memo;
    auto coef_id = [&](uint32_t key, const uint32_t m4[4]) {
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
        bool pec = false;
        double se = 0, ss = 0;
        for (int q = 0; q < 4; ++q) {
            const fdtd_material &m = P.mats[m4[q]];
            pec = pec || m.is_pec;
            se += m.eps_r;
            ss += m.sigma;
        }
        double ca = 0, cb = 0;
        if (!pec) {
            const double eps = P.eps0 * (se / 4.0);
            const double sig = ss / 4.0;
            const double half_loss = sig * P.dt / (2.0 * eps);
            ca = (1.0 - half_loss) / (1.0 + half_loss);
            cb = (P.dt / eps) / (1.0 + half_loss);
        }
        const int id = lookup(ca, cb);
        memo.emplace(key, id);
        return id;
    };
    const int pec_id = lookup(0.0, 0.0);
    for (int comp = 0; comp < 3; ++comp) {
        P.ids[comp].assign(P.id_elems, 0);
        // the two axes across the edge
        const int a1 = (comp + 1) % 3, a2 = (comp + 2) % 3;
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j) {
                uint32_t last_key = 0xffffffffu;
                int last_id = 0;
                for (int i = 0; i < nx; ++i) {
                    const int pos[3] = {i, j, k};
                    int id;
                    if (pos[a1] == 0 || pos[a2] == 0) {
                        id = pec_id;
                    } else {
                        uint32_t m4[4], key = 0;
                        int q = 0;
                        for (int d2 = -1; d2 <= 0; ++d2)
                            for (int d1 = -1; d1 <= 0; ++d1) {
                                int c[3] = {i, j, k};
                                c[a1] += d1;
                                c[a2] += d2;
                                m4[q] = cell(c[0], c[1], c[2]);
                                key = (key << 8) | m4[q];
                                ++q;
                            }
                        id = key == last_key ? last_id : coef_id(key, m4);
                        last_key = key;
                        last_id = id;
                    }
                    P.ids[comp][(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)] =
                        (uint16_t)std::min(id, 65535);
                }
            }
    }
    REQUIRE(table.size() <= 65536, FDTD_E_UNSUPPORTED,
            "more than 65536 distinct edge coefficients");
    P.id16 = table.size() > 256 ? 1 : 0;
    P.id_bits = table.size() <= 32 && !P.wide_ids ? 5 : 8;
    const double d[3] = {P.g.dx, P.g.dy, P.g.dz};
    for (int comp = 0; comp < 3; ++comp) {
        // E_comp = Ca E + Cb/d_first * diff_first - Cb/d_second * diff_second,
        // first axis = comp+1, second = comp+2 (cyclic)
        const double d1 = d[(comp + 1) % 3], d2 = d[(comp + 2) % 3];
        P.lut[comp].assign(table.size() * 4, 0.0);
        for (size_t t = 0; t < table.size(); ++t) {
            P.lut[comp][4 * t + 0] = table[t].first;
            P.lut[comp][4 * t + 1] = table[t].second / d1;
            P.lut[comp][4 * t + 2] = table[t].second / d2;
        }
    }
}

// Convolutional-PML tables along one axis (Roden-Gedney form with the
// polynomial grading of the fdtd_boundary documentation).
static void build_profiles(Plan &P, int axis)
{
    const int n = axis == 0 ? P.g.nx : axis == 1 ? P.g.ny : P.g.nz;
    const double dl = axis == 0 ? P.g.dx : axis == 1 ? P.g.dy : P.g.dz;
    const int lo = P.lo[axis], hi = P.hi[axis];
    const fdtd_boundary &B = P.bnd;
    const double eta0 = P.mu0 * P.c0;
    const double smax = B.sigma_max > 0 ? B.sigma_max : 0.8 * (B.m + 1.0) / (eta0 * dl);
    P.prof[axis].assign((size_t)PR_COUNT * n, 0.0);
    auto put = [&](int base, int idx, double x_cells) {
        double rho = 0, depth = 1;
        if (lo > 0 && x_cells < lo) { rho = lo - x_cells; depth = lo; }
        if (hi > 0 && x_cells > n - hi) { rho = x_cells - (n - hi); depth = hi; }
        double b = 1, c = 0, ik = 1;
        if (rho > 0) {
            const double u = rho / depth, um = std::pow(u, B.m);
            const double sg = smax * um;
            const double ka = 1.0 + (B.kappa_max - 1.0) * um;
            const double al = B.alpha_max * (1.0 - u);
            b = std::exp(-(sg / ka + al) * P.dt / P.eps0);
            const double den = ka * (sg + ka * al);
            c = den > 0 ? sg * (b - 1.0) / den : 0.0;
            ik = 1.0 / ka;
        }
        P.prof[axis][(size_t)(base + 0) * n + idx] = b;
        P.prof[axis][(size_t)(base + 1) * n + idx] = c;
        P.prof[axis][(size_t)(base + 2) * n + idx] = ik;
    };
    for (int p = 0; p < n; ++p) {
        put(PR_BE, p, (double)p);
        put(PR_BH, p, p + 0.5);
    }
}

static int64_t field_index(const Plan &P, int i, int j, int k)
{
    return (int64_t)(64 + (size_t)P.px * (1 + (size_t)P.py)) + i + (int64_t)P.px * j +
           (int64_t)P.px * P.py * k;
}

static void add_term(Plan &P, int comp, int i, int j, int k, double w)
{
    P.toff.push_back(field_index(P, i, j, k));
    P.tcomp.push_back(comp);
    P.tw.push_back(w);
}

// Probe term lists.  Port voltage: -(1/w) sum_j omega_j sum_k Ez dz dy over
// the Ez edges of the plane between ground and strip (trapezoid across the
// strip width).  Port current: dir * 1/2 * (loop(i-1/2) + loop(i+1/2)), each
// loop the counter-clockwise (seen from +x) integral of H over the H nodes
// half a cell outside the strip.
static void build_probes(Plan &P)
{
    P.toff.clear(); P.tcomp.clear(); P.tw.clear(); P.prange.clear();
    const double dy = P.g.dy, dz = P.g.dz;
    for (const fdtd_port &q : P.ports) {
        const int v0 = (int)P.tw.size();
        const double width = (q.y1 - q.y0) * dy;
        for (int j = q.y0; j <= q.y1; ++j) {
            const double om = (j == q.y0 || j == q.y1) ? 0.5 : 1.0;
            for (int k = 0; k < q.z0; ++k) add_term(P, FDTD_EZ, q.i, j, k, -om * dz * dy / width);
        }
        const int v1 = (int)P.tw.size();
        for (int m = q.i - 1; m <= q.i; ++m) {
            const double h = 0.5 * q.dir;
            for (int j = q.y0; j <= q.y1; ++j) add_term(P, FDTD_HY, m, j, q.z0 - 1, h * dy);
            for (int k = q.z0; k <= q.z1; ++k) add_term(P, FDTD_HZ, m, q.y1, k, h * dz);
            for (int j = q.y0; j <= q.y1; ++j) add_term(P, FDTD_HY, m, j, q.z1, -h * dy);
            for (int k = q.z0; k <= q.z1; ++k) add_term(P, FDTD_HZ, m, q.y0 - 1, k, -h * dz);
        }
        const int i1 = (int)P.tw.size();
        P.prange.insert(P.prange.end(), {v0, v1, v1, i1});
    }
    for (const Plan::Point &q : P.points) {
        const int v0 = (int)P.tw.size();
        add_term(P, q.comp, q.i, q.j, q.k, 1.0);
        const int v1 = (int)P.tw.size();
        P.prange.insert(P.prange.end(), {v0, v1, v1, v1});
    }
}

static void layout(Plan &P)
{
    size_t cur = 0;
    auto take = [&](Region &r, size_t bytes) {
        r.off = cur;
        r.bytes = bytes;
        cur = align256(cur + bytes);
    };
    const size_t elt = P.elt;
    // static tables
    P.r_static.off = 0;
    if (P.g.kernel == FDTD_KERNEL_FUSED) {
        // fused plans: the three ids of a cell packed into one 32-bit word
        take(P.r_ids[0], P.id_elems * (P.id_bits == 5 ? 2 : 4));
        take(P.r_ids[1], 0);
        take(P.r_ids[2], 0);
    } else {
        for (int c = 0; c < 3; ++c) take(P.r_ids[c], P.id_elems * (P.id16 ? 2 : 1));
    }
    for (int c = 0; c < 3; ++c) take(P.r_lut[c], P.lut[c].size() * elt);
    for (int a = 0; a < 3; ++a) take(P.r_prof[a], P.prof[a].size() * elt);
    take(P.r_toff, std::max<size_t>(1, P.toff.size()) * 8);
    take(P.r_tcomp, std::max<size_t>(1, P.tcomp.size()) * 4);
    take(P.r_tw, std::max<size_t>(1, P.tw.size()) * 8);
    take(P.r_range, std::max<size_t>(1, P.prange.size()) * 4);
    take(P.r_freq, std::max<size_t>(1, P.freqs.size()) * 8);
    take(P.r_src, std::max<size_t>(1, P.src_samples.size()) * 8);
    take(P.r_grid, GRID_PROBES2_OFF + sizeof(DevProbes) + 64);
    take(P.r_tbflag, P.tb ? tb_max_tiles(P.g.nx, P.g.ny, P.g.nz) : 1);
    P.r_static.bytes = cur;
    // mutable state
    P.r_mut.off = cur;
    for (int b = 0; b < P.nbuf; ++b)
        for (int c = 0; c < 3; ++c) {
            take(P.r_E[b][c], P.field_elems * elt);
            take(P.r_H[b][c], P.field_elems * elt);
        }
    // ping-pong only for the H auxiliaries: tile halos read those of
    // neighbouring cells, while an E auxiliary is read and written by the
    // thread that owns its cell alone, so it is updated in place
    // (two copies at most: with three field buffers the H auxiliaries still
    // alternate level by level, and only the single-level passes use them)
    for (int b = 0; b < std::min(P.nbuf, 2); ++b)
        for (int q = 0; q < PSI_COUNT; ++q) {
            if (b > 0 && q >= PSI_EXY) P.r_psi[b][q] = P.r_psi[0][q];
            else take(P.r_psi[b][q], std::max<size_t>(1, P.psi_elems[q]) * elt);
        }
    if (P.nbuf == 1)
        for (int q = 0; q < PSI_COUNT; ++q) P.r_psi[1][q] = P.r_psi[0][q];
    // the components of every field sit at one fixed stride (E and H interleave)
    P.cstride = P.r_E[0][1].off - P.r_E[0][0].off;
    for (int b = 0; b < P.nbuf; ++b)
        for (int c = 1; c < 3; ++c)
            REQUIRE(P.r_E[b][c].off - P.r_E[b][c - 1].off == P.cstride &&
                        P.r_H[b][c].off - P.r_H[b][c - 1].off == P.cstride,
                    FDTD_E_UNSUPPORTED, "field components are not evenly spaced");
    take(P.r_hist, std::max<size_t>(1, (size_t)P.nprobe() * 2 * P.K) * 8);
    take(P.r_acc, std::max<size_t>(1, (size_t)P.nprobe() * 2 * P.nf() * 2) * 8);
    P.r_mut.bytes = cur - P.r_mut.off;
    P.ws_bytes = cur;
}

static void finalize(Plan &P)
{
    if (P.finalized) return;
    const fdtd_grid &g = P.g;
    REQUIRE(!P.cells.empty(), FDTD_E_STATE, "materials not set");
    REQUIRE(!P.freqs.empty(), FDTD_E_STATE, "frequencies not set");
    REQUIRE(P.src.kind != FDTD_WAVE_SAMPLED || !P.src_samples.empty(), FDTD_E_STATE,
            "sampled source without samples");
    const bool norm = g.units == FDTD_NORMALIZED;
    P.c0 = norm ? 1.0 : 299792458.0;
    P.mu0 = norm ? 1.0 : 4.0e-7 * M_PI;
    P.eps0 = 1.0 / (P.mu0 * P.c0 * P.c0);
    const double s = 1.0 / (g.dx * g.dx) + 1.0 / (g.dy * g.dy) + 1.0 / (g.dz * g.dz);
    P.dt = g.courant / (P.c0 * std::sqrt(s));
    // x rows padded to 32 elements: 64-lane row loads stay on whole 128-byte lines
    P.px = (int32_t)(((size_t)g.nx + 2 + 31) / 32 * 32);
    P.py = g.ny + 2;
    P.pz = g.nz + 2;
    // trailing guard: tile halo rows of the fused kernel may run up to 17 rows
    // past the last plane; then 64 sink elements that only receive the
    // stores of fused-kernel lanes without a cell (never read)
    P.sink = 64 + (size_t)P.px * P.py * P.pz + (size_t)P.px * 18;
    P.field_elems = P.sink + 64;
    P.id_elems = (size_t)g.nx * g.ny * g.nz;
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
        P.lo[a] = P.bnd.face[2 * a] == FDTD_FACE_CPML ? P.bnd.cells[2 * a] : 0;
        P.hi[a] = P.bnd.face[2 * a + 1] == FDTD_FACE_CPML ? P.bnd.cells[2 * a + 1] : 0;
        REQUIRE(P.lo[a] + P.hi[a] <= n[a], FDTD_E_INVALID_ARG, "absorbing layers overlap");
    }
    P.elt = g.precision == FDTD_FP64 ? 8 : 4;
    P.nbuf = g.kernel == FDTD_KERNEL_FUSED ? 2 : 1;
    // the fused kernel addresses every array with 32-bit byte offsets
    REQUIRE(g.kernel != FDTD_KERNEL_FUSED || P.field_elems * 4 < ((size_t)1 << 32),
            FDTD_E_UNSUPPORTED, "grid too large for one fused plan (field array >= 4 GiB)");
    const size_t Lx = P.lo[0] + P.hi[0], Ly = P.lo[1] + P.hi[1], Lz = P.lo[2] + P.hi[2];
    const size_t xl = Lx * g.ny * g.nz, yl = (size_t)g.nx * Ly * g.nz,
                 zl = (size_t)g.nx * g.ny * Lz;
    const size_t sz[PSI_COUNT] = {yl, zl, zl, xl, xl, yl, yl, zl, zl, xl, xl, yl};
    for (int q = 0; q < PSI_COUNT; ++q) P.psi_elems[q] = sz[q];
    build_coefficients(P);
    // the fused kernel keeps the coefficient tables in LDS, indexed by 8-bit ids
    REQUIRE(g.kernel != FDTD_KERNEL_FUSED || !P.id16, FDTD_E_UNSUPPORTED,
            "the fused kernel supports at most 256 distinct edge coefficients");
    for (int a = 0; a < 3; ++a) build_profiles(P, a);
    build_probes(P);
    // two-level steps need a third field buffer: on request, or (automatic)
    // for a state that streams from HBM (beyond twice the memory-side
    // cache) whose default launch shape leaves two-level tiles
    P.tb = false;
    layout(P);
    if (g.kernel == FDTD_KERNEL_FUSED && P.tb_mode != 0) {
        bool want = P.tb_mode == 1;
        if (P.tb_mode < 0 && P.ws_bytes > STREAM_BYTES) {
            TileSet t = make_tileset(P, P.cfg);
            want = make_tbset(P, P.cfg, t).n > 0;
        }
        if (want) {
            P.tb = true;
            P.nbuf = 3;
            layout(P);
        }
    }
    P.finalized = true;
}

template <typename T>
DevGrid<T> Plan::dev_grid() const
{
    DevGrid<T> d{};
    const int b = parity, o = nbuf == 2 ? 1 - parity : (nbuf == 3 ? (parity + 1) % 3 : parity);
    // H auxiliaries: copy (step & 1) with three field buffers
    const int pb = nbuf == 3 ? (int)(step & 1) : (nbuf == 2 ? b : 0);
    const int po = nbuf == 1 ? pb : 1 - pb;
    for (int c = 0; c < 3; ++c) {
        d.E[c] = reinterpret_cast<T *>(base + r_E[b][c].off);
        d.H[c] = reinterpret_cast<T *>(base + r_H[b][c].off);
        d.Eo[c] = reinterpret_cast<T *>(base + r_E[o][c].off);
        d.Ho[c] = reinterpret_cast<T *>(base + r_H[o][c].off);
        d.Em[c] = d.Eo[c];
        d.Hm[c] = d.Ho[c];
        d.ids[c] = base + r_ids[c].off;
        d.lut[c] = reinterpret_cast<const T *>(base + r_lut[c].off);
        d.prof[c] = reinterpret_cast<const T *>(base + r_prof[c].off);
    }
    for (int q = 0; q < PSI_COUNT; ++q) {
        d.psi[q] = reinterpret_cast<T *>(base + r_psi[pb][q].off);
        d.psi_o[q] = reinterpret_cast<T *>(base + r_psi[po][q].off);
    }
    d.tbflag = reinterpret_cast<const uint8_t *>(base + r_tbflag.off);
    d.off = 64 + (int64_t)px * (1 + py);
    d.cstride = (int64_t)cstride;
    d.sink = (int64_t)sink;
    d.nx = g.nx; d.ny = g.ny; d.nz = g.nz; d.px = px; d.py = py;
    d.id16 = id16;
    d.nlut = (int32_t)(lut[0].size() / 4);
    for (int a = 0; a < 3; ++a) { d.lo[a] = lo[a]; d.hi[a] = hi[a]; }
    d.ch[0] = (T)(dt / (mu0 * g.dx));
    d.ch[1] = (T)(dt / (mu0 * g.dy));
    d.ch[2] = (T)(dt / (mu0 * g.dz));
    d.src_kind = src.kind;
    for (int q = 0; q < 6; ++q) d.src_box[q] = src.box[q];
    d.dt = dt;
    d.src_samples = reinterpret_cast<const double *>(base + r_src.off);
    d.src_nsamp = (int64_t)src_samples.size();
    d.src_amp = src.amplitude;
    d.src_fc = src.fc;
    d.src_w = src.width;
    d.src_tau = src.bandwidth > 0 ? 2.0 * std::sqrt(std::log(1000.0)) / (M_PI * src.bandwidth) : 0.0;
    if (src.kind == FDTD_WAVE_GAUSS_SINE)
        d.src_t0 = src.t0 > 0 ? src.t0 : 3.0 * d.src_tau;
    else if (src.kind == FDTD_WAVE_DIFF_GAUSSIAN)
        d.src_t0 = src.t0 > 0 ? src.t0 : 3.0 * src.width;
    else
        d.src_t0 = src.t0;
    return d;
}

DevGrid<float> Plan::dev_grid_at(int cur, int pp) const
{
    DevGrid<float> d = dev_grid<float>();
    const int o = nbuf == 1 ? cur : (cur + 1) % nbuf;
    for (int c = 0; c < 3; ++c) {
        d.E[c] = reinterpret_cast<float *>(base + r_E[cur][c].off);
        d.H[c] = reinterpret_cast<float *>(base + r_H[cur][c].off);
        d.Eo[c] = reinterpret_cast<float *>(base + r_E[o][c].off);
        d.Ho[c] = reinterpret_cast<float *>(base + r_H[o][c].off);
        d.Em[c] = d.Eo[c];
        d.Hm[c] = d.Ho[c];
    }
    const int po = nbuf == 1 ? pp : 1 - pp;
    for (int q = 0; q < PSI_COUNT; ++q) {
        d.psi[q] = reinterpret_cast<float *>(base + r_psi[pp][q].off);
        d.psi_o[q] = reinterpret_cast<float *>(base + r_psi[po][q].off);
    }
    return d;
}

DevGrid<float> Plan::dev_grid_tb(int cur) const
{
    DevGrid<float> d = dev_grid_at(cur % nbuf, 0);
    const int m = (cur + 1) % nbuf, o = (cur + 2) % nbuf;
    for (int c = 0; c < 3; ++c) {
        d.Em[c] = reinterpret_cast<float *>(base + r_E[m][c].off);
        d.Hm[c] = reinterpret_cast<float *>(base + r_H[m][c].off);
        d.Eo[c] = reinterpret_cast<float *>(base + r_E[o][c].off);
        d.Ho[c] = reinterpret_cast<float *>(base + r_H[o][c].off);
    }
    return d;
}

template DevGrid<float> Plan::dev_grid<float>() const;
template DevGrid<double> Plan::dev_grid<double>() const;

LaunchCfg default_launch(const Plan *const *plans, size_t n)
{
    // 8-row tiles, and the longest z-chunk (16, 8 or 4 planes) that still
    // gives each of the 256 CUs about 8 tiles
    LaunchCfg c;
    c.rows = 8;
    for (c.zchunk = 16; c.zchunk > 4; c.zchunk /= 2) {
        int64_t tiles = 0;
        for (size_t q = 0; q < n; ++q) {
            const fdtd_grid &g = plans[q]->g;
            tiles += (int64_t)((g.nx + 63) / 64) * ((g.ny + 7) / 8) * ((g.nz + c.zchunk - 1) / c.zchunk);
        }
        if (tiles >= 2048) break;
    }
    return c;
}

TileSet make_tileset(const Plan &P, const LaunchCfg &cfg)
{
    TileSet t{};
    const int n[3] = {P.g.nx, P.g.ny, P.g.nz};
    const int w[3] = {64, cfg.rows, cfg.zchunk};
    // a last x column of 1..32 cells goes to 16-wide tiles
    const int rx = P.g.nx % 64;
    t.nxw = (rx > 0 && rx <= 32) ? (rx + 15) / 16 : 0;
    t.nty = (P.g.ny + 4 * cfg.rows - 1) / (4 * cfg.rows);
    int cnt[3], b0[3], b1[3];
    bool empty = false;
    for (int a = 0; a < 3; ++a) {
        cnt[a] = (n[a] + w[a] - 1) / w[a];
        if (a == 0 && t.nxw > 0) cnt[a] = n[a] / 64;
        b0[a] = b1[a] = 0;
        int first = -1, last = -1;
        for (int q = 0; q < cnt[a]; ++q) {
            // cells the tile touches along a: its own, the halo (or first
            // input plane) one below
            const int lo = std::max(q * w[a] - 1, 0), hi = std::min(q * w[a] + w[a], n[a]);
            if (lo >= P.lo[a] && hi <= n[a] - P.hi[a]) {
                if (first < 0) first = q;
                last = q;
            }
        }
        if (first < 0) empty = true;
        else { b0[a] = first; b1[a] = last + 1; }
    }
    if (empty)
        for (int a = 0; a < 3; ++a) b0[a] = b1[a] = 0;
    t.tx = cnt[0]; t.ty = cnt[1]; t.tz = cnt[2];
    t.ix0 = b0[0]; t.ix1 = b1[0];
    t.iy0 = b0[1]; t.iy1 = b1[1];
    t.iz0 = b0[2]; t.iz1 = b1[2];
    t.ni = (b1[0] - b0[0]) * (b1[1] - b0[1]) * (b1[2] - b0[2]);
    t.nb = cnt[0] * cnt[1] * cnt[2] - t.ni + t.nxw * t.nty * cnt[2];
    return t;
}

// Two-level tiles for the tile decomposition t (made by make_tileset with the
// same cfg).  The two-level pass recomputes two cells around every cell it
// writes, so the box of interior tiles is shrunk, a tile row or plane at a
// time, until that margin avoids the absorbing layers and the grid's x and y
// faces and the planes it reads exist: x0 - 2 >= lo, x1 + 2 <= n - hi (also
// y), and z0 = 0 on a grid without a lower z layer or z0 - 2 >= lo, and
// z1 + 1 <= nz - hi.  The tiles taken off join the boundary launch.  Returns
// the cell box cut into TB_W x cfg.tb_rows x cfg.tb_zchunk tiles (n = 0
// when none is left).
TBSet make_tbset(const Plan &P, const LaunchCfg &cfg, TileSet &t)
{
    const int n[3] = {P.g.nx, P.g.ny, P.g.nz};
    const int w[3] = {64, cfg.rows, cfg.zchunk};
    int *b0[3] = {&t.ix0, &t.iy0, &t.iz0}, *b1[3] = {&t.ix1, &t.iy1, &t.iz1};
    int c0[3], c1[3];
    for (int a = 0; a < 3; ++a) {
        auto lo_ok = [&](int q) {
            const int c = q * w[a];
            if (a == 2 && c == 0) return P.lo[2] == 0;
            return c - 2 >= P.lo[a];
        };
        auto hi_ok = [&](int q) {
            const int c = std::min(q * w[a], n[a]);
            return a == 2 ? c + 1 <= n[a] - P.hi[a] : c + 2 <= n[a] - P.hi[a];
        };
        while (*b0[a] < *b1[a] && !lo_ok(*b0[a])) ++*b0[a];
        while (*b0[a] < *b1[a] && !hi_ok(*b1[a])) --*b1[a];
        c0[a] = *b0[a] * w[a];
        c1[a] = std::min(*b1[a] * w[a], n[a]);
    }
    if (t.ix0 >= t.ix1 || t.iy0 >= t.iy1 || t.iz0 >= t.iz1) {
        t.ix0 = t.ix1 = t.iy0 = t.iy1 = t.iz0 = t.iz1 = 0;
        c0[0] = c1[0] = c0[1] = c1[1] = c0[2] = c1[2] = 0;
    }
    const int rx = P.g.nx % 64;
    const int cntx = (rx > 0 && rx <= 32) ? n[0] / 64 : (n[0] + 63) / 64;
    const int cnty = (n[1] + w[1] - 1) / w[1], cntz = (n[2] + w[2] - 1) / w[2];
    t.ni = (t.ix1 - t.ix0) * (t.iy1 - t.iy0) * (t.iz1 - t.iz0);
    t.nb = cntx * cnty * cntz - t.ni + t.nxw * t.nty * cntz;
    TBSet b{};
    b.x0 = c0[0]; b.x1 = c1[0];
    b.y0 = c0[1]; b.y1 = c1[1];
    b.z0 = c0[2]; b.z1 = c1[2];
    b.rows = cfg.tb_rows;
    b.zc = cfg.tb_zchunk;
    if (t.ni > 0) {
        b.ntx = (b.x1 - b.x0 + TB_W - 1) / TB_W;
        b.nty = (b.y1 - b.y0 + b.rows - 1) / b.rows;
        b.ntz = (b.z1 - b.z0 + b.zc - 1) / b.zc;
        b.n = b.ntx * b.nty * b.ntz;
    }
    return b;
}

static DevProbes dev_probes(const Plan &P)
{
    DevProbes p{};
    p.toff = reinterpret_cast<const int64_t *>(P.base + P.r_toff.off);
    p.tcomp = reinterpret_cast<const int32_t *>(P.base + P.r_tcomp.off);
    p.tw = reinterpret_cast<const double *>(P.base + P.r_tw.off);
    p.range = reinterpret_cast<const int32_t *>(P.base + P.r_range.off);
    p.hist = reinterpret_cast<double *>(P.base + P.r_hist.off);
    p.K = P.K;
    p.nprobe = P.nprobe();
    return p;
}

static DevDft dev_dft(const Plan &P)
{
    DevDft d{};
    d.hist = reinterpret_cast<const double *>(P.base + P.r_hist.off);
    d.acc = reinterpret_cast<double *>(P.base + P.r_acc.off);
    d.freqs = reinterpret_cast<const double *>(P.base + P.r_freq.off);
    d.nf = P.nf();
    d.nprobe = P.nprobe();
    d.K = P.K;
    d.dt = P.dt;
    return d;
}

// upload helpers: convert FP64 host tables to the field type
static void upload(Plan &P, const Region &r, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return;
    hip_check(hipMemcpyAsync(P.base + r.off, src, bytes, hipMemcpyHostToDevice, s), "upload");
}

static void upload_real(Plan &P, const Region &r, const std::vector<double> &v, hipStream_t s,
                        std::vector<std::vector<char>> &keep)
{
    if (v.empty()) return;
    if (P.elt == 8) {
        upload(P, r, v.data(), v.size() * 8, s);
        return;
    }
    keep.emplace_back(v.size() * 4);
    float *f = reinterpret_cast<float *>(keep.back().data());
    for (size_t q = 0; q < v.size(); ++q) f[q] = (float)v[q];
    upload(P, r, f, v.size() * 4, s);
}

// Tile decomposition of the plan's launch shape; with three field buffers
// also the two-level tiles and, per two-level tile, whether it holds a
// probe term (such a tile writes the intermediate level of all its cells,
// for the probes of that level).
static void plan_tiles(Plan &P)
{
    P.tiles = make_tileset(P, P.cfg);
    P.tbset = TBSet{};
    P.tbflags.assign(1, 0);
    if (P.tb) {
        P.tbset = make_tbset(P, P.cfg, P.tiles);
        const TBSet &b = P.tbset;
        P.tbflags.assign((size_t)std::max(1, b.n), 0);
        REQUIRE(P.tbflags.size() <= P.r_tbflag.bytes, FDTD_E_INVALID_ARG,
                "two-level tile shape too small for the plan");
        const int64_t off = 64 + (int64_t)P.px * (1 + P.py);
        const int64_t plane = (int64_t)P.px * P.py;
        for (size_t q = 0; q < P.toff.size() && b.n > 0; ++q) {
            const int64_t u = P.toff[q] - off + 1 + P.px + plane;
            const int i = (int)(u % P.px) - 1, j = (int)((u / P.px) % P.py) - 1,
                      k = (int)(u / plane) - 1;
            if (i < b.x0 || i >= b.x1 || j < b.y0 || j >= b.y1 || k < b.z0 || k >= b.z1) continue;
            const int tx = (i - b.x0) / TB_W, ty = (j - b.y0) / b.rows, tz = (k - b.z0) / b.zc;
            P.tbflags[(size_t)tx + (size_t)b.ntx * (ty + (size_t)b.nty * tz)] = 1;
        }
    }
    P.tiles_cfg = P.cfg;
}

// The tile sets and flags of plan_tiles into the launch table.
static void upload_tiles(Plan &P, hipStream_t s)
{
    upload(P, Region{P.r_grid.off + GRID_SET_OFF, sizeof(TileSet)}, &P.tiles, sizeof(TileSet), s);
    upload(P, Region{P.r_grid.off + GRID_TBSET_OFF, sizeof(TBSet)}, &P.tbset, sizeof(TBSet), s);
    if (P.tb) upload(P, P.r_tbflag, P.tbflags.data(), P.tbflags.size(), s);
}

static void bind_plan(Plan &P, char *base, size_t bytes, hipStream_t s)
{
    finalize(P);
    REQUIRE(base != nullptr, FDTD_E_INVALID_ARG, "null workspace");
    REQUIRE(((uintptr_t)base & 255) == 0, FDTD_E_INVALID_ARG, "workspace not 256-byte aligned");
    REQUIRE(bytes >= P.ws_bytes, FDTD_E_NOMEM, "workspace smaller than fdtd_plan_workspace_size");
    P.base = base;
    P.ring_dev = -1;
    P.ring = nullptr;
    {
        int dev = -1;
        double *ring = nullptr;
        if (scratch_ring(dev, ring) == hipSuccess) {
            P.ring_dev = dev;
            P.ring = ring;
        }
    }
    std::vector<std::vector<char>> keep;
    if (P.g.kernel == FDTD_KERNEL_FUSED) {
        const int b = P.id_bits;
        const size_t word = b == 5 ? 2 : 4;
        keep.emplace_back(P.id_elems * word);
        char *q = keep.back().data();
        for (size_t t = 0; t < P.id_elems; ++t) {
            const uint32_t w = (uint32_t)P.ids[0][t] | (uint32_t)P.ids[1][t] << b |
                               (uint32_t)P.ids[2][t] << (2 * b);
            if (word == 2) reinterpret_cast<uint16_t *>(q)[t] = (uint16_t)w;
            else reinterpret_cast<uint32_t *>(q)[t] = w;
        }
        upload(P, P.r_ids[0], q, P.id_elems * word, s);
    }
    for (int c = 0; c < 3; ++c) {
        if (P.g.kernel == FDTD_KERNEL_FUSED) {
            // packed above
        } else if (P.id16) {
            upload(P, P.r_ids[c], P.ids[c].data(), P.id_elems * 2, s);
        } else {
            keep.emplace_back(P.id_elems);
            char *q = keep.back().data();
            for (size_t t = 0; t < P.id_elems; ++t) q[t] = (char)(uint8_t)P.ids[c][t];
            upload(P, P.r_ids[c], q, P.id_elems, s);
        }
        upload_real(P, P.r_lut[c], P.lut[c], s, keep);
        upload_real(P, P.r_prof[c], P.prof[c], s, keep);
    }
    upload(P, P.r_toff, P.toff.data(), P.toff.size() * 8, s);
    upload(P, P.r_tcomp, P.tcomp.data(), P.tcomp.size() * 4, s);
    upload(P, P.r_tw, P.tw.data(), P.tw.size() * 8, s);
    upload(P, P.r_range, P.prange.data(), P.prange.size() * 4, s);
    upload(P, P.r_freq, P.freqs.data(), P.freqs.size() * 8, s);
    upload(P, P.r_src, P.src_samples.data(), P.src_samples.size() * 8, s);
    if (P.g.kernel == FDTD_KERNEL_FUSED) {
        // launch table of the fused kernels: the descriptors of every step
        // (single-level from each buffer with each auxiliary copy, two-level
        // from each buffer), the tile sets (written again before each run
        // whose launch shape differs from the uploaded one) and the probes
        DevGrid<float> g9[9];
        for (int q = 0; q < 6; ++q) g9[q] = P.dev_grid_at((q / 2) % P.nbuf, q % 2);
        for (int q = 0; q < 3; ++q) g9[6 + q] = P.dev_grid_tb(q % P.nbuf);
        const DevProbes pr = dev_probes(P);
        keep.emplace_back(P.r_grid.bytes, 0);
        std::memcpy(keep.back().data(), g9, sizeof g9);
        std::memcpy(keep.back().data() + GRID_PROBES_OFF, &pr, sizeof pr);
        DevProbes pr2 = pr;
        pr2.hist = P.ring;
        std::memcpy(keep.back().data() + GRID_PROBES2_OFF, &pr2, sizeof pr2);
        plan_tiles(P);
        std::memcpy(keep.back().data() + GRID_SET_OFF, &P.tiles, sizeof P.tiles);
        std::memcpy(keep.back().data() + GRID_TBSET_OFF, &P.tbset, sizeof P.tbset);
        upload(P, P.r_grid, keep.back().data(), P.r_grid.bytes, s);
        if (P.tb) upload(P, P.r_tbflag, P.tbflags.data(), P.tbflags.size(), s);
    }
    hip_check(hipMemsetAsync(P.base + P.r_mut.off, 0, P.r_mut.bytes, s), "clear state");
    hip_check(hipStreamSynchronize(s), "bind sync");
    P.step = 0;
    P.dft_n = 0;
    P.sampled = 0;
    P.parity = 0;
    P.bound = true;
}

static void reset_plan(Plan &P, hipStream_t s)
{
    REQUIRE(P.bound, FDTD_E_STATE, "plan not bound");
    hip_check(hipMemsetAsync(P.base + P.r_mut.off, 0, P.r_mut.bytes, s), "reset");
    P.step = 0;
    P.dft_n = 0;
    P.sampled = 0;
    P.parity = 0;
}

// Fold the samples dft_n+1 .. sampled of the history ring into the DFTs.
static void flush_dft(Plan &P, hipStream_t s, const double *ring = nullptr)
{
    if (P.sampled > P.dft_n) {
        DevDft d = dev_dft(P);
        if (ring) d.hist = ring;
        hip_check(launch_dft(d, P.dft_n + 1, P.sampled - P.dft_n, s), "dft");
        P.dft_n = P.sampled;
    }
}

}  // namespace fdtd

hipError_t fdtd::KernelTimer::step(hipEvent_t &a, hipEvent_t &b, bool first, bool last,
                                   int32_t count)
{
    a = b = nullptr;
    if (!on) return hipSuccess;
    if (first) open = -1;
    if (open < 0) {
        if (ev.empty()) {
            ev.assign(2 * SLOTS, nullptr);
            used.assign(SLOTS, 0);
            for (auto &e : ev) {
                const hipError_t r = hipEventCreate(&e);
                if (r != hipSuccess) return r;
            }
        }
        if (used[next]) {
            hipError_t r = hipEventSynchronize(ev[2 * next + 1]);
            if (r != hipSuccess) return r;
            float t = 0;
            r = hipEventElapsedTime(&t, ev[2 * next], ev[2 * next + 1]);
            if (r != hipSuccess) return r;
            ms += t;
            launches += used[next];
            used[next] = 0;
        }
        open = (long)next;
        next = (next + 1) % SLOTS;
        in_window = 0;
        a = ev[2 * open];
    }
    in_window += count;
    if (in_window >= every || last) {
        b = ev[2 * open + 1];
        used[open] = in_window;
        open = -1;
    }
    return hipSuccess;
}

hipError_t fdtd::KernelTimer::drain()
{
    for (size_t q = 0; q < used.size(); ++q) {
        if (!used[q]) continue;
        hipError_t r = hipEventSynchronize(ev[2 * q + 1]);
        if (r != hipSuccess) return r;
        float t = 0;
        r = hipEventElapsedTime(&t, ev[2 * q], ev[2 * q + 1]);
        if (r != hipSuccess) return r;
        ms += t;
        launches += used[q];
        used[q] = 0;
    }
    return hipSuccess;
}

void fdtd::KernelTimer::reset()
{
    for (auto &u : used) u = 0;
    ms = 0;
    launches = 0;
    open = -1;
    in_window = 0;
}

void fdtd::KernelTimer::destroy()
{
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    ev.clear();
    used.clear();
}

namespace fdtd {

// ring: the probe history ring to use instead of the workspace's (the
// static one of fdtd_run_noalloc); the kernel timer is then left out.
static void run_plan(Plan &P, int64_t nsteps, hipStream_t s, double *ring = nullptr)
{
    REQUIRE(P.bound, FDTD_E_STATE, "plan not bound");
    REQUIRE(!P.in_batch, FDTD_E_STATE, "plan belongs to a batch; use fdtd_batch_run");
    REQUIRE(nsteps >= 0, FDTD_E_INVALID_ARG, "negative step count");
    DevProbes pr = dev_probes(P);
    if (ring) pr.hist = ring;
    const bool fused = P.g.kernel == FDTD_KERNEL_FUSED;
    if (fused && nsteps > 0 &&
        (P.tiles_cfg.rows != P.cfg.rows || P.tiles_cfg.zchunk != P.cfg.zchunk ||
         P.tiles_cfg.tb_rows != P.cfg.tb_rows || P.tiles_cfg.tb_zchunk != P.cfg.tb_zchunk)) {
        plan_tiles(P);
        upload_tiles(P, s);
    }
    const char *tab = P.base + P.r_grid.off;
    const auto *grids = reinterpret_cast<const DevGrid<float> *>(tab);
    const auto *tset = reinterpret_cast<const TileSet *>(tab + GRID_SET_OFF);
    const auto *probes = reinterpret_cast<const DevProbes *>(tab + (ring ? GRID_PROBES2_OFF : GRID_PROBES_OFF));
    const int32_t lut_cap = std::max<int32_t>(1, (int32_t)(P.lut[0].size() / 4));
    LaunchCfg cfg = P.cfg;
    cfg.order = tile_order(P.cfg, P.ws_bytes);
    cfg.stream = stream_stores(P.cfg, P.ws_bytes);
    for (int64_t t = 0; t < nsteps;) {
        // two levels per pass where the plan has two-level tiles
        const bool pair = fused && P.tb && P.cfg.tb_depth == 2 && P.tbset.n > 0 && nsteps - t >= 2;
        const int adv = pair ? 2 : 1;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (!ring) hip_check(P.timer.step(e0, e1, t == 0, t + adv >= nsteps, adv), "timer");
        if (pair) {
            // boundary tiles n -> n+1 into the next buffer (sampling level
            // n), the two-level pass n -> n+2 of the interior tiles (level
            // n+1 of its rim and probe tiles into the next buffer too), then
            // the boundary tiles n+1 -> n+2 (sampling level n+1)
            const int cur = P.parity, pp = (int)(P.step & 1), mid = (cur + 1) % 3;
            hip_check(launch_fused(grids + 2 * cur + pp, tset, 1, P.tiles.nb, 0, cfg, lut_cap,
                                   P.id_bits, P.step, probes, P.nprobe(), P.nprobe() > 0, s, e0,
                                   nullptr),
                      "boundary step");
            hip_check(launch_tb(grids + 6 + cur,
                                reinterpret_cast<const TBSet *>(tab + GRID_TBSET_OFF), P.tbset.n,
                                cfg, lut_cap, P.id_bits, P.step, s),
                      "two-level step");
            hip_check(launch_fused(grids + 2 * mid + (1 - pp), tset, 1, P.tiles.nb, 0, cfg,
                                   lut_cap, P.id_bits, P.step + 1, probes, P.nprobe(),
                                   P.nprobe() > 0, s, nullptr, e1),
                      "boundary step");
            P.parity = (cur + 2) % 3;
            if (P.nprobe() > 0) P.sampled = std::max(P.sampled, P.step + 1);
        } else if (fused) {
            // the launch samples its input level P.step (if >= 1) as well
            hip_check(launch_fused(grids + 2 * P.parity + (int)(P.step & 1), tset, 1, P.tiles.nb,
                                   P.tiles.ni, cfg, lut_cap, P.id_bits, P.step, probes,
                                   P.nprobe(), P.nprobe() > 0, s, e0, e1),
                      "fused step");
            P.parity = (P.parity + 1) % P.nbuf;
            if (P.nprobe() > 0 && P.step >= 1) P.sampled = std::max(P.sampled, P.step);
        } else if (P.g.precision == FDTD_FP64) {
            const DevGrid<double> d = P.dev_grid<double>();
            hip_check(launch_plain_step(d, P.step, s, e0, e1), "plain step");
            hip_check(launch_probe(d, pr, P.step + 1, s), "probe");
            P.sampled = P.step + 1;
        } else {
            const DevGrid<float> d = P.dev_grid<float>();
            hip_check(launch_plain_step(d, P.step, s, e0, e1), "plain step");
            hip_check(launch_probe(d, pr, P.step + 1, s), "probe");
            P.sampled = P.step + 1;
        }
        P.step += adv;
        t += adv;
        // the ring holds K samples: fold them in before a later one would
        // overwrite an unfolded slot (a pass samples at most two levels)
        if (P.sampled - P.dft_n >= P.K - 2) flush_dft(P, s, ring);
    }
    if (fused && P.sampled < P.step) {
        // the last level of the run has not been sampled by a launch yet
        hip_check(launch_probe(P.dev_grid<float>(), pr, P.step, s), "probe");
        P.sampled = P.step;
    }
    flush_dft(P, s, ring);
}

// entry points for the batch code
void plan_bind_slice(Plan &P, char *base, size_t bytes, hipStream_t s) { bind_plan(P, base, bytes, s); }
void plan_reset(Plan &P, hipStream_t s) { reset_plan(P, s); }
void plan_finalize(Plan &P) { finalize(P); }
DevProbes plan_dev_probes(const Plan &P) { return dev_probes(P); }
DevDft plan_dev_dft(const Plan &P) { return dev_dft(P); }

}  // namespace fdtd

using namespace fdtd;

// ---------------------------------------------------------------------------
// C interface
// ---------------------------------------------------------------------------
extern "C" {

const char *fdtd_status_string(fdtd_status s)
{
    switch (s) {
    case FDTD_OK: return "ok";
    case FDTD_E_INVALID_ARG: return "invalid argument";
    case FDTD_E_STATE: return "wrong call order";
    case FDTD_E_UNSUPPORTED: return "unsupported";
    case FDTD_E_HIP: return "HIP runtime error";
    case FDTD_E_NOMEM: return "out of memory";
    case FDTD_E_DIVERGED: return "diverged";
    default: return "unknown status";
    }
}

fdtd_status fdtd_plan_create(const fdtd_grid *grid, fdtd_plan **out)
{
    if (!grid || !out) return FDTD_E_INVALID_ARG;
    *out = nullptr;
    const fdtd_grid &g = *grid;
    if (g.nx < 2 || g.ny < 2 || g.nz < 2) return FDTD_E_INVALID_ARG;
    if ((int64_t)g.nx * g.ny * g.nz > (int64_t)1 << 34) return FDTD_E_INVALID_ARG;
    if (!(g.dx > 0) || !(g.dy > 0) || !(g.dz > 0) || !(g.courant > 0)) return FDTD_E_INVALID_ARG;
    if (g.precision != FDTD_FP32 && g.precision != FDTD_FP64) return FDTD_E_INVALID_ARG;
    if (g.units != FDTD_SI && g.units != FDTD_NORMALIZED) return FDTD_E_INVALID_ARG;
    if (g.kernel != FDTD_KERNEL_PLAIN && g.kernel != FDTD_KERNEL_FUSED) return FDTD_E_INVALID_ARG;
    if (g.kernel == FDTD_KERNEL_FUSED && g.precision != FDTD_FP32) return FDTD_E_UNSUPPORTED;
    fdtd_plan *p = new (std::nothrow) fdtd_plan();
    if (!p) return FDTD_E_NOMEM;
    p->g = g;
    p->bnd.m = 3.0;
    p->bnd.kappa_max = 1.0;
    const Plan *one = p;
    p->cfg = default_launch(&one, 1);
    *out = p;
    return FDTD_OK;
}

void fdtd_plan_destroy(fdtd_plan *plan)
{
    if (!plan) return;
    plan->timer.destroy();
    delete plan;
}

const char *fdtd_last_error(const fdtd_plan *plan) { return plan ? plan->err.c_str() : ""; }

#define PLAN_GUARD(plan) \
    if (!(plan)) return FDTD_E_INVALID_ARG; \
    return guarded(plan, [&]()

#define NOT_FINAL(P) REQUIRE(!(P).finalized, FDTD_E_STATE, "plan already finalized")

fdtd_status fdtd_plan_set_materials(fdtd_plan *plan, const uint8_t *cells,
                                    const fdtd_material *table, int32_t n)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        NOT_FINAL(P);
        REQUIRE(cells && table, FDTD_E_INVALID_ARG, "null material arrays");
        REQUIRE(n >= 1 && n <= 256, FDTD_E_INVALID_ARG, "material count outside [1, 256]");
        for (int q = 0; q < n; ++q)
            REQUIRE(table[q].is_pec || (table[q].eps_r > 0 && table[q].sigma >= 0),
                    FDTD_E_INVALID_ARG, "bad material parameters");
        const size_t nc = (size_t)P.g.nx * P.g.ny * P.g.nz;
        for (size_t q = 0; q < nc; ++q)
            REQUIRE(cells[q] < n, FDTD_E_INVALID_ARG, "cell material id out of range");
        P.cells.assign(cells, cells + nc);
        P.mats.assign(table, table + n);
    });
}

fdtd_status fdtd_plan_set_boundary(fdtd_plan *plan, const fdtd_boundary *b)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        NOT_FINAL(P);
        REQUIRE(b, FDTD_E_INVALID_ARG, "null boundary");
        const int n[3] = {P.g.nx, P.g.ny, P.g.nz};
        for (int f = 0; f < 6; ++f) {
            REQUIRE(b->face[f] == FDTD_FACE_PEC || b->face[f] == FDTD_FACE_CPML,
                    FDTD_E_INVALID_ARG, "unknown face kind");
            REQUIRE(b->cells[f] >= 0, FDTD_E_INVALID_ARG, "negative layer thickness");
        }
        for (int a = 0; a < 3; ++a) {
            const int L = (b->face[2 * a] == FDTD_FACE_CPML ? b->cells[2 * a] : 0) +
                          (b->face[2 * a + 1] == FDTD_FACE_CPML ? b->cells[2 * a + 1] : 0);
            REQUIRE(L <= n[a], FDTD_E_INVALID_ARG, "absorbing layers overlap");
        }
        REQUIRE(b->m >= 0 && b->kappa_max >= 1.0 && b->alpha_max >= 0, FDTD_E_INVALID_ARG,
                "bad layer grading");
        P.bnd = *b;
    });
}

fdtd_status fdtd_plan_add_port(fdtd_plan *plan, const fdtd_port *q, int32_t *id)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        NOT_FINAL(P);
        REQUIRE(q, FDTD_E_INVALID_ARG, "null port");
        REQUIRE(q->dir == 1 || q->dir == -1, FDTD_E_INVALID_ARG, "port direction must be +1/-1");
        REQUIRE(q->i >= 1 && q->i < P.g.nx, FDTD_E_INVALID_ARG, "port plane outside the grid");
        REQUIRE(q->y0 >= 1 && q->y1 > q->y0 && q->y1 < P.g.ny, FDTD_E_INVALID_ARG,
                "port strip y-range must leave room for the current loop");
        REQUIRE(q->z0 >= 1 && q->z1 > q->z0 && q->z1 < P.g.nz, FDTD_E_INVALID_ARG,
                "port strip z-range must leave room for the current loop");
        REQUIRE(P.points.empty(), FDTD_E_STATE, "add ports before point probes");
        P.ports.push_back(*q);
        if (id) *id = (int32_t)P.ports.size() - 1;
    });
}

fdtd_status fdtd_plan_add_point_probe(fdtd_plan *plan, int32_t comp, int32_t i, int32_t j,
                                      int32_t k, int32_t *id)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        NOT_FINAL(P);
        REQUIRE(comp >= 0 && comp < 6, FDTD_E_INVALID_ARG, "bad component");
        REQUIRE(i >= 0 && i <= P.g.nx && j >= 0 && j <= P.g.ny && k >= 0 && k <= P.g.nz,
                FDTD_E_INVALID_ARG, "probe outside the grid");
        P.points.push_back({comp, i, j, k});
        if (id) *id = (int32_t)(P.ports.size() + P.points.size()) - 1;
    });
}

fdtd_status fdtd_plan_set_source(fdtd_plan *plan, const fdtd_source *src)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        NOT_FINAL(P);
        REQUIRE(src, FDTD_E_INVALID_ARG, "null source");
        const fdtd_source &s = *src;
        REQUIRE(s.kind >= FDTD_WAVE_NONE && s.kind <= FDTD_WAVE_SAMPLED,
                FDTD_E_INVALID_ARG, "unknown waveform");
        if (s.kind != FDTD_WAVE_NONE) {
            const int *b = s.box;
            REQUIRE(b[0] >= 0 && b[0] <= b[1] && b[1] < P.g.nx && b[2] >= 0 && b[2] <= b[3] &&
                        b[3] < P.g.ny && b[4] >= 0 && b[4] <= b[5] && b[5] < P.g.nz,
                    FDTD_E_INVALID_ARG, "source box outside the grid");
            if (s.kind == FDTD_WAVE_GAUSS_SINE)
                REQUIRE(s.bandwidth > 0, FDTD_E_INVALID_ARG, "bandwidth must be positive");
            else if (s.kind != FDTD_WAVE_SAMPLED)
                REQUIRE(s.width > 0, FDTD_E_INVALID_ARG, "pulse width must be positive");
        }
        P.src = s;
    });
}

fdtd_status fdtd_plan_set_source_samples(fdtd_plan *plan, const double *samples, int64_t n)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        NOT_FINAL(P);
        REQUIRE(samples && n >= 1, FDTD_E_INVALID_ARG, "no source samples");
        P.src_samples.assign(samples, samples + n);
    });
}

fdtd_status fdtd_plan_set_frequencies(fdtd_plan *plan, const double *f, int32_t nf)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        NOT_FINAL(P);
        REQUIRE(f && nf >= 1 && nf <= 4096, FDTD_E_INVALID_ARG, "frequency count outside [1, 4096]");
        P.freqs.assign(f, f + nf);
    });
}

fdtd_status fdtd_plan_workspace_size(fdtd_plan *plan, size_t *bytes)
{
    PLAN_GUARD(plan) {
        REQUIRE(bytes, FDTD_E_INVALID_ARG, "null output");
        finalize(*plan);
        *bytes = plan->ws_bytes;
    });
}

fdtd_status fdtd_plan_get_dt(const fdtd_plan *plan, double *dt)
{
    if (!plan || !dt) return FDTD_E_INVALID_ARG;
    if (!plan->finalized) return FDTD_E_STATE;
    *dt = plan->dt;
    return FDTD_OK;
}

fdtd_status fdtd_plan_bind(fdtd_plan *plan, void *dptr, size_t bytes, void *stream)
{
    PLAN_GUARD(plan) {
        REQUIRE(!plan->in_batch, FDTD_E_STATE, "plan belongs to a batch");
        bind_plan(*plan, static_cast<char *>(dptr), bytes, static_cast<hipStream_t>(stream));
    });
}

fdtd_status fdtd_reset(fdtd_plan *plan, void *stream)
{
    PLAN_GUARD(plan) { reset_plan(*plan, static_cast<hipStream_t>(stream)); });
}

fdtd_status fdtd_run(fdtd_plan *plan, int64_t nsteps, void *stream)
{
    PLAN_GUARD(plan) { run_plan(*plan, nsteps, static_cast<hipStream_t>(stream)); });
}

fdtd_status fdtd_run_noalloc(fdtd_plan *plan, int64_t nsteps, void *stream)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        REQUIRE(P.bound, FDTD_E_STATE, "plan not bound");
        REQUIRE(!P.in_batch, FDTD_E_STATE, "plan belongs to a batch; use fdtd_batch_run");
        const size_t need = (size_t)P.nprobe() * 2 * (size_t)P.K * sizeof(double);
        REQUIRE(need <= NOALLOC_RING_BYTES, FDTD_E_INVALID_ARG,
                "probe history ring of " + std::to_string(need) + " bytes exceeds the " +
                    std::to_string(NOALLOC_RING_BYTES) + "-byte static ring of fdtd_run_noalloc");
        REQUIRE(P.ring != nullptr, FDTD_E_HIP, "static ring address unavailable on the bound device");
        int dev = -1;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        REQUIRE(dev == P.ring_dev, FDTD_E_STATE,
                "current device " + std::to_string(dev) + " is not the device the plan was bound on (" +
                    std::to_string(P.ring_dev) + ")");
        run_plan(P, nsteps, static_cast<hipStream_t>(stream), P.ring);
    });
}

fdtd_status fdtd_get_step(const fdtd_plan *plan, int64_t *step)
{
    if (!plan || !step) return FDTD_E_INVALID_ARG;
    *step = plan->step;
    return FDTD_OK;
}

fdtd_status fdtd_get_spectra(fdtd_plan *plan, int32_t probe, double *V, double *I, void *stream)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        REQUIRE(P.bound, FDTD_E_STATE, "plan not bound");
        REQUIRE(probe >= 0 && probe < P.nprobe(), FDTD_E_INVALID_ARG, "bad probe index");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t n = (size_t)P.nf() * 2;
        std::vector<double> buf(2 * n);
        hip_check(hipMemcpyAsync(buf.data(), P.base + P.r_acc.off + (size_t)probe * 2 * n * 8,
                                 2 * n * 8, hipMemcpyDeviceToHost, s), "spectra copy");
        hip_check(hipStreamSynchronize(s), "spectra sync");
        for (double v : buf) REQUIRE(std::isfinite(v), FDTD_E_DIVERGED, "non-finite spectrum");
        if (V) std::memcpy(V, buf.data(), n * 8);
        if (I) std::memcpy(I, buf.data() + n, n * 8);
    });
}

static const Region &field_region(const Plan &P, int comp)
{
    return comp < 3 ? P.r_E[P.parity][comp] : P.r_H[P.parity][comp - 3];
}

fdtd_status fdtd_read_field(fdtd_plan *plan, int32_t comp, double *host, void *stream)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        REQUIRE(P.bound, FDTD_E_STATE, "plan not bound");
        REQUIRE(comp >= 0 && comp < 6 && host, FDTD_E_INVALID_ARG, "bad component or buffer");
        hipStream_t s = static_cast<hipStream_t>(stream);
        std::vector<char> raw(P.field_elems * P.elt);
        hip_check(hipMemcpyAsync(raw.data(), P.base + field_region(P, comp).off, raw.size(),
                                 hipMemcpyDeviceToHost, s), "field copy");
        hip_check(hipStreamSynchronize(s), "field sync");
        const int nx = P.g.nx, ny = P.g.ny, nz = P.g.nz;
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i <= nx; ++i) {
                    const int64_t q = field_index(P, i, j, k);
                    double v = P.elt == 8 ? reinterpret_cast<const double *>(raw.data())[q]
                                          : (double)reinterpret_cast<const float *>(raw.data())[q];
                    host[(size_t)i + (size_t)(nx + 1) * ((size_t)j + (size_t)(ny + 1) * k)] = v;
                }
    });
}

fdtd_status fdtd_write_field(fdtd_plan *plan, int32_t comp, const double *host, void *stream)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        REQUIRE(P.bound, FDTD_E_STATE, "plan not bound");
        REQUIRE(comp >= 0 && comp < 6 && host, FDTD_E_INVALID_ARG, "bad component or buffer");
        hipStream_t s = static_cast<hipStream_t>(stream);
        std::vector<char> raw(P.field_elems * P.elt, 0);
        const int nx = P.g.nx, ny = P.g.ny, nz = P.g.nz;
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const int64_t q = field_index(P, i, j, k);
                    const double v =
                        host[(size_t)i + (size_t)(nx + 1) * ((size_t)j + (size_t)(ny + 1) * k)];
                    if (P.elt == 8) reinterpret_cast<double *>(raw.data())[q] = v;
                    else reinterpret_cast<float *>(raw.data())[q] = (float)v;
                }
        hip_check(hipMemcpyAsync(P.base + field_region(P, comp).off, raw.data(), raw.size(),
                                 hipMemcpyHostToDevice, s), "field copy");
        hip_check(hipStreamSynchronize(s), "field sync");
    });
}

struct CkHeader {
    uint64_t magic, mut_bytes;
    int64_t step, dft_n, sampled;
    int32_t parity, pad;
};
static const uint64_t CK_MAGIC = 0x46445444434b5031ull;

fdtd_status fdtd_checkpoint_size(const fdtd_plan *plan, size_t *bytes)
{
    if (!plan || !bytes) return FDTD_E_INVALID_ARG;
    if (!plan->finalized) return FDTD_E_STATE;
    *bytes = sizeof(CkHeader) + plan->r_mut.bytes;
    return FDTD_OK;
}

fdtd_status fdtd_checkpoint_save(fdtd_plan *plan, void *host, size_t bytes, void *stream)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        REQUIRE(P.bound, FDTD_E_STATE, "plan not bound");
        REQUIRE(host, FDTD_E_INVALID_ARG, "null buffer");
        REQUIRE(bytes >= sizeof(CkHeader) + P.r_mut.bytes, FDTD_E_NOMEM, "checkpoint buffer too small");
        hipStream_t s = static_cast<hipStream_t>(stream);
        CkHeader h{CK_MAGIC, P.r_mut.bytes, P.step, P.dft_n, P.sampled, P.parity, 0};
        std::memcpy(host, &h, sizeof h);
        hip_check(hipMemcpyAsync(static_cast<char *>(host) + sizeof h, P.base + P.r_mut.off,
                                 P.r_mut.bytes, hipMemcpyDeviceToHost, s), "checkpoint copy");
        hip_check(hipStreamSynchronize(s), "checkpoint sync");
    });
}

fdtd_status fdtd_checkpoint_load(fdtd_plan *plan, const void *host, size_t bytes, void *stream)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        REQUIRE(P.bound, FDTD_E_STATE, "plan not bound");
        REQUIRE(host && bytes >= sizeof(CkHeader), FDTD_E_INVALID_ARG, "bad checkpoint");
        CkHeader h;
        std::memcpy(&h, host, sizeof h);
        REQUIRE(h.magic == CK_MAGIC && h.mut_bytes == P.r_mut.bytes &&
                    bytes >= sizeof h + P.r_mut.bytes,
                FDTD_E_INVALID_ARG, "checkpoint belongs to a different plan");
        hipStream_t s = static_cast<hipStream_t>(stream);
        hip_check(hipMemcpyAsync(P.base + P.r_mut.off, static_cast<const char *>(host) + sizeof h,
                                 P.r_mut.bytes, hipMemcpyHostToDevice, s), "checkpoint copy");
        hip_check(hipStreamSynchronize(s), "checkpoint sync");
        P.step = h.step;
        P.dft_n = h.dft_n;
        P.sampled = h.sampled;
        P.parity = h.parity;
    });
}

fdtd_status fdtd_plan_get_config(const fdtd_plan *plan, int32_t *rows, int32_t *zchunk)
{
    if (!plan) return FDTD_E_INVALID_ARG;
    if (rows) *rows = plan->cfg.rows;
    if (zchunk) *zchunk = plan->cfg.zchunk;
    return FDTD_OK;
}

fdtd_status fdtd_plan_set_config(fdtd_plan *plan, int32_t rows, int32_t zchunk)
{
    PLAN_GUARD(plan) {
        REQUIRE(valid_rows(rows), FDTD_E_INVALID_ARG, "tile rows must be 2, 4, 8, 12 or 16");
        REQUIRE(zchunk >= 1 && zchunk <= 64, FDTD_E_INVALID_ARG, "z-chunk must be in [1, 64]");
        plan->cfg.rows = rows;
        plan->cfg.zchunk = zchunk;
    });
}

fdtd_status fdtd_plan_set_tile_order(fdtd_plan *plan, int32_t order)
{
    PLAN_GUARD(plan) {
        REQUIRE(valid_order(order), FDTD_E_INVALID_ARG, "tile order must be -1 or in [0, 4096]");
        plan->cfg.order = order;
    });
}

fdtd_status fdtd_plan_get_tile_order(const fdtd_plan *plan, int32_t *order, int32_t *used)
{
    if (!plan) return FDTD_E_INVALID_ARG;
    if (order) *order = plan->cfg.order;
    if (used) *used = tile_order(plan->cfg, plan->ws_bytes);
    return FDTD_OK;
}

fdtd_status fdtd_plan_set_stream_stores(fdtd_plan *plan, int32_t mode)
{
    PLAN_GUARD(plan) {
        REQUIRE(mode >= -1 && mode <= 1, FDTD_E_INVALID_ARG, "stream-store mode must be -1, 0 or 1");
        plan->cfg.stream = mode;
    });
}

fdtd_status fdtd_plan_get_stream_stores(const fdtd_plan *plan, int32_t *mode, int32_t *used)
{
    if (!plan) return FDTD_E_INVALID_ARG;
    if (mode) *mode = plan->cfg.stream;
    if (used) *used = stream_stores(plan->cfg, plan->ws_bytes);
    return FDTD_OK;
}

fdtd_status fdtd_plan_set_temporal(fdtd_plan *plan, int32_t mode)
{
    PLAN_GUARD(plan) {
        REQUIRE(mode >= -1 && mode <= 1, FDTD_E_INVALID_ARG, "two-level mode must be -1, 0 or 1");
        REQUIRE(!plan->finalized, FDTD_E_STATE, "two-level mode is set before the plan is finalized");
        REQUIRE(mode != 1 || plan->g.kernel == FDTD_KERNEL_FUSED, FDTD_E_UNSUPPORTED,
                "two-level steps need the fused FP32 kernel");
        plan->tb_mode = mode;
    });
}

fdtd_status fdtd_plan_set_temporal_config(fdtd_plan *plan, int32_t tile_rows, int32_t zchunk)
{
    PLAN_GUARD(plan) {
        REQUIRE(valid_tb_rows(tile_rows), FDTD_E_INVALID_ARG, "two-level tile rows must be 8, 10 or 13");
        REQUIRE(zchunk >= 4 && zchunk <= 256, FDTD_E_INVALID_ARG,
                "two-level z-chunk must be in [4, 256]");
        plan->cfg.tb_rows = tile_rows;
        plan->cfg.tb_zchunk = zchunk;
        plan->cfg.tb_depth = 2;
    });
}

fdtd_status fdtd_plan_get_temporal(const fdtd_plan *plan, int32_t *mode, int32_t *used,
                                   int32_t *tile_rows, int32_t *zchunk, int32_t *tiles)
{
    if (!plan) return FDTD_E_INVALID_ARG;
    if (mode) *mode = plan->tb_mode;
    const bool on = plan->tb && plan->cfg.tb_depth == 2;
    if (used) *used = on ? 1 : 0;
    if (tile_rows) *tile_rows = plan->cfg.tb_rows;
    if (zchunk) *zchunk = plan->cfg.tb_zchunk;
    if (tiles) {
        if (!on) {
            *tiles = 0;
        } else {
            TileSet t = make_tileset(*plan, plan->cfg);
            *tiles = make_tbset(*plan, plan->cfg, t).n;
        }
    }
    return FDTD_OK;
}

fdtd_status fdtd_plan_autotune(fdtd_plan *plan, int32_t trial_steps, const char *cache_path,
                               void *stream, int32_t *best_index)
{
    PLAN_GUARD(plan) {
        Plan &P = *plan;
        REQUIRE(P.bound, FDTD_E_STATE, "plan not bound");
        REQUIRE(!P.in_batch, FDTD_E_STATE, "plan belongs to a batch; use fdtd_batch_autotune");
        REQUIRE(P.g.kernel == FDTD_KERNEL_FUSED, FDTD_E_UNSUPPORTED,
                "only the fused kernel has a launch shape to tune");
        REQUIRE(trial_steps >= 1, FDTD_E_INVALID_ARG, "trial_steps must be >= 1");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const Plan *self = &P;
        // plans with the third buffer search more: their own cache entries
        const std::string key = tune_device_name() + "|" + tune_shape_key(&self, 1) +
                                (P.tb ? "two-level" : "");
        TimerPause pause(P.timer);   // trial launches are not the caller's
        TuneHooks h;
        h.apply = [&](const LaunchCfg &c) { P.cfg = c; };
        h.run = [&](int32_t n) { run_plan(P, n, s); };
        h.two_level = P.tb;
        LaunchCfg best = P.cfg;
        int32_t best_i = -1;
        hip_check(tune_search(h, trial_steps, cache_path, key, s, best, best_i), "autotune");
        if (best_i >= 0) {
            reset_plan(P, s);
            hip_check(hipStreamSynchronize(s), "sync");
        }
        if (best_index) *best_index = best_i;
    });
}

fdtd_status fdtd_plan_set_timing(fdtd_plan *plan, int32_t enable)
{
    PLAN_GUARD(plan) {
        REQUIRE(enable >= 0, FDTD_E_INVALID_ARG, "negative timing stride");
        hip_check(plan->timer.drain(), "timer drain");
        plan->timer.reset();
        plan->timer.on = enable != 0;
        plan->timer.every = enable > 1 ? enable : 1;
    });
}

fdtd_status fdtd_plan_get_kernel_time(fdtd_plan *plan, double *ms, int64_t *launches)
{
    PLAN_GUARD(plan) {
        hip_check(plan->timer.drain(), "timer drain");
        if (ms) *ms = plan->timer.ms;
        if (launches) *launches = plan->timer.launches;
    });
}

}  // extern "C"
