// Fused FP32 Yee step: H^{n+1/2} and E^{n+1} (with the absorbing-layer
// auxiliaries and the soft source) in one pass over the grid.
//
// A block owns a tile of 64 (x) by R (y) cells and marches through a chunk of
// z planes.  For plane k it needs E^n of planes k and k+1 with a one-cell
// halo in x and y: three E planes rotate through LDS (k and k+1 in use, k+2
// being filled from registers loaded one iteration earlier).  H^{n+1/2}(k)
// is computed for the tile plus the low-x column and low-y row (the halo the
// E update needs, recomputed instead of exchanged) and kept in LDS; E^{n+1}(k)
// follows from it and the H^{n+1/2}(k-1) values each thread carries in
// registers from the previous plane.
//
// Latency hiding: everything plane k+1 needs from HBM (E of plane k+2, H^{n-1/2},
// material ids, auxiliaries) is requested at the top of iteration k and only
// consumed one iteration later; the block barriers order LDS only, so those
// loads stay in flight across them.
//
// Reads and writes go to separate buffers (fields and auxiliaries are
// ping-ponged between steps), so the halo a block recomputes never races
// with the block that owns those cells.  Neighbouring tiles are kept on the
// same XCD so their halo re-reads hit that XCD's L2.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "probe.hpp"

namespace fdtd {

namespace {

constexpr int TW = 64;        // tile width in x = one wavefront
constexpr int LUT_LDS = 64;   // LUTs up to this many entries live in LDS

// Block barrier that orders LDS accesses only: outstanding global loads
// (the prefetch of the next plane) stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ bool layer_slot(int p, int lo, int hi, int n, int &s)
{
    if (p < lo) { s = p; return true; }
    if (p >= n - hi) { s = p - (n - hi) + lo; return true; }
    return false;
}

__device__ double src_value(const DevGrid<float> &d, int64_t level)
{
    if (d.src_kind == FDTD_WAVE_GAUSSIAN_STEPS) {
        const double u = ((double)level - d.src_t0) / d.src_w;
        return d.src_amp * exp(-u * u);
    }
    const double t = (double)level * d.dt;
    if (d.src_kind == FDTD_WAVE_GAUSS_SINE) {
        const double u = (t - d.src_t0) / d.src_tau;
        return d.src_amp * exp(-u * u) * sin(2.0 * M_PI * d.src_fc * (t - d.src_t0));
    }
    if (d.src_kind == FDTD_WAVE_DIFF_GAUSSIAN) {
        const double u = (t - d.src_t0) / d.src_w;
        return d.src_amp * (-2.0 * u) * exp(-u * u);
    }
    return 0.0;
}

// Every device array is accessed through the global address space with a
// 32-bit byte offset from a uniform base: the loads become global (not flat)
// instructions with the scalar-base + 32-bit vector-offset form, and since
// global loads do not count against the LDS wait counter, the LDS-only block
// barriers leave them in flight.  (Every array of a fused plan is smaller
// than 4 GiB, checked on the host.)
#define GLOBAL_AS __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ T gld(const T *base, uint32_t idx)
{
    const GLOBAL_AS char *b = (const GLOBAL_AS char *)base;
    return *(const GLOBAL_AS T *)(b + idx * (uint32_t)sizeof(T));
}

template <typename T>
__device__ __forceinline__ void gst(T *base, uint32_t idx, T v)
{
    GLOBAL_AS char *b = (GLOBAL_AS char *)base;
    *(GLOBAL_AS T *)(b + idx * (uint32_t)sizeof(T)) = v;
}

__device__ __forceinline__ float ldf(const float *base, uint32_t idx) { return gld(base, idx); }
__device__ __forceinline__ void stf(float *base, uint32_t idx, float v) { gst(base, idx, v); }

// One {Ca, Cb/d1, Cb/d2, 0} LUT entry as a single 16-byte global load.
__device__ __forceinline__ float4 lut_entry(const float *lut, int id)
{
    typedef float f4v __attribute__((ext_vector_type(4)));
    const f4v v = gld(reinterpret_cast<const f4v *>(lut), (uint32_t)id);
    return make_float4(v.x, v.y, v.z, v.w);
}

// Layer-modified difference: diff/kappa + psi with psi <- b psi + c diff
// (b, c, 1/kappa of the position, from the block's LDS profile cache).
__device__ __forceinline__ float lterm(float diff, float b, float c, float ik, float psi_old,
                                       float &psi_new)
{
    psi_new = b * psi_old + c * diff;
    return diff * ik + psi_new;
}

// Auxiliary slots of one cell: which layers it is in and its index in each.
struct LayerPos {
    bool inx, iny, inz;
    uint32_t qx, qy, qz;
};

__device__ __forceinline__ LayerPos layer_pos(const DevGrid<float> &d, int i, int j, int k)
{
    LayerPos L;
    int s;
    L.inx = layer_slot(i, d.lo[0], d.hi[0], d.nx, s);
    L.qx = L.inx ? (uint32_t)(s + (d.lo[0] + d.hi[0]) * (j + d.ny * k)) : 0u;
    L.iny = layer_slot(j, d.lo[1], d.hi[1], d.ny, s);
    L.qy = L.iny ? (uint32_t)(i + d.px * (s + (d.lo[1] + d.hi[1]) * k)) : 0u;
    L.inz = layer_slot(k, d.lo[2], d.hi[2], d.nz, s);
    L.qz = L.inz ? (uint32_t)(i + d.px * (j + d.ny * s)) : 0u;
    return L;
}

// The six H auxiliaries of one cell (the first six PsiId values), zero
// outside the layers.
struct Psi6 {
    float v[6];
};

__device__ __forceinline__ void load_psi_h(const DevGrid<float> &d, const LayerPos &L, Psi6 &p)
{
    p.v[PSI_HXY] = L.iny ? ldf(d.psi[PSI_HXY], L.qy) : 0.f;
    p.v[PSI_HZY] = L.iny ? ldf(d.psi[PSI_HZY], L.qy) : 0.f;
    p.v[PSI_HYX] = L.inx ? ldf(d.psi[PSI_HYX], L.qx) : 0.f;
    p.v[PSI_HZX] = L.inx ? ldf(d.psi[PSI_HZX], L.qx) : 0.f;
    p.v[PSI_HXZ] = L.inz ? ldf(d.psi[PSI_HXZ], L.qz) : 0.f;
    p.v[PSI_HYZ] = L.inz ? ldf(d.psi[PSI_HYZ], L.qz) : 0.f;
}

// The six E auxiliaries (indexed PsiId - 6).
__device__ __forceinline__ void load_psi_e(const DevGrid<float> &d, const LayerPos &L, Psi6 &p)
{
    p.v[PSI_EXY - 6] = L.iny ? ldf(d.psi[PSI_EXY], L.qy) : 0.f;
    p.v[PSI_EZY - 6] = L.iny ? ldf(d.psi[PSI_EZY], L.qy) : 0.f;
    p.v[PSI_EYX - 6] = L.inx ? ldf(d.psi[PSI_EYX], L.qx) : 0.f;
    p.v[PSI_EZX - 6] = L.inx ? ldf(d.psi[PSI_EZX], L.qx) : 0.f;
    p.v[PSI_EXZ - 6] = L.inz ? ldf(d.psi[PSI_EXZ], L.qz) : 0.f;
    p.v[PSI_EYZ - 6] = L.inz ? ldf(d.psi[PSI_EYZ], L.qz) : 0.f;
}

struct HDiff {
    float ez_y, ey_z, ex_z, ez_x, ey_x, ex_y;
};

constexpr int ZMAX = 64;   // longest z-chunk (its profiles are cached in LDS)

template <int R>
struct Smem {
    float e[3][3][R + 2][TW + 2];   // 3 rotating E^n planes: rows y0-1..y0+R, cols x0-1..x0+64
    float h[3][R + 1][TW + 1];      // H^{n+1/2}(k): rows y0-1..y0+R-1, cols x0-1..x0+63
    float4 lut[3][LUT_LDS];
    float px[PR_COUNT][TW + 2];     // x profiles at x0-1 .. x0+64
    float py[PR_COUNT][R + 2];      // y profiles at y0-1 .. y0+R
    float pz[PR_COUNT][ZMAX + 1];   // z profiles at z0-1 .. z0+ZMAX-1
};

// H^{n+1/2} from H^{n-1/2} and the six forward differences of E^n at the
// LDS-cache positions (lx, ly, lz) of the block.  With `store` the updated
// auxiliaries of the H components are written.
template <int R>
__device__ __forceinline__ void h_apply(const DevGrid<float> &d, const Smem<R> &sm,
                                        const LayerPos &L, int lx, int ly, int lz, HDiff df,
                                        const Psi6 &ps, bool store, float hx, float hy, float hz,
                                        float &ox, float &oy, float &oz)
{
    float pn;
    if (L.inx) {
        const float b = sm.px[PR_BH][lx], c = sm.px[PR_CH][lx], ik = sm.px[PR_KH][lx];
        df.ez_x = lterm(df.ez_x, b, c, ik, ps.v[PSI_HYX], pn);
        if (store) stf(d.psi_o[PSI_HYX], L.qx, pn);
        df.ey_x = lterm(df.ey_x, b, c, ik, ps.v[PSI_HZX], pn);
        if (store) stf(d.psi_o[PSI_HZX], L.qx, pn);
    }
    if (L.iny) {
        const float b = sm.py[PR_BH][ly], c = sm.py[PR_CH][ly], ik = sm.py[PR_KH][ly];
        df.ez_y = lterm(df.ez_y, b, c, ik, ps.v[PSI_HXY], pn);
        if (store) stf(d.psi_o[PSI_HXY], L.qy, pn);
        df.ex_y = lterm(df.ex_y, b, c, ik, ps.v[PSI_HZY], pn);
        if (store) stf(d.psi_o[PSI_HZY], L.qy, pn);
    }
    if (L.inz) {
        const float b = sm.pz[PR_BH][lz], c = sm.pz[PR_CH][lz], ik = sm.pz[PR_KH][lz];
        df.ey_z = lterm(df.ey_z, b, c, ik, ps.v[PSI_HXZ], pn);
        if (store) stf(d.psi_o[PSI_HXZ], L.qz, pn);
        df.ex_z = lterm(df.ex_z, b, c, ik, ps.v[PSI_HYZ], pn);
        if (store) stf(d.psi_o[PSI_HYZ], L.qz, pn);
    }
    ox = hx - d.ch[1] * df.ez_y + d.ch[2] * df.ey_z;
    oy = hy - d.ch[2] * df.ex_z + d.ch[0] * df.ez_x;
    oz = hz - d.ch[0] * df.ey_x + d.ch[1] * df.ex_y;
}

// Rows of the E patch a wave loads: R waves share the R+2 rows of each
// component; halo columns x0-1 and x0+64 are loaded by the first threads.
template <int R>
struct EPatch {
    static constexpr int Q = (R + 2 + R - 1) / R;   // rows per wave and component
    float v[3][Q];
    float halo;
};

template <int R>
__device__ __forceinline__ void epatch_load(const DevGrid<float> &d, EPatch<R> &p, int x0, int y0,
                                            int k)
{
    const int t = threadIdx.x, lane = t & (TW - 1), w = t / TW;
    const uint32_t base = (uint32_t)(d.off + x0 + d.px * (y0 - 1) + d.px * d.py * k);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < EPatch<R>::Q; ++q) {
            const int row = w + R * q;
            if (row < R + 2) p.v[c][q] = ldf(d.E[c], base + d.px * row + lane);
        }
    // halo columns: thread t -> side t & 1, component and row from t >> 1
    if (t < 6 * (R + 2)) {
        const int side = t & 1, rest = t >> 1;
        const int c = rest / (R + 2), row = rest % (R + 2);
        const uint32_t a = base + d.px * row + (side ? TW : 0) - (side ? 0 : 1);
        p.halo = ldf(c == 0 ? d.E[0] : (c == 1 ? d.E[1] : d.E[2]), a);
    }
}

template <int R>
__device__ __forceinline__ void epatch_store(Smem<R> &sm, const EPatch<R> &p, int slot)
{
    const int t = threadIdx.x, lane = t & (TW - 1), w = t / TW;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < EPatch<R>::Q; ++q) {
            const int row = w + R * q;
            if (row < R + 2) sm.e[slot][c][row][lane + 1] = p.v[c][q];
        }
    if (t < 6 * (R + 2)) {
        const int side = t & 1, rest = t >> 1;
        const int c = rest / (R + 2), row = rest % (R + 2);
        sm.e[slot][c][row][side ? TW + 1 : 0] = p.halo;
    }
}

// What plane k of the own cell (and the halo cell of this thread) needs
// from HBM besides the E patch; loaded one plane ahead.
struct PlaneRegs {
    float hx, hy, hz;          // H^{n-1/2} own
    int idx, idy, idz;         // edge ids own
    float hhx, hhy, hhz;       // H^{n-1/2} of the halo cell
    Psi6 ph;                   // H auxiliaries of the own cell
};

__device__ __forceinline__ void plane_load(const DevGrid<float> &d, PlaneRegs &r, bool own, int i,
                                           int j, int k, bool has_halo, int hi_, int hj_)
{
    if (own) {
        const uint32_t c = (uint32_t)(d.off + i + d.px * j + d.px * d.py * k);
        r.hx = ldf(d.H[0], c);
        r.hy = ldf(d.H[1], c);
        r.hz = ldf(d.H[2], c);
        const uint32_t qi = (uint32_t)(i + d.px * (j + d.ny * k));
        if (d.id16) {
            r.idx = gld(static_cast<const uint16_t *>(d.ids[0]), qi);
            r.idy = gld(static_cast<const uint16_t *>(d.ids[1]), qi);
            r.idz = gld(static_cast<const uint16_t *>(d.ids[2]), qi);
        } else {
            r.idx = gld(static_cast<const uint8_t *>(d.ids[0]), qi);
            r.idy = gld(static_cast<const uint8_t *>(d.ids[1]), qi);
            r.idz = gld(static_cast<const uint8_t *>(d.ids[2]), qi);
        }
        load_psi_h(d, layer_pos(d, i, j, k), r.ph);
    }
    if (has_halo) {
        const uint32_t c = (uint32_t)(d.off + hi_ + d.px * hj_ + d.px * d.py * k);
        r.hhx = ldf(d.H[0], c);
        r.hhy = ldf(d.H[1], c);
        r.hhz = ldf(d.H[2], c);
    }
}

// Profile value of table `tab` at position p of an axis of length n (the
// tables cover [0, n); positions outside never enter an update).
__device__ __forceinline__ float prof_at(const float *prof, int tab, int n, int p)
{
    return (p >= 0 && p < n) ? gld(prof, (uint32_t)(tab * n + p)) : 0.f;
}

template <int R>
__device__ void fused_tile(const DevGrid<float> &d, int tile, int zchunk, int64_t level,
                           Smem<R> &sm)
{
    const int tiles_x = (d.nx + TW - 1) / TW, tiles_y = (d.ny + R - 1) / R;
    const int tx = tile % tiles_x;
    const int ty = (tile / tiles_x) % tiles_y;
    const int tz = tile / (tiles_x * tiles_y);
    const int x0 = tx * TW, y0 = ty * R, z0 = tz * zchunk;
    const int z1 = min(z0 + zchunk, d.nz);
    const int t = threadIdx.x;
    const int lane = t & (TW - 1), row = t / TW;
    const int i = x0 + lane, j = y0 + row;
    const bool own = i < d.nx && j < d.ny;
    const int sy = d.px, sz = d.px * d.py;
    const int lx = lane + 1, ly = row + 1;

    // the halo cell this thread recomputes H for (low-y row, then low-x column)
    int hi_ = 0, hj_ = 0;
    const bool halo_thread = t < TW + R + 1;
    if (halo_thread) {
        if (t < TW) { hi_ = x0 + t; hj_ = y0 - 1; }
        else { hi_ = x0 - 1; hj_ = y0 - 1 + (t - TW); }
    }
    // only halo cells inside the grid matter: the others feed PEC edges only
    const bool halo_live = halo_thread && hi_ >= 0 && hj_ >= 0 && hi_ < d.nx && hj_ < d.ny;
    const int hlx = hi_ - x0 + 1, hly = hj_ - y0 + 1;

    // ---- block caches: LUTs and the layer profiles of the tile ------------
    const int nlut = d.nlut;
    const bool lut_lds = nlut <= LUT_LDS;
    if (lut_lds)
        for (int q = t; q < 3 * nlut; q += TW * R) {
            const int c = q / nlut, e = q % nlut;
            sm.lut[c][e] = lut_entry(c == 0 ? d.lut[0] : (c == 1 ? d.lut[1] : d.lut[2]), e);
        }
    for (int q = t; q < PR_COUNT * (TW + 2); q += TW * R) {
        const int tab = q / (TW + 2), p = q % (TW + 2);
        sm.px[tab][p] = prof_at(d.prof[0], tab, d.nx, x0 - 1 + p);
    }
    for (int q = t; q < PR_COUNT * (R + 2); q += TW * R) {
        const int tab = q / (R + 2), p = q % (R + 2);
        sm.py[tab][p] = prof_at(d.prof[1], tab, d.ny, y0 - 1 + p);
    }
    for (int q = t; q < PR_COUNT * (ZMAX + 1); q += TW * R) {
        const int tab = q / (ZMAX + 1), p = q % (ZMAX + 1);
        sm.pz[tab][p] = prof_at(d.prof[2], tab, d.nz, z0 - 1 + p);
    }

    // ---- prologue: request everything the first plane needs at once -------
    EPatch<R> pa, pb;
    epatch_load<R>(d, pa, x0, y0, z0);
    epatch_load<R>(d, pb, x0, y0, z0 + 1);
    PlaneRegs cur_r{}, nxt_r{};
    plane_load(d, cur_r, own, i, j, z0, halo_live, hi_, hj_);
    // inputs of H^{n+1/2}(z0-1) at the own cell, needed by E(z0); on the
    // bottom face the E edges it feeds are PEC, so it is not needed there
    const bool pro = own && z0 > 0;
    HDiff pdf{};
    float phx = 0.f, phy = 0.f, phz = 0.f;
    Psi6 pps{};
    LayerPos pL{};
    if (pro) {
        const uint32_t c = (uint32_t)(d.off + i + sy * j + sz * (z0 - 1));
        const float ex = ldf(d.E[0], c), ey = ldf(d.E[1], c), ez = ldf(d.E[2], c);
        pdf.ez_y = ldf(d.E[2], c + sy) - ez;
        pdf.ey_z = ldf(d.E[1], c + sz) - ey;
        pdf.ex_z = ldf(d.E[0], c + sz) - ex;
        pdf.ez_x = ldf(d.E[2], c + 1) - ez;
        pdf.ey_x = ldf(d.E[1], c + 1) - ey;
        pdf.ex_y = ldf(d.E[0], c + sy) - ex;
        phx = ldf(d.H[0], c);
        phy = ldf(d.H[1], c);
        phz = ldf(d.H[2], c);
        pL = layer_pos(d, i, j, z0 - 1);
        load_psi_h(d, pL, pps);
    }
    float sval = 0.f;
    const bool src_col = d.src_kind != 0 && own && i >= d.src_box[0] && i <= d.src_box[1] &&
                         j >= d.src_box[2] && j <= d.src_box[3];
    if (src_col) sval = (float)src_value(d, level + 1);
    lds_barrier();   // caches visible

    float hx_prev = 0.f, hy_prev = 0.f;
    if (pro) {
        float oz;
        h_apply<R>(d, sm, pL, lx, ly, 0, pdf, pps, false, phx, phy, phz, hx_prev, hy_prev, oz);
    }
    epatch_store<R>(sm, pa, 0);
    epatch_store<R>(sm, pb, 1);
    lds_barrier();

    int s0 = 0, s1 = 1, s2 = 2;   // LDS slots of planes k, k+1, k+2
    for (int k = z0; k < z1; ++k) {
        const int lz = k - z0 + 1;
        // ---- requests: this plane's E and halo auxiliaries, and everything
        //      plane k+1 needs from HBM (consumed one iteration later) ------
        const LayerPos L = layer_pos(d, i, j, k);
        Psi6 pe_cur{}, ph_halo{};
        if (own) load_psi_e(d, L, pe_cur);
        LayerPos Lh{};
        if (halo_live) {
            Lh = layer_pos(d, hi_, hj_, k);
            load_psi_h(d, Lh, ph_halo);
        }
        EPatch<R> pe;
        const bool more_e = k + 2 <= z1;
        if (more_e) epatch_load<R>(d, pe, x0, y0, k + 2);
        if (k + 1 < z1) plane_load(d, nxt_r, own, i, j, k + 1, halo_live, hi_, hj_);

        const uint32_t c = (uint32_t)(d.off + i + sy * j + sz * k);
        // ---- H^{n+1/2}(k): own cell ---------------------------------------
        {
            HDiff df;
            const float ex = sm.e[s0][0][ly][lx], ey = sm.e[s0][1][ly][lx], ez = sm.e[s0][2][ly][lx];
            df.ez_y = sm.e[s0][2][ly + 1][lx] - ez;
            df.ey_z = sm.e[s1][1][ly][lx] - ey;
            df.ex_z = sm.e[s1][0][ly][lx] - ex;
            df.ez_x = sm.e[s0][2][ly][lx + 1] - ez;
            df.ey_x = sm.e[s0][1][ly][lx + 1] - ey;
            df.ex_y = sm.e[s0][0][ly + 1][lx] - ex;
            float ox = 0.f, oy = 0.f, oz = 0.f;
            if (own) {
                h_apply<R>(d, sm, L, lx, ly, lz, df, cur_r.ph, true, cur_r.hx, cur_r.hy, cur_r.hz,
                           ox, oy, oz);
                stf(d.Ho[0], c, ox);
                stf(d.Ho[1], c, oy);
                stf(d.Ho[2], c, oz);
            }
            sm.h[0][ly][lx] = ox;
            sm.h[1][ly][lx] = oy;
            sm.h[2][ly][lx] = oz;
        }
        // ---- H^{n+1/2}(k): halo row y0-1 and halo column x0-1 -------------
        if (halo_thread) {
            float ox = 0.f, oy = 0.f, oz = 0.f;
            if (halo_live) {
                HDiff df;
                const float ex = sm.e[s0][0][hly][hlx], ey = sm.e[s0][1][hly][hlx],
                            ez = sm.e[s0][2][hly][hlx];
                df.ez_y = sm.e[s0][2][hly + 1][hlx] - ez;
                df.ey_z = sm.e[s1][1][hly][hlx] - ey;
                df.ex_z = sm.e[s1][0][hly][hlx] - ex;
                df.ez_x = sm.e[s0][2][hly][hlx + 1] - ez;
                df.ey_x = sm.e[s0][1][hly][hlx + 1] - ey;
                df.ex_y = sm.e[s0][0][hly + 1][hlx] - ex;
                h_apply<R>(d, sm, Lh, hlx, hly, lz, df, ph_halo, false, cur_r.hhx, cur_r.hhy,
                           cur_r.hhz, ox, oy, oz);
            }
            sm.h[0][hly][hlx] = ox;
            sm.h[1][hly][hlx] = oy;
            sm.h[2][hly][hlx] = oz;
        }
        lds_barrier();

        // ---- E^{n+1}(k): own cell -----------------------------------------
        if (own) {
            const float hx = sm.h[0][ly][lx], hy = sm.h[1][ly][lx], hz = sm.h[2][ly][lx];
            float dHz_y = hz - sm.h[2][ly - 1][lx];
            float dHy_z = hy - hy_prev;
            float dHx_z = hx - hx_prev;
            float dHz_x = hz - sm.h[2][ly][lx - 1];
            float dHy_x = hy - sm.h[1][ly][lx - 1];
            float dHx_y = hx - sm.h[0][ly - 1][lx];
            float pn;
            if (L.inx) {
                const float b = sm.px[PR_BE][lx], cc = sm.px[PR_CE][lx], ik = sm.px[PR_KE][lx];
                dHz_x = lterm(dHz_x, b, cc, ik, pe_cur.v[PSI_EYX - 6], pn);
                stf(d.psi_o[PSI_EYX], L.qx, pn);
                dHy_x = lterm(dHy_x, b, cc, ik, pe_cur.v[PSI_EZX - 6], pn);
                stf(d.psi_o[PSI_EZX], L.qx, pn);
            }
            if (L.iny) {
                const float b = sm.py[PR_BE][ly], cc = sm.py[PR_CE][ly], ik = sm.py[PR_KE][ly];
                dHz_y = lterm(dHz_y, b, cc, ik, pe_cur.v[PSI_EXY - 6], pn);
                stf(d.psi_o[PSI_EXY], L.qy, pn);
                dHx_y = lterm(dHx_y, b, cc, ik, pe_cur.v[PSI_EZY - 6], pn);
                stf(d.psi_o[PSI_EZY], L.qy, pn);
            }
            if (L.inz) {
                const float b = sm.pz[PR_BE][lz], cc = sm.pz[PR_CE][lz], ik = sm.pz[PR_KE][lz];
                dHy_z = lterm(dHy_z, b, cc, ik, pe_cur.v[PSI_EXZ - 6], pn);
                stf(d.psi_o[PSI_EXZ], L.qz, pn);
                dHx_z = lterm(dHx_z, b, cc, ik, pe_cur.v[PSI_EYZ - 6], pn);
                stf(d.psi_o[PSI_EYZ], L.qz, pn);
            }
            float4 cx, cy, cz;
            if (lut_lds) {
                cx = sm.lut[0][cur_r.idx];
                cy = sm.lut[1][cur_r.idy];
                cz = sm.lut[2][cur_r.idz];
            } else {
                cx = lut_entry(d.lut[0], cur_r.idx);
                cy = lut_entry(d.lut[1], cur_r.idy);
                cz = lut_entry(d.lut[2], cur_r.idz);
            }
            stf(d.Eo[0], c, cx.x * sm.e[s0][0][ly][lx] + cx.y * dHz_y - cx.z * dHy_z);
            stf(d.Eo[1], c, cy.x * sm.e[s0][1][ly][lx] + cy.y * dHx_z - cy.z * dHz_x);
            float ez = cz.x * sm.e[s0][2][ly][lx] + cz.y * dHy_x - cz.z * dHx_y;
            if (src_col && k >= d.src_box[4] && k <= d.src_box[5]) ez += sval;
            stf(d.Eo[2], c, ez);
            hx_prev = hx;
            hy_prev = hy;
        }
        // ---- rotate: plane k+2 into LDS, next plane's registers current ----
        if (more_e) epatch_store<R>(sm, pe, s2);
        cur_r = nxt_r;
        const int sf = s0;
        s0 = s1;
        s1 = s2;
        s2 = sf;
        lds_barrier();
    }
}

// Block b of n is dispatched to XCD b % 8; give each XCD a contiguous run
// of tiles so that neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int xcd = b & 7, idx = b >> 3;
    const int q = n >> 3, r = n & 7;
    return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + idx;
}

// One launch = one leapfrog step of every instance in the table.  The first
// `nprobe_blocks` blocks sample the probes of the input level (so sampling
// overlaps the update instead of costing a launch of its own); the others
// update tiles.
template <int R>
__global__ void __launch_bounds__(TW *R)
k_fused(const DevGrid<float> *__restrict__ grids, const int32_t *__restrict__ block_start,
        int ninst, int zchunk, int ntiles, int64_t level, const DevProbes *__restrict__ probes,
        int nprobe_blocks, int max_probes)
{
    __shared__ Smem<R> sm;
    const int b = blockIdx.x;
    if (b < nprobe_blocks) {
        const int inst = b / max_probes, q = b % max_probes;
        if (q < probes[inst].nprobe)
            probe_one(grids[inst], probes[inst], q, level, reinterpret_cast<double *>(&sm));
        return;
    }
    const int tb = xcd_tile(b - nprobe_blocks, ntiles);
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {          // last instance whose first block <= tb
        const int mid = (lo + hi + 1) >> 1;
        if (block_start[mid] <= tb) lo = mid;
        else hi = mid - 1;
    }
    fused_tile<R>(grids[lo], tb - block_start[lo], zchunk, level, sm);
}

template <int R>
hipError_t launch_r(const DevGrid<float> *g, const int32_t *bs, int ninst, int ntiles, int zchunk,
                    int64_t level, const DevProbes *probes, int nprobe_blocks, int max_probes,
                    hipStream_t s)
{
    k_fused<R><<<ntiles + nprobe_blocks, TW * R, 0, s>>>(g, bs, ninst, zchunk, ntiles, level,
                                                         probes, nprobe_blocks, max_probes);
    return hipGetLastError();
}

}  // namespace

int32_t fused_tiles(int32_t nx, int32_t ny, int32_t nz, const LaunchCfg &cfg)
{
    const int tx = (nx + TW - 1) / TW, ty = (ny + cfg.rows - 1) / cfg.rows;
    const int tz = (nz + cfg.zchunk - 1) / cfg.zchunk;
    return tx * ty * tz;
}

hipError_t launch_fused(const DevGrid<float> *grids_dev, const int32_t *block_start_dev,
                        int32_t ninst, int32_t ntiles, const LaunchCfg &cfg, int64_t level,
                        const DevProbes *probes_dev, int32_t max_probes, bool sample_input,
                        hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const int npb = (sample_input && level >= 1) ? ninst * max_probes : 0;
    if (e0) (void)hipEventRecord(e0, s);
    hipError_t err;
    switch (cfg.rows) {
    case 2: err = launch_r<2>(grids_dev, block_start_dev, ninst, ntiles, cfg.zchunk, level, probes_dev, npb, max_probes, s); break;
    case 4: err = launch_r<4>(grids_dev, block_start_dev, ninst, ntiles, cfg.zchunk, level, probes_dev, npb, max_probes, s); break;
    case 8: err = launch_r<8>(grids_dev, block_start_dev, ninst, ntiles, cfg.zchunk, level, probes_dev, npb, max_probes, s); break;
    case 16: err = launch_r<16>(grids_dev, block_start_dev, ninst, ntiles, cfg.zchunk, level, probes_dev, npb, max_probes, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e1) (void)hipEventRecord(e1, s);
    return err;
}

}  // namespace fdtd
