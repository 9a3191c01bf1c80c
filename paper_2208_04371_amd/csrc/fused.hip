// Fused FP32 Yee step: H^{n+1/2} and E^{n+1} (with the absorbing-layer
// auxiliaries and the soft source) in one pass over the grid.
//
// A block of 64 x R threads owns a tile of 64 (x) by R (y) cells, or in the
// last x column of a grid whose width leaves a remainder of at most 32, a
// narrow tile of 16 by 4R cells, and marches through a chunk of z planes.  For plane k it needs E^n of planes k and k+1 with a one-cell
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

#include <type_traits>

#include "internal.hpp"
#include "probe.hpp"
#include "source.hpp"

namespace fdtd {

namespace {

constexpr int TW = 64;        // tile width in x = one wavefront
constexpr int NW = 16;        // width of the narrow tiles of a ragged last column
constexpr int LUT_LDS = 256;  // coefficient sets per component (8-bit ids)

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

// Field store of the step's output.  NT: streaming (non-temporal) store,
// for states larger than the memory-side cache: the value is not read again
// until the next step, so caching it only evicts this step's inputs.  For a
// cache-resident state the plain store keeps the next step's inputs cached.
template <bool NT>
__device__ __forceinline__ void field_st(float *base, uint32_t idx, float v)
{
    if constexpr (NT) {
        GLOBAL_AS char *b = (GLOBAL_AS char *)base;
        __builtin_nontemporal_store(v, (GLOBAL_AS float *)(b + idx * (uint32_t)sizeof(float)));
    } else {
        gst(base, idx, v);
    }
}

// One {Ca, Cb/d1, Cb/d2, 0} LUT entry as a single 16-byte global load.
__device__ __forceinline__ float4 lut_entry(const float *lut, int id)
{
    typedef float f4v __attribute__((ext_vector_type(4)));
    const f4v v = gld(reinterpret_cast<const f4v *>(lut), (uint32_t)id);
    return make_float4(v.x, v.y, v.z, v.w);
}

// The two update formulas with their rounding pinned (fused multiply-adds in
// a fixed order), so that the single-level and the two-level kernels give the
// same bits for the same inputs whatever the compiler contracts elsewhere:
//   H' = (H - c1 d1) + c2 d2            (c = dt / (mu0 delta))
//   E' = (Ca E + Cb1 d1) - Cb2 d2       (Cb1, Cb2 = Cb / delta of the two axes)
__device__ __forceinline__ float h_upd(float h, float c1, float d1, float c2, float d2)
{
    return __builtin_fmaf(c2, d2, __builtin_fmaf(-c1, d1, h));
}
__device__ __forceinline__ float e_upd(float e, const float4 &c, float d1, float d2)
{
    return __builtin_fmaf(-c.z, d2, __builtin_fmaf(c.y, d1, c.x * e));
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
    L.qy = L.iny ? (uint32_t)(i + d.nx * (s + (d.lo[1] + d.hi[1]) * k)) : 0u;
    L.inz = layer_slot(k, d.lo[2], d.hi[2], d.nz, s);
    L.qz = L.inz ? (uint32_t)(i + d.nx * (j + d.ny * s)) : 0u;
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

// LDS of a tile of X columns by Y rows.
template <int X, int Y>
struct Smem {
    float e[3][3][Y + 2][X + 2];    // 3 rotating E^n planes: rows y0-1..y0+Y, cols x0-1..x0+X
    float h[3][Y + 1][X + 1];       // H^{n+1/2}(k): rows y0-1..y0+Y-1, cols x0-1..x0+X-1
    float dummy[TW];                // target of the writes of repeated items
};

// The block's tables in the dynamic part of LDS, sized per launch: the
// coefficient LUTs ([3][cap] entries) and, in boundary launches, the layer
// profiles of the tile.
template <int X, int Y>
struct Tabs {
    float4 *lut;
    float *px, *py, *pz;            // [PR_COUNT][X+2] at x0-1.., [PR_COUNT][Y+2] at y0-1..,
    int cap;                        // [PR_COUNT][ZMAX+1] at z0-1..
    __device__ float4 coef(int c, uint32_t id) const { return lut[c * cap + (int)id]; }
    __device__ float prx(int tab, int p) const { return px[tab * (X + 2) + p]; }
    __device__ float pry(int tab, int p) const { return py[tab * (Y + 2) + p]; }
    __device__ float prz(int tab, int p) const { return pz[tab * (ZMAX + 1) + p]; }
    __device__ void place(float4 *dyn, int lut_cap)
    {
        cap = lut_cap;
        lut = dyn;
        px = reinterpret_cast<float *>(dyn + 3 * lut_cap);
        py = px + PR_COUNT * (X + 2);
        pz = py + PR_COUNT * (Y + 2);
    }
};

// Dynamic LDS of a launch: the LUTs, and in boundary launches the profiles
// of the larger of the two tile shapes.
template <int R>
constexpr size_t tabs_bytes(int cap, bool layers)
{
    constexpr int xy = (TW + 2 + R + 2) > (NW + 2 + TW * R / NW + 2) ? (TW + 2 + R + 2)
                                                                      : (NW + 2 + TW * R / NW + 2);
    return (size_t)cap * 3 * sizeof(float4) +
           (layers ? (size_t)PR_COUNT * (xy + ZMAX + 1) * sizeof(float) : 0);
}

// H^{n+1/2} from H^{n-1/2} and the six forward differences of E^n at the
// LDS-cache positions (lx, ly, lz) of the block.  Inside the layers (LAYERS
// kernels only) the differences take their auxiliaries; with `store` the
// updated auxiliaries of the H components are written.
template <int X, int Y, bool LAYERS>
__device__ __forceinline__ void h_apply(const DevGrid<float> &d, const Tabs<X, Y> &tb,
                                        const LayerPos &L, int lx, int ly, int lz, HDiff df,
                                        const Psi6 &ps, bool store, float hx, float hy, float hz,
                                        float &ox, float &oy, float &oz)
{
    if constexpr (LAYERS) {
        float pn;
        if (L.inx) {
            const float b = tb.prx(PR_BH, lx), c = tb.prx(PR_CH, lx), ik = tb.prx(PR_KH, lx);
            df.ez_x = lterm(df.ez_x, b, c, ik, ps.v[PSI_HYX], pn);
            if (store) stf(d.psi_o[PSI_HYX], L.qx, pn);
            df.ey_x = lterm(df.ey_x, b, c, ik, ps.v[PSI_HZX], pn);
            if (store) stf(d.psi_o[PSI_HZX], L.qx, pn);
        }
        if (L.iny) {
            const float b = tb.pry(PR_BH, ly), c = tb.pry(PR_CH, ly), ik = tb.pry(PR_KH, ly);
            df.ez_y = lterm(df.ez_y, b, c, ik, ps.v[PSI_HXY], pn);
            if (store) stf(d.psi_o[PSI_HXY], L.qy, pn);
            df.ex_y = lterm(df.ex_y, b, c, ik, ps.v[PSI_HZY], pn);
            if (store) stf(d.psi_o[PSI_HZY], L.qy, pn);
        }
        if (L.inz) {
            const float b = tb.prz(PR_BH, lz), c = tb.prz(PR_CH, lz), ik = tb.prz(PR_KH, lz);
            df.ey_z = lterm(df.ey_z, b, c, ik, ps.v[PSI_HXZ], pn);
            if (store) stf(d.psi_o[PSI_HXZ], L.qz, pn);
            df.ex_z = lterm(df.ex_z, b, c, ik, ps.v[PSI_HYZ], pn);
            if (store) stf(d.psi_o[PSI_HYZ], L.qz, pn);
        }
    }
    ox = h_upd(hx, d.ch[1], df.ez_y, d.ch[2], df.ey_z);
    oy = h_upd(hy, d.ch[2], df.ex_z, d.ch[0], df.ez_x);
    oz = h_upd(hz, d.ch[0], df.ey_x, d.ch[1], df.ex_y);
}

// The E^n patch of one plane: rows y0-1 .. y0+Y (Y+2) of the three
// components over columns x0 .. x0+X-1, and the halo columns x0-1, x0+X.
// The threads of row group g (X consecutive threads; one wave in 64-wide
// tiles) load row g of each component (rows 0..Y-1), NX more row loads from
// the six remaining (component, row Y or Y+1) items, and one halo value per
// thread.  Every wave issues the same loads: items past the last repeat it
// and land in a dummy LDS row, so no load sits behind a branch (a branch
// around a load makes the compiler wait for every load and store in flight).
// Narrow tiles clamp their rows to the top guard row: their Y can run past
// the end of the array, and rows beyond the grid only feed discarded cells.
template <int X, int Y>
struct EPatch {
    static constexpr int NX = (6 + Y - 1) / Y;       // extra row loads per row group
    static constexpr int NHALO = 6 * (Y + 2);        // 2 sides x 3 comps x rows
    float v[3];
    float x[NX];
    float halo;
};

__device__ __forceinline__ const float *comp_ptr(const float *c0, int64_t stride, int c)
{
    return reinterpret_cast<const float *>(reinterpret_cast<const char *>(c0) + c * stride);
}

// Patch row of a load (see EPatch).
template <int X>
__device__ __forceinline__ int patch_row(const DevGrid<float> &d, int y0, int row)
{
    if constexpr (X < TW) return min(row, d.ny + 1 - y0);
    else return row;
}

template <int X, int Y>
__device__ __forceinline__ void epatch_load(const DevGrid<float> &d, EPatch<X, Y> &p, int x0, int y0,
                                            int k, int g, int gx)
{
    const int t = threadIdx.x;
    const uint32_t base = (uint32_t)(d.off + x0 + d.px * (y0 - 1) + d.px * d.py * k);
    const int vr = patch_row<X>(d, y0, g);
#pragma unroll
    for (int c = 0; c < 3; ++c) p.v[c] = ldf(d.E[c], base + d.px * vr + gx);
#pragma unroll
    for (int q = 0; q < EPatch<X, Y>::NX; ++q) {
        const int e = min(g * EPatch<X, Y>::NX + q, 5);      // uniform per wave if X = 64
        const int xr = patch_row<X>(d, y0, Y + (e & 1));
        p.x[q] = ldf(comp_ptr(d.E[0], d.cstride, e >> 1), base + d.px * xr + gx);
    }
    const int tt = min(t, EPatch<X, Y>::NHALO - 1);
    const int side = tt & 1, rest = tt >> 1;
    const int c = rest / (Y + 2), row = patch_row<X>(d, y0, rest % (Y + 2));
    p.halo = ldf(comp_ptr(d.E[0], d.cstride, c), base + d.px * row + (side ? X : 0) - (side ? 0 : 1));
}

template <int X, int Y>
__device__ __forceinline__ void epatch_store(Smem<X, Y> &sm, const EPatch<X, Y> &p, int slot, int g,
                                             int gx)
{
    const int t = threadIdx.x, lane = t & (TW - 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) sm.e[slot][c][g][gx + 1] = p.v[c];
#pragma unroll
    for (int q = 0; q < EPatch<X, Y>::NX; ++q) {
        const int e = g * EPatch<X, Y>::NX + q;
        float *dst = e < 6 ? &sm.e[slot][e >> 1][Y + (e & 1)][gx + 1] : &sm.dummy[lane];
        *dst = p.x[q];
    }
    const int side = t & 1, rest = t >> 1;
    const int c = rest / (Y + 2), row = rest % (Y + 2);
    float *dst = t < EPatch<X, Y>::NHALO ? &sm.e[slot][c][row][side ? X + 1 : 0] : &sm.dummy[lane];
    *dst = p.halo;
}

// The packed edge ids of a cell: IDB bits per component (x lowest), in a
// 16-bit word for IDB = 5, a 32-bit word for IDB = 8.
template <int IDB>
using IdWord = typename std::conditional<IDB == 5, uint16_t, uint32_t>::type;

// What plane k of the own cell (and the halo cell of this thread) needs
// from HBM besides the E patch; loaded one plane ahead.
struct PlaneRegs {
    float hx, hy, hz;          // H^{n-1/2} own
    uint32_t ids;              // packed edge ids own
    float hhx, hhy, hhz;       // H^{n-1/2} of the halo cell
    Psi6 ph;                   // H auxiliaries of the own cell (boundary tiles)
};

// Per-thread constants of one tile.
struct TileCtx {
    int x0, y0, z0, z1;
    int g;                     // row group: tile row of the thread (uniform per
                               // wave in 64-wide tiles)
    int i, j, lx, ly;          // own cell and its LDS position
    int ci, cj;                // own cell clamped into the grid (load address)
    int hi_, hj_, hlx, hly;    // halo cell and its LDS position
    int chi, chj;              // halo cell clamped into the grid (load address)
    bool own, halo_thread, halo_live, src_col;
    float sval;                // source value of the output level
    uint32_t sy, sz;           // field strides
};

// Loads for plane k: unconditional (lanes without a cell load a clamped
// one and discard it); only the auxiliaries of boundary tiles depend on the
// lane.
template <bool LAYERS, int IDB>
__device__ __forceinline__ void plane_load(const DevGrid<float> &d, PlaneRegs &r, const TileCtx &t,
                                           int k)
{
    const uint32_t c = (uint32_t)(d.off + t.ci) + t.sy * t.cj + t.sz * k;
    r.hx = ldf(d.H[0], c);
    r.hy = ldf(d.H[1], c);
    r.hz = ldf(d.H[2], c);
    r.ids = (uint32_t)gld(static_cast<const IdWord<IDB> *>(d.ids[0]),
                (uint32_t)(t.ci + d.nx * (t.cj + d.ny * k)));
    const uint32_t h = (uint32_t)(d.off + t.chi) + t.sy * t.chj + t.sz * k;
    r.hhx = ldf(d.H[0], h);
    r.hhy = ldf(d.H[1], h);
    r.hhz = ldf(d.H[2], h);
    if constexpr (LAYERS) {
        if (t.own) load_psi_h(d, layer_pos(d, t.i, t.j, k), r.ph);
    }
}

// Profile value of table `tab` at position p of an axis of length n (the
// tables cover [0, n); positions outside never enter an update).
__device__ __forceinline__ float prof_at(const float *prof, int tab, int n, int p)
{
    return (p >= 0 && p < n) ? gld(prof, (uint32_t)(tab * n + p)) : 0.f;
}

// Rotating state of the march through the planes.
struct MarchState {
    int s0, s1, s2;            // LDS slots of E^n planes k, k+1, k+2
    float hx_prev, hy_prev;    // H^{n+1/2}(k-1) of the own cell
};

// One plane k (< z1) of the march.  `cur` holds what plane k needs from
// HBM (loaded during plane k-1); `nxt` receives what plane k+1 needs.  The
// caller alternates the two register sets instead of copying them: a copy
// would have to wait for the loads in flight.  Past the end of the chunk
// the prefetches repeat the last plane (cache hits, results unused).
template <int X, int Y, bool LAYERS, int IDB, bool NT>
__device__ __forceinline__ void march_plane(const DevGrid<float> &d, Smem<X, Y> &sm,
                                            const Tabs<X, Y> &tb, const TileCtx &t, int k,
                                            const PlaneRegs &cur, PlaneRegs &nxt, MarchState &m)
{
    const int lx = t.lx, ly = t.ly, hlx = t.hlx, hly = t.hly, lane = threadIdx.x & (TW - 1);
    const int s0 = m.s0, s1 = m.s1, s2 = m.s2;
    const int lz = k - t.z0 + 1;
    // ---- requests: this plane's auxiliaries (boundary tiles), then
    //      everything plane k+1 needs (consumed one plane later) -------------
    LayerPos L{}, Lh{};
    Psi6 pe_cur{}, ph_halo{};
    if constexpr (LAYERS) {
        L = layer_pos(d, t.i, t.j, k);
        if (t.own) load_psi_e(d, L, pe_cur);
        if (t.halo_live) {
            Lh = layer_pos(d, t.hi_, t.hj_, k);
            load_psi_h(d, Lh, ph_halo);
        }
    }
    EPatch<X, Y> pe;
    epatch_load<X, Y>(d, pe, t.x0, t.y0, min(k + 2, t.z1), t.g, lx - 1);
    plane_load<LAYERS, IDB>(d, nxt, t, min(k + 1, t.z1 - 1));

    // lanes without a cell store into the sink
    const uint32_t c = t.own ? (uint32_t)(d.off + t.i) + t.sy * t.j + t.sz * k
                             : (uint32_t)d.sink + (uint32_t)lane;
    // ---- H^{n+1/2}(k): own cell -------------------------------------------
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
        if (!LAYERS || t.own)
            h_apply<X, Y, LAYERS>(d, tb, L, lx, ly, lz, df, cur.ph, true, cur.hx, cur.hy, cur.hz,
                               ox, oy, oz);
        field_st<NT>(d.Ho[0], c, ox);
        field_st<NT>(d.Ho[1], c, oy);
        field_st<NT>(d.Ho[2], c, oz);
        sm.h[0][ly][lx] = t.own ? ox : 0.f;
        sm.h[1][ly][lx] = t.own ? oy : 0.f;
        sm.h[2][ly][lx] = t.own ? oz : 0.f;
    }
    // ---- H^{n+1/2}(k): halo row y0-1 and halo column x0-1 -----------------
    {
        HDiff df;
        const float ex = sm.e[s0][0][hly][hlx], ey = sm.e[s0][1][hly][hlx],
                    ez = sm.e[s0][2][hly][hlx];
        df.ez_y = sm.e[s0][2][hly + 1][hlx] - ez;
        df.ey_z = sm.e[s1][1][hly][hlx] - ey;
        df.ex_z = sm.e[s1][0][hly][hlx] - ex;
        df.ez_x = sm.e[s0][2][hly][hlx + 1] - ez;
        df.ey_x = sm.e[s0][1][hly][hlx + 1] - ey;
        df.ex_y = sm.e[s0][0][hly + 1][hlx] - ex;
        float ox, oy, oz;
        h_apply<X, Y, LAYERS>(d, tb, Lh, hlx, hly, lz, df, ph_halo, false, cur.hhx, cur.hhy,
                           cur.hhz, ox, oy, oz);
        // halo cells outside the grid only feed PEC edges: keep them zero
        const bool live = t.halo_live;
        float *hx = t.halo_thread ? &sm.h[0][hly][hlx] : &sm.dummy[lane];
        float *hy = t.halo_thread ? &sm.h[1][hly][hlx] : &sm.dummy[lane];
        float *hz = t.halo_thread ? &sm.h[2][hly][hlx] : &sm.dummy[lane];
        *hx = live ? ox : 0.f;
        *hy = live ? oy : 0.f;
        *hz = live ? oz : 0.f;
    }
    lds_barrier();

    // ---- E^{n+1}(k): own cell ---------------------------------------------
    {
        const float hx = sm.h[0][ly][lx], hy = sm.h[1][ly][lx], hz = sm.h[2][ly][lx];
        float dHz_y = hz - sm.h[2][ly - 1][lx];
        float dHy_z = hy - m.hy_prev;
        float dHx_z = hx - m.hx_prev;
        float dHz_x = hz - sm.h[2][ly][lx - 1];
        float dHy_x = hy - sm.h[1][ly][lx - 1];
        float dHx_y = hx - sm.h[0][ly - 1][lx];
        if constexpr (LAYERS) {
            if (t.own) {
                float pn;
                if (L.inx) {
                    const float b = tb.prx(PR_BE, lx), cc = tb.prx(PR_CE, lx), ik = tb.prx(PR_KE, lx);
                    dHz_x = lterm(dHz_x, b, cc, ik, pe_cur.v[PSI_EYX - 6], pn);
                    stf(d.psi_o[PSI_EYX], L.qx, pn);
                    dHy_x = lterm(dHy_x, b, cc, ik, pe_cur.v[PSI_EZX - 6], pn);
                    stf(d.psi_o[PSI_EZX], L.qx, pn);
                }
                if (L.iny) {
                    const float b = tb.pry(PR_BE, ly), cc = tb.pry(PR_CE, ly), ik = tb.pry(PR_KE, ly);
                    dHz_y = lterm(dHz_y, b, cc, ik, pe_cur.v[PSI_EXY - 6], pn);
                    stf(d.psi_o[PSI_EXY], L.qy, pn);
                    dHx_y = lterm(dHx_y, b, cc, ik, pe_cur.v[PSI_EZY - 6], pn);
                    stf(d.psi_o[PSI_EZY], L.qy, pn);
                }
                if (L.inz) {
                    const float b = tb.prz(PR_BE, lz), cc = tb.prz(PR_CE, lz), ik = tb.prz(PR_KE, lz);
                    dHy_z = lterm(dHy_z, b, cc, ik, pe_cur.v[PSI_EXZ - 6], pn);
                    stf(d.psi_o[PSI_EXZ], L.qz, pn);
                    dHx_z = lterm(dHx_z, b, cc, ik, pe_cur.v[PSI_EYZ - 6], pn);
                    stf(d.psi_o[PSI_EYZ], L.qz, pn);
                }
            }
        }
        constexpr uint32_t IDM = (1u << IDB) - 1u;
        const float4 cx = tb.coef(0, cur.ids & IDM);
        const float4 cy = tb.coef(1, (cur.ids >> IDB) & IDM);
        const float4 cz = tb.coef(2, (cur.ids >> (2 * IDB)) & IDM);
        const float ex = e_upd(sm.e[s0][0][ly][lx], cx, dHz_y, dHy_z);
        const float ey = e_upd(sm.e[s0][1][ly][lx], cy, dHx_z, dHz_x);
        float ez = e_upd(sm.e[s0][2][ly][lx], cz, dHy_x, dHx_y);
        if (t.src_col && k >= d.src_box[4] && k <= d.src_box[5]) ez += t.sval;
        field_st<NT>(d.Eo[0], c, ex);
        field_st<NT>(d.Eo[1], c, ey);
        field_st<NT>(d.Eo[2], c, ez);
        m.hx_prev = hx;
        m.hy_prev = hy;
    }
    // ---- rotate: plane k+2 into the LDS slot plane k leaves ----------------
    epatch_store<X, Y>(sm, pe, s2, t.g, lx - 1);
    m.s0 = s1;
    m.s1 = s2;
    m.s2 = s0;
    lds_barrier();
}

// The tile of X by Y cells at (x0, y0), z-chunk tz.
template <int X, int Y, bool LAYERS, int IDB, bool NT>
__device__ void fused_tile(const DevGrid<float> &d, int x0, int y0, int tz, int zchunk,
                           int64_t level, Smem<X, Y> &sm, const Tabs<X, Y> &tb)
{
    constexpr int NTH = X * Y;  // threads of the block
    TileCtx tc;
    tc.x0 = x0;
    tc.y0 = y0;
    tc.z0 = tz * zchunk;
    tc.z1 = min(tc.z0 + zchunk, d.nz);
    const int z0 = tc.z0;
    const int t = threadIdx.x;
    const int col = t % X, row = t / X;
    tc.g = X == TW ? __builtin_amdgcn_readfirstlane(row) : row;
    const int i = x0 + col, j = y0 + row;
    tc.i = i;
    tc.j = j;
    tc.ci = min(i, d.nx - 1);
    tc.cj = min(j, d.ny - 1);
    tc.own = i < d.nx && j < d.ny;
    tc.sy = (uint32_t)d.px;
    tc.sz = (uint32_t)(d.px * d.py);
    tc.lx = col + 1;
    tc.ly = row + 1;
    const int lx = tc.lx, ly = tc.ly;

    // the halo cell this thread recomputes H for: the low-y row, then the
    // low-x column; the other threads repeat the last one (writing to a
    // dummy LDS row) so that the halo work has no branch either
    const int nh = X + Y + 1;
    const int th = min(t, nh - 1);
    const int hi_ = th < X ? x0 + th : x0 - 1;
    const int hj_ = th < X ? y0 - 1 : y0 - 1 + (th - X);
    tc.halo_thread = t < nh;
    // only halo cells inside the grid matter: the others feed PEC edges only
    tc.halo_live = hi_ >= 0 && hj_ >= 0 && hi_ < d.nx && hj_ < d.ny;
    tc.hi_ = hi_;
    tc.hj_ = hj_;
    tc.chi = max(min(hi_, d.nx - 1), 0);
    tc.chj = max(min(hj_, d.ny - 1), 0);
    tc.hlx = hi_ - x0 + 1;
    tc.hly = hj_ - y0 + 1;

    // ---- block caches: LUTs (and the layer profiles of boundary tiles) ------
    const int nlut = d.nlut;
    for (int q = t; q < 3 * nlut; q += NTH) {
        const int c = q / nlut, e = q % nlut;
        tb.lut[c * tb.cap + e] = lut_entry(c == 0 ? d.lut[0] : (c == 1 ? d.lut[1] : d.lut[2]), e);
    }
    if constexpr (LAYERS) {
        for (int q = t; q < PR_COUNT * (X + 2); q += NTH) {
            const int tab = q / (X + 2), p = q % (X + 2);
            tb.px[q] = prof_at(d.prof[0], tab, d.nx, x0 - 1 + p);
        }
        for (int q = t; q < PR_COUNT * (Y + 2); q += NTH) {
            const int tab = q / (Y + 2), p = q % (Y + 2);
            tb.py[q] = prof_at(d.prof[1], tab, d.ny, y0 - 1 + p);
        }
        for (int q = t; q < PR_COUNT * (ZMAX + 1); q += NTH) {
            const int tab = q / (ZMAX + 1), p = q % (ZMAX + 1);
            tb.pz[q] = prof_at(d.prof[2], tab, d.nz, z0 - 1 + p);
        }
    }

    // ---- prologue: request everything the first plane needs at once -------
    EPatch<X, Y> pa, pb;
    epatch_load<X, Y>(d, pa, x0, y0, z0, tc.g, col);
    epatch_load<X, Y>(d, pb, x0, y0, z0 + 1, tc.g, col);
    PlaneRegs ra{}, rb{};
    plane_load<LAYERS, IDB>(d, ra, tc, z0);
    // inputs of H^{n+1/2}(z0-1) at the own cell, needed by E(z0); on the
    // bottom face the E edges it feeds are PEC, so it is not needed there
    const bool pro = z0 > 0;
    HDiff pdf{};
    float phx = 0.f, phy = 0.f, phz = 0.f;
    Psi6 pps{};
    LayerPos pL{};
    if (pro) {
        const uint32_t c = (uint32_t)(d.off + tc.ci) + tc.sy * tc.cj + tc.sz * (z0 - 1);
        const float ex = ldf(d.E[0], c), ey = ldf(d.E[1], c), ez = ldf(d.E[2], c);
        pdf.ez_y = ldf(d.E[2], c + tc.sy) - ez;
        pdf.ey_z = ldf(d.E[1], c + tc.sz) - ey;
        pdf.ex_z = ldf(d.E[0], c + tc.sz) - ex;
        pdf.ez_x = ldf(d.E[2], c + 1) - ez;
        pdf.ey_x = ldf(d.E[1], c + 1) - ey;
        pdf.ex_y = ldf(d.E[0], c + tc.sy) - ex;
        phx = ldf(d.H[0], c);
        phy = ldf(d.H[1], c);
        phz = ldf(d.H[2], c);
        if constexpr (LAYERS) {
            if (tc.own) {
                pL = layer_pos(d, i, j, z0 - 1);
                load_psi_h(d, pL, pps);
            }
        }
    }
    tc.sval = 0.f;
    tc.src_col = d.src_kind != 0 && tc.own && i >= d.src_box[0] && i <= d.src_box[1] &&
                 j >= d.src_box[2] && j <= d.src_box[3];
    if (tc.src_col) tc.sval = (float)source_at(d, level + 1);
    lds_barrier();   // caches visible

    MarchState m;
    m.hx_prev = 0.f;
    m.hy_prev = 0.f;
    if (pro) {
        float oz;
        h_apply<X, Y, LAYERS>(d, tb, pL, lx, ly, 0, pdf, pps, false, phx, phy, phz, m.hx_prev,
                           m.hy_prev, oz);
    }
    epatch_store<X, Y>(sm, pa, 0, tc.g, col);
    epatch_store<X, Y>(sm, pb, 1, tc.g, col);
    lds_barrier();

    m.s0 = 0;
    m.s1 = 1;
    m.s2 = 2;
    // two planes per iteration with the register sets swapping roles; an
    // odd last plane runs after the loop
    int k = z0;
    for (; k + 1 < tc.z1; k += 2) {
        march_plane<X, Y, LAYERS, IDB, NT>(d, sm, tb, tc, k, ra, rb, m);
        march_plane<X, Y, LAYERS, IDB, NT>(d, sm, tb, tc, k + 1, rb, ra, m);
    }
    if (k < tc.z1) march_plane<X, Y, LAYERS, IDB, NT>(d, sm, tb, tc, k, ra, rb, m);
}

// Tile of block b of n.  Block b is dispatched to XCD b % 8.  Order 0: each
// XCD gets one contiguous run of tiles, so neighbouring tiles share its L2.
// Order k >= 1: runs of k tiles are dealt to the XCDs in turn; blocks past
// the last whole round of 8k take the tile of their own index.
__device__ __forceinline__ int xcd_tile(int b, int n, int order)
{
    const int xcd = b & 7, idx = b >> 3;
    if (order == 0) {
        const int q = n >> 3, r = n & 7;
        return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + idx;
    }
    const int whole = n / (8 * order) * (8 * order);
    return b >= whole ? b : ((idx / order) * 8 + xcd) * order + idx % order;
}

// Tile q of the interior box, x fastest.
__device__ __forceinline__ void interior_tile(const TileSet &s, int q, int &tx, int &ty, int &tz)
{
    const int nx = s.ix1 - s.ix0, ny = s.iy1 - s.iy0;
    tx = s.ix0 + q % nx;
    ty = s.iy0 + (q / nx) % ny;
    tz = s.iz0 + q / (nx * ny);
}

// Tile q of the complement of the interior box among the 64-wide tiles:
// whole xy-planes of tiles outside [iz0, iz1) first, then whole x-rows
// outside [iy0, iy1) of the planes inside, then the tiles outside [ix0, ix1)
// of the rows inside.  (The narrow tiles of a ragged last column are
// interleaved with these in the boundary launch.)
__device__ __forceinline__ void boundary_tile(const TileSet &s, int q, int &tx, int &ty, int &tz)
{
    const int nix = s.ix1 - s.ix0, niy = s.iy1 - s.iy0, niz = s.iz1 - s.iz0;
    const int plane = s.tx * s.ty;
    const int a = (s.tz - niz) * plane;
    if (q < a) {
        const int z = q / plane, r = q % plane;
        tz = z < s.iz0 ? z : z + niz;
        ty = r / s.tx;
        tx = r % s.tx;
        return;
    }
    q -= a;
    const int rows = (s.ty - niy) * s.tx;
    const int b = niz * rows;
    if (q < b) {
        const int z = q / rows, r = q % rows;
        const int y = r / s.tx;
        tz = s.iz0 + z;
        ty = y < s.iy0 ? y : y + niy;
        tx = r % s.tx;
        return;
    }
    q -= b;
    const int cols = s.tx - nix;
    const int z = q / (niy * cols), r = q % (niy * cols);
    const int x = r % cols;
    tz = s.iz0 + z;
    ty = s.iy0 + r / cols;
    tx = x < s.ix0 ? x : x + nix;
}

// One launch of one tile class for every instance in the table.  In the
// boundary launch the first `nprobe_blocks` blocks sample the probes of the
// input level (so sampling overlaps the update instead of costing a launch
// of its own).
// Occupancy targets: boundary kernels of 8 or more rows need just over 128
// VGPRs, one more wave per SIMD than they would get (3 -> 4) is worth the
// few registers spilled; interior kernels hold 6 waves.
template <int R, bool LAYERS>
constexpr int min_waves() { return LAYERS ? (R >= 8 ? 4 : 1) : (R >= 4 ? 6 : 1); }

template <int R, bool LAYERS, int IDB, bool NT>
__global__ void __launch_bounds__(TW *R)
__attribute__((amdgpu_waves_per_eu(min_waves<R, LAYERS>(), 8)))
k_fused(const DevGrid<float> *__restrict__ grids, const TileSet *__restrict__ sets, int ninst,
        int zchunk, int ntiles, int64_t level, const DevProbes *__restrict__ probes,
        int nprobe_blocks, int max_probes, int lut_cap, int order)
{
    constexpr int YN = TW * R / NW;   // rows of a narrow tile
    using SmW = Smem<TW, R>;
    using SmN = Smem<NW, YN>;
    constexpr size_t SMB = LAYERS && sizeof(SmN) > sizeof(SmW) ? sizeof(SmN) : sizeof(SmW);
    __shared__ __attribute__((aligned(16))) char smraw[SMB];
    extern __shared__ float4 dyn_lds[];
    const int b = blockIdx.x;
    if (b < nprobe_blocks) {
        const int inst = b / max_probes, q = b % max_probes;
        if (q < probes[inst].nprobe)
            probe_one(grids[inst], probes[inst], q, level, reinterpret_cast<double *>(smraw));
        return;
    }
    const int tl = xcd_tile(b - nprobe_blocks, ntiles, order);
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {          // last instance whose first block <= tl
        const int mid = (lo + hi + 1) >> 1;
        if ((LAYERS ? sets[mid].sb : sets[mid].si) <= tl) lo = mid;
        else hi = mid - 1;
    }
    const TileSet s = sets[lo];
    int tx, ty, tz;
    if constexpr (LAYERS) {
        // the narrow tiles sit at every st-th position of the grid's range,
        // spread over all XCDs
        int q = tl - s.sb;
        const int nn = s.nxw * s.nty * s.tz;
        const int st = nn > 0 ? s.nb / nn : 1;
        const int before = min(q / st + 1, nn);         // narrow positions <= q
        if (nn > 0 && q % st == 0 && q / st < nn) {
            const int n = q / st, sub = n % s.nxw, rest = n / s.nxw;
            Tabs<NW, YN> tb;
            tb.place(dyn_lds, lut_cap);
            fused_tile<NW, YN, true, IDB, NT>(grids[lo], s.tx * TW + sub * NW, (rest % s.nty) * YN,
                                          rest / s.nty, zchunk, level,
                                          *reinterpret_cast<SmN *>(smraw), tb);
            return;
        }
        boundary_tile(s, nn > 0 ? q - before : q, tx, ty, tz);
    } else {
        interior_tile(s, tl - s.si, tx, ty, tz);
    }
    Tabs<TW, R> tb;
    tb.place(dyn_lds, lut_cap);
    fused_tile<TW, R, LAYERS, IDB, NT>(grids[lo], tx * TW, ty * R, tz, zchunk, level,
                                   *reinterpret_cast<SmW *>(smraw), tb);
}

template <int R, bool LAYERS, int IDB, bool NT>
hipError_t launch_r(const DevGrid<float> *g, const TileSet *sets, int ninst, int ntiles,
                    int zchunk, int64_t level, const DevProbes *probes, int nprobe_blocks,
                    int max_probes, int lut_cap, int order, hipStream_t s)
{
    k_fused<R, LAYERS, IDB, NT><<<ntiles + nprobe_blocks, TW * R, tabs_bytes<R>(lut_cap, LAYERS), s>>>(
        g, sets, ninst, zchunk, ntiles, level, probes, nprobe_blocks, max_probes, lut_cap, order);
    return hipGetLastError();
}

template <bool LAYERS, int IDB, bool NT>
hipError_t launch_class(const DevGrid<float> *g, const TileSet *sets, int ninst, int ntiles,
                        const LaunchCfg &cfg, int64_t level, const DevProbes *probes, int npb,
                        int max_probes, int lut_cap, hipStream_t s)
{
    switch (cfg.rows) {
    case 2: return launch_r<2, LAYERS, IDB, NT>(g, sets, ninst, ntiles, cfg.zchunk, level, probes, npb, max_probes, lut_cap, cfg.order, s);
    case 4: return launch_r<4, LAYERS, IDB, NT>(g, sets, ninst, ntiles, cfg.zchunk, level, probes, npb, max_probes, lut_cap, cfg.order, s);
    case 8: return launch_r<8, LAYERS, IDB, NT>(g, sets, ninst, ntiles, cfg.zchunk, level, probes, npb, max_probes, lut_cap, cfg.order, s);
    case 12: return launch_r<12, LAYERS, IDB, NT>(g, sets, ninst, ntiles, cfg.zchunk, level, probes, npb, max_probes, lut_cap, cfg.order, s);
    case 16: return launch_r<16, LAYERS, IDB, NT>(g, sets, ninst, ntiles, cfg.zchunk, level, probes, npb, max_probes, lut_cap, cfg.order, s);
    default: return hipErrorInvalidValue;
    }
}


// ---------------------------------------------------------------------------
// Two-level (temporally blocked) pass over the interior tiles
// ---------------------------------------------------------------------------
// A block of 64 x (R+3) threads owns a tile of TB_W = 60 x R cells and
// marches through a z-chunk, taking the fields from level n (E^n,
// H^{n-1/2}) to level n+2 (E^{n+2}, H^{n+3/2}) in one pass: HBM sees the
// level-n inputs read once and the level-n+2 outputs written once.  Thread
// (lane, w) owns the column x = x0-2+lane, y = y0-2+w, so that a wavefront
// covers one row of the tile plus two halo cells on each side.  Level n+1
// is recomputed on the halo the second level needs (never exchanged between
// blocks) and lives in registers and LDS only, except on the one-cell rim
// of the two-level box and in tiles that hold probe terms, where it is also
// written out for the single-level passes of the other tiles and the probes.
//
// At march position m the block computes H^{n+1/2}(m) and E^{n+1}(m), then
// H^{n+3/2}(m-1) and E^{n+2}(m-1): the second level trails by a plane, since
// H^{n+3/2}(m-1) needs E^{n+1}(m).  The values are right on these regions
// (the other lanes compute values nothing uses):
//   H^{n+1/2}:  x0-2 .. x0+60, y0-2 .. y0+R      lanes 0..62, waves 0..R+2
//   E^{n+1}:    x0-1 .. x0+60, y0-1 .. y0+R      lanes 1..62, waves 1..R+2
//   H^{n+3/2}:  x0-1 .. x0+59, y0-1 .. y0+R-1    lanes 1..61, waves 1..R+1
//   E^{n+2}:    x0   .. x0+59, y0   .. y0+R-1    lanes 2..61, waves 2..R+1
// E^n is needed on x0-2 .. x0+61, y0-2 .. y0+R+1: each thread loads its own
// column, the first three waves the extra row y0+R+1 (one component each).
// Update formulas and their rounding are those of the single-level kernel
// (h_upd, e_upd): a two-level pass gives the bits of two single steps.
template <int R>
struct TBSmem {
    // Only the y neighbours go through LDS (x neighbours are lanes of the
    // same wavefront), and only the two components each difference needs.
    // E^n and E^{n+1} alternate between two slots, so each march position
    // needs two block barriers.
    float e0[2][2][R + 4][TW];   // Ex, Ez of E^n(m), rows y0-2 .. y0+R+1
    float h1[2][R + 3][TW];      // Hx, Hz of H^{n+1/2}(m)
    float e1[2][2][R + 3][TW];   // Ex, Ez of E^{n+1}(m-1)
    float h2[2][R + 3][TW];      // Hx, Hz of H^{n+3/2}(m-1)
    float dummy[TW];             // target of the extra-row stores of waves >= 2
};

// Value of the lane one to the right (x + 1) / left (x - 1) in the
// wavefront (the lanes at the ends get values nothing uses).
__device__ __forceinline__ float lane_next(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_prev(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}

// Loads of one march position, issued a position ahead.
struct TBRegs {
    float e[3];                // E^n(m+1), own column
    float ex;                  // E^n(m+1) on the extra row (Ex in wave 0, Ez in the others)
    float h[3];                // H^{n-1/2}(m), own column
    uint32_t id;               // packed edge ids of plane m
};

// Values carried from one march position to the next.
struct TBState {
    float e0[3];               // E^n(m)
    float h1p[3];              // H^{n+1/2}(m-1)
    float e1p[3];              // E^{n+1}(m-1)
    float h2p[2];              // Hx, Hy of H^{n+3/2}(m-2)
    uint32_t idp;              // ids of plane m-1
};

struct TBCtx {
    int lane, w;
    int x, y;                  // column of the thread
    int z0, z1;                // the tile's chunk
    int zlast;                 // last plane of E^n the pass reads (z1 + 1)
    uint32_t col;              // field index of (x, y) clamped into storage, plane 0
    uint32_t xcol;             // same for the extra-row load
    uint32_t idcol;            // id index of (x, y) clamped into the grid, plane 0
    uint32_t sz;               // plane stride
    int exc;                   // component of the extra-row load (0 or 2)
    bool own;                  // (x, y) is a cell of the tile and of the box
    bool rim_xy;               // ... on the box's x or y rim
    bool all;                  // the tile holds probe terms
    bool src_col;
    int sk0, sk1;              // source planes (empty range without a source)
    int bz0, bz1;              // the box's z range
    float sval1, sval2;        // source values of levels n+1 and n+2
};

// What the march needs of the grid descriptor, kept in registers: the
// first component of each field (the others follow at cstride bytes).
struct TBPtr {
    const float *E, *H;        // level n
    float *Eo, *Ho;            // level n+2
    float *Em, *Hm;            // level n+1 (rim and probe tiles)
    const void *ids;
    int64_t cstride;
    uint32_t sink;
    uint32_t idplane;          // nx * ny
    float ch[3];
};

__device__ __forceinline__ float *comp_out(float *c0, int64_t stride, int c)
{
    return reinterpret_cast<float *>(reinterpret_cast<char *>(c0) + c * stride);
}

template <int R, int IDB>
__device__ __forceinline__ void tb_load(const TBPtr &d, TBRegs &r, const TBCtx &t, int ke, int kh)
{
    const uint32_t pe = t.sz * (uint32_t)ke, ph = t.sz * (uint32_t)kh;
    r.e[0] = ldf(d.E, t.col + pe);
    r.e[1] = ldf(comp_ptr(d.E, d.cstride, 1), t.col + pe);
    r.e[2] = ldf(comp_ptr(d.E, d.cstride, 2), t.col + pe);
    r.ex = ldf(comp_ptr(d.E, d.cstride, t.exc), t.xcol + pe);
    r.h[0] = ldf(d.H, t.col + ph);
    r.h[1] = ldf(comp_ptr(d.H, d.cstride, 1), t.col + ph);
    r.h[2] = ldf(comp_ptr(d.H, d.cstride, 2), t.col + ph);
    r.id = (uint32_t)gld(static_cast<const IdWord<IDB> *>(d.ids), t.idcol + d.idplane * (uint32_t)kh);
}

// Ex, Ez of E^n(k) of the own column and the extra row into LDS slot q.
template <int R>
__device__ __forceinline__ void tb_store_e0(TBSmem<R> &sm, const TBCtx &t, int q, const float *e,
                                            float ex)
{
    sm.e0[q][0][t.w][t.lane] = e[0];
    sm.e0[q][1][t.w][t.lane] = e[2];
    float *dst = t.w < 2 ? &sm.e0[q][t.w][R + 3][t.lane] : &sm.dummy[t.lane];
    *dst = ex;
}

// One march position m (see the comment above k_tb).  No branch inside:
// every phase runs at every position, and a store that does not apply (a
// lane without an own cell, a plane outside the chunk, the positions before
// the second level starts) goes to the sink, so the compiler's wait counts
// follow the straight-line order of the loads.  RIM: the tile writes level
// n+1 of its rim cells (or, in a probe tile, of all its cells).
template <int R, int IDB, bool NT, bool RIM>
__device__ __forceinline__ void tb_plane(const TBPtr &d, TBSmem<R> &sm, const float4 *lut, int cap,
                                         const TBCtx &t, int m, int q, const TBRegs &cur,
                                         TBRegs &nxt, TBState &st)
{
    const int lane = t.lane, w = t.w;
    const int ym = max(w - 1, 0), yp = min(w + 1, R + 2);
    const uint32_t sink = d.sink + (uint32_t)lane;
    // ---- requests for position m+1 (consumed one position later) ----------
    tb_load<R, IDB>(d, nxt, t, min(m + 2, t.zlast), min(m + 1, t.z1));

    // ---- H^{n+1/2}(m) ------------------------------------------------------
    const float ex = st.e0[0], ey = st.e0[1], ez = st.e0[2];
    const float ezx = lane_next(ez), eyx = lane_next(ey);
    const float h1x = h_upd(cur.h[0], d.ch[1], sm.e0[q][1][w + 1][lane] - ez, d.ch[2], cur.e[1] - ey);
    const float h1y = h_upd(cur.h[1], d.ch[2], cur.e[0] - ex, d.ch[0], ezx - ez);
    const float h1z = h_upd(cur.h[2], d.ch[0], eyx - ey, d.ch[1], sm.e0[q][0][w + 1][lane] - ex);
    sm.h1[0][w][lane] = h1x;
    sm.h1[1][w][lane] = h1z;
    lds_barrier();

    // ---- E^{n+1}(m) --------------------------------------------------------
    constexpr uint32_t IDM = (1u << IDB) - 1u;
    float e1x, e1y, e1z;
    {
        const float h1zx = lane_prev(h1z), h1yx = lane_prev(h1y);
        const float dHz_y = h1z - sm.h1[1][ym][lane];
        const float dHy_z = h1y - st.h1p[1];
        const float dHx_z = h1x - st.h1p[0];
        const float dHz_x = h1z - h1zx;
        const float dHy_x = h1y - h1yx;
        const float dHx_y = h1x - sm.h1[0][ym][lane];
        const float4 cx = lut[cur.id & IDM];
        const float4 cy = lut[cap + ((cur.id >> IDB) & IDM)];
        const float4 cz = lut[2 * cap + ((cur.id >> (2 * IDB)) & IDM)];
        e1x = e_upd(ex, cx, dHz_y, dHy_z);
        e1y = e_upd(ey, cy, dHx_z, dHz_x);
        e1z = e_upd(ez, cz, dHy_x, dHx_y);
        // (sval1 is zero off the source columns)
        if (m >= t.sk0 && m <= t.sk1) e1z += t.sval1;
    }
    // E^{n+1}(m) and E^n(m+1) into the other slots, for position m+1 (the
    // barrier after the next H update orders them)
    sm.e1[1 - q][0][w][lane] = e1x;
    sm.e1[1 - q][1][w][lane] = e1z;
    tb_store_e0<R>(sm, t, 1 - q, cur.e, cur.ex);
    if constexpr (RIM) {
        // level n+1 of the rim (read by the single-level passes of the
        // neighbouring tiles) and of probe tiles (read by the probes)
        const bool on = t.own && m >= t.z0 && m < t.z1 &&
                        (t.all || t.rim_xy || m == t.bz0 || m == t.bz1 - 1);
        const uint32_t c = on ? t.col + t.sz * (uint32_t)m : sink;
        stf(d.Em, c, e1x);
        stf(comp_out(d.Em, d.cstride, 1), c, e1y);
        stf(comp_out(d.Em, d.cstride, 2), c, e1z);
        stf(d.Hm, c, h1x);
        stf(comp_out(d.Hm, d.cstride, 1), c, h1y);
        stf(comp_out(d.Hm, d.cstride, 2), c, h1z);
    }

    // ---- H^{n+3/2}(m-1) ----------------------------------------------------
    // (at m = 0, only in the bottom chunk of a grid without a lower layer,
    // this is H^{n+3/2}(-1) below the grid: zero, it feeds only the
    // tangential E edges of the ground face)
    const bool below = m == 0;
    const float e1pzx = lane_next(st.e1p[2]), e1pyx = lane_next(st.e1p[1]);
    float h2x = h_upd(st.h1p[0], d.ch[1], sm.e1[q][1][yp][lane] - st.e1p[2], d.ch[2], e1y - st.e1p[1]);
    float h2y = h_upd(st.h1p[1], d.ch[2], e1x - st.e1p[0], d.ch[0], e1pzx - st.e1p[2]);
    float h2z = h_upd(st.h1p[2], d.ch[0], e1pyx - st.e1p[1], d.ch[1], sm.e1[q][0][yp][lane] - st.e1p[0]);
    h2x = below ? 0.f : h2x;
    h2y = below ? 0.f : h2y;
    h2z = below ? 0.f : h2z;
    sm.h2[0][w][lane] = h2x;
    sm.h2[1][w][lane] = h2z;
    // the second level's outputs: planes z0 .. z1-1
    const uint32_t co = (t.own && m - 1 >= t.z0) ? t.col + t.sz * (uint32_t)(m - 1) : sink;
    field_st<NT>(d.Ho, co, h2x);
    field_st<NT>(comp_out(d.Ho, d.cstride, 1), co, h2y);
    field_st<NT>(comp_out(d.Ho, d.cstride, 2), co, h2z);
    lds_barrier();

    // ---- E^{n+2}(m-1) ------------------------------------------------------
    {
        const float h2zx = lane_prev(h2z), h2yx = lane_prev(h2y);
        const float dHz_y = h2z - sm.h2[1][ym][lane];
        const float dHy_z = h2y - st.h2p[1];
        const float dHx_z = h2x - st.h2p[0];
        const float dHz_x = h2z - h2zx;
        const float dHy_x = h2y - h2yx;
        const float dHx_y = h2x - sm.h2[0][ym][lane];
        const float4 cx = lut[st.idp & IDM];
        const float4 cy = lut[cap + ((st.idp >> IDB) & IDM)];
        const float4 cz = lut[2 * cap + ((st.idp >> (2 * IDB)) & IDM)];
        const float e2x = e_upd(st.e1p[0], cx, dHz_y, dHy_z);
        const float e2y = e_upd(st.e1p[1], cy, dHx_z, dHz_x);
        float e2z = e_upd(st.e1p[2], cz, dHy_x, dHx_y);
        if (m - 1 >= t.sk0 && m - 1 <= t.sk1) e2z += t.sval2;
        field_st<NT>(d.Eo, co, e2x);
        field_st<NT>(comp_out(d.Eo, d.cstride, 1), co, e2y);
        field_st<NT>(comp_out(d.Eo, d.cstride, 2), co, e2z);
    }
    st.h2p[0] = h2x;
    st.h2p[1] = h2y;
    st.e0[0] = cur.e[0];
    st.e0[1] = cur.e[1];
    st.e0[2] = cur.e[2];
    st.h1p[0] = h1x;
    st.h1p[1] = h1y;
    st.h1p[2] = h1z;
    st.e1p[0] = e1x;
    st.e1p[1] = e1y;
    st.e1p[2] = e1z;
    st.idp = cur.id;
}

// The march of one tile from its first position to z1.
template <int R, int IDB, bool NT, bool RIM>
__device__ __forceinline__ void tb_march(const TBPtr &d, TBSmem<R> &sm, const float4 *lut, int cap,
                                         const TBCtx &t, int mfirst, TBRegs &ra, TBRegs &rb,
                                         TBState &st)
{
    int m = mfirst;
    for (; m + 1 <= t.z1; m += 2) {
        tb_plane<R, IDB, NT, RIM>(d, sm, lut, cap, t, m, 0, ra, rb, st);
        tb_plane<R, IDB, NT, RIM>(d, sm, lut, cap, t, m + 1, 1, rb, ra, st);
    }
    if (m <= t.z1) tb_plane<R, IDB, NT, RIM>(d, sm, lut, cap, t, m, 0, ra, rb, st);
}

// Occupancy: two blocks of 11 waves (8 rows) per CU need 6 waves per SIMD
// (at most 80 VGPRs), two of 13 (10 rows) 7 (72 VGPRs); a block of 16 waves
// (13 rows) fills 4.
template <int R>
constexpr int tb_min_waves() { return R >= 13 ? 4 : (R >= 10 ? 7 : 6); }

template <int R, int IDB, bool NT>
__global__ void __launch_bounds__(TW *(R + 3))
__attribute__((amdgpu_waves_per_eu(tb_min_waves<R>(), 8)))
k_tb(const DevGrid<float> *__restrict__ grid, const TBSet *__restrict__ set, int64_t level,
     int lut_cap, int order)
{
    __shared__ __attribute__((aligned(16))) TBSmem<R> sm;
    extern __shared__ float4 dyn_lds[];
    const DevGrid<float> &d = *grid;
    const TBSet s = *set;
    // what the march reads of the descriptor, in registers: its fields are
    // then not reloaded after each store of the march
    TBPtr g;
    g.E = d.E[0];
    g.H = d.H[0];
    g.Eo = d.Eo[0];
    g.Ho = d.Ho[0];
    g.Em = d.Em[0];
    g.Hm = d.Hm[0];
    g.ids = d.ids[0];
    g.cstride = d.cstride;
    g.sink = (uint32_t)d.sink;
    g.idplane = (uint32_t)(d.nx * d.ny);
    g.ch[0] = d.ch[0];
    g.ch[1] = d.ch[1];
    g.ch[2] = d.ch[2];
    const int tl = xcd_tile(blockIdx.x, s.n, order);
    const int tx = tl % s.ntx, ty = (tl / s.ntx) % s.nty, tz = tl / (s.ntx * s.nty);
    const int x0 = s.x0 + tx * TB_W, y0 = s.y0 + ty * R;
    TBCtx t;
    t.z0 = s.z0 + tz * s.zc;
    t.z1 = min(t.z0 + s.zc, s.z1);
    t.zlast = t.z1 + 1;
    t.bz0 = s.z0;
    t.bz1 = s.z1;
    t.lane = threadIdx.x & (TW - 1);
    t.w = __builtin_amdgcn_readfirstlane(threadIdx.x / TW);
    t.x = x0 - 2 + t.lane;
    t.y = y0 - 2 + t.w;
    t.sz = (uint32_t)(d.px * d.py);
    // storage holds x in [-1, nx], y in [-1, ny]; the box keeps x, y >= 0
    const int cx = min(t.x, d.nx), cy = min(t.y, d.ny);
    t.col = (uint32_t)(d.off + cx) + (uint32_t)d.px * (uint32_t)cy;
    t.exc = t.w == 0 ? 0 : 2;
    t.xcol = (uint32_t)(d.off + cx) + (uint32_t)d.px * (uint32_t)min(y0 + R + 1, d.ny);
    t.idcol = (uint32_t)min(t.x, d.nx - 1) + (uint32_t)d.nx * (uint32_t)min(t.y, d.ny - 1);
    t.own = t.lane >= 2 && t.lane < TB_W + 2 && t.w >= 2 && t.w < R + 2 && t.x < s.x1 && t.y < s.y1;
    t.rim_xy = t.x == s.x0 || t.x == s.x1 - 1 || t.y == s.y0 || t.y == s.y1 - 1;
    t.all = __builtin_amdgcn_readfirstlane((int)d.tbflag[tl]) != 0;
    const bool rim_tile = t.all || tx == 0 || tx == s.ntx - 1 || ty == 0 || ty == s.nty - 1 ||
                          tz == 0 || tz == s.ntz - 1;
    t.src_col = d.src_kind != 0 && t.x < d.nx && t.y < d.ny && t.x >= d.src_box[0] &&
                t.x <= d.src_box[1] && t.y >= d.src_box[2] && t.y <= d.src_box[3];
    t.sk0 = d.src_kind != 0 ? d.src_box[4] : 1;
    t.sk1 = d.src_kind != 0 ? d.src_box[5] : 0;
    t.sval1 = t.src_col ? (float)source_at(d, level + 1) : 0.f;
    t.sval2 = t.src_col ? (float)source_at(d, level + 2) : 0.f;

    // ---- the coefficient LUTs into LDS ---------------------------------------
    constexpr int NTH = TW * (R + 3);
    const int nlut = d.nlut;
    for (int q = threadIdx.x; q < 3 * nlut; q += NTH) {
        const int c = q / nlut, e = q % nlut;
        dyn_lds[c * lut_cap + e] = lut_entry(c == 0 ? d.lut[0] : (c == 1 ? d.lut[1] : d.lut[2]), e);
    }

    // ---- prologue ------------------------------------------------------------
    TBState st;
    TBRegs ra, rb;
    const int mfirst = t.z0 == 0 ? 0 : t.z0 - 1;
    // E^n(mfirst) with its extra row, and the loads of position mfirst
    TBRegs p0;
    tb_load<R, IDB>(g, p0, t, mfirst, mfirst);
    tb_load<R, IDB>(g, ra, t, mfirst + 1, mfirst);
    st.h1p[0] = st.h1p[1] = st.h1p[2] = 0.f;
    st.e1p[0] = st.e1p[1] = st.e1p[2] = 0.f;
    st.h2p[0] = st.h2p[1] = 0.f;
    st.idp = 0;
    if (t.z0 > 0) {
        // Hx, Hy of H^{n+1/2}(z0-2), for the z difference of E^{n+1}(z0-1)
        const uint32_t c = t.col + t.sz * (uint32_t)(t.z0 - 2);
        const float ex = ldf(d.E[0], c), ey = ldf(d.E[1], c), ez = ldf(d.E[2], c);
        const float ezy = ldf(d.E[2], c + (uint32_t)d.px), ezx = ldf(d.E[2], c + 1u);
        const float hx = ldf(d.H[0], c), hy = ldf(d.H[1], c);
        st.h1p[0] = h_upd(hx, g.ch[1], ezy - ez, g.ch[2], p0.e[1] - ey);
        st.h1p[1] = h_upd(hy, g.ch[2], p0.e[0] - ex, g.ch[0], ezx - ez);
    }
    st.e0[0] = p0.e[0];
    st.e0[1] = p0.e[1];
    st.e0[2] = p0.e[2];
    tb_store_e0<R>(sm, t, 0, p0.e, p0.ex);
    // E^{n+1}(-1) below the grid for the bottom chunk (read at m = 0)
    sm.e1[0][0][t.w][t.lane] = 0.f;
    sm.e1[0][1][t.w][t.lane] = 0.f;
    lds_barrier();

    if (rim_tile) tb_march<R, IDB, NT, true>(g, sm, dyn_lds, lut_cap, t, mfirst, ra, rb, st);
    else tb_march<R, IDB, NT, false>(g, sm, dyn_lds, lut_cap, t, mfirst, ra, rb, st);
}

template <int R, int IDB, bool NT>
hipError_t launch_tb_r(const DevGrid<float> *g, const TBSet *set, int ntiles, int64_t level,
                       int lut_cap, int order, hipStream_t s)
{
    k_tb<R, IDB, NT><<<ntiles, TW * (R + 3), (size_t)lut_cap * 3 * sizeof(float4), s>>>(
        g, set, level, lut_cap, order);
    return hipGetLastError();
}

template <int IDB, bool NT>
hipError_t launch_tb_rows(const DevGrid<float> *g, const TBSet *set, int ntiles, int rows,
                          int64_t level, int lut_cap, int order, hipStream_t s)
{
    switch (rows) {
    case 10: return launch_tb_r<10, IDB, NT>(g, set, ntiles, level, lut_cap, order, s);
    case 8: return launch_tb_r<8, IDB, NT>(g, set, ntiles, level, lut_cap, order, s);
    case 13: return launch_tb_r<13, IDB, NT>(g, set, ntiles, level, lut_cap, order, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fused(const DevGrid<float> *grids_dev, const TileSet *sets_dev, int32_t ninst,
                        int32_t nb, int32_t ni, const LaunchCfg &cfg, int32_t lut_cap,
                        int32_t id_bits, int64_t level, const DevProbes *probes_dev,
                        int32_t max_probes, bool sample_input, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1)
{
    if (!valid_rows(cfg.rows) || cfg.order < 0 || !valid_order(cfg.order) || cfg.stream < 0)
        return hipErrorInvalidValue;
    if (lut_cap < 1 || lut_cap > LUT_LDS) return hipErrorInvalidValue;
    if (id_bits != 5 && id_bits != 8) return hipErrorInvalidValue;
    if (id_bits == 5 && lut_cap > 32) return hipErrorInvalidValue;
    const int npb = (sample_input && level >= 1) ? ninst * max_probes : 0;
    if (e0) (void)hipEventRecord(e0, s);
    hipError_t err = hipSuccess;
    // the two classes write disjoint cells and read only the input level
    auto launch = [&](auto layers, int32_t n, int32_t probe_blocks) {
        constexpr bool L = decltype(layers)::value;
        if (id_bits == 5)
            return cfg.stream ? launch_class<L, 5, true>(grids_dev, sets_dev, ninst, n, cfg, level,
                                                         probes_dev, probe_blocks, max_probes, lut_cap, s)
                              : launch_class<L, 5, false>(grids_dev, sets_dev, ninst, n, cfg, level,
                                                          probes_dev, probe_blocks, max_probes, lut_cap, s);
        return cfg.stream ? launch_class<L, 8, true>(grids_dev, sets_dev, ninst, n, cfg, level,
                                                     probes_dev, probe_blocks, max_probes, lut_cap, s)
                          : launch_class<L, 8, false>(grids_dev, sets_dev, ninst, n, cfg, level,
                                                      probes_dev, probe_blocks, max_probes, lut_cap, s);
    };
    if (nb + npb > 0) err = launch(std::true_type{}, nb, npb);
    if (err == hipSuccess && ni > 0) err = launch(std::false_type{}, ni, 0);
    if (e1) (void)hipEventRecord(e1, s);
    return err;
}


hipError_t launch_tb(const DevGrid<float> *g_dev, const TBSet *set_dev, int32_t ntiles,
                     const LaunchCfg &cfg, int32_t lut_cap, int32_t id_bits, int64_t level,
                     hipStream_t s)
{
    if (!valid_tb_rows(cfg.tb_rows) || cfg.order < 0 || !valid_order(cfg.order) || cfg.stream < 0)
        return hipErrorInvalidValue;
    if (lut_cap < 1 || lut_cap > LUT_LDS) return hipErrorInvalidValue;
    if (id_bits != 5 && id_bits != 8) return hipErrorInvalidValue;
    if (id_bits == 5 && lut_cap > 32) return hipErrorInvalidValue;
    if (ntiles <= 0) return hipSuccess;
    // Cached stores whatever the plan's stream-store setting: the tiles are
    // 60 cells wide, so their rows do not start on 128-byte lines, and
    // streaming stores would reach memory as partial lines where cached ones
    // let L2 merge the parts that neighbouring tiles write (1591 against
    // 1650 us per pass on the 1024x512x256 line)
    if (id_bits == 5)
        return launch_tb_rows<5, false>(g_dev, set_dev, ntiles, cfg.tb_rows, level, lut_cap, cfg.order, s);
    return launch_tb_rows<8, false>(g_dev, set_dev, ntiles, cfg.tb_rows, level, lut_cap, cfg.order, s);
}

}  // namespace fdtd
