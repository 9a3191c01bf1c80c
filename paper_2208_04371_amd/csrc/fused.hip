// Fused FP32 Yee step: H^{n+1/2} and E^{n+1} (with the absorbing-layer
// auxiliaries and the soft source) in one pass over the grid.
//
// A block owns a tile of 64 (x) by R (y) cells and marches through a chunk of
// z planes.  For plane k it needs E^n of planes k and k+1 with a one-cell
// halo in x and y: both planes sit in LDS (double-buffered, the k+1 plane of
// one iteration is the k plane of the next).  H^{n+1/2}(k) is computed for
// the tile plus the low-x column and low-y row (the halo the E update needs),
// kept in LDS, and E^{n+1}(k) follows from it and the H^{n+1/2}(k-1) values
// each thread carries in registers from the previous plane.
//
// Reads and writes go to separate buffers (fields and auxiliaries are
// ping-ponged between steps), so the halo a block recomputes never races
// with the block that owns those cells.  Every cell value is read once from
// HBM and written once per step; halo re-reads hit L2, helped by a block ->
// tile map that keeps neighbouring tiles on the same XCD.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace fdtd {

namespace {

constexpr int TW = 64;   // tile width in x = one wavefront

__device__ __forceinline__ bool layer_slot(int p, int lo, int hi, int n, int &s)
{
    if (p < lo) { s = p; return true; }
    if (p >= n - hi) { s = p - (n - hi) + lo; return true; }
    return false;
}

__device__ __forceinline__ float lterm(float diff, const float *prof, int n, int pos, bool is_h,
                                       const float *psi_in, float *psi_out, int64_t q, bool store)
{
    const float b = prof[(is_h ? PR_BH : PR_BE) * n + pos];
    const float c = prof[(is_h ? PR_CH : PR_CE) * n + pos];
    const float ik = prof[(is_h ? PR_KH : PR_KE) * n + pos];
    const float p = b * psi_in[q] + c * diff;
    if (store) psi_out[q] = p;
    return diff * ik + p;
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

// H^{n+1/2} at (i, j, k) from the six forward differences of E^n.  `store`
// writes the updated auxiliaries (only the owner of a cell does).
struct HDiff {
    float ez_y, ey_z, ex_z, ez_x, ey_x, ex_y;
};

__device__ __forceinline__ void h_apply(const DevGrid<float> &d, int i, int j, int k, HDiff df,
                                        float hx, float hy, float hz, bool store, float &ox,
                                        float &oy, float &oz)
{
    int s;
    if (layer_slot(i, d.lo[0], d.hi[0], d.nx, s)) {
        const int64_t q = s + (int64_t)(d.lo[0] + d.hi[0]) * (j + (int64_t)d.ny * k);
        df.ez_x = lterm(df.ez_x, d.prof[0], d.nx, i, true, d.psi[PSI_HYX], d.psi_o[PSI_HYX], q, store);
        df.ey_x = lterm(df.ey_x, d.prof[0], d.nx, i, true, d.psi[PSI_HZX], d.psi_o[PSI_HZX], q, store);
    }
    if (layer_slot(j, d.lo[1], d.hi[1], d.ny, s)) {
        const int64_t q = i + (int64_t)d.px * (s + (int64_t)(d.lo[1] + d.hi[1]) * k);
        df.ez_y = lterm(df.ez_y, d.prof[1], d.ny, j, true, d.psi[PSI_HXY], d.psi_o[PSI_HXY], q, store);
        df.ex_y = lterm(df.ex_y, d.prof[1], d.ny, j, true, d.psi[PSI_HZY], d.psi_o[PSI_HZY], q, store);
    }
    if (layer_slot(k, d.lo[2], d.hi[2], d.nz, s)) {
        const int64_t q = i + (int64_t)d.px * (j + (int64_t)d.ny * s);
        df.ey_z = lterm(df.ey_z, d.prof[2], d.nz, k, true, d.psi[PSI_HXZ], d.psi_o[PSI_HXZ], q, store);
        df.ex_z = lterm(df.ex_z, d.prof[2], d.nz, k, true, d.psi[PSI_HYZ], d.psi_o[PSI_HYZ], q, store);
    }
    ox = hx - d.ch[1] * df.ez_y + d.ch[2] * df.ey_z;
    oy = hy - d.ch[2] * df.ex_z + d.ch[0] * df.ez_x;
    oz = hz - d.ch[0] * df.ey_x + d.ch[1] * df.ex_y;
}

template <int R>
struct Smem {
    float e[2][3][R + 2][TW + 2];   // E^n planes k / k+1: rows y0-1..y0+R, cols x0-1..x0+64
    float h[3][R + 1][TW + 1];      // H^{n+1/2}(k): rows y0-1..y0+R-1, cols x0-1..x0+63
};

template <int R>
__device__ void load_e_plane(const DevGrid<float> &d, Smem<R> &sm, int buf, int x0, int y0, int k)
{
    const int t = threadIdx.x;
    const int lane = t & (TW - 1), w = t / TW;
    const int64_t sy = d.px, sz = (int64_t)d.px * d.py;
    const int64_t base = d.off + x0 + sy * (y0 - 1) + sz * k;
    // main columns: R waves over 3 * (R + 2) rows, aligned 64-wide loads
    for (int r = w; r < 3 * (R + 2); r += R) {
        const int comp = r / (R + 2), row = r % (R + 2);
        sm.e[buf][comp][row][lane + 1] = d.E[comp][base + sy * row + lane];
    }
    // halo columns x0-1 and x0+64
    for (int q = t; q < 3 * (R + 2) * 2; q += TW * R) {
        const int side = q & 1, rest = q >> 1;
        const int comp = rest / (R + 2), row = rest % (R + 2);
        const int col = side ? TW : -1;
        sm.e[buf][comp][row][col + 1] = d.E[comp][base + sy * row + col];
    }
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
    const int64_t sy = d.px, sz = (int64_t)d.px * d.py;

    // H^{n+1/2}(z0-1) at the own cell, needed by E(z0).  On the bottom face
    // the E edges it feeds are PEC, so it is not needed there.
    float hx_prev = 0.f, hy_prev = 0.f;
    if (own && z0 > 0) {
        const int k = z0 - 1;
        const int64_t c = d.off + i + sy * j + sz * k;
        HDiff df;
        const float ex = d.E[0][c], ey = d.E[1][c], ez = d.E[2][c];
        df.ez_y = d.E[2][c + sy] - ez;
        df.ey_z = d.E[1][c + sz] - ey;
        df.ex_z = d.E[0][c + sz] - ex;
        df.ez_x = d.E[2][c + 1] - ez;
        df.ey_x = d.E[1][c + 1] - ey;
        df.ex_y = d.E[0][c + sy] - ex;
        float oz;
        h_apply(d, i, j, k, df, d.H[0][c], d.H[1][c], d.H[2][c], false, hx_prev, hy_prev, oz);
    }

    int cur = 0;
    load_e_plane<R>(d, sm, cur, x0, y0, z0);
    const bool src_tile = d.src_kind != 0;
    double sval = 0.0;
    if (src_tile && own && i >= d.src_box[0] && i <= d.src_box[1] && j >= d.src_box[2] &&
        j <= d.src_box[3])
        sval = src_value(d, level + 1);

    for (int k = z0; k < z1; ++k) {
        const int nxt = cur ^ 1;
        load_e_plane<R>(d, sm, nxt, x0, y0, k + 1);
        __syncthreads();

        // ---- H^{n+1/2}(k): own cell ---------------------------------------
        const int64_t c = d.off + i + sy * j + sz * k;
        {
            const int lx = lane + 1, ly = row + 1;
            HDiff df;
            const float ex = sm.e[cur][0][ly][lx], ey = sm.e[cur][1][ly][lx], ez = sm.e[cur][2][ly][lx];
            df.ez_y = sm.e[cur][2][ly + 1][lx] - ez;
            df.ey_z = sm.e[nxt][1][ly][lx] - ey;
            df.ex_z = sm.e[nxt][0][ly][lx] - ex;
            df.ez_x = sm.e[cur][2][ly][lx + 1] - ez;
            df.ey_x = sm.e[cur][1][ly][lx + 1] - ey;
            df.ex_y = sm.e[cur][0][ly + 1][lx] - ex;
            float ox = 0.f, oy = 0.f, oz = 0.f;
            if (own) {
                h_apply(d, i, j, k, df, d.H[0][c], d.H[1][c], d.H[2][c], true, ox, oy, oz);
                d.Ho[0][c] = ox;
                d.Ho[1][c] = oy;
                d.Ho[2][c] = oz;
            }
            sm.h[0][row + 1][lane + 1] = ox;
            sm.h[1][row + 1][lane + 1] = oy;
            sm.h[2][row + 1][lane + 1] = oz;
        }
        // ---- H^{n+1/2}(k): halo row y0-1 and halo column x0-1 -------------
        for (int hq = t; hq < TW + R + 1; hq += TW * R) {
            int hi_, hj_;
            if (hq < TW) { hi_ = x0 + hq; hj_ = y0 - 1; }
            else { hi_ = x0 - 1; hj_ = y0 - 1 + (hq - TW); }
            const int lx = hi_ - x0 + 1, ly = hj_ - y0 + 1;
            float ox = 0.f, oy = 0.f, oz = 0.f;
            if (hi_ >= 0 && hj_ >= 0 && hi_ < d.nx && hj_ < d.ny) {
                HDiff df;
                const float ex = sm.e[cur][0][ly][lx], ey = sm.e[cur][1][ly][lx],
                            ez = sm.e[cur][2][ly][lx];
                df.ez_y = sm.e[cur][2][ly + 1][lx] - ez;
                df.ey_z = sm.e[nxt][1][ly][lx] - ey;
                df.ex_z = sm.e[nxt][0][ly][lx] - ex;
                df.ez_x = sm.e[cur][2][ly][lx + 1] - ez;
                df.ey_x = sm.e[cur][1][ly][lx + 1] - ey;
                df.ex_y = sm.e[cur][0][ly + 1][lx] - ex;
                const int64_t ch = d.off + hi_ + sy * hj_ + sz * k;
                h_apply(d, hi_, hj_, k, df, d.H[0][ch], d.H[1][ch], d.H[2][ch], false, ox, oy, oz);
            }
            sm.h[0][ly][lx] = ox;
            sm.h[1][ly][lx] = oy;
            sm.h[2][ly][lx] = oz;
        }
        __syncthreads();

        // ---- E^{n+1}(k): own cell -----------------------------------------
        if (own) {
            const int lx = lane + 1, ly = row + 1;
            const float hx = sm.h[0][ly][lx], hy = sm.h[1][ly][lx], hz = sm.h[2][ly][lx];
            float dHz_y = hz - sm.h[2][ly - 1][lx];
            float dHy_z = hy - hy_prev;
            float dHx_z = hx - hx_prev;
            float dHz_x = hz - sm.h[2][ly][lx - 1];
            float dHy_x = hy - sm.h[1][ly][lx - 1];
            float dHx_y = hx - sm.h[0][ly - 1][lx];
            int s;
            if (layer_slot(i, d.lo[0], d.hi[0], d.nx, s)) {
                const int64_t q = s + (int64_t)(d.lo[0] + d.hi[0]) * (j + (int64_t)d.ny * k);
                dHz_x = lterm(dHz_x, d.prof[0], d.nx, i, false, d.psi[PSI_EYX], d.psi_o[PSI_EYX], q, true);
                dHy_x = lterm(dHy_x, d.prof[0], d.nx, i, false, d.psi[PSI_EZX], d.psi_o[PSI_EZX], q, true);
            }
            if (layer_slot(j, d.lo[1], d.hi[1], d.ny, s)) {
                const int64_t q = i + (int64_t)d.px * (s + (int64_t)(d.lo[1] + d.hi[1]) * k);
                dHz_y = lterm(dHz_y, d.prof[1], d.ny, j, false, d.psi[PSI_EXY], d.psi_o[PSI_EXY], q, true);
                dHx_y = lterm(dHx_y, d.prof[1], d.ny, j, false, d.psi[PSI_EZY], d.psi_o[PSI_EZY], q, true);
            }
            if (layer_slot(k, d.lo[2], d.hi[2], d.nz, s)) {
                const int64_t q = i + (int64_t)d.px * (j + (int64_t)d.ny * s);
                dHy_z = lterm(dHy_z, d.prof[2], d.nz, k, false, d.psi[PSI_EXZ], d.psi_o[PSI_EXZ], q, true);
                dHx_z = lterm(dHx_z, d.prof[2], d.nz, k, false, d.psi[PSI_EYZ], d.psi_o[PSI_EYZ], q, true);
            }
            const int64_t qi = i + (int64_t)d.px * (j + (int64_t)d.ny * k);
            int idx, idy, idz;
            if (d.id16) {
                idx = static_cast<const uint16_t *>(d.ids[0])[qi];
                idy = static_cast<const uint16_t *>(d.ids[1])[qi];
                idz = static_cast<const uint16_t *>(d.ids[2])[qi];
            } else {
                idx = static_cast<const uint8_t *>(d.ids[0])[qi];
                idy = static_cast<const uint8_t *>(d.ids[1])[qi];
                idz = static_cast<const uint8_t *>(d.ids[2])[qi];
            }
            const float4 cx = reinterpret_cast<const float4 *>(d.lut[0])[idx];
            const float4 cy = reinterpret_cast<const float4 *>(d.lut[1])[idy];
            const float4 cz = reinterpret_cast<const float4 *>(d.lut[2])[idz];
            d.Eo[0][c] = cx.x * sm.e[cur][0][ly][lx] + cx.y * dHz_y - cx.z * dHy_z;
            d.Eo[1][c] = cy.x * sm.e[cur][1][ly][lx] + cy.y * dHx_z - cy.z * dHz_x;
            float ez = cz.x * sm.e[cur][2][ly][lx] + cz.y * dHy_x - cz.z * dHx_y;
            if (sval != 0.0 && k >= d.src_box[4] && k <= d.src_box[5]) ez += (float)sval;
            d.Eo[2][c] = ez;
            hx_prev = hx;
            hy_prev = hy;
        }
        cur = nxt;
        __syncthreads();
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

template <int R>
__global__ void __launch_bounds__(TW *R) k_fused(DevGrid<float> d, int zchunk, int ntiles,
                                                 int64_t level)
{
    __shared__ Smem<R> sm;
    fused_tile<R>(d, xcd_tile(blockIdx.x, ntiles), zchunk, level, sm);
}

template <int R>
__global__ void __launch_bounds__(TW *R)
k_fused_batch(const DevGrid<float> *grids, const int32_t *block_start, int ninst, int zchunk,
              int ntiles, int64_t level)
{
    __shared__ Smem<R> sm;
    const int b = xcd_tile(blockIdx.x, ntiles);
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {          // last instance whose first block <= b
        const int mid = (lo + hi + 1) >> 1;
        if (block_start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    fused_tile<R>(grids[lo], b - block_start[lo], zchunk, level, sm);
}

template <int R>
hipError_t launch_r(const DevGrid<float> &d, int zchunk, int64_t level, hipStream_t s)
{
    const int n = fused_tiles(d.nx, d.ny, d.nz, LaunchCfg{R, zchunk});
    k_fused<R><<<n, TW * R, 0, s>>>(d, zchunk, n, level);
    return hipGetLastError();
}

template <int R>
hipError_t launch_batch_r(const DevGrid<float> *g, const int32_t *bs, int ninst, int total,
                          int zchunk, int64_t level, hipStream_t s)
{
    k_fused_batch<R><<<total, TW * R, 0, s>>>(g, bs, ninst, zchunk, total, level);
    return hipGetLastError();
}

}  // namespace

int32_t fused_tiles(int32_t nx, int32_t ny, int32_t nz, const LaunchCfg &cfg)
{
    const int tx = (nx + TW - 1) / TW, ty = (ny + cfg.rows - 1) / cfg.rows;
    const int tz = (nz + cfg.zchunk - 1) / cfg.zchunk;
    return tx * ty * tz;
}

hipError_t launch_fused_step(const DevGrid<float> &d, const LaunchCfg &cfg, int64_t level,
                             hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (e0) hipEventRecord(e0, s);
    hipError_t err;
    switch (cfg.rows) {
    case 1: err = launch_r<1>(d, cfg.zchunk, level, s); break;
    case 2: err = launch_r<2>(d, cfg.zchunk, level, s); break;
    case 4: err = launch_r<4>(d, cfg.zchunk, level, s); break;
    case 8: err = launch_r<8>(d, cfg.zchunk, level, s); break;
    case 16: err = launch_r<16>(d, cfg.zchunk, level, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e1) hipEventRecord(e1, s);
    return err;
}

hipError_t launch_fused_batch(const DevGrid<float> *grids_dev, const int32_t *block_start_dev,
                              int32_t ninst, int32_t total_blocks, const LaunchCfg &cfg,
                              int64_t level, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (e0) hipEventRecord(e0, s);
    hipError_t err;
    switch (cfg.rows) {
    case 1: err = launch_batch_r<1>(grids_dev, block_start_dev, ninst, total_blocks, cfg.zchunk, level, s); break;
    case 2: err = launch_batch_r<2>(grids_dev, block_start_dev, ninst, total_blocks, cfg.zchunk, level, s); break;
    case 4: err = launch_batch_r<4>(grids_dev, block_start_dev, ninst, total_blocks, cfg.zchunk, level, s); break;
    case 8: err = launch_batch_r<8>(grids_dev, block_start_dev, ninst, total_blocks, cfg.zchunk, level, s); break;
    case 16: err = launch_batch_r<16>(grids_dev, block_start_dev, ninst, total_blocks, cfg.zchunk, level, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e1) hipEventRecord(e1, s);
    return err;
}

}  // namespace fdtd
