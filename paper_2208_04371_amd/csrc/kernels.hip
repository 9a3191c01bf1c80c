// Plain (unfused) Yee kernels, probe sampling and the running DFT.
//
// One step n -> n+1 of the leapfrog (Yee 1966, the grid of Sec. II-A):
//   H^{n+1/2} = H^{n-1/2} - dt/mu0 curl E^n            (k_h_plain)
//   E^{n+1}   = Ca E^n + Cb curl H^{n+1/2}, Ez += s     (k_e_plain)
// with convolutional-PML auxiliary terms inside the absorbing layers: every
// difference along an axis w becomes diff/kappa_w + psi, psi <- b psi + c diff
// (psi kept in difference units, i.e. multiplied by the cell size).
// The kernels are templated on the field type: FP64 for the plain FP64
// path, FP32 for the plain FP32 path.  One thread per cell (i, j, k) updates
// the three components stored at that index.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "probe.hpp"
#include "source.hpp"

namespace fdtd {

namespace {

constexpr int BX = 64;   // one wavefront along x
constexpr int BY = 4;

__device__ __forceinline__ bool in_layer(int p, int lo, int hi, int n, int &s)
{
    if (p < lo) { s = p; return true; }
    if (p >= n - hi) { s = p - (n - hi) + lo; return true; }
    return false;
}

template <typename T>
__device__ __forceinline__ int edge_id(const DevGrid<T> &d, int comp, int64_t q)
{
    return d.id16 ? (int)static_cast<const uint16_t *>(d.ids[comp])[q]
                  : (int)static_cast<const uint8_t *>(d.ids[comp])[q];
}

// Layer-modified difference: diff * (1/kappa) + psi, psi <- b psi + c diff.
template <typename T>
__device__ __forceinline__ T layer_term(T diff, const T *prof, int n, int pos, int slot,
                                        bool is_h, T *psi, int64_t q)
{
    const T b = prof[(is_h ? PR_BH : PR_BE) * n + pos];
    const T c = prof[(is_h ? PR_CH : PR_CE) * n + pos];
    const T ik = prof[(is_h ? PR_KH : PR_KE) * n + pos];
    T p = b * psi[q] + c * diff;
    psi[q] = p;
    (void)slot;
    return diff * ik + p;
}

template <typename T>
__global__ void __launch_bounds__(BX *BY) k_h_plain(DevGrid<T> d)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    const int64_t sy = d.px, sz = (int64_t)d.px * d.py;
    const int64_t c = d.off + i + sy * j + sz * k;
    const T ex = d.E[0][c], ey = d.E[1][c], ez = d.E[2][c];
    // forward differences of E around the three H nodes of this cell
    T dEz_y = d.E[2][c + sy] - ez, dEy_z = d.E[1][c + sz] - ey;   // Hx
    T dEx_z = d.E[0][c + sz] - ex, dEz_x = d.E[2][c + 1] - ez;    // Hy
    T dEy_x = d.E[1][c + 1] - ey, dEx_y = d.E[0][c + sy] - ex;    // Hz

    int xs, ys, zs;
    const int Lx = d.lo[0] + d.hi[0], Ly = d.lo[1] + d.hi[1], Lz = d.lo[2] + d.hi[2];
    if (in_layer(i, d.lo[0], d.hi[0], d.nx, xs)) {
        const int64_t q = xs + (int64_t)Lx * (j + (int64_t)d.ny * k);
        dEz_x = layer_term(dEz_x, d.prof[0], d.nx, i, 0, true, d.psi[PSI_HYX], q);
        dEy_x = layer_term(dEy_x, d.prof[0], d.nx, i, 0, true, d.psi[PSI_HZX], q);
    }
    if (in_layer(j, d.lo[1], d.hi[1], d.ny, ys)) {
        const int64_t q = i + (int64_t)d.nx * (ys + (int64_t)Ly * k);
        dEz_y = layer_term(dEz_y, d.prof[1], d.ny, j, 0, true, d.psi[PSI_HXY], q);
        dEx_y = layer_term(dEx_y, d.prof[1], d.ny, j, 0, true, d.psi[PSI_HZY], q);
    }
    if (in_layer(k, d.lo[2], d.hi[2], d.nz, zs)) {
        const int64_t q = i + (int64_t)d.nx * (j + (int64_t)d.ny * zs);
        dEy_z = layer_term(dEy_z, d.prof[2], d.nz, k, 0, true, d.psi[PSI_HXZ], q);
        dEx_z = layer_term(dEx_z, d.prof[2], d.nz, k, 0, true, d.psi[PSI_HYZ], q);
    }
    d.Ho[0][c] = d.H[0][c] - d.ch[1] * dEz_y + d.ch[2] * dEy_z;
    d.Ho[1][c] = d.H[1][c] - d.ch[2] * dEx_z + d.ch[0] * dEz_x;
    d.Ho[2][c] = d.H[2][c] - d.ch[0] * dEy_x + d.ch[1] * dEx_y;
}

template <typename T>
__global__ void __launch_bounds__(BX *BY) k_e_plain(DevGrid<T> d, int64_t level)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    const int64_t sy = d.px, sz = (int64_t)d.px * d.py;
    const int64_t c = d.off + i + sy * j + sz * k;
    const T hx = d.H[0][c], hy = d.H[1][c], hz = d.H[2][c];
    // backward differences of H around the three E edges of this cell
    T dHz_y = hz - d.H[2][c - sy], dHy_z = hy - d.H[1][c - sz];   // Ex
    T dHx_z = hx - d.H[0][c - sz], dHz_x = hz - d.H[2][c - 1];    // Ey
    T dHy_x = hy - d.H[1][c - 1], dHx_y = hx - d.H[0][c - sy];    // Ez

    int xs, ys, zs;
    const int Lx = d.lo[0] + d.hi[0], Ly = d.lo[1] + d.hi[1], Lz = d.lo[2] + d.hi[2];
    (void)Lz;
    if (in_layer(i, d.lo[0], d.hi[0], d.nx, xs)) {
        const int64_t q = xs + (int64_t)Lx * (j + (int64_t)d.ny * k);
        dHz_x = layer_term(dHz_x, d.prof[0], d.nx, i, 0, false, d.psi[PSI_EYX], q);
        dHy_x = layer_term(dHy_x, d.prof[0], d.nx, i, 0, false, d.psi[PSI_EZX], q);
    }
    if (in_layer(j, d.lo[1], d.hi[1], d.ny, ys)) {
        const int64_t q = i + (int64_t)d.nx * (ys + (int64_t)Ly * k);
        dHz_y = layer_term(dHz_y, d.prof[1], d.ny, j, 0, false, d.psi[PSI_EXY], q);
        dHx_y = layer_term(dHx_y, d.prof[1], d.ny, j, 0, false, d.psi[PSI_EZY], q);
    }
    if (in_layer(k, d.lo[2], d.hi[2], d.nz, zs)) {
        const int64_t q = i + (int64_t)d.nx * (j + (int64_t)d.ny * zs);
        dHy_z = layer_term(dHy_z, d.prof[2], d.nz, k, 0, false, d.psi[PSI_EXZ], q);
        dHx_z = layer_term(dHx_z, d.prof[2], d.nz, k, 0, false, d.psi[PSI_EYZ], q);
    }
    const int64_t qi = i + (int64_t)d.nx * (j + (int64_t)d.ny * k);
    const T *cx = d.lut[0] + 4 * edge_id(d, 0, qi);
    const T *cy = d.lut[1] + 4 * edge_id(d, 1, qi);
    const T *cz = d.lut[2] + 4 * edge_id(d, 2, qi);
    d.Eo[0][c] = cx[0] * d.E[0][c] + cx[1] * dHz_y - cx[2] * dHy_z;
    d.Eo[1][c] = cy[0] * d.E[1][c] + cy[1] * dHx_z - cy[2] * dHz_x;
    T ez = cz[0] * d.E[2][c] + cz[1] * dHy_x - cz[2] * dHx_y;
    if (d.src_kind && i >= d.src_box[0] && i <= d.src_box[1] && j >= d.src_box[2] &&
        j <= d.src_box[3] && k >= d.src_box[4] && k <= d.src_box[5]) {
        ez += (T)source_at(d, level + 1);
    }
    d.Eo[2][c] = ez;
}

constexpr int PROBE_THREADS = 256;

template <typename T>
__global__ void __launch_bounds__(PROBE_THREADS) k_probe(DevGrid<T> d, DevProbes p, int64_t sample)
{
    __shared__ double red[PROBE_THREADS];
    probe_one(d, p, blockIdx.x, sample, red);
}

__global__ void __launch_bounds__(PROBE_THREADS)
k_probe_batch(const DevGrid<float> *grids, const DevProbes *probes, int64_t sample)
{
    __shared__ double red[PROBE_THREADS];
    const int inst = blockIdx.y;
    const DevProbes &p = probes[inst];
    if ((int)blockIdx.x >= p.nprobe) return;
    probe_one(grids[inst], p, blockIdx.x, sample, red);
}

// Running DFT: one thread per (probe, signal, frequency) adds the samples
// n_first .. n_first+count-1 in order.  Phase 2 pi frac(f dt t_n) in FP64;
// t_n = n for voltages / point values, n - 1/2 for currents.
__device__ void dft_one(const DevDft &d, int idx, int64_t n_first, int64_t count)
{
    const int nf = d.nf;
    if (idx >= d.nprobe * 2 * nf) return;
    const int f = idx % nf;
    const int sig = (idx / nf) % 2;
    const int q = idx / (2 * nf);
    const double *h = d.hist + ((int64_t)q * 2 + sig) * d.K;
    double re = d.acc[(int64_t)idx * 2 + 0], im = d.acc[(int64_t)idx * 2 + 1];
    for (int64_t s = 0; s < count; ++s) {
        const int64_t n = n_first + s;
        const double x = h[(n - 1) % d.K];
        const double tn = sig ? (double)n - 0.5 : (double)n;
        const double cyc = d.freqs[f] * d.dt * tn;
        const double ph = 2.0 * M_PI * (cyc - floor(cyc));
        double sn, cs;
        sincos(ph, &sn, &cs);
        re += x * cs * d.dt;
        im -= x * sn * d.dt;
    }
    d.acc[(int64_t)idx * 2 + 0] = re;
    d.acc[(int64_t)idx * 2 + 1] = im;
}

__global__ void __launch_bounds__(256) k_dft(DevDft d, int64_t n_first, int64_t count)
{
    dft_one(d, blockIdx.x * 256 + threadIdx.x, n_first, count);
}

__global__ void __launch_bounds__(256)
k_dft_batch(const DevDft *table, int64_t n_first, int64_t count)
{
    dft_one(table[blockIdx.y], blockIdx.x * 256 + threadIdx.x, n_first, count);
}

}  // namespace

template <typename T>
hipError_t launch_plain_step(const DevGrid<T> &d, int64_t level, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1)
{
    dim3 block(BX, BY, 1);
    dim3 grid((d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, d.nz);
    if (e0) {
        const hipError_t r = hipEventRecord(e0, s);
        if (r != hipSuccess) return r;
    }
    k_h_plain<T><<<grid, block, 0, s>>>(d);
    k_e_plain<T><<<grid, block, 0, s>>>(d, level);
    hipError_t r = hipGetLastError();
    if (r == hipSuccess && e1) r = hipEventRecord(e1, s);
    return r;
}

template <typename T>
hipError_t launch_probe(const DevGrid<T> &d, const DevProbes &p, int64_t sample, hipStream_t s)
{
    if (p.nprobe <= 0) return hipSuccess;
    k_probe<T><<<p.nprobe, PROBE_THREADS, 0, s>>>(d, p, sample);
    return hipGetLastError();
}

hipError_t launch_dft(const DevDft &d, int64_t n_first, int64_t count, hipStream_t s)
{
    const int n = d.nprobe * 2 * d.nf;
    if (n <= 0 || count <= 0) return hipSuccess;
    k_dft<<<(n + 255) / 256, 256, 0, s>>>(d, n_first, count);
    return hipGetLastError();
}

hipError_t launch_probe_batch(const DevGrid<float> *grids_dev, const DevProbes *probes_dev,
                              int32_t ninst, int32_t max_probes, int64_t sample, hipStream_t s)
{
    if (max_probes <= 0) return hipSuccess;
    k_probe_batch<<<dim3(max_probes, ninst), PROBE_THREADS, 0, s>>>(grids_dev, probes_dev, sample);
    return hipGetLastError();
}

hipError_t launch_dft_batch(const DevDft *dft_dev, int32_t ninst, int32_t max_probes,
                            int32_t max_nf, int64_t n_first, int64_t count, hipStream_t s)
{
    const int n = max_probes * 2 * max_nf;
    if (n <= 0 || count <= 0) return hipSuccess;
    k_dft_batch<<<dim3((n + 255) / 256, ninst), 256, 0, s>>>(dft_dev, n_first, count);
    return hipGetLastError();
}

template hipError_t launch_plain_step<float>(const DevGrid<float> &, int64_t, hipStream_t,
                                             hipEvent_t, hipEvent_t);
template hipError_t launch_plain_step<double>(const DevGrid<double> &, int64_t, hipStream_t,
                                              hipEvent_t, hipEvent_t);
template hipError_t launch_probe<float>(const DevGrid<float> &, const DevProbes &, int64_t,
                                        hipStream_t);
template hipError_t launch_probe<double>(const DevGrid<double> &, const DevProbes &, int64_t,
                                         hipStream_t);

}  // namespace fdtd
