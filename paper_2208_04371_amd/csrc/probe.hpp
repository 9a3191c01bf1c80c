// Probe sampling shared by the probe kernels and the fused step kernel.
//
// Every probe is a weighted sum of field samples (the port voltage and
// current of eq. 4, or one field value).  The sum runs in FP64 in a fixed
// order: thread t adds terms t, t+B, ... (B = block size), the partials
// above the largest power of two P <= B are folded onto the first B - P,
// then a fixed pairwise tree over P, so results do not depend on timing.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace fdtd {

template <typename T>
__device__ __forceinline__ double probe_sum(const DevGrid<T> &d, const DevProbes &p, int r0,
                                            int r1, double *red)
{
    const int t = threadIdx.x, B = blockDim.x;
    double acc = 0.0;
    for (int q = r0 + t; q < r1; q += B) {
        const int comp = p.tcomp[q];
        const T *F = comp < 3 ? d.E[comp] : d.H[comp - 3];   // the level held in E/H
        acc += (double)F[p.toff[q]] * p.tw[q];
    }
    red[t] = acc;
    __syncthreads();
    int P = 1;
    while (2 * P <= B) P *= 2;
    if (t < B - P) red[t] += red[t + P];
    __syncthreads();
    for (int w = P / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double v = red[0];
    __syncthreads();
    return v;
}

// Sample probe `probe` of grid d into history slot (sample - 1) % K.
template <typename T>
__device__ __forceinline__ void probe_one(const DevGrid<T> &d, const DevProbes &p, int probe,
                                          int64_t sample, double *red)
{
    const int *r = p.range + 4 * probe;
    const double v = probe_sum(d, p, r[0], r[1], red);
    const double cur = probe_sum(d, p, r[2], r[3], red);
    if (threadIdx.x == 0) {
        const int64_t slot = (sample - 1) % p.K;
        p.hist[((int64_t)probe * 2 + 0) * p.K + slot] = v;
        p.hist[((int64_t)probe * 2 + 1) * p.K + slot] = cur;
    }
}

}  // namespace fdtd
