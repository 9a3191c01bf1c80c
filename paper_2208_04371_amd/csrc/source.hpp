// Value of the soft source for an E level (eq. 3 and the pulses beside it),
// shared by the plain and the fused kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace fdtd {

// s(level): what the soft source adds to its E nodes when they reach `level`
// (time level * dt).  Evaluated in FP64; kind/parameters from the plan.
template <typename T>
__device__ __forceinline__ double source_at(const DevGrid<T> &d, int64_t level)
{
    if (d.src_kind == FDTD_WAVE_GAUSSIAN_STEPS) {
        const double u = ((double)level - d.src_t0) / d.src_w;
        return d.src_amp * exp(-u * u);
    }
    if (d.src_kind == FDTD_WAVE_SAMPLED)
        return (level >= 1 && level <= d.src_nsamp) ? d.src_amp * d.src_samples[level - 1] : 0.0;
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

}  // namespace fdtd
