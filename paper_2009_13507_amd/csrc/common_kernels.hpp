// common_kernels.hpp -- the small single-workgroup reduction kernels
// (fixed-order sums, run-to-run reproducible).  Included by one translation
// unit only.
#pragma once
#include "adjoint_kernels.hpp"
#include "batch_kernels.hpp"
#include "obs_kernels.hpp"
#include "step_kernels.hpp"

namespace ssgp {

// Sums the per-tile |psi|^2 partials (wave_tile_sums: the order every
// x-pass workgroup uses too) and writes
// out = {d_+1, d_0, d_-1, N_+1, N_0, N_-1, fallback}.  One wavefront.
__global__ void __launch_bounds__(64) renorm_finalize_kernel(const double *partials, int ntiles, RenormSpec sp,
                                                             double *out) {
    double s[3];
    wave_tile_sums(partials, ntiles, s);
    if (threadIdx.x == 0) {
        double N[3] = {s[0] * sp.dA, s[1] * sp.dA, s[2] * sp.dA};
        double d[3], fb = 0.0;
        renorm_factors(sp, N, d, &fb);
        for (int j = 0; j < 3; ++j) {
            out[j] = d[j];
            out[3 + j] = N[j];
        }
        out[6] = fb;
    }
}

__global__ void __launch_bounds__(1024) obs_finalize_kernel(const double *partials, int nblocks, double *out) {
    __shared__ double red[OBS_NQ][16];
    double s[OBS_NQ];
#pragma unroll
    for (int q = 0; q < OBS_NQ; ++q) s[q] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 1024)
#pragma unroll
        for (int q = 0; q < OBS_NQ; ++q) s[q] += partials[(long long)b * OBS_NQ + q];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < OBS_NQ; ++q) {
        double t = s[q];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) t += __shfl_down(t, d, 64);
        if (lane == 0) red[q][wave] = t;
    }
    __syncthreads();
    if (threadIdx.x < OBS_NQ) {
        const int q = threadIdx.x;
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += red[q][w];
        out[q] = t;
    }
}

// dL/dOmega over a call's adjoint steps.  The per-row partials of the k-th
// step of the call are partials[k * nrows + row].  omega_step_sums_kernel
// sums each step's rows in a fixed tree (one workgroup per step);
// omega_accumulate_kernel then adds the step sums to their Omega segments in
// the order the steps are taken back (k = nsteps - 1 down to 0; step index
// n0 + k, segment (n0 + k) / steps_per_seg clamped to [0, nseg), or 0
// without a schedule, nseg = 0).
__global__ void __launch_bounds__(256) omega_step_sums_kernel(const double *partials, int nrows, double *sums) {
    __shared__ double red[256];
    const double *p = partials + (long long)blockIdx.x * nrows;
    double s = 0.0;
    for (int q = threadIdx.x; q < nrows; q += 256) s += p[q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__global__ void omega_accumulate_kernel(const double *sums, int nsteps, long long n0, int steps_per_seg, int nseg,
                                        double *acc) {
    if (threadIdx.x != 0) return;
    for (int k = nsteps - 1; k >= 0; --k) {
        long long seg = 0;
        if (nseg > 0) {
            seg = (n0 + k) / steps_per_seg;
            seg = seg < 0 ? 0 : seg >= nseg ? nseg - 1 : seg;
        }
        acc[seg] += sums[k];
    }
}

// Clears the batched step's barrier words before a launch; a barrier
// timeout of the previous launch is kept in the sticky flag bar[3] for the
// host.
__global__ void batch_reset_kernel(unsigned *bar) {
    if (threadIdx.x == 0) {
        if (bar[2] != 0u) bar[3] = 1u;
        bar[0] = 0u;
        bar[2] = 0u;
    }
}

} // namespace ssgp
