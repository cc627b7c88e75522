// obs_kernels.hpp -- norms, magnetisation, energy (Eq. (5)) and rms sizes.
//
// One pass over the state: every thread accumulates, in FP64, for its grid
// points
//   N_j, sum r^2 rho_j (j = +1, 0, -1), the kinetic term (forward differences
//   over every link, including the link from the zero ghost before the first
//   point of each line), the trap, c0, c2, Rabi and spin-orbit terms of
//   Eq. (5); the workgroup sums go to a partial array and a one-workgroup
//   kernel adds them in a fixed order (run-to-run reproducible).
#pragma once
#include "cplx.hpp"

namespace ssgp {

constexpr int OBS_NQ = 12;  // N[3], r2w[3], kin, trap, c0, c2, rabi, so

template <typename R> struct ObsArgs {
    const cx<R> *psi;
    int dim, nx, ny;
    long long plane;
    double dx, dy, x0, y0, kappa2;
    double c0, c2, om_t;
    cx<double> hx[9], hy[9];  // H_SO psi_j = sum_j' hx[j][j'] d_x psi_j' + hy[j][j'] d_y psi_j'
    unsigned hxmask, hymask;
    double *partials;         // [gridDim.x][OBS_NQ]
};

template <typename R>
__device__ __forceinline__ cx<double> ld64(const cx<R> *p) {
    const cx<R> v = *p;
    return cx<double>{(double)v.x, (double)v.y};
}

template <typename R>
__global__ void __launch_bounds__(256) obs_kernel(ObsArgs<R> a) {
    __shared__ double red[OBS_NQ][4];
    double acc[OBS_NQ];
#pragma unroll
    for (int q = 0; q < OBS_NQ; ++q) acc[q] = 0.0;
    const long long n = a.plane;
    const double ix2 = 1.0 / (a.dx * a.dx), iy2 = 1.0 / (a.dy * a.dy);
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x) {
        const int ix = (int)(p % a.nx), iy = (int)(p / a.nx);
        const double x = a.x0 + ix * a.dx, y = a.dim == 2 ? a.y0 + iy * a.dy : 0.0;
        const double V = 0.5 * (x * x + a.kappa2 * y * y);
        cx<double> v[3];
        double rj[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            v[j] = ld64(a.psi + j * n + p);
            rj[j] = abs2(v[j]);
            acc[j] += rj[j];
            acc[3 + j] += (x * x + y * y) * rj[j];
            const cx<double> vr = ix + 1 < a.nx ? ld64(a.psi + j * n + p + 1) : czero<double>();
            double kin = 0.5 * abs2(vr - v[j]) * ix2;
            if (ix == 0) kin += 0.5 * rj[j] * ix2;
            if (a.dim == 2) {
                const cx<double> vu = iy + 1 < a.ny ? ld64(a.psi + j * n + p + a.nx) : czero<double>();
                kin += 0.5 * abs2(vu - v[j]) * iy2;
                if (iy == 0) kin += 0.5 * rj[j] * iy2;
            }
            acc[6] += kin;
        }
        const double rho = rj[0] + rj[1] + rj[2];
        acc[7] += V * rho;
        acc[8] += 0.5 * a.c0 * rho * rho;
        const cx<double> t4 = conj(v[2]) * v[1] * v[1] * conj(v[0]);
        acc[9] += 0.5 * a.c2 * (rj[0] * rj[0] + rj[2] * rj[2] + 2.0 * rj[0] * rj[1] + 2.0 * rj[2] * rj[1]
                                - 2.0 * rj[0] * rj[2] + 4.0 * t4.x);
        acc[10] += 2.0 * a.om_t * ((conj(v[0]) + conj(v[2])) * v[1]).x;
        if (a.hxmask | a.hymask) {
            cx<double> dxv[3], dyv[3];
#pragma unroll
            for (int jp = 0; jp < 3; ++jp) {
                const cx<R> *b = a.psi + jp * n + p;
                const cx<double> r = ix + 1 < a.nx ? ld64(b + 1) : czero<double>();
                const cx<double> l = ix >= 1 ? ld64(b - 1) : czero<double>();
                dxv[jp] = (0.5 / a.dx) * (r - l);
                dyv[jp] = czero<double>();
                if (a.dim == 2 && a.hymask) {
                    const cx<double> u = iy + 1 < a.ny ? ld64(b + a.nx) : czero<double>();
                    const cx<double> d = iy >= 1 ? ld64(b - a.nx) : czero<double>();
                    dyv[jp] = (0.5 / a.dy) * (u - d);
                }
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                cx<double> h = czero<double>();
#pragma unroll
                for (int jp = 0; jp < 3; ++jp) {
                    if (a.hxmask & (1u << (3 * j + jp))) h = cfma(a.hx[3 * j + jp], dxv[jp], h);
                    if (a.hymask & (1u << (3 * j + jp))) h = cfma(a.hy[3 * j + jp], dyv[jp], h);
                }
                acc[11] += (conj(v[j]) * h).x;
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < OBS_NQ; ++q) {
        double t = acc[q];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) t += __shfl_down(t, d, 64);
        if (lane == 0) red[q][wave] = t;
    }
    __syncthreads();
    if (threadIdx.x < OBS_NQ) {
        const int q = threadIdx.x;
        a.partials[(long long)blockIdx.x * OBS_NQ + q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
    }
}

} // namespace ssgp
