// obs_kernels.hpp -- norms, magnetisation, energy (Eq. (5)) and rms sizes.
//
// One pass over the state: every thread accumulates, in FP64, for its grid
// points
//   N_j, sum r^2 rho_j (j = +1, 0, -1), the kinetic term (forward differences
//   over every link, including the link from the zero ghost before the first
//   point of each line), the trap, c0, c2, Rabi and spin-orbit terms of
//   Eq. (5); the workgroup sums go to a partial array and a one-workgroup
//   kernel adds them in a fixed order (run-to-run reproducible): thread t
//   takes blocks t, t + 1024, ... of all twelve quantities in one pass, then
//   the wavefronts' shuffle trees and the sixteen wavefront sums in order.
// Measured at 1024^2 (one record, rocprofv3): 25.0 + 8.5 us, against 29.2 +
// 16.3 us with a per-point 64-bit index division and twelve tree reductions
// in turn (2048 workgroups: 29.6 us; one point per thread over 4096: 37.5).
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
    // what the kernel reads of hx and hy (set by its launcher, so_pattern_of):
    // pattern 1 couples neighbouring components (a = [0][1] = [1][2],
    // b = [1][0] = [2][1]), pattern 2 is diagonal (a = [0][0], b = [2][2]),
    // 0 none
    int xpat, ypat;
    cx<double> hxa, hxb, hya, hyb;
    double *partials;         // [gridDim.x][OBS_NQ]
};

// The coefficient of entry (j, jp) under an SO pattern (false: no term).
__device__ __forceinline__ bool so_entry(int pat, int j, int jp, cx<double> qa, cx<double> qb, cx<double> &q) {
    if (pat == 1) {
        if ((j == 0 && jp == 1) || (j == 1 && jp == 2)) q = qa;
        else if ((j == 1 && jp == 0) || (j == 2 && jp == 1)) q = qb;
        else return false;
        return true;
    }
    if (pat == 2) {
        if (j == 0 && jp == 0) q = qa;
        else if (j == 2 && jp == 2) q = qb;
        else return false;
        return true;
    }
    return false;
}

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
    // segments of 256 points of a row, one point per thread: the row and the
    // segment come from the workgroup-uniform segment index (no per-point
    // integer division)
    const int nseg = (a.nx + 255) / 256;
    const long long segs = (long long)a.ny * nseg;
    for (long long sg = blockIdx.x; sg < segs; sg += gridDim.x) {
        const int iy = (int)(sg / nseg), ix = (int)(sg % nseg) * 256 + (int)threadIdx.x;
        if (ix >= a.nx) continue;
        const long long p = (long long)iy * a.nx + ix;
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
        if (a.xpat | a.ypat) {
            cx<double> dxv[3], dyv[3];
#pragma unroll
            for (int jp = 0; jp < 3; ++jp) {
                const cx<R> *b = a.psi + jp * n + p;
                const cx<double> r = ix + 1 < a.nx ? ld64(b + 1) : czero<double>();
                const cx<double> l = ix >= 1 ? ld64(b - 1) : czero<double>();
                dxv[jp] = (0.5 / a.dx) * (r - l);
                dyv[jp] = czero<double>();
                if (a.dim == 2 && a.ypat) {
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
                    cx<double> q;
                    if (so_entry(a.xpat, j, jp, a.hxa, a.hxb, q)) h = cfma(q, dxv[jp], h);
                    if (so_entry(a.ypat, j, jp, a.hya, a.hyb, q)) h = cfma(q, dyv[jp], h);
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
