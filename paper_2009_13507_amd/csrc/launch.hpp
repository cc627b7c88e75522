// launch.hpp -- host launchers of the kernels, one translation unit per
// kernel family and state precision (compiled in parallel).  Each returns
// hipSuccess or the HIP error of the launch.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstring>

#include "adjoint_kernels.hpp"
#include "batch_kernels.hpp"
#include "obs_kernels.hpp"
#include "step_kernels.hpp"

namespace ssgp {

struct Launch {
    hipStream_t stream;
    int ncu;  // compute units of the device
    // optional events that take the start and end time of the x-pass or
    // y-pass kernel itself (hipExtLaunchKernel), for live kernel timing
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
};

// Launches kernel<<<grid, block, lds, c.stream>>>(args), with c's timing
// events attached when it has them.
template <typename K, typename A>
inline hipError_t launch_timed(const Launch &c, K kern, dim3 grid, dim3 block, size_t lds, const A &args) {
    if (!c.ev_start) {
        kern<<<grid, block, lds, c.stream>>>(args);
        return hipGetLastError();
    }
    void *argv[] = {(void *)&args};
    return hipExtLaunchKernel((const void *)kern, grid, block, argv, lds, c.stream, c.ev_start, c.ev_stop, 0);
}

// The SO coefficient pattern of a row kernel's arguments (sopat, qa, qb)
// from qx and qxmask.  The x-derivative SO forms give one of two: sopat 1
// (S_x, S_y, the equal mixture) couples neighbouring components, with
// qa = qx[0][1] = qx[1][2] and qb = qx[1][0] = qx[2][1]; sopat 2 (S_z) is
// diagonal, qa = qx[0][0], qb = qx[2][2]; sopat 0: no SO terms.  Compared
// bitwise, so that a kernel adds the same numbers as the sum over all nine
// entries would; false for another pattern (no SO form gives one).
template <typename C> inline bool so_pattern_of(const C (&q)[9], unsigned mask, int &pat, C &qa, C &qb) {
    auto same = [](const C &p, const C &r) { return std::memcmp(&p, &r, sizeof p) == 0; };
    pat = 0;
    if (mask == 0) return true;
    if (mask == 0xAAu && same(q[1], q[5]) && same(q[3], q[7])) {  // (0,1) (1,0) (1,2) (2,1)
        pat = 1;
        qa = q[1];
        qb = q[3];
        return true;
    }
    if (mask == 0x101u) {  // (0,0) (2,2)
        pat = 2;
        qa = q[0];
        qb = q[8];
        return true;
    }
    return false;
}
template <typename A> inline bool so_pattern(A &a) { return so_pattern_of(a.qx, a.qxmask, a.sopat, a.qa, a.qb); }

// Dynamic LDS of the 1D and adjoint row kernels: all three components.
template <typename R> inline size_t row_lds(int nx, int L) { return (size_t)3 * (nx + nx / L + 1) * sizeof(cx<R>); }

template <typename R> hipError_t launch_xpass(const Launch &c, const XArgs<R> &a, int km, int rows);
template <typename R> hipError_t launch_ypass(const Launch &c, const YArgs<R> &a, int L, int tx, int threads);
template <typename R> hipError_t launch_step1d(const Launch &c, const Args1D<R> &a, int L);
template <typename R> hipError_t launch_adj_xpass(const Launch &c, const AdjXArgs<R> &a, int L, int rows);
template <typename R> hipError_t launch_pointwise(const Launch &c, const PArgs<R> &a, int blocks);
template <typename R> hipError_t launch_pso(const Launch &c, const SOArgs<R> &a);
template <typename R> hipError_t launch_scale(const Launch &c, cx<R> *psi, long long plane, const double *d, int blocks);
template <typename R> hipError_t launch_obs(const Launch &c, const ObsArgs<R> &a, int blocks);
hipError_t launch_renorm_finalize(const Launch &c, const double *partials, int ntiles, RenormSpec sp, double *out);
hipError_t launch_obs_finalize(const Launch &c, const double *partials, int nblocks, double *out);
hipError_t launch_omega_accumulate(const Launch &c, const double *partials, int nrows, int nsteps, double *sums,
                                   long long n0, int steps_per_seg, int nseg, double *acc);

// batched imaginary-time step
enum { BATCH_PHASE_X = 0, BATCH_PHASE_Y = 1, BATCH_PHASE_R = 2, BATCH_PHASE_SCALE = 3 };
template <typename R> hipError_t batch_occupancy(int *per_cu);
template <typename R> hipError_t launch_batch_persistent(hipStream_t s, const BatchArgs<R> &a, int grid);
template <typename R> hipError_t launch_batch_phase(hipStream_t s, const BatchArgs<R> &a, int phase, int apply_renorm);
hipError_t launch_batch_reset(hipStream_t s, unsigned *bar);

// chunk lengths with compiled kernels (row kernels: one 64-lane wavefront
// per line, so nx <= 64 L <= 2048) and coefficient modes (coef_mode)
#define SSGP_SWITCH_L(L, CMV, CALL)                                                                   \
    switch (L) {                                                                                      \
    case 1: return CALL(1, 0);                                                                        \
    case 2: return CALL(2, 0);                                                                        \
    case 4: return CMV == 4 ? CALL(4, 4) : CALL(4, 0);                                                \
    case 8: return CMV == 4 ? CALL(8, 4) : CMV == 8 ? CALL(8, 8) : CALL(8, 0);                        \
    case 16: return CMV == 4 ? CALL(16, 4) : CMV == 8 ? CALL(16, 8) : CALL(16, 0);                    \
    case 32: return CMV == 4 ? CALL(32, 4) : CMV == 8 ? CALL(32, 8) : CALL(32, 0);                    \
    default: return hipErrorInvalidValue;                                                             \
    }


} // namespace ssgp
