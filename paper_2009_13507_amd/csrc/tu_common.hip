// single-workgroup reduction kernels and their launchers
#include "common_kernels.hpp"
#include "launch.hpp"

namespace ssgp {

hipError_t launch_renorm_finalize(const Launch &c, const double *partials, int ntiles, RenormSpec sp, double *out) {
    renorm_finalize_kernel<<<1, 64, 0, c.stream>>>(partials, ntiles, sp, out);
    return hipGetLastError();
}

hipError_t launch_obs_finalize(const Launch &c, const double *partials, int nblocks, double *out) {
    obs_finalize_kernel<<<1, 1024, 0, c.stream>>>(partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_omega_accumulate(const Launch &c, const double *partials, int nrows, int nsteps, double *sums,
                                   long long n0, int steps_per_seg, int nseg, double *acc) {
    if (nsteps < 1) return hipSuccess;
    omega_step_sums_kernel<<<nsteps, 256, 0, c.stream>>>(partials, nrows, sums);
    omega_accumulate_kernel<<<1, 64, 0, c.stream>>>(sums, nsteps, n0, steps_per_seg, nseg, acc);
    return hipGetLastError();
}

hipError_t launch_batch_reset(hipStream_t s, unsigned *bar) {
    batch_reset_kernel<<<1, 64, 0, s>>>(bar);
    return hipGetLastError();
}

} // namespace ssgp
