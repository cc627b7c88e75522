// single-workgroup reduction kernels and their launchers
#include "common_kernels.hpp"
#include "launch.hpp"

namespace ssgp {

hipError_t launch_renorm_finalize(const Launch &c, const double *partials, int ntiles, RenormSpec sp, double *out) {
    renorm_finalize_kernel<<<1, 64, 0, c.stream>>>(partials, ntiles, sp, out);
    return hipGetLastError();
}

hipError_t launch_obs_finalize(const Launch &c, const double *partials, int nblocks, double *out) {
    obs_finalize_kernel<<<1, 256, 0, c.stream>>>(partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_omega_accumulate(const Launch &c, const double *partials, int nrows, double *acc, int seg) {
    omega_accumulate_kernel<<<1, 256, 0, c.stream>>>(partials, nrows, acc, seg);
    return hipGetLastError();
}

hipError_t launch_batch_reset(hipStream_t s, unsigned *bar) {
    batch_reset_kernel<<<1, 64, 0, s>>>(bar);
    return hipGetLastError();
}

} // namespace ssgp
