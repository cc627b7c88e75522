// batch_host.inl -- batched API (included by ssgp.hip).
struct ssgp_batch_s {
    int n = 0;
};
extern "C" int ssgp_create_batch(int, const int *, const int *, const double *, const ssgp_params *, int, void *,
                                 const long long *, void *, ssgp_batch *out) {
    if (out) *out = nullptr;
    return fail(SSGP_EINVAL, "batched mode not built yet");
}
extern "C" int ssgp_batch_step_imag(ssgp_batch, int) { return fail(SSGP_EINVAL, "batched mode not built yet"); }
extern "C" int ssgp_batch_step_imag_serial(ssgp_batch, int) { return fail(SSGP_EINVAL, "batched mode not built yet"); }
extern "C" int ssgp_batch_observables(ssgp_batch, ssgp_obs *) { return fail(SSGP_EINVAL, "batched mode not built yet"); }
extern "C" int ssgp_destroy_batch(ssgp_batch b) { delete b; return SSGP_OK; }
