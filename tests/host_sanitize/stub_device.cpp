// Device layer stand-in for host-only builds of libpf's setup and C ABI
// (sanitizer test): every device entry reports that no GPU is present.
#include "pf_internal.hpp"

namespace pf {
struct DevPlan {};
int dev_create(HostPlan &, DevPlan **out) {
    *out = nullptr;
    return fail(PF_EDEVICE, "no device in the host-only binary");
}
void dev_destroy(DevPlan *dp) { delete dp; }
int dev_upload_tiles(HostPlan &, DevPlan *) { return PF_OK; }
int dev_set_params(HostPlan &, DevPlan *, const double *, void *) { return PF_EDEVICE; }
int dev_eval_single(HostPlan &, DevPlan *, const double *, double *, double *, void *) {
    return PF_EDEVICE;
}
int dev_eval_batch(HostPlan &, DevPlan *, const double *, double *, double *, void *) {
    return PF_EDEVICE;
}
int dev_vjp(HostPlan &, DevPlan *, const double *, const double *, int32_t, double *, double *,
            void *) {
    return PF_EDEVICE;
}
int dev_newton(HostPlan &, DevPlan *, double *, const pf_newton_opts *, pf_linsolve_fn, void *,
               pf_newton_report *) {
    return PF_EDEVICE;
}
int dev_autotune(HostPlan &, DevPlan *, const double *, double *, double *, int32_t, void *,
                 const char *, pf_schedule *, int32_t *) {
    return PF_EDEVICE;
}
int dev_fetch_params(HostPlan &, DevPlan *) { return PF_EDEVICE; }
int q_limits_valid(const HostPlan &, const double *, const double *, double) { return PF_EDEVICE; }
}  // namespace pf
