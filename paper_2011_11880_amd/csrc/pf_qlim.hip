// Reactive limits of PV generators (Section II-A): the extended formulation
// keeps a generator's Q_g variable when it stops controlling its voltage, so
// holding it at a reactive target only changes its control row from
// V - V_set to Q_g - Q_target.  Plans set up with q_limits carry both slots
// in that row; the mode lives in the generator table the kernels already
// read (see kGenHeld).  This file holds the host side: setting modes and
// the switching rule, used by one check against a state and by the Newton
// loop that checks the limits inside its iterations.
#include <cmath>
#include <vector>

#include <hip/hip_runtime.h>

#include "pf_internal.hpp"

using namespace pf;

namespace {

int need_slots(const pf_plan *plan) {
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    if (!plan->host.q_slots)
        return fail(PF_EINVAL, "the plan was set up without q_limits (no Q_g slot in PV rows)");
    return PF_OK;
}

// Write the modes into the generator table (host) and upload it.
int apply(HostPlan &hp, DevPlan *dp) {
    for (int32_t k = 0; k < hp.NPVt; ++k) {
        const size_t g = size_t(hp.pv_gen[size_t(k)]);
        const bool held = hp.pv_mode[size_t(k)] != 0;
        hp.gen4[4 * g + 2] = held ? kGenHeld : kGenVoltageSlot;
        hp.gen2[2 * g] = held ? hp.pv_qt[size_t(k)] : hp.pv_vset[size_t(k)];
    }
    if (hp.host_only || !dp) return PF_OK;
    return dev_upload_gens(hp, dp);
}

}  // namespace

namespace pf {

int q_limits_valid(const HostPlan &hp, const double *q_min, const double *q_max, double tol) {
    if (!hp.q_slots)
        return fail(PF_EINVAL, "the plan was set up without q_limits (no Q_g slot in PV rows)");
    if (hp.kind == KIND_BATCH) return fail(PF_EINVAL, "reactive-limit checks need a non-batched plan");
    if (hp.NPVt && (!q_min || !q_max)) return fail(PF_EINVAL, "q_min or q_max is NULL");
    if (!(tol >= 0.0)) return fail(PF_EINVAL, "the switching tolerance must be >= 0");
    for (size_t k = 0; k < size_t(hp.NPVt); ++k)
        if (!(q_min[k] <= q_max[k])) return fail(PF_EINVAL, "q_min[%zu] > q_max[%zu]", k, k);
    return PF_OK;
}

// The switching rule at the state xh (host copy): a unit under voltage
// control whose Q_g leaves [q_min - tol, q_max + tol] is held at the limit
// it crossed; a held unit returns to voltage control when its bus voltage
// has moved past V_set on the side that the limit no longer justifies
// (above V_set while held at q_max, below it while held at q_min).
int q_switch(HostPlan &hp, DevPlan *dp, const double *xh, const double *q_min,
             const double *q_max, double tol, int32_t *n_switched) {
    int32_t switched = 0;
    for (size_t k = 0; k < size_t(hp.NPVt); ++k) {
        const size_t g = size_t(hp.pv_gen[k]);
        const double qg = xh[size_t(hp.gen4[4 * g])];
        // the unit's bus: its V variable is the only V column of its row,
        // i.e. the first slot's column
        const double v = xh[size_t(hp.colidx[size_t(hp.gen4[4 * g + 1])])];
        if (hp.pv_mode[k] == 0) {
            if (qg > q_max[k] + tol) {
                hp.pv_mode[k] = 1;
                hp.pv_qt[k] = q_max[k];
                ++switched;
            } else if (qg < q_min[k] - tol) {
                hp.pv_mode[k] = 1;
                hp.pv_qt[k] = q_min[k];
                ++switched;
            }
        } else {
            const bool at_max = hp.pv_qt[k] == q_max[k];
            if ((at_max && v > hp.pv_vset[k] + tol) || (!at_max && v < hp.pv_vset[k] - tol)) {
                hp.pv_mode[k] = 0;
                hp.pv_qt[k] = 0.0;
                ++switched;
            }
        }
    }
    if (n_switched) *n_switched = switched;
    return switched ? apply(hp, dp) : PF_OK;
}

bool pivots_switch_safe(const HostPlan &hp, const int32_t *pivP, const int32_t *pivQ) {
    if (!hp.q_slots || hp.kind == KIND_BATCH) return false;
    std::vector<int32_t> at(size_t(hp.n));   // position of each column
    for (int64_t k = 0; k < hp.n; ++k) at[size_t(pivQ[k])] = int32_t(k);
    for (size_t k = 0; k < size_t(hp.NPVt); ++k) {
        const size_t g = size_t(hp.pv_gen[k]);
        const int32_t qg = hp.gen4[4 * g];                               // Q_g column = control row
        const int32_t v = hp.colidx[size_t(hp.rowptr[size_t(qg)])];       // V column = bus Q row
        const int32_t kq = at[size_t(qg)], kv = at[size_t(v)];
        if (!(kq < kv) || pivP[kq] != v || pivP[kv] != qg) return false;
    }
    return true;
}

}  // namespace pf

extern "C" {

int pf_set_gen_modes(pf_plan *plan, const int32_t *mode, const double *q_target) {
    clear_error();
    int rc = need_slots(plan);
    if (rc) return rc;
    HostPlan &hp = plan->host;
    const size_t NPV = size_t(hp.NPVt);
    if (NPV && !mode) return fail(PF_EINVAL, "mode is NULL");
    for (size_t k = 0; k < NPV; ++k) {
        if (mode[k] != 0 && mode[k] != 1) return fail(PF_EINVAL, "mode[%zu] must be 0 or 1", k);
        if (mode[k] == 1) {
            if (!q_target) return fail(PF_EINVAL, "q_target is NULL but mode[%zu] is 1", k);
            if (!std::isfinite(q_target[k]))
                return fail(PF_EINVAL, "q_target[%zu] is not finite", k);
        }
    }
    for (size_t k = 0; k < NPV; ++k) {
        hp.pv_mode[k] = mode[k];
        hp.pv_qt[k] = mode[k] ? q_target[k] : 0.0;
    }
    return apply(plan->host, plan->dev);
}

int pf_get_gen_modes(const pf_plan *plan, int32_t *mode, double *q_target) {
    clear_error();
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    const HostPlan &hp = plan->host;
    for (size_t k = 0; k < size_t(hp.NPVt); ++k) {
        if (mode) mode[k] = hp.pv_mode.empty() ? 0 : hp.pv_mode[k];
        if (q_target) q_target[k] = hp.pv_qt.empty() ? 0.0 : hp.pv_qt[k];
    }
    return PF_OK;
}

int pf_q_limit_check(pf_plan *plan, const double *x, const double *q_min, const double *q_max,
                     double tol, int32_t *n_switched, void *stream) {
    clear_error();
    int rc = need_slots(plan);
    if (rc) return rc;
    HostPlan &hp = plan->host;
    if (hp.host_only || !plan->dev) return fail(PF_EINVAL, "plan is host-only");
    if (hp.kind == KIND_BATCH) return fail(PF_EINVAL, "pf_q_limit_check needs a non-batched plan");
    if (!x) return fail(PF_EINVAL, "NULL argument");
    rc = q_limits_valid(hp, q_min, q_max, tol);
    if (rc) return rc;
    std::vector<double> xh(size_t(hp.n));
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return fail(PF_EDEVICE, "hipGetDevice failed");
    if (prev != hp.device && hipSetDevice(hp.device) != hipSuccess)
        return fail(PF_EDEVICE, "cannot select device %d", hp.device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(xh.data(), x, xh.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (prev != hp.device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail(PF_EDEVICE, "copy of x failed: %s", hipGetErrorString(e));
    return q_switch(hp, plan->dev, xh.data(), q_min, q_max, tol, n_switched);
}

}  // extern "C"
