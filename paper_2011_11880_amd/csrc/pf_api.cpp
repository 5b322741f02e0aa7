// C ABI of libpf (declared in include/pf.h): argument checks and dispatch to
// the host setup and the device layer.  No computation of the hot path
// happens here.
#include <cstdlib>
#include <cstring>
#include <new>

#include "pf_internal.hpp"

namespace pf {
const char *last_error();
}

using namespace pf;

namespace {

int finish_setup(pf_plan *p, const pf_setup_opts *opt, pf_plan **out) {
    int rc = normalise_schedule(p->host, opt ? &opt->sched : nullptr, p->host.sched);
    if (rc) return rc;
    build_tiles(p->host);
    p->host.host_only = opt && opt->host_only;
    p->host.device = opt ? opt->device : -1;
    if (!p->host.host_only) {
        rc = dev_create(p->host, &p->dev);
        if (rc) return rc;
    }
    *out = p;
    return PF_OK;
}

int check_eval(const pf_plan *plan, bool want_batch) {
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    if (plan->host.host_only || !plan->dev) return fail(PF_EINVAL, "plan is host-only");
    if (want_batch && plan->host.kind != KIND_BATCH)
        return fail(PF_EINVAL, "pf_eval_batch needs a batched plan");
    if (!want_batch && plan->host.kind == KIND_BATCH)
        return fail(PF_EINVAL, "batched plans are evaluated with pf_eval_batch");
    return PF_OK;
}

}  // namespace

extern "C" {

const char *pf_last_error(void) { return last_error(); }

int pf_setup(const pf_network *net, const pf_setup_opts *opt, pf_plan **out) {
    clear_error();
    if (!out) return fail(PF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!net) return fail(PF_EINVAL, "network is NULL");
    pf_plan *p = new (std::nothrow) pf_plan();
    if (!p) return fail(PF_ENOMEM, "host allocation failed");
    int rc;
    try {
        p->host.q_slots = (opt && opt->q_limits) ? 1 : 0;
        rc = build_host_plan(net, 1, p->host);
    } catch (const std::bad_alloc &) {
        rc = fail(PF_ENOMEM, "host allocation failed");
    }
    if (!rc) rc = finish_setup(p, opt, out);
    if (rc) delete p;
    return rc;
}

int pf_setup_batch(const pf_network *net, const pf_batch_spec *spec, const pf_setup_opts *opt,
                   pf_plan **out) {
    clear_error();
    if (!out) return fail(PF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!net) return fail(PF_EINVAL, "network is NULL");
    pf_plan *p = new (std::nothrow) pf_plan();
    if (!p) return fail(PF_ENOMEM, "host allocation failed");
    int rc;
    try {
        p->host.q_slots = (opt && opt->q_limits) ? 1 : 0;
        rc = build_host_plan(net, 1, p->host);
        if (!rc) rc = attach_batch(spec, p->host);
    } catch (const std::bad_alloc &) {
        rc = fail(PF_ENOMEM, "host allocation failed");
    }
    if (!rc) rc = finish_setup(p, opt, out);
    if (rc) delete p;
    return rc;
}

int pf_setup_multi(const pf_network *nets, int32_t n_grids, const pf_setup_opts *opt,
                   pf_plan **out) {
    clear_error();
    if (!out) return fail(PF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!nets || n_grids < 1) return fail(PF_EINVAL, "need n_grids >= 1 networks");
    pf_plan *p = new (std::nothrow) pf_plan();
    if (!p) return fail(PF_ENOMEM, "host allocation failed");
    int rc;
    try {
        p->host.q_slots = (opt && opt->q_limits) ? 1 : 0;
        rc = build_host_plan(nets, n_grids, p->host);
        p->host.kind = KIND_MULTI;
    } catch (const std::bad_alloc &) {
        rc = fail(PF_ENOMEM, "host allocation failed");
    }
    if (!rc) rc = finish_setup(p, opt, out);
    if (rc) delete p;
    return rc;
}

void pf_destroy(pf_plan *plan) {
    if (!plan) return;
    dev_destroy(plan->dev);
    delete plan;
}

int pf_info(const pf_plan *plan, int64_t *n, int64_t *nnz) {
    clear_error();
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    if (n) *n = plan->host.n;
    if (nnz) *nnz = plan->host.nnz;
    return PF_OK;
}

int pf_info_ex(const pf_plan *plan, pf_info_t *info) {
    clear_error();
    if (!plan || !info) return fail(PF_EINVAL, "NULL argument");
    const HostPlan &h = plan->host;
    std::memset(info, 0, sizeof *info);
    info->n = h.n;
    info->nnz = h.nnz;
    info->n_params = h.n_params();
    info->n_entries = h.n_y;
    info->n_bus = h.Nt;
    info->n_branch = h.Bt;
    info->n_load = h.NLt;
    info->n_pv = h.NPVt;
    info->n_slack = h.NSt;
    info->n_shunt = h.NSHt;
    info->n_inst = h.n_inst;
    info->inst_stride = h.panels ? 64 : h.ld;
    info->layout = h.panels ? PF_LAYOUT_PANELS : PF_LAYOUT_ROWS;
    info->n_grids = int32_t(h.grids.size());
    info->n_tiles = h.n_tiles();
    info->kind = h.kind;
    return PF_OK;
}

int pf_info_multi(const pf_plan *plan, int64_t *x_off, int64_t *j_off) {
    clear_error();
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    const HostPlan &h = plan->host;
    const size_t G = h.grids.size();
    for (size_t g = 0; g < G; ++g) {
        if (x_off) x_off[g] = h.grids[g].xoff;
        if (j_off) j_off[g] = h.grids[g].joff;
    }
    if (x_off) x_off[G] = h.n;
    if (j_off) j_off[G] = h.nnz;
    return PF_OK;
}

int pf_pattern(const pf_plan *plan, int32_t *rowptr, int32_t *colidx) {
    clear_error();
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    const HostPlan &h = plan->host;
    if (rowptr) std::memcpy(rowptr, h.rowptr.data(), h.rowptr.size() * sizeof(int32_t));
    if (colidx) std::memcpy(colidx, h.colidx.data(), h.colidx.size() * sizeof(int32_t));
    return PF_OK;
}

int pf_jacobian_row_order(const pf_plan *plan, int32_t *order) {
    clear_error();
    if (!plan || !order) return fail(PF_EINVAL, "NULL argument");
    const HostPlan &h = plan->host;
    for (int64_t r = 0; r < h.n; ++r) order[r] = int32_t(r);
    // a control row's first slot is its V (angle) column, whose index equals
    // that of the bus's Q (P) row
    for (size_t g = 0; g < size_t(h.NGt); ++g) {
        const int32_t v_row = h.gen4[4 * g];
        const int32_t th_row = h.gen4[4 * g + 2];
        // a unit held at a reactive target keeps its row: its +1 sits on
        // its own Q_g column, the diagonal
        if (th_row != kGenHeld) {
            const int32_t q_row = h.colidx[size_t(h.rowptr[size_t(v_row)])];
            order[q_row] = v_row;
            order[v_row] = q_row;
        }
        if (th_row >= 0) {
            const int32_t p_row = h.colidx[size_t(h.rowptr[size_t(th_row)])];
            order[p_row] = th_row;
            order[th_row] = p_row;
        }
    }
    return PF_OK;
}

int pf_eval(pf_plan *plan, const double *x, double *F, double *Jval, void *stream) {
    clear_error();
    int rc = check_eval(plan, false);
    if (rc) return rc;
    if (!x) return fail(PF_EINVAL, "x is NULL");
    if (!F && !Jval) return fail(PF_EINVAL, "F and Jval are both NULL");
    return dev_eval_single(plan->host, plan->dev, x, F, Jval, stream);
}

int pf_eval_residual(pf_plan *plan, const double *x, double *F, void *stream) {
    if (!F) return fail(PF_EINVAL, "F is NULL");
    return pf_eval(plan, x, F, nullptr, stream);
}

int pf_eval_jacobian(pf_plan *plan, const double *x, double *Jval, void *stream) {
    if (!Jval) return fail(PF_EINVAL, "Jval is NULL");
    return pf_eval(plan, x, nullptr, Jval, stream);
}

int pf_eval_batch(pf_plan *plan, const double *X, double *F, double *Jval, void *stream) {
    clear_error();
    int rc = check_eval(plan, true);
    if (rc) return rc;
    if (!X) return fail(PF_EINVAL, "X is NULL");
    if (!F && !Jval) return fail(PF_EINVAL, "F and Jval are both NULL");
    return dev_eval_batch(plan->host, plan->dev, X, F, Jval, stream);
}

int pf_set_params(pf_plan *plan, const double *params, void *stream) {
    clear_error();
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    if (plan->host.host_only || !plan->dev) return fail(PF_EINVAL, "plan is host-only");
    if (!params && plan->host.n_params() > 0) return fail(PF_EINVAL, "params is NULL");
    const int rc = dev_set_params(plan->host, plan->dev, params, stream);
    if (!rc) plan->host.params_stale = true;
    return rc;
}

int pf_vjp(pf_plan *plan, const double *x, const double *W, int32_t k, double *gx,
           double *gparam, void *stream) {
    clear_error();
    int rc = check_eval(plan, false);
    if (rc) return rc;
    if (!x || !W) return fail(PF_EINVAL, "x or W is NULL");
    if (k < 1 || k > 1024) return fail(PF_EINVAL, "k must be in [1, 1024]");
    if (!gx && !gparam) return fail(PF_EINVAL, "gx and gparam are both NULL");
    return dev_vjp(plan->host, plan->dev, x, W, k, gx, gparam, stream);
}

int pf_get_schedule(const pf_plan *plan, pf_schedule *sched) {
    clear_error();
    if (!plan || !sched) return fail(PF_EINVAL, "NULL argument");
    *sched = plan->host.sched;
    return PF_OK;
}

int pf_set_schedule(pf_plan *plan, const pf_schedule *sched) {
    clear_error();
    if (!plan || !sched) return fail(PF_EINVAL, "NULL argument");
    pf_schedule s{};
    int rc = normalise_schedule(plan->host, sched, s);
    if (rc) return rc;
    const int32_t old_tiles = plan->host.sched.tile_entries;
    plan->host.sched = s;
    if (s.tile_entries != old_tiles || plan->host.tiles.empty()) {
        build_tiles(plan->host);
        if (plan->dev) return dev_upload_tiles(plan->host, plan->dev);
    }
    return PF_OK;
}

int pf_autotune_cached(pf_plan *plan, const double *x, double *F, double *Jval, int32_t reps,
                       void *stream, const char *cache_path, pf_schedule *best, int32_t *hit) {
    clear_error();
    if (hit) *hit = 0;
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    if (plan->host.host_only || !plan->dev) return fail(PF_EINVAL, "plan is host-only");
    if (!x || (!F && !Jval)) return fail(PF_EINVAL, "need x and at least one output");
    if (reps < 1) return fail(PF_EINVAL, "reps must be >= 1");
    return dev_autotune(plan->host, plan->dev, x, F, Jval, reps, stream, cache_path, best, hit);
}

int pf_autotune(pf_plan *plan, const double *x, double *F, double *Jval, int32_t reps,
                void *stream, pf_schedule *best) {
    return pf_autotune_cached(plan, x, F, Jval, reps, stream, std::getenv("PF_TUNE_CACHE"), best,
                              nullptr);
}

int pf_newton(pf_plan *plan, double *x, const pf_newton_opts *opts, pf_linsolve_fn solve,
              void *user, pf_newton_report *report) {
    clear_error();
    int rc = check_eval(plan, false);
    if (rc) return rc;
    if (!x || !solve) return fail(PF_EINVAL, "x or solve is NULL");
    if (opts && opts->max_iter > 64) return fail(PF_EINVAL, "max_iter must be <= 64");
    return dev_newton(plan->host, plan->dev, x, opts, solve, user, report);
}

}  // extern "C"
