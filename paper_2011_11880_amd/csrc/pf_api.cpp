// C ABI of libpf (declared in include/pf.h): argument checks and dispatch to
// the host setup and the device layer.  No computation of the hot path
// happens here.
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "pf_internal.hpp"

namespace pf {
const char *last_error();
}

using namespace pf;

namespace {

// A network with its buses renumbered for locality: breadth-first over the
// in-service branches, from bus 0 and then from the lowest-numbered bus not
// yet reached, so neighbouring buses get nearby numbers and the states a
// wavefront gathers share cache lines.  order[k] = input bus at position k.
struct Renumbered {
    pf_network net{};
    std::vector<int32_t> order, from, to, load_bus, pv_bus, slack_bus, shunt_bus;
};

bool in_range(const int32_t *a, int32_t n, int32_t hi) {
    if (n > 0 && !a) return false;
    for (int32_t k = 0; k < n; ++k)
        if (a[k] < 0 || a[k] >= hi) return false;
    return true;
}

// False (and no renumbering) for networks whose sizes or bus indices are
// malformed: build_host_plan then reports the error on the input itself.
bool renumber(const pf_network &in, Renumbered &r) {
    const int32_t N = in.n_bus;
    if (N < 1 || in.n_branch < 0 || in.n_load < 0 || in.n_pv < 0 || in.n_slack < 0 ||
        in.n_shunt < 0)
        return false;
    if (!in_range(in.br_from, in.n_branch, N) || !in_range(in.br_to, in.n_branch, N) ||
        !in_range(in.load_bus, in.n_load, N) || !in_range(in.pv_bus, in.n_pv, N) ||
        !in_range(in.slack_bus, in.n_slack, N) || !in_range(in.shunt_bus, in.n_shunt, N))
        return false;
    std::vector<int32_t> deg(size_t(N) + 1, 0), adj;
    auto on = [&](int32_t e) { return !in.br_status || in.br_status[e]; };
    for (int32_t e = 0; e < in.n_branch; ++e)
        if (on(e)) {
            ++deg[size_t(in.br_from[e]) + 1];
            ++deg[size_t(in.br_to[e]) + 1];
        }
    for (int32_t i = 0; i < N; ++i) deg[size_t(i) + 1] += deg[size_t(i)];
    adj.resize(size_t(deg[size_t(N)]));
    std::vector<int32_t> fill(deg.begin(), deg.end() - 1);
    for (int32_t e = 0; e < in.n_branch; ++e)
        if (on(e)) {
            adj[size_t(fill[size_t(in.br_from[e])]++)] = in.br_to[e];
            adj[size_t(fill[size_t(in.br_to[e])]++)] = in.br_from[e];
        }
    r.order.clear();
    r.order.reserve(size_t(N));
    std::vector<int32_t> pos(size_t(N), -1);
    for (int32_t s = 0; s < N; ++s) {
        if (pos[size_t(s)] >= 0) continue;
        pos[size_t(s)] = int32_t(r.order.size());
        r.order.push_back(s);
        for (size_t h = r.order.size() - 1; h < r.order.size(); ++h) {
            const int32_t b = r.order[h];
            for (int32_t q = deg[size_t(b)]; q < deg[size_t(b) + 1]; ++q) {
                const int32_t c = adj[size_t(q)];
                if (pos[size_t(c)] < 0) {
                    pos[size_t(c)] = int32_t(r.order.size());
                    r.order.push_back(c);
                }
            }
        }
    }
    auto map = [&](const int32_t *a, int32_t n, std::vector<int32_t> &out) -> const int32_t * {
        out.resize(size_t(n));
        for (int32_t k = 0; k < n; ++k) out[size_t(k)] = pos[size_t(a[k])];
        return out.data();
    };
    r.net = in;
    r.net.br_from = map(in.br_from, in.n_branch, r.from);
    r.net.br_to = map(in.br_to, in.n_branch, r.to);
    r.net.load_bus = map(in.load_bus, in.n_load, r.load_bus);
    r.net.pv_bus = map(in.pv_bus, in.n_pv, r.pv_bus);
    r.net.slack_bus = map(in.slack_bus, in.n_slack, r.slack_bus);
    r.net.shunt_bus = map(in.shunt_bus, in.n_shunt, r.shunt_bus);
    return true;
}

// The host plan of n_grids networks, each renumbered first when the options
// ask for the locality order; records the plan's bus order.
int build_ordered(const pf_network *nets, int32_t n_grids, const pf_setup_opts *opt,
                  HostPlan &hp) {
    const int32_t how = opt ? opt->bus_order : PF_ORDER_INPUT;
    if (how != PF_ORDER_INPUT && how != PF_ORDER_LOCALITY)
        return fail(PF_EINVAL, "unknown bus_order %d", how);
    if (how == PF_ORDER_INPUT) {
        const int rc = build_host_plan(nets, n_grids, hp);
        if (!rc) {
            hp.bus_order.clear();
            for (const GridInfo &g : hp.grids)
                for (int32_t i = 0; i < g.N; ++i) hp.bus_order.push_back(i);
        }
        return rc;
    }
    std::vector<Renumbered> rn(static_cast<size_t>(n_grids));
    std::vector<pf_network> nn(static_cast<size_t>(n_grids));
    for (int32_t g = 0; g < n_grids; ++g) {
        if (!renumber(nets[g], rn[size_t(g)])) return build_host_plan(nets, n_grids, hp);
        nn[size_t(g)] = rn[size_t(g)].net;
    }
    const int rc = build_host_plan(nn.data(), n_grids, hp);
    if (!rc) {
        hp.bus_order_kind = PF_ORDER_LOCALITY;
        hp.bus_order.clear();
        for (const Renumbered &r : rn) hp.bus_order.insert(hp.bus_order.end(), r.order.begin(),
                                                           r.order.end());
    }
    return rc;
}

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

// Row order of the Jacobian whose diagonal holds the pivots (see
// pf_jacobian_row_order).  A control row's first slot is its V (angle)
// column, whose index equals that of the bus's Q (P) row; the two rows trade
// places.  A PV unit held at a reactive target keeps its row (its +1 at its
// own Q_g is then the diagonal) unless every unit is to be taken under
// voltage control (all_voltage), as for pivots that must survive a switch.
static void jacobian_row_order(const HostPlan &h, int32_t *order, bool all_voltage) {
    for (int64_t r = 0; r < h.n; ++r) order[r] = int32_t(r);
    for (size_t g = 0; g < size_t(h.NGt); ++g) {
        const int32_t v_row = h.gen4[4 * g];
        const int32_t th_row = h.gen4[4 * g + 2];
        if (th_row != kGenHeld || all_voltage) {
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
}

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
        rc = build_ordered(net, 1, opt, p->host);
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
        rc = build_ordered(net, 1, opt, p->host);
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
        rc = build_ordered(nets, n_grids, opt, p->host);
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

int pf_bus_order(const pf_plan *plan, int32_t *order) {
    clear_error();
    if (!plan || !order) return fail(PF_EINVAL, "NULL argument");
    const std::vector<int32_t> &o = plan->host.bus_order;
    if (!o.empty()) std::memcpy(order, o.data(), o.size() * sizeof(int32_t));
    return PF_OK;
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
    jacobian_row_order(plan->host, order, false);
    return PF_OK;
}

int pf_jacobian_switch_order(const pf_plan *plan, int32_t *order, int32_t *qv) {
    clear_error();
    if (!plan || !order) return fail(PF_EINVAL, "NULL argument");
    const HostPlan &h = plan->host;
    if (!h.q_slots)
        return fail(PF_EINVAL, "the plan was set up without q_limits (no Q_g slot in PV rows)");
    jacobian_row_order(h, order, true);
    if (qv) {
        for (size_t k = 0; k < size_t(h.NPVt); ++k) {
            const size_t g = size_t(h.pv_gen[k]);
            qv[2 * k] = h.gen4[4 * g];
            qv[2 * k + 1] = h.colidx[size_t(h.rowptr[size_t(h.gen4[4 * g])])];
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
    if (opts && (opts->q_min || opts->q_max)) {
        rc = q_limits_valid(plan->host, opts->q_min, opts->q_max,
                            opts->q_switch_tol >= 0 ? opts->q_switch_tol : 1e-9);
        if (rc) return rc;
    }
    return dev_newton(plan->host, plan->dev, x, opts, solve, user, report);
}

}  // extern "C"
