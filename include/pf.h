/*
 * pf.h - C ABI of the MI355X power-flow evaluation library (libpf.so).
 *
 * The library evaluates, in FP64 on a gfx950 GPU, the hot path of Newton
 * power flow as formulated in Section II-A of Cui, Li & Fang, "Effective
 * Parallelism for Equation and Jacobian Evaluation in Large-Scale Power Flow
 * Calculation":
 *
 *   g(y) = 0                                   (eq. 1)
 *   g = [g_p, g_q, g_V, g_theta]               (eq. 2: P and Q mismatch per
 *                                               bus, voltage-control error per
 *                                               generator, angle-control error
 *                                               per slack)
 *   y = [theta, V, Q_g, P_s]                   (eq. 3: bus angles, bus voltage
 *                                               magnitudes, reactive output of
 *                                               every generator (PV units first,
 *                                               then slacks), slack active output)
 *
 * Models (Section II-A): bus, constant-power PQ load, PV generator, slack
 * generator, line (pi-model) and two-winding transformer (ideal tap ratio t
 * and phase shift phi on the from side), shunt admittance.  Line injections
 * are computed per line and summed at the two buses (eq. 4 is the t = 1,
 * phi = 0 case of the from/to active power).
 *
 * Sign convention: a bus row is the power leaving the bus into branches,
 * shunts and loads minus the power produced there; g_V = V - V_set and
 * g_theta = theta - theta_set.  Units are per unit; angles in y are radians;
 * transformer phase shifts are given in degrees.
 *
 * Sizes: n = 2N + N_g + N_s variables and equations; the Jacobian has the
 * fixed CSR pattern of nnz = 4N + 8B_u + 2N_g + 2N_s entries, where B_u is the
 * number of distinct connected bus pairs (parallel branches share entries).
 * Row P_i holds [theta cols of sorted({i} U adj(i))][V cols, same order]
 * [P_s col if a slack sits at i]; row Q_i the same with the Q_g col of the
 * generator at i; every control row has a single +1 entry.  Columns are
 * sorted within each row.
 *
 * Conventions for every entry point:
 *  - Return value: PF_OK (0) or a negative PF_E* status; pf_last_error()
 *    then returns a thread-local message (valid until the next call on the
 *    same thread).
 *  - Pointers named "host" are read (or written) only during the call; the
 *    caller keeps ownership.  Device pointers (x, F, Jval, X, W, gx, gparam,
 *    params) are caller-owned GPU buffers on the plan's device; the library
 *    never frees or retains them.
 *  - Evaluation calls are asynchronous on the given HIP stream (NULL = the
 *    default stream), allocate nothing, and check their arguments
 *    synchronously; faults inside a kernel surface at the caller's next
 *    synchronisation.  Evaluation calls (pf_eval*, pf_vjp) only read the
 *    plan's device data, so several may run at once on different streams;
 *    pf_set_params, pf_set_schedule, pf_autotune and pf_newton must not
 *    overlap any other call on the same plan.
 *  - All floating-point data are IEEE FP64, all indices int32, 0-based.
 *  - Results are deterministic: every bus sum is a fixed-order left fold, no
 *    floating-point atomics are used, and every schedule gives bit-identical
 *    outputs.
 */
#ifndef PF_H
#define PF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PF_OK 0
#define PF_EINVAL (-1)   /* bad argument or malformed network data */
#define PF_ETOPO (-2)    /* self-loop, two voltage controllers on one bus, isolated bus */
#define PF_EDEVICE (-3)  /* HIP runtime error, or no usable GPU */
#define PF_ENOMEM (-4)   /* device or host allocation failed */
#define PF_ESOLVE (-5)   /* linear-solve callback failed (e.g. singular Jacobian) */
#define PF_ENOCONV (-6)  /* Newton reached max_iter without convergence */

/*
 * One network, host structure of arrays (Section II-A models).
 *   br_from/br_to      branch terminal buses; the transformer is on br_from
 *   br_r, br_x         series resistance and reactance (not both zero)
 *   br_b               total line charging susceptance, split b/2 per end
 *   br_tap             off-nominal ratio (> 0; 1 for a line)
 *   br_shift_deg       phase shift in degrees (0 for a line)
 *   br_status          1 in service / 0 out of service; NULL = all in service
 *   load_*             constant-power loads; several may share a bus
 *   pv_*               PV units: bus, active setpoint P, voltage setpoint V
 *   slack_*            slack units: bus, voltage setpoint, angle setpoint (rad)
 *   shunt_*            shunt admittance g + jb to ground; several may share a bus
 * A bus carries at most one generator (PV or slack).  Array pointers for
 * zero-length groups may be NULL.
 */
typedef struct pf_network {
    int32_t n_bus, n_branch, n_load, n_pv, n_slack, n_shunt;
    const int32_t *br_from, *br_to;
    const double *br_r, *br_x, *br_b, *br_tap, *br_shift_deg;
    const int32_t *br_status;
    const int32_t *load_bus;
    const double *load_p, *load_q;
    const int32_t *pv_bus;
    const double *pv_p, *pv_v;
    const int32_t *slack_bus;
    const double *slack_v, *slack_theta;
    const int32_t *shunt_bus;
    const double *shunt_g, *shunt_b;
} pf_network;

/*
 * Launch schedule.  A zero field means "library default".  Any schedule
 * yields bit-identical results; only speed differs.
 *   tile_entries    single-instance kernel: admittance entries per wavefront
 *                   tile (multiple of 64; rows are never split)
 *   waves_per_block wavefronts per workgroup, 1..8
 *   grid_blocks     persistent grid size in workgroups, each wavefront
 *                   walking a contiguous range of work; -1 = no persistence
 *                   (one tile / work item per wavefront, grid sized to the
 *                   work); 0 = library default
 *   batch_buses     batched kernel: buses per work item
 *   batch_order     batched kernel bus order: 1 natural, 2 breadth-first
 *                   from the lowest-numbered bus
 *   xcd_remap       1: give each of the 8 XCDs a contiguous range of work
 *                   items (L2 locality), 2: round-robin (hardware order)
 *   batch_group     batched kernel work order: number of instance chunks
 *                   of a bus processed back to back (1..64); a chunk is 64
 *                   instances, or 128 where two instances share a lane
 *                   (plans without overlays whose instance count and pitch
 *                   are even).  Work runs over
 *                   groups of this many chunks, and inside a group bus by
 *                   bus: 1 = one chunk at a time over all buses (small state
 *                   footprint per bus, good cache reuse between neighbouring
 *                   buses); >= the chunk count = bus by bus (whole instance
 *                   rows of the outputs written together)
 */
typedef struct pf_schedule {
    int32_t tile_entries;
    int32_t waves_per_block;
    int32_t grid_blocks;
    int32_t batch_buses;
    int32_t batch_order;
    int32_t xcd_remap;
    int32_t batch_group;
} pf_schedule;

/*
 * Setup options (NULL = defaults).
 *   host_only  1: build and validate host structures only (pattern, sizes,
 *              schedule) without touching a GPU; evaluation calls then fail
 *              with PF_EINVAL.  Used for CPU-side checks.
 *   device     HIP device ordinal; -1 = the calling thread's current device
 *   sched      initial schedule
 *   q_limits   1: every PV generator's control row also holds its Q_g column
 *              (the row then has two slots, V then Q_g; nnz grows by the
 *              number of PV units), so that pf_set_gen_modes can hold the
 *              generator at a reactive target without changing the pattern
 *   bus_order  PF_ORDER_INPUT (0): the plan keeps the network's bus numbers.
 *              PF_ORDER_LOCALITY (1): the plan numbers each grid's buses
 *              breadth-first over its in-service branches (from bus 0, then
 *              from the lowest-numbered bus not yet reached), so that
 *              neighbouring buses sit close together in every bus-indexed
 *              array: the single-instance kernel's state gathers then share
 *              cache lines (Section II-D's point about contiguous data).
 *              Every bus-indexed array the library takes or returns (the
 *              angle and voltage blocks of x and F, the rows and columns of
 *              the pattern, bus lists) is then in the plan's order;
 *              pf_bus_order gives the map.  Branch, load and generator
 *              numbering (and so the parameter vector and the generator
 *              blocks of x and F) are unchanged.
 */
#define PF_ORDER_INPUT 0
#define PF_ORDER_LOCALITY 1
typedef struct pf_setup_opts {
    int32_t host_only;
    int32_t device;
    pf_schedule sched;
    int32_t q_limits;
    int32_t bus_order;
} pf_setup_opts;

typedef struct pf_plan pf_plan;

/*
 * Build a single-instance plan: validate the network, build the fixed
 * Jacobian pattern, the per-bus admittance rows and every setup-time
 * coefficient, and upload them (Section III: evaluation calls allocate
 * nothing; the paper's per-call triplet assembly is replaced by the fixed
 * pattern).  On success *out owns all device memory of the plan.
 * Errors: PF_EINVAL (NULL pointers, sizes < 0, n_bus < 1, index out of
 * range, r = x = 0, tap <= 0, non-finite data), PF_ETOPO (self-loop, two
 * generators on one bus, a bus without in-service branches when n_bus > 1),
 * PF_EDEVICE, PF_ENOMEM.
 */
int pf_setup(const pf_network *net, const pf_setup_opts *opt, pf_plan **out);

/*
 * Batch specification over one base network (scenarios and N-1 cases; the
 * paper runs such jobs as separate processes, Section II-C / IV-C).
 *   n_inst       number of instances (>= 1)
 *   load_scale   host [n_inst][n_load]; instance k's load l draws
 *                scale * (P_l, Q_l); NULL = all 1
 *   pv_scale     host [n_inst][n_pv]; scales PV active setpoints; NULL = all 1
 *   outage       host [n_inst]; branch taken out of service in instance k,
 *                or -1; the branch must be in service in the base network.
 *                Its Jacobian slots keep their place in the shared pattern
 *                and receive 0 when nothing else connects the bus pair.
 *   inst_stride  row pitch, in elements, of the batched X, F and Jval arrays
 *                (>= n_inst; 0 = n_inst).  Padding rows to a multiple of 16
 *                instances aligns every 64-instance segment to 128 B; the
 *                padding columns are neither read for results nor written.
 *   layout       PF_LAYOUT_ROWS (0): X[n][ld], F[n][ld], Jval[nnz][ld];
 *                PF_LAYOUT_PANELS (1): instances in panels of 64,
 *                X[P][n][64], F[P][n][64], Jval[P][nnz][64] with
 *                P = ceil(n_inst / 64); instance k lives in panel k / 64,
 *                column k % 64 (inst_stride is ignored).  Each panel is one
 *                contiguous block, so a pass over one panel streams its
 *                outputs and keeps its state slice cache-resident.
 */
#define PF_LAYOUT_ROWS 0
#define PF_LAYOUT_PANELS 1
typedef struct pf_batch_spec {
    int32_t n_inst;
    const double *load_scale;
    const double *pv_scale;
    const int32_t *outage;
    int32_t inst_stride;
    int32_t layout;
} pf_batch_spec;

/*
 * Build a batched plan: n_inst instances that share the base network's
 * pattern and data, each with its own state and overlay.  All batched
 * arrays are instance-fastest with row pitch ld = inst_stride:
 * X[n][ld], F[n][ld], Jval[nnz][ld] (instance k of variable i at i*ld + k).
 * Errors as pf_setup, plus PF_EINVAL for a bad spec.
 */
int pf_setup_batch(const pf_network *net, const pf_batch_spec *spec,
                   const pf_setup_opts *opt, pf_plan **out);

/*
 * Build a multi-grid plan over n_grids independent networks evaluated in
 * one launch.  Their state, residual and Jacobian vectors are concatenated
 * in grid order (block-diagonal system); pf_info_multi gives the offsets.
 * Errors as pf_setup (for any grid), PF_EINVAL for n_grids < 1.
 */
int pf_setup_multi(const pf_network *nets, int32_t n_grids,
                   const pf_setup_opts *opt, pf_plan **out);

/* Sizes: n (state length of one instance, or of the concatenation) and nnz. */
int pf_info(const pf_plan *plan, int64_t *n, int64_t *nnz);

/* Extended sizes of a plan. */
typedef struct pf_info_t {
    int64_t n, nnz;        /* per instance (batch) or total (multi) */
    int64_t n_params;      /* length of the parameter vector (pf_set_params) */
    int64_t n_entries;     /* admittance-row entries (N + 2 B_u) */
    int32_t n_bus, n_branch, n_load, n_pv, n_slack, n_shunt;
    int32_t n_inst;        /* 1 unless batched */
    int32_t inst_stride;   /* batched row pitch (elements); 1 unless batched */
    int32_t layout;        /* batched layout: PF_LAYOUT_ROWS or PF_LAYOUT_PANELS */
    int32_t n_grids;       /* 1 unless multi-grid */
    int32_t n_tiles;       /* wavefront tiles of the single-instance kernel */
    int32_t kind;          /* 0 single, 1 batched, 2 multi-grid */
} pf_info_t;
int pf_info_ex(const pf_plan *plan, pf_info_t *info);

/* Host copies of per-grid offsets into the concatenated vectors of a
 * multi-grid plan: x_off and j_off each receive n_grids + 1 entries. */
int pf_info_multi(const pf_plan *plan, int64_t *x_off, int64_t *j_off);

/* Host copy of the plan's bus order: order[k] (host [total buses]) is the
 * input bus (numbered within its grid) that plan bus k of that grid stands
 * for; the identity unless the plan was set up with PF_ORDER_LOCALITY.  For
 * a state y in input numbering, the plan's x has x[k] = y[order[k]] and
 * x[N + k] = y[N + order[k]] per grid, the generator entries unchanged. */
int pf_bus_order(const pf_plan *plan, int32_t *order);

/* Host copy of the fixed CSR pattern: rowptr[n + 1], colidx[nnz]. */
int pf_pattern(const pf_plan *plan, int32_t *rowptr, int32_t *colidx);

/*
 * A row order of the Jacobian (host output [n]: row k of the reordered
 * matrix is row order[k]) under which every diagonal entry is a structural
 * nonzero that no branch outage can remove: each generator's voltage-control
 * row (+1 at its bus voltage) trades places with its bus's Q row (whose -1 at
 * Q_g then sits on the diagonal), each slack angle row with its bus's P row;
 * the other diagonals are the buses' own sums over their branches.  A PV
 * unit held at a reactive target (pf_set_gen_modes) keeps its row, whose +1
 * at its own Q_g is then the diagonal; the order follows the current modes.
 * An LU
 * that pivots on the diagonal of the reordered matrix therefore keeps usable
 * pivots for every instance of a batch (outages, scenarios) and for later
 * Newton iterates.  Works on host-only plans.
 */
int pf_jacobian_row_order(const pf_plan *plan, int32_t *order);

/*
 * Row order and pivot pairs for an LU whose pivots stay usable when PV units
 * switch between voltage control and a held reactive output inside the
 * Newton iterations (Section II-A: the extended formulation keeps Q_g as a
 * variable in both modes, so a switch only moves the control row's +1 from
 * the bus voltage column to the Q_g column; a plan set up with q_limits
 * carries both slots).  order [n] (host output): as pf_jacobian_row_order
 * with every PV unit taken under voltage control, whatever its current mode:
 * the bus's Q row sits on the unit's Q_g column (its -1 there in both modes)
 * and the unit's control row on the bus voltage column.  qv [2 * n_pv] (host
 * output, may be NULL): qv[2k] = the Q_g column of PV unit k (also the index
 * of its control row), qv[2k + 1] = its bus voltage column (also the index
 * of the bus's Q row).  Under this pairing a held unit's control row takes
 * its voltage pivot from the bus's Q row, which elimination adds to it once
 * the Q_g column is gone: an LU that eliminates column qv[2k] before column
 * qv[2k + 1] has the pivots of a bus without a generator there when the unit
 * is held and a unit pivot when it is not.  pf_batch_lu_create checks this
 * for every PV unit, and pf_newton_batch then accepts reactive limits.
 * Errors: PF_EINVAL (NULL order or plan, plan set up without q_limits).
 * Works on host-only plans.
 */
int pf_jacobian_switch_order(const pf_plan *plan, int32_t *order, int32_t *qv);

/*
 * Residual F(x) (task 1 of the Newton loop, Section I).  x, F: device [n].
 * Errors: PF_EINVAL (NULL buffer, batched plan, host-only plan), PF_EDEVICE.
 */
int pf_eval_residual(pf_plan *plan, const double *x, double *F, void *stream);

/* Jacobian values (task 2): writes all nnz values of Jval (device [nnz]) in
 * pf_pattern order, constants and explicit zeros included. */
int pf_eval_jacobian(pf_plan *plan, const double *x, double *Jval, void *stream);

/* Fused residual + Jacobian in one launch; F or Jval may be NULL (not both). */
int pf_eval(pf_plan *plan, const double *x, double *F, double *Jval, void *stream);

/* Batched fused evaluation: X, F (nullable) and Jval (nullable, not both
 * NULL) in the plan's batched layout (rows of pitch inst_stride, or panels
 * of 64 instances).  Batched plans only. */
int pf_eval_batch(pf_plan *plan, const double *X, double *F, double *Jval,
                  void *stream);

/*
 * Replace the differentiable network data from a device vector laid out as
 * [r(B), x(B), b(B), tap(B), shift_deg(B), load_p(N_L), load_q(N_L)]
 * (n_params doubles; concatenated in grid order for multi-grid plans) and
 * rebuild every derived coefficient on the device.  The pattern is fixed:
 * r = x = 0 or tap <= 0 are not checked here and yield non-finite values.
 * The fast decoupled matrices (pf_fdlf_matrices, pf_fdlf_create) are built
 * on the host; the first such call after pf_set_params waits for the device
 * and copies the new parameters back before building them.
 */
int pf_set_params(pf_plan *plan, const double *params, void *stream);

/*
 * Adjoint: for k cotangents W (device [n][k], cotangent-fastest) computes
 *   gx     = J(x)^T W                              device [n][k]
 *   gparam = (dF/dp)^T W  for p as in pf_set_params device [n_params][k]
 * (shift gradient per degree, the unit the data is given in).  Either
 * output may be NULL.  Single-instance plans only; 1 <= k <= 1024.
 */
int pf_vjp(pf_plan *plan, const double *x, const double *W, int32_t k,
           double *gx, double *gparam, void *stream);

/* Current and new launch schedule (setting may reallocate the plan's
 * schedule tables; not an evaluation call). */
int pf_get_schedule(const pf_plan *plan, pf_schedule *sched);
int pf_set_schedule(pf_plan *plan, const pf_schedule *sched);

/*
 * Autotuner: coordinate descent over the plan kernel's schedules (tile
 * size, work-item size, bus order, instance-chunk grouping, waves per
 * block, grid size, XCD mapping), each candidate timed on the given buffers
 * (single: x, F, Jval as pf_eval; batched: as pf_eval_batch) as the median
 * of reps >= 1 launches; a candidate must be 1.5% faster than the best so
 * far to replace it.  The winner becomes the plan's schedule and is
 * returned in *best (nullable).  Synchronises the stream.  Every schedule
 * gives bit-identical outputs.
 *
 * Tune cache: with cache_path non-NULL and non-empty, the text file there
 * is searched first for a line keyed by the GPU (architecture, compute
 * units), the kernel source the library was built from and the plan's
 * shape (kind, bus order, sizes, grids, instances, pitch, layout, overlays,
 * outputs asked for).  On a hit that schedule is applied without timing anything
 * and *hit (nullable) is set to 1; on a miss the search runs and appends its
 * result to the file (PF_EINVAL if the file cannot be written).
 * pf_autotune is pf_autotune_cached with the path taken from the
 * environment variable PF_TUNE_CACHE (unset or empty: no cache).
 */
int pf_autotune(pf_plan *plan, const double *x, double *F, double *Jval,
                int32_t reps, void *stream, pf_schedule *best);
int pf_autotune_cached(pf_plan *plan, const double *x, double *F, double *Jval,
                       int32_t reps, void *stream, const char *cache_path,
                       pf_schedule *best, int32_t *hit);

/*
 * Newton power flow (tasks 1-4, Section I): full steps
 *   x <- x - J(x)^{-1} F(x)   until ||F||_inf < tol or max_iter steps.
 * The sparse solve (task 3) is the caller's: the library copies J values and
 * F to host and calls solve(user, n, rowptr, colidx, Jval_host, rhs_host,
 * dx_host), which must fill dx and return 0 (non-zero -> PF_ESOLVE).
 * x: device [n], updated in place.  Runs on the default stream and
 * synchronises; work queued on other (non-blocking) streams that writes x
 * must be complete before the call.  report (nullable) receives iteration counts, per-iteration
 * norms (up to 64) and times.  Returns PF_ENOCONV if max_iter is reached.
 *
 * Reactive limits inside the iterations (Section II-A: the extended
 * formulation keeps one set of equations whether a PV unit controls its
 * voltage or is held at a reactive target, so the limits may be checked at
 * any iterate): with q_min and q_max
 * set (host [n_pv], read during the call; plan set up with q_limits = 1,
 * not batched), at every iterate x_k whose ||F||_inf is below
 * q_check_below the switching rule of pf_q_limit_check (tolerance
 * q_switch_tol) is applied to x_k; after a switch F and J are evaluated
 * again at x_k under the new modes before the step.  norm[k] is then the
 * norm under the modes in force after the check, switched[k] the number of
 * units that changed mode at x_k, and convergence needs ||F||_inf < tol
 * under modes that the check at that iterate left unchanged.  The modes
 * stay on the plan (pf_get_gen_modes).  A switch moves the held row's
 * nonzero from the V column to the Q_g column.  pf_newton refactorises on
 * the host each step and follows it; pf_newton_batch (on a plan of one
 * instance: limits are per plan, not per instance) and pf_newton_device
 * follow it when their factorisation was made along pivots that pair and
 * order every PV unit's rows as pf_jacobian_switch_order describes.  Other
 * fixed pivots, and the constant B' / B'' of pf_fdlf_solve, cannot follow
 * it: those return PF_EINVAL when q_min or q_max is set.
 */
typedef int (*pf_linsolve_fn)(void *user, int64_t n, const int32_t *rowptr,
                              const int32_t *colidx, const double *Jval_host,
                              const double *rhs_host, double *dx_host);

typedef struct pf_newton_opts {
    double tol;            /* <= 0: 1e-10 */
    int32_t max_iter;      /* <= 0: 10 */
    const double *q_min;   /* both NULL: no limit checks (pf_newton, pf_newton_batch) */
    const double *q_max;
    double q_check_below;  /* <= 0: 1e-3 */
    double q_switch_tol;   /* < 0: 1e-9; 0 compares exactly */
} pf_newton_opts;

typedef struct pf_newton_report {
    int32_t iterations;   /* solves performed */
    int32_t converged;
    double norm[65];      /* ||F||_inf at x_0 .. x_iterations */
    double t_eval_s;      /* device evaluation time (residual + Jacobian) */
    double t_solve_s;     /* host solve callback time */
    double t_total_s;
    int32_t switched[65]; /* units that changed mode at x_k (limit checks) */
    int32_t n_switches;   /* sum of switched[] */
} pf_newton_report;

int pf_newton(pf_plan *plan, double *x, const pf_newton_opts *opts,
              pf_linsolve_fn solve, void *user, pf_newton_report *report);

/*
 * Reactive limits of PV generators (Section II-A: in the extended
 * formulation one set of equations covers a PV unit under voltage control
 * and held at a reactive target, so the limits can be checked during the
 * iterations).  A held
 * generator keeps its Q_g variable; its control row becomes
 * Q_g - Q_target (slot values 0 at V, 1 at Q_g) instead of V - V_set (1 at
 * V, 0 at Q_g).  Needs a plan set up with q_limits = 1 (else PF_EINVAL).
 * Modes apply to every instance of a batched plan.
 *
 * pf_set_gen_modes: host arrays over the plan's PV units (grid by grid, in
 *   input order): mode[k] 0 = voltage control, 1 = held at q_target[k]
 *   (q_target may be NULL when every mode is 0).  Synchronous; must not
 *   overlap an evaluation on the plan.
 * pf_get_gen_modes: the current modes and targets (either pointer may be
 *   NULL).
 * pf_q_limit_check: one check against q_min, q_max (host [n_pv]) at the
 *   state x (device [n], non-batched plans): a unit under voltage control
 *   whose Q_g is outside [q_min - tol, q_max + tol] is held at the violated
 *   limit; a held unit returns to voltage control when its bus voltage
 *   exceeds V_set + tol while held at q_max, or falls below V_set - tol
 *   while held at q_min (a unit held at any other target, set by
 *   pf_set_gen_modes, counts as held at q_min).  The new modes are applied as by pf_set_gen_modes;
 *   *n_switched (nullable) receives the number of changes.  Copies x to the
 *   host on the given stream (after the work queued there) and synchronises
 *   it.  A Newton solve with limits either repeats solve -> check until
 *   nothing switches, or lets pf_newton check inside its iterations.
 */
int pf_set_gen_modes(pf_plan *plan, const int32_t *mode, const double *q_target);
int pf_get_gen_modes(const pf_plan *plan, int32_t *mode, double *q_target);
int pf_q_limit_check(pf_plan *plan, const double *x, const double *q_min,
                     const double *q_max, double tol, int32_t *n_switched, void *stream);

/*
 * Device-resident Newton (tasks 1-4 of Section I with task 3 on the GPU).
 * The Jacobian pattern of a plan never changes, so one LU factorisation with
 * pivoting of one Jacobian M of the plan,  P M Q = L U,  fixes the pattern of
 * T = (L - I) + U and the row and column orders; rocSOLVER's sparse
 * re-factorisation (csrrf) then factorises every later Jacobian of the plan
 * on the device along that pattern, without pivoting again, and solves there.
 * (pf_batch_lu_create and pf_newton_batch below give the same Newton on this
 * library's own factorisation, with the plan as one instance; they are faster
 * on sparse factors, and rocSOLVER remains for factors whose rows are too
 * long for them.)
 *
 * pf_refact_create: host inputs, read during the call only.
 *   Jval_host  [nnz]   the values of M in pf_pattern order
 *   T_rowptr   [n+1], T_colidx [nnzT], T_val [nnzT]: CSR of (L - I) + U, the
 *              strictly lower part holding L without its unit diagonal;
 *              columns strictly increasing within a row, diagonal present,
 *              and every fill entry of the symbolic factorisation present
 *              (pf_lu_symbolic; a numeric LU may omit entries whose values
 *              vanish for M, and the re-factorisation would then be
 *              incomplete for other matrices -> PF_EINVAL)
 *   pivP, pivQ [n]     row k of P M Q is row pivP[k] of M; column k is column
 *              pivQ[k] of M
 * The plan must be a non-batched device plan; the object keeps a pointer to
 * it (destroy the object first) and owns its own device buffers (F, J, step,
 * the factors).  rocSOLVER is loaded on the first call (PF_EDEVICE if it
 * cannot be).  Malformed T or permutations -> PF_EINVAL.  Synchronises.
 */
typedef struct pf_refact pf_refact;

int pf_refact_create(pf_plan *plan, const double *Jval_host, int64_t nnzT,
                     const int32_t *T_rowptr, const int32_t *T_colidx,
                     const double *T_val, const int32_t *pivP, const int32_t *pivQ,
                     pf_refact **out);

/* Refactorise with the Jacobian values Jval (device [nnz], pf_pattern order)
 * and solve J y = b in place (b: device [n]).  Asynchronous on the stream;
 * the factors are held in the object, so calls on one object must not
 * overlap.  A zero pivot gives non-finite results rather than an error. */
int pf_refact_solve(pf_refact *rf, const double *Jval, double *b, void *stream);

/*
 * Newton power flow with every step on the device: per iteration one fused
 * evaluation (pf_eval), ||F||_inf by a device reduction (the only value
 * copied to the host, for the convergence test), refactorisation and solve
 * by rf, and x <- x - dx.  x: device [n], updated in place; opts and report
 * as pf_newton, with t_eval_s the device time of the evaluations and
 * t_solve_s the device time from the end of each evaluation to the end of
 * its step (norm, refactorisation, triangular solves, update).  Runs on the
 * given stream and synchronises it once per iteration.  Returns PF_ENOCONV if
 * max_iter is reached.  Reactive limits (q_min / q_max) are checked inside
 * the iterations as pf_newton does when rf's pivots survive a switch
 * (pf_jacobian_switch_order; pf_refact_create records it), else PF_EINVAL;
 * each check copies x to the host.
 */
int pf_newton_device(pf_plan *plan, pf_refact *rf, double *x,
                     const pf_newton_opts *opts, pf_newton_report *report,
                     void *stream);

/* Release the refactorisation object.  NULL is ignored. */
void pf_refact_destroy(pf_refact *rf);

/*
 * Fast decoupled power flow, XB variant (Section V names it as another
 * method that reuses the same equation evaluation).  Constant matrices,
 * built from the network given at setup (single-grid plans):
 *   B'  over the buses without a slack: per in-service branch the weight
 *       1/x only (the weighted Laplacian, slack rows and columns removed);
 *   B'' over the buses without a voltage controller: -Im(Y_bus) of the full
 *       pi-models with taps, charging and bus shunts, phase shifts left out.
 * Rows follow ascending bus number; columns are sorted.
 *
 * pf_fdlf_matrices: host outputs, all nullable; call once with NULL arrays
 *   to learn nnz_bp and nnz_bpp.  Row counts are N - N_slack (B') and
 *   N - N_gen (B'').  bp_bus / bpp_bus receive the bus of every row.
 */
int pf_fdlf_matrices(const pf_plan *plan, int64_t *nnz_bp, int32_t *bp_rowptr,
                     int32_t *bp_colidx, double *bp_val, int32_t *bp_bus,
                     int64_t *nnz_bpp, int32_t *bpp_rowptr, int32_t *bpp_colidx,
                     double *bpp_val, int32_t *bpp_bus);

/*
 * A constant sparse factorisation on the device: the n x n CSR matrix M and
 * one host LU of it (P M Q = L U in the form pf_refact_create takes), all
 * host arrays read during the call.  The factor values T_val are used as
 * given (M is only checked against them); the rows of T are grouped into
 * elimination levels at creation.  device < 0: the current device.
 * pf_lu_solve solves M y = b in place (b: device [n]) on the stream with
 * level-scheduled forward and backward solves of this library (runs of small
 * consecutive levels in one block); calls on one object must not overlap.
 * Errors as pf_refact_create.
 */
typedef struct pf_lu pf_lu;

/* Symbolic LU without pivoting of P M Q for the n x n CSR pattern
 * (rowptr, colidx) of M and the orders pivP, pivQ (as above): the CSR
 * pattern of T = (L - I) + U that holds every entry an elimination along it
 * can reach, whatever the values (a numeric LU may return fewer entries
 * where values happen to vanish; the device re-factorisations need the full
 * pattern).  Call with NULL T arrays to learn *nnzT.  Host arrays. */
int pf_lu_symbolic(int64_t n, const int32_t *rowptr, const int32_t *colidx,
                   const int32_t *pivP, const int32_t *pivQ, int64_t *nnzT,
                   int32_t *T_rowptr, int32_t *T_colidx);

int pf_lu_create(int32_t device, int64_t n, int64_t nnz, const int32_t *rowptr,
                 const int32_t *colidx, const double *val, int64_t nnzT,
                 const int32_t *T_rowptr, const int32_t *T_colidx,
                 const double *T_val, const int32_t *pivP, const int32_t *pivQ,
                 pf_lu **out);
int pf_lu_solve(pf_lu *lu, double *b, void *stream);

/*
 * For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * solve of pf_lu_solve, bit for bit, with its permuted working vector (n
 * doubles) in a static device array of the library instead of the object's
 * buffer.  The array holds 1,048,576 doubles (8 MiB) on every device the
 * library runs on, until the process ends; n above that -> PF_EINVAL.  The
 * call allocates nothing (the array's address is looked up once per
 * device).  Every call on one device shares the array and leaves it holding
 * its last working vector: calls that overlap on one device (other streams,
 * graphs replayed concurrently) race.  Errors as pf_lu_solve.
 */
int pf_lu_solve_noalloc(pf_lu *lu, double *b, void *stream);
void pf_lu_destroy(pf_lu *lu);

/*
 * pf_fdlf_create: bind a plan and the factorisations of its B' and B'' (NULL
 * for an empty matrix); the object keeps pointers to all three (destroy it
 * first) and owns its device buffers.
 * pf_fdlf_solve: x (device [n]) updated in place.  Controlled voltages and
 * slack angles are set to their set points (the method never steps them);
 * then per iteration, each step from a fresh residual (pf_eval_residual's
 * kernel), theta[B' buses] -= B'^-1 (F_p / V) and V[B'' buses] -=
 * B''^-1 (F_q / V), until max |F| over those rows < tol; then Q_g and P_s
 * take the values that zero their buses' rows.  report: norm[k] = that
 * maximum before iteration k (k = 0..iterations), norm[iterations + 1] =
 * ||F||_inf at the end; converged if that is below tol too; t_eval_s the
 * device time of the residual evaluations, t_solve_s the wall time of the
 * half-steps.  Needs every PV unit under voltage control.  PF_ENOCONV if
 * max_iter (<= 64) is reached.  Synchronises the stream once per iteration.
 */
typedef struct pf_fdlf pf_fdlf;

int pf_fdlf_create(pf_plan *plan, pf_lu *bp, pf_lu *bpp, pf_fdlf **out);
int pf_fdlf_solve(pf_fdlf *fd, double *x, const pf_newton_opts *opts,
                  pf_newton_report *report, void *stream);
void pf_fdlf_destroy(pf_fdlf *fd);

/*
 * Batched Newton (every instance of a batched plan solved together, e.g. N-1
 * contingencies).  The Jacobians of a batched plan share one pattern, so one
 * host LU with pivoting of one of them, P M Q = L U (T = (L - I) + U and
 * pivP, pivQ as for pf_refact_create; T must hold every Jacobian entry and be
 * closed under elimination, as the filled pattern of an LU is), serves every
 * instance: each is factorised on the device along T without pivoting again
 * (a zero pivot gives non-finite values for that instance only).
 *
 * pf_batch_lu_create: batched plan in the row layout, or a single-instance
 *   or multi-grid plan (one instance: its x, F and Jval are the row layout
 *   with pitch 1, and the same calls give a device-resident Newton whose
 *   factorisation is this library's own); host arrays read during the call; the object keeps a pointer to the plan (destroy it
 *   first) and owns its device buffers (T values for every instance: nnzT x
 *   the plan's row pitch doubles, plus F, J and work rows).  Rows of T
 *   longer than the device's LDS allows for 16 instances give PF_EINVAL.
 * pf_batch_lu_factor: factorise every instance from J (device, the plan's
 *   batched Jacobian layout [nnz][pitch]).
 * pf_batch_lu_solve: after a factorisation, Xout[., i] = J_i^-1 B[., i] for
 *   every instance (device [n][pitch], must not alias).  Asynchronous.
 * pf_newton_batch: X (device [n][pitch]) updated in place; per iteration one
 *   evaluation (pf_eval_batch's kernel, or pf_eval's for a plan of one
 *   instance), per-instance ||F||_inf (the
 *   norms are copied to the host), the factorisation and solves, and
 *   x <- x - dx for the instances still above tol; an instance that reaches
 *   tol is not stepped again.  inst_iters / inst_norm (host [n_inst],
 *   nullable) receive each instance's steps and last norm.  report:
 *   iterations = steps taken, converged = number of converged instances,
 *   norm[k] = largest norm among unconverged instances before step k,
 *   t_eval_s = evaluations, t_solve_s = factorisations + solves + updates
 *   (device time).  PF_ENOCONV if some instance has not converged after
 *   max_iter (<= 64) steps.  Calls on one object must not overlap.
 *   With q_min / q_max set (plan of one instance set up with q_limits,
 *   factorisation whose pivots pair and order every PV unit's Q row and
 *   control row as pf_jacobian_switch_order describes, else PF_EINVAL) the
 *   limits are checked inside the iterations exactly as pf_newton does
 *   (same options, same report fields switched / n_switches; the state is
 *   copied to the host for each check); the factorisation of each step
 *   then follows the modes in force.
 */
typedef struct pf_batch_lu pf_batch_lu;

int pf_batch_lu_create(pf_plan *plan, int64_t nnzT, const int32_t *T_rowptr,
                       const int32_t *T_colidx, const int32_t *pivP,
                       const int32_t *pivQ, pf_batch_lu **out);
int pf_batch_lu_factor(pf_batch_lu *b, const double *J, void *stream);
int pf_batch_lu_solve(pf_batch_lu *b, const double *B, double *Xout, void *stream);
int pf_newton_batch(pf_plan *plan, pf_batch_lu *b, double *X, const pf_newton_opts *opts,
                    int32_t *inst_iters, double *inst_norm, pf_newton_report *report,
                    void *stream);
void pf_batch_lu_destroy(pf_batch_lu *b);

/* Release the plan and all its device memory.  NULL is ignored. */
void pf_destroy(pf_plan *plan);

/* Message describing the last failure on this thread ("" if none). */
const char *pf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PF_H */
