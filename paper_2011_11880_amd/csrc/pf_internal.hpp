// Internal structures of libpf: the host-side plan built at setup, and the
// device mirror that the kernels read.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "pf.h"

namespace pf {

// Status helpers ------------------------------------------------------------
int fail(int code, const char *fmt, ...);
void clear_error();

// Contribution kinds of a branch to an admittance-row entry (from/to ends).
enum ContribKind : int32_t { K_FF = 0, K_FT = 1, K_TF = 2, K_TT = 3 };

// Row-start flag kept in bit 31 of an admittance column index.
constexpr int32_t kRowStart = int32_t(0x80000000u);
constexpr int32_t kColMask = 0x7fffffff;

// One grid inside a plan (a plan has one grid unless it is multi-grid).
struct GridInfo {
    int32_t N, NPV, NS, NG;      // buses, PV units, slacks, generators
    int32_t NB, NL, NSH;         // branches, loads, shunts
    int64_t xoff;                // first variable / equation of the grid
    int64_t joff;                // first Jacobian value of the grid
    int64_t nnz;                 // Jacobian values of the grid
    int32_t bus_off, br_off, load_off, pv_off, gen_off, shunt_off;
    int32_t y_off, n_y;          // admittance entries
};

// Grid descriptor read by the single-instance kernel (one per grid).
struct GridDev {
    int32_t N;
    int32_t bus_off;
    int64_t xoff;
};

enum PlanKind : int32_t { KIND_SINGLE = 0, KIND_BATCH = 1, KIND_MULTI = 2 };

// Third field of a PV unit's gen4 record (a slack's holds its P_s index):
// voltage control with a single control-row slot, voltage control with the
// Q_g slot present (written 0), or reactive output held at gen2.x.
constexpr int32_t kGenVoltage = -1, kGenVoltageSlot = -2, kGenHeld = -3;

// Entries per tile of the adjoint's row walk (a longer row forms a tile of
// its own); small tiles give more, shorter wavefronts.
constexpr int32_t kAdjTileEntries = 16;

struct HostPlan {
    int32_t kind = KIND_SINGLE;
    int32_t n_inst = 1;
    int32_t ld = 1;                    // batched row pitch (>= n_inst)
    int32_t panels = 0;                // 1: batched arrays in panels of 64 instances
    bool host_only = false;
    int device = 0;
    std::vector<GridInfo> grids;

    // totals over grids
    int64_t n = 0, nnz = 0;
    int32_t Nt = 0, Bt = 0, NLt = 0, NPVt = 0, NSt = 0, NGt = 0, NSHt = 0;
    int64_t n_y = 0;

    // fixed Jacobian pattern (concatenated, absolute indices)
    std::vector<int32_t> rowptr, colidx;

    // admittance rows over all buses (global bus numbering); columns are the
    // local bus index inside the grid, with kRowStart on each row's first entry
    std::vector<int32_t> yptr;      // Nt + 1 (global entry index)
    std::vector<int32_t> ycol;      // n_y
    std::vector<int32_t> cptr;      // n_y + 1: contributions per entry
    std::vector<int32_t> clist;     // (global branch id << 2) | kind

    // per bus
    std::vector<int32_t> bus4;      // Nt * 4: ystart, yend, jP (row P start), jQ
    std::vector<int32_t> bus2;      // Nt * 2: diagonal position, generator (global) or -1
    std::vector<int32_t> busx;      // Nt * 2: theta and V variable (= P and Q row) index
    std::vector<int32_t> ytr;       // n_y: entry (j, i) of row j for entry (i, j), -1 on the diagonal
    std::vector<int32_t> shptr, shlist;  // shunts per bus (global shunt ids)
    std::vector<int32_t> ldptr, ldlist;  // loads per bus (global load ids)

    // per generator (global: grid by grid, PV units then slacks)
    std::vector<int32_t> gen4;      // NGt * 4: Q_g var (= V row), V-row slot,
                                    //          P_s var (= theta row) or a PV mode (kGen*),
                                    //          theta-row slot (-1 for PV units)
    std::vector<double> gen2;       // NGt * 2: V setpoint (Q target when held), theta setpoint
    std::vector<int32_t> genpv;     // NGt: PV unit id (global) or -1 for a slack
    // reactive-limit support: with q_slots every PV unit's control row also
    // holds its Q_g column (the row's second slot), so the unit can be held
    // at a reactive target; pv_gen maps PV unit -> generator
    int32_t q_slots = 0;
    std::vector<int32_t> pv_gen, pv_mode;   // NPVt each
    std::vector<double> pv_vset, pv_qt;      // NPVt each

    // per branch / device (global ids)
    std::vector<int32_t> br_f, br_t;   // global bus ids
    std::vector<int32_t> br_on;        // 1 in service
    std::vector<double> params;        // [r][x][b][tap][shift_deg][load_p][load_q]
    bool params_stale = false;         // device copy replaced by pf_set_params since the
                                       // host copy was last refreshed
    std::vector<double> pv_p;          // NPVt
    std::vector<double> shunt_g, shunt_b;
    std::vector<int32_t> load_bus;     // global bus id

    // single-instance schedule
    pf_schedule sched{};
    std::vector<int32_t> tiles;        // ntiles * 8: e0, e1, b0 (global bus), grid,
                                       //   J range of the P rows, J range of the Q rows

    // batched overlay
    std::vector<double> load_scale_t;  // [NL][ld] or empty
    std::vector<double> pv_scale_t;    // [NPV][ld] or empty
    std::vector<int32_t> outage;       // [I] or empty
    std::vector<int32_t> order_natural, order_bfs;   // bus processing orders
    // input bus (grid-local) of every plan bus: the identity unless the
    // network was renumbered for locality at setup (bus_order_kind 1)
    std::vector<int32_t> bus_order;
    int32_t bus_order_kind = 0;

    // adjoint work order (single-instance and multi-grid plans): admittance
    // rows taken in breadth-first order, so that a contiguous range of work,
    // which one XCD runs, covers neighbouring buses and its L2 serves the
    // cotangent rows they share
    std::vector<int32_t> adj_src;      // n_y: entry index, rows in order_bfs order
    std::vector<int32_t> adj_tiles;    // n * 4: e0, e1 (positions in adj_src),
                                       //   position of the first row in order_bfs, grid
    // parameter gradients: each in-service branch belongs to the entry
    // (from bus, to bus) of its from bus's row, which evaluates it next to
    // that entry; adj_own holds that branch per position of adj_src (or -1).
    // A second branch on the same entry and out-of-service branches go to
    // adj_left, evaluated by a separate pass.
    std::vector<int32_t> adj_own;      // n_y
    std::vector<int32_t> adj_left;

    int64_t n_params() const { return 5LL * Bt + 2LL * NLt; }
    int32_t n_tiles() const { return int32_t(tiles.size() / 8); }
    int32_t n_adj_tiles() const { return int32_t(adj_tiles.size() / 4); }
};

// Host setup (pf_setup.cpp)
int build_host_plan(const pf_network *nets, int32_t n_grids, HostPlan &hp);
int attach_batch(const pf_batch_spec *spec, HostPlan &hp);
int normalise_schedule(const HostPlan &hp, const pf_schedule *in, pf_schedule &out);
void build_tiles(HostPlan &hp);
void build_adjoint_order(HostPlan &hp);

// Device side (pf_device.hip)
struct DevPlan;
int dev_create(HostPlan &hp, DevPlan **out);
void dev_destroy(DevPlan *dp);
int dev_upload_tiles(HostPlan &hp, DevPlan *dp);
int dev_set_params(HostPlan &hp, DevPlan *dp, const double *params_dev, void *stream);
int dev_fetch_params(HostPlan &hp, DevPlan *dp);
int dev_upload_gens(const HostPlan &hp, DevPlan *dp);
int dev_eval_single(HostPlan &hp, DevPlan *dp, const double *x, double *F,
                    double *J, void *stream);
int dev_eval_batch(HostPlan &hp, DevPlan *dp, const double *X, double *F,
                   double *J, void *stream);
int dev_vjp(HostPlan &hp, DevPlan *dp, const double *x, const double *W,
            int32_t k, double *gx, double *gp, void *stream);
int dev_newton(HostPlan &hp, DevPlan *dp, double *x, const pf_newton_opts *opts,
               pf_linsolve_fn solve, void *user, pf_newton_report *rep);
// Reactive limits (pf_qlim.hip): argument checks, and the switching rule
// at a host copy of the state (uploads the generator table on a switch).
int q_limits_valid(const HostPlan &hp, const double *q_min, const double *q_max, double tol);
int q_switch(HostPlan &hp, DevPlan *dp, const double *xh, const double *q_min,
             const double *q_max, double tol, int32_t *n_switched);
// Whether an LU's pivots (M[pivP][:, pivQ] = L U) survive any PV unit's
// switch: each unit's bus Q row on its Q_g column, its control row on the bus
// voltage column, the Q_g column first.  False for batched plans (modes are
// per plan) and plans without Q_g slots.
bool pivots_switch_safe(const HostPlan &hp, const int32_t *pivP, const int32_t *pivQ);
int dev_autotune(HostPlan &hp, DevPlan *dp, const double *x, double *F,
                 double *J, int32_t reps, void *stream, const char *cache,
                 pf_schedule *best, int32_t *hit);

}  // namespace pf

struct pf_plan {
    pf::HostPlan host;
    pf::DevPlan *dev = nullptr;
};
