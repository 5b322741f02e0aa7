/*
 * CPU oracle for power-flow equation and Jacobian evaluation.
 *
 * TEST INFRASTRUCTURE.  This is the plain, slow, FP64 reference that the
 * HIP library is checked against.  Only the test suite, the package's smoke
 * check and the benchmark's CPU-baseline leg load it; the library itself
 * never does, and the two share no code.  Build:
 *   gcc -O2 -ffp-contract=off -fPIC -shared pf_oracle.c -o liboracle.so -lm
 *
 * It follows the paper's model-based formulation (Section II-A, eqs. 1-4):
 * every model (PQ load, PV generator, slack generator, line/transformer,
 * shunt) evaluates its own equations and Jacobian elements, and results on
 * the same bus are joined by summation.  The Jacobian comes out as triplets
 * (Section III: triplets assembled into a sparse matrix), which the Python
 * side sums into CSR.
 *
 * Exports:
 *   ora_residual      F(y) and, per row, the sum of |terms| (for tolerances)
 *   ora_residual_cs   F(y) in complex arithmetic (complex-step derivatives)
 *   ora_branch_flows  one branch's four terminal injections
 *   ora_jacobian      dF/dy as COO triplets, model by model, with each
 *                     triplet's sum of |products| (for tolerances)
 *   ora_vjp_params    gradient of w.F with respect to branch and load data
 *   ora_vjp_params_scale  sum of |terms| behind each of those gradients
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>
#include <string.h>

#define ORA_PI 3.14159265358979323846

typedef struct {
    int n_bus, n_branch, n_load, n_pv, n_slack, n_shunt;
    const int *br_from, *br_to, *br_status;
    const int *load_bus, *pv_bus, *slack_bus, *shunt_bus;
    /* per PV generator: 0 = voltage control, 1 = reactive output held at a
       target (a PV generator switched to a PQ injection); NULL = all 0 */
    const int *pv_mode;
} ora_topo;

/* numeric data of a network, real build */
typedef struct {
    const double *br_r, *br_x, *br_b, *br_tap, *br_shift_deg;
    const double *load_p, *load_q, *pv_p, *pv_v, *slack_v, *slack_theta;
    const double *shunt_g, *shunt_b;
    const double *pv_qtarget;   /* per PV generator; read where pv_mode is 1 */
} ora_data;

/*
 * Rounding scale of a branch's four terminal injections: for each flow, the
 * sum of the absolute values of the products it is made of (with the
 * charging half split from the series susceptance).  A flow is itself a
 * difference of nearly equal products when the angle across the branch is
 * small, so |flow| alone would understate the rounding of either side's sum.
 */
static void branch_flow_scales(double r, double x, double bc, double tap,
                               double shift_deg, double vf, double vt,
                               double thf, double tht, double out[4])
{
    const double d = r * r + x * x;
    const double g = r / d, b = -x / d;
    const double delta = thf - tht - shift_deg * (ORA_PI / 180.0);
    const double c = cos(delta), s = sin(delta);
    const double u = vf * vt / tap, t2 = tap * tap;
    const double ugc = fabs(u * g * c), ubs = fabs(u * b * s);
    const double ugs = fabs(u * g * s), ubc = fabs(u * b * c);
    out[0] = fabs(vf * vf * g / t2) + ugc + ubs;
    out[1] = fabs(vf * vf * b / t2) + fabs(vf * vf * bc / (2.0 * t2)) + ugs + ubc;
    out[2] = fabs(vt * vt * g) + ugc + ubs;
    out[3] = fabs(vt * vt * b) + fabs(vt * vt * bc / 2.0) + ugs + ubc;
}

/* ---- real instantiation ---- */
#define ORA_T double
#define ORA_SIN sin
#define ORA_COS cos
#define ORA_NAME(x) x##_d
#define ORA_ACC(S, i, v) do { if (S) (S)[i] += fabs(v); } while (0)
#define ORA_ACC_FLOWS(S, N, f, t, r, x, bc, tap, sh, vf, vt, thf, tht)         \
    do {                                                                       \
        if (S) {                                                               \
            double m_[4];                                                      \
            branch_flow_scales(r, x, bc, tap, sh, vf, vt, thf, tht, m_);       \
            (S)[f] += m_[0];                                                   \
            (S)[(N) + (f)] += m_[1];                                           \
            (S)[t] += m_[2];                                                   \
            (S)[(N) + (t)] += m_[3];                                           \
        }                                                                      \
    } while (0)
#include "ora_core.inc"
#undef ORA_T
#undef ORA_SIN
#undef ORA_COS
#undef ORA_NAME
#undef ORA_ACC
#undef ORA_ACC_FLOWS

/* ---- complex instantiation (complex-step differentiation) ---- */
#define ORA_T double complex
#define ORA_SIN csin
#define ORA_COS ccos
#define ORA_NAME(x) x##_z
#define ORA_ACC(S, i, v) do { (void)(S); } while (0)
#define ORA_ACC_FLOWS(S, N, f, t, r, x, bc, tap, sh, vf, vt, thf, tht) do { (void)(S); } while (0)
#include "ora_core.inc"
#undef ORA_T
#undef ORA_SIN
#undef ORA_COS
#undef ORA_NAME
#undef ORA_ACC
#undef ORA_ACC_FLOWS

void ora_residual(const ora_topo *tp, const ora_data *d, const double *y,
                  double *F, double *S)
{
    residual_d(tp, d->br_r, d->br_x, d->br_b, d->br_tap, d->br_shift_deg,
               d->load_p, d->load_q, d->pv_p, d->pv_v, d->slack_v,
               d->slack_theta, d->shunt_g, d->shunt_b, d->pv_qtarget, y, F, S);
}

/*
 * Complex residual.  Every numeric array is interleaved (re, im) pairs, so a
 * perturbation i*h on any state entry or parameter gives
 * dF/dz = Im F / h without subtractive cancellation.
 */
void ora_residual_cs(const ora_topo *tp, const double *br_r, const double *br_x,
                     const double *br_b, const double *br_tap,
                     const double *br_shift_deg, const double *load_p,
                     const double *load_q, const double *pv_p,
                     const double *pv_v, const double *slack_v,
                     const double *slack_theta, const double *shunt_g,
                     const double *shunt_b, const double *pv_qtarget,
                     const double *y, double *F)
{
#define Z(p) ((const double complex *)(const void *)(p))
    residual_z(tp, Z(br_r), Z(br_x), Z(br_b), Z(br_tap), Z(br_shift_deg),
               Z(load_p), Z(load_q), Z(pv_p), Z(pv_v), Z(slack_v),
               Z(slack_theta), Z(shunt_g), Z(shunt_b), Z(pv_qtarget), Z(y),
               (double complex *)(void *)F, NULL);
#undef Z
}

void ora_branch_flows(double r, double x, double bc, double tap,
                      double shift_deg, double vf, double vt, double thf,
                      double tht, double out[4])
{
    branch_flows_d(r, x, bc, tap, shift_deg, vf, vt, thf, tht, out);
}

/* Store one triplet and, when asked for, its rounding scale m (the sum of
 * the absolute values of the products the value is made of). */
static long put(int *rows, int *cols, double *vals, double *scales, long k,
                int r, int c, double v, double m)
{
    rows[k] = r;
    cols[k] = c;
    vals[k] = v;
    if (scales) scales[k] = m;
    return k + 1;
}

/* Upper bound on the number of triplets ora_jacobian emits. */
long ora_jacobian_size(const ora_topo *tp)
{
    return 16L * tp->n_branch + 2L * tp->n_shunt + 2L * tp->n_pv +
           4L * tp->n_slack;
}

/*
 * Jacobian elements dF/dy as triplets (row, col, value), model by model.
 * Duplicated (row, col) pairs are meant to be summed.  Returns the count.
 *
 * Line/transformer partials, with u = V_f V_t / tap, delta = th_f - th_t - phi,
 * C = cos delta, S = sin delta and
 *   A1 = u (g C + b S), B1 = u (g S - b C),
 *   A2 = u (g C - b S), B2 = u (g S + b C):
 *   dP_f/dth_f =  B1   dP_f/dth_t = -B1
 *   dQ_f/dth_f = -A1   dQ_f/dth_t =  A1
 *   dP_t/dth_f =  B2   dP_t/dth_t = -B2
 *   dQ_t/dth_f =  A2   dQ_t/dth_t = -A2
 *   dP_f/dV_f = 2 V_f g / tap^2 - A1 / V_f     dP_f/dV_t = -A1 / V_t
 *   dQ_f/dV_f = -2 V_f (b + bc/2) / tap^2 - B1 / V_f   dQ_f/dV_t = -B1 / V_t
 *   dP_t/dV_f = -A2 / V_f     dP_t/dV_t = 2 V_t g - A2 / V_t
 *   dQ_t/dV_f =  B2 / V_f     dQ_t/dV_t = -2 V_t (b + bc/2) + B2 / V_t
 * (the divisions by V are carried out as products with the other voltage).
 */
long ora_jacobian(const ora_topo *tp, const ora_data *dd, const double *y,
                  int *rows, int *cols, double *vals, double *scales)
{
    const int N = tp->n_bus, NPV = tp->n_pv, NS = tp->n_slack;
    const int NG = NPV + NS;
    const double *th = y, *V = y + N;
    long k = 0;
    int e, i;
#define PUT(r, c, v, m) (k = put(rows, cols, vals, scales, k, (r), (c), (v), (m)))
    /* PQ loads: constant power, no state dependence. */
    /* PV generators */
    for (e = 0; e < NPV; ++e) {
        i = tp->pv_bus[e];
        PUT(N + i, 2 * N + e, -1.0, 1.0);                 /* dFq/dQg */
        if (tp->pv_mode && tp->pv_mode[e])
            PUT(2 * N + e, 2 * N + e, 1.0, 1.0);          /* d(Qg - Qt)/dQg */
        else
            PUT(2 * N + e, N + i, 1.0, 1.0);              /* dFV/dV */
    }
    /* Slack generators */
    for (e = 0; e < NS; ++e) {
        i = tp->slack_bus[e];
        PUT(i, 2 * N + NG + e, -1.0, 1.0);                /* dFp/dPs */
        PUT(N + i, 2 * N + NPV + e, -1.0, 1.0);           /* dFq/dQg */
        PUT(2 * N + NPV + e, N + i, 1.0, 1.0);            /* dFV/dV */
        PUT(2 * N + NG + e, i, 1.0, 1.0);                 /* dFth/dth */
    }
    /* Lines and transformers */
    for (e = 0; e < tp->n_branch; ++e) {
        int f, t;
        double r, x, bc, tap, phi, d, g, b, delta, C, S, u, t2;
        double A1, B1, A2, B2, vf, vt, mA, mB, af, at;
        if (tp->br_status && !tp->br_status[e]) continue;
        f = tp->br_from[e];
        t = tp->br_to[e];
        r = dd->br_r[e];
        x = dd->br_x[e];
        bc = dd->br_b[e];
        tap = dd->br_tap[e];
        phi = dd->br_shift_deg[e] * (ORA_PI / 180.0);
        d = r * r + x * x;
        g = r / d;
        b = -x / d;
        vf = V[f];
        vt = V[t];
        delta = th[f] - th[t] - phi;
        C = cos(delta);
        S = sin(delta);
        u = vf * vt / tap;
        t2 = tap * tap;
        A1 = u * (g * C + b * S);
        B1 = u * (g * S - b * C);
        A2 = u * (g * C - b * S);
        B2 = u * (g * S + b * C);
        /* scales: A1, A2 are made of u g C and u b S; B1, B2 of u g S and
           u b C; the V partials of the same products over V_f or V_t */
        mA = fabs(u * g * C) + fabs(u * b * S);
        mB = fabs(u * g * S) + fabs(u * b * C);
        af = vf / tap;
        at = vt / tap;
        /* theta columns */
        PUT(f, f, B1, mB);
        PUT(f, t, -B1, mB);
        PUT(N + f, f, -A1, mA);
        PUT(N + f, t, A1, mA);
        PUT(t, f, B2, mB);
        PUT(t, t, -B2, mB);
        PUT(N + t, f, A2, mA);
        PUT(N + t, t, -A2, mA);
        /* V columns */
        PUT(f, N + f, 2.0 * vf * g / t2 - (vt / tap) * (g * C + b * S),
            fabs(2.0 * vf * g / t2) + fabs(at * g * C) + fabs(at * b * S));
        PUT(f, N + t, -(vf / tap) * (g * C + b * S), fabs(af * g * C) + fabs(af * b * S));
        PUT(N + f, N + f, -2.0 * vf * (b + bc / 2.0) / t2 - (vt / tap) * (g * S - b * C),
            fabs(2.0 * vf * b / t2) + fabs(vf * bc / t2) + fabs(at * g * S) + fabs(at * b * C));
        PUT(N + f, N + t, -(vf / tap) * (g * S - b * C), fabs(af * g * S) + fabs(af * b * C));
        PUT(t, N + f, -(vt / tap) * (g * C - b * S), fabs(at * g * C) + fabs(at * b * S));
        PUT(t, N + t, 2.0 * vt * g - (vf / tap) * (g * C - b * S),
            fabs(2.0 * vt * g) + fabs(af * g * C) + fabs(af * b * S));
        PUT(N + t, N + f, (vt / tap) * (g * S + b * C), fabs(at * g * S) + fabs(at * b * C));
        PUT(N + t, N + t, -2.0 * vt * (b + bc / 2.0) + (vf / tap) * (g * S + b * C),
            fabs(2.0 * vt * b) + fabs(vt * bc) + fabs(af * g * S) + fabs(af * b * C));
    }
    /* Shunts */
    for (e = 0; e < tp->n_shunt; ++e) {
        double vg, vb;
        i = tp->shunt_bus[e];
        vg = 2.0 * dd->shunt_g[e] * V[i];
        vb = -2.0 * dd->shunt_b[e] * V[i];
        PUT(i, N + i, vg, fabs(vg));
        PUT(N + i, N + i, vb, fabs(vb));
    }
#undef PUT
    return k;
}

/*
 * Gradient of L = w . F(y; p) with respect to the network data p, for one
 * cotangent w (length n).  Outputs (all length n_branch except the loads):
 *   g_r, g_x, g_b (line charging), g_tap, g_shift (per degree),
 *   g_lp, g_lq (length n_load).
 *
 * With D = r^2 + x^2: dg/dr = (x^2 - r^2)/D^2, dg/dx = -2 r x / D^2,
 * db/dr = 2 r x / D^2, db/dx = (x^2 - r^2)/D^2, and the flow partials
 *   dP_f/dg = V_f^2/tap^2 - u C   dP_f/db = -u S
 *   dQ_f/dg = -u S                dQ_f/db = -V_f^2/tap^2 + u C
 *   dP_t/dg = V_t^2 - u C         dP_t/db = u S
 *   dQ_t/dg = u S                 dQ_t/db = -V_t^2 + u C
 *   dQ_f/dbc = -V_f^2/(2 tap^2)   dQ_t/dbc = -V_t^2/2
 *   dP_f/dtap = -2 V_f^2 g / tap^3 + A1/tap
 *   dQ_f/dtap = 2 V_f^2 (b + bc/2)/tap^3 + B1/tap
 *   dP_t/dtap = A2/tap            dQ_t/dtap = -B2/tap
 *   dX/dphi = -dX/dth_f for every flow X (phi in radians).
 */
void ora_vjp_params(const ora_topo *tp, const ora_data *dd, const double *y,
                    const double *w, double *g_r, double *g_x, double *g_b,
                    double *g_tap, double *g_shift, double *g_lp, double *g_lq)
{
    const int N = tp->n_bus;
    const double *th = y, *V = y + N;
    int e;
    for (e = 0; e < tp->n_branch; ++e) {
        int f, t;
        double r, x, bc, tap, phi, D, D2, g, b, delta, C, S, u, t2, vf, vt;
        double A1, B1, A2, B2, dg_dr, dg_dx, db_dr, db_dx;
        double wpf, wqf, wpt, wqt, dLdg, dLdb;
        g_r[e] = g_x[e] = g_b[e] = g_tap[e] = g_shift[e] = 0.0;
        if (tp->br_status && !tp->br_status[e]) continue;
        f = tp->br_from[e];
        t = tp->br_to[e];
        r = dd->br_r[e];
        x = dd->br_x[e];
        bc = dd->br_b[e];
        tap = dd->br_tap[e];
        phi = dd->br_shift_deg[e] * (ORA_PI / 180.0);
        D = r * r + x * x;
        D2 = D * D;
        g = r / D;
        b = -x / D;
        vf = V[f];
        vt = V[t];
        delta = th[f] - th[t] - phi;
        C = cos(delta);
        S = sin(delta);
        u = vf * vt / tap;
        t2 = tap * tap;
        A1 = u * (g * C + b * S);
        B1 = u * (g * S - b * C);
        A2 = u * (g * C - b * S);
        B2 = u * (g * S + b * C);
        wpf = w[f];
        wqf = w[N + f];
        wpt = w[t];
        wqt = w[N + t];
        dLdg = wpf * (vf * vf / t2 - u * C) + wqf * (-u * S) +
               wpt * (vt * vt - u * C) + wqt * (u * S);
        dLdb = wpf * (-u * S) + wqf * (-vf * vf / t2 + u * C) +
               wpt * (u * S) + wqt * (-vt * vt + u * C);
        dg_dr = (x * x - r * r) / D2;
        dg_dx = -2.0 * r * x / D2;
        db_dr = 2.0 * r * x / D2;
        db_dx = (x * x - r * r) / D2;
        g_r[e] = dLdg * dg_dr + dLdb * db_dr;
        g_x[e] = dLdg * dg_dx + dLdb * db_dx;
        g_b[e] = wqf * (-vf * vf / (2.0 * t2)) + wqt * (-vt * vt / 2.0);
        g_tap[e] = wpf * (-2.0 * vf * vf * g / (t2 * tap) + A1 / tap) +
                   wqf * (2.0 * vf * vf * (b + bc / 2.0) / (t2 * tap) + B1 / tap) +
                   wpt * (A2 / tap) + wqt * (-B2 / tap);
        /* dX/dphi = -dX/dth_f, then per degree */
        g_shift[e] = -(wpf * B1 + wqf * (-A1) + wpt * B2 + wqt * A2) *
                     (ORA_PI / 180.0);
    }
    for (e = 0; e < tp->n_load; ++e) {
        g_lp[e] = w[tp->load_bus[e]];
        g_lq[e] = w[N + tp->load_bus[e]];
    }
}

/*
 * Tolerance scale for ora_vjp_params: for each gradient, the sum of the
 * absolute values of the product terms it is made of, with every difference
 * or sum of products counted as its separate products (x^2 - r^2 contributes
 * x^2 + r^2, u (g C + b S) contributes |u g C| + |u b S|, b + b_c/2
 * contributes |b| + |b_c|/2).  The rounding error of the gradient, evaluated
 * in any order or grouping of those terms, is bounded by a small multiple of
 * the machine epsilon times this sum.  It only bounds rounding differences
 * under cancellation; it is not part of the reference values.
 *
 * With sg, sb the scales of dL/dg and dL/db (the flow partials of
 * Section II-A's pi-model dotted with |w|) and D = r^2 + x^2:
 *   s_r = (sg (x^2 + r^2) + sb 2|r x|) / D^2   (g_r = dL/dg dg/dr + dL/db db/dr)
 *   s_x = (sg 2|r x| + sb (x^2 + r^2)) / D^2   (g_x = dL/dg dg/dx + dL/db db/dx)
 */
void ora_vjp_params_scale(const ora_topo *tp, const ora_data *dd, const double *y,
                          const double *w, double *s_r, double *s_x, double *s_b,
                          double *s_tap, double *s_shift)
{
    const int N = tp->n_bus;
    const double *th = y, *V = y + N;
    int e;
    for (e = 0; e < tp->n_branch; ++e) {
        int f, t;
        double r, x, bc, tap, phi, D, D2, g, b, delta, C, S, u, t2, vf, vt;
        double aC, aS, ag, ab, A1, B1, A2, B2, wpf, wqf, wpt, wqt, sg, sb;
        s_r[e] = s_x[e] = s_b[e] = s_tap[e] = s_shift[e] = 0.0;
        if (tp->br_status && !tp->br_status[e]) continue;
        f = tp->br_from[e];
        t = tp->br_to[e];
        r = dd->br_r[e];
        x = dd->br_x[e];
        bc = dd->br_b[e];
        tap = dd->br_tap[e];
        phi = dd->br_shift_deg[e] * (ORA_PI / 180.0);
        D = r * r + x * x;
        D2 = D * D;
        g = r / D;
        b = -x / D;
        vf = V[f];
        vt = V[t];
        delta = th[f] - th[t] - phi;
        C = cos(delta);
        S = sin(delta);
        u = vf * vt / tap;
        t2 = tap * tap;
        aC = fabs(u * C);
        aS = fabs(u * S);
        ag = fabs(g);
        ab = fabs(b);
        /* |terms| of A1 = u(gC + bS), B1 = u(gS - bC), A2 = u(gC - bS),
           B2 = u(gS + bC) */
        A1 = ag * aC + ab * aS;
        B1 = ag * aS + ab * aC;
        A2 = A1;
        B2 = B1;
        wpf = fabs(w[f]);
        wqf = fabs(w[N + f]);
        wpt = fabs(w[t]);
        wqt = fabs(w[N + t]);
        sg = wpf * (vf * vf / t2 + aC) + wqf * aS + wpt * (vt * vt + aC) + wqt * aS;
        sb = wpf * aS + wqf * (vf * vf / t2 + aC) + wpt * aS + wqt * (vt * vt + aC);
        s_r[e] = (sg * (x * x + r * r) + sb * fabs(2.0 * r * x)) / D2;
        s_x[e] = (sg * fabs(2.0 * r * x) + sb * (x * x + r * r)) / D2;
        s_b[e] = wqf * vf * vf / (2.0 * t2) + wqt * vt * vt / 2.0;
        s_tap[e] = wpf * (2.0 * vf * vf * ag / (t2 * tap) + A1 / tap) +
                   wqf * (2.0 * vf * vf * (ab + fabs(bc) / 2.0) / (t2 * tap) + B1 / tap) +
                   wpt * (A2 / tap) + wqt * (B2 / tap);
        s_shift[e] = (wpf * B1 + wqf * A1 + wpt * B2 + wqt * A2) * (ORA_PI / 180.0);
    }
}
