// Device side of libpf for gfx950 (CDNA4): plan buffers, setup-time
// coefficient kernels and the evaluation kernels of the power-flow hot path
// (Section II-A equations, tasks 1 and 2 of the Newton loop).
//
// Layout and arithmetic (all FP64):
//  * Every in-service branch's pi-model (series g + jb = 1/(r + jx), charging
//    b/2 per end, ideal transformer t e^{j phi} on the from side) is folded at
//    setup into bus-admittance rows: row i holds one entry per column of
//    sorted({i} U adj(i)) with the summed admittance G_ij + jB_ij of every
//    branch joining i and j (and the shunts on the diagonal).  An entry is
//    4 B of column + 16 B of coefficients.
//  * The injections of row i are the join of its entries (Section II-B):
//      P_i = sum_j V_i V_j (G_ij cos th_ij + B_ij sin th_ij)
//      Q_i = sum_j V_i V_j (G_ij sin th_ij - B_ij cos th_ij)
//    (diagonal term V_i^2 G_ii and -V_i^2 B_ii), summed by a left fold over
//    the row in column order -- the same order in every kernel and for every
//    schedule, so all outputs are bit-reproducible.  No atomics.
//  * Jacobian values go straight to slots fixed at setup: off-diagonal
//    entries by the lane that owns the admittance entry, the four diagonal
//    sums and the constant +-1 entries by the lane that finishes the row.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "pf_internal.hpp"

namespace pf {

#define HIP_TRY(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return fail(PF_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Relative margin by which a candidate schedule must beat the best so far in
// the autotuner's search.
constexpr float kTuneMargin = 0.015f;

// Trailing padding of the admittance-entry arrays (>= the batched kernel's
// entry group size minus one).
constexpr int kEntryPad = 8;

// Largest tile size whose Jacobian rows are assembled in LDS (6 x 256 values
// = 12 KB per wavefront).
constexpr int kStageMaxTile = 256;
// LDS a workgroup of the single-instance kernel may claim.
constexpr size_t kMaxBlockLds = 64 * 1024;

struct DevPlan {
    int device = 0;
    std::vector<void *> allocs;
    // structure
    int32_t *yptr = nullptr, *ycol = nullptr, *cptr = nullptr, *clist = nullptr;
    int4 *bus4 = nullptr;
    int2 *bus2 = nullptr;
    int32_t *shptr = nullptr, *shlist = nullptr, *ldptr = nullptr, *ldlist = nullptr;
    int4 *gen4 = nullptr;
    double2 *gen2 = nullptr;
    int32_t *genpv = nullptr;
    int32_t *br_f = nullptr, *br_t = nullptr, *br_on = nullptr, *load_bus = nullptr;
    int2 *busx = nullptr;
    int32_t *ytr = nullptr;
    GridDev *grids = nullptr;
    int4 *tiles = nullptr;
    int32_t ntiles_alloc = 0;
    // data
    double *params = nullptr, *pv_p = nullptr, *shunt_g = nullptr, *shunt_b = nullptr;
    // derived
    double *yG = nullptr, *yB = nullptr;
    double2 *spec = nullptr;
    // batched overlay
    double *lscale = nullptr, *pscale = nullptr;
    int32_t *outage = nullptr;
    int2 *out_ft = nullptr;   // per instance: buses of its outaged branch, or -1
    double *otab = nullptr;
    int32_t *order_nat = nullptr, *order_bfs = nullptr;
    // adjoint work lists (single-instance and multi-grid plans)
    int4 *adj_tiles = nullptr;
    int32_t *adj_src = nullptr, *adj_own = nullptr, *adj_left = nullptr;
    // Newton scratch (allocated at setup for single-instance plans)
    double *nw_F = nullptr, *nw_J = nullptr, *nw_dx = nullptr;
};

template <typename T>
static int dalloc(DevPlan *dp, T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return PF_OK;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess) return fail(PF_ENOMEM, "hipMalloc(%zu bytes): %s", count * sizeof(T),
                                     hipGetErrorString(e));
    dp->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return PF_OK;
}

template <typename T, typename S>
static int dupload(DevPlan *dp, T **p, const std::vector<S> &v) {
    static_assert(sizeof(S) <= sizeof(T), "element size");
    const size_t bytes = v.size() * sizeof(S);
    const size_t count = (bytes + sizeof(T) - 1) / sizeof(T);
    int rc = dalloc(dp, p, count);
    if (rc) return rc;
    if (bytes) HIP_TRY(hipMemcpy(*p, v.data(), bytes, hipMemcpyHostToDevice));
    return PF_OK;
}

// ---------------------------------------------------------------------------
// setup-time coefficients
// ---------------------------------------------------------------------------

// Admittance contribution of one branch end pair to entry (i, j):
//   FF: (y + j b/2) / t^2          TT: y + j b/2
//   FT: -y e^{j phi} / t           TF: -y e^{-j phi} / t
// with y = g + jb = 1/(r + jx).
__device__ __forceinline__ void branch_term(const double *__restrict__ P, int64_t B, int br,
                                            int kind, double &G, double &Bv) {
    const double r = P[br], x = P[B + br], bc = P[2 * B + br];
    const double tap = P[3 * B + br], sh = P[4 * B + br];
    const double d = r * r + x * x;
    const double g = r / d;
    const double b = -x / d;
    if (kind == K_FF) {
        const double t2 = tap * tap;
        G = g / t2;
        Bv = (b + 0.5 * bc) / t2;
    } else if (kind == K_TT) {
        G = g;
        Bv = b + 0.5 * bc;
    } else {
        double sp, cp;
        sincos(sh * (M_PI / 180.0), &sp, &cp);
        if (kind == K_FT) {
            G = -(g * cp - b * sp) / tap;
            Bv = -(g * sp + b * cp) / tap;
        } else {
            G = -(g * cp + b * sp) / tap;
            Bv = -(b * cp - g * sp) / tap;
        }
    }
}

// One lane per bus: admittance entries of its row, then its specified
// injection (loads minus PV setpoint).  Sums run in fixed list order.
__global__ void __launch_bounds__(256)
k_build_coeffs(int Nt, int64_t B, const int32_t *__restrict__ yptr, const int2 *__restrict__ bus2,
               const int32_t *__restrict__ cptr, const int32_t *__restrict__ clist,
               const int32_t *__restrict__ shptr, const int32_t *__restrict__ shlist,
               const double *__restrict__ shg, const double *__restrict__ shb,
               const int32_t *__restrict__ ldptr, const int32_t *__restrict__ ldlist,
               const double *__restrict__ P, int64_t NL, const int32_t *__restrict__ genpv,
               const double *__restrict__ pv_p, double *__restrict__ yG,
               double *__restrict__ yB, double2 *__restrict__ spec) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= Nt) return;
    const int32_t ys = yptr[b], ye = yptr[b + 1];
    const int2 b2 = bus2[b];
    for (int32_t e = ys; e < ye; ++e) {
        double G = 0.0, Bv = 0.0;
        for (int32_t c = cptr[e]; c < cptr[e + 1]; ++c) {
            const int32_t code = clist[c];
            double g, bb;
            branch_term(P, B, code >> 2, code & 3, g, bb);
            G += g;
            Bv += bb;
        }
        if (e - ys == b2.x) {
            for (int32_t s = shptr[b]; s < shptr[b + 1]; ++s) {
                G += shg[shlist[s]];
                Bv += shb[shlist[s]];
            }
        }
        yG[e] = G;
        yB[e] = Bv;
    }
    const double *lp = P + 5 * B;
    const double *lq = lp + NL;
    double sp = 0.0, sq = 0.0;
    for (int32_t l = ldptr[b]; l < ldptr[b + 1]; ++l) {
        sp += lp[ldlist[l]];
        sq += lq[ldlist[l]];
    }
    if (b2.y >= 0 && genpv[b2.y] >= 0) sp = sp - pv_p[genpv[b2.y]];
    spec[b] = make_double2(sp, sq);
}

// One lane per branch: the four admittance terms it adds (FF, FT, TF, TT as
// G, B pairs), used to take a branch out in N-1 instances.
__global__ void __launch_bounds__(256)
k_outage_table(int64_t B, const double *__restrict__ P, double *__restrict__ otab) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B) return;
    for (int k = 0; k < 4; ++k) {
        double G, Bv;
        branch_term(P, B, e, k, G, Bv);
        otab[8 * int64_t(e) + 2 * k] = G;
        otab[8 * int64_t(e) + 2 * k + 1] = Bv;
    }
}

// ---------------------------------------------------------------------------
// evaluation
// ---------------------------------------------------------------------------

// Contribution of admittance entry (i, j) to row i.
//   c[0..5]: P_i, Q_i, dP_i/dth_i, dP_i/dV_i, dQ_i/dth_i, dQ_i/dV_i
//   o[0..3]: dP_i/dth_j, dP_i/dV_j, dQ_i/dth_j, dQ_i/dV_j   (j != i only)
__device__ __forceinline__ void entry_eval(bool diag, double G, double B, double thi, double vi,
                                           double thj, double vj, double c[6], double o[4]) {
    if (diag) {
        const double vi2 = vi * vi;
        c[0] = vi2 * G;
        c[1] = -(vi2 * B);
        c[2] = 0.0;
        c[3] = 2.0 * vi * G;
        c[4] = 0.0;
        c[5] = -(2.0 * vi * B);
        o[0] = o[1] = o[2] = o[3] = 0.0;
    } else {
        double s, co;
        sincos(thi - thj, &s, &co);
        const double t1 = fma(G, co, B * s);     // G cos + B sin
        const double t2 = fma(G, s, -(B * co));  // G sin - B cos
        const double vv = vi * vj;
        const double a = vv * t1;
        const double q = vv * t2;
        c[0] = a;
        c[1] = q;
        c[2] = -q;
        c[3] = vj * t1;
        c[4] = a;
        c[5] = vj * t2;
        o[0] = q;
        o[1] = vi * t1;
        o[2] = -a;
        o[3] = vi * t2;
    }
}

// Logical workgroup id that gives each XCD a contiguous range: the hardware
// hands workgroup ids to the 8 XCDs round-robin.
__device__ __forceinline__ int xcd_logical_block(int bid, int nb) {
    const int q = nb >> 3, r = nb & 7, x = bid & 7;
    return x * q + min(x, r) + (bid >> 3);
}

// Output stores are streamed (non-temporal): the residual and Jacobian
// values are written once and never re-read by the kernel, and keeping them
// out of L2 leaves it to the state gathers, which neighbouring buses reuse.
__device__ __forceinline__ void st(double *p, double v) { __builtin_nontemporal_store(v, p); }
// Scattered 8-byte output stores (single-instance kernel) stay cached so that
// L2 can merge them into whole lines before they are written back.
__device__ __forceinline__ void stc(double *p, double v) { *p = v; }

// A row of cotangent-fastest data addressed as a raw buffer: the row base in
// scalar registers, each lane's byte offset in one vector register shared by
// every row it touches.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const double *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(p), 0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ double rld(const double *row, int off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(row_rsrc(row), off, 0, 0));
}
__device__ __forceinline__ void rst(double *row, int off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), row_rsrc(row), off, 0, 2);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Single-instance fused residual + Jacobian.  Each wavefront walks a
// contiguous range of tiles; a tile is a run of whole admittance rows,
// processed 64 entries (one per lane) at a time.  The six per-entry row
// contributions are staged in LDS and left-folded by the lane that holds the
// first entry of each row (or lane 0 for a row continuing from the previous
// chunk, which picks up the carried partial sums).  The tile's Jacobian rows
// P_i and Q_i occupy two contiguous value ranges; when they fit the wave's
// staging area they are assembled in LDS and written out as whole runs,
// otherwise (a very long row) values go straight to their slots.
template <bool WF, bool WJ>
__global__ void __launch_bounds__(512)
k_eval_single(const int4 *__restrict__ tiles, int ntiles, int tiles_per_wave, int remap,
              int stage_cap, const GridDev *__restrict__ grids, const int4 *__restrict__ bus4,
              const int2 *__restrict__ bus2, const double2 *__restrict__ spec,
              const int32_t *__restrict__ ycol, const double *__restrict__ yG,
              const double *__restrict__ yB, const int4 *__restrict__ gen4,
              const double2 *__restrict__ gen2, const double *__restrict__ x,
              double *__restrict__ F, double *__restrict__ J) {
    extern __shared__ double lds[];
    const int lane = threadIdx.x & 63;
    // wave index is uniform across the wavefront; telling the compiler so
    // keeps the tile walk and every row-structure load in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    double *L = lds + size_t(wv) * (6 * 64 + stage_cap);
    double *S = L + 6 * 64;
    const int lb = remap ? xcd_logical_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int lw = lb * wpb + wv;
    const int t_begin = lw * tiles_per_wave;
    const int t_end = min(ntiles, t_begin + tiles_per_wave);
    const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    for (int t = t_begin; t < t_end; ++t) {
        const int4 td = tiles[2 * t];
        const int4 tj = tiles[2 * t + 1];
        const int e0 = td.x, e1 = td.y, b0 = td.z;
        const int jP0 = tj.x, nP = tj.y - tj.x, jQ0 = tj.z, nQ = tj.w - tj.z;
        const bool staged = WJ && (nP + nQ <= stage_cap);
        // the tile's walk, compiled once with the Jacobian rows assembled in
        // LDS and once with values stored straight to their slots, so that
        // each store has one address space
        auto walk = [&](auto staged_c) {
            constexpr bool STG = decltype(staged_c)::value;
            // Jacobian value of row P_i (slot s) / row Q_i: LDS image or global
            auto putP = [&](int slot, double v) {
                if constexpr (STG)
                    S[slot - jP0] = v;
                else
                    stc(&J[slot], v);
            };
            auto putQ = [&](int slot, double v) {
                if constexpr (STG)
                    S[nP + slot - jQ0] = v;
                else
                    stc(&J[slot], v);
            };
            const GridDev gd = grids[td.w];
            const double *xt = x + gd.xoff;
            const double *xv = xt + gd.N;
            double cy[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int rows_seen = 0;
            // entry data of the first chunk; later chunks are fetched one chunk
            // ahead, while the current one computes
            int raw_n = lane < e1 - e0 ? ycol[e0 + lane] : 0;
            double G_n = lane < e1 - e0 ? yG[e0 + lane] : 0.0;
            double B_n = lane < e1 - e0 ? yB[e0 + lane] : 0.0;
            for (int c0 = e0; c0 < e1; c0 += 64) {
                const int nvalid = min(64, e1 - c0);
                const bool valid = lane < nvalid;
                const int e = c0 + lane;
                const int raw = raw_n;
                const double Ge = G_n, Be = B_n;
                const bool start = raw < 0;
                const int j = raw & kColMask;
                const uint64_t smask = __ballot(start);
                const int r = rows_seen + __popcll(smask & le) - 1;
                // lanes past the tile end read a valid duplicate (the tile's
                // first bus) so every per-bus load is issued at once, unmasked
                const int b = valid ? b0 + r : b0;
                const int i = b - gd.bus_off;
                const int4 bi = bus4[b];
                const int2 b2 = bus2[b];
                const double2 sp = spec[b];
                const double thi = xt[i], vi = xv[i];
                const double thj = xt[j], vj = xv[j];
                const bool more = c0 + 64 < e1;
                if (more) {
                    const int en = c0 + 64 + lane;
                    const bool vn = en < e1;
                    raw_n = vn ? ycol[en] : 0;
                    G_n = vn ? yG[en] : 0.0;
                    B_n = vn ? yB[en] : 0.0;
                }
                double c[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                if (valid) {
                    double o[4];
                    const bool diag = (j == i);
                    entry_eval(diag, Ge, Be, thi, vi, thj, vj, c, o);
                    if (WJ && !diag) {
                        const int p = e - bi.x, Lr = bi.y - bi.x;
                        putP(bi.z + p, o[0]);
                        putP(bi.z + Lr + p, o[1]);
                        putQ(bi.w + p, o[2]);
                        putQ(bi.w + Lr + p, o[3]);
                    }
                }
    #pragma unroll
                for (int k = 0; k < 6; ++k) L[k * 64 + lane] = c[k];
                wave_sync();
                const bool carry_row = !(smask & 1ull);
                const bool folder = start || (lane == 0 && carry_row);
                const uint64_t after = smask & ~le;
                const int next = after ? (__ffsll((unsigned long long)after) - 1) : nvalid;
                // the entry after this chunk opens a row iff its column carries
                // the row-start flag (that entry is lane 0 of the prefetch)
                const bool next_is_start = more ? (__shfl(raw_n, 0) < 0) : true;
                const bool complete = (next < nvalid) || next_is_start;
                double a[6];
    #pragma unroll
                for (int k = 0; k < 6; ++k) a[k] = (lane == 0 && carry_row) ? cy[k] : 0.0;
                if (folder) {
                    for (int q = lane; q < next; ++q) {
    #pragma unroll
                        for (int k = 0; k < 6; ++k) a[k] += L[k * 64 + q];
                    }
                }
                if (!next_is_start) {
                    const int lastf = smask ? 63 - __clzll((long long)smask) : 0;
    #pragma unroll
                    for (int k = 0; k < 6; ++k) cy[k] = __shfl(a[k], lastf);
                }
                if (folder && complete) {
                    const int Lr = bi.y - bi.x;
                    double fp = a[0] + sp.x;
                    double fq = a[1] + sp.y;
                    const int g = b2.y;
                    if (g >= 0) {
                        const int4 g4 = gen4[g];
                        const double2 gs = gen2[g];
                        const double qg = x[g4.x];
                        const bool held = g4.z == kGenHeld;
                        fq = fq - qg;
                        if (WF) stc(&F[g4.x], held ? qg - gs.x : vi - gs.x);
                        if (WJ) {
                            putQ(bi.w + 2 * Lr, -1.0);
                            stc(&J[g4.y], held ? 0.0 : 1.0);
                            if (g4.z <= kGenVoltageSlot) stc(&J[g4.y + 1], held ? 1.0 : 0.0);
                        }
                        if (g4.z >= 0) {
                            fp = fp - x[g4.z];
                            if (WF) stc(&F[g4.z], thi - gs.y);
                            if (WJ) {
                                putP(bi.z + 2 * Lr, -1.0);
                                stc(&J[g4.w], 1.0);
                            }
                        }
                    }
                    if (WF) {
                        stc(&F[gd.xoff + i], fp);
                        stc(&F[gd.xoff + gd.N + i], fq);
                    }
                    if (WJ) {
                        putP(bi.z + b2.x, a[2]);
                        putP(bi.z + Lr + b2.x, a[3]);
                        putQ(bi.w + b2.x, a[4]);
                        putQ(bi.w + Lr + b2.x, a[5]);
                    }
                }
                rows_seen += __popcll(smask);
                wave_sync();
            }
            if constexpr (STG) {
                // every slot of both ranges has been written above; stream the
                // assembled rows out as contiguous runs
                for (int q = lane; q < nP; q += 64) st(&J[jP0 + q], S[q]);
                for (int q = lane; q < nQ; q += 64) st(&J[jQ0 + q], S[nP + q]);
                wave_sync();
            }
        };
        if (staged)
            walk(std::true_type{});
        else
            walk(std::false_type{});
    }
}

// Batched fused residual + Jacobian, instance-fastest layout: lane = instance
// (64 instances per wavefront), so every state gather and every output store
// is a contiguous 512 B row segment, while the row structure and coefficients
// are wave-uniform scalar loads.  A work item is (instance chunk, run of
// buses in the chosen order); each wavefront walks a contiguous item range.
// Per-instance overlays: load / PV scale factors (SCEN) and one branch taken
// out (OUTG), whose admittance terms are subtracted from the entries it
// joins -- exactly cancelling them when no parallel branch remains.
template <bool WF, bool WJ, bool SCEN, bool OUTG>
__global__ void __launch_bounds__(512)
k_eval_batch(int N, int I, int LD, int panel, int64_t rows_x, int64_t rows_j, int n_btiles,
             int n_chunks, int TB, int n_items, int items_per_wave,
             int remap, int group,
             const int32_t *__restrict__ order, const int4 *__restrict__ bus4,
             const int2 *__restrict__ bus2, const double2 *__restrict__ spec,
             const int32_t *__restrict__ ycol, const double *__restrict__ yG,
             const double *__restrict__ yB, const int4 *__restrict__ gen4,
             const double2 *__restrict__ gen2, const int32_t *__restrict__ genpv,
             const int32_t *__restrict__ ldptr, const int32_t *__restrict__ ldlist,
             const double *__restrict__ lp, const double *__restrict__ lq,
             const double *__restrict__ pv_p, const double *__restrict__ lscale,
             const double *__restrict__ pscale, const int32_t *__restrict__ outage,
             const int2 *__restrict__ out_ft, const double *__restrict__ otab,
             const double *__restrict__ X,
             double *__restrict__ F, double *__restrict__ J) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    const int lb = remap ? xcd_logical_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int lw = lb * wpb + wv;
    const int w_begin = lw * items_per_wave;
    const int w_end = min(n_items, w_begin + items_per_wave);
    const size_t OLD = size_t(LD);   // row pitch of the overlay tables
    int cur_chunk = -1;
    int of = -1, ot = -1;   // buses of this lane's outaged branch
    for (int w = w_begin; w < w_end; ++w) {
        // item -> (chunk group, bus run, chunk inside the group)
        const int per_group = n_btiles * group;
        const int sg = w / per_group;
        const int rem = w - sg * per_group;
        const int bt = rem / group;
        const int ch = sg * group + (rem - bt * group);
        if (ch >= n_chunks) continue;
        const int k = ch * 64 + lane;
        const bool valid = k < I;
        if (OUTG && ch != cur_chunk) {
            cur_chunk = ch;
            const int2 ft = valid ? out_ft[k] : make_int2(-1, -1);
            of = ft.x;
            ot = ft.y;
        }
        const int q0 = bt * TB;
        const int q1 = min(N, q0 + TB);
        // rows of pitch LD (column k), or the chunk's panel of 64 (column lane)
        const size_t SI = panel ? 64 : size_t(LD);
        const size_t kq = panel ? size_t(lane) : size_t(k);
        const size_t xo = panel ? size_t(ch) * size_t(rows_x) * 64 : 0;
        const size_t jo = panel ? size_t(ch) * size_t(rows_j) * 64 : 0;
        const double *Xc = X + xo;
        double *Fc = F ? F + xo : nullptr;
        double *Jc = J ? J + jo : nullptr;
        // masked lanes read a valid duplicate address so loads need no
        // masking (a panel is always 64 columns wide)
        const size_t kk = panel ? kq : size_t(valid ? k : I - 1);
        constexpr int EU = 4;
        if constexpr (!SCEN && !OUTG) {
            // Without an overlay, every vector load of a row (own state,
            // generator variables, the first EU partners) is issued before the
            // row's first store. A wavefront's loads complete in order behind
            // its earlier stores, so a load issued after a store also waits for
            // that store's write. The overlay walk below instead fetches the
            // next row's header and state one row ahead: it keeps fewer
            // registers live there, and measured faster for it.
            for (int qq = q0; qq < q1; ++qq) {
                const int b = order[qq];
                const int4 bi = bus4[b];
                const int2 b2 = bus2[b];
                const int L = bi.y - bi.x;
                const double thi = Xc[size_t(b) * SI + kk];
                const double vi = Xc[size_t(N + b) * SI + kk];
                int4 g4 = make_int4(0, 0, 0, 0);
                double2 gs = make_double2(0.0, 0.0);
                double qg = 0.0, ps = 0.0;
                if (b2.y >= 0) {
                    g4 = gen4[b2.y];
                    gs = gen2[b2.y];
                    qg = Xc[size_t(g4.x) * SI + kk];
                    if (g4.z >= 0) ps = Xc[size_t(g4.z) * SI + kk];
                }
                // entry arrays carry kEntryPad trailing entries, so the first
                // group's coefficients are read unconditionally
                int jj[EU];
                double GG[EU], BB[EU], thj[EU], vj[EU];
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    jj[u] = ycol[bi.x + u] & kColMask;
                    GG[u] = yG[bi.x + u];
                    BB[u] = yB[bi.x + u];
                }
                // the diagonal entry needs no partner state: its loads
                // would only repeat the bus's own
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    thj[u] = thi;
                    vj[u] = vi;
                    if (u < L && u != b2.x) {
                        thj[u] = Xc[size_t(jj[u]) * SI + kk];
                        vj[u] = Xc[size_t(N + jj[u]) * SI + kk];
                    }
                }
                double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                auto entry = [&](int p, int j, double G, double Bv, double tj, double vjj) {
                    const bool diag = (j == b);
                    double c[6], o[4];
                    entry_eval(diag, G, Bv, thi, vi, tj, vjj, c, o);
                    if (WJ && !diag && valid) {
                        st(&Jc[size_t(bi.z + p) * SI + kq], o[0]);
                        st(&Jc[size_t(bi.z + L + p) * SI + kq], o[1]);
                        st(&Jc[size_t(bi.w + p) * SI + kq], o[2]);
                        st(&Jc[size_t(bi.w + L + p) * SI + kq], o[3]);
                    }
#pragma unroll
                    for (int q = 0; q < 6; ++q) a[q] += c[q];
                };
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    if (u >= L) break;
                    entry(u, jj[u], GG[u], BB[u], thj[u], vj[u]);
                }
                // a longer row continues in groups of EU
                for (int e0 = bi.x + EU; e0 < bi.y; e0 += EU) {
                    int j2[EU];
                    double G2[EU], B2[EU], t2[EU], v2[EU];
#pragma unroll
                    for (int u = 0; u < EU; ++u) {
                        j2[u] = ycol[e0 + u] & kColMask;
                        G2[u] = yG[e0 + u];
                        B2[u] = yB[e0 + u];
                    }
#pragma unroll
                    for (int u = 0; u < EU; ++u) {
                        t2[u] = thi;
                        v2[u] = vi;
                        if (e0 + u < bi.y && j2[u] != b) {
                            t2[u] = Xc[size_t(j2[u]) * SI + kk];
                            v2[u] = Xc[size_t(N + j2[u]) * SI + kk];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < EU; ++u) {
                        if (e0 + u >= bi.y) break;
                        entry(e0 + u - bi.x, j2[u], G2[u], B2[u], t2[u], v2[u]);
                    }
                }
                if (!valid) continue;
                const double2 sp = spec[b];
                double fp = a[0] + sp.x;
                double fq = a[1] + sp.y;
                if (b2.y >= 0) {
                    const bool held = g4.z == kGenHeld;
                    fq = fq - qg;
                    if (WF) st(&Fc[size_t(g4.x) * SI + kq], held ? qg - gs.x : vi - gs.x);
                    if (WJ) {
                        st(&Jc[size_t(bi.w + 2 * L) * SI + kq], -1.0);
                        st(&Jc[size_t(g4.y) * SI + kq], held ? 0.0 : 1.0);
                        if (g4.z <= kGenVoltageSlot)
                            st(&Jc[size_t(g4.y + 1) * SI + kq], held ? 1.0 : 0.0);
                    }
                    if (g4.z >= 0) {
                        fp = fp - ps;
                        if (WF) st(&Fc[size_t(g4.z) * SI + kq], thi - gs.y);
                        if (WJ) {
                            st(&Jc[size_t(bi.z + 2 * L) * SI + kq], -1.0);
                            st(&Jc[size_t(g4.w) * SI + kq], 1.0);
                        }
                    }
                }
                if (WF) {
                    st(&Fc[size_t(b) * SI + kq], fp);
                    st(&Fc[size_t(N + b) * SI + kq], fq);
                }
                if (WJ) {
                    st(&Jc[size_t(bi.z + b2.x) * SI + kq], a[2]);
                    st(&Jc[size_t(bi.z + L + b2.x) * SI + kq], a[3]);
                    st(&Jc[size_t(bi.w + b2.x) * SI + kq], a[4]);
                    st(&Jc[size_t(bi.w + L + b2.x) * SI + kq], a[5]);
                }
            }
            continue;
        }
        // the next bus's row header and own state are fetched one bus ahead
        int b_nx = order[q0];
        int4 bi_nx = bus4[b_nx];
        double thi_nx = Xc[size_t(b_nx) * SI + kk];
        double vi_nx = Xc[size_t(N + b_nx) * SI + kk];
        for (int qq = q0; qq < q1; ++qq) {
            const int b = b_nx;
            const int4 bi = bi_nx;
            const double thi = thi_nx, vi = vi_nx;
            if (qq + 1 < q1) {
                b_nx = order[qq + 1];
                bi_nx = bus4[b_nx];
                thi_nx = Xc[size_t(b_nx) * SI + kk];
                vi_nx = Xc[size_t(N + b_nx) * SI + kk];
            }
            const int Lr = bi.y - bi.x;
            // a lane whose outaged branch touches this bus fetches the terms
            // that branch adds to the diagonal and to the other end's entry
            int oc = -1;
            double dGd = 0.0, dBd = 0.0, dGo = 0.0, dBo = 0.0;
            if (OUTG && (of == b || ot == b)) {
                const size_t o8 = 8 * size_t(outage[k]);
                const bool from = of == b;
                oc = from ? ot : of;
                dGd = otab[o8 + (from ? 0 : 6)];
                dBd = otab[o8 + (from ? 1 : 7)];
                dGo = otab[o8 + (from ? 2 : 4)];
                dBo = otab[o8 + (from ? 3 : 5)];
            }
            double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            // entries in groups of EU: all gathers of a group are issued
            // before any of its arithmetic, so they are in flight together
            for (int e0 = bi.x; e0 < bi.y; e0 += EU) {
                int jj[EU];
                double GG[EU], BB[EU], thj[EU], vj[EU];
                // the entry arrays carry kEntryPad trailing entries (column 0,
                // zero admittance), so a group may read past the last row
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    jj[u] = ycol[e0 + u] & kColMask;
                    GG[u] = yG[e0 + u];
                    BB[u] = yB[e0 + u];
                }
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    thj[u] = thi;
                    vj[u] = vi;
                    if (e0 + u < bi.y && jj[u] != b) {
                        thj[u] = Xc[size_t(jj[u]) * SI + kk];
                        vj[u] = Xc[size_t(N + jj[u]) * SI + kk];
                    }
                }
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    const int e = e0 + u;
                    if (e >= bi.y) break;
                    const int j = jj[u];
                    double G = GG[u], Bv = BB[u];
                    const bool diag = (j == b);
                    if (OUTG && oc >= 0) {
                        if (diag) {
                            G -= dGd;
                            Bv -= dBd;
                        } else if (j == oc) {
                            G -= dGo;
                            Bv -= dBo;
                        }
                    }
                    double c[6], o[4];
                    entry_eval(diag, G, Bv, thi, vi, thj[u], vj[u], c, o);
                    if (WJ && !diag && valid) {
                        const int p = e - bi.x;
                        st(&Jc[size_t(bi.z + p) * SI + kq], o[0]);
                        st(&Jc[size_t(bi.z + Lr + p) * SI + kq], o[1]);
                        st(&Jc[size_t(bi.w + p) * SI + kq], o[2]);
                        st(&Jc[size_t(bi.w + Lr + p) * SI + kq], o[3]);
                    }
#pragma unroll
                    for (int q = 0; q < 6; ++q) a[q] += c[q];
                }
            }
            if (!valid) continue;
            const int2 b2 = bus2[b];
            double spx, spy;
            if (SCEN) {
                spx = 0.0;
                spy = 0.0;
                for (int l = ldptr[b]; l < ldptr[b + 1]; ++l) {
                    const int ld = ldlist[l];
                    const double s = lscale ? lscale[size_t(ld) * OLD + k] : 1.0;
                    spx += lp[ld] * s;
                    spy += lq[ld] * s;
                }
                if (b2.y >= 0) {
                    const int pv = genpv[b2.y];
                    if (pv >= 0) {
                        const double s = pscale ? pscale[size_t(pv) * OLD + k] : 1.0;
                        spx = spx - pv_p[pv] * s;
                    }
                }
            } else {
                const double2 sp = spec[b];
                spx = sp.x;
                spy = sp.y;
            }
            double fp = a[0] + spx;
            double fq = a[1] + spy;
            const int g = b2.y;
            if (g >= 0) {
                const int4 g4 = gen4[g];
                const double2 gs = gen2[g];
                const double qg = Xc[size_t(g4.x) * SI + kq];
                const bool held = g4.z == kGenHeld;
                fq = fq - qg;
                if (WF) st(&Fc[size_t(g4.x) * SI + kq], held ? qg - gs.x : vi - gs.x);
                if (WJ) {
                    st(&Jc[size_t(bi.w + 2 * Lr) * SI + kq], -1.0);
                    st(&Jc[size_t(g4.y) * SI + kq], held ? 0.0 : 1.0);
                    if (g4.z <= kGenVoltageSlot)
                        st(&Jc[size_t(g4.y + 1) * SI + kq], held ? 1.0 : 0.0);
                }
                if (g4.z >= 0) {
                    fp = fp - Xc[size_t(g4.z) * SI + kq];
                    if (WF) st(&Fc[size_t(g4.z) * SI + kq], thi - gs.y);
                    if (WJ) {
                        st(&Jc[size_t(bi.z + 2 * Lr) * SI + kq], -1.0);
                        st(&Jc[size_t(g4.w) * SI + kq], 1.0);
                    }
                }
            }
            if (WF) {
                st(&Fc[size_t(b) * SI + kq], fp);
                st(&Fc[size_t(N + b) * SI + kq], fq);
            }
            if (WJ) {
                st(&Jc[size_t(bi.z + b2.x) * SI + kq], a[2]);
                st(&Jc[size_t(bi.z + Lr + b2.x) * SI + kq], a[3]);
                st(&Jc[size_t(bi.w + b2.x) * SI + kq], a[4]);
                st(&Jc[size_t(bi.w + Lr + b2.x) * SI + kq], a[5]);
            }
        }
    }
}

// Batched fused residual + Jacobian without overlays, two instances per lane:
// a wavefront covers 128 instances, every state gather and output store is
// 16 bytes per lane (1 KB per instruction), and each bus's structure, row
// coefficients and scalar lookups serve twice the data.  For row layouts
// whose instance count and pitch are even (so every pair is 16-byte
// aligned).  The walk and its arithmetic are those of k_eval_batch's
// overlay-free path, per instance, so the outputs are bit-identical.
typedef double d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ d2 ld2(const double *p) { return *reinterpret_cast<const d2 *>(p); }
__device__ __forceinline__ void st2(double *p, d2 v) {
    __builtin_nontemporal_store(v, reinterpret_cast<d2 *>(p));
}
template <bool WF, bool WJ>
__global__ void __launch_bounds__(512)
k_eval_batch2(int N, int I, int LD, int n_btiles, int n_chunks, int TB, int n_items,
              int items_per_wave, int remap, int group, const int32_t *__restrict__ order,
              const int4 *__restrict__ bus4, const int2 *__restrict__ bus2,
              const double2 *__restrict__ spec, const int32_t *__restrict__ ycol,
              const double *__restrict__ yG, const double *__restrict__ yB,
              const int4 *__restrict__ gen4, const double2 *__restrict__ gen2,
              const double *__restrict__ X, double *__restrict__ F, double *__restrict__ J) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    const int lb = remap ? xcd_logical_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int lw = lb * wpb + wv;
    const int w_begin = lw * items_per_wave;
    const int w_end = min(n_items, w_begin + items_per_wave);
    const size_t SI = size_t(LD);
    for (int w = w_begin; w < w_end; ++w) {
        const int per_group = n_btiles * group;
        const int sg = w / per_group;
        const int rem = w - sg * per_group;
        const int bt = rem / group;
        const int ch = sg * group + (rem - bt * group);
        if (ch >= n_chunks) continue;
        const int k0 = ch * 128 + 2 * lane;
        const bool valid = k0 < I;
        const size_t kk = size_t(valid ? k0 : I - 2);
        const size_t kq = size_t(k0);
        const int q0 = bt * TB;
        const int q1 = min(N, q0 + TB);
        constexpr int EU = 4;
        for (int qq = q0; qq < q1; ++qq) {
            const int b = order[qq];
            const int4 bi = bus4[b];
            const int2 b2 = bus2[b];
            const int L = bi.y - bi.x;
            const d2 thi = ld2(X + size_t(b) * SI + kk);
            const d2 vi = ld2(X + size_t(N + b) * SI + kk);
            int4 g4 = make_int4(0, 0, 0, 0);
            double2 gs = make_double2(0.0, 0.0);
            d2 qg = {0.0, 0.0}, ps = {0.0, 0.0};
            if (b2.y >= 0) {
                g4 = gen4[b2.y];
                gs = gen2[b2.y];
                qg = ld2(X + size_t(g4.x) * SI + kk);
                if (g4.z >= 0) ps = ld2(X + size_t(g4.z) * SI + kk);
            }
            int jj[EU];
            double GG[EU], BB[EU];
            d2 thj[EU], vj[EU];
#pragma unroll
            for (int u = 0; u < EU; ++u) {
                jj[u] = ycol[bi.x + u] & kColMask;
                GG[u] = yG[bi.x + u];
                BB[u] = yB[bi.x + u];
            }
#pragma unroll
            for (int u = 0; u < EU; ++u) {
                thj[u] = thi;
                vj[u] = vi;
                if (u < L && u != b2.x) {
                    thj[u] = ld2(X + size_t(jj[u]) * SI + kk);
                    vj[u] = ld2(X + size_t(N + jj[u]) * SI + kk);
                }
            }
            double ax[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            double ay[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            auto entry = [&](int p, int j, double G, double Bv, d2 tj, d2 vjj) {
                const bool diag = (j == b);
                double cx[6], ox[4], cy[6], oy[4];
                entry_eval(diag, G, Bv, thi.x, vi.x, tj.x, vjj.x, cx, ox);
                entry_eval(diag, G, Bv, thi.y, vi.y, tj.y, vjj.y, cy, oy);
                if (WJ && !diag && valid) {
                    st2(J + size_t(bi.z + p) * SI + kq, d2{ox[0], oy[0]});
                    st2(J + size_t(bi.z + L + p) * SI + kq, d2{ox[1], oy[1]});
                    st2(J + size_t(bi.w + p) * SI + kq, d2{ox[2], oy[2]});
                    st2(J + size_t(bi.w + L + p) * SI + kq, d2{ox[3], oy[3]});
                }
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    ax[q] += cx[q];
                    ay[q] += cy[q];
                }
            };
#pragma unroll
            for (int u = 0; u < EU; ++u) {
                if (u >= L) break;
                entry(u, jj[u], GG[u], BB[u], thj[u], vj[u]);
            }
            for (int e0 = bi.x + EU; e0 < bi.y; e0 += EU) {
                int j2[EU];
                double G2[EU], B2[EU];
                d2 t2[EU], v2[EU];
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    j2[u] = ycol[e0 + u] & kColMask;
                    G2[u] = yG[e0 + u];
                    B2[u] = yB[e0 + u];
                }
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    t2[u] = thi;
                    v2[u] = vi;
                    if (e0 + u < bi.y && j2[u] != b) {
                        t2[u] = ld2(X + size_t(j2[u]) * SI + kk);
                        v2[u] = ld2(X + size_t(N + j2[u]) * SI + kk);
                    }
                }
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    if (e0 + u >= bi.y) break;
                    entry(e0 + u - bi.x, j2[u], G2[u], B2[u], t2[u], v2[u]);
                }
            }
            if (!valid) continue;
            const double2 sp = spec[b];
            d2 fp = {ax[0] + sp.x, ay[0] + sp.x};
            d2 fq = {ax[1] + sp.y, ay[1] + sp.y};
            if (b2.y >= 0) {
                const bool held = g4.z == kGenHeld;
                fq = fq - qg;
                if (WF) st2(F + size_t(g4.x) * SI + kq, held ? qg - gs.x : vi - gs.x);
                if (WJ) {
                    st2(J + size_t(bi.w + 2 * L) * SI + kq, d2{-1.0, -1.0});
                    const double cv = held ? 0.0 : 1.0;
                    st2(J + size_t(g4.y) * SI + kq, d2{cv, cv});
                    if (g4.z <= kGenVoltageSlot) {
                        const double cq = held ? 1.0 : 0.0;
                        st2(J + size_t(g4.y + 1) * SI + kq, d2{cq, cq});
                    }
                }
                if (g4.z >= 0) {
                    fp = fp - ps;
                    if (WF) st2(F + size_t(g4.z) * SI + kq, thi - gs.y);
                    if (WJ) {
                        st2(J + size_t(bi.z + 2 * L) * SI + kq, d2{-1.0, -1.0});
                        st2(J + size_t(g4.w) * SI + kq, d2{1.0, 1.0});
                    }
                }
            }
            if (WF) {
                st2(F + size_t(b) * SI + kq, fp);
                st2(F + size_t(N + b) * SI + kq, fq);
            }
            if (WJ) {
                st2(J + size_t(bi.z + b2.x) * SI + kq, d2{ax[2], ay[2]});
                st2(J + size_t(bi.z + L + b2.x) * SI + kq, d2{ax[3], ay[3]});
                st2(J + size_t(bi.w + b2.x) * SI + kq, d2{ax[4], ay[4]});
                st2(J + size_t(bi.w + L + b2.x) * SI + kq, d2{ax[5], ay[5]});
            }
        }
    }
}

// x <- x - dx (Newton update, task 4).
__global__ void __launch_bounds__(256) k_newton_update(int64_t n, double *__restrict__ x,
                                                       const double *__restrict__ dx) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] = x[i] - dx[i];
}

// ---------------------------------------------------------------------------
// adjoint (vector-Jacobian products)
// ---------------------------------------------------------------------------

// Cotangent group of the second phase (gathers of a group are issued
// together) and branches per wavefront of the separate branch pass.
constexpr int kVjpGroup = 8;
constexpr int kVjpTile = 16;
// Entries per first-phase pass of the row walk (the adjoint tile size).
constexpr int kVjpChunk = kAdjTileEntries;

// Partials of a branch's four terminal injections P_f, Q_f, P_t, Q_t with
// respect to r, x, line charging b, tap and phase shift (per degree), from
// the pi-model with series g + jb = 1/(r + jx):
//   dg/dr = db/dx = (x^2 - r^2)/D^2, dg/dx = -2rx/D^2, db/dr = 2rx/D^2
//   (D = r^2 + x^2), chained through the flows' g and b partials; the charging
//   enters Q only; the tap partials follow from the 1/t^2 and 1/t factors;
//   a phase shift acts as -theta_f.  d[4 p + f] = dFlow_f / dParam_p.
__device__ __forceinline__ void branch_partials(double r, double xx, double bc, double tap,
                                                double sh, double thf, double vf, double tht,
                                                double vt, double d[20]) {
    const double Dd = r * r + xx * xx;
    const double D2 = Dd * Dd;
    const double g = r / Dd;
    const double b = -xx / Dd;
    const double delta = thf - tht - sh * (M_PI / 180.0);
    double S, Cc;
    sincos(delta, &S, &Cc);
    const double u = vf * vt / tap;
    const double t2 = tap * tap;
    const double A1 = u * (g * Cc + b * S), B1 = u * (g * S - b * Cc);
    const double A2 = u * (g * Cc - b * S), B2 = u * (g * S + b * Cc);
    const double vf2 = vf * vf, vt2 = vt * vt;
    // flow partials w.r.t. series g and b: [Pf, Qf, Pt, Qt]
    const double dg[4] = {vf2 / t2 - u * Cc, -(u * S), vt2 - u * Cc, u * S};
    const double db[4] = {-(u * S), -(vf2 / t2) + u * Cc, u * S, -vt2 + u * Cc};
    const double dg_dr = (xx * xx - r * r) / D2, dg_dx = -(2.0 * r * xx) / D2;
    const double db_dr = (2.0 * r * xx) / D2, db_dx = (xx * xx - r * r) / D2;
    const double deg = -(M_PI / 180.0);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        d[f] = dg[f] * dg_dr + db[f] * db_dr;
        d[4 + f] = dg[f] * dg_dx + db[f] * db_dx;
    }
    d[8] = 0.0;
    d[9] = -(vf2 / (2.0 * t2));
    d[10] = 0.0;
    d[11] = -(vt2 / 2.0);
    d[12] = -(2.0 * vf2 * g) / (t2 * tap) + A1 / tap;
    d[13] = (2.0 * vf2 * (b + 0.5 * bc)) / (t2 * tap) + B1 / tap;
    d[14] = A2 / tap;
    d[15] = -(B2 / tap);
    d[16] = deg * B1;
    d[17] = deg * (-A1);
    d[18] = deg * B2;
    d[19] = deg * A2;
}

// The adjoint, gx = J(x)^T W (WGX) and gparam = (dF/dparams)^T W (WGP), one
// wavefront per (tile of whole admittance rows, 64-cotangent chunk).
// Column a of J collects, for every entry (a, c) of row a, the entry's share
// of the diagonal sums of rows P_a and Q_a and the off-diagonal values
// J[P_c, .a], J[Q_c, .a] of the transpose-partner entry (c, a).  Phase 1
// (lane = entry) evaluates these eight state-only coefficients once per
// entry into LDS, and the 20 partials of the branch the entry carries (the
// branch from a to c); phase 2 (lane = cotangent) walks the entries in row
// order, folding the coefficients against the W rows of P_a, Q_a, P_c, Q_c,
// and writes column a when its row ends.  The same four W rows give the
// carried branch's five gradient rows (its partials dotted with them), and
// each load's two rows are the W rows of its bus (dF_p/dP_load =
// dF_q/dQ_load = 1), written when the bus's row opens.  Rows are taken in
// breadth-first order (tiles over `src`, the entry indices in that order)
// and each XCD runs a contiguous range of tiles.
// Five wavefronts per SIMD (at most 96 registers) outrun four: each
// wavefront's walk is a chain of dependent loads, so more of them in flight
// is what helps.  Every row of W, gx and gparam a wavefront touches is the
// same for all its lanes (read from LDS, made uniform), so rows are
// addressed as buffers with a scalar base and one lane offset: that keeps
// the walk within 96 registers without spilling.
template <bool WGX, bool WGP>
__global__ void __launch_bounds__(256, 5)
k_vjp(const int4 *__restrict__ tiles, int ntiles, int n_kchunks, const int32_t *__restrict__ order,
      const int32_t *__restrict__ src, const int32_t *__restrict__ own,
      const GridDev *__restrict__ grids, const int2 *__restrict__ bus2,
      const int32_t *__restrict__ ycol, const int32_t *__restrict__ ytr,
      const double *__restrict__ yG, const double *__restrict__ yB,
      const int4 *__restrict__ gen4, const int32_t *__restrict__ ldptr,
      const int32_t *__restrict__ ldlist, const double *__restrict__ P, int B, int NL,
      const double *__restrict__ x, const double *__restrict__ W, int K,
      double *__restrict__ gx, double *__restrict__ gp) {
    constexpr int CH = kVjpChunk;
    __shared__ double sc[4][8][CH];
    __shared__ double sd[4][WGP ? 20 : 1][CH];
    __shared__ int si[4][6][CH];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wid = xcd_logical_block(blockIdx.x, gridDim.x) * 4 + wv;
    if (wid >= ntiles * n_kchunks) return;
    const int t = wid / n_kchunks;
    const int kc = wid - t * n_kchunks;
    const int k = kc * 64 + lane;
    const bool kvalid = k < K;
    const size_t kk = size_t(kvalid ? k : K - 1);
    const size_t SK = size_t(K);
    const int lo = int(kk) * 8, so = k * 8;   // byte offsets of this lane's cotangent
    const int64_t B64 = B;
    double(*C)[CH] = sc[wv];
    double(*D)[CH] = sd[wv];
    int *PC = si[wv][0];   // partner column, -1 on the diagonal
    int *PB = si[wv][1];   // bus of the entry's row
    int *OB = si[wv][2];   // carried branch or -1
    int *LF = si[wv][3];   // first load of the row's bus or -1 (row-start entries)
    int *LS = si[wv][4];   // position of that load in ldlist
    int *LN = si[wv][5];   // loads at the bus
    const int4 td = tiles[t];
    const int e0 = td.x, e1 = td.y, p0 = td.z;
    const GridDev gd = grids[td.w];
    const double *xt = x + gd.xoff;
    const double *xv = xt + gd.N;
    const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    int rows_seen = 0;
    // open row (phase 2 state, uniform except the per-lane accumulators)
    int row_bus = -1;
    double wPa = 0.0, wQa = 0.0, accT = 0.0, accV = 0.0;
    auto flush = [&](int b) {
        const int ia = b - gd.bus_off;
        const int2 b2 = bus2[b];
        double gt = accT, gv = accV;
        if (b2.y >= 0) {
            const int4 g4 = gen4[b2.y];
            const double wv = rld(W + size_t(g4.x) * SK, lo);
            const bool held = g4.z == kGenHeld;
            // control row: +1 at (V row, V_a) under voltage control, +1 at
            // (V row, Q_g) when the output is held; Q_g column: -1 in row Q_a
            if (!held) gv = gv + wv;
            if (kvalid) rst(gx + size_t(g4.x) * SK, so, held ? wv - wQa : -wQa);
            if (g4.z >= 0) {
                gt = gt + rld(W + size_t(g4.z) * SK, lo);   // angle row: +1 at (theta row, theta_a)
                if (kvalid) rst(gx + size_t(g4.z) * SK, so, -wPa);   // P_s column
            }
        }
        if (kvalid) {
            rst(gx + size_t(gd.xoff + ia) * SK, so, gt);
            rst(gx + size_t(gd.xoff + gd.N + ia) * SK, so, gv);
        }
    };
    for (int c0 = e0; c0 < e1; c0 += CH) {
        const int nvalid = min(CH, e1 - c0);
        // ---- phase 1: one entry per lane; the entry's coefficients go to
        // LDS before its branch's partials are formed, so the two sets are
        // never live together
        uint64_t smask;
        {
            const bool valid = lane < nvalid;
            const int e = valid ? src[c0 + lane] : 0;
            const int raw = valid ? ycol[e] : 0;
            const bool start = raw < 0;
            const int ic = raw & kColMask;
            smask = __ballot(start);
            const int r = rows_seen + __popcll(smask & le) - 1;
            const int b = valid ? order[p0 + r] : 0;   // bus of the entry's row
            const int ia = b - gd.bus_off;
            double cf[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            int partner = -1;
            double tha = 0.0, va = 0.0, thc = 0.0, vc = 0.0;
            if (valid) {
                tha = xt[ia];
                va = xv[ia];
                const double G = yG[e], Bc = yB[e];
                if (ic == ia) {
                    cf[2] = 2.0 * va * G;      // dP_a/dV_a (diagonal term)
                    cf[3] = -(2.0 * va * Bc);  // dQ_a/dV_a
                } else {
                    thc = xt[ic];
                    vc = xv[ic];
                    const int et = ytr[e];
                    const double Gp = yG[et], Bp = yB[et];
                    double s, co;
                    sincos(tha - thc, &s, &co);
                    const double t1 = fma(G, co, Bc * s);
                    const double t2 = fma(G, s, -(Bc * co));
                    const double t1p = fma(Gp, co, -(Bp * s));
                    const double t2p = -fma(Gp, s, Bp * co);
                    const double vv = va * vc;
                    cf[0] = -(vv * t2);   // dP_a/dth_a share   (x W[P_a])
                    cf[1] = vv * t1;      // dQ_a/dth_a share   (x W[Q_a])
                    cf[2] = vc * t1;      // dP_a/dV_a share
                    cf[3] = vc * t2;      // dQ_a/dV_a share
                    cf[4] = vv * t2p;     // dP_c/dth_a         (x W[P_c])
                    cf[5] = -(vv * t1p);  // dQ_c/dth_a         (x W[Q_c])
                    cf[6] = vc * t1p;     // dP_c/dV_a
                    cf[7] = vc * t2p;     // dQ_c/dV_a
                    partner = ic;
                }
            }
            if (lane < CH) {
#pragma unroll
                for (int q = 0; q < 8; ++q) C[q][lane] = cf[q];
                PC[lane] = partner;
                PB[lane] = b;
            }
            if constexpr (WGP) {
                double d[20];
#pragma unroll
                for (int q = 0; q < 20; ++q) d[q] = 0.0;
                int ob = -1, lf = -1, ls = 0, ln = 0;
                if (valid) {
                    if (partner >= 0) {
                        ob = own[c0 + lane];
                        if (ob >= 0)
                            branch_partials(P[ob], P[B64 + ob], P[2 * B64 + ob], P[3 * B64 + ob],
                                            P[4 * B64 + ob], tha, va, thc, vc, d);
                    }
                    if (start) {
                        ls = ldptr[b];
                        ln = ldptr[b + 1] - ls;
                        lf = ln > 0 ? ldlist[ls] : -1;
                    }
                }
                if (lane < CH) {
#pragma unroll
                    for (int q = 0; q < 20; ++q) D[q][lane] = d[q];
                    OB[lane] = ob;
                    LF[lane] = lf;
                    LS[lane] = ls;
                    LN[lane] = ln;
                }
            }
        }
        wave_sync();
        // ---- phase 2: one cotangent per lane, entries in order; the W rows
        // of a group's partners are gathered together before the group's
        // arithmetic
        for (int q0 = 0; q0 < nvalid; q0 += kVjpGroup) {
            double wPc[kVjpGroup], wQc[kVjpGroup];
#pragma unroll
            for (int u = 0; u < kVjpGroup; ++u) {
                const int q = q0 + u;
                wPc[u] = 0.0;
                wQc[u] = 0.0;
                if (q < nvalid) {
                    // every lane reads the same LDS word: the row is uniform
                    const int icp = __builtin_amdgcn_readfirstlane(PC[q]);
                    if (icp >= 0) {
                        wPc[u] = rld(W + size_t(gd.xoff + icp) * SK, lo);
                        wQc[u] = rld(W + size_t(gd.xoff + gd.N + icp) * SK, lo);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kVjpGroup; ++u) {
                const int q = q0 + u;
                if (q >= nvalid) break;
                if ((smask >> q) & 1ull) {   // a row starts here
                    if (WGX && row_bus >= 0) flush(row_bus);
                    row_bus = __builtin_amdgcn_readfirstlane(PB[q]);
                    ++rows_seen;
                    const int ia = row_bus - gd.bus_off;
                    wPa = rld(W + size_t(gd.xoff + ia) * SK, lo);
                    wQa = rld(W + size_t(gd.xoff + gd.N + ia) * SK, lo);
                    accT = 0.0;
                    accV = 0.0;
                    if (WGP && kvalid) {
                        const int lf = __builtin_amdgcn_readfirstlane(LF[q]);
                        if (lf >= 0) {
                            rst(gp + size_t(5 * B64 + lf) * SK, so, wPa);
                            rst(gp + size_t(5 * B64 + NL + lf) * SK, so, wQa);
                            const int ls = __builtin_amdgcn_readfirstlane(LS[q]);
                            const int ln = __builtin_amdgcn_readfirstlane(LN[q]);
                            for (int j = ls + 1; j < ls + ln; ++j) {
                                const int l = ldlist[j];
                                rst(gp + size_t(5 * B64 + l) * SK, so, wPa);
                                rst(gp + size_t(5 * B64 + NL + l) * SK, so, wQa);
                            }
                        }
                    }
                }
                if (WGX) {
                    accT = accT + C[0][q] * wPa + C[1][q] * wQa + C[4][q] * wPc[u] +
                           C[5][q] * wQc[u];
                    accV = accV + C[2][q] * wPa + C[3][q] * wQa + C[6][q] * wPc[u] +
                           C[7][q] * wQc[u];
                }
                if constexpr (WGP) {
                    const int ob = __builtin_amdgcn_readfirstlane(OB[q]);
                    if (ob >= 0 && kvalid) {
#pragma unroll
                        for (int pr = 0; pr < 5; ++pr) {
                            const double v = D[4 * pr][q] * wPa + D[4 * pr + 1][q] * wQa +
                                             D[4 * pr + 2][q] * wPc[u] + D[4 * pr + 3][q] * wQc[u];
                            rst(gp + size_t(pr * B64 + ob) * SK, so, v);
                        }
                    }
                }
            }
        }
        wave_sync();
    }
    if (WGX && row_bus >= 0) flush(row_bus);
}

// Parameter gradients of the branches no admittance entry carries: a second
// branch joining the same pair of buses in the same direction, and
// out-of-service branches (zero rows).  Phase 1 (lane = branch in `list`):
// the partials; phase 2 (lane = cotangent): each gradient row is the four
// partials dotted with the W rows of the branch's bus equations.
__global__ void __launch_bounds__(256)
k_vjp_branches(int B, int nlist, int n_tiles, int n_kchunks, const int32_t *__restrict__ list,
               const int32_t *__restrict__ br_f, const int32_t *__restrict__ br_t,
               const int32_t *__restrict__ br_on, const int2 *__restrict__ busx,
               const double *__restrict__ P, const double *__restrict__ x,
               const double *__restrict__ W, int K, double *__restrict__ gp) {
    __shared__ double sd[4][20][kVjpTile];
    __shared__ int4 sr[4][kVjpTile];
    __shared__ int se[4][kVjpTile];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wid = blockIdx.x * 4 + wv;
    if (wid >= n_tiles * n_kchunks) return;
    const int t = wid / n_kchunks;
    const int kc = wid - t * n_kchunks;
    const int k = kc * 64 + lane;
    const bool kvalid = k < K;
    const size_t kk = size_t(kvalid ? k : K - 1);
    const size_t SK = size_t(K);
    const int64_t B64 = B;
    double(*D)[kVjpTile] = sd[wv];
    int4 *R = sr[wv];
    int *RE = se[wv];
    const int e0 = t * kVjpTile;
    const int nb = min(kVjpTile, nlist - e0);
    {   // phase 1
        const int e = lane < nb ? list[e0 + lane] : 0;
        double d[20];
#pragma unroll
        for (int q = 0; q < 20; ++q) d[q] = 0.0;
        int4 rows = make_int4(0, 0, 0, 0);
        if (lane < nb && br_on[e]) {
            const int2 xf = busx[br_f[e]], xt = busx[br_t[e]];
            rows = make_int4(xf.x, xf.y, xt.x, xt.y);
            branch_partials(P[e], P[B64 + e], P[2 * B64 + e], P[3 * B64 + e], P[4 * B64 + e],
                            x[xf.x], x[xf.y], x[xt.x], x[xt.y], d);
        }
        if (lane < kVjpTile) {
#pragma unroll
            for (int q = 0; q < 20; ++q) D[q][lane] = d[q];
            R[lane] = rows;
            RE[lane] = e;
        }
    }
    wave_sync();
    for (int q0 = 0; q0 < nb; q0 += kVjpGroup) {   // phase 2
        double w[kVjpGroup][4];
#pragma unroll
        for (int u = 0; u < kVjpGroup; ++u) {
            if (q0 + u < nb) {
                const int4 rr = R[q0 + u];
                w[u][0] = W[size_t(rr.x) * SK + kk];
                w[u][1] = W[size_t(rr.y) * SK + kk];
                w[u][2] = W[size_t(rr.z) * SK + kk];
                w[u][3] = W[size_t(rr.w) * SK + kk];
            }
        }
#pragma unroll
        for (int u = 0; u < kVjpGroup; ++u) {
            const int q = q0 + u;
            if (q >= nb) break;
            const int e = RE[q];
#pragma unroll
            for (int pr = 0; pr < 5; ++pr) {
                const double v = D[4 * pr][q] * w[u][0] + D[4 * pr + 1][q] * w[u][1] +
                                 D[4 * pr + 2][q] * w[u][2] + D[4 * pr + 3][q] * w[u][3];
                if (kvalid) st(&gp[size_t(pr * B64 + e) * SK + k], v);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

void dev_destroy(DevPlan *dp) {
    if (!dp) return;
    int prev = 0;
    bool switched = hipGetDevice(&prev) == hipSuccess && prev != dp->device &&
                    hipSetDevice(dp->device) == hipSuccess;
    for (void *p : dp->allocs) (void)hipFree(p);
    if (switched) (void)hipSetDevice(prev);
    delete dp;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) {
            ok = false;
            return;
        }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

static int build_coeffs(HostPlan &hp, DevPlan *dp, hipStream_t st) {
    if (hp.Nt > 0) {
        hipLaunchKernelGGL(k_build_coeffs, dim3((hp.Nt + 255) / 256), dim3(256), 0, st, hp.Nt,
                           int64_t(hp.Bt), dp->yptr, dp->bus2, dp->cptr, dp->clist, dp->shptr,
                           dp->shlist, dp->shunt_g, dp->shunt_b, dp->ldptr, dp->ldlist,
                           dp->params, int64_t(hp.NLt), dp->genpv, dp->pv_p, dp->yG, dp->yB,
                           dp->spec);
        HIP_TRY(hipGetLastError());
    }
    if (dp->otab && hp.Bt > 0) {
        hipLaunchKernelGGL(k_outage_table, dim3((hp.Bt + 255) / 256), dim3(256), 0, st,
                           int64_t(hp.Bt), dp->params, dp->otab);
        HIP_TRY(hipGetLastError());
    }
    return PF_OK;
}

int dev_upload_tiles(HostPlan &hp, DevPlan *dp) {
    DeviceGuard g(dp->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", dp->device);
    const int32_t nt = hp.n_tiles();
    if (nt > dp->ntiles_alloc) {
        int4 *p = nullptr;
        int rc = dalloc(dp, &p, 2 * size_t(nt));
        if (rc) return rc;
        dp->tiles = p;
        dp->ntiles_alloc = nt;
    }
    if (nt) HIP_TRY(hipMemcpy(dp->tiles, hp.tiles.data(), 2 * size_t(nt) * sizeof(int4),
                              hipMemcpyHostToDevice));
    return PF_OK;
}

int dev_upload_gens(const HostPlan &hp, DevPlan *dp) {
    DeviceGuard g(dp->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", dp->device);
    if (hp.NGt == 0) return PF_OK;
    HIP_TRY(hipMemcpy(dp->gen4, hp.gen4.data(), hp.gen4.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dp->gen2, hp.gen2.data(), hp.gen2.size() * sizeof(double),
                      hipMemcpyHostToDevice));
    return PF_OK;
}

int dev_create(HostPlan &hp, DevPlan **out) {
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(PF_EDEVICE, "no HIP device available");
    if (hp.device < 0) HIP_TRY(hipGetDevice(&hp.device));
    if (hp.device >= ndev) return fail(PF_EINVAL, "device %d does not exist", hp.device);
    DeviceGuard guard(hp.device);
    if (!guard.ok) return fail(PF_EDEVICE, "cannot select device %d", hp.device);
    DevPlan *dp = new DevPlan();
    dp->device = hp.device;
    int rc = PF_OK;
#define UP(field, vec) \
    if (!rc) rc = dupload(dp, &dp->field, hp.vec)
    UP(yptr, yptr);
    UP(cptr, cptr);
    UP(clist, clist);
    UP(bus4, bus4);
    UP(bus2, bus2);
    UP(shptr, shptr);
    UP(shlist, shlist);
    UP(ldptr, ldptr);
    UP(ldlist, ldlist);
    UP(gen4, gen4);
    UP(gen2, gen2);
    UP(genpv, genpv);
    UP(br_f, br_f);
    UP(br_t, br_t);
    UP(br_on, br_on);
    UP(load_bus, load_bus);
    UP(busx, busx);
    UP(ytr, ytr);
    UP(params, params);
    UP(pv_p, pv_p);
    UP(shunt_g, shunt_g);
    UP(shunt_b, shunt_b);
#undef UP
    std::vector<GridDev> gd(hp.grids.size());
    for (size_t g = 0; g < hp.grids.size(); ++g)
        gd[g] = GridDev{hp.grids[g].N, hp.grids[g].bus_off, hp.grids[g].xoff};
    if (!rc) rc = dupload(dp, &dp->grids, gd);
    // admittance entries with kEntryPad zeroed trailing entries
    const size_t ny_pad = size_t(hp.n_y) + kEntryPad;
    if (!rc) rc = dalloc(dp, &dp->ycol, ny_pad);
    if (!rc) rc = dalloc(dp, &dp->yG, ny_pad);
    if (!rc) rc = dalloc(dp, &dp->yB, ny_pad);
    if (!rc) {
        hipError_t e = hipMemset(dp->ycol, 0, ny_pad * sizeof(int32_t));
        if (e == hipSuccess) e = hipMemset(dp->yG, 0, ny_pad * sizeof(double));
        if (e == hipSuccess) e = hipMemset(dp->yB, 0, ny_pad * sizeof(double));
        if (e == hipSuccess && hp.n_y)
            e = hipMemcpy(dp->ycol, hp.ycol.data(), size_t(hp.n_y) * sizeof(int32_t),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = fail(PF_EDEVICE, "entry upload: %s", hipGetErrorString(e));
    }
    if (!rc) rc = dalloc(dp, &dp->spec, size_t(hp.Nt));
    if (hp.kind == KIND_BATCH) {
        if (!rc) rc = dupload(dp, &dp->lscale, hp.load_scale_t);
        if (!rc) rc = dupload(dp, &dp->pscale, hp.pv_scale_t);
        if (!rc) rc = dupload(dp, &dp->outage, hp.outage);
        if (!rc && !hp.outage.empty()) {
            std::vector<int32_t> ft(2 * hp.outage.size(), -1);
            for (size_t k = 0; k < hp.outage.size(); ++k)
                if (hp.outage[k] >= 0) {
                    ft[2 * k] = hp.br_f[hp.outage[k]];
                    ft[2 * k + 1] = hp.br_t[hp.outage[k]];
                }
            rc = dupload(dp, &dp->out_ft, ft);
        }
        if (!rc && !hp.outage.empty()) rc = dalloc(dp, &dp->otab, size_t(hp.Bt) * 8);
        if (!rc) rc = dupload(dp, &dp->order_nat, hp.order_natural);
        if (!rc) rc = dupload(dp, &dp->order_bfs, hp.order_bfs);
    } else {
        if (!rc) rc = dupload(dp, &dp->order_bfs, hp.order_bfs);
        if (!rc) rc = dupload(dp, &dp->adj_tiles, hp.adj_tiles);
        if (!rc) rc = dupload(dp, &dp->adj_src, hp.adj_src);
        if (!rc) rc = dupload(dp, &dp->adj_own, hp.adj_own);
        if (!rc) rc = dupload(dp, &dp->adj_left, hp.adj_left);
        if (!rc) rc = dalloc(dp, &dp->nw_F, size_t(hp.n));
        if (!rc) rc = dalloc(dp, &dp->nw_J, size_t(hp.nnz));
        if (!rc) rc = dalloc(dp, &dp->nw_dx, size_t(hp.n));
    }
    if (!rc) rc = dev_upload_tiles(hp, dp);
    if (!rc) rc = build_coeffs(hp, dp, nullptr);
    if (!rc) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = fail(PF_EDEVICE, "setup kernels: %s", hipGetErrorString(e));
    }
    if (rc) {
        dev_destroy(dp);
        return rc;
    }
    *out = dp;
    return PF_OK;
}

int dev_set_params(HostPlan &hp, DevPlan *dp, const double *params_dev, void *stream) {
    DeviceGuard g(dp->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", dp->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t np = size_t(hp.n_params());
    if (np) HIP_TRY(hipMemcpyAsync(dp->params, params_dev, np * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
    return build_coeffs(hp, dp, st);
}

// Host copy of the parameters after pf_set_params (read by the host-side
// builders of the fast decoupled matrices): waits for the device, then copies.
int dev_fetch_params(HostPlan &hp, DevPlan *dp) {
    DeviceGuard g(dp->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", dp->device);
    const size_t np = size_t(hp.n_params());
    HIP_TRY(hipDeviceSynchronize());
    if (np) HIP_TRY(hipMemcpy(hp.params.data(), dp->params, np * sizeof(double),
                              hipMemcpyDeviceToHost));
    hp.params_stale = false;
    return PF_OK;
}

static void wave_grid(int64_t units, const pf_schedule &s, int &blocks, int &units_per_wave) {
    const int wpb = s.waves_per_block;
    if (units <= 0) {
        blocks = 0;
        units_per_wave = 0;
        return;
    }
    if (s.grid_blocks > 0) {
        const int64_t waves = int64_t(s.grid_blocks) * wpb;
        units_per_wave = int((units + waves - 1) / waves);
    } else {
        units_per_wave = 1;
    }
    const int64_t waves_needed = (units + units_per_wave - 1) / units_per_wave;
    blocks = int((waves_needed + wpb - 1) / wpb);
}

int dev_eval_single(HostPlan &hp, DevPlan *dp, const double *x, double *F, double *J,
                    void *stream) {
    DeviceGuard g(dp->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", dp->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const pf_schedule &s = hp.sched;
    int blocks, tpw;
    wave_grid(hp.n_tiles(), s, blocks, tpw);
    if (blocks == 0) return PF_OK;
    const int threads = 64 * s.waves_per_block;
    // staging area per wave: a tile's P and Q row ranges hold at most
    // 3 x tile_entries values each; larger tile sizes write directly
    int stage_cap = (J && s.tile_entries <= kStageMaxTile) ? 6 * s.tile_entries : 0;
    if (size_t(s.waves_per_block) * (6 * 64 + stage_cap) * sizeof(double) > kMaxBlockLds)
        stage_cap = 0;
    const size_t shm = size_t(s.waves_per_block) * (6 * 64 + stage_cap) * sizeof(double);
    const int remap = s.xcd_remap == 1 ? 1 : 0;
#define LAUNCH(WF, WJ)                                                                       \
    hipLaunchKernelGGL((k_eval_single<WF, WJ>), dim3(blocks), dim3(threads), shm, st,       \
                       dp->tiles, hp.n_tiles(), tpw, remap, stage_cap, dp->grids, dp->bus4, \
                       dp->bus2, dp->spec, dp->ycol, dp->yG, dp->yB, dp->gen4, dp->gen2, x, \
                       F, J)
    if (F && J)
        LAUNCH(true, true);
    else if (F)
        LAUNCH(true, false);
    else
        LAUNCH(false, true);
#undef LAUNCH
    HIP_TRY(hipGetLastError());
    return PF_OK;
}

int dev_eval_batch(HostPlan &hp, DevPlan *dp, const double *X, double *F, double *J,
                   void *stream) {
    DeviceGuard g(dp->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", dp->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const pf_schedule &s = hp.sched;
    const int N = hp.Nt;
    const int I = hp.n_inst;
    const int TB = s.batch_buses;
    const int n_btiles = (N + TB - 1) / TB;
    // overlay-free row layouts with an even instance count and pitch take two
    // instances per lane (chunks of 128)
    const bool pairs = !dp->lscale && !dp->pscale && !dp->outage && !hp.panels && I % 2 == 0 &&
                       hp.ld % 2 == 0;
    const int n_chunks = pairs ? (I + 127) / 128 : (I + 63) / 64;
    const int group = std::min(s.batch_group, n_chunks);
    const int64_t n_items = int64_t(n_btiles) * group * ((n_chunks + group - 1) / group);
    if (n_items > (int64_t(1) << 31) - 1) return fail(PF_EINVAL, "batch work list too long");
    int blocks, ipw;
    wave_grid(n_items, s, blocks, ipw);
    if (blocks == 0) return PF_OK;
    const int threads = 64 * s.waves_per_block;
    const int remap = s.xcd_remap == 1 ? 1 : 0;
    const int32_t *order = s.batch_order == 2 ? dp->order_bfs : dp->order_nat;
    const bool scen = dp->lscale || dp->pscale;
    const bool outg = dp->outage != nullptr;
    const double *lp = dp->params + 5LL * hp.Bt;
    const double *lq = lp + hp.NLt;
#define LAUNCH(WF, WJ, SC, OG)                                                                 \
    hipLaunchKernelGGL((k_eval_batch<WF, WJ, SC, OG>), dim3(blocks), dim3(threads), 0, st, N, \
                       I, hp.ld, hp.panels, hp.n, hp.nnz, n_btiles, n_chunks, TB, int(n_items), ipw, remap, group, order,     \
                       dp->bus4, dp->bus2,                                                    \
                       dp->spec, dp->ycol, dp->yG, dp->yB, dp->gen4, dp->gen2, dp->genpv,     \
                       dp->ldptr, dp->ldlist, lp, lq, dp->pv_p, dp->lscale, dp->pscale,       \
                       dp->outage, dp->out_ft, dp->otab, X, F, J)
#define LAUNCH_OV(WF, WJ)              \
    if (scen && outg)                  \
        LAUNCH(WF, WJ, true, true);    \
    else if (scen)                     \
        LAUNCH(WF, WJ, true, false);   \
    else if (outg)                     \
        LAUNCH(WF, WJ, false, true);   \
    else                               \
        LAUNCH(WF, WJ, false, false)
    if (pairs) {
#define LAUNCH2(WF, WJ)                                                                           \
    hipLaunchKernelGGL((k_eval_batch2<WF, WJ>), dim3(blocks), dim3(threads), 0, st, N, I, hp.ld,   \
                       n_btiles, n_chunks, TB, int(n_items), ipw, remap, group, order, dp->bus4, \
                       dp->bus2, dp->spec, dp->ycol, dp->yG, dp->yB, dp->gen4, dp->gen2, X, F, J)
        if (F && J)
            LAUNCH2(true, true);
        else if (F)
            LAUNCH2(true, false);
        else
            LAUNCH2(false, true);
#undef LAUNCH2
    } else if (F && J) {
        LAUNCH_OV(true, true);
    } else if (F) {
        LAUNCH_OV(true, false);
    } else {
        LAUNCH_OV(false, true);
    }
#undef LAUNCH_OV
#undef LAUNCH
    HIP_TRY(hipGetLastError());
    return PF_OK;
}

int dev_vjp(HostPlan &hp, DevPlan *dp, const double *x, const double *W, int32_t K, double *gx,
            double *gp, void *stream) {
    DeviceGuard g(dp->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", dp->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n_kchunks = (K + 63) / 64;
    if (hp.n_adj_tiles() > 0) {
        const int64_t waves = int64_t(hp.n_adj_tiles()) * n_kchunks;
#define LAUNCH(WGX, WGP)                                                                        \
    hipLaunchKernelGGL((k_vjp<WGX, WGP>), dim3(unsigned((waves + 3) / 4)), dim3(256), 0, st,     \
                       dp->adj_tiles, hp.n_adj_tiles(), n_kchunks, dp->order_bfs, dp->adj_src,   \
                       dp->adj_own, dp->grids, dp->bus2, dp->ycol, dp->ytr, dp->yG, dp->yB,      \
                       dp->gen4, dp->ldptr, dp->ldlist, dp->params, hp.Bt, hp.NLt, x, W, int(K), \
                       gx, gp)
        if (gx && gp)
            LAUNCH(true, true);
        else if (gx)
            LAUNCH(true, false);
        else
            LAUNCH(false, true);
#undef LAUNCH
        HIP_TRY(hipGetLastError());
    }
    const int nleft = int(hp.adj_left.size());
    if (gp && nleft > 0) {
        const int nt = (nleft + kVjpTile - 1) / kVjpTile;
        const int64_t waves = int64_t(nt) * n_kchunks;
        hipLaunchKernelGGL(k_vjp_branches, dim3(unsigned((waves + 3) / 4)), dim3(256), 0, st,
                           hp.Bt, nleft, nt, n_kchunks, dp->adj_left, dp->br_f, dp->br_t,
                           dp->br_on, dp->busx, dp->params, x, W, int(K), gp);
        HIP_TRY(hipGetLastError());
    }
    return PF_OK;
}

// ---------------------------------------------------------------------------
// Host-side drivers: the Newton loop with a host solve, and the schedule
// search with its cache.  They launch the kernels above and change none of
// them; the kernel source identity carried in tune-cache keys and counter
// summaries covers the code above this line only.
// ---------------------------------------------------------------------------

int dev_newton(HostPlan &hp, DevPlan *dp, double *x, const pf_newton_opts *opts,
               pf_linsolve_fn solve, void *user, pf_newton_report *rep) {
    DeviceGuard g(dp->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", dp->device);
    const double tol = (opts && opts->tol > 0) ? opts->tol : 1e-10;
    const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 10;
    const bool limits = opts && (opts->q_min || opts->q_max);
    const double check_below = (limits && opts->q_check_below > 0) ? opts->q_check_below : 1e-3;
    const double switch_tol = (limits && opts->q_switch_tol >= 0) ? opts->q_switch_tol : 1e-9;
    const int64_t n = hp.n, nnz = hp.nnz;
    std::vector<double> Fh(static_cast<size_t>(n)), Jh(static_cast<size_t>(nnz)),
        dxh(static_cast<size_t>(n)), xh(limits ? static_cast<size_t>(n) : 0);
    pf_newton_report r{};
    hipEvent_t ev0, ev1;
    HIP_TRY(hipEventCreate(&ev0));
    HIP_TRY(hipEventCreate(&ev1));
    // F and J at x under the current modes; F to the host and its max norm
    auto evaluate = [&](double &nf) -> int {
        HIP_TRY(hipEventRecord(ev0, nullptr));
        const int e = dev_eval_single(hp, dp, x, dp->nw_F, dp->nw_J, nullptr);
        if (e) return e;
        HIP_TRY(hipEventRecord(ev1, nullptr));
        HIP_TRY(hipMemcpy(Fh.data(), dp->nw_F, size_t(n) * sizeof(double), hipMemcpyDeviceToHost));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
        r.t_eval_s += ms * 1e-3;
        nf = 0.0;
        for (int64_t q = 0; q < n; ++q) {
            const double v = std::fabs(Fh[q]);
            if (v != v) {  // a NaN anywhere makes the norm NaN
                nf = v;
                break;
            }
            if (v > nf) nf = v;
        }
        return PF_OK;
    };
    auto t_start = std::chrono::steady_clock::now();
    // the iterations; the events are released on every path below
    auto iterate = [&]() -> int {
        int rc = PF_ENOCONV;
        for (int it = 0;; ++it) {
            double nf = 0.0;
            int e = evaluate(nf);
            if (e) {
                rc = e;
                break;
            }
            int32_t ns = 0;
            if (limits && nf < check_below) {
                HIP_TRY(hipMemcpy(xh.data(), x, size_t(n) * sizeof(double),
                                  hipMemcpyDeviceToHost));
                e = q_switch(hp, dp, xh.data(), opts->q_min, opts->q_max, switch_tol, &ns);
                if (!e && ns) e = evaluate(nf);
                if (e) {
                    rc = e;
                    break;
                }
            }
            if (it < 65) {
                r.norm[it] = nf;
                r.switched[it] = ns;
            }
            r.n_switches += ns;
            if (nf < tol && ns == 0) {
                r.converged = 1;
                rc = PF_OK;
                break;
            }
            if (it >= max_iter) {
                rc = fail(PF_ENOCONV, "Newton did not converge in %d iterations (|F| = %g)",
                          max_iter, nf);
                break;
            }
            HIP_TRY(hipMemcpy(Jh.data(), dp->nw_J, size_t(nnz) * sizeof(double),
                              hipMemcpyDeviceToHost));
            auto ts = std::chrono::steady_clock::now();
            const int sr = solve(user, n, hp.rowptr.data(), hp.colidx.data(), Jh.data(), Fh.data(),
                                 dxh.data());
            r.t_solve_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count();
            if (sr != 0) {
                rc = fail(PF_ESOLVE, "linear solve callback returned %d at iteration %d", sr, it);
                break;
            }
            HIP_TRY(hipMemcpy(dp->nw_dx, dxh.data(), size_t(n) * sizeof(double),
                              hipMemcpyHostToDevice));
            hipLaunchKernelGGL(k_newton_update, dim3(unsigned((n + 255) / 256)), dim3(256), 0, nullptr,
                               n, x, dp->nw_dx);
            HIP_TRY(hipGetLastError());
            r.iterations = it + 1;
        }
        HIP_TRY(hipDeviceSynchronize());
        return rc;
    };
    const int rc = iterate();
    r.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (rep) *rep = r;
    return rc;
}


// Median time (ms) of `reps` launches of the plan's kernel under its
// current schedule, each bracketed by its own pair of events (released on
// every path).
static int time_schedule(HostPlan &hp, DevPlan *dp, const double *x, double *F, double *J,
                         int reps, hipStream_t st, float &ms_out) {
    std::vector<hipEvent_t> ev(2 * size_t(reps), nullptr);
    auto launch = [&]() {
        return hp.kind == KIND_BATCH ? dev_eval_batch(hp, dp, x, F, J, st)
                                     : dev_eval_single(hp, dp, x, F, J, st);
    };
    auto run = [&]() -> int {
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
        int rc = launch();  // warm-up
        for (int r = 0; r < reps && !rc; ++r) {
            HIP_TRY(hipEventRecord(ev[2 * r], st));
            rc = launch();
            if (!rc) HIP_TRY(hipEventRecord(ev[2 * r + 1], st));
        }
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(st));
        std::vector<float> t(size_t(reps), 0.f);
        for (int r = 0; r < reps; ++r) HIP_TRY(hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]));
        std::sort(t.begin(), t.end());
        ms_out = t[size_t(reps) / 2];
        return PF_OK;
    };
    const int rc = run();
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

// Coordinate descent over the schedule space: starting from the current
// schedule, each parameter in turn is set to the fastest of its candidate
// values while the others stay fixed; two sweeps, then a joint pass over the
// axes that interact most (below).  A candidate replaces the
// best so far only when it is faster by more than kTuneMargin, so that
// timing noise between near-equal schedules does not decide.  Every candidate gives
// bit-identical results, so only time decides.
static int autotune_search(HostPlan &hp, DevPlan *dp, const double *x, double *F, double *J,
                           int32_t reps, void *stream, pf_schedule *best_out, float *best_ms_out) {
    DeviceGuard g(dp->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", dp->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool batch = hp.kind == KIND_BATCH;
    struct Axis {
        int32_t pf_schedule::*field;
        std::vector<int32_t> values;
    };
    std::vector<Axis> axes;
    if (batch) {
        axes.push_back({&pf_schedule::batch_buses, {1, 2, 4, 8, 16, 32, 64}});
        axes.push_back({&pf_schedule::batch_order, {1, 2}});
        axes.push_back({&pf_schedule::batch_group, {1, 2, 4, 8, 64}});
    } else {
        axes.push_back({&pf_schedule::tile_entries, {64, 128, 256, 512, 1024, 2048}});
    }
    axes.push_back({&pf_schedule::waves_per_block, {1, 2, 4, 8}});
    axes.push_back({&pf_schedule::grid_blocks, {-1, 256, 512, 1024, 2048, 4096}});
    axes.push_back({&pf_schedule::xcd_remap, {1, 2}});

    pf_schedule best = hp.sched;
    auto apply = [&](const pf_schedule &s) -> int {
        const bool retile = s.tile_entries != hp.sched.tile_entries;
        hp.sched = s;
        if (retile) {
            build_tiles(hp);
            return dev_upload_tiles(hp, dp);
        }
        return PF_OK;
    };
    float best_ms = 0.f;
    int rc = apply(best);
    if (!rc) rc = time_schedule(hp, dp, x, F, J, reps, st, best_ms);
    auto consider = [&](const pf_schedule &cand) -> int {
        float ms = 0.f;
        int r = apply(cand);
        if (!r) r = time_schedule(hp, dp, x, F, J, reps, st, ms);
        if (!r && ms < best_ms * (1.0f - kTuneMargin)) {
            best_ms = ms;
            best = cand;
        }
        return r;
    };
    for (int sweep = 0; sweep < 2 && !rc; ++sweep) {
        for (const Axis &ax : axes) {
            for (int32_t v : ax.values) {
                if (best.*(ax.field) == v) continue;
                pf_schedule cand = best;
                cand.*(ax.field) = v;
                rc = consider(cand);
                if (rc) break;
            }
            if (rc) break;
        }
    }
    // Work-item size, waves per block and chunk grouping interact (tile
    // size and waves per block for single-instance plans), so single-axis
    // moves can stall short of a better corner: try every combination of
    // them around the best of the other axes.
    if (!rc) {
        const size_t a0 = 0, a1 = batch ? 3 : 1, a2 = 2;
        const std::vector<int32_t> v2s =
            batch ? axes[a2].values : std::vector<int32_t>{best.*(axes[a2].field)};
        for (int32_t v0 : axes[a0].values) {
            for (int32_t v1 : axes[a1].values) {
                for (int32_t v2 : v2s) {
                    pf_schedule cand = best;
                    cand.*(axes[a0].field) = v0;
                    cand.*(axes[a1].field) = v1;
                    cand.*(axes[a2].field) = v2;
                    if (cand.*(axes[a0].field) == best.*(axes[a0].field) &&
                        cand.*(axes[a1].field) == best.*(axes[a1].field) &&
                        cand.*(axes[a2].field) == best.*(axes[a2].field))
                        continue;
                    rc = consider(cand);
                    if (rc) break;
                }
                if (rc) break;
            }
            if (rc) break;
        }
    }
    const int rc2 = apply(best);
    if (!rc) rc = rc2;
    if (!rc && best_out) *best_out = best;
    if (!rc && best_ms_out) *best_ms_out = best_ms;
    return rc;
}

// ---------------------------------------------------------------------------
// tune cache: one text line per tuned plan shape,
//   <key> tile_entries waves_per_block grid_blocks batch_buses batch_order
//         xcd_remap batch_group <ms>
// The key names the GPU (architecture, compute units), the kernel source the
// library was built from, and everything about the plan that the kernel's
// work depends on; the last line with a matching key wins.
// ---------------------------------------------------------------------------

#ifndef PF_KERNEL_SHA
#define PF_KERNEL_SHA "unversioned"
#endif

static int tune_key(const HostPlan &hp, const DevPlan *dp, bool wf, bool wj, std::string &key) {
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dp->device));
    // FNV-1a over the grids' bus and entry counts (multi-grid plans)
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= uint64_t((v >> (8 * b)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (const GridInfo &g : hp.grids) {
        mix(g.N);
        mix(g.n_y);
        mix(g.NG);
    }
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "arch=%s;cus=%d;src=%s;kind=%d;order=%d;grids=%zu;gh=%016llx;n=%lld;nnz=%lld;"
                  "inst=%d;ld=%d;panels=%d;scen=%d;outg=%d;out=%d%d",
                  prop.gcnArchName, prop.multiProcessorCount, PF_KERNEL_SHA, hp.kind,
                  hp.bus_order_kind,
                  hp.grids.size(), (unsigned long long)h, (long long)hp.n, (long long)hp.nnz,
                  hp.n_inst, hp.ld, hp.panels,
                  int(!hp.load_scale_t.empty() || !hp.pv_scale_t.empty()),
                  int(!hp.outage.empty()), int(wf), int(wj));
    key = buf;
    return PF_OK;
}

static bool cache_lookup(const char *path, const std::string &key, pf_schedule &out) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    std::vector<char> line(4096);
    while (std::fgets(line.data(), int(line.size()), f)) {
        const size_t len = std::strlen(line.data());
        if (len <= key.size() || std::strncmp(line.data(), key.c_str(), key.size()) != 0 ||
            line[key.size()] != ' ')
            continue;
        pf_schedule s{};
        if (std::sscanf(line.data() + key.size(), "%d %d %d %d %d %d %d", &s.tile_entries,
                        &s.waves_per_block, &s.grid_blocks, &s.batch_buses, &s.batch_order,
                        &s.xcd_remap, &s.batch_group) == 7) {
            out = s;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static int cache_append(const char *path, const std::string &key, const pf_schedule &s,
                        float ms) {
    FILE *f = std::fopen(path, "a");
    if (!f) return fail(PF_EINVAL, "cannot open tune cache %s for appending", path);
    std::fprintf(f, "%s %d %d %d %d %d %d %d %.6f\n", key.c_str(), s.tile_entries,
                 s.waves_per_block, s.grid_blocks, s.batch_buses, s.batch_order, s.xcd_remap,
                 s.batch_group, double(ms));
    const bool bad = std::fclose(f) != 0;
    return bad ? fail(PF_EINVAL, "cannot write tune cache %s", path) : PF_OK;
}

int dev_autotune(HostPlan &hp, DevPlan *dp, const double *x, double *F, double *J, int32_t reps,
                 void *stream, const char *cache, pf_schedule *best_out, int32_t *hit) {
    DeviceGuard g(dp->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", dp->device);
    if (hit) *hit = 0;
    std::string key;
    if (cache && cache[0]) {
        int rc = tune_key(hp, dp, F != nullptr, J != nullptr, key);
        if (rc) return rc;
        pf_schedule s{};
        if (cache_lookup(cache, key, s)) {
            pf_schedule n{};
            rc = normalise_schedule(hp, &s, n);
            if (rc) return rc;
            const bool retile = n.tile_entries != hp.sched.tile_entries;
            hp.sched = n;
            if (retile) {
                build_tiles(hp);
                rc = dev_upload_tiles(hp, dp);
                if (rc) return rc;
            }
            if (best_out) *best_out = n;
            if (hit) *hit = 1;
            return PF_OK;
        }
    }
    pf_schedule best{};
    float ms = 0.f;
    int rc = autotune_search(hp, dp, x, F, J, reps, stream, &best, &ms);
    if (rc) return rc;
    if (best_out) *best_out = best;
    if (!key.empty()) rc = cache_append(cache, key, best, ms);
    return rc;
}

}  // namespace pf
