// Batched Newton power flow: thousands of instances of one grid (N-1
// contingencies, scenarios) solved together, every step on the device.  The
// Jacobians of a batched plan share one pattern, so one host LU with pivoting
// of one of them (P M Q = L U) fixes the pattern of T = (L - I) + U and both
// orders for all instances; every instance is then factorised along that
// pattern without pivoting again, in the same instance-fastest layout as the
// evaluation (a wavefront's lanes are instances, so every access to a T entry
// is one contiguous segment and the row structure is wave-uniform).
//
// Factorisation, row by row (row r of T in the permuted order):
//   t_r. <- the permuted Jacobian row (0 on fill entries);
//   for each k < r with t_rk in the pattern, in increasing k:
//       t_rk <- t_rk / t_kk;   t_rj <- t_rj - t_rk t_kj  for every j > k of row k;
// rows are grouped into levels (a row only needs rows of earlier levels) and
// each level is one launch; a wave keeps its row in LDS for all instances of
// its chunk.  A row's work is one stream of items, each reading one value of
// T: a step's divide (by t_kk) followed by its updates (by t_kj).  The
// values of a group of items are loaded together across step boundaries,
// so a row waits on memory once per group rather than once per step.
// Solves: forward over the same levels, backward over levels of U, then the
// update x[pivQ[k]] -= z[k].
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include <hip/hip_runtime.h>

#include "pf_internal.hpp"
#include "pf_trisolve.hpp"

#define BL_HIP(expr)                                                               \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return fail(PF_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

using namespace pf;

struct pf_batch_lu {
    pf_plan *plan = nullptr;
    int device = 0;
    int n = 0, nnzT = 0, n_inst = 0, ld = 0;
    // host copies of the level structure
    std::vector<int32_t> flev_ptr, blev_ptr;  // levels -> rows (offsets into the row lists)
    std::vector<int32_t> flev_w, blev_w;      // lanes used per wave (64, 32 or 16) per level
    std::vector<int32_t> flev_maxr;           // longest row per factor level
    std::vector<int32_t> flev_maxi;           // most items of a row per factor level
    // one instance: runs of consecutive small levels done by one block, as
    // {first level, end level, waves, LDS bytes per wave} (factorisation) and
    // {first level, end level, waves} (forward, backward solves)
    std::vector<int32_t> fchain_factor;
    TriLevels tri;   // the solves: row records (host copies); one instance: levels and runs
    int32_t *flev_ptr_d = nullptr, *blev_ptr_d = nullptr;
    int4 *frec = nullptr, *brec = nullptr;   // the solves' row records in level order
    int4 *frec_factor = nullptr;  // factorisation rows in level order: {T start, T end,
                                  // first item, items end}
    // device structure
    int32_t *trp = nullptr;   // n + 1
    int32_t *tci = nullptr;   // nnzT
    int32_t *tsrc = nullptr;  // nnzT: Jacobian slot of each T entry, -1 for fill
    int32_t *item_ptr = nullptr;  // n + 1: items of each row
    int2 *item = nullptr;     // {-(local index of t_rk) - 1, T position of t_kk} opens a step;
                              // {local index of t_rj, T position of t_kj} is an update
    int32_t *frows = nullptr;  // factorisation rows in level order
    int32_t *pivQ = nullptr;
    // device work arrays, instance-fastest with row pitch ld
    double *T = nullptr, *F = nullptr, *J = nullptr, *Y = nullptr;
    double *part = nullptr, *norm = nullptr;  // per-instance norms
    int32_t *active = nullptr;
    double *norm_host = nullptr;              // pinned [ld]
    int part_rows = 0;
    size_t lds_limit = 0;     // dynamic LDS a block may use
    // every PV unit's Q row pivots on its Q_g column and its control row on
    // the bus voltage column, Q_g eliminated first: the pivots survive a
    // switch of any unit's mode (pf_jacobian_switch_order)
    bool switch_safe = false;
};

namespace {

constexpr int kNormRowBlocks = 512;  // row blocks of the per-instance norm
constexpr int kG = 8;               // loads issued together in the solves and row loads
constexpr int kItems = 32;          // factorisation items whose loads are issued together
// The index arrays (tci, tsrc, item) and T carry padding past their ends so
// that a group's reads need no bounds test: the loads of a group are then
// issued back to back, and only the use of an entry is guarded.  Padding
// entries point at T row 0, Jacobian slot -1 (none) and column 0.
constexpr int kPad = kItems;
// Levels whose rows times instances are at most this many run a wavefront
// per (row, instance) rather than a lane per instance (at 1024 instances:
// levels of up to 16 rows; 2048 to 16384 measured alike, 65536 slower).
constexpr int64_t kInstWaves = 16384;

struct BGuard {
    int prev = -1;
    bool ok = true;
    explicit BGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) {
            ok = false;
            return;
        }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~BGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <class T>
int balloc(T **dst, const T *src, size_t count) {
    BL_HIP(hipMalloc(dst, (count ? count : 1) * sizeof(T)));
    if (src && count) BL_HIP(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return PF_OK;
}

void release(pf_batch_lu *b) {
    if (!b) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    for (void *p : {(void *)b->trp, (void *)b->tci, (void *)b->tsrc,
                    (void *)b->item_ptr, (void *)b->item, (void *)b->frows,
                    (void *)b->pivQ, (void *)b->T,
                    (void *)b->F, (void *)b->J, (void *)b->Y, (void *)b->part, (void *)b->norm,
                    (void *)b->active, (void *)b->flev_ptr_d, (void *)b->blev_ptr_d,
                    (void *)b->frec, (void *)b->brec, (void *)b->frec_factor})
        if (p) (void)hipFree(p);
    if (b->norm_host) (void)hipHostFree(b->norm_host);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete b;
}

bool is_perm(const int32_t *p, int n) {
    std::vector<char> seen(size_t(n), 0);
    for (int i = 0; i < n; ++i) {
        if (p[i] < 0 || p[i] >= n || seen[size_t(p[i])]) return false;
        seen[size_t(p[i])] = 1;
    }
    return true;
}

// lanes per wave for rows of length maxr so that a block's LDS row fits
int lanes_for(int maxr, size_t lds_limit) {
    for (int w = 64; w >= 16; w >>= 1)
        if (size_t(maxr) * size_t(w) * sizeof(double) <= lds_limit) return w;
    return 0;
}

// ---------------------------------------------------------------------------
// kernels (one wavefront per block; lane < W handles instance chunk*W + lane)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(64) k_blu_factor(
    const int32_t *__restrict__ rows, int n_chunks, int W, int n_inst, int SI,
    const int32_t *__restrict__ trp, const int32_t *__restrict__ tsrc,
    const int32_t *__restrict__ item_ptr, const int2 *__restrict__ item,
    const double *__restrict__ J, double *__restrict__ T) {
    extern __shared__ double Lrow[];
    const int lane = threadIdx.x;
    const int r = rows[blockIdx.x / n_chunks];
    const int inst = (blockIdx.x % n_chunks) * W + lane;
    const bool live = lane < W && inst < n_inst;
    const int r0 = trp[r], R = trp[r + 1] - r0;
    if (live) {
        // the row's Jacobian values, kG loads in flight at a time
        for (int q0 = 0; q0 < R; q0 += kG) {
            int sl[kG];
            double v[kG];
#pragma unroll
            for (int q = 0; q < kG; ++q) sl[q] = tsrc[r0 + q0 + q];
#pragma unroll
            for (int q = 0; q < kG; ++q) v[q] = J[size_t(max(sl[q], 0)) * SI + inst];
#pragma unroll
            for (int q = 0; q < kG; ++q)
                if (q0 + q < R) Lrow[(q0 + q) * W + lane] = sl[q] >= 0 ? v[q] : 0.0;
        }
        // the row's items in groups: a group's loads are issued before its
        // divides and read-modify-writes of the LDS row, which follow the
        // stream's order, so every result is that of the plain loop
        const int i0 = item_ptr[r], i1 = item_ptr[r + 1];
        double lik = 0.0;
        for (int g0 = i0; g0 < i1; g0 += kItems) {
            double t[kItems];
            int2 it[kItems];
#pragma unroll
            for (int q = 0; q < kItems; ++q) it[q] = item[g0 + q];
#pragma unroll
            for (int q = 0; q < kItems; ++q) t[q] = T[size_t(it[q].y) * SI + inst];
#pragma unroll
            for (int q = 0; q < kItems; ++q) {
                if (g0 + q < i1) {
                    if (it[q].x < 0) {   // a step opens: t_rk <- t_rk / t_kk
                        const int xk = -it[q].x - 1;
                        lik = Lrow[xk * W + lane] / t[q];
                        Lrow[xk * W + lane] = lik;
                    } else {
                        Lrow[it[q].x * W + lane] = fma(-lik, t[q], Lrow[it[q].x * W + lane]);
                    }
                }
            }
        }
        for (int q = 0; q < R; ++q) T[size_t(r0 + q) * SI + inst] = Lrow[q * W + lane];
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One row of one instance (instance inst of rows of pitch SI): a wavefront
// per row, its lanes spread over the row.  The row and the values its items
// read (final entries of rows of earlier levels) are loaded into LDS by all
// lanes at once; the steps then run in order, each step's divide on the
// wave-uniform value and its updates over the lanes.  A step's updates change
// distinct entries of the row, so every result equals that of the one-lane
// loop of k_blu_factor.
__device__ __forceinline__ void factor_row1(int4 m, int lane, const int32_t *__restrict__ tsrc,
                                            const int2 *__restrict__ item,
                                            const double *__restrict__ J, double *__restrict__ T,
                                            double *sm, size_t SI = 1, int inst = 0) {
    // the row's record: {first entry, end, first item, end of its items}
    const int r0 = m.x, R = m.y - r0;
    const int i0 = m.z, NI = m.w - i0;
    double *Lrow = sm;
    double *tv = sm + R;
    int *ix = reinterpret_cast<int *>(tv + NI);
    for (int q = lane; q < R; q += 64) {
        const int s = tsrc[r0 + q];
        Lrow[q] = s >= 0 ? J[size_t(s) * SI + inst] : 0.0;
    }
    for (int q = lane; q < NI; q += 64) {
        const int2 it = item[i0 + q];
        ix[q] = it.x;
        tv[q] = T[size_t(it.y) * SI + inst];
    }
    wave_sync();
    int q = 0;
    while (q < NI) {
        // item q opens a step: t_rk <- t_rk / t_kk
        const int xk = -ix[q] - 1;
        const double lik = Lrow[xk] / tv[q];
        wave_sync();
        if (lane == 0) Lrow[xk] = lik;
        // its updates run up to the next opening item
        int next = NI;
        for (int u0 = q + 1; u0 < NI; u0 += 64) {
            const int uq = u0 + lane;
            const bool stop = uq >= NI || ix[uq] < 0;
            const uint64_t m = __ballot(stop);
            const int lim = m ? __ffsll((unsigned long long)m) - 1 : 64;
            if (lane < lim) Lrow[ix[uq]] = fma(-lik, tv[uq], Lrow[ix[uq]]);
            if (m) {
                next = u0 + lim;
                break;
            }
        }
        wave_sync();
        q = next;
    }
    for (int q2 = lane; q2 < R; q2 += 64) T[size_t(r0 + q2) * SI + inst] = Lrow[q2];
}

// Several instances, levels of few rows: a wavefront per (row, instance) as
// for one instance, instead of one lane per instance walking the row's long
// chain of items alone.
__global__ void __launch_bounds__(64) k_blu_factor_inst(
    const int4 *__restrict__ rec, int n_inst, int SI, const int32_t *__restrict__ tsrc,
    const int2 *__restrict__ item, const double *__restrict__ J, double *__restrict__ T) {
    extern __shared__ double sm[];
    const int4 m = rec[blockIdx.x / n_inst];
    const int inst = blockIdx.x % n_inst;
    factor_row1(m, threadIdx.x, tsrc, item, J, T, sm, size_t(SI), inst);
}

__global__ void __launch_bounds__(64) k_blu_factor1(
    const int4 *__restrict__ rec, const int32_t *__restrict__ tsrc,
    const int2 *__restrict__ item, const double *__restrict__ J, double *__restrict__ T) {
    extern __shared__ double sm[];
    factor_row1(rec[blockIdx.x], threadIdx.x, tsrc, item, J, T, sm);
}

// Levels of at most kTriChainRows rows, when consecutive, run in one block:
// wavefront w takes row w of each level, and a block barrier separates the
// levels (a row reads only rows of earlier levels, whose writes the barrier
// makes visible to the block).  This saves a launch per level where the
// levels are small.
__global__ void __launch_bounds__(64 * kTriChainRows) k_blu_factor1_chain(
    int l0, int l1, const int32_t *__restrict__ lev_ptr, const int4 *__restrict__ rec,
    int stride, const int32_t *__restrict__ tsrc, const int2 *__restrict__ item,
    const double *__restrict__ J, double *__restrict__ T) {
    extern __shared__ double sm[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    for (int l = l0; l < l1; ++l) {
        const int q0 = lev_ptr[l];
        if (wv < lev_ptr[l + 1] - q0)
            factor_row1(rec[q0 + wv], lane, tsrc, item, J, T, sm + size_t(wv) * size_t(stride));
        __syncthreads();
    }
}

// forward: Y[r] = F[pivP[r]] - sum_{k < r} t_rk Y[k]
// (rec: the rows' records in level order, {row, first entry, diagonal,
// pivP[row]} forward and {row, diagonal, row end, 0} backward)
__global__ void __launch_bounds__(64) k_blu_fwd(
    const int4 *__restrict__ rec, int n_chunks, int W, int n_inst, int SI,
    const int32_t *__restrict__ tci, const double *__restrict__ T, const double *__restrict__ F,
    double *__restrict__ Y) {
    const int lane = threadIdx.x;
    const int4 m = rec[blockIdx.x / n_chunks];
    const int r = m.x;
    const int inst = (blockIdx.x % n_chunks) * W + lane;
    if (lane >= W || inst >= n_inst) return;
    double s = F[size_t(m.w) * SI + inst];
    const int e1 = m.z;   // the strictly lower part ends at the diagonal
    for (int e0 = m.y; e0 < e1; e0 += kG) {
        int c[kG];
        double t[kG], y[kG];
#pragma unroll
        for (int q = 0; q < kG; ++q) c[q] = tci[e0 + q];
#pragma unroll
        for (int q = 0; q < kG; ++q) {
            t[q] = T[size_t(e0 + q) * SI + inst];
            y[q] = Y[size_t(c[q]) * SI + inst];
        }
#pragma unroll
        for (int q = 0; q < kG; ++q)
            if (e0 + q < e1) s = fma(-t[q], y[q], s);
    }
    Y[size_t(r) * SI + inst] = s;
}

// backward: Y[r] = (Y[r] - sum_{j > r} t_rj Y[j]) / t_rr
__global__ void __launch_bounds__(64) k_blu_bwd(
    const int4 *__restrict__ rec, int n_chunks, int W, int n_inst, int SI,
    const int32_t *__restrict__ tci, const double *__restrict__ T, double *__restrict__ Y) {
    const int lane = threadIdx.x;
    const int4 m = rec[blockIdx.x / n_chunks];
    const int r = m.x;
    const int inst = (blockIdx.x % n_chunks) * W + lane;
    if (lane >= W || inst >= n_inst) return;
    double s = Y[size_t(r) * SI + inst];
    const int e1 = m.z;
    for (int e0 = m.y + 1; e0 < e1; e0 += kG) {
        int c[kG];
        double t[kG], y[kG];
#pragma unroll
        for (int q = 0; q < kG; ++q) c[q] = tci[e0 + q];
#pragma unroll
        for (int q = 0; q < kG; ++q) {
            t[q] = T[size_t(e0 + q) * SI + inst];
            y[q] = Y[size_t(c[q]) * SI + inst];
        }
#pragma unroll
        for (int q = 0; q < kG; ++q)
            if (e0 + q < e1) s = fma(-t[q], y[q], s);
    }
    Y[size_t(r) * SI + inst] = s / T[size_t(m.y) * SI + inst];
}


// x[pivQ[k]] -= z[k] for active instances (subtract = 1), or x[pivQ[k]] = z[k]
// (subtract = 0); one block per (row k, 256 instances)
__global__ void __launch_bounds__(256) k_blu_step(int n, int n_inst, int SI, int inst_blocks,
                                                  int subtract,
                                                  const int32_t *__restrict__ pivQ,
                                                  const int32_t *__restrict__ active,
                                                  const double *__restrict__ Z,
                                                  double *__restrict__ X) {
    const int k = blockIdx.x / inst_blocks;
    const int inst = (blockIdx.x % inst_blocks) * 256 + threadIdx.x;
    if (inst >= n_inst || k >= n) return;
    const size_t dst = size_t(pivQ[k]) * SI + inst;
    const double z = Z[size_t(k) * SI + inst];
    if (!subtract)
        X[dst] = z;
    else if (active[inst])
        X[dst] -= z;
}

__device__ __forceinline__ double bmax(double m, double a) {
    return (a > m || a != a) && !(m != m) ? a : m;
}

// per-instance max |F| over rows: part[rb][inst] over row block rb
__global__ void __launch_bounds__(256) k_blu_norm_part(int n, int n_inst, int SI, int rows_per,
                                                       const double *__restrict__ F,
                                                       double *__restrict__ part) {
    const int inst = blockIdx.x * 256 + threadIdx.x;
    if (inst >= n_inst) return;
    const int r0 = blockIdx.y * rows_per, r1 = min(n, r0 + rows_per);
    double m = 0.0;
    for (int r = r0; r < r1; ++r) m = bmax(m, fabs(F[size_t(r) * SI + inst]));
    part[size_t(blockIdx.y) * SI + inst] = m;
}

// fold the row blocks' maxima: 64 instances per block, 4 slices of the row
// blocks per instance (loads issued kG at a time), combined in LDS
__global__ void __launch_bounds__(256) k_blu_norm_fold(int nb, int n_inst, int SI,
                                                       const double *__restrict__ part,
                                                       double *__restrict__ norm) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int inst = blockIdx.x * 64 + lane;
    double m = 0.0;
    if (inst < n_inst) {
        for (int b0 = sl * kG; b0 < nb; b0 += 4 * kG) {
            double v[kG];
#pragma unroll
            for (int q = 0; q < kG; ++q) v[q] = b0 + q < nb ? part[size_t(b0 + q) * SI + inst] : 0.0;
#pragma unroll
            for (int q = 0; q < kG; ++q) m = bmax(m, v[q]);
        }
    }
    red[sl][lane] = m;
    __syncthreads();
    if (sl == 0 && inst < n_inst)
        norm[inst] = bmax(bmax(red[0][lane], red[1][lane]), bmax(red[2][lane], red[3][lane]));
}

// ---------------------------------------------------------------------------
// host-side structure
// ---------------------------------------------------------------------------

int build(pf_batch_lu *b, const HostPlan &hp, int64_t nnzT, const int32_t *trp,
          const int32_t *tci, const int32_t *pivP, const int32_t *pivQ, size_t lds_limit) {
    const int n = int(hp.n);
    std::vector<int32_t> tdiag(size_t(n), -1), tsrc(size_t(nnzT) + kPad, -1);
    // Jacobian slot of each T entry: entry (r, c) of P M Q is (pivP[r], pivQ[c]) of M
    for (int r = 0; r < n; ++r) {
        const int32_t mr = pivP[r];
        const int32_t *b0 = hp.colidx.data() + hp.rowptr[size_t(mr)];
        const int32_t *b1 = hp.colidx.data() + hp.rowptr[size_t(mr) + 1];
        for (int32_t e = trp[r]; e < trp[r + 1]; ++e) {
            if (tci[e] == r) tdiag[size_t(r)] = e;
            const int32_t mc = pivQ[tci[e]];
            const int32_t *p = std::lower_bound(b0, b1, mc);
            if (p != b1 && *p == mc) tsrc[size_t(e)] = int32_t(p - hp.colidx.data());
        }
        if (tdiag[size_t(r)] < 0) return fail(PF_EINVAL, "T lacks the diagonal of row %d", r);
    }
    // every Jacobian slot must land in T
    {
        std::vector<char> hit(size_t(hp.nnz), 0);
        for (int32_t s : tsrc)
            if (s >= 0) hit[size_t(s)] = 1;
        for (int64_t s = 0; s < hp.nnz; ++s)
            if (!hit[size_t(s)])
                return fail(PF_EINVAL, "T does not hold every Jacobian entry (slot %lld)", (long long)s);
    }
    // elimination items; T must be closed under elimination
    std::vector<int32_t> item_ptr(size_t(n) + 1, 0);
    std::vector<int2> item;
    std::vector<int32_t> flev(size_t(n), 0);
    for (int r = 0; r < n; ++r) {
        const int32_t r0 = trp[r], r1 = trp[r + 1];
        int lev = 0;
        for (int32_t e = r0; e < r1 && tci[e] < r; ++e) {
            const int k = tci[e];
            lev = std::max(lev, flev[size_t(k)] + 1);
            item.push_back(make_int2(-(e - r0) - 1, tdiag[size_t(k)]));
            for (int32_t f = tdiag[size_t(k)] + 1; f < trp[k + 1]; ++f) {
                const int32_t j = tci[f];
                const int32_t *p = std::lower_bound(tci + r0, tci + r1, j);
                if (p == tci + r1 || *p != j)
                    return fail(PF_EINVAL, "T is not closed under elimination (row %d, column %d)", r, j);
                item.push_back(make_int2(int32_t(p - (tci + r0)), f));
            }
            if (item.size() > size_t(INT32_MAX)) return fail(PF_EINVAL, "elimination too large");
        }
        flev[size_t(r)] = lev;
        item_ptr[size_t(r) + 1] = int32_t(item.size());
    }
    // backward levels over U
    std::vector<int32_t> blev(size_t(n), 0);
    for (int r = n - 1; r >= 0; --r) {
        int lev = 0;
        for (int32_t e = tdiag[size_t(r)] + 1; e < trp[r + 1]; ++e)
            lev = std::max(lev, blev[size_t(tci[e])] + 1);
        blev[size_t(r)] = lev;
    }
    auto group = [&](const std::vector<int32_t> &lev, std::vector<int32_t> &ptr,
                     std::vector<int32_t> &rows) {
        const int nl = n ? 1 + *std::max_element(lev.begin(), lev.end()) : 0;
        ptr.assign(size_t(nl) + 1, 0);
        for (int r = 0; r < n; ++r) ptr[size_t(lev[size_t(r)]) + 1]++;
        for (int l = 0; l < nl; ++l) ptr[size_t(l) + 1] += ptr[size_t(l)];
        rows.assign(size_t(n), 0);
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int r = 0; r < n; ++r) rows[size_t(fill[size_t(lev[size_t(r)])]++)] = r;
    };
    std::vector<int32_t> frows, brows;
    group(flev, b->flev_ptr, frows);
    group(blev, b->blev_ptr, brows);
    const size_t nfl = b->flev_ptr.size() - 1;
    b->flev_w.assign(nfl, 64);
    b->flev_maxr.assign(nfl, 0);
    b->flev_maxi.assign(nfl, 0);
    for (size_t l = 0; l < nfl; ++l) {
        int maxr = 0;
        for (int32_t q = b->flev_ptr[l]; q < b->flev_ptr[l + 1]; ++q) {
            const int r = frows[size_t(q)];
            maxr = std::max(maxr, trp[r + 1] - trp[r]);
            b->flev_maxi[l] = std::max(b->flev_maxi[l], item_ptr[size_t(r) + 1] - item_ptr[size_t(r)]);
        }
        b->flev_maxr[l] = maxr;
        // no more lanes than the instances need (16, 32 or 64), at most what
        // the LDS allows for the level's longest row
        const int wneed = b->n_inst <= 16 ? 16 : b->n_inst <= 32 ? 32 : 64;
        b->flev_w[l] = std::min(lanes_for(maxr, lds_limit), wneed);
        if (!b->flev_w[l])
            return fail(PF_EINVAL, "a row of T has %d entries: too long for the batched factorisation", maxr);
    }
    b->blev_w.assign(b->blev_ptr.size() - 1, 64);
    if (b->n_inst == 1 && b->ld == 1) {
        auto nrows = [](const std::vector<int32_t> &ptr, size_t l) { return ptr[l + 1] - ptr[l]; };
        // LDS of a factorisation level's row, in doubles per wavefront
        auto lds_of = [&](size_t l) {
            const size_t bytes = size_t(b->flev_maxr[l] + b->flev_maxi[l]) * sizeof(double) +
                                 size_t(b->flev_maxi[l]) * sizeof(int32_t);
            return (bytes + sizeof(double) - 1) / sizeof(double);
        };
        // factorisation: runs of small levels whose rows fit the block's LDS together
        for (size_t l = 0; l < nfl;) {
            size_t e = l;
            int w = 0;
            size_t stride = 0;
            while (e < nfl && nrows(b->flev_ptr, e) <= kTriChainRows) {
                const int w2 = std::max(w, nrows(b->flev_ptr, e));
                const size_t s2 = std::max(stride, lds_of(e));
                if (size_t(w2) * s2 * sizeof(double) > lds_limit) break;
                w = w2;
                stride = s2;
                ++e;
            }
            if (e - l >= 2) {
                b->fchain_factor.insert(b->fchain_factor.end(),
                                        {int32_t(l), int32_t(e), int32_t(w), int32_t(stride)});
                l = e;
            } else {
                l = std::max(e, l + 1);
            }
        }
        b->tri.flev_ptr = b->flev_ptr;
        b->tri.blev_ptr = b->blev_ptr;
        tri_chains(b->tri.flev_ptr, b->tri.fchain);
        tri_chains(b->tri.blev_ptr, b->tri.bchain);
    }
    // the solves' row records (every instance count)
    b->tri.tdiag = tdiag;
    b->tri.frows = frows;
    b->tri.brows = brows;
    tri_records(trp, pivP, b->tri);
    int rc = PF_OK;
    if (!rc) rc = balloc(&b->trp, trp, size_t(n) + 1);
    std::vector<int32_t> tci_pad(tci, tci + nnzT);
    tci_pad.resize(size_t(nnzT) + kPad, 0);
    item.resize(item.size() + kPad, make_int2(0, 0));
    if (!rc) rc = balloc(&b->tci, tci_pad.data(), tci_pad.size());
    if (!rc) rc = balloc(&b->tsrc, tsrc.data(), tsrc.size());
    if (!rc) rc = balloc(&b->item_ptr, item_ptr.data(), item_ptr.size());
    if (!rc) rc = balloc(&b->item, item.data(), item.size());
    if (!rc) rc = balloc(&b->frows, frows.data(), frows.size());
    if (!rc) rc = balloc(&b->flev_ptr_d, b->flev_ptr.data(), b->flev_ptr.size());
    if (!rc) rc = balloc(&b->blev_ptr_d, b->blev_ptr.data(), b->blev_ptr.size());
    if (!rc) rc = balloc(&b->pivQ, pivQ, size_t(n));
    {
        std::vector<int4> fr(frows.size());
        for (size_t q = 0; q < frows.size(); ++q) {
            const int r = frows[q];
            fr[q] = make_int4(trp[r], trp[r + 1], item_ptr[size_t(r)], item_ptr[size_t(r) + 1]);
        }
        if (!rc) rc = balloc(&b->frec_factor, fr.data(), fr.size());
    }
    if (!rc) rc = balloc(&b->frec, b->tri.frec.data(), b->tri.frec.size());
    if (!rc) rc = balloc(&b->brec, b->tri.brec.data(), b->tri.brec.size());
    return rc;
}

int factor_levels(pf_batch_lu *b, const double *J, hipStream_t st) {
    const int I = b->n_inst, SI = b->ld;
    const bool one = I == 1 && SI == 1;
    size_t ci = 0;   // next run of small levels
    for (size_t l = 0; l + 1 < b->flev_ptr.size(); ++l) {
        const int nr = b->flev_ptr[l + 1] - b->flev_ptr[l];
        if (one && ci < b->fchain_factor.size() && size_t(b->fchain_factor[ci]) == l) {
            const int l1 = b->fchain_factor[ci + 1], w = b->fchain_factor[ci + 2];
            const int stride = b->fchain_factor[ci + 3];
            hipLaunchKernelGGL(k_blu_factor1_chain, dim3(1), dim3(unsigned(64 * w)),
                               size_t(w) * size_t(stride) * sizeof(double), st, int(l), l1,
                               b->flev_ptr_d, b->frec_factor, stride, b->tsrc, b->item, J, b->T);
            l = size_t(l1) - 1;
            ci += 4;
            continue;
        }
        if (one) {   // one instance: lanes spread over the row
            const size_t shm1 = size_t(b->flev_maxr[l] + b->flev_maxi[l]) * sizeof(double) +
                                size_t(b->flev_maxi[l]) * sizeof(int32_t);
            if (shm1 <= b->lds_limit) {
                hipLaunchKernelGGL(k_blu_factor1, dim3(unsigned(nr)), dim3(64), shm1, st,
                                   b->frec_factor + b->flev_ptr[l], b->tsrc, b->item, J, b->T);
                continue;
            }
        }
        if (!one && int64_t(nr) * I <= kInstWaves) {
            const size_t shm1 = size_t(b->flev_maxr[l] + b->flev_maxi[l]) * sizeof(double) +
                                size_t(b->flev_maxi[l]) * sizeof(int32_t);
            if (shm1 <= b->lds_limit) {
                hipLaunchKernelGGL(k_blu_factor_inst, dim3(unsigned(int64_t(nr) * I)), dim3(64), shm1,
                                   st, b->frec_factor + b->flev_ptr[l], I, SI, b->tsrc, b->item,
                                   J, b->T);
                continue;
            }
        }
        const int W = b->flev_w[l];
        const int nc = (I + W - 1) / W;
        const size_t shm = size_t(b->flev_maxr[l]) * size_t(W) * sizeof(double);
        hipLaunchKernelGGL(k_blu_factor, dim3(unsigned(int64_t(nr) * nc)), dim3(64), shm, st,
                           b->frows + b->flev_ptr[l], nc, W, I, SI, b->trp, b->tsrc,
                           b->item_ptr, b->item, J, b->T);
    }
    BL_HIP(hipGetLastError());
    return PF_OK;
}

int solve_levels(pf_batch_lu *b, const double *Fin, double *Y, hipStream_t st) {
    const int I = b->n_inst, SI = b->ld;
    const int nc = (I + 63) / 64;
    if (I == 1 && SI == 1) {   // one instance: lanes over each row's entries
        const TriDev d{b->flev_ptr_d, b->blev_ptr_d, b->frec, b->brec, b->tci, b->T};
        tri_solve(b->tri, d, Fin, Y, st);
        BL_HIP(hipGetLastError());
        return PF_OK;
    }
    for (size_t l = 0; l + 1 < b->flev_ptr.size(); ++l) {
        const int nr = b->flev_ptr[l + 1] - b->flev_ptr[l];
        hipLaunchKernelGGL(k_blu_fwd, dim3(unsigned(int64_t(nr) * nc)), dim3(64), 0, st,
                           b->frec + b->flev_ptr[l], nc, 64, I, SI, b->tci, b->T, Fin, Y);
    }
    for (size_t l = 0; l + 1 < b->blev_ptr.size(); ++l) {
        const int nr = b->blev_ptr[l + 1] - b->blev_ptr[l];
        hipLaunchKernelGGL(k_blu_bwd, dim3(unsigned(int64_t(nr) * nc)), dim3(64), 0, st,
                           b->brec + b->blev_ptr[l], nc, 64, I, SI, b->tci, b->T, Y);
    }
    BL_HIP(hipGetLastError());
    return PF_OK;
}

}  // namespace

extern "C" {

int pf_batch_lu_create(pf_plan *plan, int64_t nnzT, const int32_t *T_rowptr,
                       const int32_t *T_colidx, const int32_t *pivP, const int32_t *pivQ,
                       pf_batch_lu **out) {
    clear_error();
    if (!out) return fail(PF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    const HostPlan &hp = plan->host;
    // single-instance and multi-grid plans are one instance of row pitch 1
    if (hp.kind != KIND_BATCH && (hp.n_inst != 1 || hp.ld != 1))
        return fail(PF_EINVAL, "unexpected instance layout of a single-instance plan");
    if (hp.panels) return fail(PF_EINVAL, "the batched factorisation needs the row layout");
    if (!T_rowptr || !T_colidx || !pivP || !pivQ) return fail(PF_EINVAL, "NULL argument");
    const int64_t n = hp.n;
    if (n < 1 || n > INT32_MAX - 1) return fail(PF_EINVAL, "bad system size");
    if (nnzT < n || nnzT > INT32_MAX) return fail(PF_EINVAL, "nnzT must be in [n, 2^31)");
    if (T_rowptr[0] != 0 || T_rowptr[n] != nnzT) return fail(PF_EINVAL, "T_rowptr must start at 0 and end at nnzT");
    for (int64_t r = 0; r < n; ++r) {
        if (T_rowptr[r + 1] < T_rowptr[r]) return fail(PF_EINVAL, "T_rowptr is not non-decreasing");
        for (int32_t e = T_rowptr[r]; e < T_rowptr[r + 1]; ++e) {
            if (T_colidx[e] < 0 || T_colidx[e] >= n) return fail(PF_EINVAL, "T_colidx out of range");
            if (e > T_rowptr[r] && T_colidx[e] <= T_colidx[e - 1])
                return fail(PF_EINVAL, "T_colidx not strictly increasing in a row");
        }
    }
    if (!is_perm(pivP, int(n)) || !is_perm(pivQ, int(n)))
        return fail(PF_EINVAL, "pivP and pivQ must be permutations of 0..n-1");
    if (hp.host_only || !plan->dev) return fail(PF_EINVAL, "plan is host-only");
    BGuard g(hp.device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", hp.device);
    int lds = 0;
    BL_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hp.device));
    // rows of the factorisation live in dynamic LDS, up to the device's limit
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_blu_factor),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_blu_factor1),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_blu_factor1_chain),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_blu_factor_inst),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    pf_batch_lu *b = new (std::nothrow) pf_batch_lu();
    if (!b) return fail(PF_ENOMEM, "host allocation failed");
    b->plan = plan;
    b->device = hp.device;
    b->n = int(n);
    b->nnzT = int(nnzT);
    b->n_inst = hp.n_inst;
    b->ld = hp.ld;
    b->lds_limit = size_t(lds);
    b->switch_safe = pivots_switch_safe(hp, pivP, pivQ);
    int rc;
    try {
        rc = build(b, hp, nnzT, T_rowptr, T_colidx, pivP, pivQ, size_t(lds));
    } catch (const std::bad_alloc &) {
        rc = fail(PF_ENOMEM, "host allocation failed");
    }
    const size_t SI = size_t(hp.ld);
    b->part_rows = int((n + kNormRowBlocks - 1) / kNormRowBlocks);
    if (!rc) rc = balloc<double>(&b->T, nullptr, (size_t(nnzT) + kPad) * SI);
    if (!rc) rc = balloc<double>(&b->F, nullptr, size_t(n) * SI);
    if (!rc) rc = balloc<double>(&b->J, nullptr, size_t(hp.nnz) * SI);
    if (!rc) rc = balloc<double>(&b->Y, nullptr, size_t(n) * SI);
    if (!rc) rc = balloc<double>(&b->part, nullptr, size_t(kNormRowBlocks) * SI);
    if (!rc) rc = balloc<double>(&b->norm, nullptr, SI);
    if (!rc) rc = balloc<int32_t>(&b->active, nullptr, SI);
    if (!rc && hipHostMalloc(&b->norm_host, SI * sizeof(double), hipHostMallocDefault) != hipSuccess)
        rc = fail(PF_ENOMEM, "pinned allocation failed");
    if (rc) {
        release(b);
        return rc;
    }
    *out = b;
    return PF_OK;
}

void pf_batch_lu_destroy(pf_batch_lu *b) { release(b); }

int pf_batch_lu_factor(pf_batch_lu *b, const double *J, void *stream) {
    clear_error();
    if (!b || !J) return fail(PF_EINVAL, "NULL argument");
    BGuard g(b->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", b->device);
    return factor_levels(b, J, static_cast<hipStream_t>(stream));
}

int pf_batch_lu_solve(pf_batch_lu *b, const double *B, double *Xout, void *stream) {
    clear_error();
    if (!b || !B || !Xout) return fail(PF_EINVAL, "NULL argument");
    if (B == Xout) return fail(PF_EINVAL, "B and Xout must not alias");
    BGuard g(b->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", b->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = solve_levels(b, B, b->Y, st);
    if (rc) return rc;
    const int ib = (b->n_inst + 255) / 256;
    hipLaunchKernelGGL(k_blu_step, dim3(unsigned(int64_t(ib) * b->n)), dim3(256), 0, st, b->n,
                       b->n_inst, b->ld, ib, 0, b->pivQ, b->active, b->Y, Xout);
    BL_HIP(hipGetLastError());
    return PF_OK;
}

int pf_newton_batch(pf_plan *plan, pf_batch_lu *b, double *X, const pf_newton_opts *opts,
                    int32_t *inst_iters, double *inst_norm, pf_newton_report *report,
                    void *stream) {
    clear_error();
    if (!plan || !b || !X) return fail(PF_EINVAL, "NULL argument");
    if (b->plan != plan) return fail(PF_EINVAL, "the factorisation belongs to another plan");
    if (opts && opts->max_iter > 64) return fail(PF_EINVAL, "max_iter must be <= 64");
    HostPlan &hp = plan->host;
    const bool limits = opts && (opts->q_min || opts->q_max);
    const double check_below = (limits && opts->q_check_below > 0) ? opts->q_check_below : 1e-3;
    const double switch_tol = (limits && opts->q_switch_tol >= 0) ? opts->q_switch_tol : 1e-9;
    if (limits) {
        const int e = q_limits_valid(hp, opts->q_min, opts->q_max, switch_tol);
        if (e) return e;
        if (!b->switch_safe)
            return fail(PF_EINVAL, "reactive limits need a factorisation whose pivots survive a "
                        "switch (pf_jacobian_switch_order); this one's do not");
    }
    BGuard g(b->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", b->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double tol = (opts && opts->tol > 0) ? opts->tol : 1e-10;
    const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 10;
    const int I = b->n_inst, SI = b->ld, n = b->n;
    std::vector<int32_t> act(size_t(SI), 0), iters(size_t(I), 0);
    // limits are checked on plans of one instance only (switch_safe): X is
    // then the plain state
    std::vector<double> xh(limits ? size_t(n) : 0);
    for (int i = 0; i < I; ++i) act[size_t(i)] = 1;
    pf_newton_report r{};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    for (auto &e : ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            for (auto &f : ev)
                if (f) (void)hipEventDestroy(f);
            return fail(PF_EDEVICE, "hipEventCreate failed");
        }
    }
    float ms = 0.f;
    auto t_start = std::chrono::steady_clock::now();
    int rc = PF_OK;
    int it = 0;
    int n_conv = 0;
    // F and J at X under the current modes, and every instance's ||F||_inf
    // on the host (norm_host)
    auto evaluate = [&]() -> int {
        (void)hipEventRecord(ev[0], st);
        const int e = hp.kind == KIND_BATCH ? dev_eval_batch(hp, plan->dev, X, b->F, b->J, st)
                                            : dev_eval_single(hp, plan->dev, X, b->F, b->J, st);
        if (e) return e;
        (void)hipEventRecord(ev[1], st);
        hipLaunchKernelGGL(k_blu_norm_part, dim3(unsigned((I + 255) / 256), kNormRowBlocks),
                           dim3(256), 0, st, n, I, SI, b->part_rows, b->F, b->part);
        hipLaunchKernelGGL(k_blu_norm_fold, dim3(unsigned((I + 63) / 64)), dim3(256), 0, st,
                           kNormRowBlocks, I, SI, b->part, b->norm);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(b->norm_host, b->norm, size_t(I) * sizeof(double),
                           hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fail(PF_EDEVICE, "device step failed in iteration %d", it);
        if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) r.t_eval_s += ms * 1e-3;
        return PF_OK;
    };
    for (;; ++it) {
        rc = evaluate();
        if (rc) break;
        // the limits at this iterate (as pf_newton): after a switch F and J
        // are evaluated again under the new modes before the step
        int32_t ns = 0;
        if (limits && b->norm_host[0] < check_below) {
            if (hipMemcpyAsync(xh.data(), X, size_t(n) * sizeof(double), hipMemcpyDeviceToHost,
                               st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = fail(PF_EDEVICE, "copy of the state failed in iteration %d", it);
                break;
            }
            rc = q_switch(hp, plan->dev, xh.data(), opts->q_min, opts->q_max, switch_tol, &ns);
            if (!rc && ns) rc = evaluate();
            if (rc) break;
        }
        if (it < 65) r.switched[it] = ns;
        r.n_switches += ns;
        // an instance stops once its norm is below tol (under modes that
        // the check left unchanged); it is not stepped again
        n_conv = 0;
        double worst = 0.0;
        for (int i = 0; i < I; ++i) {
            const double v = b->norm_host[i];
            if (act[size_t(i)] && v < tol && ns == 0) act[size_t(i)] = 0;
            if (!act[size_t(i)]) ++n_conv;
            else if (v != v || worst != worst) worst = NAN;
            else if (v > worst) worst = v;
        }
        if (it < 65) r.norm[it] = worst;
        if (n_conv == I) {
            rc = PF_OK;
            break;
        }
        if (it >= max_iter) {
            rc = fail(PF_ENOCONV, "%d of %d instances did not converge in %d iterations", I - n_conv,
                      I, max_iter);
            break;
        }
        for (int i = 0; i < I; ++i)
            if (act[size_t(i)]) iters[size_t(i)] = it + 1;
        if (hipMemcpyAsync(b->active, act.data(), size_t(SI) * sizeof(int32_t),
                           hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = fail(PF_EDEVICE, "copy of the active mask failed");
            break;
        }
        (void)hipEventRecord(ev[2], st);
        rc = factor_levels(b, b->J, st);
        if (rc) break;
        rc = solve_levels(b, b->F, b->Y, st);
        if (rc) break;
        const int ib = (I + 255) / 256;
        hipLaunchKernelGGL(k_blu_step, dim3(unsigned(int64_t(ib) * n)), dim3(256), 0, st, n, I,
                           SI, ib, 1, b->pivQ, b->active, b->Y, X);
        (void)hipEventRecord(ev[3], st);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(PF_EDEVICE, "device step failed in iteration %d", it);
            break;
        }
        if (hipEventElapsedTime(&ms, ev[2], ev[3]) == hipSuccess) r.t_solve_s += ms * 1e-3;
        r.iterations = it + 1;
    }
    (void)hipStreamSynchronize(st);
    r.converged = n_conv;
    r.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (inst_iters) std::memcpy(inst_iters, iters.data(), size_t(I) * sizeof(int32_t));
    if (inst_norm) std::memcpy(inst_norm, b->norm_host, size_t(I) * sizeof(double));
    if (report) *report = r;
    return rc;
}

}  // extern "C"
