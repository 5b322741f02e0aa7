// Level-scheduled triangular solves with one right-hand side along the
// factor T = (L - I) + U of P M Q = L U (CSR, unit lower part below the
// diagonal, U on and above it):
//   forward:   Y[r] = B[pivP[r]] - sum_{k < r} t_rk Y[k]
//   backward:  Y[r] = (Y[r] - sum_{j > r} t_rj Y[j]) / t_rr
//   result:    X[pivQ[k]] = Y[k]   (left to the caller)
// Rows of one level depend only on rows of earlier levels.  A wavefront takes
// a row, its lanes over the row's entries, and combines the lanes' partial
// sums by a fixed butterfly (deterministic).  Each row's bounds come from one
// record in level order ({row, first entry, diagonal, pivP[row]} forward,
// {row, diagonal, row end, 0} backward), so a row waits on one load before
// its entries rather than on the row id and then its bounds.  Consecutive levels of at most
// kTriChainRows rows run in one block, a wavefront per row and a block
// barrier between levels, which saves a launch per level where levels are
// small.  Internal to libpf; included by the device sources that solve.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

namespace {

// Rows of a level in a run, and wavefronts of a run's block, at most (runs of
// levels up to 32 rows, two rows per wavefront, measured no faster; up to 64,
// slower).
constexpr int kTriChainRows = 16;

__device__ __forceinline__ double tri_wave_sum(double p) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off);
    return p;
}

__device__ __forceinline__ void tri_fwd_row(int4 m, int lane, const int32_t *__restrict__ tci,
                                            const double *__restrict__ T,
                                            const double *__restrict__ B, double *__restrict__ Y) {
    const double bv = B[m.w];
    double p = 0.0;
    for (int e = m.y + lane; e < m.z; e += 64) p = fma(T[e], Y[tci[e]], p);
    p = tri_wave_sum(p);
    if (lane == 0) Y[m.x] = bv - p;
}

__device__ __forceinline__ void tri_bwd_row(int4 m, int lane, const int32_t *__restrict__ tci,
                                            const double *__restrict__ T, double *__restrict__ Y) {
    const double yr = Y[m.x], td = T[m.y];
    double p = 0.0;
    for (int e = m.y + 1 + lane; e < m.z; e += 64) p = fma(T[e], Y[tci[e]], p);
    p = tri_wave_sum(p);
    if (lane == 0) Y[m.x] = (yr - p) / td;
}

// one level: a block (one wavefront) per row
__global__ void __launch_bounds__(64) k_tri_fwd(
    const int4 *__restrict__ rec, const int32_t *__restrict__ tci, const double *__restrict__ T,
    const double *__restrict__ B, double *__restrict__ Y) {
    tri_fwd_row(rec[blockIdx.x], threadIdx.x, tci, T, B, Y);
}

__global__ void __launch_bounds__(64) k_tri_bwd(
    const int4 *__restrict__ rec, const int32_t *__restrict__ tci, const double *__restrict__ T,
    double *__restrict__ Y) {
    tri_bwd_row(rec[blockIdx.x], threadIdx.x, tci, T, Y);
}

// levels l0 .. l1-1 of at most kTriChainRows rows in one block: wavefront w
// takes rows w, w + (wavefronts), ... of each level; the barrier makes a
// level's results visible to the block before the next level reads them
__global__ void __launch_bounds__(64 * kTriChainRows) k_tri_fwd_chain(
    int l0, int l1, const int32_t *__restrict__ lev_ptr, const int4 *__restrict__ rec,
    const int32_t *__restrict__ tci, const double *__restrict__ T, const double *__restrict__ B,
    double *__restrict__ Y) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int l = l0; l < l1; ++l) {
        const int q0 = lev_ptr[l], nr = lev_ptr[l + 1] - q0;
        for (int i = wv; i < nr; i += nw) tri_fwd_row(rec[q0 + i], lane, tci, T, B, Y);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(64 * kTriChainRows) k_tri_bwd_chain(
    int l0, int l1, const int32_t *__restrict__ lev_ptr, const int4 *__restrict__ rec,
    const int32_t *__restrict__ tci, const double *__restrict__ T, double *__restrict__ Y) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int l = l0; l < l1; ++l) {
        const int q0 = lev_ptr[l], nr = lev_ptr[l + 1] - q0;
        for (int i = wv; i < nr; i += nw) tri_bwd_row(rec[q0 + i], lane, tci, T, Y);
        __syncthreads();
    }
}

// Host: runs of at least two consecutive levels of at most kTriChainRows
// rows, as {first level, end level, widest level's rows}.
inline void tri_chains(const std::vector<int32_t> &ptr, std::vector<int32_t> &out) {
    out.clear();
    const size_t nl = ptr.empty() ? 0 : ptr.size() - 1;
    for (size_t l = 0; l < nl;) {
        size_t e = l;
        int w = 0;
        while (e < nl && ptr[e + 1] - ptr[e] <= kTriChainRows) {
            w = std::max(w, ptr[e + 1] - ptr[e]);
            ++e;
        }
        if (e - l >= 2) {
            out.insert(out.end(), {int32_t(l), int32_t(e), int32_t(w)});
            l = e;
        } else {
            l = std::max(e, l + 1);
        }
    }
}

// Host: the level structure of the forward and backward solves of T.
struct TriLevels {
    std::vector<int32_t> tdiag;              // diagonal position of each row
    std::vector<int32_t> flev_ptr, blev_ptr; // levels -> offsets into frows / brows
    std::vector<int32_t> frows, brows;       // rows in level order
    std::vector<int32_t> fchain, bchain;     // runs of small levels
    std::vector<int4> frec, brec;            // the rows' records, in level order
};

// Host: the rows' records in level order (see the kernels above).
inline void tri_records(const int32_t *trp, const int32_t *pivP, TriLevels &t) {
    t.frec.resize(t.frows.size());
    t.brec.resize(t.brows.size());
    for (size_t q = 0; q < t.frows.size(); ++q) {
        const int32_t r = t.frows[q];
        t.frec[q] = make_int4(r, trp[r], t.tdiag[size_t(r)], pivP[r]);
    }
    for (size_t q = 0; q < t.brows.size(); ++q) {
        const int32_t r = t.brows[q];
        t.brec[q] = make_int4(r, t.tdiag[size_t(r)], trp[r + 1], 0);
    }
}

inline void tri_group(int n, const std::vector<int32_t> &lev, std::vector<int32_t> &ptr,
                      std::vector<int32_t> &rows) {
    const int nl = n ? 1 + *std::max_element(lev.begin(), lev.end()) : 0;
    ptr.assign(size_t(nl) + 1, 0);
    for (int r = 0; r < n; ++r) ptr[size_t(lev[size_t(r)]) + 1]++;
    for (int l = 0; l < nl; ++l) ptr[size_t(l) + 1] += ptr[size_t(l)];
    rows.assign(size_t(n), 0);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int r = 0; r < n; ++r) rows[size_t(fill[size_t(lev[size_t(r)])]++)] = r;
}

// T's rows must hold their diagonal (checked by the caller).
inline void tri_levels(int n, const int32_t *trp, const int32_t *tci, TriLevels &t) {
    t.tdiag.assign(size_t(n), 0);
    std::vector<int32_t> flev(size_t(n), 0), blev(size_t(n), 0);
    for (int r = 0; r < n; ++r) {
        int lev = 0;
        for (int32_t e = trp[r]; e < trp[r + 1]; ++e) {
            if (tci[e] < r) lev = std::max(lev, flev[size_t(tci[e])] + 1);
            if (tci[e] == r) t.tdiag[size_t(r)] = e;
        }
        flev[size_t(r)] = lev;
    }
    for (int r = n - 1; r >= 0; --r) {
        int lev = 0;
        for (int32_t e = t.tdiag[size_t(r)] + 1; e < trp[r + 1]; ++e)
            lev = std::max(lev, blev[size_t(tci[e])] + 1);
        blev[size_t(r)] = lev;
    }
    tri_group(n, flev, t.flev_ptr, t.frows);
    tri_group(n, blev, t.blev_ptr, t.brows);
    tri_chains(t.flev_ptr, t.fchain);
    tri_chains(t.blev_ptr, t.bchain);
}

// Device copies of what the solve kernels read.
struct TriDev {
    const int32_t *flev_ptr, *blev_ptr;
    const int4 *frec, *brec;
    const int32_t *tci;
    const double *T;
};

// Forward then backward solve of one right-hand side B into Y (device, n),
// on the stream; Y must not alias B.  Launch errors are left for the caller
// to collect.
inline void tri_solve(const TriLevels &h, const TriDev &d, const double *B, double *Y,
                      hipStream_t st) {
    size_t ci = 0;
    for (size_t l = 0; l + 1 < h.flev_ptr.size(); ++l) {
        if (ci < h.fchain.size() && size_t(h.fchain[ci]) == l) {
            const int l1 = h.fchain[ci + 1], w = h.fchain[ci + 2];
            hipLaunchKernelGGL(k_tri_fwd_chain, dim3(1), dim3(unsigned(64 * w)), 0, st, int(l), l1,
                               d.flev_ptr, d.frec, d.tci, d.T, B, Y);
            l = size_t(l1) - 1;
            ci += 3;
            continue;
        }
        const int nr = h.flev_ptr[l + 1] - h.flev_ptr[l];
        hipLaunchKernelGGL(k_tri_fwd, dim3(unsigned(nr)), dim3(64), 0, st, d.frec + h.flev_ptr[l],
                           d.tci, d.T, B, Y);
    }
    ci = 0;
    for (size_t l = 0; l + 1 < h.blev_ptr.size(); ++l) {
        if (ci < h.bchain.size() && size_t(h.bchain[ci]) == l) {
            const int l1 = h.bchain[ci + 1], w = h.bchain[ci + 2];
            hipLaunchKernelGGL(k_tri_bwd_chain, dim3(1), dim3(unsigned(64 * w)), 0, st, int(l), l1,
                               d.blev_ptr, d.brec, d.tci, d.T, Y);
            l = size_t(l1) - 1;
            ci += 3;
            continue;
        }
        const int nr = h.blev_ptr[l + 1] - h.blev_ptr[l];
        hipLaunchKernelGGL(k_tri_bwd, dim3(unsigned(nr)), dim3(64), 0, st, d.brec + h.blev_ptr[l],
                           d.tci, d.T, Y);
    }
}

}  // namespace
