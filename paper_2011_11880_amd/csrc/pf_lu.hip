// Device-resident Newton power flow (tasks 1-4 of the Newton loop, Section I)
// with the linear solve (task 3) done on the GPU by rocSOLVER's sparse
// re-factorisation.  The Jacobian pattern is fixed at setup, so one LU
// factorisation with pivoting (P J Q = L U, computed once by the caller on the
// host) fixes the pattern of T = (L - I) + U and both permutations; every
// later Jacobian of the same plan is refactorised numerically on the device
// along that pattern and solved there.  Nothing but the convergence test's
// one scalar per iteration leaves the GPU.
//
// rocSOLVER is loaded on first use (dlopen), so that callers that never ask
// for the device solve do not pay for loading it.
#include <dlfcn.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <vector>

#include <hip/hip_runtime.h>
#include <rocsolver/rocsolver.h>

#include "pf_internal.hpp"
#include "pf_trisolve.hpp"

#define LU_HIP(expr)                                                               \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return fail(PF_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LU_RS(expr)                                                                    \
    do {                                                                               \
        rocblas_status s_ = (expr);                                                    \
        if (s_ != rocblas_status_success)                                              \
            return fail(PF_ESOLVE, "%s failed: rocblas status %d", #expr, int(s_));   \
    } while (0)

namespace pf {
namespace {

// rocSOLVER / rocBLAS entry points used here, resolved at run time.
struct RfApi {
    decltype(&rocblas_create_handle) create_handle = nullptr;
    decltype(&rocblas_destroy_handle) destroy_handle = nullptr;
    decltype(&rocblas_set_stream) set_stream = nullptr;
    decltype(&rocsolver_create_rfinfo) create_rfinfo = nullptr;
    decltype(&rocsolver_destroy_rfinfo) destroy_rfinfo = nullptr;
    decltype(&rocsolver_dcsrrf_analysis) analysis = nullptr;
    decltype(&rocsolver_dcsrrf_refactlu) refactlu = nullptr;
    decltype(&rocsolver_dcsrrf_solve) solve = nullptr;
    bool ok = false;
    char why[256] = "";
};

const RfApi &rf_api() {
    static RfApi api;
    static std::once_flag once;
    std::call_once(once, [] {
        void *hs = dlopen("librocsolver.so.0", RTLD_NOW | RTLD_GLOBAL);
        if (!hs) hs = dlopen("/opt/rocm/lib/librocsolver.so.0", RTLD_NOW | RTLD_GLOBAL);
        void *hb = dlopen("librocblas.so.5", RTLD_NOW | RTLD_GLOBAL);
        if (!hb) hb = dlopen("/opt/rocm/lib/librocblas.so.5", RTLD_NOW | RTLD_GLOBAL);
        if (!hs || !hb) {
            snprintf(api.why, sizeof api.why, "cannot load rocSOLVER/rocBLAS: %s", dlerror());
            return;
        }
#define SYM(h, field, name)                                                     \
    api.field = reinterpret_cast<decltype(api.field)>(dlsym(h, name));          \
    if (!api.field) {                                                           \
        snprintf(api.why, sizeof api.why, "symbol %s missing", name);           \
        return;                                                                 \
    }
        SYM(hb, create_handle, "rocblas_create_handle");
        SYM(hb, destroy_handle, "rocblas_destroy_handle");
        SYM(hb, set_stream, "rocblas_set_stream");
        SYM(hs, create_rfinfo, "rocsolver_create_rfinfo");
        SYM(hs, destroy_rfinfo, "rocsolver_destroy_rfinfo");
        SYM(hs, analysis, "rocsolver_dcsrrf_analysis");
        SYM(hs, refactlu, "rocsolver_dcsrrf_refactlu");
        SYM(hs, solve, "rocsolver_dcsrrf_solve");
#undef SYM
        api.ok = true;
    });
    return api;
}

// ||F||_inf in two launches: kAbsBlocks partial maxima, then one block folds
// them.  A NaN anywhere makes the result NaN (it is never replaced).
constexpr int kAbsBlocks = 256;

__device__ __forceinline__ double absmax2(double m, double a) {
    return (a > m || a != a) && !(m != m) ? a : m;
}

__global__ void __launch_bounds__(256) k_absmax_part(int64_t n, const double *__restrict__ F,
                                                     double *__restrict__ part) {
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256)
        m = absmax2(m, fabs(F[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) red[threadIdx.x] = absmax2(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_absmax_fold(int nb, const double *__restrict__ part,
                                                     double *__restrict__ out) {
    __shared__ double red[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) m = absmax2(m, part[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) red[threadIdx.x] = absmax2(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// x <- x - dx  (the full Newton step)
__global__ void __launch_bounds__(256) k_step(int64_t n, double *__restrict__ x,
                                              const double *__restrict__ dx) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) x[i] -= dx[i];
}

}  // namespace
}  // namespace pf

using namespace pf;

struct pf_refact {
    pf_plan *plan = nullptr;
    int device = 0;
    int n = 0;
    int nnzA = 0;
    int nnzT = 0;
    int *ptrA = nullptr, *indA = nullptr;  // the plan's Jacobian pattern
    int *ptrT = nullptr, *indT = nullptr;  // pattern of (L - I) + U
    double *valT = nullptr;
    int *pivP = nullptr, *pivQ = nullptr;
    double *F = nullptr, *J = nullptr, *dx = nullptr, *part = nullptr, *norm = nullptr;
    double *norm_host = nullptr;  // pinned
    rocblas_handle handle = nullptr;
    rocsolver_rfinfo info = nullptr;
    bool switch_safe = false;     // pivots survive a PV unit's switch (pivots_switch_safe)
};

namespace {

void release(pf_refact *rf) {
    if (!rf) return;
    const RfApi &api = rf_api();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(rf->device);
    if (rf->info && api.ok) (void)api.destroy_rfinfo(rf->info);
    if (rf->handle && api.ok) (void)api.destroy_handle(rf->handle);
    for (void *p : {(void *)rf->ptrA, (void *)rf->indA, (void *)rf->ptrT, (void *)rf->indT,
                    (void *)rf->valT, (void *)rf->pivP, (void *)rf->pivQ, (void *)rf->F,
                    (void *)rf->J, (void *)rf->dx, (void *)rf->part, (void *)rf->norm})
        if (p) (void)hipFree(p);
    if (rf->norm_host) (void)hipHostFree(rf->norm_host);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete rf;
}

template <class T>
int alloc_copy(T **dst, const T *src, size_t count) {
    LU_HIP(hipMalloc(dst, (count ? count : 1) * sizeof(T)));
    if (src && count) LU_HIP(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return PF_OK;
}

bool is_permutation(const int32_t *p, int n) {
    std::vector<char> seen(size_t(n), 0);
    for (int i = 0; i < n; ++i) {
        if (p[i] < 0 || p[i] >= n || seen[size_t(p[i])]) return false;
        seen[size_t(p[i])] = 1;
    }
    return true;
}

// CSR with rowptr[0] = 0, non-decreasing, rowptr[n] = nnz, strictly increasing
// columns in range, and the diagonal present in every row.
const char *check_T(int n, int64_t nnz, const int32_t *rp, const int32_t *ci) {
    if (rp[0] != 0 || rp[n] != nnz) return "T_rowptr must start at 0 and end at nnzT";
    for (int i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return "T_rowptr is not non-decreasing";
        bool diag = false;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] < 0 || ci[k] >= n) return "T_colidx out of range";
            if (k > rp[i] && ci[k] <= ci[k - 1]) return "T_colidx not strictly increasing in a row";
            diag |= ci[k] == i;
        }
        if (!diag) return "T lacks a diagonal entry (U must have a full diagonal)";
    }
    return nullptr;
}

int symbolic(int n, const int32_t *rp, const int32_t *ci, const int32_t *pivP,
             const int32_t *pivQ, std::vector<int32_t> &trp, std::vector<int32_t> &tci);

// T must hold every entry that elimination along it reaches for matrices of
// M's pattern (the full symbolic pattern); a pattern with missing fill would
// make the device re-factorisation an incomplete one.
int check_closure(int n, const int32_t *rp, const int32_t *ci, const int32_t *pivP,
                  const int32_t *pivQ, const int32_t *T_rowptr, const int32_t *T_colidx) {
    std::vector<int32_t> srp, sci;
    int rc;
    try {
        rc = symbolic(n, rp, ci, pivP, pivQ, srp, sci);
    } catch (const std::bad_alloc &) {
        rc = fail(PF_ENOMEM, "host allocation failed");
    }
    if (rc) return rc;
    for (int r = 0; r < n; ++r) {
        int32_t t = T_rowptr[r];
        for (int32_t e = srp[size_t(r)]; e < srp[size_t(r) + 1]; ++e) {
            while (t < T_rowptr[r + 1] && T_colidx[t] < sci[size_t(e)]) ++t;
            if (t == T_rowptr[r + 1] || T_colidx[t] != sci[size_t(e)])
                return fail(PF_EINVAL,
                            "T lacks fill entry (%d, %d) of the symbolic factorisation "
                            "(pf_lu_symbolic gives the full pattern)", r, sci[size_t(e)]);
        }
    }
    return PF_OK;
}

int solve_on_stream(pf_refact *rf, const double *Jval, double *b, hipStream_t st) {
    const RfApi &api = rf_api();
    LU_RS(api.set_stream(rf->handle, st));
    LU_RS(api.refactlu(rf->handle, rf->n, rf->nnzA, rf->ptrA, rf->indA, const_cast<double *>(Jval),
                       rf->nnzT, rf->ptrT, rf->indT, rf->valT, rf->pivP, rf->pivQ, rf->info));
    LU_RS(api.solve(rf->handle, rf->n, 1, rf->nnzT, rf->ptrT, rf->indT, rf->valT, rf->pivP,
                    rf->pivQ, b, rf->n, rf->info));
    return PF_OK;
}

int absmax_on_stream(pf_refact *rf, const double *F, hipStream_t st) {
    const int nb = int(std::min<int64_t>(kAbsBlocks, (int64_t(rf->n) + 255) / 256));
    hipLaunchKernelGGL(k_absmax_part, dim3(nb), dim3(256), 0, st, int64_t(rf->n), F, rf->part);
    hipLaunchKernelGGL(k_absmax_fold, dim3(1), dim3(256), 0, st, nb, rf->part, rf->norm);
    LU_HIP(hipGetLastError());
    LU_HIP(hipMemcpyAsync(rf->norm_host, rf->norm, sizeof(double), hipMemcpyDeviceToHost, st));
    return PF_OK;
}

struct Guard {
    int prev = -1;
    bool ok = true;
    explicit Guard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) {
            ok = false;
            return;
        }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~Guard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int create(pf_plan *plan, const double *Jval_host, int64_t nnzT, const int32_t *T_rowptr,
           const int32_t *T_colidx, const double *T_val, const int32_t *pivP,
           const int32_t *pivQ, pf_refact *rf) {
    const HostPlan &hp = plan->host;
    const int n = int(hp.n);
    const RfApi &api = rf_api();
    if (!api.ok) return fail(PF_EDEVICE, "%s", api.why);
    Guard g(hp.device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", hp.device);
    rf->plan = plan;
    rf->device = hp.device;
    rf->n = n;
    rf->nnzA = int(hp.nnz);
    rf->nnzT = int(nnzT);
    int rc = PF_OK;
    if (!rc) rc = alloc_copy(&rf->ptrA, hp.rowptr.data(), hp.rowptr.size());
    if (!rc) rc = alloc_copy(&rf->indA, hp.colidx.data(), hp.colidx.size());
    if (!rc) rc = alloc_copy(&rf->ptrT, T_rowptr, size_t(n) + 1);
    if (!rc) rc = alloc_copy(&rf->indT, T_colidx, size_t(nnzT));
    if (!rc) rc = alloc_copy(&rf->valT, T_val, size_t(nnzT));
    if (!rc) rc = alloc_copy(&rf->pivP, pivP, size_t(n));
    if (!rc) rc = alloc_copy(&rf->pivQ, pivQ, size_t(n));
    if (!rc) rc = alloc_copy(&rf->J, Jval_host, size_t(hp.nnz));
    if (!rc) rc = alloc_copy<double>(&rf->F, nullptr, size_t(n));
    if (!rc) rc = alloc_copy<double>(&rf->dx, nullptr, size_t(n));
    if (!rc) rc = alloc_copy<double>(&rf->part, nullptr, kAbsBlocks);
    if (!rc) rc = alloc_copy<double>(&rf->norm, nullptr, 1);
    if (rc) return rc;
    LU_HIP(hipHostMalloc(&rf->norm_host, sizeof(double), hipHostMallocDefault));
    LU_HIP(hipMemset(rf->dx, 0, size_t(n) * sizeof(double)));
    LU_RS(api.create_handle(&rf->handle));
    LU_RS(api.create_rfinfo(&rf->info, rf->handle));
    LU_RS(api.analysis(rf->handle, n, 1, rf->nnzA, rf->ptrA, rf->indA, rf->J, rf->nnzT, rf->ptrT,
                       rf->indT, rf->valT, rf->pivP, rf->pivQ, rf->dx, n, rf->info));
    LU_HIP(hipDeviceSynchronize());
    return PF_OK;
}

}  // namespace

extern "C" {

int pf_refact_create(pf_plan *plan, const double *Jval_host, int64_t nnzT,
                     const int32_t *T_rowptr, const int32_t *T_colidx, const double *T_val,
                     const int32_t *pivP, const int32_t *pivQ, pf_refact **out) {
    clear_error();
    if (!out) return fail(PF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    const HostPlan &hp = plan->host;
    if (hp.kind == KIND_BATCH) return fail(PF_EINVAL, "pf_refact_create needs a non-batched plan");
    if (!Jval_host || !T_rowptr || !T_colidx || !T_val || !pivP || !pivQ)
        return fail(PF_EINVAL, "NULL argument");
    const int64_t n = hp.n;
    if (n < 1) return fail(PF_EINVAL, "the plan has no variables");
    if (n > INT32_MAX - 1 || hp.nnz > INT32_MAX) return fail(PF_EINVAL, "system too large");
    if (nnzT < n || nnzT > INT32_MAX) return fail(PF_EINVAL, "nnzT must be in [n, 2^31)");
    if (const char *why = check_T(int(n), nnzT, T_rowptr, T_colidx)) return fail(PF_EINVAL, "%s", why);
    if (!is_permutation(pivP, int(n)) || !is_permutation(pivQ, int(n)))
        return fail(PF_EINVAL, "pivP and pivQ must be permutations of 0..n-1");
    if (int e = check_closure(int(n), hp.rowptr.data(), hp.colidx.data(), pivP, pivQ, T_rowptr,
                              T_colidx))
        return e;
    if (hp.host_only || !plan->dev) return fail(PF_EINVAL, "plan is host-only");
    pf_refact *rf = new (std::nothrow) pf_refact();
    if (!rf) return fail(PF_ENOMEM, "host allocation failed");
    int rc = create(plan, Jval_host, nnzT, T_rowptr, T_colidx, T_val, pivP, pivQ, rf);
    if (rc) {
        release(rf);
        return rc;
    }
    rf->switch_safe = pivots_switch_safe(hp, pivP, pivQ);
    *out = rf;
    return PF_OK;
}

void pf_refact_destroy(pf_refact *rf) { release(rf); }

int pf_refact_solve(pf_refact *rf, const double *Jval, double *b, void *stream) {
    clear_error();
    if (!rf) return fail(PF_EINVAL, "refactorisation is NULL");
    if (!Jval || !b) return fail(PF_EINVAL, "Jval or b is NULL");
    Guard g(rf->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", rf->device);
    return solve_on_stream(rf, Jval, b, static_cast<hipStream_t>(stream));
}

int pf_newton_device(pf_plan *plan, pf_refact *rf, double *x, const pf_newton_opts *opts,
                     pf_newton_report *report, void *stream) {
    clear_error();
    if (!plan || !rf) return fail(PF_EINVAL, "plan or refactorisation is NULL");
    if (rf->plan != plan) return fail(PF_EINVAL, "the refactorisation belongs to another plan");
    if (!x) return fail(PF_EINVAL, "x is NULL");
    if (opts && opts->max_iter > 64) return fail(PF_EINVAL, "max_iter must be <= 64");
    HostPlan &hp = plan->host;
    const bool limits = opts && (opts->q_min || opts->q_max);
    const double check_below = (limits && opts->q_check_below > 0) ? opts->q_check_below : 1e-3;
    const double switch_tol = (limits && opts->q_switch_tol >= 0) ? opts->q_switch_tol : 1e-9;
    if (limits) {
        const int e = q_limits_valid(hp, opts->q_min, opts->q_max, switch_tol);
        if (e) return e;
        if (!rf->switch_safe)
            return fail(PF_EINVAL, "reactive limits need a refactorisation whose pivots survive a "
                        "switch (pf_jacobian_switch_order); this one's do not");
    }
    Guard g(rf->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", rf->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double tol = (opts && opts->tol > 0) ? opts->tol : 1e-10;
    const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 10;
    const int64_t n = hp.n;
    std::vector<double> xh(limits ? size_t(n) : 0);
    pf_newton_report r{};
    // events: per iteration [eval start, eval end, solve end]
    std::vector<hipEvent_t> ev(3 * size_t(max_iter + 1), nullptr);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) e = nullptr;
    auto t_start = std::chrono::steady_clock::now();
    int rc = PF_ENOCONV;
    int it = 0;
    for (;; ++it) {
        hipEvent_t *e = &ev[3 * size_t(it)];
        if (e[0]) (void)hipEventRecord(e[0], st);
        rc = dev_eval_single(hp, plan->dev, x, rf->F, rf->J, st);
        if (rc) break;
        if (e[1]) (void)hipEventRecord(e[1], st);
        rc = absmax_on_stream(rf, rf->F, st);
        if (rc) break;
        if (hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(PF_EDEVICE, "stream synchronisation failed in Newton iteration %d", it);
            break;
        }
        float ms = 0.f;
        if (e[0] && e[1] && hipEventElapsedTime(&ms, e[0], e[1]) == hipSuccess) r.t_eval_s += ms * 1e-3;
        double nf = *rf->norm_host;
        // the limits at this iterate (as pf_newton): after a switch F and J
        // are evaluated again under the new modes before the step (its time
        // counts as evaluation; the step's is measured from its end)
        int32_t ns = 0;
        if (limits && nf < check_below) {
            if (hipMemcpyAsync(xh.data(), x, size_t(n) * sizeof(double), hipMemcpyDeviceToHost,
                               st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = fail(PF_EDEVICE, "copy of the state failed in Newton iteration %d", it);
                break;
            }
            rc = q_switch(hp, plan->dev, xh.data(), opts->q_min, opts->q_max, switch_tol, &ns);
            if (!rc && ns) {
                if (e[0]) (void)hipEventRecord(e[0], st);
                rc = dev_eval_single(hp, plan->dev, x, rf->F, rf->J, st);
                if (!rc && e[1]) (void)hipEventRecord(e[1], st);
                if (!rc) rc = absmax_on_stream(rf, rf->F, st);
                if (!rc && hipStreamSynchronize(st) != hipSuccess)
                    rc = fail(PF_EDEVICE, "stream synchronisation failed in Newton iteration %d", it);
                if (!rc && e[0] && e[1] && hipEventElapsedTime(&ms, e[0], e[1]) == hipSuccess)
                    r.t_eval_s += ms * 1e-3;
                nf = *rf->norm_host;
            }
            if (rc) break;
        }
        r.norm[it] = nf;
        r.switched[it] = ns;
        r.n_switches += ns;
        if (nf < tol && ns == 0) {
            r.converged = 1;
            rc = PF_OK;
            break;
        }
        if (it >= max_iter) {
            rc = fail(PF_ENOCONV, "Newton did not converge in %d iterations (|F| = %g)", max_iter, nf);
            break;
        }
        if (hipMemcpyAsync(rf->dx, rf->F, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, st) !=
            hipSuccess) {
            rc = fail(PF_EDEVICE, "copy of F failed");
            break;
        }
        rc = solve_on_stream(rf, rf->J, rf->dx, st);
        if (rc) break;
        hipLaunchKernelGGL(k_step, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, n, x, rf->dx);
        if (hipGetLastError() != hipSuccess) {
            rc = fail(PF_EDEVICE, "Newton step launch failed");
            break;
        }
        if (e[2]) (void)hipEventRecord(e[2], st);
        r.iterations = it + 1;
    }
    if (hipStreamSynchronize(st) != hipSuccess && rc == PF_OK)
        rc = fail(PF_EDEVICE, "stream synchronisation failed");
    r.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    for (int k = 0; k < std::min(r.iterations, max_iter + 1); ++k) {
        hipEvent_t *e = &ev[3 * size_t(k)];
        float ms = 0.f;
        if (e[1] && e[2] && hipEventElapsedTime(&ms, e[1], e[2]) == hipSuccess) r.t_solve_s += ms * 1e-3;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (report) *report = r;
    return rc;
}

}  // extern "C"

// ===========================================================================
// Fast decoupled power flow, XB variant (Section V names the method as
// another user of the same residual evaluation).  The constant matrices
// B' (angle step, over the buses without a slack) and B'' (voltage step, over
// the buses without a voltage controller) are built here from the network
// data of the plan; each is factorised once (one host LU handed over as for
// pf_refact_create) and every iteration reuses the residual kernel:
//   F = F(x);  theta[B' buses] -= B'^-1 (F_p / V);
//   F = F(x);  V[B'' buses]    -= B''^-1 (F_q / V);
// until the stepped rows are below tol, then Q_g and P_s take the values that
// zero their buses' rows.
// ===========================================================================

struct pf_lu {
    int device = 0;
    int n = 0, nnzT = 0;
    int *indT = nullptr;
    double *valT = nullptr, *Y = nullptr;
    int *pivP = nullptr, *pivQ = nullptr;
    int *flev_ptr = nullptr, *blev_ptr = nullptr;
    int4 *frec = nullptr, *brec = nullptr;   // the rows' records in level order
    TriLevels tri;   // host copy of the level structure
};

struct pf_fdlf {
    pf_plan *plan = nullptr;
    pf_lu *bp = nullptr, *bpp = nullptr;
    int device = 0;
    int np = 0, nq = 0, ng = 0;
    int32_t *bus_p = nullptr, *bus_q = nullptr;  // row -> bus of B', B''
    int4 *gens = nullptr;                        // {bus, Q_g index, P_s index or -1, 0}
    double2 *setp = nullptr;                     // per generator (V_set, theta_set)
    double *F = nullptr, *rp = nullptr, *rq = nullptr, *part = nullptr, *norm = nullptr;
    double *norm_host = nullptr;
};

namespace {

// B' and B'' of a single-grid plan in CSR (columns sorted), with the bus of
// every row.  Entries are summed branch by branch in input order, then the
// bus shunts (B'' only).
struct FdMats {
    std::vector<int32_t> rp_p, ci_p, bus_p, rp_q, ci_q, bus_q;
    std::vector<double> v_p, v_q;
};

void csr_from_rows(std::vector<std::vector<std::pair<int32_t, double>>> &rows,
                   std::vector<int32_t> &rp, std::vector<int32_t> &ci, std::vector<double> &v) {
    rp.assign(1, 0);
    ci.clear();
    v.clear();
    for (auto &r : rows) {
        std::stable_sort(r.begin(), r.end(),
                         [](const std::pair<int32_t, double> &a,
                            const std::pair<int32_t, double> &b) { return a.first < b.first; });
        for (size_t k = 0; k < r.size();) {
            const int32_t c = r[k].first;
            double s = 0.0;
            for (; k < r.size() && r[k].first == c; ++k) s += r[k].second;
            ci.push_back(c);
            v.push_back(s);
        }
        rp.push_back(int32_t(ci.size()));
    }
}

int build_fd(const HostPlan &hp, FdMats &m) {
    if (hp.kind != KIND_SINGLE) return fail(PF_EINVAL, "the fast decoupled method needs a single-grid plan");
    const int N = hp.Nt;
    const int64_t B = hp.Bt;
    std::vector<int32_t> ip(size_t(N), -1), iq(size_t(N), -1);
    m.bus_p.clear();
    m.bus_q.clear();
    for (int i = 0; i < N; ++i) {
        const int g = hp.bus2[2 * size_t(i) + 1];
        const bool ctrl = g >= 0;
        const bool slack = ctrl && hp.gen4[4 * size_t(g) + 2] >= 0;
        if (!slack) {
            ip[size_t(i)] = int32_t(m.bus_p.size());
            m.bus_p.push_back(i);
        }
        if (!ctrl) {
            iq[size_t(i)] = int32_t(m.bus_q.size());
            m.bus_q.push_back(i);
        }
    }
    std::vector<std::vector<std::pair<int32_t, double>>> P(m.bus_p.size()), Q(m.bus_q.size());
    auto add = [](std::vector<std::vector<std::pair<int32_t, double>>> &D,
                  const std::vector<int32_t> &idx, int i, int j, double v) {
        const int32_t a = idx[size_t(i)], b = idx[size_t(j)];
        if (a >= 0 && b >= 0) D[size_t(a)].push_back({b, v});
    };
    for (int64_t e = 0; e < B; ++e) {
        if (!hp.br_on[size_t(e)]) continue;
        const int f = hp.br_f[size_t(e)], t = hp.br_t[size_t(e)];
        const double r = hp.params[size_t(e)], x = hp.params[size_t(B + e)];
        const double bc = hp.params[size_t(2 * B + e)], tap = hp.params[size_t(3 * B + e)];
        const double w = 1.0 / x;
        add(P, ip, f, f, w);
        add(P, ip, t, t, w);
        add(P, ip, f, t, -w);
        add(P, ip, t, f, -w);
        const double b = -x / (r * r + x * x);
        add(Q, iq, f, f, -(b + bc / 2) / (tap * tap));
        add(Q, iq, t, t, -(b + bc / 2));
        add(Q, iq, f, t, b / tap);
        add(Q, iq, t, f, b / tap);
    }
    for (int i = 0; i < N; ++i)
        for (int32_t k = hp.shptr[size_t(i)]; k < hp.shptr[size_t(i) + 1]; ++k)
            add(Q, iq, i, i, -hp.shunt_b[size_t(hp.shlist[size_t(k)])]);
    csr_from_rows(P, m.rp_p, m.ci_p, m.v_p);
    csr_from_rows(Q, m.rp_q, m.ci_q, m.v_q);
    return PF_OK;
}

void release_lu(pf_lu *lu) {
    if (!lu) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(lu->device);
    for (void *p : {(void *)lu->indT, (void *)lu->valT,
                    (void *)lu->Y, (void *)lu->pivP, (void *)lu->pivQ, (void *)lu->frec,
                    (void *)lu->brec, (void *)lu->flev_ptr, (void *)lu->blev_ptr})
        if (p) (void)hipFree(p);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete lu;
}

void release_fd(pf_fdlf *fd) {
    if (!fd) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(fd->device);
    for (void *p : {(void *)fd->bus_p, (void *)fd->bus_q, (void *)fd->gens, (void *)fd->setp, (void *)fd->F,
                    (void *)fd->rp, (void *)fd->rq, (void *)fd->part, (void *)fd->norm})
        if (p) (void)hipFree(p);
    if (fd->norm_host) (void)hipHostFree(fd->norm_host);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete fd;
}

const char *check_csr(int n, int64_t nnz, const int32_t *rp, const int32_t *ci) {
    if (rp[0] != 0 || rp[n] != nnz) return "rowptr must start at 0 and end at nnz";
    for (int i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return "rowptr is not non-decreasing";
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] < 0 || ci[k] >= n) return "column index out of range";
            if (k > rp[i] && ci[k] <= ci[k - 1]) return "columns not strictly increasing in a row";
        }
    }
    return nullptr;
}

// The factors are the host LU's own: T's values are uploaded as given and
// every solve runs this library's level-scheduled kernels along them (the
// matrix M itself is only checked).
int create_lu(int device, int n, const int32_t *T_rowptr, const int32_t *T_colidx,
              const double *T_val, const int32_t *pivP, const int32_t *pivQ, pf_lu *lu) {
    Guard g(device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", device);
    lu->device = device;
    lu->n = n;
    lu->nnzT = T_rowptr[n];
    try {
        tri_levels(n, T_rowptr, T_colidx, lu->tri);
        tri_records(T_rowptr, pivP, lu->tri);
    } catch (const std::bad_alloc &) {
        return fail(PF_ENOMEM, "host allocation failed");
    }
    const TriLevels &t = lu->tri;
    int rc = PF_OK;
    if (!rc) rc = alloc_copy(&lu->indT, T_colidx, size_t(lu->nnzT));
    if (!rc) rc = alloc_copy(&lu->valT, T_val, size_t(lu->nnzT));
    if (!rc) rc = alloc_copy(&lu->pivP, pivP, size_t(n));
    if (!rc) rc = alloc_copy(&lu->pivQ, pivQ, size_t(n));
    if (!rc) rc = alloc_copy(&lu->frec, t.frec.data(), t.frec.size());
    if (!rc) rc = alloc_copy(&lu->brec, t.brec.data(), t.brec.size());
    if (!rc) rc = alloc_copy(&lu->flev_ptr, t.flev_ptr.data(), t.flev_ptr.size());
    if (!rc) rc = alloc_copy(&lu->blev_ptr, t.blev_ptr.data(), t.blev_ptr.size());
    if (!rc) rc = alloc_copy(&lu->Y, static_cast<const double *>(nullptr), size_t(n));
    return rc;
}

// X[pivQ[k]] = Y[k]
__global__ void __launch_bounds__(256) k_lu_unpermute(int n, const int32_t *__restrict__ pivQ,
                                                      const double *__restrict__ Y,
                                                      double *__restrict__ X) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) X[pivQ[k]] = Y[k];
}

// Solve with the permuted working vector Y (n doubles, written in full by
// the forward solve before anything reads it).
int lu_solve_in(pf_lu *lu, double *b, double *Y, hipStream_t st) {
    const TriDev d{lu->flev_ptr, lu->blev_ptr, lu->frec, lu->brec, lu->indT, lu->valT};
    tri_solve(lu->tri, d, b, Y, st);
    hipLaunchKernelGGL(k_lu_unpermute, dim3(unsigned((lu->n + 255) / 256)), dim3(256), 0, st,
                       lu->n, lu->pivQ, Y, b);
    LU_HIP(hipGetLastError());
    return PF_OK;
}

int lu_solve(pf_lu *lu, double *b, hipStream_t st) { return lu_solve_in(lu, b, lu->Y, st); }

// ---------------------------------------------------------------------------
// Working vector of pf_lu_solve_noalloc: a static device array, one copy per
// device, held until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress returns on each device (the array's name is a
// host-side stand-in there).
// ---------------------------------------------------------------------------
constexpr int64_t kStaticScratchDoubles = int64_t(1) << 20;   // 8 MiB
static __device__ __align__(256) double scratch[kStaticScratchDoubles];
constexpr int kMaxScratchDevices = 64;

// The array's address on `device`, which must be current; looked up once per
// device.
int static_scratch(int device, double **out) {
    static std::mutex mu;
    static double *addr[kMaxScratchDevices] = {};
    if (device < 0 || device >= kMaxScratchDevices)
        return fail(PF_EINVAL, "device %d is out of range for the static scratch", device);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PF_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                        hipGetErrorString(e));
        addr[device] = static_cast<double *>(p);
    }
    *out = addr[device];
    return PF_OK;
}

// rhs[r] = F[bus[r]] / V[bus[r]] (when rhs is not NULL); part[block] = max |F[bus]|
__global__ void __launch_bounds__(256) k_fd_gather(int m, const int32_t *__restrict__ bus,
                                                   const double *__restrict__ Fpart,
                                                   const double *__restrict__ V,
                                                   double *__restrict__ rhs,
                                                   double *__restrict__ part) {
    __shared__ double red[256];
    double mx = 0.0;
    for (int r = blockIdx.x * 256 + threadIdx.x; r < m; r += gridDim.x * 256) {
        const int i = bus[r];
        const double f = Fpart[i];
        if (rhs) rhs[r] = f / V[i];
        mx = absmax2(mx, fabs(f));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) red[threadIdx.x] = absmax2(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// xpart[bus[r]] -= d[r]
__global__ void __launch_bounds__(256) k_fd_scatter(int m, const int32_t *__restrict__ bus,
                                                    double *__restrict__ xpart,
                                                    const double *__restrict__ d) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < m) xpart[bus[r]] -= d[r];
}

// generator variables that zero their buses' rows: Q_g += F_q[bus], P_s += F_p[bus]
__global__ void __launch_bounds__(256) k_fd_gens(int ng, int N, const int4 *__restrict__ gens,
                                                 const double *__restrict__ F,
                                                 double *__restrict__ x) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= ng) return;
    const int4 q = gens[g];
    x[q.y] += F[N + q.x];
    if (q.z >= 0) x[q.z] += F[q.x];
}

// the method never steps controlled voltages or slack angles: put them at
// their set points
__global__ void __launch_bounds__(256) k_fd_init(int ng, int N, const int4 *__restrict__ gens,
                                                 const double2 *__restrict__ setp,
                                                 double *__restrict__ x) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= ng) return;
    const int4 q = gens[g];
    x[N + q.x] = setp[g].x;
    if (q.z >= 0) x[q.x] = setp[g].y;
}

int fd_blocks(int m) { return std::max(1, std::min(kAbsBlocks, (m + 255) / 256)); }

}  // namespace

namespace {

// Symbolic LU without pivoting of B = P M Q (row k of B is row pivP[k] of M,
// column k is column pivQ[k]): row by row, the pattern of row r is that of
// B's row r united with the upper part of every earlier row k it reaches
// (k < r in the pattern, in increasing k, including entries that this union
// itself adds).  The result holds every entry an elimination along it can
// touch, whatever the values.
int symbolic(int n, const int32_t *rp, const int32_t *ci, const int32_t *pivP,
             const int32_t *pivQ, std::vector<int32_t> &trp, std::vector<int32_t> &tci) {
    std::vector<int32_t> qinv(static_cast<size_t>(n));
    for (int k = 0; k < n; ++k) qinv[size_t(pivQ[k])] = k;
    std::vector<int32_t> mark(size_t(n), -1);
    std::vector<int32_t> udiag(size_t(n), 0);  // start of row k's upper part in tci
    std::vector<int32_t> row, heap;
    trp.assign(1, 0);
    tci.clear();
    for (int r = 0; r < n; ++r) {
        row.clear();
        heap.clear();
        auto add = [&](int32_t c) {
            if (mark[size_t(c)] == r) return;
            mark[size_t(c)] = r;
            row.push_back(c);
            if (c < r) {
                heap.push_back(c);
                std::push_heap(heap.begin(), heap.end(), std::greater<int32_t>());
            }
        };
        const int32_t m = pivP[r];
        for (int32_t e = rp[m]; e < rp[m + 1]; ++e) add(qinv[size_t(ci[e])]);
        add(r);
        while (!heap.empty()) {
            std::pop_heap(heap.begin(), heap.end(), std::greater<int32_t>());
            const int32_t k = heap.back();
            heap.pop_back();
            for (int32_t f = udiag[size_t(k)]; f < trp[size_t(k) + 1]; ++f) add(tci[size_t(f)]);
        }
        std::sort(row.begin(), row.end());
        const size_t base = tci.size();
        if (base + row.size() > size_t(INT32_MAX)) return fail(PF_EINVAL, "LU pattern too large");
        tci.insert(tci.end(), row.begin(), row.end());
        trp.push_back(int32_t(tci.size()));
        const auto d = std::upper_bound(row.begin(), row.end(), r);   // first entry past the diagonal
        udiag[size_t(r)] = int32_t(base + size_t(d - row.begin()));
    }
    return PF_OK;
}

}  // namespace

extern "C" {

int pf_lu_symbolic(int64_t n, const int32_t *rowptr, const int32_t *colidx, const int32_t *pivP,
                   const int32_t *pivQ, int64_t *nnzT, int32_t *T_rowptr, int32_t *T_colidx) {
    clear_error();
    if (!rowptr || !colidx || !pivP || !pivQ || !nnzT) return fail(PF_EINVAL, "NULL argument");
    if (n < 1 || n > INT32_MAX - 1) return fail(PF_EINVAL, "n must be in [1, 2^31 - 1)");
    if (const char *why = check_csr(int(n), rowptr[n], rowptr, colidx))
        return fail(PF_EINVAL, "matrix: %s", why);
    if (!is_permutation(pivP, int(n)) || !is_permutation(pivQ, int(n)))
        return fail(PF_EINVAL, "pivP and pivQ must be permutations of 0..n-1");
    std::vector<int32_t> trp, tci;
    int rc;
    try {
        rc = symbolic(int(n), rowptr, colidx, pivP, pivQ, trp, tci);
    } catch (const std::bad_alloc &) {
        rc = fail(PF_ENOMEM, "host allocation failed");
    }
    if (rc) return rc;
    *nnzT = int64_t(tci.size());
    if (T_rowptr) std::memcpy(T_rowptr, trp.data(), trp.size() * sizeof(int32_t));
    if (T_colidx) std::memcpy(T_colidx, tci.data(), tci.size() * sizeof(int32_t));
    return PF_OK;
}

// The matrices are built on the host from the plan's parameters; after
// pf_set_params the host copy is refreshed from the device first.
static int fresh_params(const pf_plan *plan) {
    if (!plan->host.params_stale || !plan->dev) return PF_OK;
    pf_plan *p = const_cast<pf_plan *>(plan);
    return dev_fetch_params(p->host, p->dev);
}

int pf_fdlf_matrices(const pf_plan *plan, int64_t *nnz_bp, int32_t *bp_rowptr,
                     int32_t *bp_colidx, double *bp_val, int32_t *bp_bus, int64_t *nnz_bpp,
                     int32_t *bpp_rowptr, int32_t *bpp_colidx, double *bpp_val,
                     int32_t *bpp_bus) {
    clear_error();
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    FdMats m;
    int rc = fresh_params(plan);
    if (rc) return rc;
    try {
        rc = build_fd(plan->host, m);
    } catch (const std::bad_alloc &) {
        rc = fail(PF_ENOMEM, "host allocation failed");
    }
    if (rc) return rc;
    if (nnz_bp) *nnz_bp = int64_t(m.ci_p.size());
    if (nnz_bpp) *nnz_bpp = int64_t(m.ci_q.size());
    auto put = [](auto *dst, const auto &src) {
        if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(src[0]));
    };
    put(bp_rowptr, m.rp_p);
    put(bp_colidx, m.ci_p);
    put(bp_val, m.v_p);
    put(bp_bus, m.bus_p);
    put(bpp_rowptr, m.rp_q);
    put(bpp_colidx, m.ci_q);
    put(bpp_val, m.v_q);
    put(bpp_bus, m.bus_q);
    return PF_OK;
}

int pf_lu_create(int32_t device, int64_t n, int64_t nnz, const int32_t *rowptr,
                 const int32_t *colidx, const double *val, int64_t nnzT, const int32_t *T_rowptr,
                 const int32_t *T_colidx, const double *T_val, const int32_t *pivP,
                 const int32_t *pivQ, pf_lu **out) {
    clear_error();
    if (!out) return fail(PF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!rowptr || !colidx || !val || !T_rowptr || !T_colidx || !T_val || !pivP || !pivQ)
        return fail(PF_EINVAL, "NULL argument");
    if (n < 1 || n > INT32_MAX - 1) return fail(PF_EINVAL, "n must be in [1, 2^31 - 1)");
    if (nnz < 0 || nnz > INT32_MAX || nnzT < n || nnzT > INT32_MAX)
        return fail(PF_EINVAL, "nnz must be in [0, 2^31), nnzT in [n, 2^31)");
    if (const char *why = check_csr(int(n), nnz, rowptr, colidx))
        return fail(PF_EINVAL, "matrix: %s", why);
    if (const char *why = check_T(int(n), nnzT, T_rowptr, T_colidx)) return fail(PF_EINVAL, "%s", why);
    if (!is_permutation(pivP, int(n)) || !is_permutation(pivQ, int(n)))
        return fail(PF_EINVAL, "pivP and pivQ must be permutations of 0..n-1");
    if (int e = check_closure(int(n), rowptr, colidx, pivP, pivQ, T_rowptr, T_colidx)) return e;
    int dev = device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return fail(PF_EDEVICE, "no current device");
    pf_lu *lu = new (std::nothrow) pf_lu();
    if (!lu) return fail(PF_ENOMEM, "host allocation failed");
    int rc = create_lu(dev, int(n), T_rowptr, T_colidx, T_val, pivP, pivQ, lu);
    if (rc) {
        release_lu(lu);
        return rc;
    }
    *out = lu;
    return PF_OK;
}

int pf_lu_solve(pf_lu *lu, double *b, void *stream) {
    clear_error();
    if (!lu || !b) return fail(PF_EINVAL, "NULL argument");
    Guard g(lu->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", lu->device);
    return lu_solve(lu, b, static_cast<hipStream_t>(stream));
}

int pf_lu_solve_noalloc(pf_lu *lu, double *b, void *stream) {
    clear_error();
    if (!lu || !b) return fail(PF_EINVAL, "NULL argument");
    if (int64_t(lu->n) > kStaticScratchDoubles)
        return fail(PF_EINVAL, "n = %d exceeds the static scratch of %lld doubles", lu->n,
                    (long long)kStaticScratchDoubles);
    Guard g(lu->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", lu->device);
    double *Y = nullptr;
    const int rc = static_scratch(lu->device, &Y);
    if (rc) return rc;
    return lu_solve_in(lu, b, Y, static_cast<hipStream_t>(stream));
}

void pf_lu_destroy(pf_lu *lu) { release_lu(lu); }

int pf_fdlf_create(pf_plan *plan, pf_lu *bp, pf_lu *bpp, pf_fdlf **out) {
    clear_error();
    if (!out) return fail(PF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plan) return fail(PF_EINVAL, "plan is NULL");
    const HostPlan &hp = plan->host;
    if (hp.host_only || !plan->dev) return fail(PF_EINVAL, "plan is host-only");
    FdMats m;
    int rc = fresh_params(plan);
    if (!rc) rc = build_fd(hp, m);
    if (rc) return rc;
    const int np = int(m.bus_p.size()), nq = int(m.bus_q.size());
    if ((np > 0) != (bp != nullptr) || (nq > 0) != (bpp != nullptr))
        return fail(PF_EINVAL, "give a factorisation exactly for each non-empty matrix");
    if ((bp && bp->n != np) || (bpp && bpp->n != nq))
        return fail(PF_EINVAL, "factorisation size does not match B' (%d) / B'' (%d)", np, nq);
    if ((bp && bp->device != hp.device) || (bpp && bpp->device != hp.device))
        return fail(PF_EINVAL, "factorisations live on another device than the plan");
    pf_fdlf *fd = new (std::nothrow) pf_fdlf();
    if (!fd) return fail(PF_ENOMEM, "host allocation failed");
    fd->plan = plan;
    fd->bp = bp;
    fd->bpp = bpp;
    fd->device = hp.device;
    fd->np = np;
    fd->nq = nq;
    std::vector<int4> gens;
    std::vector<double2> setp;
    for (int i = 0; i < hp.Nt; ++i) {
        const int g = hp.bus2[2 * size_t(i) + 1];
        if (g < 0) continue;
        const int32_t ps = hp.gen4[4 * size_t(g) + 2];
        gens.push_back(make_int4(i, hp.gen4[4 * size_t(g)], ps >= 0 ? ps : -1, 0));
        const int32_t pv = hp.genpv[size_t(g)];
        setp.push_back(make_double2(pv >= 0 ? hp.pv_vset[size_t(pv)] : hp.gen2[2 * size_t(g)],
                                    hp.gen2[2 * size_t(g) + 1]));
    }
    fd->ng = int(gens.size());
    {
        Guard g(hp.device);
        if (!g.ok) rc = fail(PF_EDEVICE, "cannot select device %d", hp.device);
        if (!rc) rc = alloc_copy(&fd->bus_p, m.bus_p.data(), m.bus_p.size());
        if (!rc) rc = alloc_copy(&fd->bus_q, m.bus_q.data(), m.bus_q.size());
        if (!rc) rc = alloc_copy(&fd->gens, gens.data(), gens.size());
        if (!rc) rc = alloc_copy(&fd->setp, setp.data(), setp.size());
        if (!rc) rc = alloc_copy<double>(&fd->F, nullptr, size_t(hp.n));
        if (!rc) rc = alloc_copy<double>(&fd->rp, nullptr, size_t(np));
        if (!rc) rc = alloc_copy<double>(&fd->rq, nullptr, size_t(nq));
        if (!rc) rc = alloc_copy<double>(&fd->part, nullptr, 2 * kAbsBlocks);
        if (!rc) rc = alloc_copy<double>(&fd->norm, nullptr, 1);
        if (!rc && hipHostMalloc(&fd->norm_host, sizeof(double), hipHostMallocDefault) != hipSuccess)
            rc = fail(PF_ENOMEM, "pinned allocation failed");
    }
    if (rc) {
        release_fd(fd);
        return rc;
    }
    *out = fd;
    return PF_OK;
}

void pf_fdlf_destroy(pf_fdlf *fd) { release_fd(fd); }

int pf_fdlf_solve(pf_fdlf *fd, double *x, const pf_newton_opts *opts, pf_newton_report *report,
                  void *stream) {
    clear_error();
    if (!fd || !x) return fail(PF_EINVAL, "NULL argument");
    if (opts && opts->max_iter > 64) return fail(PF_EINVAL, "max_iter must be <= 64");
    if (opts && (opts->q_min || opts->q_max))
        return fail(PF_EINVAL, "reactive limits are checked inside the iterations by the Newton "
                    "solvers only: the constant B' and B'' cannot follow a switch");
    HostPlan &hp = fd->plan->host;
    for (int32_t k = 0; k < hp.NPVt; ++k)
        if (!hp.pv_mode.empty() && hp.pv_mode[size_t(k)])
            return fail(PF_EINVAL, "the fast decoupled method needs every PV unit under voltage control");
    Guard g(fd->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", fd->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double tol = (opts && opts->tol > 0) ? opts->tol : 1e-10;
    const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 10;
    const int N = hp.Nt;
    const int bp_blocks = fd_blocks(fd->np), bq_blocks = fd_blocks(fd->nq);
    pf_newton_report r{};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float ms = 0.f;
    auto t_start = std::chrono::steady_clock::now();
    auto eval = [&]() -> int {
        if (e0) (void)hipEventRecord(e0, st);
        int rc = dev_eval_single(hp, fd->plan->dev, x, fd->F, nullptr, st);
        if (e1) (void)hipEventRecord(e1, st);
        return rc;
    };
    auto eval_time = [&]() {
        if (e0 && e1 && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            r.t_eval_s += ms * 1e-3;
    };
    int rc = PF_OK;
    int it = 0;
    if (fd->ng) {
        hipLaunchKernelGGL(k_fd_init, dim3((fd->ng + 255) / 256), dim3(256), 0, st, fd->ng, N,
                           fd->gens, fd->setp, x);
        if (hipGetLastError() != hipSuccess) rc = fail(PF_EDEVICE, "launch failed");
    }
    bool stepped_ok = false;
    for (; !rc; ++it) {
        rc = eval();
        if (rc) break;
        // mismatch of the stepped rows, and the angle-step right-hand side
        if (fd->np)
            hipLaunchKernelGGL(k_fd_gather, dim3(bp_blocks), dim3(256), 0, st, fd->np, fd->bus_p,
                               fd->F, x + N, fd->rp, fd->part);
        if (fd->nq)
            hipLaunchKernelGGL(k_fd_gather, dim3(bq_blocks), dim3(256), 0, st, fd->nq, fd->bus_q,
                               fd->F + N, x + N, nullptr, fd->part + bp_blocks);
        hipLaunchKernelGGL(k_absmax_fold, dim3(1), dim3(256), 0, st,
                           (fd->np ? bp_blocks : 0) + (fd->nq ? bq_blocks : 0),
                           fd->np ? fd->part : fd->part + bp_blocks, fd->norm);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(fd->norm_host, fd->norm, sizeof(double), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(PF_EDEVICE, "device step failed in iteration %d", it);
            break;
        }
        eval_time();
        const double nf = *fd->norm_host;
        if (it < 65) r.norm[it] = nf;
        if (nf < tol) {
            stepped_ok = true;
            break;
        }
        if (it >= max_iter) {
            rc = fail(PF_ENOCONV, "fast decoupled iteration did not converge in %d iterations (%g)",
                      max_iter, nf);
            break;
        }
        auto ts = std::chrono::steady_clock::now();
        if (fd->np) {
            rc = lu_solve(fd->bp, fd->rp, st);
            if (rc) break;
            hipLaunchKernelGGL(k_fd_scatter, dim3((fd->np + 255) / 256), dim3(256), 0, st, fd->np,
                               fd->bus_p, x, fd->rp);
        }
        rc = eval();
        if (rc) break;
        if (fd->nq) {
            hipLaunchKernelGGL(k_fd_gather, dim3(bq_blocks), dim3(256), 0, st, fd->nq, fd->bus_q,
                               fd->F + N, x + N, fd->rq, fd->part);
            rc = lu_solve(fd->bpp, fd->rq, st);
            if (rc) break;
            hipLaunchKernelGGL(k_fd_scatter, dim3((fd->nq + 255) / 256), dim3(256), 0, st, fd->nq,
                               fd->bus_q, x + N, fd->rq);
        }
        if (hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(PF_EDEVICE, "device step failed in iteration %d", it);
            break;
        }
        eval_time();
        r.t_solve_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count();
        r.iterations = it + 1;
    }
    if (rc == PF_OK && stepped_ok) {
        // generator variables, then the full norm of F
        rc = eval();
        if (!rc && fd->ng)
            hipLaunchKernelGGL(k_fd_gens, dim3((fd->ng + 255) / 256), dim3(256), 0, st, fd->ng, N,
                               fd->gens, fd->F, x);
        if (!rc) rc = eval();
        if (!rc) {
            const int nb = fd_blocks(int(hp.n));
            hipLaunchKernelGGL(k_absmax_part, dim3(nb), dim3(256), 0, st, hp.n, fd->F, fd->part);
            hipLaunchKernelGGL(k_absmax_fold, dim3(1), dim3(256), 0, st, nb, fd->part, fd->norm);
            if (hipMemcpyAsync(fd->norm_host, fd->norm, sizeof(double), hipMemcpyDeviceToHost,
                               st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = fail(PF_EDEVICE, "final norm failed");
        }
        if (!rc) {
            r.norm[std::min(it + 1, 64)] = *fd->norm_host;
            r.converged = *fd->norm_host < tol;
            if (!r.converged)
                rc = fail(PF_ENOCONV, "generator rows did not close (|F| = %g)", *fd->norm_host);
        }
    }
    (void)hipStreamSynchronize(st);
    r.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (report) *report = r;
    return rc;
}

}  // extern "C"
