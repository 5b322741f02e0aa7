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
#include <mutex>
#include <new>
#include <vector>

#include <hip/hip_runtime.h>
#include <rocsolver/rocsolver.h>

#include "pf_internal.hpp"

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
    if (hp.host_only || !plan->dev) return fail(PF_EINVAL, "plan is host-only");
    pf_refact *rf = new (std::nothrow) pf_refact();
    if (!rf) return fail(PF_ENOMEM, "host allocation failed");
    int rc = create(plan, Jval_host, nnzT, T_rowptr, T_colidx, T_val, pivP, pivQ, rf);
    if (rc) {
        release(rf);
        return rc;
    }
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
    Guard g(rf->device);
    if (!g.ok) return fail(PF_EDEVICE, "cannot select device %d", rf->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double tol = (opts && opts->tol > 0) ? opts->tol : 1e-10;
    const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 10;
    const int64_t n = hp.n;
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
        const double nf = *rf->norm_host;
        r.norm[it] = nf;
        if (nf < tol) {
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
    for (int k = 0; k <= std::min(it, max_iter); ++k) {
        hipEvent_t *e = &ev[3 * size_t(k)];
        float ms = 0.f;
        if (e[0] && e[1] && hipEventElapsedTime(&ms, e[0], e[1]) == hipSuccess) r.t_eval_s += ms * 1e-3;
        if (k < r.iterations && e[1] && e[2] && hipEventElapsedTime(&ms, e[1], e[2]) == hipSuccess)
            r.t_solve_s += ms * 1e-3;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (report) *report = r;
    return rc;
}

}  // extern "C"
