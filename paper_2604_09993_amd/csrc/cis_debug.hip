// Debug mode of the single-trajectory entry points: with the environment
// variable CIS_DEBUG_FINITE set (non-empty, not "0"), a call that launched
// successfully then counts the non-finite values of each of its inputs and
// outputs, synchronizes its stream and returns CIS_ERR_NONFINITE naming every
// array that holds one.  Not a hot path: it allocates a small counter array,
// copies it back and frees it.  Without the variable nothing is checked and
// non-finite values propagate through the arithmetic like any others.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../include/cis.h"
#include "cis_debug.hpp"
#include "cis_host.hpp"

namespace cis {

bool debug_finite_enabled() {
    const char* v = std::getenv("CIS_DEBUG_FINITE");
    return v && *v && std::strcmp(v, "0") != 0;
}

namespace {

// Non-finite elements of the [rows][cols] block of a [rows][ld] array.
template <class T>
__global__ void __launch_bounds__(256) k_count_nonfinite(const T* __restrict__ p, int64_t rows,
                                                         int64_t cols, int64_t ld,
                                                         unsigned long long* cnt) {
    const int64_t n = rows * cols;
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / cols;
        if (!__builtin_isfinite(p[r * ld + (i - r * cols)])) ++c;
    }
    if (c) atomicAdd(cnt, c);
}

}  // namespace

cis_status debug_scan(const char* call, int32_t dtype, void* stream, const DebugArr* arr, int n) {
    if (n < 1 || n > kDebugMaxArrays) return fail(CIS_ERR_DIM, "%s: debug scan of %d arrays", call, n);
    hipStream_t hs = (hipStream_t)stream;
    unsigned long long* d = nullptr;
    if (hipMalloc(&d, n * sizeof(unsigned long long)) != hipSuccess)
        return fail(CIS_ERR_HIP, "%s: debug scan: counter allocation failed", call);
    cis_status st = CIS_OK;
    if (hipMemsetAsync(d, 0, n * sizeof(unsigned long long), hs) != hipSuccess)
        st = fail(CIS_ERR_HIP, "%s: debug scan: counter clear failed", call);
    for (int i = 0; i < n && st == CIS_OK; ++i) {
        const DebugArr& a = arr[i];
        const int64_t total = a.rows * a.cols;
        if (!a.p || total <= 0) continue;
        const int64_t blocks = (total + 255) / 256;
        const dim3 grid((unsigned)(blocks < 1024 ? blocks : 1024));
        if (dtype == CIS_F32)
            hipLaunchKernelGGL(k_count_nonfinite<float>, grid, dim3(256), 0, hs,
                               (const float*)a.p, a.rows, a.cols, a.ld, d + i);
        else
            hipLaunchKernelGGL(k_count_nonfinite<double>, grid, dim3(256), 0, hs,
                               (const double*)a.p, a.rows, a.cols, a.ld, d + i);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            st = fail(CIS_ERR_HIP, "%s: debug scan launch: %s", call, hipGetErrorString(e));
    }
    unsigned long long h[kDebugMaxArrays] = {};
    if (st == CIS_OK &&
        (hipMemcpyAsync(h, d, n * sizeof(unsigned long long), hipMemcpyDeviceToHost, hs) !=
             hipSuccess ||
         hipStreamSynchronize(hs) != hipSuccess))
        st = fail(CIS_ERR_HIP, "%s: debug scan: copy back failed", call);
    (void)hipFree(d);
    if (st != CIS_OK) return st;
    std::string msg;
    for (int i = 0; i < n; ++i) {
        if (!h[i]) continue;
        char part[96];
        std::snprintf(part, sizeof(part), "%s%s %s %llu", msg.empty() ? "" : ", ",
                      arr[i].output ? "output" : "input", arr[i].name, h[i]);
        msg += part;
    }
    if (msg.empty()) return CIS_OK;
    return fail(CIS_ERR_NONFINITE, "%s: non-finite values: %s", call, msg.c_str());
}

cis_status debug_scan_forward(const char* call, const cis_model* m, const cis_shape* sh,
                              int32_t nx, int32_t nu, const void* X, const void* U,
                              const void* s, const void* params, const void* A, const void* Bm,
                              const void* Bp, const void* S, const void* defect,
                              const void* xprop, const void* err, void* stream) {
    const int64_t N = sh->N, ln = sh->ld_node, li = sh->ld_int;
    const DebugArr arr[] = {
        {"X", X, nx, N + 1, ln, false},      {"U", U, nu, N + 1, ln, false},
        {"s", s, 1, N, N, false},            {"params", params, 1, m->np, m->np, false},
        {"A", A, (int64_t)nx * nx, N, li, true},
        {"Bm", Bm, (int64_t)nx * nu, N, li, true},
        {"Bp", Bp, (int64_t)nx * nu, N, li, true},
        {"S", S, nx, N, li, true},           {"defect", defect, nx, N, li, true},
        {"xprop", xprop, nx, N, li, true},   {"err", err, 1, N, N, true},
    };
    return debug_scan(call, sh->dtype, stream, arr, (int)(sizeof(arr) / sizeof(arr[0])));
}

}  // namespace cis
