// Debug-mode non-finite scan of the single-trajectory entry points (host).
#pragma once
#include <stdint.h>

#include "../../include/cis.h"

namespace cis {

constexpr int kDebugMaxArrays = 16;

// One array of an entry point: the [rows][cols] block of a [rows][ld] array.
struct DebugArr {
    const char* name;
    const void* p;   // NULL: not given, skipped
    int64_t rows, cols, ld;
    bool output;
};

// CIS_DEBUG_FINITE set (non-empty, not "0")
bool debug_finite_enabled();

// Counts the non-finite values of n <= kDebugMaxArrays arrays on `stream`,
// synchronizes it, and returns CIS_ERR_NONFINITE (naming every array with
// its count) if any was found.
cis_status debug_scan(const char* call, int32_t dtype, void* stream, const DebugArr* arr, int n);

// The inputs and outputs of a discretize-type call with nx augmented states
// and nu controls (err: the RKF estimate [N], or NULL).
cis_status debug_scan_forward(const char* call, const cis_model* m, const cis_shape* sh,
                              int32_t nx, int32_t nu, const void* X, const void* U,
                              const void* s, const void* params, const void* A, const void* Bm,
                              const void* Bp, const void* S, const void* defect,
                              const void* xprop, const void* err, void* stream);

}  // namespace cis
