// Host-side model object and argument validation shared by the kernel files.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cis.h"

// Compiled (legs, depth) topologies; see cis.h.
#define CIS_TOPOLOGIES(X) X(0, 0) X(1, 0) X(1, 1) X(1, 2) X(2, 1) X(2, 2) X(2, 3) X(4, 3)

struct cis_model {
    int32_t nb, nj, nc;   // bodies, joints, contacts
    int32_t L, D;         // legs, links per leg
    int32_t n, ny, nx, m, np;
    std::vector<double> len, rp, rc, ks, ds, cr;
    double g, A, kappa;
};

namespace cis {

// Record the failure text for cis_last_error() and return st.
cis_status fail(cis_status st, const char* fmt, ...);

inline size_t elem_size(int32_t dtype) { return dtype == CIS_F32 ? 4 : 8; }
inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Checks shared by every entry point: model, shape, and the input pointers.
cis_status check_common(const cis_model* m, const cis_shape* sh, const void* X, const void* U,
                        const void* s, const void* params);

// Tuning cache (CIS_TUNE_CACHE): choices per key, -1 where not made; the file
// is read and rewritten under g_cache_mu.
struct TuneChoice {
    int split = -1, waves = -1, persist = -1, def_lane = -1, adj_waves = -1;
    int blocks = -1, compose = -1, form = -1, layout = -1;
};
extern std::mutex g_cache_mu;
std::map<std::string, TuneChoice> cache_read(const std::string& path);
bool cache_write(const std::string& path, const std::map<std::string, TuneChoice>& m);
// "<architecture>/<compute units>cu" of a device
std::string device_tag(int dev);

}  // namespace cis
