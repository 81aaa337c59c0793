// A prepared kernel launch: function, grid and a private copy of the argument
// values.  The same record is launched eagerly on a stream or added to a HIP
// graph as a kernel node (whose parameters HIP copies when the node is added).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstring>

#include "../../include/cis.h"
#include "cis_host.hpp"

namespace cis {

struct KLaunch {
    static constexpr int MAX_ARGS = 8;
    static constexpr size_t BUF = 4096;
    const void* func = nullptr;
    dim3 grid{1, 1, 1}, block{1, 1, 1};
    int nargs = 0;
    size_t off[MAX_ARGS] = {};
    size_t end = 0;
    alignas(16) unsigned char buf[BUF];

    template <class A>
    void arg(const A& v) {
        const size_t al = alignof(A) < 16 ? alignof(A) : 16;
        const size_t o = (end + al - 1) / al * al;
        if (nargs >= MAX_ARGS || o + sizeof(A) > BUF) {
            func = nullptr;   // refused in launch()/node()
            return;
        }
        std::memcpy(buf + o, &v, sizeof(A));
        off[nargs++] = o;
        end = o + sizeof(A);
    }
    bool ok() const { return func != nullptr && grid.x > 0 && grid.y > 0 && grid.z > 0; }
    void pointers(void** a) { for (int i = 0; i < nargs; ++i) a[i] = buf + off[i]; }

    hipError_t launch(hipStream_t s) {
        if (!ok()) return hipErrorInvalidValue;
        void* a[MAX_ARGS];
        pointers(a);
        return hipLaunchKernel(func, grid, block, a, 0, s);
    }
    // Adds this launch to `g` after the `ndep` nodes in `deps`.
    hipError_t node(hipGraph_t g, const hipGraphNode_t* deps, size_t ndep, hipGraphNode_t* out) {
        if (!ok()) return hipErrorInvalidValue;
        void* a[MAX_ARGS];
        pointers(a);
        hipKernelNodeParams p;
        std::memset(&p, 0, sizeof(p));
        p.func = const_cast<void*>(func);
        p.gridDim = grid;
        p.blockDim = block;
        p.sharedMemBytes = 0;
        p.kernelParams = a;
        p.extra = nullptr;
        return hipGraphAddKernelNode(out, g, deps, ndep, &p);
    }
};

// One model's slice of a batch as the kernels see it (device pointers).
struct BatchGroupDev {
    const void* fdesc;   // FwdArgs<T>[n_traj] (discretize / defects)
    const void* adesc;   // AdjArgs<double>[n_traj] (reverse sweep)
    const int2* items;   // work list, sorted by decreasing substep count
    int n_items;
    int* cursor;         // [2], zero between launches
    void* rec;           // split form: stage records of every item
    const int64_t* rec_off;   // [n_items] element offset of an item's records
};

// Launch preparation for one model group (implemented next to the kernels).
// `persist_blocks` = 0 selects one workgroup per work unit, otherwise that many
// persistent workgroups draw units from the cursor.  `waves` (1 or 2; 2 in
// FP64 only): waves per SIMD the kernel's registers are budgeted for.
cis_status prep_discretize_batch(const cis_model* m, int32_t dtype, const BatchGroupDev& g,
                                 int persist_blocks, int waves, KLaunch* out);
// (body_lanes: the two-wave body-lane kernel, else one element-lane wave per interval)
cis_status prep_defects_batch(const cis_model* m, int32_t dtype, const BatchGroupDev& g,
                              bool body_lanes, KLaunch* out);
// (max_ckpt_every: largest checkpoint spacing of the group's trajectories;
// waves per interval: 3 = evaluation a stage ahead of the reverse sweep (when
// the spacing is at most 8), 2 = replay a chunk ahead, 1 = one wave)
cis_status prep_adjoint_batch(const cis_model* m, const BatchGroupDev& g, int max_ckpt_every,
                              int waves, KLaunch* out);
// gU, gX_N and gp of n_traj trajectories from their partials (RedDesc array).
cis_status prep_adjoint_reduce_batch(const void* rdesc, int n_traj, KLaunch* out);
// Split form of the discretize step (coefficient records, then tangent
// columns): the two launches of one model group.
// (waves: register budget of the tangent kernel in waves per SIMD, 1 or 2)
cis_status prep_split_batch(const cis_model* m, int32_t dtype, const BatchGroupDev& g, int waves,
                            KLaunch* coefrec, KLaunch* tangent);
bool split_form_supported(const cis_model* m);
// elements of one interval's part of the split workspace (-1: not offered)
int64_t split_elems_per_interval(const cis_model* m, int K);
// Column groups (work units per item) of the discretize kernel.
int discretize_units_per_item(const cis_model* m, int32_t dtype);

// Substep blocks, passes 1 and 2 (FP64): checkpoints [B][n][ld_int] at the
// block starts, defect and F~ of the whole interval, and the block
// sensitivities Ab [nx][nx][B N], Bmb / Bpb [nx][m][B N], Sb [nx][B N].
cis_status blocked_passes(const cis_model* m, const cis_shape* sh, const void* X, const void* U,
                          const void* s, const void* prm, int B, double* ckpt, double* Ab,
                          double* Bmb, double* Bpb, double* Sb, void* defect, void* xprop,
                          hipStream_t stream);

// Per-trajectory inputs of the batched reduction.
struct RedDesc {
    const double* ws_uk;
    const double* ws_uk1;
    const double* ws_p;
    double* gU;
    double* gX;
    double* gp;
    int N, m, nxt, np;
    int64_t ldn;
};

}  // namespace cis
