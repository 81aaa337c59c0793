// Substep-blocked discretization (FP64).  The K substeps of every interval
// are split into B blocks of K/B substeps whose sensitivities are integrated
// independently from checkpointed block-start states (passes 1 and 2 in
// cis.hip); pass 3, here, chains them: with X_b = [Phi_b | B-_b | B+_b | S_b]
// of block b (over [tau_b, tau_b+1], Sec. VI variational equations restricted
// to the block),
//     Phi = Phi_{B-1} ... Phi_0,
//     [B- | B+ | S] = sum_b Phi_{B-1} ... Phi_{b+1} [B-_b | B+_b | S_b],
// accumulated from the last block backwards: P = Phi_{B-1}; for b = B-2..0:
// acc += P [B-_b | B+_b | S_b], P = P Phi_b.  The products are dense
// nx-by-nx times nx-by-(nx + 2m + 1), one workgroup per interval, either on
// the vector ALUs or on FP64 MFMA (v_mfma_f64_16x16x4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/cis.h"
#include "cis_debug.hpp"
#include "cis_host.hpp"
#include "cis_launch.hpp"
#include "cis_model.hpp"

namespace cis {

struct ComposeArgs {
    const double* Ab;    // [nx][nx][ldb], column b N + k
    const double* Bmb;   // [nx][m][ldb]
    const double* Bpb;
    const double* Sb;    // [nx][ldb]
    double* A;           // [nx][nx][ldi]
    double* Bm;          // [nx][m][ldi]
    double* Bp;
    double* S;           // [nx][ldi]
    int64_t ldb, ldi;
    int N, B;
};

// element (r, c) of X_b = [Phi_b | B-_b | B+_b | S_b] of interval k, or of
// the output [A | B- | B+ | S] (column index `col` = b N + k or k)
template <class TP>
__device__ __forceinline__ int64_t blk_off(int r, int c, int64_t ld, int64_t col, int& which) {
    constexpr int NXT = TP::NXT, M = TP::M;
    if (c < NXT) { which = 0; return ((int64_t)r * NXT + c) * ld + col; }
    if (c < NXT + M) { which = 1; return ((int64_t)r * M + c - NXT) * ld + col; }
    if (c < NXT + 2 * M) { which = 2; return ((int64_t)r * M + c - NXT - M) * ld + col; }
    which = 3;
    return (int64_t)r * ld + col;
}
template <class TP>
__device__ __forceinline__ double load_blk(const ComposeArgs& a, int r, int c, int b, int k) {
    int w;
    const int64_t o = blk_off<TP>(r, c, a.ldb, (int64_t)b * a.N + k, w);
    const double* p = w == 0 ? a.Ab : (w == 1 ? a.Bmb : (w == 2 ? a.Bpb : a.Sb));
    return p[o];
}
template <class TP>
__device__ __forceinline__ void store_out(const ComposeArgs& a, int r, int c, int k, double v) {
    int w;
    const int64_t o = blk_off<TP>(r, c, a.ldi, k, w);
    double* p = w == 0 ? a.A : (w == 1 ? a.Bm : (w == 2 ? a.Bp : a.S));
    p[o] = v;
}

// ---------------------------------------------------------------------------
// Vector-ALU composition: thread c owns column c of the running products
// (its nx rows in registers); P lives in LDS column-major.
// ---------------------------------------------------------------------------
template <class TP>
struct ComposeValuShared {
    double P[TP::NXT * TP::NXT];   // column-major: P(r, q) at [q * NXT + r]
};

template <class TP>
__global__ void __launch_bounds__(256) k_compose_valu(ComposeArgs a) {
    constexpr int NXT = TP::NXT, M = TP::M, NCOLS = NXT + 2 * M + 1;
    static_assert(NCOLS <= 256, "one thread per column");
    __shared__ ComposeValuShared<TP> sh;
    const int k = xcd_slot(blockIdx.x, gridDim.x);
    const int c = threadIdx.x;
    const bool active = c < NCOLS;
    const bool phi_col = c < NXT;
    double acc[NXT];
    // last block: P = Phi_{B-1}, acc = its B-/B+/S columns
    {
        const int b = a.B - 1;
#pragma unroll
        for (int r = 0; r < NXT; ++r) {
            const double v = active ? load_blk<TP>(a, r, c, b, k) : 0.0;
            acc[r] = v;
            if (phi_col) sh.P[c * NXT + r] = v;
        }
    }
    __syncthreads();
    for (int b = a.B - 2; b >= 0; --b) {
        if (phi_col) {
#pragma unroll
            for (int r = 0; r < NXT; ++r) acc[r] = 0.0;
        }
        // acc += P x, x = column c of X_b, streamed eight rows at a time
#pragma unroll 1
        for (int q0 = 0; q0 < NXT; q0 += 8) {
            double x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                x[i] = (active && q0 + i < NXT) ? load_blk<TP>(a, q0 + i, c, b, k) : 0.0;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (q0 + i < NXT) {
                    const double* pc = sh.P + (q0 + i) * NXT;
#pragma unroll
                    for (int r = 0; r < NXT; ++r) acc[r] = fma(pc[r], x[i], acc[r]);
                }
            }
        }
        __syncthreads();   // every thread has read P
        if (phi_col) {
#pragma unroll
            for (int r = 0; r < NXT; ++r) sh.P[c * NXT + r] = acc[r];
        }
        __syncthreads();
    }
    if (active) {
#pragma unroll
        for (int r = 0; r < NXT; ++r) store_out<TP>(a, r, c, k, phi_col ? sh.P[c * NXT + r] : acc[r]);
    }
}

// ---------------------------------------------------------------------------
// MFMA composition: D(16x16) += A(16x4) B(4x16) with v_mfma_f64_16x16x4.
// Operand layout per lane l (gfx950, checked on the device): A(i = l % 16,
// k = l / 16), B(k = l / 16, j = l % 16); register v = 0..3 of the result
// holds D(l / 16 + 4 v, l % 16).
// The padded product P (NP x NP, NP = nx rounded up to 16) is in LDS,
// column-major; wave w owns column tiles w, w + 4, ...
// ---------------------------------------------------------------------------
template <class TP>
struct ComposeMfmaShared {
    static constexpr int NP = (TP::NXT + 15) / 16 * 16;
    double P[NP * NP];
};

typedef double double4_t __attribute__((ext_vector_type(4)));

template <class TP>
__global__ void __launch_bounds__(256) k_compose_mfma(ComposeArgs a) {
    constexpr int NXT = TP::NXT, M = TP::M, NCOLS = NXT + 2 * M + 1;
    constexpr int NP = ComposeMfmaShared<TP>::NP;
    constexpr int MT = NP / 16, KT = NP / 4;
    constexpr int NT = (NCOLS + 15) / 16;          // column tiles
    constexpr int TPW = (NT + 3) / 4;              // column tiles per wave
    __shared__ ComposeMfmaShared<TP> sh;
    const int k = xcd_slot(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    // accumulators of the owned tiles (Phi tiles hold the new product)
    double4_t acc[TPW][MT];
    auto tile_col = [&](int t) { return (wave + 4 * t) * 16 + li; };
    // last block
    for (int e = tid; e < NP * NP; e += 256) {
        const int q = e / NP, r = e % NP;
        sh.P[e] = (q < NXT && r < NXT) ? load_blk<TP>(a, r, q, a.B - 1, k) : 0.0;
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int c = tile_col(t);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = mt * 16 + lk + 4 * v;
                acc[t][mt][v] = (c >= NXT && c < NCOLS && r < NXT) ? load_blk<TP>(a, r, c, a.B - 1, k)
                                                                    : 0.0;
            }
    }
    __syncthreads();
    for (int b = a.B - 2; b >= 0; --b) {
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int c0 = (wave + 4 * t) * 16;
            if (c0 >= NCOLS) continue;                 // wave-uniform
            const int c = c0 + li;
            // a tile may straddle column nx: the column (lane) decides whether
            // it starts a new product (Phi columns) or accumulates (B-/B+/S)
            const bool phi_lane = c < NXT;
            // B operand of every k step: X_b(4 kt + lk, c)
            double bop[KT];
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) {
                const int r = 4 * kt + lk;
                bop[kt] = (c < NCOLS && r < NXT) ? load_blk<TP>(a, r, c, b, k) : 0.0;
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const double4_t zero = {0.0, 0.0, 0.0, 0.0};
                double4_t d = phi_lane ? zero : acc[t][mt];
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) {
                    const double aop = sh.P[(4 * kt + lk) * NP + mt * 16 + li];
                    d = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[kt], d, 0, 0, 0);
                }
                acc[t][mt] = d;
            }
        }
        __syncthreads();   // every wave has read P
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int c0 = (wave + 4 * t) * 16;
            if (c0 >= NXT) continue;
            const int c = c0 + li;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = mt * 16 + lk + 4 * v;
                    // keep the padding of P zero
                    sh.P[c * NP + r] = (c < NXT && r < NXT) ? acc[t][mt][v] : 0.0;
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int c0 = (wave + 4 * t) * 16;
        if (c0 >= NCOLS) continue;
        const int c = c0 + li;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = mt * 16 + lk + 4 * v;
                if (c < NCOLS && r < NXT)
                    store_out<TP>(a, r, c, k, c < NXT ? sh.P[c * NP + r] : acc[t][mt][v]);
            }
    }
}

template <int L, int D>
static cis_status launch_compose(const ComposeArgs& ca, int mode, hipStream_t stream) {
    using TP = Topo<L, D>;
    ComposeArgs a = ca;
    void* args[] = {&a};
    const void* fn = mode == CIS_COMPOSE_MFMA ? (const void*)&k_compose_mfma<TP>
                                              : (const void*)&k_compose_valu<TP>;
    const int nth = mode == CIS_COMPOSE_MFMA ? 256 : (TP::NXT + 2 * TP::M + 1 + 63) / 64 * 64;
    hipError_t e = hipLaunchKernel(fn, dim3(a.N), dim3(nth), args, 0, stream);
    if (e != hipSuccess) return fail(CIS_ERR_HIP, "k_compose launch: %s", hipGetErrorString(e));
    return CIS_OK;
}

struct BlockedLayout {
    size_t ckpt, Ab, Bmb, Bpb, Sb, total;   // byte offsets into the workspace
};

static size_t al256(size_t v) { return (v + 255) / 256 * 256; }

static BlockedLayout blocked_layout(const cis_model* m, const cis_shape* sh, int B) {
    BlockedLayout l;
    const size_t nx = m->nx, mm = m->m, N = sh->N;
    size_t o = 0;
    l.ckpt = o;
    o = al256(o + (size_t)B * m->n * sh->ld_int * sizeof(double));
    l.Ab = o;
    o = al256(o + nx * nx * B * N * sizeof(double));
    l.Bmb = o;
    o = al256(o + nx * mm * B * N * sizeof(double));
    l.Bpb = o;
    o = al256(o + nx * mm * B * N * sizeof(double));
    l.Sb = o;
    o = al256(o + nx * B * N * sizeof(double));
    l.total = o;
    return l;
}

}  // namespace cis

using namespace cis;

extern "C" cis_status cis_blocked_workspace_size(const cis_model* model, const cis_shape* shape,
                                                 int32_t blocks, size_t* bytes) {
    if (!model || !shape || !bytes)
        return fail(CIS_ERR_NULL, "cis_blocked_workspace_size: null argument");
    if (shape->N < 1 || blocks < 2 || shape->substeps < 1 || shape->substeps % blocks != 0 ||
        shape->ld_int < shape->N)
        return fail(CIS_ERR_DIM, "cis_blocked_workspace_size: need N >= 1, ld_int >= N, blocks >= 2 dividing K");
    *bytes = blocked_layout(model, shape, blocks).total;
    return CIS_OK;
}

static cis_status discretize_blocked_impl(const cis_model* model, const cis_shape* shape,
                                          const void* X, const void* U, const void* s,
                                          const void* params, int32_t blocks,
                                          int32_t compose, void* A, void* Bm, void* Bp,
                                          void* S, void* defect, void* xprop, void* ws,
                                          size_t ws_bytes, void* stream) {
    cis_status st = check_common(model, shape, X, U, s, params);
    if (st != CIS_OK) return st;
    if (shape->dtype != CIS_F64)
        return fail(CIS_ERR_DTYPE, "cis_discretize_blocked: only CIS_F64 is offered");
    if (blocks < 2 || shape->substeps % blocks != 0)
        return fail(CIS_ERR_DIM, "cis_discretize_blocked: blocks=%d must be >= 2 and divide K=%d",
                    blocks, shape->substeps);
    if (compose != CIS_COMPOSE_VALU && compose != CIS_COMPOSE_MFMA)
        return fail(CIS_ERR_DIM, "cis_discretize_blocked: unknown composition %d", compose);
    const bool hasm = model->m > 0;
    if (!A || !S || !defect || (hasm && (!Bm || !Bp)))
        return fail(CIS_ERR_NULL, "cis_discretize_blocked: A, S, defect (and Bm, Bp when m > 0) are required");
    if (!aligned(A, 8) || !aligned(S, 8) || !aligned(defect, 8) || !aligned(xprop, 8) ||
        !aligned(Bm, 8) || !aligned(Bp, 8) || !aligned(ws, 8))
        return fail(CIS_ERR_LAYOUT, "cis_discretize_blocked: pointer not aligned to 8 bytes");
    const BlockedLayout l = blocked_layout(model, shape, blocks);
    if (!ws || ws_bytes < l.total)
        return fail(CIS_ERR_WORKSPACE, "cis_discretize_blocked: workspace of %zu bytes needed",
                    l.total);
    unsigned char* w = (unsigned char*)ws;
    hipStream_t hs = (hipStream_t)stream;
    ComposeArgs ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.Ab = (const double*)(w + l.Ab);
    ca.Bmb = (const double*)(w + l.Bmb);
    ca.Bpb = (const double*)(w + l.Bpb);
    ca.Sb = (const double*)(w + l.Sb);
    ca.A = (double*)A;
    ca.Bm = (double*)Bm;
    ca.Bp = (double*)Bp;
    ca.S = (double*)S;
    ca.ldb = (int64_t)blocks * shape->N;
    ca.ldi = shape->ld_int;
    ca.N = shape->N;
    ca.B = blocks;
    st = blocked_passes(model, shape, X, U, s, params, blocks, (double*)(w + l.ckpt),
                        (double*)(w + l.Ab), (double*)(w + l.Bmb), (double*)(w + l.Bpb),
                        (double*)(w + l.Sb), defect, xprop, hs);
    if (st != CIS_OK) return st;
#define CIS_COMPOSE(LL, DD) \
    if (model->L == LL && model->D == DD) return launch_compose<LL, DD>(ca, compose, hs);
    CIS_TOPOLOGIES(CIS_COMPOSE)
#undef CIS_COMPOSE
    return fail(CIS_ERR_UNSUPPORTED, "cis_discretize_blocked: topology has no compiled kernel");
}

extern "C" cis_status cis_discretize_blocked(const cis_model* model, const cis_shape* shape,
                                             const void* X, const void* U, const void* s,
                                             const void* params, int32_t blocks,
                                             int32_t compose, void* A, void* Bm, void* Bp,
                                             void* S, void* defect, void* xprop, void* ws,
                                             size_t ws_bytes, void* stream) {
    const cis_status st = discretize_blocked_impl(model, shape, X, U, s, params, blocks, compose,
                                                  A, Bm, Bp, S, defect, xprop, ws, ws_bytes,
                                                  stream);
    if (st != CIS_OK || !debug_finite_enabled()) return st;
    return debug_scan_forward("cis_discretize_blocked", model, shape, model->nx, model->m, X, U,
                              s, params, A, Bm, Bp, S, defect, xprop, nullptr, stream);
}

// ---------------------------------------------------------------------------
// Tuner of the discretize step for one trajectory shape: one-launch layouts,
// split form, blocked forms, timed on the caller's data.
// ---------------------------------------------------------------------------
namespace {

// Best of `reps` timed runs (HIP events on the stream) after one untimed run.
template <class F>
float time_ms(F run, hipStream_t hs, int reps, cis_status& st) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = fail(CIS_ERR_HIP, "cis_single_tune: event creation failed");
        return 0.0f;
    }
    float best = -1.0f;
    st = run();
    for (int r = 0; r < reps && st == CIS_OK; ++r) {
        hipEventRecord(e0, hs);
        st = run();
        hipEventRecord(e1, hs);
        if (hipEventSynchronize(e1) != hipSuccess) st = fail(CIS_ERR_HIP, "cis_single_tune: sync failed");
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        if (best < 0.0f || ms < best) best = ms;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return best;
}

bool valid_choice(const cis_single_choice& c, const cis_model* m, const cis_shape* sh) {
    const bool legs = m->L >= 1 && m->D >= 1;
    switch (c.form) {
    case CIS_FORM_ONE_LAUNCH: return c.layout >= 1 && c.layout <= 4;
    case CIS_FORM_SPLIT: return legs && (c.waves == 1 || c.waves == 2);
    case CIS_FORM_BLOCKED:
        return sh->dtype == CIS_F64 && c.blocks >= 2 && c.blocks <= 8 &&
               sh->substeps % c.blocks == 0 &&
               (c.compose == CIS_COMPOSE_VALU || c.compose == CIS_COMPOSE_MFMA);
    default: return false;
    }
}

}  // namespace

extern "C" cis_status cis_single_tune(const cis_model* model, const cis_shape* shape,
                                      const void* X, const void* U, const void* s,
                                      const void* params, void* A, void* Bm, void* Bp, void* S,
                                      void* defect, void* xprop, cis_single_choice* choice,
                                      void* stream) {
    cis_status st = check_common(model, shape, X, U, s, params);
    if (st != CIS_OK) return st;
    if (!choice) return fail(CIS_ERR_NULL, "cis_single_tune: choice output is required");
    if (shape->layout != 0) return fail(CIS_ERR_DIM, "cis_single_tune: shape->layout must be 0");
    hipStream_t hs = (hipStream_t)stream;
    const int K = shape->substeps;
    const bool f64 = shape->dtype == CIS_F64;
    const bool legs = model->L >= 1 && model->D >= 1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(CIS_ERR_HIP, "cis_single_tune: no device");
    std::memset(choice, 0, sizeof(*choice));
    // cache lookup
    const char* cpath = std::getenv("CIS_TUNE_CACHE");
    char key[256];
    std::snprintf(key, sizeof(key), "single|%s|L%dD%d|%s|N%d|K%d", device_tag(dev).c_str(),
                  model->L, model->D, f64 ? "f64" : "f32", shape->N, K);
    bool hit = false;
    if (cpath && *cpath) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        const auto cache = cache_read(cpath);
        const auto it = cache.find(key);
        if (it != cache.end()) {
            cis_single_choice c{};
            c.form = it->second.form;
            c.layout = it->second.layout;
            c.waves = it->second.waves;
            c.blocks = it->second.blocks;
            c.compose = it->second.compose;
            if (valid_choice(c, model, shape)) {
                *choice = c;
                choice->from_cache = 1;
                hit = true;
            }
        }
    }
    // workspace for the largest candidate (split records, blocked passes)
    size_t wsz = 0;
    if (legs) {
        size_t b = 0;
        st = cis_split_workspace_size(model, shape, &b);
        if (st != CIS_OK) return st;
        wsz = std::max(wsz, b);
    }
    for (int b = 2; f64 && b <= 8 && b <= K; ++b)
        if (K % b == 0) wsz = std::max(wsz, blocked_layout(model, shape, b).total);
    void* ws = nullptr;
    if (wsz && hipMalloc(&ws, wsz) != hipSuccess)
        return fail(CIS_ERR_HIP, "cis_single_tune: workspace of %zu bytes", wsz);
    auto run = [&](const cis_single_choice& c) -> cis_status {
        if (c.form == CIS_FORM_SPLIT)
            return cis_discretize_split(model, shape, X, U, s, params, c.waves, A, Bm, Bp, S,
                                        defect, xprop, ws, wsz, stream);
        if (c.form == CIS_FORM_BLOCKED)
            return cis_discretize_blocked(model, shape, X, U, s, params, c.blocks, c.compose, A,
                                          Bm, Bp, S, defect, xprop, ws, wsz, stream);
        cis_shape sh = *shape;
        sh.layout = c.layout;
        return cis_discretize(model, &sh, X, U, s, params, A, Bm, Bp, S, defect, xprop, stream);
    };
    if (!hit) {
        std::vector<cis_single_choice> cands;
        for (int l = 1; l <= 4; ++l) cands.push_back({CIS_FORM_ONE_LAUNCH, l, 0, 0, 0, 0, 0.0f});
        if (legs)
            for (int w = 1; w <= 2; ++w) cands.push_back({CIS_FORM_SPLIT, 0, w, 0, 0, 0, 0.0f});
        for (int b = 2; f64 && b <= 8 && b <= K; ++b)
            if (K % b == 0)
                for (int c = CIS_COMPOSE_VALU; c <= CIS_COMPOSE_MFMA; ++c)
                    cands.push_back({CIS_FORM_BLOCKED, 0, 0, b, c, 0, 0.0f});
        int best = -1;
        float best_ms = 0.0f;
        for (int i = 0; i < (int)cands.size() && st == CIS_OK; ++i) {
            const float ms = time_ms([&] { return run(cands[i]); }, hs, 3, st);
            if (st == CIS_OK && (best < 0 || ms < best_ms)) {
                best = i;
                best_ms = ms;
            }
        }
        if (st != CIS_OK) {
            if (ws) (void)hipFree(ws);
            return st;
        }
        *choice = cands[best];
        choice->ms = best_ms;
        if (cpath && *cpath) {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto cur = cache_read(cpath);
            TuneChoice& tc = cur[key];
            tc.form = choice->form;
            tc.layout = choice->layout;
            tc.waves = choice->waves;
            tc.blocks = choice->blocks;
            tc.compose = choice->compose;
            (void)cache_write(cpath, cur);
        }
    }
    // the outputs hold the chosen configuration's results
    st = run(*choice);
    if (st == CIS_OK && hipStreamSynchronize(hs) != hipSuccess)
        st = fail(CIS_ERR_HIP, "cis_single_tune: stream synchronization failed");
    if (ws) (void)hipFree(ws);
    return st;
}
