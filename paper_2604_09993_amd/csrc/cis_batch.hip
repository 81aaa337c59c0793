// Batched multiple shooting over many trajectories: plan creation (work
// lists, descriptors, schedule tuning, HIP graphs) and the hot run calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/cis.h"
#include "cis_host.hpp"
#include "cis_launch.hpp"
#include "cis_model.hpp"

using namespace cis;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Group {
    const cis_model* model = nullptr;
    std::vector<int> trajs;    // indices into the plan's trajectory list
    std::vector<int2> items;   // {group-local trajectory, interval}
    int units_per_item = 0;
    int persist_blocks = 0;
    int disc_waves = 0;        // register budget of the discretize kernel (waves per SIMD)
    int adj_waves = 0;         // waves per interval of the chosen reverse sweep
    int def_waves = 0;         // waves per interval of the chosen defects pass
    size_t fdesc_off = 0, ddesc_off = 0, adesc_off = 0, items_off = 0, cursor_off = 0;
    // split form: record offsets per item (device), the group's part of the
    // record memory (elements), and whether the chosen discretize form is it
    bool split_ok = false, split = false;
    size_t recoff_off = 0, rec_base = 0;
    std::vector<int64_t> rec_off;
    BatchGroupDev dev{};
    KLaunch disc, disc_b, def, adj;   // disc_b: tangent launch of the split form
    bool from_cache = false;          // every tuned choice came from the tuning cache
};

}  // namespace

namespace cis {

// ---------------------------------------------------------------------------
// Tuning cache: the choices CIS_SCHED_TUNE makes per model group (and the
// single-trajectory tuner per trajectory shape), kept in the JSON file named
// by CIS_TUNE_CACHE (no variable: no cache) as
//   {"version": 1, "entries": {"<key>": {"split": s, "waves": w, "persist": p,
//                                        "def_lane": d, "adj_waves": a,
//                                        "blocks": b, "compose": c,
//                                        "form": f, "layout": l}, ...}}
// keyed by device (architecture, compute units), topology, dtype, operations,
// work-list length and substep range (and checkpoint spacing with the reverse
// sweep); -1 marks a choice that was not made.  A missing or unreadable file
// is an empty cache; writes replace the file through a temporary.
// ---------------------------------------------------------------------------
std::mutex g_cache_mu;

// minimal reader of the cache's own format (objects, strings, integers)
struct CacheParser {
    const std::string& t;
    size_t i = 0;
    explicit CacheParser(const std::string& s) : t(s) {}
    void ws() { while (i < t.size() && std::strchr(" \t\r\n", t[i])) ++i; }
    bool lit(char c) { ws(); if (i < t.size() && t[i] == c) { ++i; return true; } return false; }
    bool str(std::string& out) {
        ws();
        if (i >= t.size() || t[i] != '"') return false;
        const size_t j = t.find('"', i + 1);
        if (j == std::string::npos) return false;
        out = t.substr(i + 1, j - i - 1);
        i = j + 1;
        return true;
    }
    bool num(long& v) {
        ws();
        char* end = nullptr;
        v = std::strtol(t.c_str() + i, &end, 10);
        if (end == t.c_str() + i) return false;
        i = end - t.c_str();
        return true;
    }
    // {"name": int, ...}
    bool choice(TuneChoice& c) {
        if (!lit('{')) return false;
        if (lit('}')) return true;
        do {
            std::string k;
            long v = 0;
            if (!str(k) || !lit(':') || !num(v)) return false;
            if (k == "split") c.split = (int)v;
            else if (k == "waves") c.waves = (int)v;
            else if (k == "persist") c.persist = (int)v;
            else if (k == "def_lane") c.def_lane = (int)v;
            else if (k == "adj_waves") c.adj_waves = (int)v;
            else if (k == "blocks") c.blocks = (int)v;
            else if (k == "compose") c.compose = (int)v;
            else if (k == "form") c.form = (int)v;
            else if (k == "layout") c.layout = (int)v;
        } while (lit(','));
        return lit('}');
    }
    bool file(std::map<std::string, TuneChoice>& m) {
        if (!lit('{')) return false;
        if (lit('}')) return true;
        do {
            std::string k;
            if (!str(k) || !lit(':')) return false;
            if (k == "entries") {
                if (!lit('{')) return false;
                if (lit('}')) continue;
                do {
                    std::string key;
                    TuneChoice c;
                    if (!str(key) || !lit(':') || !choice(c)) return false;
                    m[key] = c;
                } while (lit(','));
                if (!lit('}')) return false;
            } else {
                long v = 0;
                if (!num(v)) return false;
            }
        } while (lit(','));
        return lit('}');
    }
};

std::map<std::string, TuneChoice> cache_read(const std::string& path) {
    std::map<std::string, TuneChoice> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    CacheParser cp(text);
    if (!cp.file(m)) m.clear();
    return m;
}

bool cache_write(const std::string& path, const std::map<std::string, TuneChoice>& m) {
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return false;
        f << "{\"version\": 1, \"entries\": {";
        bool first = true;
        for (const auto& kv : m) {
            const TuneChoice& c = kv.second;
            f << (first ? "\n  " : ",\n  ") << '"' << kv.first << "\": {\"split\": " << c.split
              << ", \"waves\": " << c.waves << ", \"persist\": " << c.persist
              << ", \"def_lane\": " << c.def_lane << ", \"adj_waves\": " << c.adj_waves
              << ", \"blocks\": " << c.blocks << ", \"compose\": " << c.compose
              << ", \"form\": " << c.form << ", \"layout\": " << c.layout << "}";
            first = false;
        }
        f << "\n}}\n";
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path.c_str()) == 0;
}

std::string device_tag(int dev) {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%s/%dcu", pr.gcnArchName, pr.multiProcessorCount);
    for (char* c = buf; *c; ++c)
        if (*c == '"' || *c == '\\') *c = '_';
    return buf;
}

}  // namespace cis

namespace {

int auto_ckpt(int K) {
    for (int c = 8; c > 1; --c)
        if (K % c == 0) return c;
    return 1;
}

}  // namespace

struct cis_batch_plan {
    int device = 0;
    int32_t dtype = CIS_F64, ops = 0;
    std::vector<cis_traj> trajs;
    std::vector<int> ckpt_every;
    std::vector<size_t> ckpt_off, ws_off;
    std::vector<Group> groups;
    size_t rdesc_off = 0;
    unsigned char* dmem = nullptr;
    unsigned char* recmem = nullptr;   // stage records of the split form
    KLaunch red;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
};

static void plan_free(cis_batch_plan* p) {
    if (!p) return;
    for (int i = 0; i < 2; ++i) {
        if (p->exec[i]) (void)hipGraphExecDestroy(p->exec[i]);
        if (p->graph[i]) (void)hipGraphDestroy(p->graph[i]);
    }
    if (p->dmem) (void)hipFree(p->dmem);
    if (p->recmem) (void)hipFree(p->recmem);
    delete p;
}

// Per-trajectory argument checks of one operation.
static cis_status check_traj(const cis_traj& t, int i, int32_t dtype, int32_t ops) {
    cis_shape sh;
    std::memset(&sh, 0, sizeof(sh));
    sh.N = t.N;
    sh.substeps = t.substeps;
    sh.dtype = (cis_dtype)dtype;
    sh.ld_node = t.ld_node;
    sh.ld_int = t.ld_int;
    cis_status st = check_common(t.model, &sh, t.X, t.U, t.s, t.params);
    if (st != CIS_OK) {
        char why[256];
        std::snprintf(why, sizeof(why), "%s", cis_last_error());
        return fail(st, "trajectory %d: %s", i, why);
    }
    const size_t es = elem_size(dtype);
    const bool hasm = t.model->m > 0;
    if (ops & CIS_BATCH_DISCRETIZE) {
        if (!t.A || !t.S || !t.defect || (hasm && (!t.Bm || !t.Bp)))
            return fail(CIS_ERR_NULL, "trajectory %d: A, S, defect (and Bm, Bp when m > 0) are required", i);
        if (!aligned(t.A, es) || !aligned(t.S, es) || !aligned(t.defect, es) ||
            !aligned(t.xprop, es) || !aligned(t.Bm, es) || !aligned(t.Bp, es))
            return fail(CIS_ERR_LAYOUT, "trajectory %d: output pointer not aligned to %zu bytes", i, es);
    }
    if (ops & CIS_BATCH_ADJOINT) {
        if (!t.defect || !t.seed || !t.gX || !t.gs || !t.gparams || (hasm && !t.gU))
            return fail(CIS_ERR_NULL, "trajectory %d: defect, seed, gX, gs, gparams (and gU when m > 0) are required", i);
        if (!aligned(t.defect, es) || !aligned(t.xprop, es) || !aligned(t.seed, es) ||
            !aligned(t.gX, es) || !aligned(t.gU, es) || !aligned(t.gs, es) || !aligned(t.gparams, es))
            return fail(CIS_ERR_LAYOUT, "trajectory %d: pointer not aligned to %zu bytes", i, es);
    }
    return CIS_OK;
}

template <class T>
static FwdArgs<T> fwd_desc(const cis_traj& t) {
    FwdArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.X = (const T*)t.X;
    a.U = (const T*)t.U;
    a.s = (const T*)t.s;
    a.prm = (const T*)t.params;
    a.ldn = t.ld_node;
    a.ldi = t.ld_int;
    a.N = t.N;
    a.K = t.substeps;
    a.C = 1;
    return a;
}

// Median time in microseconds of `reps` launches of one group's discretize kernel.
static float time_launch(KLaunch& l, hipStream_t s, int reps) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.f;
    }
    std::vector<float> ts;
    bool ok = l.launch(s) == hipSuccess;   // warm-up
    for (int r = 0; ok && r < reps; ++r) {
        ok = hipEventRecord(e0, s) == hipSuccess && l.launch(s) == hipSuccess &&
             hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        if (ok) ok = hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        ts.push_back(ms * 1e3f);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok || ts.empty()) return -1.f;
    std::sort(ts.begin(), ts.end());
    return ts[ts.size() / 2];
}

// Median time in microseconds of `reps` launches of a pair (the split form).
static float time_pair(KLaunch& a, KLaunch& b, hipStream_t s, int reps) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.f;
    }
    std::vector<float> ts;
    bool ok = a.launch(s) == hipSuccess && b.launch(s) == hipSuccess;   // warm-up
    for (int r = 0; ok && r < reps; ++r) {
        ok = hipEventRecord(e0, s) == hipSuccess && a.launch(s) == hipSuccess &&
             b.launch(s) == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
             hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        if (ok) ok = hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        ts.push_back(ms * 1e3f);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok || ts.empty()) return -1.f;
    std::sort(ts.begin(), ts.end());
    return ts[ts.size() / 2];
}

static cis_status build_graph(cis_batch_plan* p, int op) {
    const int gi = op == CIS_BATCH_DISCRETIZE ? 0 : 1;
    hipGraph_t g = nullptr;
    if (hipGraphCreate(&g, 0) != hipSuccess) return fail(CIS_ERR_HIP, "hipGraphCreate failed");
    p->graph[gi] = g;
    std::vector<hipGraphNode_t> tails;
    for (Group& gr : p->groups) {
        hipGraphNode_t n0 = nullptr, n1 = nullptr;
        if (op == CIS_BATCH_DISCRETIZE) {
            if (gr.disc.node(g, nullptr, 0, &n0) != hipSuccess)
                return fail(CIS_ERR_HIP, "graph: discretize node refused");
            if (gr.split && gr.disc_b.node(g, &n0, 1, &n1) != hipSuccess)
                return fail(CIS_ERR_HIP, "graph: tangent node refused");
        } else {
            if (gr.def.node(g, nullptr, 0, &n0) != hipSuccess ||
                gr.adj.node(g, &n0, 1, &n1) != hipSuccess)
                return fail(CIS_ERR_HIP, "graph: defects/adjoint node refused");
            tails.push_back(n1);
        }
    }
    if (op == CIS_BATCH_ADJOINT) {
        hipGraphNode_t nr = nullptr;
        if (p->red.node(g, tails.data(), tails.size(), &nr) != hipSuccess)
            return fail(CIS_ERR_HIP, "graph: reduction node refused");
    }
    hipError_t e = hipGraphInstantiate(&p->exec[gi], g, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(CIS_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return CIS_OK;
}

static bool sched_bits_unknown(int32_t s) { return (s & ~0x1FFF) != 0; }

extern "C" cis_status cis_batch_plan_create(const cis_traj* trajs, int32_t n_traj,
                                            cis_dtype dtype, int32_t ops, int32_t sched,
                                            int32_t ckpt_every, int32_t graph, void* stream,
                                            cis_batch_plan** out) {
    const int32_t sched_all = sched;
    if (!out) return fail(CIS_ERR_NULL, "cis_batch_plan_create: plan output is required");
    *out = nullptr;
    if (!trajs) return fail(CIS_ERR_NULL, "cis_batch_plan_create: trajs is required");
    if (n_traj < 1) return fail(CIS_ERR_DIM, "cis_batch_plan_create: n_traj=%d must be >= 1", n_traj);
    if (dtype != CIS_F64 && dtype != CIS_F32)
        return fail(CIS_ERR_DTYPE, "cis_batch_plan_create: unknown dtype %d", dtype);
    if (ops < 1 || ops > 3) return fail(CIS_ERR_DIM, "cis_batch_plan_create: ops=%d is not a mask of operations", ops);
    if ((ops & CIS_BATCH_ADJOINT) && dtype != CIS_F64)
        return fail(CIS_ERR_DTYPE, "cis_batch_plan_create: the reverse sweep is offered in CIS_F64 only");
    int adj_force = (sched >> 4) & 3;   // 0: default, else waves of the reverse sweep
    const bool adj4 = (sched & CIS_SCHED_ADJ_4) != 0;
    const int waves_force = (sched >> 6) & 3;   // 0: default, 1 or 2: register budget
    const int def_force = (sched >> 9) & 3;     // 0: default, 1: body lanes, 2: element lanes
    const int split_force = (sched >> 11) & 3;  // 0: default, 1: split form, 2: fused form
    sched &= 0xF;
    if (sched < CIS_SCHED_GRID || sched > CIS_SCHED_TUNE || sched_bits_unknown(sched_all) ||
        waves_force == 3 || def_force == 3 || split_force == 3 || (adj4 && adj_force))
        return fail(CIS_ERR_DIM, "cis_batch_plan_create: unknown schedule %d", sched_all);
    if (adj4) adj_force = 4;
    if (waves_force == 2 && dtype != CIS_F64 && split_force != 1)
        return fail(CIS_ERR_DTYPE, "cis_batch_plan_create: CIS_SCHED_WAVES_2 is offered in CIS_F64 "
                                   "only (FP32: with CIS_SCHED_SPLIT)");
    if (ckpt_every < 0) return fail(CIS_ERR_DIM, "cis_batch_plan_create: ckpt_every=%d < 0", ckpt_every);
    for (int i = 0; i < n_traj; ++i) {
        cis_status st = check_traj(trajs[i], i, dtype, ops);
        if (st != CIS_OK) return st;
        if ((ops & CIS_BATCH_ADJOINT) && ckpt_every > 0 && trajs[i].substeps % ckpt_every != 0)
            return fail(CIS_ERR_DIM, "trajectory %d: ckpt_every=%d must divide K=%d", i, ckpt_every,
                        trajs[i].substeps);
        if ((int64_t)trajs[i].N > (1 << 30))
            return fail(CIS_ERR_DIM, "trajectory %d: N too large", i);
    }
    cis_batch_plan* p = new cis_batch_plan();
    p->dtype = dtype;
    p->ops = ops;
    p->trajs.assign(trajs, trajs + n_traj);
    (void)hipGetDevice(&p->device);
    hipStream_t hs = (hipStream_t)stream;

    // group by model, work items sorted by decreasing K (then trajectory, interval)
    for (int i = 0; i < n_traj; ++i) {
        const cis_model* m = trajs[i].model;
        auto it = std::find_if(p->groups.begin(), p->groups.end(),
                               [&](const Group& g) { return g.model == m; });
        if (it == p->groups.end()) {
            p->groups.emplace_back();
            p->groups.back().model = m;
            it = p->groups.end() - 1;
        }
        it->trajs.push_back(i);
    }
    int64_t total_items = 0;
    for (Group& g : p->groups) {
        for (int lt = 0; lt < (int)g.trajs.size(); ++lt)
            for (int k = 0; k < trajs[g.trajs[lt]].N; ++k) g.items.push_back(make_int2(lt, k));
        std::stable_sort(g.items.begin(), g.items.end(), [&](const int2& a, const int2& b) {
            return trajs[g.trajs[a.x]].substeps > trajs[g.trajs[b.x]].substeps;
        });
        g.units_per_item = discretize_units_per_item(g.model, dtype);
        total_items += (int64_t)g.items.size();
        if ((int64_t)g.items.size() * g.units_per_item > (int64_t)1 << 30) {
            plan_free(p);
            return fail(CIS_ERR_DIM, "cis_batch_plan_create: work list too long");
        }
    }
    (void)total_items;

    // device memory: descriptors, work lists, cursors; checkpoints and partials
    const size_t es = elem_size(dtype);
    const size_t fsz = dtype == CIS_F64 ? sizeof(FwdArgs<double>) : sizeof(FwdArgs<float>);
    size_t off = 0;
    for (Group& g : p->groups) {
        const size_t nt = g.trajs.size();
        g.fdesc_off = off;
        off = align_up(off + nt * fsz);
        g.ddesc_off = off;
        off = align_up(off + nt * fsz);
        g.adesc_off = off;
        off = align_up(off + nt * sizeof(AdjArgs<double>));
        g.items_off = off;
        off = align_up(off + g.items.size() * sizeof(int2));
        g.cursor_off = off;
        off = align_up(off + 2 * sizeof(int));
        // split form: candidate when forced, or timed with CIS_SCHED_TUNE
        g.split_ok = (ops & CIS_BATCH_DISCRETIZE) && split_form_supported(g.model) &&
                     split_force != 2 && (split_force == 1 || sched == CIS_SCHED_TUNE);
        if (g.split_ok) {
            g.recoff_off = off;
            off = align_up(off + g.items.size() * sizeof(int64_t));
        }
    }
    size_t rec_total = 0;   // elements
    for (Group& g : p->groups) {
        if (!g.split_ok) continue;
        g.rec_base = rec_total;
        int64_t cum = 0;
        g.rec_off.resize(g.items.size());
        for (size_t it = 0; it < g.items.size(); ++it) {
            g.rec_off[it] = cum;
            cum += split_elems_per_interval(g.model, trajs[g.trajs[g.items[it].x]].substeps);
        }
        rec_total += (size_t)cum;
        rec_total = (rec_total + 31) / 32 * 32;
    }
    p->rdesc_off = off;
    off = align_up(off + (ops & CIS_BATCH_ADJOINT ? n_traj * sizeof(RedDesc) : 0));
    const size_t host_part = off;
    p->ckpt_every.assign(n_traj, 1);
    p->ckpt_off.assign(n_traj, 0);
    p->ws_off.assign(n_traj, 0);
    if (ops & CIS_BATCH_ADJOINT) {
        for (int i = 0; i < n_traj; ++i) {
            const cis_traj& t = trajs[i];
            const int C = ckpt_every > 0 ? ckpt_every : auto_ckpt(t.substeps);
            p->ckpt_every[i] = C;
            p->ckpt_off[i] = off;
            off = align_up(off + (size_t)(t.substeps / C) * t.model->n * t.ld_int * es);
            p->ws_off[i] = off;
            off = align_up(off + (size_t)(2 * t.model->m + t.model->np) * t.N * sizeof(double));
        }
    }
    hipError_t e = hipMalloc((void**)&p->dmem, off);
    if (e != hipSuccess) {
        plan_free(p);
        return fail(CIS_ERR_HIP, "cis_batch_plan_create: hipMalloc(%zu): %s", off, hipGetErrorString(e));
    }
    unsigned char* d = p->dmem;
    if (rec_total > 0) {
        e = hipMalloc((void**)&p->recmem, rec_total * es);
        if (e != hipSuccess) {
            plan_free(p);
            return fail(CIS_ERR_HIP, "cis_batch_plan_create: hipMalloc(%zu) of the stage records: %s",
                        rec_total * es, hipGetErrorString(e));
        }
    }

    // host image of the descriptor part
    std::vector<unsigned char> img(host_part, 0);
    for (Group& g : p->groups) {
        for (size_t lt = 0; lt < g.trajs.size(); ++lt) {
            const int i = g.trajs[lt];
            const cis_traj& t = trajs[i];
            if (dtype == CIS_F64) {
                FwdArgs<double> a = fwd_desc<double>(t);
                a.A = (double*)t.A;
                a.Bm = (double*)t.Bm;
                a.Bp = (double*)t.Bp;
                a.S = (double*)t.S;
                a.defect = (double*)t.defect;
                a.xprop = (double*)t.xprop;
                std::memcpy(&img[g.fdesc_off + lt * fsz], &a, fsz);
                FwdArgs<double> f = fwd_desc<double>(t);
                f.defect = (double*)t.defect;
                f.xprop = (double*)t.xprop;
                if (ops & CIS_BATCH_ADJOINT) {
                    f.ckpt = (double*)(d + p->ckpt_off[i]);
                    f.C = p->ckpt_every[i];
                }
                std::memcpy(&img[g.ddesc_off + lt * fsz], &f, fsz);
                AdjArgs<double> ad;
                std::memset(&ad, 0, sizeof(ad));
                ad.f = f;
                ad.seed = (const double*)t.seed;
                ad.gX = (double*)t.gX;
                ad.gs = (double*)t.gs;
                if (ops & CIS_BATCH_ADJOINT) {
                    double* w = (double*)(d + p->ws_off[i]);
                    ad.ws_uk = w;
                    ad.ws_uk1 = w + (size_t)t.model->m * t.N;
                    ad.ws_p = w + (size_t)2 * t.model->m * t.N;
                }
                std::memcpy(&img[g.adesc_off + lt * sizeof(ad)], &ad, sizeof(ad));
            } else {
                FwdArgs<float> a = fwd_desc<float>(t);
                a.A = (float*)t.A;
                a.Bm = (float*)t.Bm;
                a.Bp = (float*)t.Bp;
                a.S = (float*)t.S;
                a.defect = (float*)t.defect;
                a.xprop = (float*)t.xprop;
                std::memcpy(&img[g.fdesc_off + lt * fsz], &a, fsz);
                FwdArgs<float> f = fwd_desc<float>(t);
                f.defect = (float*)t.defect;
                f.xprop = (float*)t.xprop;
                std::memcpy(&img[g.ddesc_off + lt * fsz], &f, fsz);
            }
        }
        if (!g.items.empty())
            std::memcpy(&img[g.items_off], g.items.data(), g.items.size() * sizeof(int2));
        if (g.split_ok && !g.items.empty())
            std::memcpy(&img[g.recoff_off], g.rec_off.data(), g.items.size() * sizeof(int64_t));
    }
    if (ops & CIS_BATCH_ADJOINT) {
        for (int i = 0; i < n_traj; ++i) {
            const cis_traj& t = trajs[i];
            RedDesc r;
            std::memset(&r, 0, sizeof(r));
            const double* w = (const double*)(d + p->ws_off[i]);
            r.ws_uk = w;
            r.ws_uk1 = w + (size_t)t.model->m * t.N;
            r.ws_p = w + (size_t)2 * t.model->m * t.N;
            r.gU = (double*)t.gU;
            r.gX = (double*)t.gX;
            r.gp = (double*)t.gparams;
            r.N = t.N;
            r.m = t.model->m;
            r.nxt = t.model->nx;
            r.np = t.model->np;
            r.ldn = t.ld_node;
            std::memcpy(&img[p->rdesc_off + i * sizeof(RedDesc)], &r, sizeof(r));
        }
    }
    e = hipMemcpyAsync(d, img.data(), host_part, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) {
        plan_free(p);
        return fail(CIS_ERR_HIP, "cis_batch_plan_create: upload: %s", hipGetErrorString(e));
    }

    // tuning cache (CIS_SCHED_TUNE only)
    std::string cpath;
    std::map<std::string, TuneChoice> cache;
    bool cache_dirty = false;
    std::string dtag;
    if (sched == CIS_SCHED_TUNE) {
        const char* cp = std::getenv("CIS_TUNE_CACHE");
        if (cp && *cp) {
            cpath = cp;
            dtag = device_tag(p->device);
            std::lock_guard<std::mutex> lk(g_cache_mu);
            cache = cache_read(cpath);
        }
    }
    // launch records
    int ncu = 0;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device);
    if (ncu < 1) ncu = 1;
    for (Group& g : p->groups) {
        g.dev.fdesc = d + g.fdesc_off;
        g.dev.adesc = d + g.adesc_off;
        g.dev.items = (const int2*)(d + g.items_off);
        g.dev.n_items = (int)g.items.size();
        g.dev.cursor = (int*)(d + g.cursor_off);
        g.dev.rec = g.split_ok ? (void*)(p->recmem + g.rec_base * es) : nullptr;
        g.dev.rec_off = g.split_ok ? (const int64_t*)(d + g.recoff_off) : nullptr;
        cis_status st;
        std::string key;
        TuneChoice want, made;
        bool cached_all = !cpath.empty();
        if (!cpath.empty()) {
            int kmin = 1 << 30, kmax = 0, cmx = 1;
            for (int i : g.trajs) {
                kmin = std::min(kmin, trajs[i].substeps);
                kmax = std::max(kmax, trajs[i].substeps);
                cmx = std::max(cmx, p->ckpt_every[i]);
            }
            char kb[256];
            std::snprintf(kb, sizeof(kb), "%s|L%dD%d|%s|ops%d|items%zu|K%d-%d|C%d", dtag.c_str(),
                          g.model->L, g.model->D, dtype == CIS_F64 ? "f64" : "f32", (int)ops,
                          g.items.size(), kmin, kmax, (ops & CIS_BATCH_ADJOINT) ? cmx : 0);
            key = kb;
            auto it = cache.find(key);
            if (it != cache.end()) want = it->second;
        }
        if (ops & CIS_BATCH_DISCRETIZE) {
            // candidates: (grid | persistent) x register budget (1 or 2 waves
            // per SIMD; FP64 only has the second); the schedule bits fix some
            const int units = g.dev.n_items * g.units_per_item;
            struct Cand { KLaunch l, lb; int pblocks, waves; bool split; };
            std::vector<Cand> cands;
            if (g.split_ok) {
                for (int w = 1; w <= 2; ++w) {
                    if (waves_force ? w != waves_force : (sched != CIS_SCHED_TUNE && w != 1))
                        continue;
                    Cand c;
                    c.pblocks = 0;
                    c.waves = w;
                    c.split = true;
                    st = prep_split_batch(g.model, dtype, g.dev, w, &c.l, &c.lb);
                    if (st != CIS_OK) {
                        plan_free(p);
                        return st;
                    }
                    cands.push_back(c);
                }
            }
            for (int w = 1; w <= (dtype == CIS_F64 ? 2 : 1); ++w) {
                if (split_force == 1 && g.split_ok) break;
                if (waves_force ? w != waves_force : (sched != CIS_SCHED_TUNE && w != 1)) continue;
                KLaunch probe;
                st = prep_discretize_batch(g.model, dtype, g.dev, 1, w, &probe);
                if (st != CIS_OK) {
                    plan_free(p);
                    return st;
                }
                int occ = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, probe.func, probe.block.x,
                                                                 0) != hipSuccess || occ < 1)
                    occ = 1;
                const int pblocks = std::min(units, occ * ncu);
                for (int pers = 0; pers < 2; ++pers) {
                    if (sched == CIS_SCHED_GRID && pers) continue;
                    if (sched == CIS_SCHED_PERSISTENT && !pers) continue;
                    Cand c;
                    c.pblocks = pers ? pblocks : 0;
                    c.waves = w;
                    c.split = false;
                    st = prep_discretize_batch(g.model, dtype, g.dev, c.pblocks, w, &c.l);
                    if (st != CIS_OK) {
                        plan_free(p);
                        return st;
                    }
                    cands.push_back(c);
                }
            }
            size_t best = 0;
            bool hit = false;
            if (cands.size() > 1 && want.split >= 0) {
                for (size_t c = 0; c < cands.size(); ++c)
                    if ((cands[c].split ? 1 : 0) == want.split && cands[c].waves == want.waves &&
                        (cands[c].pblocks > 0 ? 1 : 0) == want.persist) {
                        best = c;
                        hit = true;
                        break;
                    }
            }
            if (cands.size() > 1 && !hit) {
                cached_all = false;
                float tbest = -1.f;
                for (size_t c = 0; c < cands.size(); ++c) {
                    const float t = cands[c].split ? time_pair(cands[c].l, cands[c].lb, hs, 3)
                                                   : time_launch(cands[c].l, hs, 3);
                    if (t < 0.f) {
                        plan_free(p);
                        return fail(CIS_ERR_HIP, "cis_batch_plan_create: tuning launch failed");
                    }
                    if (tbest < 0.f || t < tbest) {
                        tbest = t;
                        best = c;
                    }
                }
            }
            g.persist_blocks = cands[best].pblocks;
            g.disc_waves = cands[best].waves;
            g.disc = cands[best].l;
            g.split = cands[best].split;
            if (g.split) g.disc_b = cands[best].lb;
            made.split = g.split ? 1 : 0;
            made.waves = g.disc_waves;
            made.persist = g.persist_blocks > 0 ? 1 : 0;
        }
        if (ops & CIS_BATCH_ADJOINT) {
            BatchGroupDev dd = g.dev;
            dd.fdesc = d + g.ddesc_off;
            KLaunch def_body, def_lane;
            st = prep_defects_batch(g.model, dtype, dd, true, &def_body);
            if (st == CIS_OK) st = prep_defects_batch(g.model, dtype, dd, false, &def_lane);
            g.def = def_force == 2 ? def_lane : def_body;
            if (st == CIS_OK && sched == CIS_SCHED_TUNE && !def_force && want.def_lane >= 0) {
                g.def = want.def_lane ? def_lane : def_body;
            } else if (st == CIS_OK && sched == CIS_SCHED_TUNE && !def_force) {
                cached_all = false;
                const float tb = time_launch(def_body, hs, 3);
                const float tl = time_launch(def_lane, hs, 3);
                if (tb < 0.f || tl < 0.f) {
                    plan_free(p);
                    return fail(CIS_ERR_HIP, "cis_batch_plan_create: tuning launch failed");
                }
                if (tl < tb) g.def = def_lane;
            }
            int cmax_g = 1;
            for (int i : g.trajs) cmax_g = std::max(cmax_g, p->ckpt_every[i]);
            // reverse sweep with 4, 3, 2 or 1 waves per interval (latency vs
            // throughput): timed when tuning, else the three-wave form
            KLaunch adjv[4];
            for (int w = 0; w < 4 && st == CIS_OK; ++w)
                st = prep_adjoint_batch(g.model, g.dev, cmax_g, 4 - w, &adjv[w]);
            if (st != CIS_OK) {
                plan_free(p);
                return st;
            }
            made.def_lane = g.def.func == def_lane.func ? 1 : 0;
            int best = adj_force ? 4 - adj_force : 1;
            if (sched == CIS_SCHED_TUNE && !adj_force && want.adj_waves >= 1 && want.adj_waves <= 4) {
                best = 4 - want.adj_waves;
            } else if (sched == CIS_SCHED_TUNE && !adj_force) {
                cached_all = false;
                if (g.def.launch(hs) != hipSuccess || hipStreamSynchronize(hs) != hipSuccess) {
                    plan_free(p);
                    return fail(CIS_ERR_HIP, "cis_batch_plan_create: tuning launch failed");
                }
                float tbest = -1.f;
                for (int w = 0; w < 4; ++w) {
                    if (w > 0 && adjv[w].func == adjv[w - 1].func) continue;
                    const float tw = time_launch(adjv[w], hs, 3);
                    if (tw < 0.f) {
                        plan_free(p);
                        return fail(CIS_ERR_HIP, "cis_batch_plan_create: tuning launch failed");
                    }
                    if (tbest < 0.f || tw < tbest) {
                        tbest = tw;
                        best = w;
                    }
                }
            }
            g.adj = adjv[best];
            g.adj_waves = adjv[best].block.x / 64;
            g.def_waves = g.def.block.x / 64;
            made.adj_waves = 4 - best;
        }
        if (!cpath.empty()) {
            g.from_cache = cached_all;
            if (!cached_all) {
                cache[key] = made;
                cache_dirty = true;
            }
        }
    }
    if (cache_dirty) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        // merge with entries other plans wrote meanwhile, then replace the file
        std::map<std::string, TuneChoice> cur = cache_read(cpath);
        for (const auto& kv : cache) cur[kv.first] = kv.second;
        (void)cache_write(cpath, cur);
    }
    if (p->recmem) {
        bool used = false;
        for (const Group& g : p->groups) used = used || g.split;
        if (!used) {
            if (hipStreamSynchronize(hs) != hipSuccess) {
                plan_free(p);
                return fail(CIS_ERR_HIP, "cis_batch_plan_create: synchronization failed");
            }
            (void)hipFree(p->recmem);
            p->recmem = nullptr;
        }
    }
    if (ops & CIS_BATCH_ADJOINT) {
        cis_status st = prep_adjoint_reduce_batch(d + p->rdesc_off, n_traj, &p->red);
        if (st != CIS_OK) {
            plan_free(p);
            return st;
        }
    }
    if (graph) {
        for (int op : {CIS_BATCH_DISCRETIZE, CIS_BATCH_ADJOINT}) {
            if (!(ops & op)) continue;
            cis_status st = build_graph(p, op);
            if (st != CIS_OK) {
                plan_free(p);
                return st;
            }
        }
    }
    *out = p;
    return CIS_OK;
}

extern "C" cis_status cis_batch_run(cis_batch_plan* p, int32_t op, void* stream) {
    if (!p) return fail(CIS_ERR_NULL, "cis_batch_run: plan is required");
    if ((op != CIS_BATCH_DISCRETIZE && op != CIS_BATCH_ADJOINT) || !(p->ops & op))
        return fail(CIS_ERR_DIM, "cis_batch_run: operation %d was not planned", op);
    hipStream_t hs = (hipStream_t)stream;
    for (Group& g : p->groups) {
        hipError_t e;
        if (op == CIS_BATCH_DISCRETIZE) {
            e = g.disc.launch(hs);
            if (e == hipSuccess && g.split) e = g.disc_b.launch(hs);
        } else {
            e = g.def.launch(hs);
            if (e == hipSuccess) e = g.adj.launch(hs);
        }
        if (e != hipSuccess) return fail(CIS_ERR_HIP, "cis_batch_run: launch: %s", hipGetErrorString(e));
    }
    if (op == CIS_BATCH_ADJOINT) {
        hipError_t e = p->red.launch(hs);
        if (e != hipSuccess) return fail(CIS_ERR_HIP, "cis_batch_run: reduction launch: %s", hipGetErrorString(e));
    }
    return CIS_OK;
}

extern "C" cis_status cis_batch_run_part(cis_batch_plan* p, int32_t op, int32_t part,
                                         void* stream) {
    if (!p) return fail(CIS_ERR_NULL, "cis_batch_run_part: plan is required");
    if ((op != CIS_BATCH_DISCRETIZE && op != CIS_BATCH_ADJOINT) || !(p->ops & op))
        return fail(CIS_ERR_DIM, "cis_batch_run_part: operation %d was not planned", op);
    if (part != 0 && part != 1 && !(op == CIS_BATCH_ADJOINT && part == 2))
        return fail(CIS_ERR_DIM, "cis_batch_run_part: part %d out of range", part);
    hipStream_t hs = (hipStream_t)stream;
    for (Group& g : p->groups) {
        hipError_t e = hipSuccess;
        if (op == CIS_BATCH_DISCRETIZE) {
            if (part == 0) e = g.disc.launch(hs);
            else if (g.split) e = g.disc_b.launch(hs);
        } else if (part == 0) {
            e = g.def.launch(hs);
        } else if (part == 1) {
            e = g.adj.launch(hs);
        }
        if (e != hipSuccess)
            return fail(CIS_ERR_HIP, "cis_batch_run_part: launch: %s", hipGetErrorString(e));
    }
    if (op == CIS_BATCH_ADJOINT && part == 2) {
        hipError_t e = p->red.launch(hs);
        if (e != hipSuccess)
            return fail(CIS_ERR_HIP, "cis_batch_run_part: reduction launch: %s", hipGetErrorString(e));
    }
    return CIS_OK;
}

extern "C" cis_status cis_batch_graph_run(cis_batch_plan* p, int32_t op, void* stream) {
    if (!p) return fail(CIS_ERR_NULL, "cis_batch_graph_run: plan is required");
    if ((op != CIS_BATCH_DISCRETIZE && op != CIS_BATCH_ADJOINT) || !(p->ops & op))
        return fail(CIS_ERR_DIM, "cis_batch_graph_run: operation %d was not planned", op);
    const int gi = op == CIS_BATCH_DISCRETIZE ? 0 : 1;
    if (!p->exec[gi]) return fail(CIS_ERR_DIM, "cis_batch_graph_run: the plan was created without graphs");
    hipError_t e = hipGraphLaunch(p->exec[gi], (hipStream_t)stream);
    if (e != hipSuccess) return fail(CIS_ERR_HIP, "cis_batch_graph_run: %s", hipGetErrorString(e));
    return CIS_OK;
}

extern "C" cis_status cis_batch_plan_info(const cis_batch_plan* p, int32_t g, int32_t* groups,
                                          int32_t* n_traj, int32_t* n_items,
                                          int32_t* units_per_item, int32_t* persist_blocks,
                                          int32_t* adjoint_waves, int32_t* waves_per_simd,
                                          int32_t* defects_waves) {
    if (!p) return fail(CIS_ERR_NULL, "cis_batch_plan_info: plan is required");
    if (groups) *groups = (int32_t)p->groups.size();
    if (g < 0 || g >= (int32_t)p->groups.size()) return CIS_OK;
    const Group& gr = p->groups[g];
    if (n_traj) *n_traj = (int32_t)gr.trajs.size();
    if (n_items) *n_items = (int32_t)gr.items.size();
    if (units_per_item) *units_per_item = gr.units_per_item;
    if (persist_blocks) *persist_blocks = gr.persist_blocks;
    if (adjoint_waves) *adjoint_waves = gr.adj_waves;
    if (waves_per_simd) *waves_per_simd = gr.disc_waves;
    if (defects_waves) *defects_waves = gr.def_waves;
    return CIS_OK;
}

extern "C" cis_status cis_batch_plan_discretize_form(const cis_batch_plan* p, int32_t g,
                                                     int32_t* split, int32_t* tangent_waves) {
    if (!p) return fail(CIS_ERR_NULL, "cis_batch_plan_discretize_form: plan is required");
    if (g < 0 || g >= (int32_t)p->groups.size())
        return fail(CIS_ERR_DIM, "cis_batch_plan_discretize_form: group %d out of range", g);
    const Group& gr = p->groups[g];
    if (split) *split = gr.split ? 1 : 0;
    if (tangent_waves) *tangent_waves = gr.split ? gr.disc_waves : 0;
    return CIS_OK;
}

extern "C" cis_status cis_batch_plan_tuned_from_cache(const cis_batch_plan* p, int32_t g,
                                                      int32_t* from_cache) {
    if (!p || !from_cache) return fail(CIS_ERR_NULL, "cis_batch_plan_tuned_from_cache: null argument");
    if (g < 0 || g >= (int32_t)p->groups.size())
        return fail(CIS_ERR_DIM, "cis_batch_plan_tuned_from_cache: group %d out of range", g);
    *from_cache = p->groups[g].from_cache ? 1 : 0;
    return CIS_OK;
}

extern "C" void cis_batch_plan_destroy(cis_batch_plan* p) {
    if (!p) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    plan_free(p);
    (void)hipSetDevice(cur);
}
