// Ragged batches: ensembles of realizations (classical-field or truncated-Wigner
// samples, section 1) of possibly different lattice shapes, expanded in one go.
//
// Problems that are identical up to their input field form a shape class and
// share one plan; a class runs in groups of G realizations stacked as the
// leading slice dimension of the pass tensors, so every pass of the schedule
// covers G fields at once. Per group: gather the caller's G input pointers
// into a contiguous staging tensor, run the plan's passes, scatter the field
// and density to the caller's outputs. The whole sequence over all classes
// and groups is captured once into a HIP graph and replayed with a single
// graph launch per run; the transform passes inside run as persistent grids
// (a capped number of workgroups looping over the tile list) when the
// autotuner finds that faster.
//
// Autotuning (per class, at batch creation): every candidate (preferred tile
// size, persistent grid or not, fused or split 1-D expansion passes) runs one
// group eagerly, timed with HIP events; the fastest is kept. Results are cached
// per process and, with FX_AUTOTUNE_CACHE=<file>, on disk.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "plan.h"

using namespace fx;

namespace {

struct Tune {
    int ts_target = 2048;
    int persist = 0;
    bool allow_split = true;
};

std::mutex g_tune_mu;
std::map<std::string, Tune> g_tune;
bool g_tune_loaded = false;

std::string class_key(const fx_problem& p, int64_t group) {
    std::ostringstream o;
    o << p.ndim << ":";
    for (int j = 0; j < p.ndim; ++j) o << p.shape[j] << "x" << p.lambda[j] << ",";
    o << "prec" << p.precision << ":sched" << p.schedule << ":G" << group;
    return o.str();
}

void load_tune_cache() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("FX_AUTOTUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string key;
    Tune t;
    int split = 1;
    while (f >> key >> t.ts_target >> t.persist >> split) {
        t.allow_split = split != 0;
        g_tune[key] = t;
    }
}

void save_tune_cache() {
    const char* path = std::getenv("FX_AUTOTUNE_CACHE");
    if (!path) return;
    std::ofstream f(path);
    for (const auto& kv : g_tune)
        f << kv.first << " " << kv.second.ts_target << " " << kv.second.persist << " "
          << (kv.second.allow_split ? 1 : 0) << "\n";
}

bool same_problem(const fx_problem& a, const fx_problem& b) {
    if (a.ndim != b.ndim || a.precision != b.precision || a.schedule != b.schedule) return false;
    if (a.m_over_hbar != b.m_over_hbar || a.t_flight != b.t_flight) return false;
    for (int j = 0; j < a.ndim; ++j) {
        if (a.shape[j] != b.shape[j] || a.lambda[j] != b.lambda[j] || a.dx[j] != b.dx[j]) return false;
        auto eq = [](double x, double y) { return (std::isnan(x) && std::isnan(y)) || x == y; };
        if (!eq(a.a[j], b.a[j]) || !eq(a.abar[j], b.abar[j])) return false;
    }
    return true;
}

}  // namespace

struct fx_batch {
    struct Class {
        fx_plan* plan = nullptr;
        std::vector<int> members;
        int64_t group = 1;
        Tune tune;
    };
    int n = 0;
    bool dbl = false;
    std::vector<Class> classes;
    void* stage_in = nullptr;  // max group * M of any class
    size_t stage_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t g_stream = nullptr;
    std::vector<const void*> g_in;
    std::vector<void*> g_out, g_rho;
};

namespace {

size_t cbytes(const fx_batch* b) { return b->dbl ? 16 : 8; }

void apply_tune(fx_plan* p, const Tune& t) {
    p->ts_target = t.ts_target;
    p->persist = t.persist;
    p->allow_split = t.allow_split;
}

// Enqueues one class group: gather -> passes -> scatter.
fx_status run_group(fx_batch* b, fx_batch::Class& c, size_t first, size_t count, const void* const* psi0,
                    void* const* psi_out, void* const* rho_out, hipStream_t st) {
    fx_plan* p = c.plan;
    const int64_t M = p->M;
    const size_t cs = cbytes(b);
    for (size_t off = 0; off < count; off += 64) {
        const int cnt = (int)std::min<size_t>(64, count - off);
        const void* srcs[64];
        for (int i = 0; i < cnt; ++i) srcs[i] = psi0[c.members[first + off + i]];
        if (launch_gather(b->dbl, srcs, (char*)b->stage_in + off * M * cs, M, cnt, st) != hipSuccess) {
            set_error("gather launch failed");
            return FX_EDEVICE;
        }
    }
    void* dst = (char*)p->ws + (size_t)2 * p->buf_elems * cs;  // the plan's output staging region
    int qb[3] = {0, 0, 0}, qn[3] = {p->ax[0].lam, p->ax[1].lam, p->ax[2].lam};
    fx_status s = run_box(p, qb, qn, b->stage_in, dst, 0, nullptr, false, st);
    if (s != FX_OK) return s;
    for (size_t off = 0; off < count; off += 64) {
        const int cnt = (int)std::min<size_t>(64, count - off);
        void* outs[64];
        void* rhos[64];
        for (int i = 0; i < cnt; ++i) {
            const int m = c.members[first + off + i];
            outs[i] = psi_out ? psi_out[m] : nullptr;
            rhos[i] = rho_out ? rho_out[m] : nullptr;
        }
        if (launch_scatter(b->dbl, (char*)dst + off * M * cs, outs, M, cnt, rho_out ? 1 : 0, rhos, st) !=
            hipSuccess) {
            set_error("scatter launch failed");
            return FX_EDEVICE;
        }
    }
    return FX_OK;
}

fx_status run_all(fx_batch* b, const void* const* psi0, void* const* psi_out, void* const* rho_out, hipStream_t st) {
    for (auto& c : b->classes) {
        for (size_t first = 0; first < c.members.size(); first += (size_t)c.group) {
            const size_t count = std::min<size_t>((size_t)c.group, c.members.size() - first);
            if ((int64_t)count != c.plan->slices) plan_setup_workspace(c.plan, (int64_t)count);
            fx_status s = run_group(b, c, first, count, psi0, psi_out, rho_out, st);
            if (s != FX_OK) return s;
        }
    }
    return FX_OK;
}

void drop_graph(fx_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Times a group of `count` realizations of class c with tuning t (eager launches, HIP events).
// Returns ms or -1.
double time_group(fx_batch* b, fx_batch::Class& c, const Tune& t, size_t count, hipStream_t st) {
    apply_tune(c.plan, t);
    plan_setup_workspace(c.plan, (int64_t)count);
    if (c.plan->ws_need > c.plan->ws_bytes) return -1.0;
    std::vector<const void*> in(b->n, b->stage_in);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -1.0; }
    // the staging input doubles as every member's source; outputs are not written (nullptr)
    double best = -1.0;
    for (int rep = 0; rep < 2; ++rep) {
        (void)hipEventRecord(e0, st);
        fx_status s = run_group(b, c, 0, count, in.data(), nullptr, nullptr, st);
        (void)hipEventRecord(e1, st);
        if (s != FX_OK || hipEventSynchronize(e1) != hipSuccess) { best = -1.0; break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep == 1) best = ms;  // first repetition warms caches and LDS attributes
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

}  // namespace

extern "C" {

fx_status fx_batch_create(const fx_problem* probs, int32_t n, fx_batch** out) {
    if (!out) { set_error("out is NULL"); return FX_EINVAL; }
    if (!probs || n < 1) { set_error("need at least one problem"); return FX_EINVAL; }
    for (int i = 0; i < n; ++i) {
        fx_status s = validate(&probs[i]);
        if (s != FX_OK) return s;
        if (probs[i].precision != probs[0].precision) {
            set_error("all problems of a batch must share one precision");
            return FX_EINVAL;
        }
    }
    fx_batch* b = new (std::nothrow) fx_batch();
    if (!b) { set_error("host allocation failed"); return FX_ENOMEM; }
    b->n = n;
    b->dbl = probs[0].precision == FX_PREC_C128;
    for (int i = 0; i < n; ++i) {
        bool found = false;
        for (auto& c : b->classes) {
            if (same_problem(c.plan->prob_in, probs[i])) {
                c.members.push_back(i);
                found = true;
                break;
            }
        }
        if (found) continue;
        fx_batch::Class c;
        fx_status s = fx_plan_create(&probs[i], &c.plan);
        if (s != FX_OK) {
            fx_batch_destroy(b);
            return s;
        }
        c.plan->prob_in = probs[i];
        c.members.push_back(i);
        b->classes.push_back(c);
    }
    // group sizes: as many realizations per group as fit the plan's workspace budget
    const size_t cs = cbytes(b);
    size_t stage_elems = 0;
    for (auto& c : b->classes) {
        int64_t G = (int64_t)c.members.size();
        while (G > 1) {
            plan_setup_workspace(c.plan, G);
            if (c.plan->ws_need <= c.plan->budget) break;
            G = (G + 1) / 2;
        }
        c.group = G;
        plan_setup_workspace(c.plan, G);
        c.plan->nb_fixed = c.plan->nb_outer;
        fx_status s = ensure_workspace(c.plan);
        if (s != FX_OK) { fx_batch_destroy(b); return s; }
        stage_elems = std::max(stage_elems, (size_t)(G * c.plan->M));
    }
    if (hipMalloc(&b->stage_in, stage_elems * cs) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of batch staging failed");
        fx_batch_destroy(b);
        return FX_ENOMEM;
    }
    b->stage_bytes = stage_elems * cs;
    if (hipMemset(b->stage_in, 0, b->stage_bytes) != hipSuccess) { fx_batch_destroy(b); return FX_EDEVICE; }
    // autotune per class (eager runs), then keep the winner
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache();
    const bool tune = std::getenv("FX_NO_AUTOTUNE") == nullptr;
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) { fx_batch_destroy(b); return FX_EDEVICE; }
    bool dirty = false;
    for (auto& c : b->classes) {
        const std::string key = class_key(c.plan->prob, c.group);
        auto it = g_tune.find(key);
        Tune best;
        if (it != g_tune.end()) {
            best = it->second;
        } else if (tune) {
            double best_ms = -1.0;
            // a few realizations per timing run keep the search short; the choice only concerns
            // tile shapes and grid sizes, which depend on the lattice, not on the group size
            const size_t tune_count = (size_t)std::min<int64_t>(c.group, 2);
            const int ts_c[] = {1024, 2048, 4096};
            const int pe_c[] = {0, 4};
            const bool sp_c[] = {true, false};
            for (int ts : ts_c)
                for (int pe : pe_c)
                    for (bool sp : sp_c) {
                        Tune t;
                        t.ts_target = ts;
                        t.persist = pe;
                        t.allow_split = sp;
                        const double ms = time_group(b, c, t, tune_count, st);
                        if (ms >= 0 && (best_ms < 0 || ms < best_ms)) {
                            best_ms = ms;
                            best = t;
                        }
                    }
            g_tune[key] = best;
            dirty = true;
        }
        c.tune = best;
        apply_tune(c.plan, best);
        plan_setup_workspace(c.plan, c.group);
        fx_status s = ensure_workspace(c.plan);
        if (s != FX_OK) { (void)hipStreamDestroy(st); fx_batch_destroy(b); return s; }
        // eager runs (full group and the last partial one) so that every kernel the graph will hold
        // has been launched once before any capture
        std::vector<const void*> in(n, b->stage_in);
        s = run_group(b, c, 0, (size_t)c.group, in.data(), nullptr, nullptr, st);
        const size_t rem = c.members.size() % (size_t)c.group;
        if (s == FX_OK && rem) {
            plan_setup_workspace(c.plan, (int64_t)rem);
            s = run_group(b, c, 0, rem, in.data(), nullptr, nullptr, st);
            plan_setup_workspace(c.plan, c.group);
        }
        if (s != FX_OK) { (void)hipStreamDestroy(st); fx_batch_destroy(b); return s; }
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("batch set-up run failed");
        (void)hipStreamDestroy(st);
        fx_batch_destroy(b);
        return FX_EDEVICE;
    }
    (void)hipStreamDestroy(st);
    if (dirty) save_tune_cache();
    *out = b;
    return FX_OK;
}

fx_status fx_batch_destroy(fx_batch* b) {
    if (!b) return FX_OK;
    drop_graph(b);
    for (auto& c : b->classes) fx_plan_destroy(c.plan);
    if (b->stage_in) (void)hipFree(b->stage_in);
    delete b;
    return FX_OK;
}

fx_status fx_batch_run(fx_batch* b, const void* const* psi0, void* const* psi_out, void* const* rho_out,
                       void* stream) {
    if (!b) { set_error("batch is NULL"); return FX_EINVAL; }
    if (!psi0) { set_error("psi0 array is NULL"); return FX_EINVAL; }
    if (!psi_out && !rho_out) { set_error("psi_out and rho_out are both NULL"); return FX_EINVAL; }
    for (int i = 0; i < b->n; ++i) {
        if (!psi0[i]) { set_error("psi0[i] is NULL"); return FX_EINVAL; }
        const bool has_psi = psi_out && psi_out[i];
        const bool has_rho = rho_out && rho_out[i];
        if (!has_psi && !has_rho) { set_error("realization without any output"); return FX_EINVAL; }
    }
    hipStream_t st = (hipStream_t)stream;
    if (st == nullptr || std::getenv("FX_NO_GRAPH")) return run_all(b, psi0, psi_out, rho_out, st);
    std::vector<const void*> in(psi0, psi0 + b->n);
    std::vector<void*> o(b->n, nullptr), r(b->n, nullptr);
    for (int i = 0; i < b->n; ++i) {
        if (psi_out) o[i] = psi_out[i];
        if (rho_out) r[i] = rho_out[i];
    }
    const bool same = b->exec && st == b->g_stream && in == b->g_in && o == b->g_out && r == b->g_rho;
    if (!same) {
        drop_graph(b);
        for (auto& c : b->classes) c.plan->timing = false;
        FX_TRY_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        fx_status s = run_all(b, psi0, psi_out, rho_out, st);
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(st, &g);
        if (s != FX_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (ce != hipSuccess) {
            set_error(std::string("graph capture failed: ") + hipGetErrorString(ce));
            return FX_EDEVICE;
        }
        b->graph = g;
        FX_TRY_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
        b->g_stream = st;
        b->g_in = in;
        b->g_out = o;
        b->g_rho = r;
    }
    FX_TRY_HIP(hipGraphLaunch(b->exec, st));
    return FX_OK;
}

}  // extern "C"
