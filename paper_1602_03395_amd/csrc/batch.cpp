// Ragged batches: ensembles of realizations (classical-field or truncated-Wigner
// samples, section 1) of possibly different lattice shapes, expanded in one go.
//
// Problems that are identical up to their input field form a shape class and
// share one plan. A class is cut into work items of G realizations by one block
// of the outermost magnification index (the q-block): an item stacks its G
// fields as the leading slice dimension of every pass of the schedule, so each
// kernel launch of the item covers G fields and a range of terms q at once, and
// the q-blocks of an item accumulate into its output (the sequential
// accumulation over q of section 7.1). Per item group: gather the caller's G
// input pointers into the class's staging tensor, run the passes over every
// q-block, scatter the field and density to the caller's outputs.
//
// Classes are independent, so each class runs on a lane stream of its own: the
// run forks from the caller's stream into the lanes and joins back, and the
// largest classes (by terms x points x members) are issued first. The whole
// fork-join sequence is captured once into a HIP graph, whose parallel branches
// let the device interleave the kernels of different classes (one class's tail
// waves fill with another's work), and replayed with a single graph launch per
// run. Inside a class the transform passes run as persistent grids where the
// tuner finds that faster.
//
// Autotuning (per class, at batch creation): first the item shape, over the
// frontier of realizations per item G against the q-block that the workspace
// budget allows; then coordinate descent from the best shape over the transform
// family (register-resident lane transforms or LDS Stockham radix-8/4/2 stages),
// the fused (one wave per tile, or eight waves sharing the terms) or split
// structured accumulate, the LDS tile size and persistent grids. Each candidate
// runs one full item eagerly three times, timed with HIP events, and the best of
// the last two runs per realization counts. Then the lane concurrency (all
// classes in parallel, or one after the other) is decided on whole runs of the
// batch, alternating between the two forms; before that, whether the largest class
// runs as two or three replicas (plans and workspaces of their own, a share of its
// items each, on lanes of their own, so that several of its items run at once) is
// decided on whole runs as well. Results are cached per process and, with
// FX_AUTOTUNE_CACHE=<file>, on disk.
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
    bool use_cfp = true;
    int use_eas = 1;
    bool use_eaw = true;
    int64_t group = 0;  // realizations per item (0: the largest that fits the workspace budget)
    int64_t qblock = 0; // outermost magnification indices per q-block (0: as the budget allows)
    bool operator==(const Tune& o) const {
        return ts_target == o.ts_target && persist == o.persist && allow_split == o.allow_split &&
               use_cfp == o.use_cfp && use_eas == o.use_eas && use_eaw == o.use_eaw && group == o.group &&
               qblock == o.qblock;
    }
};

std::mutex g_tune_mu;
std::map<std::string, Tune> g_tune;
std::map<std::string, int> g_conc;
std::map<std::string, int> g_repl;  // replicas of the largest class per batch key
bool g_tune_loaded = false;

std::string class_key(const fx_problem& p, size_t members) {
    std::ostringstream o;
    o << p.ndim << ":";
    for (int j = 0; j < p.ndim; ++j) o << p.shape[j] << "x" << p.lambda[j] << ",";
    o << "prec" << p.precision << ":sched" << p.schedule << ":n" << members;
    return o.str();
}

void load_tune_cache() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("FX_AUTOTUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string kind, key;
    while (f >> kind >> key) {
        if (kind == "class") {
            Tune t;
            int split = 1, cfp = 1, eaw = 1;
            long long g = 0, qb = 0;
            if (!(f >> t.ts_target >> t.persist >> split >> cfp >> t.use_eas >> eaw >> g >> qb)) break;
            t.allow_split = split != 0;
            t.use_cfp = cfp != 0;
            t.use_eaw = eaw != 0;
            t.group = g;
            t.qblock = qb;
            g_tune[key] = t;
        } else if (kind == "batch") {
            int c = 1, r = 1;
            if (!(f >> c >> r)) break;
            g_conc[key] = c;
            g_repl[key] = r;
        } else {
            break;
        }
    }
}

void save_tune_cache() {
    const char* path = std::getenv("FX_AUTOTUNE_CACHE");
    if (!path) return;
    std::ofstream f(path);
    for (const auto& kv : g_tune)
        f << "class " << kv.first << " " << kv.second.ts_target << " " << kv.second.persist << " "
          << (kv.second.allow_split ? 1 : 0) << " " << (kv.second.use_cfp ? 1 : 0) << " " << kv.second.use_eas << " "
          << (kv.second.use_eaw ? 1 : 0) << " " << kv.second.group << " " << kv.second.qblock << "\n";
    for (const auto& kv : g_conc) {
        auto r = g_repl.find(kv.first);
        f << "batch " << kv.first << " " << kv.second << " " << (r != g_repl.end() ? r->second : 1) << "\n";
    }
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
        int64_t group = 1;      // realizations per item
        Tune tune;
        void* stage = nullptr;  // gather target: group * M input values
        size_t stage_bytes = 0;
        int lane = 0;
        double cost = 0;        // terms x points x members (issue order)
    };
    int n = 0;
    bool dbl = false;
    std::vector<Class> classes;  // in issue order (largest cost first)
    int concurrency = 1;         // lanes in use (1: every class on the caller's stream)
    int tuned_concurrency = 1;   // the value batch creation chose
    std::vector<hipStream_t> lanes;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t g_stream = nullptr;
    std::vector<const void*> g_in;
    std::vector<void*> g_out, g_rho;
};

namespace {

size_t cbytes(const fx_batch* b) { return b->dbl ? 16 : 8; }

// Applies the tuning knobs to the class plan and lays out its workspace for G realizations.
void apply_tune(fx_plan* p, const Tune& t, int64_t G) {
    p->ts_target = t.ts_target;
    p->persist = t.persist;
    p->allow_split = t.allow_split;
    p->use_cfp = t.use_cfp;
    p->use_eas = t.use_eas;
    p->use_eaw = t.use_eaw;
    p->nb_fixed = t.qblock;
    plan_setup_workspace(p, G);
}

fx_status ensure_stage(fx_batch* b, fx_batch::Class& c, int64_t G) {
    const size_t need = (size_t)(G * c.plan->M) * cbytes(b);
    if (c.stage && c.stage_bytes >= need) return FX_OK;
    if (c.stage) (void)hipFree(c.stage);
    c.stage = nullptr;
    c.stage_bytes = 0;
    if (hipMalloc(&c.stage, need) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of batch staging failed");
        return FX_ENOMEM;
    }
    c.stage_bytes = need;
    // the tuner reads the staging tensor as every realization's input: give it defined values
    if (hipMemset(c.stage, 0, need) != hipSuccess) {
        set_error("clearing the batch staging failed");
        return FX_EDEVICE;
    }
    return FX_OK;
}

// Enqueues one item group: gather -> passes over every q-block -> scatter.
fx_status run_group(fx_batch* b, fx_batch::Class& c, size_t first, size_t count, const void* const* psi0,
                    void* const* psi_out, void* const* rho_out, hipStream_t st) {
    fx_plan* p = c.plan;
    const int64_t M = p->M;
    const size_t cs = cbytes(b);
    for (size_t off = 0; off < count; off += 64) {
        const int cnt = (int)std::min<size_t>(64, count - off);
        const void* srcs[64];
        for (int i = 0; i < cnt; ++i) srcs[i] = psi0[c.members[first + off + i]];
        if (launch_gather(b->dbl, srcs, (char*)c.stage + off * M * cs, M, cnt, st) != hipSuccess) {
            set_error("gather launch failed");
            return FX_EDEVICE;
        }
    }
    void* dst = (char*)p->ws + (size_t)2 * p->buf_elems * cs;  // the plan's output staging region
    int qb[3] = {0, 0, 0}, qn[3] = {p->ax[0].lam, p->ax[1].lam, p->ax[2].lam};
    fx_status s = run_box(p, qb, qn, c.stage, dst, 0, nullptr, false, st);
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

// Every item of one class, in member order, on stream st.
fx_status run_class(fx_batch* b, fx_batch::Class& c, const void* const* psi0, void* const* psi_out,
                    void* const* rho_out, hipStream_t st) {
    for (size_t first = 0; first < c.members.size(); first += (size_t)c.group) {
        const size_t count = std::min<size_t>((size_t)c.group, c.members.size() - first);
        if ((int64_t)count != c.plan->slices) plan_setup_workspace(c.plan, (int64_t)count);
        fx_status s = run_group(b, c, first, count, psi0, psi_out, rho_out, st);
        if (s != FX_OK) return s;
    }
    if (c.plan->slices != c.group) plan_setup_workspace(c.plan, c.group);
    return FX_OK;
}

// Forks the lanes from st (every lane waits for what st holds so far).
fx_status fork_lanes(fx_batch* b, int L, hipStream_t st) {
    FX_TRY_HIP(hipEventRecord(b->fork, st));
    for (int k = 0; k < L; ++k) FX_TRY_HIP(hipStreamWaitEvent(b->lanes[k], b->fork, 0));
    return FX_OK;
}

// Joins the lanes back into st (st waits for everything the lanes hold).
fx_status join_lanes(fx_batch* b, int L, hipStream_t st) {
    for (int k = 0; k < L; ++k) {
        FX_TRY_HIP(hipEventRecord(b->joins[k], b->lanes[k]));
        FX_TRY_HIP(hipStreamWaitEvent(st, b->joins[k], 0));
    }
    return FX_OK;
}

// The classes on their lanes: fork from st, one lane per class (classes beyond the lane count share
// lanes round-robin in issue order), join back into st. With one lane every class runs on st.
fx_status run_all(fx_batch* b, const void* const* psi0, void* const* psi_out, void* const* rho_out, hipStream_t st) {
    if (b->concurrency <= 1) {
        for (auto& c : b->classes) {
            fx_status s = run_class(b, c, psi0, psi_out, rho_out, st);
            if (s != FX_OK) return s;
        }
        return FX_OK;
    }
    const int L = b->concurrency;
    fx_status s = fork_lanes(b, L, st);
    if (s != FX_OK) return s;
    for (auto& c : b->classes) {
        s = run_class(b, c, psi0, psi_out, rho_out, b->lanes[c.lane % L]);
        if (s != FX_OK) break;
    }
    // join even after a failed enqueue, so that st never runs ahead of work already on the lanes
    fx_status sj = join_lanes(b, L, st);
    return s != FX_OK ? s : sj;
}

void drop_graph(fx_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = false;
    Timer() { ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess; }
    ~Timer() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Times one item of class c (G realizations, every q-block) with tuning t; returns ms per
// realization or -1 when the tuning does not fit (workspace budget, 32-bit indexing) or fails.
double time_item(fx_batch* b, fx_batch::Class& c, const Tune& t, hipStream_t st) {
    const int64_t G = t.group;
    apply_tune(c.plan, t, G);
    if (!c.plan->index_ok || c.plan->ws_need > c.plan->budget) return -1.0;
    if (ensure_workspace(c.plan) != FX_OK || ensure_stage(b, c, G) != FX_OK) return -1.0;
    std::vector<const void*> in(b->n, c.stage);  // the staging tensor doubles as every input
    Timer tm;
    double best = -1.0;
    if (tm.ok) {
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(tm.e0, st);
            fx_status s = run_group(b, c, 0, (size_t)G, in.data(), nullptr, nullptr, st);
            (void)hipEventRecord(tm.e1, st);
            if (s != FX_OK || hipEventSynchronize(tm.e1) != hipSuccess) { best = -1.0; break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, tm.e0, tm.e1);
            // the first repetition sets LDS attributes and warms caches; the best of the others counts
            if (rep >= 1 && (best < 0 || ms / (double)G < best)) best = ms / (double)G;
        }
    }
    (void)hipGetLastError();
    return best;
}

// The largest item (<= members) whose workspace fits the budget at the tuning's q-block.
int64_t largest_group(fx_batch::Class& c, Tune t) {
    int64_t G = (int64_t)c.members.size();
    while (G > 1) {
        apply_tune(c.plan, t, G);
        if (c.plan->ws_need <= c.plan->budget && c.plan->index_ok) break;
        G = (G + 1) / 2;
    }
    return G;
}

// The largest item (<= members) whose workspace fits the budget at q-block qb.
int64_t largest_group_at(fx_batch::Class& c, Tune t, int64_t qb) {
    t.qblock = qb;
    return largest_group(c, t);
}

// Autotuning of one class. First the item shape: the workspace holds G realizations times a
// q-block of the outermost magnification index, so the candidates are the points of that frontier
// (for every q-block lam, lam/2, ..., 1 the largest G that fits, and half of it), from one
// realization with every term in one block (the single-field layout) to many realizations with
// short blocks. Then coordinate descent over the kernel knobs from the best item shape.
Tune tune_class(fx_batch* b, fx_batch::Class& c, hipStream_t st) {
    const int k = c.plan->nact;
    const int64_t lam_outer = k > 0 ? c.plan->ax[c.plan->act[k - 1]].lam : 1;
    Tune best;
    double best_ms = -1.0;
    auto consider = [&](Tune t) {
        if (t.group < 1) return;
        if (best_ms >= 0 && t == best) return;
        const double ms = time_item(b, c, t, st);
        if (ms >= 0 && (best_ms < 0 || ms < best_ms * 0.995)) {
            best_ms = ms;
            best = t;
        }
    };
    std::vector<int64_t> qbs;
    for (int64_t qb = lam_outer; qb >= 1; qb = (qb > 1) ? (qb + 1) / 2 : 0) {
        if (qbs.empty() || qbs.back() != qb) qbs.push_back(qb);
        if (qb == 1) break;
    }
    for (int64_t qb : qbs) {
        Tune t;
        t.qblock = qb;
        t.group = largest_group_at(c, t, qb);
        apply_tune(c.plan, t, t.group);
        if (c.plan->nb_outer != qb && qb != lam_outer) continue;  // the budget cut the block: a smaller one follows
        consider(t);
        if (t.group > 1) {
            t.group = (t.group + 1) / 2;
            consider(t);
        }
    }
    for (int sweep = 0; sweep < 2; ++sweep) {
        for (bool v : {true, false}) { Tune t = best; t.use_cfp = v; consider(t); }
        for (bool v : {true, false}) { Tune t = best; t.use_eaw = v; consider(t); }
        for (int v : {0, 1, 2}) { Tune t = best; t.use_eas = v; consider(t); }
        for (bool v : {true, false}) { Tune t = best; t.allow_split = v; consider(t); }
        for (int v : {0, 4}) { Tune t = best; t.persist = v; consider(t); }
        for (int v : {1024, 2048, 4096}) { Tune t = best; t.ts_target = v; consider(t); }
    }
    if (best.group < 1) {
        best = Tune();
        best.group = largest_group(c, best);
    }
    if (best.qblock == 0) {
        apply_tune(c.plan, best, best.group);
        best.qblock = c.plan->nb_outer;
    }
    return best;
}

// ms of one whole run of the batch (every item of every class, each class's staging tensor as the
// input of all its realizations, no outputs) with the given lane count; -1 on failure.
double time_full(fx_batch* b, int lanes, hipStream_t st) {
    Timer tm;
    if (!tm.ok) return -1.0;
    const int saved = b->concurrency;
    b->concurrency = lanes;
    double ms_out = -1.0;
    (void)hipEventRecord(tm.e0, st);
    fx_status s = lanes > 1 ? fork_lanes(b, lanes, st) : FX_OK;
    for (auto& c : b->classes) {
        if (s != FX_OK) break;
        std::vector<const void*> in(b->n, c.stage);
        s = run_class(b, c, in.data(), nullptr, nullptr, lanes > 1 ? b->lanes[c.lane % lanes] : st);
    }
    if (lanes > 1) (void)join_lanes(b, lanes, st);
    (void)hipEventRecord(tm.e1, st);
    if (s == FX_OK && hipEventSynchronize(tm.e1) == hipSuccess) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, tm.e0, tm.e1);
        ms_out = ms;
    }
    b->concurrency = saved;
    (void)hipGetLastError();
    return ms_out;
}

// Adds a lane stream (and its join event) for one more class.
fx_status add_lane(fx_batch* b) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        set_error("creating a batch lane failed");
        return FX_EDEVICE;
    }
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(s);
        set_error("creating a batch lane failed");
        return FX_EDEVICE;
    }
    b->lanes.push_back(s);
    b->joins.push_back(e);
    return FX_OK;
}

// Splits class k: its members after the first keep_items items (0: half of them) go to a copy of the
// class with a plan and workspace of its own, issued right after it on a lane of its own, so that
// items of both run at once. Returns FX_EUNSUPPORTED when either part would be empty.
fx_status split_class(fx_batch* b, size_t k, hipStream_t st, size_t keep_items = 0) {
    fx_batch::Class& c = b->classes[k];
    const size_t G = (size_t)c.group;
    const size_t items = (c.members.size() + G - 1) / G;
    if (keep_items == 0) keep_items = (items + 1) / 2;
    if (items < 2 || keep_items >= items) return FX_EUNSUPPORTED;
    fx_batch::Class r;
    fx_status s = fx_plan_create(&c.plan->prob_in, &r.plan);
    if (s != FX_OK) return s;
    r.plan->prob_in = c.plan->prob_in;
    r.tune = c.tune;
    r.group = c.group;
    r.cost = c.cost;
    const size_t keep = keep_items * G;
    r.members.assign(c.members.begin() + keep, c.members.end());
    apply_tune(r.plan, r.tune, r.group);
    if ((s = ensure_workspace(r.plan)) == FX_OK) s = ensure_stage(b, r, r.group);
    if (s == FX_OK) s = add_lane(b);
    if (s != FX_OK) {
        fx_plan_destroy(r.plan);
        if (r.stage) (void)hipFree(r.stage);
        return s;
    }
    b->classes[k].members.resize(keep);
    b->classes.insert(b->classes.begin() + (k + 1), r);
    for (size_t i = 0; i < b->classes.size(); ++i) b->classes[i].lane = (int)i;
    // one eager item before any capture (the replica's workspace is new)
    fx_batch::Class& rr = b->classes[k + 1];
    std::vector<const void*> in(b->n, rr.stage);
    return run_group(b, rr, 0, std::min(G, rr.members.size()), in.data(), nullptr, nullptr, st);
}

// Undoes split_class: the replica's members go back to the class, its plan, staging and lane are freed.
void merge_class(fx_batch* b, size_t k) {
    fx_batch::Class& r = b->classes[k + 1];
    b->classes[k].members.insert(b->classes[k].members.end(), r.members.begin(), r.members.end());
    fx_plan_destroy(r.plan);
    if (r.stage) (void)hipFree(r.stage);
    b->classes.erase(b->classes.begin() + (k + 1));
    if (!b->lanes.empty()) {
        (void)hipStreamDestroy(b->lanes.back());
        (void)hipEventDestroy(b->joins.back());
        b->lanes.pop_back();
        b->joins.pop_back();
    }
    for (size_t i = 0; i < b->classes.size(); ++i) b->classes[i].lane = (int)i;
}

// Every output range (psi_out[i], rho_out[i]) must be disjoint from every other output range and
// from every input; inputs may be shared between realizations. Sort-and-sweep over the ranges.
fx_status check_batch_disjoint(const fx_batch* b, const void* const* psi0, void* const* psi_out,
                               void* const* rho_out) {
    struct Range { uintptr_t lo, hi; int member; };
    std::vector<Range> outs, ins;
    const size_t cs = cbytes(b);
    std::vector<int64_t> M(b->n, 0);
    for (const auto& c : b->classes)
        for (int m : c.members) M[m] = c.plan->M;
    for (int i = 0; i < b->n; ++i) {
        const size_t cb = (size_t)M[i] * cs;
        ins.push_back({(uintptr_t)psi0[i], (uintptr_t)psi0[i] + cb, i});
        if (psi_out && psi_out[i]) outs.push_back({(uintptr_t)psi_out[i], (uintptr_t)psi_out[i] + cb, i});
        if (rho_out && rho_out[i]) outs.push_back({(uintptr_t)rho_out[i], (uintptr_t)rho_out[i] + cb / 2, i});
    }
    auto by_lo = [](const Range& x, const Range& y) { return x.lo < y.lo; };
    std::sort(outs.begin(), outs.end(), by_lo);
    for (size_t k = 1; k < outs.size(); ++k)
        if (outs[k].lo < outs[k - 1].hi) {
            set_error("output buffers of realizations " + std::to_string(outs[k - 1].member) + " and " +
                      std::to_string(outs[k].member) + " overlap");
            return FX_EINVAL;
        }
    for (const Range& r : ins) {
        // outputs are sorted and disjoint, so their ends ascend too: the last output starting below
        // r.hi has the largest end of all outputs that could reach into r
        auto it = std::lower_bound(outs.begin(), outs.end(), Range{r.hi, 0, 0}, by_lo);
        if (it != outs.begin()) {
            const Range& o = *(it - 1);
            if (o.hi > r.lo) {
                set_error("input of realization " + std::to_string(r.member) + " overlaps an output of realization " +
                          std::to_string(o.member));
                return FX_EINVAL;
            }
        }
    }
    return FX_OK;
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
    // issue order: largest classes first (terms x points x members)
    for (auto& c : b->classes) c.cost = (double)c.plan->Q * (double)c.plan->M * (double)c.members.size();
    std::stable_sort(b->classes.begin(), b->classes.end(),
                     [](const fx_batch::Class& x, const fx_batch::Class& y) { return x.cost > y.cost; });
    const int ncls = (int)b->classes.size();
    for (int k = 0; k < ncls; ++k) b->classes[k].lane = k;
    b->lanes.assign(ncls, nullptr);
    b->joins.assign(ncls, nullptr);
    for (int k = 0; k < ncls; ++k) {
        if (hipStreamCreateWithFlags(&b->lanes[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->joins[k], hipEventDisableTiming) != hipSuccess) {
            set_error("creating the batch lanes failed");
            fx_batch_destroy(b);
            return FX_EDEVICE;
        }
    }
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
        set_error("creating the batch lanes failed");
        fx_batch_destroy(b);
        return FX_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache();
    const bool tune = std::getenv("FX_NO_AUTOTUNE") == nullptr;
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) { fx_batch_destroy(b); return FX_EDEVICE; }
    auto fail = [&](fx_status s) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
        fx_batch_destroy(b);
        return s;
    };
    bool dirty = false;
    std::string bkey;
    for (auto& c : b->classes) {
        const std::string key = class_key(c.plan->prob, c.members.size());
        bkey += key + ";";
        auto it = g_tune.find(key);
        Tune best;
        if (it != g_tune.end()) {
            best = it->second;
        } else if (tune) {
            best = tune_class(b, c, st);
            g_tune[key] = best;
            dirty = true;
        } else {
            best.group = largest_group(c, best);
        }
        if (best.group < 1) best.group = 1;
        c.tune = best;
        c.group = best.group;
        apply_tune(c.plan, best, c.group);
        fx_status s = ensure_workspace(c.plan);
        if (s == FX_OK) s = ensure_stage(b, c, c.group);
        if (s != FX_OK) return fail(s);
        // eager runs (a full item and the last partial one) so that every kernel the graph will hold
        // has been launched once before any capture
        std::vector<const void*> in(n, c.stage);
        s = run_group(b, c, 0, (size_t)c.group, in.data(), nullptr, nullptr, st);
        const size_t rem = c.members.size() % (size_t)c.group;
        if (s == FX_OK && rem) {
            plan_setup_workspace(c.plan, (int64_t)rem);
            s = run_group(b, c, 0, rem, in.data(), nullptr, nullptr, st);
            plan_setup_workspace(c.plan, c.group);
        }
        if (s != FX_OK) return fail(s);
    }
    // replicas of the largest class (R items of it at once, on R lanes), when whole runs say so
    {
        // R replicas of class 0 from one: items split into near-equal whole-item parts
        auto make_replicas = [&](int R) -> fx_status {
            for (int r = 0; r + 1 < R; ++r) {
                const fx_batch::Class& c = b->classes[r];
                const size_t items = (c.members.size() + (size_t)c.group - 1) / (size_t)c.group;
                fx_status s2 = split_class(b, (size_t)r, st, (items + (size_t)(R - r) - 1) / (size_t)(R - r));
                if (s2 != FX_OK) return s2;
            }
            return FX_OK;
        };
        auto undo_replicas = [&](int R) {
            for (int r = R - 2; r >= 0; --r) merge_class(b, (size_t)r);
        };
        auto best_of = [&]() {
            const int L = (int)b->classes.size();
            double t = -1.0;
            for (int rep = 0; rep < 3; ++rep) {
                const double a = time_full(b, L, st);
                if (rep > 0 && a >= 0 && (t < 0 || a < t)) t = a;
            }
            return t;
        };
        auto it = g_repl.find(bkey);
        int repl = 1;
        const char* forced = std::getenv("FX_BATCH_REPLICAS");
        if (forced || it != g_repl.end()) {
            repl = forced ? std::max(1, std::min(4, std::atoi(forced))) : it->second;
            if (repl > 1) {
                fx_status s2 = make_replicas(repl);
                if (s2 != FX_OK && s2 != FX_EUNSUPPORTED) return fail(s2);
            }
        } else if (tune && b->classes[0].members.size() >= 2 * (size_t)b->classes[0].group) {
            double best_t = best_of();
            for (int R = 2; R <= 3; ++R) {
                fx_status s2 = make_replicas(R);
                if (s2 == FX_EUNSUPPORTED) { undo_replicas((int)b->classes.size() - ncls + 1); break; }
                if (s2 != FX_OK) return fail(s2);
                const double t = best_of();
                undo_replicas(R);
                if (t >= 0 && (best_t < 0 || t < best_t * 0.99)) {
                    best_t = t;
                    repl = R;
                } else {
                    break;
                }
            }
            if (repl > 1) {
                fx_status s2 = make_replicas(repl);
                if (s2 != FX_OK) return fail(s2);
            }
            g_repl[bkey] = repl;
            dirty = true;
        }
    }
    const int ncl = (int)b->classes.size();
    // lane concurrency: every class on its own lane, or all on the caller's stream
    b->concurrency = 1;
    if (ncl > 1) {
        auto it = g_conc.find(bkey);
        if (it != g_conc.end()) {
            b->concurrency = std::min(it->second, ncl);
        } else if (tune) {
            // whole runs, alternating between the two forms, best of two each after one warm-up
            double t1 = -1.0, tn = -1.0;
            for (int rep = 0; rep < 3; ++rep) {
                const double a = time_full(b, 1, st), c = time_full(b, ncl, st);
                if (rep == 0) continue;
                if (a >= 0 && (t1 < 0 || a < t1)) t1 = a;
                if (c >= 0 && (tn < 0 || c < tn)) tn = c;
            }
            b->concurrency = (tn >= 0 && (t1 < 0 || tn < t1)) ? ncl : 1;
            g_conc[bkey] = b->concurrency;
            dirty = true;
        } else {
            b->concurrency = ncl;
        }
    }
    if (const char* e = std::getenv("FX_BATCH_LANES")) b->concurrency = std::max(1, std::min(ncl, std::atoi(e)));
    b->tuned_concurrency = b->concurrency;
    if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("batch set-up run failed");
        return fail(FX_EDEVICE);
    }
    (void)hipStreamDestroy(st);
    if (dirty) save_tune_cache();
    *out = b;
    return FX_OK;
}

fx_status fx_batch_destroy(fx_batch* b) {
    if (!b) return FX_OK;
    drop_graph(b);
    for (auto& c : b->classes) {
        fx_plan_destroy(c.plan);
        if (c.stage) (void)hipFree(c.stage);
    }
    for (hipStream_t s : b->lanes)
        if (s) (void)hipStreamDestroy(s);
    for (hipEvent_t e : b->joins)
        if (e) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
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
    fx_status ov = check_batch_disjoint(b, psi0, psi_out, rho_out);
    if (ov != FX_OK) return ov;
    hipStream_t st = (hipStream_t)stream;
    bool timing = false;
    for (auto& c : b->classes) timing = timing || c.plan->timing;
    // per-pass timing records events around every launch, which a captured graph would not replay:
    // such runs (and runs on the legacy default stream, which cannot be captured) go out eagerly
    if (st == nullptr || timing || std::getenv("FX_NO_GRAPH")) return run_all(b, psi0, psi_out, rho_out, st);
    std::vector<const void*> in(psi0, psi0 + b->n);
    std::vector<void*> o(b->n, nullptr), r(b->n, nullptr);
    for (int i = 0; i < b->n; ++i) {
        if (psi_out) o[i] = psi_out[i];
        if (rho_out) r[i] = rho_out[i];
    }
    const bool same = b->exec && st == b->g_stream && in == b->g_in && o == b->g_out && r == b->g_rho;
    if (!same) {
        drop_graph(b);
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

fx_status fx_batch_num_classes(const fx_batch* b, int32_t* n) {
    if (!b || !n) { set_error("NULL argument"); return FX_EINVAL; }
    *n = (int32_t)b->classes.size();
    return FX_OK;
}

fx_status fx_batch_class(fx_batch* b, int32_t i, fx_plan** plan, int32_t* members, int64_t* group,
                         int32_t* lane) {
    if (!b) { set_error("batch is NULL"); return FX_EINVAL; }
    if (i < 0 || i >= (int32_t)b->classes.size()) { set_error("class index out of range"); return FX_EINVAL; }
    const auto& c = b->classes[i];
    if (plan) *plan = c.plan;
    if (members) *members = (int32_t)c.members.size();
    if (group) *group = c.group;
    if (lane) *lane = b->concurrency > 1 ? c.lane % b->concurrency : 0;
    return FX_OK;
}

fx_status fx_batch_set_lanes(fx_batch* b, int32_t lanes) {
    if (!b) { set_error("batch is NULL"); return FX_EINVAL; }
    if (lanes < 0) { set_error("lanes must be >= 0"); return FX_EINVAL; }
    const int ncl = (int)b->classes.size();
    const int want = lanes == 0 ? b->tuned_concurrency : std::min(lanes, ncl);
    if (want != b->concurrency) {
        drop_graph(b);
        b->concurrency = want;
    }
    return FX_OK;
}

fx_status fx_batch_class_members(const fx_batch* b, int32_t i, int32_t* members, int32_t max) {
    if (!b || !members) { set_error("NULL argument"); return FX_EINVAL; }
    if (i < 0 || i >= (int32_t)b->classes.size()) { set_error("class index out of range"); return FX_EINVAL; }
    const auto& c = b->classes[i];
    for (int32_t k = 0; k < max && k < (int32_t)c.members.size(); ++k) members[k] = c.members[k];
    return FX_OK;
}

}  // extern "C"
