// Plan object and schedule helpers shared by the host runtime files (not public ABI).
#pragma once

#include <string>
#include <vector>

#include "fx_internal.h"

#define FX_TRY_HIP(call)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            fx::set_error(std::string(#call) + ": " + hipGetErrorString(e_));                  \
            return FX_EDEVICE;                                                             \
        }                                                                                  \
    } while (0)

namespace fx {

struct Op {
    Kind kind;
    int axis;          // padded axis 0..2
    PassGeom g;
    int64_t in_elems;  // per op, elements read tensor size
    int64_t out_elems;
    int axis2 = -1;    // AA: the second (later) axis
    AAGeom aa;         // AA: geometry of the fused pair
};

constexpr int64_t kMaxAxis = 4096;

}  // namespace fx

struct fx_plan {
    fx_problem prob{};             // with default offsets resolved
    fx_problem prob_in{};          // as given by the caller
    bool dbl = true;
    int ndim = 1;
    int64_t len[3] = {1, 1, 1};   // padded shape
    fx::AxisParams par[3];
    fx::AxisDev ax[3];
    int act[3] = {0, 0, 0};
    int nact = 0;
    int64_t M = 1;                 // total points
    int64_t Q = 1;                 // prod lam
    void* dtab = nullptr;
    size_t dtab_bytes = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    int64_t nb_outer = 1;          // block of the outermost magnification index
    int64_t nb_fixed = 0;          // >0: use this block instead of fitting the budget
    int64_t slices = 1;            // leading slices (batched realizations)
    size_t ws_need = 0;
    int64_t buf_elems = 0;         // elements of each of the two ping-pong buffers
    int schedule = FX_SCHED_PAPER;
    int ts_target = 2048;
    bool allow_split = true;       // split a starved fused EA pass into E + A
    bool spectrum[3] = {false, false, false};  // axis built from a caller spectrum table
    void* ff_tab = nullptr;        // far-field comparator: per-axis dense matrices (built on first use)
    void* ff_buf = nullptr;        // far-field comparator: two M-point buffers
    size_t ff_off[3] = {0, 0, 0};
    void* bf_state = nullptr;      // brute-force comparator: tables and buffers (built on first use)
    bool use_cfp = true;           // register E kernel where the pruned length allows it
    bool use_asr = true;           // register structured accumulate (k_ASR) for g <= asr_max_g
    bool use_eh2 = true;           // compile-time power-of-two EH kernel (FX_NO_EH2 disables)
    int use_aa = 1;                // fuse the last two accumulate passes: 0 never (FX_AA=0), 1 in
                                   // registers where g_u = g_v is 16 or 32 and they are the last two
                                   // axes, 2 also through the LDS form elsewhere (FX_AA=1)
    int use_eas = 1;               // EA through the structured register kernel: 0 never (FX_NO_EAS),
                                   // 1 where it applies with P >= 8 and g <= 16 (smaller transforms
                                   // are dominated by the per-wave overheads; its table-row traffic
                                   // per line grows as g^2 / 64 times the line's output), 2 wherever
                                   // it applies (FX_EAS=1)
    bool use_eaw = true;           // EA for g = 8 through the one-wave-per-tile structured kernel
    int use_erw = 1;               // E with P lanes per line (g = 8): 0 never, 1 for P >= 32, 2 also P = 16
                                   // (FX_NO_EAW disables)
    int asr_max_g = 64;            // above this the LDS-transform form (k_AS) is used
    int cfp_blocks = 1024;         // register E kernel: target workgroups per launch
    bool use_p2 = true;            // compile-time specialised kernels for power-of-two axes
    bool index_ok = true;          // every tensor of the current layout indexes in 32 bits (see workspace_layout)
    int persist = 0;               // >0: tile passes run as persistent grids of persist x CUs workgroups
    size_t budget = 0;
    // per-pass timing
    bool timing = false;
    struct Pending { int op; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::vector<int64_t> t_launch;
    std::vector<double> t_ms;
};

namespace fx {

size_t csize(const fx_plan* p);
std::vector<Op> build_ops(const fx_plan* p, const int qb[3], const int qn[3], int64_t slices0, bool adjoint);
int64_t max_intermediate(const std::vector<Op>& ops);
fx_status validate(const fx_problem* pr);
// Outer block, ping-pong buffer elements and workspace bytes for `slices` leading slices.
void workspace_layout(const fx_plan* p, int64_t slices, int64_t* nb, int64_t* buf, size_t* need);
// The same for the forward schedule alone (with_adjoint = false) or both schedules (true).
void workspace_layout_for(const fx_plan* p, int64_t slices, bool with_adjoint, int64_t* nb, int64_t* buf,
                          size_t* need);
fx_status plan_setup_workspace(fx_plan* p, int64_t slices);
fx_status ensure_workspace(fx_plan* p);
// slot0: first timing slot of the list (0 forward, FX_ADJOINT_SLOT0 adjoint)
fx_status run_ops(fx_plan* p, const std::vector<Op>& ops, const void* src, void* dst, int accumulate, void* rho,
                  hipStream_t st, int slot0);
fx_status run_box(fx_plan* p, const int qb[3], const int qn[3], const void* src, void* dst, int accumulate,
                  void* rho, bool adjoint, hipStream_t st);
fx_status check_ptr(const void* ptr, const char* what);
int64_t stack_chunk(fx_plan* p, int64_t count, size_t extra_bytes_per_field);
// FX_EINVAL when the byte ranges [a, a + na) and [b, b + nb) intersect; a NULL pointer is never checked.
fx_status check_disjoint(const void* a, size_t na, const char* an, const void* b, size_t nb, const char* bn);
// Elements below which every pass tensor, tile count and grid size indexes in 32 bits.
constexpr int64_t kIndexLimit = (int64_t(1) << 31) - (int64_t(1) << 28);
void bf_release(fx_plan* p);

}  // namespace fx
