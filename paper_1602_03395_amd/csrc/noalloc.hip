// The expansion without any device allocation: fx_expand_noalloc runs the same passes as
// fx_expand, with the ping-pong intermediates and the output staging in a fixed scratch array
// that is part of the library's device image, instead of a workspace the plan allocates.
//
// The array's address on a device comes from hipGetSymbolAddress, resolved once per device on
// the first call there (with that device current) and cached; in host code the array's own name
// is only a stand-in for the symbol, never a device address, so it is used nowhere else. Every
// call on one device shares that device's array: calls that overlap in time on one device (two
// streams, two threads) race on it. No pass reads scratch memory it has not written in the same
// call, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "plan.h"

namespace fx {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // FX_NOALLOC_SCRATCH_BYTES in include/fx.h
static_assert(kScratchBytes == FX_NOALLOC_SCRATCH_BYTES, "scratch size and its public value differ");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device (resolved on first use).
fx_status scratch_on_current_device(void** out) {
    int dev = 0;
    FX_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the library's scratch table");
        return FX_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
            return FX_EDEVICE;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FX_OK;
}

}  // namespace
}  // namespace fx

using namespace fx;

extern "C" fx_status fx_expand_noalloc(fx_plan* p, const void* psi0, void* psi_out, void* rho_out, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    fx_status s = check_ptr(psi0, "psi0");
    if (s != FX_OK) return s;
    if (!psi_out && !rho_out) { set_error("psi_out and rho_out are both NULL"); return FX_EINVAL; }
    const size_t cb = (size_t)p->M * csize(p), rb = cb / 2;
    if ((s = check_disjoint(psi0, cb, "psi0", psi_out, cb, "psi_out")) != FX_OK) return s;
    if ((s = check_disjoint(psi0, cb, "psi0", rho_out, rb, "rho_out")) != FX_OK) return s;
    if ((s = check_disjoint(psi_out, cb, "psi_out", rho_out, rb, "rho_out")) != FX_OK) return s;
    void* base = nullptr;
    if ((s = scratch_on_current_device(&base)) != FX_OK) return s;

    // Lay the single-field schedule out in the scratch array: the outermost magnification index is
    // blocked until the intermediates fit (the sequential accumulation of section 7.1). The plan's
    // own workspace settings are restored afterwards.
    const size_t budget = p->budget;
    const int64_t nb_fixed = p->nb_fixed, slices = p->slices;
    void* ws = p->ws;
    const size_t ws_bytes = p->ws_bytes;
    const bool ws_owned = p->ws_owned, timing = p->timing;
    auto restore = [&]() {
        p->budget = budget;
        p->nb_fixed = nb_fixed;
        p->ws = ws;
        p->ws_bytes = ws_bytes;
        p->ws_owned = ws_owned;
        p->timing = timing;
        plan_setup_workspace(p, slices);
    };
    // the layout's budget bounds the two intermediates; the output staging (one field) comes on top
    const size_t staging = (size_t)p->M * csize(p) + 1024;
    p->budget = kScratchBytes > staging ? kScratchBytes - staging : 0;
    p->nb_fixed = 0;
    p->timing = false;  // per-pass timing would create events
    plan_setup_workspace(p, 1);
    // only the forward schedule runs here: its own (smaller) intermediates set the layout
    workspace_layout_for(p, 1, false, &p->nb_outer, &p->buf_elems, &p->ws_need);
    p->index_ok = p->M < kIndexLimit && p->buf_elems < kIndexLimit;
    if (!p->index_ok || p->ws_need > kScratchBytes) {
        const size_t need = p->ws_need;
        const bool idx = p->index_ok;
        restore();
        if (!idx) {
            set_error("a pass tensor of this problem reaches 2^31 elements, beyond the kernels' 32-bit indexing");
            return FX_EUNSUPPORTED;
        }
        set_error("fx_expand_noalloc: the problem needs " + std::to_string(need) + " bytes of scratch even with "
                  "one outermost magnification index per block, more than the library's fixed " +
                  std::to_string(kScratchBytes) + " bytes (FX_NOALLOC_SCRATCH_BYTES); use fx_expand");
        return FX_ENOMEM;
    }
    p->ws = base;
    p->ws_bytes = kScratchBytes;
    p->ws_owned = false;
    void* dst = psi_out ? psi_out : (char*)base + (size_t)2 * p->buf_elems * csize(p);
    int qb[3] = {0, 0, 0}, qn[3] = {p->ax[0].lam, p->ax[1].lam, p->ax[2].lam};
    s = run_box(p, qb, qn, psi0, dst, 0, rho_out, false, (hipStream_t)stream);
    restore();
    return s;
}
