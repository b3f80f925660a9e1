// Positive-P pairs (section 7.4, generalisations): the fields psi and psi^+ that stand for
// the annihilation and creation operators are expanded together, as the two leading
// slices of one run of the plan's passes. psi^+ obeys the complex-conjugate free
// equation, so its expansion is conj(U conj(psi^+)): the input slice is conjugated on
// the way in and the output slice on the way out. The density estimator is
// n = psibar^+ psibar (complex; its real part is the estimator of the mean density).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "plan.h"

namespace fx {
namespace {

// stage[0:n] = psi, stage[n:2n] = conj(psi_plus)
template <typename T>
__global__ void k_pair_in(const C<T>* __restrict__ psi, const C<T>* __restrict__ psi_plus, C<T>* __restrict__ stage,
                          int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        stage[i] = psi[i];
        const C<T> v = psi_plus[i];
        stage[n + i] = mk<T>(v.x, -v.y);
    }
}

// psibar = res[0:n], psibar^+ = conj(res[n:2n]), n = psibar^+ * psibar; every output optional
template <typename T>
__global__ void k_pair_out(const C<T>* __restrict__ res, C<T>* __restrict__ out, C<T>* __restrict__ out_plus,
                           C<T>* __restrict__ dens, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const C<T> a = res[i];
        const C<T> b = res[n + i];
        const C<T> bp = mk<T>(b.x, -b.y);
        if (out) out[i] = a;
        if (out_plus) out_plus[i] = bp;
        if (dens) dens[i] = cmul<T>(bp, a);
    }
}

// g = 2 grad_rho psibar: the derivative of a real function of rho = |psibar|^2 in PyTorch's
// complex convention (dL/dRe + i dL/dIm)
template <typename T>
__global__ void k_density_grad(const C<T>* __restrict__ psibar, const T* __restrict__ grad_rho, C<T>* __restrict__ g,
                               int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T w = (T)2 * grad_rho[i];
        const C<T> v = psibar[i];
        g[i] = mk<T>(w * v.x, w * v.y);
    }
}

int blocks_for(int64_t n) {
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

// Workspace of a pair call: the plan's two ping-pong buffers and output staging for two
// slices, then the two-slice input staging.
void setup_pair(fx_plan* p) {
    plan_setup_workspace(p, 2);
    p->ws_need += (size_t)(2 * p->M) * csize(p);
}

}  // namespace
}  // namespace fx

using namespace fx;

extern "C" {

fx_status fx_plan_pair_workspace_size(const fx_plan* p, size_t* bytes) {
    if (!p || !bytes) { set_error("NULL argument"); return FX_EINVAL; }
    int64_t nb = 0, buf = 0;
    size_t need = 0;
    workspace_layout(p, 2, &nb, &buf, &need);
    *bytes = need + (size_t)(2 * p->M) * csize(p);
    return FX_OK;
}

fx_status fx_expand_pair(fx_plan* p, const void* psi, const void* psi_plus, void* psi_out, void* psi_plus_out,
                         void* n_out, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    fx_status s = check_ptr(psi, "psi");
    if (s != FX_OK) return s;
    if ((s = check_ptr(psi_plus, "psi_plus")) != FX_OK) return s;
    if (!psi_out && !psi_plus_out && !n_out) { set_error("every output is NULL"); return FX_EINVAL; }
    {
        const size_t cb = (size_t)p->M * csize(p);
        const void* ins[2] = {psi, psi_plus};
        const char* in_names[2] = {"psi", "psi_plus"};
        const void* outs[3] = {psi_out, psi_plus_out, n_out};
        const char* out_names[3] = {"psi_out", "psi_plus_out", "n_out"};
        for (int o = 0; o < 3; ++o) {
            for (int i = 0; i < 2; ++i)
                if ((s = check_disjoint(ins[i], cb, in_names[i], outs[o], cb, out_names[o])) != FX_OK) return s;
            for (int o2 = o + 1; o2 < 3; ++o2)
                if ((s = check_disjoint(outs[o], cb, out_names[o], outs[o2], cb, out_names[o2])) != FX_OK) return s;
        }
    }
    if (p->slices != 2) setup_pair(p);  // the single-field entry points reset slices to 1
    if ((s = ensure_workspace(p)) != FX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const size_t cs = csize(p);
    const int64_t n = p->M;
    char* dst = (char*)p->ws + (size_t)2 * p->buf_elems * cs;
    char* stage = dst + (size_t)(2 * n) * cs;
    if (p->dbl)
        hipLaunchKernelGGL(k_pair_in<double>, dim3(blocks_for(n)), dim3(kThreads), 0, st, (const double2*)psi,
                           (const double2*)psi_plus, (double2*)stage, n);
    else
        hipLaunchKernelGGL(k_pair_in<float>, dim3(blocks_for(n)), dim3(kThreads), 0, st, (const float2*)psi,
                           (const float2*)psi_plus, (float2*)stage, n);
    FX_TRY_HIP(hipGetLastError());
    int qb[3] = {0, 0, 0}, qn[3] = {p->ax[0].lam, p->ax[1].lam, p->ax[2].lam};
    if ((s = run_box(p, qb, qn, stage, dst, 0, nullptr, false, st)) != FX_OK) return s;
    if (p->dbl)
        hipLaunchKernelGGL(k_pair_out<double>, dim3(blocks_for(n)), dim3(kThreads), 0, st, (const double2*)dst,
                           (double2*)psi_out, (double2*)psi_plus_out, (double2*)n_out, n);
    else
        hipLaunchKernelGGL(k_pair_out<float>, dim3(blocks_for(n)), dim3(kThreads), 0, st, (const float2*)dst,
                           (float2*)psi_out, (float2*)psi_plus_out, (float2*)n_out, n);
    FX_TRY_HIP(hipGetLastError());
    return FX_OK;
}

fx_status fx_density_adjoint(fx_plan* p, const void* psibar, const void* grad_rho, void* grad_psi0, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    fx_status s = check_ptr(psibar, "psibar");
    if (s != FX_OK) return s;
    if ((s = check_ptr(grad_rho, "grad_rho")) != FX_OK) return s;
    if ((s = check_ptr(grad_psi0, "grad_psi0")) != FX_OK) return s;
    const size_t cb = (size_t)p->M * csize(p);
    if ((s = check_disjoint(psibar, cb, "psibar", grad_psi0, cb, "grad_psi0")) != FX_OK) return s;
    if ((s = check_disjoint(grad_rho, cb / 2, "grad_rho", grad_psi0, cb, "grad_psi0")) != FX_OK) return s;
    if (p->slices != 1) plan_setup_workspace(p, 1);
    if ((s = ensure_workspace(p)) != FX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = p->M;
    // 2 grad_rho psibar goes to the output staging region, which the adjoint passes do not use
    void* g = (char*)p->ws + (size_t)2 * p->buf_elems * csize(p);
    if (p->dbl)
        hipLaunchKernelGGL(k_density_grad<double>, dim3(blocks_for(n)), dim3(kThreads), 0, st,
                           (const double2*)psibar, (const double*)grad_rho, (double2*)g, n);
    else
        hipLaunchKernelGGL(k_density_grad<float>, dim3(blocks_for(n)), dim3(kThreads), 0, st,
                           (const float2*)psibar, (const float*)grad_rho, (float2*)g, n);
    FX_TRY_HIP(hipGetLastError());
    int qb[3] = {0, 0, 0}, qn[3] = {p->ax[0].lam, p->ax[1].lam, p->ax[2].lam};
    return run_box(p, qb, qn, g, grad_psi0, 0, nullptr, true, st);
}

fx_status fx_density_adjoint_many(fx_plan* p, int64_t count, const void* psibar, const void* grad_rho,
                                  void* grad_psi0, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    if (count < 1) { set_error("count must be >= 1"); return FX_EINVAL; }
    fx_status s = check_ptr(psibar, "psibar");
    if (s != FX_OK) return s;
    if ((s = check_ptr(grad_rho, "grad_rho")) != FX_OK) return s;
    if ((s = check_ptr(grad_psi0, "grad_psi0")) != FX_OK) return s;
    const size_t cb = (size_t)p->M * csize(p);
    if ((s = check_disjoint(psibar, count * cb, "psibar", grad_psi0, count * cb, "grad_psi0")) != FX_OK) return s;
    if ((s = check_disjoint(grad_rho, count * cb / 2, "grad_rho", grad_psi0, count * cb, "grad_psi0")) != FX_OK)
        return s;
    const int64_t chunk = stack_chunk(p, count, 0);
    if ((s = ensure_workspace(p)) != FX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    int qb[3] = {0, 0, 0}, qn[3] = {p->ax[0].lam, p->ax[1].lam, p->ax[2].lam};
    for (int64_t f = 0; f < count; f += chunk) {
        const int64_t c = std::min(chunk, count - f);
        if (c != p->slices) plan_setup_workspace(p, c);
        const int64_t n = c * p->M;
        // 2 grad_rho psibar of the chunk goes to the output staging region (c fields), which the
        // adjoint passes do not use
        void* g = (char*)p->ws + (size_t)2 * p->buf_elems * csize(p);
        const char* pb = (const char*)psibar + (size_t)f * cb;
        const char* gr = (const char*)grad_rho + (size_t)f * cb / 2;
        if (p->dbl)
            hipLaunchKernelGGL(k_density_grad<double>, dim3(blocks_for(n)), dim3(kThreads), 0, st,
                               (const double2*)pb, (const double*)gr, (double2*)g, n);
        else
            hipLaunchKernelGGL(k_density_grad<float>, dim3(blocks_for(n)), dim3(kThreads), 0, st,
                               (const float2*)pb, (const float*)gr, (float2*)g, n);
        FX_TRY_HIP(hipGetLastError());
        if ((s = run_box(p, qb, qn, g, (char*)grad_psi0 + (size_t)f * cb, 0, nullptr, true, st)) != FX_OK) return s;
    }
    return FX_OK;
}

}  // extern "C"
