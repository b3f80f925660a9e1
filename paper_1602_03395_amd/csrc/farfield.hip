// Far-field estimate on the magnified output lattice (eq. (farfieldk)): the comparator that the
// finite-time expansion replaces. With kappa_j(nbar) = (m / hbar t) xbar_j(nbar) the norm-preserving
// transform of eq. (FT), summed over the lattice as in eq. (Psiwtm) but at off-grid kappa,
// factorises over axes:
//   amp[nbar] = (m / hbar t)^(d/2) dV / (2 pi)^(d/2) sum_n Psi[n] prod_j exp(-i kappa_j(nbar_j) x_j(n_j)),
// rho_ff = |amp|^2. Each axis is a dense M_j x M_j complex matrix (built on the host in FP64 with
// the phase reduced modulo 2 pi in long double) applied along that axis: a batched complex GEMM,
// computed here with LDS-tiled VALU kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "plan.h"

namespace fx {
namespace {

constexpr int kTI = 64, kTJ = 64, kTK = 16;

// C[b][i][j] = sum_k A(b, i, k) B(b, k, j), complex, with element strides; I x J x K, batch nb.
struct GemmArgs {
    const void* A;
    const void* B;
    void* C;
    void* rho;  // optional |C|^2, same indexing as C
    int64_t I, J, K, nb;
    int64_t sai, sak, sab;  // A strides (elements): i, k, batch
    int64_t sbk, sbj, sbb;
    int64_t sci, scj, scb;
};

template <typename T>
__global__ __launch_bounds__(256) void k_cgemm(GemmArgs g) {
    __shared__ C<T> As[kTK][kTI + 1];
    __shared__ C<T> Bs[kTK][kTJ + 1];
    const C<T>* Ap = (const C<T>*)g.A;
    const C<T>* Bp = (const C<T>*)g.B;
    C<T>* Cp = (C<T>*)g.C;
    T* Rp = (T*)g.rho;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t ti = (g.I + kTI - 1) / kTI, tj = (g.J + kTJ - 1) / kTJ;
    const int64_t tiles = ti * tj * g.nb;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int64_t b = t / (ti * tj);
        const int64_t r = t - b * ti * tj;
        const int64_t i0 = (r / tj) * kTI, j0 = (r % tj) * kTJ;
        C<T> acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = mk<T>(0, 0);
        for (int64_t k0 = 0; k0 < g.K; k0 += kTK) {
            // 1024 elements of each tile, 4 per thread
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int idx = threadIdx.x + 256 * e;
                const int kk = idx & (kTK - 1), ii = idx >> 4;  // A tile: 64 rows x 16 k
                const int64_t gi = i0 + ii, gk = k0 + kk;
                As[kk][ii] = (gi < g.I && gk < g.K) ? Ap[b * g.sab + gi * g.sai + gk * g.sak] : mk<T>(0, 0);
                const int jj = idx & (kTJ - 1), kb = idx >> 6;   // B tile: 16 k x 64 cols
                const int64_t gj = j0 + jj, gk2 = k0 + kb;
                Bs[kb][jj] = (gj < g.J && gk2 < g.K) ? Bp[b * g.sbb + gk2 * g.sbk + gj * g.sbj] : mk<T>(0, 0);
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < kTK; ++kk) {
                C<T> a[4], bb[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) a[u] = As[kk][ty + 16 * u];
#pragma unroll
                for (int v = 0; v < 4; ++v) bb[v] = Bs[kk][tx + 16 * v];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] = cfma<T>(acc[u][v], a[u], bb[v]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t gi = i0 + ty + 16 * u;
            if (gi >= g.I) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gj = j0 + tx + 16 * v;
                if (gj >= g.J) continue;
                const int64_t o = b * g.scb + gi * g.sci + gj * g.scj;
                Cp[o] = acc[u][v];
                if (Rp) Rp[o] = acc[u][v].x * acc[u][v].x + acc[u][v].y * acc[u][v].y;
            }
        }
    }
}

int blocks_for_tiles(int64_t tiles) { return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, 65536)); }

// Dense axis matrices W_j[nbar][n] = exp(-i kappa_j(nbar) x_j(n)), the prefactor folded into the
// first real axis; phases reduced modulo 2 pi in long double.
fx_status build_ff(fx_plan* p) {
    if (p->ff_tab) return FX_OK;
    const int off = 3 - p->ndim;
    const size_t cs = csize(p);
    const long double two_pi = 6.283185307179586476925286766559L;
    const long double kap = (long double)p->prob.m_over_hbar / (long double)p->prob.t_flight;
    double dV = 1.0;
    for (int j = 0; j < p->ndim; ++j) dV *= p->prob.dx[j];
    const double pref = std::pow(std::fabs((double)kap), 0.5 * p->ndim) * dV / std::pow(2.0 * M_PI, 0.5 * p->ndim);
    size_t total = 0;
    for (int pa = off; pa < 3; ++pa) {
        p->ff_off[pa] = total;
        total += (((size_t)p->len[pa] * p->len[pa] * cs + 255) / 256) * 256;
    }
    std::vector<unsigned char> host(total, 0);
    for (int pa = off; pa < 3; ++pa) {
        const int j = pa - off;
        const int64_t M = p->len[pa];
        const long double a = p->prob.a[j], ab = p->prob.abar[j];
        const long double dx = p->prob.dx[j], ldx = (long double)p->prob.lambda[j] * dx;
        const double amp = (pa == off) ? pref : 1.0;
        for (int64_t nb = 0; nb < M; ++nb) {
            const long double k = kap * (ab + (long double)nb * ldx);
            for (int64_t n = 0; n < M; ++n) {
                long double ph = -k * (a + (long double)n * dx);
                ph -= two_pi * std::nearbyint(ph / two_pi);
                const double c = amp * std::cos((double)ph), sn = amp * std::sin((double)ph);
                const size_t i = p->ff_off[pa] + (size_t)(nb * M + n) * cs;
                if (p->dbl) {
                    double v[2] = {c, sn};
                    std::memcpy(&host[i], v, sizeof(v));
                } else {
                    float v[2] = {(float)c, (float)sn};
                    std::memcpy(&host[i], v, sizeof(v));
                }
            }
        }
    }
    void* d = nullptr;
    if (hipMalloc(&d, total) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of far-field tables failed");
        return FX_ENOMEM;
    }
    if (hipMemcpy(d, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        set_error("far-field table upload failed");
        return FX_EDEVICE;
    }
    void* b = nullptr;
    if (hipMalloc(&b, (size_t)2 * p->M * cs) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(d);
        set_error("hipMalloc of far-field buffers failed");
        return FX_ENOMEM;
    }
    p->ff_tab = d;
    p->ff_buf = b;
    return FX_OK;
}

}  // namespace
}  // namespace fx

using namespace fx;

extern "C" fx_status fx_far_field(fx_plan* p, const void* psi0, void* amp_out, void* rho_out, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    fx_status s = check_ptr(psi0, "psi0");
    if (s != FX_OK) return s;
    if (!amp_out && !rho_out) { set_error("amp_out and rho_out are both NULL"); return FX_EINVAL; }
    if (p->prob.t_flight == 0.0) { set_error("the far-field estimate needs t_flight != 0"); return FX_EINVAL; }
    {
        const size_t cb = (size_t)p->M * csize(p);
        if ((s = check_disjoint(psi0, cb, "psi0", amp_out, cb, "amp_out")) != FX_OK) return s;
        if ((s = check_disjoint(psi0, cb, "psi0", rho_out, cb / 2, "rho_out")) != FX_OK) return s;
        if ((s = check_disjoint(amp_out, cb, "amp_out", rho_out, cb / 2, "rho_out")) != FX_OK) return s;
    }
    for (int pa = 0; pa < 3; ++pa)
        if (p->spectrum[pa]) {
            set_error("the far-field estimate is defined for the free-particle spectrum only");
            return FX_EUNSUPPORTED;
        }
    if ((s = build_ff(p)) != FX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const size_t cs = csize(p);
    const int off = 3 - p->ndim;
    const void* cur = psi0;
    char* bufs[2] = {(char*)p->ff_buf, (char*)p->ff_buf + (size_t)p->M * cs};
    for (int pa = off; pa < 3; ++pa) {
        const bool last = (pa == 2);
        void* dst = (last && amp_out) ? amp_out : bufs[(pa - off) & 1];
        int64_t A = 1, S = 1;
        for (int i = 0; i < pa; ++i) A *= p->len[i];
        for (int i = pa + 1; i < 3; ++i) S *= p->len[i];
        const int64_t L = p->len[pa];
        GemmArgs g;
        const void* W = (const char*)p->ff_tab + p->ff_off[pa];
        g.C = dst;
        g.rho = last ? rho_out : nullptr;
        if (S > 1) {  // out[a][nbar][s] = sum_n W[nbar][n] in[a][n][s]
            g.A = W; g.sai = L; g.sak = 1; g.sab = 0;
            g.B = cur; g.sbk = S; g.sbj = 1; g.sbb = L * S;
            g.sci = S; g.scj = 1; g.scb = L * S;
            g.I = L; g.J = S; g.K = L; g.nb = A;
        } else {      // out[a][nbar] = sum_n in[a][n] W[nbar][n]
            g.A = cur; g.sai = L; g.sak = 1; g.sab = 0;
            g.B = W; g.sbk = 1; g.sbj = L; g.sbb = 0;
            g.sci = L; g.scj = 1; g.scb = 0;
            g.I = A; g.J = L; g.K = L; g.nb = 1;
        }
        const int64_t tiles = ((g.I + kTI - 1) / kTI) * ((g.J + kTJ - 1) / kTJ) * g.nb;
        if (p->dbl)
            hipLaunchKernelGGL(k_cgemm<double>, dim3(blocks_for_tiles(tiles)), dim3(256), 0, st, g);
        else
            hipLaunchKernelGGL(k_cgemm<float>, dim3(blocks_for_tiles(tiles)), dim3(256), 0, st, g);
        FX_TRY_HIP(hipGetLastError());
        cur = dst;
    }
    return FX_OK;
}
