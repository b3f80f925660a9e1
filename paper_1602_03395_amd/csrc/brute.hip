// Brute-force comparator (section 3 and the comparison of section 6): the free flight evaluated
// on the vacuum-padded lattice itself, without the method. Per axis the field is padded to
// N = lam M points (eq. (vacuum)), transformed (eq. (DFT)), multiplied by
//   Phi[l] = exp(i kappa_l (abar - a) - i hbar t kappa_l^2 / 2m),  kappa_l = 2 pi l / (N dx)
// (eqs. (free0), (Psin) with the output offset), transformed back and sampled at every lam-th
// point. Because the free propagator factorises over axes this equals eq. (Psin) on the full
// padded lattice, at a fraction of its memory. Lines longer than one workgroup's LDS are
// transformed in two passes each way (N = N1 N2, twiddles between the passes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "device_common.h"
#include "plan.h"

namespace fx {
namespace {

enum class BfMode { SINGLE, F1, F2, I1, I2 };

struct BfPass {
    BfMode mode;
    int64_t A, S;      // lengths before / after the axis
    int M, N, N1, N2;  // axis length, padded length, N = N1 N2 when two passes are used
    int lam;
    int L;             // transform length of this pass
    int TS;            // lines per tile
    int64_t nlines;
    const void* in;
    void* out;
    void* rho;         // SINGLE / I2 of the last axis: |out|^2
    const void* tw;    // exp(-2 pi i k / N), k < N
    const void* phi;   // Phi in transform order, N values
    RadixPlan pl;      // plan of the L-point transform
};

// Element i of line `line` of the pass: input address (or -1 for a padded zero) and output
// address (or -1 when the element is not kept).
template <typename T>
__device__ __forceinline__ void bf_addr(const BfPass& b, int64_t line, int i, int64_t& src, int64_t& dst) {
    const int64_t S = b.S;
    const int64_t s = line % S;
    const int64_t r = line / S;
    switch (b.mode) {
        case BfMode::SINGLE: {  // line (a, s), i = n (in) = k (transform) = m (out)
            const int64_t a = r;
            src = (i < b.M) ? (a * b.M + i) * S + s : -1;
            dst = (i % b.lam == 0) ? (a * b.M + i / b.lam) * S + s : -1;
            break;
        }
        case BfMode::F1: {  // line (a, n2, s), i = n1 in, k1 out
            const int64_t n2 = r % b.N2, a = r / b.N2;
            const int64_t n = (int64_t)b.N2 * i + n2;
            src = (n < b.M) ? (a * b.M + n) * S + s : -1;
            dst = (a * b.N + (int64_t)i * b.N2 + n2) * S + s;
            break;
        }
        case BfMode::F2:
        case BfMode::I1: {  // line (a, k1, s), i = n2 -> k2 (F2) or k2 -> m2 (I1), in place
            const int64_t k1 = r % b.N1, a = r / b.N1;
            src = dst = (a * b.N + k1 * b.N2 + i) * S + s;
            break;
        }
        case BfMode::I2: {  // line (a, m2, s), i = k1 in, m1 out; m = m2 + N2 m1
            const int64_t m2 = r % b.N2, a = r / b.N2;
            src = (a * b.N + (int64_t)i * b.N2 + m2) * S + s;
            const int64_t m = m2 + (int64_t)b.N2 * i;
            dst = (m % b.lam == 0) ? (a * b.M + m / b.lam) * S + s : -1;
            break;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_bf(BfPass b) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = b.L, TS = b.TS;
    C<T>* X = (C<T>*)smem;
    C<T>* Y = X + TS * L;
    C<T>* rl = Y + TS * L;  // exp(-2 pi i k / L)
    const C<T>* twN = (const C<T>*)b.tw;
    const C<T>* phi = (const C<T>*)b.phi;
    const C<T>* in = (const C<T>*)b.in;
    C<T>* out = (C<T>*)b.out;
    T* rho = (T*)b.rho;
    const int stride = b.N / L;
    for (int k = threadIdx.x; k < L; k += blockDim.x) rl[k] = twN[(int64_t)k * stride];
    __syncthreads();
    const int64_t ntiles = (b.nlines + TS - 1) / TS;
    const T invN = (T)(1.0 / (double)b.N);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t l0 = t * TS;
        const int nl = (int)min((int64_t)TS, b.nlines - l0);
        // load: consecutive threads take consecutive lines of one element index
        for (int e = threadIdx.x; e < nl * L; e += blockDim.x) {
            const int i = e / nl, li = e - (e / nl) * nl;
            int64_t src, dst;
            bf_addr<T>(b, l0 + li, i, src, dst);
            X[li * L + i] = (src >= 0) ? in[src] : mk<T>(0, 0);
        }
        __syncthreads();
        const bool inv = (b.mode == BfMode::I1 || b.mode == BfMode::I2);
        C<T>* R = lds_fft<T>(X, Y, nl, L, b.pl, rl, 1, inv);
        if (b.mode == BfMode::SINGLE) {
            // Phi, then the inverse transform, in the same workgroup
            for (int e = threadIdx.x; e < nl * L; e += blockDim.x) R[e] = cmul<T>(R[e], phi[e % L]);
            __syncthreads();
            C<T>* other = (R == X) ? Y : X;
            R = lds_fft<T>(R, other, nl, L, b.pl, rl, 1, true);
        }
        for (int e = threadIdx.x; e < nl * L; e += blockDim.x) {
            const int i = e / nl, li = e - (e / nl) * nl;
            const int64_t line = l0 + li;
            int64_t src, dst;
            bf_addr<T>(b, line, i, src, dst);
            if (dst < 0) continue;
            C<T> v = R[li * L + i];
            const int64_t r = line / b.S;
            switch (b.mode) {
                case BfMode::F1: {  // twiddle exp(-2 pi i n2 k1 / N)
                    const int64_t n2 = r % b.N2;
                    v = cmul<T>(v, twN[(n2 * i) % b.N]);
                    break;
                }
                case BfMode::F2: {  // Phi at transform index k1 + N1 k2
                    const int64_t k1 = r % b.N1;
                    v = cmul<T>(v, phi[k1 + (int64_t)b.N1 * i]);
                    break;
                }
                case BfMode::I1: {  // twiddle exp(+2 pi i k1 m2 / N)
                    const int64_t k1 = r % b.N1;
                    v = cmulc<T>(v, twN[(k1 * i) % b.N]);
                    break;
                }
                default:  // SINGLE, I2: normalise the inverse transform
                    v = cscale<T>(v, invN);
                    break;
            }
            out[dst] = v;
            if (rho) rho[dst] = v.x * v.x + v.y * v.y;
        }
        __syncthreads();
    }
}

size_t bf_lds(bool dbl, int L, int TS) { return (size_t)(2 * TS + 1) * L * (dbl ? 16 : 8); }

// Transform length that fits one workgroup with a tile of one line.
int bf_lmax(bool dbl) {
    const int lim = lds_limit_bytes();
    return lim / (3 * (dbl ? 16 : 8));
}

// exp(-2 pi i k / N) and Phi over the transform order for one axis, in FP64 with the phase
// reduced modulo 1 cycle in long double before the exponential.
void bf_tables(const fx_plan* p, int pa, int N, std::vector<double>& tw, std::vector<double>& phi) {
    const int j = pa - (3 - p->ndim);
    const long double dx = p->prob.dx[j];
    const long double delta = ((long double)p->prob.abar[j] - (long double)p->prob.a[j]) / dx;
    const long double pi = 3.14159265358979323846264338327950288L;
    const long double Lb = (long double)N * dx;
    const long double beta = pi * ((long double)p->prob.t_flight / (long double)p->prob.m_over_hbar) / (Lb * Lb);
    tw.assign(2 * (size_t)N, 0.0);
    phi.assign(2 * (size_t)N, 0.0);
    auto put = [pi](std::vector<double>& v, size_t i, long double cyc) {
        cyc -= std::nearbyint((double)cyc);
        const double ang = (double)(2.0L * pi * cyc);
        v[2 * i] = std::cos(ang);
        v[2 * i + 1] = std::sin(ang);
    };
    for (int k = 0; k < N; ++k) put(tw, (size_t)k, -(long double)k / (long double)N);
    for (int idx = 0; idx < N; ++idx) {
        const int64_t l = (2 * (int64_t)idx < (int64_t)N) ? idx : (int64_t)idx - N;  // Nyquist negative (eq. (kj))
        // cycles: l delta / N - beta l^2 (shift to the output offset, free evolution)
        long double c = (long double)l * delta / (long double)N;
        c -= std::nearbyint((double)c);
        long double q = beta * (long double)(l * l);
        q -= std::nearbyint((double)q);
        put(phi, (size_t)idx, c - q);  // indexed by the transform index idx
    }
}

fx_status launch_bf(const fx_plan* p, BfPass b, hipStream_t st) {
    const size_t lds = bf_lds(p->dbl, b.L, b.TS);
    const void* k = p->dbl ? (const void*)k_bf<double> : (const void*)k_bf<float>;
    if (lds > 65536) FX_TRY_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit_bytes()));
    b.pl = make_radix_plan(b.L);
    const int64_t tiles = (b.nlines + b.TS - 1) / b.TS;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, 1 << 20));
    if (p->dbl) hipLaunchKernelGGL(k_bf<double>, dim3(blocks), dim3(kThreads), lds, st, b);
    else hipLaunchKernelGGL(k_bf<float>, dim3(blocks), dim3(kThreads), lds, st, b);
    FX_TRY_HIP(hipGetLastError());
    return FX_OK;
}

struct BfAxis {
    int N = 1, N1 = 1, N2 = 1;
    bool two = false;
    size_t tw_off = 0, phi_off = 0;
};

}  // namespace
}  // namespace fx

namespace fx {

// Per-plan brute-force state (tables and buffers), built on first use and released with the plan.
struct BfState {
    void* tab = nullptr;
    void* buf = nullptr;   // padded intermediate of the two-pass transforms
    void* io = nullptr;    // two M-point buffers between axes
    BfAxis ax[3];
};

void bf_release(fx_plan* p) {
    BfState* bs = (BfState*)p->bf_state;
    if (!bs) return;
    if (bs->tab) (void)hipFree(bs->tab);
    if (bs->buf) (void)hipFree(bs->buf);
    if (bs->io) (void)hipFree(bs->io);
    delete bs;
    p->bf_state = nullptr;
}

}  // namespace fx

using namespace fx;

extern "C" fx_status fx_brute_force(fx_plan* p, const void* psi0, void* psi_out, void* rho_out, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    fx_status s = check_ptr(psi0, "psi0");
    if (s != FX_OK) return s;
    if (!psi_out && !rho_out) { set_error("psi_out and rho_out are both NULL"); return FX_EINVAL; }
    {
        const size_t cb = (size_t)p->M * csize(p);
        if ((s = check_disjoint(psi0, cb, "psi0", psi_out, cb, "psi_out")) != FX_OK) return s;
        if ((s = check_disjoint(psi0, cb, "psi0", rho_out, cb / 2, "rho_out")) != FX_OK) return s;
        if ((s = check_disjoint(psi_out, cb, "psi_out", rho_out, cb / 2, "rho_out")) != FX_OK) return s;
    }
    for (int pa = 0; pa < 3; ++pa)
        if (p->spectrum[pa]) {
            set_error("the brute-force comparator is built for the free-particle spectrum only");
            return FX_EUNSUPPORTED;
        }
    const int off = 3 - p->ndim;
    const size_t cs = csize(p);
    const int lmax = bf_lmax(p->dbl);
    if (!p->bf_state) {
        BfState* ns = new (std::nothrow) BfState();
        if (!ns) { set_error("host allocation failed"); return FX_ENOMEM; }
        p->bf_state = ns;
        size_t tab_bytes = 0, buf_elems = 0;
        std::vector<std::vector<double>> tws(3), phis(3);
        fx_status err = FX_OK;
        for (int pa = off; pa < 3 && err == FX_OK; ++pa) {
            BfAxis& a = ns->ax[pa];
            const int64_t N = (int64_t)p->ax[pa].lam * p->len[pa];
            a.N = (int)N;
            if (N > lmax) {
                // N = N1 N2 with both factors fitting one workgroup, as balanced as possible
                int best = 0;
                for (int f = 2; (int64_t)f * f <= N; ++f)
                    if (N % f == 0 && f <= lmax && N / f <= lmax) best = f;
                if (!best) {
                    set_error("padded axis length has no factorisation into workgroup-sized transforms");
                    err = FX_EUNSUPPORTED;
                    break;
                }
                a.two = true;
                a.N1 = (int)(N / best);
                a.N2 = best;
                int64_t A = 1, S = 1;
                for (int i = 0; i < pa; ++i) A *= p->len[i];
                for (int i = pa + 1; i < 3; ++i) S *= p->len[i];
                buf_elems = std::max<size_t>(buf_elems, (size_t)(A * N * S));
            }
            bf_tables(p, pa, a.N, tws[pa], phis[pa]);
            a.tw_off = tab_bytes;
            tab_bytes += ((size_t)N * cs + 255) / 256 * 256;
            a.phi_off = tab_bytes;
            tab_bytes += ((size_t)N * cs + 255) / 256 * 256;
        }
        if (err == FX_OK) {
            std::vector<unsigned char> host(tab_bytes, 0);
            for (int pa = off; pa < 3; ++pa) {
                const BfAxis& a = ns->ax[pa];
                for (int k = 0; k < 2 * a.N; ++k) {
                    if (p->dbl) {
                        std::memcpy(&host[a.tw_off + 8 * k], &tws[pa][k], 8);
                        std::memcpy(&host[a.phi_off + 8 * k], &phis[pa][k], 8);
                    } else {
                        const float t = (float)tws[pa][k], f = (float)phis[pa][k];
                        std::memcpy(&host[a.tw_off + 4 * k], &t, 4);
                        std::memcpy(&host[a.phi_off + 4 * k], &f, 4);
                    }
                }
            }
            if (hipMalloc(&ns->tab, std::max<size_t>(tab_bytes, 256)) != hipSuccess ||
                hipMalloc(&ns->io, (size_t)2 * p->M * cs) != hipSuccess ||
                (buf_elems && hipMalloc(&ns->buf, buf_elems * cs) != hipSuccess)) {
                (void)hipGetLastError();
                set_error("hipMalloc for the brute-force comparator failed");
                err = FX_ENOMEM;
            } else if (hipMemcpy(ns->tab, host.data(), tab_bytes, hipMemcpyHostToDevice) != hipSuccess) {
                set_error("brute-force table upload failed");
                err = FX_EDEVICE;
            }
        }
        if (err != FX_OK) {
            bf_release(p);
            return err;
        }
    }
    BfState* bs = (BfState*)p->bf_state;
    hipStream_t st = (hipStream_t)stream;
    const void* cur = psi0;
    char* io[2] = {(char*)bs->io, (char*)bs->io + (size_t)p->M * cs};
    for (int pa = off; pa < 3; ++pa) {
        const bool last = (pa == 2);
        void* dst = (last && psi_out) ? psi_out : io[(pa - off) & 1];
        int64_t A = 1, S = 1;
        for (int i = 0; i < pa; ++i) A *= p->len[i];
        for (int i = pa + 1; i < 3; ++i) S *= p->len[i];
        const BfAxis& a = bs->ax[pa];
        BfPass b{};
        b.A = A;
        b.S = S;
        b.M = (int)p->len[pa];
        b.N = a.N;
        b.N1 = a.N1;
        b.N2 = a.N2;
        b.lam = p->ax[pa].lam;
        b.tw = (const char*)bs->tab + a.tw_off;
        b.phi = (const char*)bs->tab + a.phi_off;
        if (!a.two) {
            b.mode = BfMode::SINGLE;
            b.L = a.N;
            b.TS = std::max(1, std::min(64, 2048 / a.N));
            while (b.TS > 1 && (int64_t)bf_lds(p->dbl, b.L, b.TS) > lds_limit_bytes()) --b.TS;
            b.nlines = A * S;
            b.in = cur;
            b.out = dst;
            b.rho = last ? rho_out : nullptr;
            if ((s = launch_bf(p, b, st)) != FX_OK) return s;
        } else {
            const BfMode modes[4] = {BfMode::F1, BfMode::F2, BfMode::I1, BfMode::I2};
            for (int k = 0; k < 4; ++k) {
                b.mode = modes[k];
                b.L = (k == 0 || k == 3) ? a.N1 : a.N2;
                b.TS = std::max(1, std::min(64, 2048 / b.L));
                while (b.TS > 1 && (int64_t)bf_lds(p->dbl, b.L, b.TS) > lds_limit_bytes()) --b.TS;
                b.nlines = (k == 0 || k == 3) ? A * a.N2 * S : A * a.N1 * S;
                b.in = (k == 0) ? cur : bs->buf;
                b.out = (k == 3) ? dst : bs->buf;
                b.rho = (k == 3 && last) ? rho_out : nullptr;
                if ((s = launch_bf(p, b, st)) != FX_OK) return s;
            }
        }
        cur = dst;
    }
    return FX_OK;
}
