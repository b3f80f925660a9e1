// Pass kernels with compile-time transforms for axis lengths 3 * 2^k (12 to 1536 points).
//
// Same operations as the generic E and EA kernels. A tile holds floor(2048/M) lines; the
// length-M transform is a Stockham sequence fixed at compile time (radix 3, then the short
// power-of-two radix, then radix 8), so every index is a constant-divisor multiply-shift
// and every loop is unrolled. The pruned inverse of length P = M/g uses the runtime
// mixed-radix stages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <set>

#include "device_common.h"
#include "fx_internal.h"

namespace fx {

namespace {

constexpr int kTileCap = 2048;

// s-th radix of the compile-time plan of length M (0 past the last stage).
constexpr int ct_rad(int M, int s) {
    int m = M, idx = 0;
    while (m % 3 == 0) {
        if (idx == s) return 3;
        m /= 3;
        ++idx;
    }
    int k = 0;
    while ((1 << k) < m) ++k;
    const int r0 = k % 3;
    if (r0 != 0) {
        if (idx == s) return 1 << r0;
        ++idx;
        k -= r0;
    }
    while (k > 0) {
        if (idx == s) return 8;
        ++idx;
        k -= 3;
    }
    return 0;
}
constexpr int ct_nst(int M) {
    int s = 0;
    while (ct_rad(M, s) != 0) ++s;
    return s;
}
constexpr int ct_ns(int M, int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= ct_rad(M, i);
    return p;
}

template <typename T, int M, int S, bool INV>
__device__ __forceinline__ void ct_stage(const C<T>* __restrict__ X, C<T>* __restrict__ Y,
                                         const C<T>* __restrict__ tw, const C<T>* __restrict__ post) {
    constexpr int R = ct_rad(M, S), NS = ct_ns(M, S);
    constexpr int NB = M / R;
    constexpr int TS = kTileCap / M;
    constexpr int TOT = TS * NB;
    constexpr int ITER = (TOT + kThreads - 1) / kThreads;
    constexpr int TSTEP = M / (NS * R);
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int j = threadIdx.x + it * kThreads;
        if ((TOT % kThreads) == 0 || j < TOT) {
            const int l = j / NB;
            const int jj = j - l * NB;
            const int k = jj % NS;
            const C<T>* x = X + l * M;
            C<T>* y = Y + l * M;
            C<T> v[R];
#pragma unroll
            for (int t = 0; t < R; ++t) v[t] = x[jj + t * NB];
            if constexpr (NS > 1) {
#pragma unroll
                for (int t = 1; t < R; ++t) v[t] = cmul<T>(v[t], root<T>(tw, t * k * TSTEP, INV));
            }
            Bfly<T, R>::run(v, INV);
            const int base = (jj - k) * R + k;
            if (post) {
#pragma unroll
                for (int t = 0; t < R; ++t) y[base + t * NS] = cmul<T>(v[t], post[base + t * NS]);
            } else {
#pragma unroll
                for (int t = 0; t < R; ++t) y[base + t * NS] = v[t];
            }
        }
    }
}

template <typename T, int M, int S, bool INV>
struct CtRun {
    static __device__ __forceinline__ C<T>* run(C<T>* X, C<T>* Y, const C<T>* tw, const C<T>* post) {
        if constexpr (S == ct_nst(M)) {
            return X;
        } else {
            constexpr bool last = (S + 1 == ct_nst(M));
            ct_stage<T, M, S, INV>(X, Y, tw, last ? post : nullptr);
            __syncthreads();
            return CtRun<T, M, S + 1, INV>::run(Y, X, tw, post);
        }
    }
};

template <typename T>
__device__ const C<T>* stage_roots_ct(C<T>* dst, const C<T>* __restrict__ src, int M) {
    for (int i = threadIdx.x; i < M; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    return dst;
}

template <typename T, int M>
__global__ __launch_bounds__(kThreads) void k_Ect(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int TS = kTileCap / M;
    constexpr int TILE = TS * M;
    constexpr int LOADS = (TILE + kThreads - 1) / kThreads;
    const int P = ax.P;
    const FDiv fP(P);
    C<T>* B0 = (C<T>*)smem;
    C<T>* B1 = B0 + TILE;
    const C<T>* tw = stage_roots_ct<T>(B1 + TILE, (const C<T>*)ax.tw, M);
    C<T>* Wsc = B1 + TILE + M;
    const C<T>* TA = (const C<T>*)ax.TA;
    const C<T>* TB = (const C<T>*)ax.TB;
    const T scale = (T)ax.scale;
    const int total = (int)(g.Qin * g.qn * g.ntiles);
    const FDiv fnt((int)g.ntiles), fqn(g.qn);
    for (int bid = blockIdx.x; bid < total; bid += gridDim.x) {
        const int rest = fnt.div(bid);
        const int tt = bid - rest * (int)g.ntiles;
        const int qi32 = fqn.div(rest);
        const int qq = rest - qi32 * g.qn;
        const int64_t qi = qi32;
        const int q = g.qb + qq;
        const Tile tl = decode_tile(g, tt);
        const FDiv fdM = tile_div(g, tl, M), fdP = tile_div(g, tl, P);
        const int nl = tl.nl;
        const C<T>* ta = TA + q * M;
#pragma unroll
        for (int k = 0; k < LOADS; ++k) {
            const int e = threadIdx.x + k * kThreads;
            if (e < nl * M) {
                int l, n;
                const int64_t off = tile_elem(g, tl, qi, M, fdM, e, l, n);
                B0[l * M + n] = cmul<T>(in[off], ta[n]);
            }
        }
        __syncthreads();
        C<T>* Y = CtRun<T, M, 0, false>::run(B0, B1, tw, TB + q * M);
        C<T>* Z = (Y == B0) ? B1 : B0;
        fold_lines<T>(Y, Z, Wsc, TS, M, P, ax.g, fP);
        C<T>* Rz = lds_fft<T>(Z, Y, TS, M, ax.fp, tw, ax.g, true);
        const int64_t qo = qi * g.qn + qq;
        for (int e = threadIdx.x; e < nl * P; e += blockDim.x) {
            int l, u;
            const int64_t off = tile_elem(g, tl, qo, P, fdP, e, l, u);
            out[off] = cscale<T>(Rz[l * M + u], scale);
        }
        __syncthreads();
    }
}

template <typename T, int M>
__global__ __launch_bounds__(kThreads) void k_EAct(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                   PassGeom g, int accumulate, T* __restrict__ rho) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int TS = kTileCap / M;
    constexpr int TILE = TS * M;
    constexpr int ACC = (TILE + kThreads - 1) / kThreads;
    const int P = ax.P;
    const FDiv fP(P);
    C<T>* RAW = (C<T>*)smem;
    C<T>* B0 = RAW + TILE;
    C<T>* B1 = B0 + TILE;
    const C<T>* tw = stage_roots_ct<T>(B1 + TILE, (const C<T>*)ax.tw, M);
    C<T>* Wsc = B1 + TILE + M;
    const C<T>* TA = (const C<T>*)ax.TA;
    const C<T>* TB = (const C<T>*)ax.TB;
    const C<T>* Tf = (const C<T>*)ax.Tf;
    const T scale = (T)ax.scale;
    const int total = (int)(g.Qin * g.ntiles);
    const FDiv fnt((int)g.ntiles);
    for (int bid = blockIdx.x; bid < total; bid += gridDim.x) {
        const int qi32 = fnt.div(bid);
        const int tt = bid - qi32 * (int)g.ntiles;
        const int64_t qi = qi32;
        const Tile tl = decode_tile(g, tt);
        const FDiv fdM = tile_div(g, tl, M);
        const int nl = tl.nl;
        const int cnt = nl * M;
        int en[ACC], es[ACC], er[ACC];
        int64_t eoff[ACC];
        C<T> acc[ACC];
#pragma unroll
        for (int k = 0; k < ACC; ++k) {
            const int e = threadIdx.x + k * kThreads;
            en[k] = es[k] = er[k] = 0;
            eoff[k] = 0;
            acc[k] = mk<T>(0, 0);
            if (e < cnt) {
                int l, n;
                eoff[k] = tile_elem(g, tl, qi, M, fdM, e, l, n);
                RAW[l * M + n] = in[eoff[k]];
                en[k] = n;
                es[k] = l * M + n;
                er[k] = l * M + fP.mod(n * ax.lg);
            }
        }
        __syncthreads();
        for (int i = 0; i < g.qn; ++i) {
            const int q = g.qb + i;
            const C<T>* ta = TA + q * M;
#pragma unroll
            for (int k = 0; k < ACC; ++k) {
                const int e = threadIdx.x + k * kThreads;
                if ((TILE % kThreads) == 0 || e < TILE) B0[e] = cmul<T>(RAW[e], ta[e % M]);
            }
            __syncthreads();
            C<T>* Y = CtRun<T, M, 0, false>::run(B0, B1, tw, TB + q * M);
            C<T>* Z = (Y == B0) ? B1 : B0;
            fold_lines<T>(Y, Z, Wsc, TS, M, P, ax.g, fP);
            C<T>* Rz = lds_fft<T>(Z, Y, TS, M, ax.fp, tw, ax.g, true);
            const C<T>* tf = Tf + q * M;
#pragma unroll
            for (int k = 0; k < ACC; ++k) {
                const int e = threadIdx.x + k * kThreads;
                if (e < cnt) acc[k] = cfma<T>(acc[k], tf[en[k]], Rz[er[k]]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < ACC; ++k) {
            const int e = threadIdx.x + k * kThreads;
            if (e < cnt) {
                C<T> v = cscale<T>(acc[k], scale);
                if (accumulate) v = cadd<T>(v, out[eoff[k]]);
                out[eoff[k]] = v;
                if (rho) rho[eoff[k]] = v.x * v.x + v.y * v.y;
            }
        }
        __syncthreads();
    }
}

template <typename K>
hipError_t prep_lds_ct(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    static std::mutex mu;
    static std::set<const void*> done;
    std::lock_guard<std::mutex> lk(mu);
    if (done.count((const void*)kernel)) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       lds_limit_bytes());
    if (e == hipSuccess) done.insert((const void*)kernel);
    return e;
}

template <typename T, int M>
hipError_t launch_m(Kind kind, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                    void* rho, hipStream_t st) {
    const size_t lds = ct_lds_bytes(kind, sizeof(T) == 8, M);
    int64_t blocks = (kind == Kind::E) ? g.Qin * g.qn * g.ntiles : g.Qin * g.ntiles;
    if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = g.max_blocks;
    blocks = std::min<int64_t>(std::max<int64_t>(blocks, 1), 1 << 22);
    if (kind == Kind::E) {
        auto k = k_Ect<T, M>;
        hipError_t e = prep_lds_ct(k, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kThreads), lds, st, (const C<T>*)in, (C<T>*)out, ax, g);
    } else {
        auto k = k_EAct<T, M>;
        hipError_t e = prep_lds_ct(k, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kThreads), lds, st, (const C<T>*)in, (C<T>*)out, ax, g,
                           accumulate, (T*)rho);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ct_T(Kind kind, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                       void* rho, hipStream_t st) {
    switch (ax.M) {
        case 12: return launch_m<T, 12>(kind, in, out, ax, g, accumulate, rho, st);
        case 24: return launch_m<T, 24>(kind, in, out, ax, g, accumulate, rho, st);
        case 48: return launch_m<T, 48>(kind, in, out, ax, g, accumulate, rho, st);
        case 96: return launch_m<T, 96>(kind, in, out, ax, g, accumulate, rho, st);
        case 192: return launch_m<T, 192>(kind, in, out, ax, g, accumulate, rho, st);
        case 384: return launch_m<T, 384>(kind, in, out, ax, g, accumulate, rho, st);
        case 768: return launch_m<T, 768>(kind, in, out, ax, g, accumulate, rho, st);
        case 1536: return launch_m<T, 1536>(kind, in, out, ax, g, accumulate, rho, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool ct_applicable(Kind kind, int M) {
    if (kind != Kind::E && kind != Kind::EA) return false;
    switch (M) {
        case 12: case 24: case 48: case 96: case 192: case 384: case 768: case 1536: return true;
        default: return false;
    }
}

int ct_tile_lines(int M) { return kTileCap / M; }

size_t ct_lds_bytes(Kind kind, bool dbl, int M) {
    const size_t c = dbl ? 16 : 8;
    const size_t nbuf = (kind == Kind::EA) ? 3 : 2;
    const size_t tile = (size_t)(kTileCap / M) * M;
    return (nbuf * tile + (size_t)M + kThreads) * c;
}

hipError_t launch_pass_ct(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                          int accumulate, void* rho, hipStream_t st) {
    if (!ct_applicable(kind, ax.M) || g.TS != ct_tile_lines(ax.M)) return hipErrorInvalidValue;
    return dbl ? launch_ct_T<double>(kind, in, out, ax, g, accumulate, rho, st)
               : launch_ct_T<float>(kind, in, out, ax, g, accumulate, rho, st);
}

}  // namespace fx
