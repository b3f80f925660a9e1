// Pass kernels specialised for power-of-two axes of 8 to 2048 points (gfx950).
//
// Same operations as the generic E and EA kernels (premultiply, forward transform,
// chirp, fold, pruned inverse, and for EA the twiddle-gather-accumulate over the
// magnification index), but the length-M transform is generated at compile time:
// a tile always holds 2048 points (2048/M lines), each of the 256 threads owns one
// radix-8 butterfly per stage (two radix-4 or four radix-2 butterflies for the one
// short stage), and every index is a shift or mask of compile-time constants. The
// length-P transform of the pruned inverse uses the runtime power-of-two stages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <set>

#include "device_common.h"
#include "fx_internal.h"

namespace fx {

namespace {

constexpr int kTilePoints2 = 2048;  // points per tile of the specialised kernels

// FP32 tiles are padded by one element per 256-byte bank row (32 complex64), which turns the
// strided Stockham stores into (nearly) conflict-free ones. FP64 tiles are not padded: there
// the extra address arithmetic and registers cost more than the conflicts (measured).
template <typename T> struct PadP { static constexpr bool on = sizeof(T) == 4; };
template <typename T> __device__ __forceinline__ int px(int i) {
    if constexpr (PadP<T>::on) return i + (i >> 5);
    else return i;
}
__host__ __device__ constexpr int padded_tile(bool dbl) { return dbl ? kTilePoints2 : kTilePoints2 + (kTilePoints2 >> 5) + 2; }

// Stage structure of a length-2^LM transform: the short radix (2 or 4) first, then radix 8.
template <int LM> struct Plan2 {
    static constexpr int LR0 = (LM % 3 != 0) ? (LM % 3) : 3;
    static constexpr int NST = 1 + (LM - LR0) / 3;
    static constexpr int lr(int s) { return s == 0 ? LR0 : 3; }
    static constexpr int lns(int s) { return s == 0 ? 0 : LR0 + 3 * (s - 1); }
};

// Twiddles of this thread's radix-8 butterfly in every stage after the first. The thread ->
// butterfly map is the same for every tile and every magnification index, so they are read
// once per workgroup and kept in registers.
// In FP64 the registers are too dear (occupancy), so the FP64 kernels read the roots from LDS.
template <typename T, int LM> struct TwReg {
    static constexpr bool kRegs = sizeof(T) == 4;
    C<T> w[kRegs ? Plan2<LM>::NST : 1][7];
    const C<T>* tw = nullptr;
    __device__ __forceinline__ void load(const C<T>* __restrict__ lds_tw) {
        tw = lds_tw;
        if constexpr (kRegs) {
            constexpr int M = 1 << LM;
            const int jj = threadIdx.x % (M / 8);
#pragma unroll
            for (int s = 1; s < Plan2<LM>::NST; ++s) {
                const int NS = 1 << Plan2<LM>::lns(s);
                const int k = jj % NS;
                const int tstep = M / (NS * 8);
#pragma unroll
                for (int t = 1; t < 8; ++t) w[s][t - 1] = lds_tw[t * k * tstep];
            }
        }
    }
    template <int S>
    __device__ __forceinline__ C<T> get(int t, int k) const {
        if constexpr (kRegs) {
            (void)k;
            return w[S][t - 1];
        } else {
            constexpr int M = 1 << LM;
            constexpr int NS = 1 << Plan2<LM>::lns(S);
            return tw[t * k * (M / (NS * 8))];
        }
    }
};

// One compile-time Stockham stage S of a length-2^LM transform over the 2048/M lines of a tile.
template <typename T, int LM, int S, bool INV>
__device__ __forceinline__ void p2_stage(const C<T>* __restrict__ X, C<T>* __restrict__ Y, const TwReg<T, LM>& tr,
                                         const C<T>* __restrict__ post) {
    constexpr int LR = Plan2<LM>::lr(S), LNS = Plan2<LM>::lns(S);
    constexpr int M = 1 << LM, R = 1 << LR, NS = 1 << LNS;
    constexpr int NB = M / R;
    constexpr int TPL = M / 8;  // threads per line
    constexpr int BPT = 8 / R;  // butterflies per thread
    const int tid = threadIdx.x;
    const int l = tid / TPL;
    const int g0 = tid % TPL;
    const int lo = l * M;
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int jj = g0 + i * TPL;
        const int k = jj % NS;
        C<T> v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) v[t] = X[px<T>(lo + jj + t * NB)];
        if constexpr (NS > 1) {
            static_assert(R == 8, "only the first stage has a short radix");
#pragma unroll
            for (int t = 1; t < R; ++t) {
                C<T> w = tr.template get<S>(t, k);
                if (INV) w.y = -w.y;
                v[t] = cmul<T>(v[t], w);
            }
        }
        Bfly<T, R>::run(v, INV);
        const int base = (jj - k) * R + k;
        if (post) {
#pragma unroll
            for (int t = 0; t < R; ++t) Y[px<T>(lo + base + t * NS)] = cmul<T>(v[t], post[base + t * NS]);
        } else {
#pragma unroll
            for (int t = 0; t < R; ++t) Y[px<T>(lo + base + t * NS)] = v[t];
        }
    }
}

template <typename T, int LM, int S, bool INV>
struct P2Run {
    static __device__ __forceinline__ C<T>* run(C<T>* X, C<T>* Y, const TwReg<T, LM>& tr, const C<T>* post) {
        if constexpr (S == Plan2<LM>::NST) {
            return X;
        } else {
            constexpr bool last = (S + 1 == Plan2<LM>::NST);
            p2_stage<T, LM, S, INV>(X, Y, tr, last ? post : nullptr);
            __syncthreads();
            return P2Run<T, LM, S + 1, INV>::run(Y, X, tr, post);
        }
    }
};

// Runtime power-of-two stage for the short pruned transforms (length 2^LP, lines at stride ls).
template <typename T, int LR>
__device__ void p2_stage_rt(const C<T>* __restrict__ X, C<T>* __restrict__ Y, int nl, int ls, int LP, int LNS,
                            const C<T>* __restrict__ tw, int tws, bool inv) {
    constexpr int R = 1 << LR;
    const int LNB = LP - LR;
    const int total = nl << LNB;
    const int tstep = (1 << (LP - LNS - LR)) * tws;
    const int nbm = (1 << LNB) - 1, nsm = (1 << LNS) - 1;
    for (int j = threadIdx.x; j < total; j += blockDim.x) {
        const int l = j >> LNB;
        const int jj = j & nbm;
        const int k = jj & nsm;
        const int lo = l * ls;
        C<T> v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) v[t] = X[px<T>(lo + jj + (t << LNB))];
        if (LNS > 0) {
#pragma unroll
            for (int t = 1; t < R; ++t) v[t] = cmul<T>(v[t], root<T>(tw, t * k * tstep, inv));
        }
        Bfly<T, R>::run(v, inv);
        const int base = ((jj - k) << LR) + k;
#pragma unroll
        for (int t = 0; t < R; ++t) Y[px<T>(lo + base + (t << LNS))] = v[t];
    }
}

template <typename T>
__device__ C<T>* p2_fft_rt(C<T>* X, C<T>* Y, int nl, int ls, int LP, const C<T>* __restrict__ tw, int tws,
                           bool inv) {
    int LNS = 0;
    while (LNS < LP) {
        const int LR = (LNS == 0 && (LP % 3) != 0) ? (LP % 3) : 3;
        if (LR == 1) p2_stage_rt<T, 1>(X, Y, nl, ls, LP, LNS, tw, tws, inv);
        else if (LR == 2) p2_stage_rt<T, 2>(X, Y, nl, ls, LP, LNS, tw, tws, inv);
        else p2_stage_rt<T, 3>(X, Y, nl, ls, LP, LNS, tw, tws, inv);
        __syncthreads();
        C<T>* t = X;
        X = Y;
        Y = t;
        LNS += LR;
    }
    return X;
}

// Z[l][u] = sum_{c<g} Y[l][u + c P] over the padded tile; P = 2^LP. Several threads share an
// output when there are few outputs; their partial sums meet in W (kThreads entries).
template <typename T>
__device__ void fold2(const C<T>* __restrict__ Y, C<T>* __restrict__ Z, C<T>* __restrict__ W, int nl, int M, int LP,
                      int g) {
    const int P = 1 << LP;
    const int outs = nl << LP;
    int K = 1;
    while (K * 2 <= g && outs * K * 2 <= kThreads) K *= 2;
    const int kb = __ffs(K) - 1;
    const int t = threadIdx.x;
    if (K == 1) {
        for (int e = t; e < outs; e += kThreads) {
            const int l = e >> LP, u = e & (P - 1);
            const int yo = l * M + u;
            C<T> acc = mk<T>(0, 0);
            for (int c = 0; c < g; ++c) acc = cadd<T>(acc, Y[px<T>(yo + c * P)]);
            Z[px<T>(yo)] = acc;
        }
        __syncthreads();
        return;
    }
    if (t < outs * K) {
        const int o = t >> kb, kk = t & (K - 1);
        const int l = o >> LP, u = o & (P - 1);
        const int yo = l * M + u;
        C<T> acc = mk<T>(0, 0);
        for (int c = kk; c < g; c += K) acc = cadd<T>(acc, Y[px<T>(yo + c * P)]);
        W[t] = acc;
    }
    __syncthreads();
    for (int e = t; e < outs; e += kThreads) {
        const int l = e >> LP, u = e & (P - 1);
        C<T> acc = W[e << kb];
        for (int kk = 1; kk < K; ++kk) acc = cadd<T>(acc, W[(e << kb) + kk]);
        Z[px<T>(l * M + u)] = acc;
    }
    __syncthreads();
}

template <typename T, int LM>
__device__ const C<T>* stage_roots_p2(C<T>* dst, const C<T>* __restrict__ src) {
    for (int i = threadIdx.x; i < (1 << LM); i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    return dst;
}

// ------------------------------------------------------------------------------------
// E for M = 2^LM: in [Qin][A][M][S] -> out [Qin*qn][A][P][S].
// ------------------------------------------------------------------------------------
template <typename T, int LM>
__global__ __launch_bounds__(kThreads) void k_E2(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                 PassGeom g, int LP) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int M = 1 << LM;
    constexpr int TS = kTilePoints2 / M;
    constexpr int PT = padded_tile(sizeof(T) == 8);
    const int P = ax.P;
    C<T>* B0 = (C<T>*)smem;
    C<T>* B1 = B0 + PT;
    const C<T>* tw = stage_roots_p2<T, LM>(B1 + PT, (const C<T>*)ax.tw);
    C<T>* Wsc = B1 + PT + M;
    TwReg<T, LM> tr;
    tr.load(tw);
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
        for (int k = 0; k < kTilePoints2 / kThreads; ++k) {
            const int e = threadIdx.x + k * kThreads;
            if (e < nl * M) {
                int l, n;
                const int64_t off = tile_elem(g, tl, qi, M, fdM, e, l, n);
                B0[px<T>(l * M + n)] = cmul<T>(in[off], ta[n]);
            }
        }
        __syncthreads();
        C<T>* Y = P2Run<T, LM, 0, false>::run(B0, B1, tr, TB + q * M);
        C<T>* Z = (Y == B0) ? B1 : B0;
        fold2<T>(Y, Z, Wsc, TS, M, LP, ax.g);
        C<T>* Rz = p2_fft_rt<T>(Z, Y, TS, M, LP, tw, ax.g, true);
        const int64_t qo = qi * g.qn + qq;
        for (int e = threadIdx.x; e < nl * P; e += blockDim.x) {
            int l, u;
            const int64_t off = tile_elem(g, tl, qo, P, fdP, e, l, u);
            out[off] = cscale<T>(Rz[px<T>(l * M + u)], scale);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// EH (adjoint of E, summed over the terms) for M = 2^LM >= kThreads: in [Qo*qn][A][P][S] ->
// out [Qo][A][M][S],
//   out = (1/M) sum_i conj(TA_q) IFFT_M( conj(TB_q) unfold( DFT_P(in_i) ) ),
// the conjugate transpose of every step of E in reverse order. One output line per workgroup:
// the rows of the 2048-point tile are 2048 / M terms of that line, transformed together, and
// each thread sums its M / kThreads output points over the rows and all terms in registers.
// ------------------------------------------------------------------------------------
template <typename T, int LM>
__global__ __launch_bounds__(kThreads) void k_EH2(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g, int accumulate, int LP) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int M = 1 << LM;
    constexpr int TS = kTilePoints2 / M;  // terms per round
    constexpr int ACC = M / kThreads;     // output points per thread
    constexpr int PT = padded_tile(sizeof(T) == 8);
    static_assert(ACC >= 1 && ACC * kThreads == M, "one line spans the workgroup");
    const int P = ax.P;
    C<T>* B0 = (C<T>*)smem;
    C<T>* B1 = B0 + PT;
    const C<T>* tw = stage_roots_p2<T, LM>(B1 + PT, (const C<T>*)ax.tw);
    TwReg<T, LM> tr;
    tr.load(tw);
    const C<T>* TA = (const C<T>*)ax.TA;
    const C<T>* TB = (const C<T>*)ax.TB;
    const T scale = (T)ax.scale;
    const int64_t S = g.S;
    const int64_t lines = g.Qin * g.A * S;  // Qin = output slices
    const int t = (int)threadIdx.x;
    // XCD-contiguous line order: workgroups are dispatched round-robin over the 8 XCDs (id mod 8),
    // so line (id mod 8) L8 + id / 8 gives each XCD a contiguous range, and the strided lines
    // (consecutive s) that share cache lines are read through one L2
    const int64_t L8 = (lines + 7) / 8;
    for (int64_t bid = blockIdx.x; bid < 8 * L8; bid += gridDim.x) {
        const int64_t L = (bid & 7) * L8 + (bid >> 3);
        if (L >= lines) continue;  // uniform over the workgroup
        const int64_t s = L % S;
        const int64_t t2 = L / S;
        const int64_t a = t2 % g.A;
        const int64_t qo = t2 / g.A;
        C<T> acc[ACC];
#pragma unroll
        for (int j = 0; j < ACC; ++j) acc[j] = mk<T>(0, 0);
        for (int i0 = 0; i0 < g.qn; i0 += TS) {
            // row r: the P inputs of term i0 + r (zero past the last term)
            for (int e = t; e < TS * P; e += kThreads) {
                const int r = e >> LP, u = e & (P - 1);
                const int i = i0 + r;
                C<T> v = mk<T>(0, 0);
                if (i < g.qn) v = in[(((qo * g.qn + i) * g.A + a) * P + u) * S + s];
                B0[px<T>(r * M + u)] = v;
            }
            __syncthreads();
            // forward P-point transform of every row (roots tw[k g])
            C<T>* Z = p2_fft_rt<T>(B0, B1, TS, M, LP, tw, ax.g, false);
            C<T>* Yb = (Z == B0) ? B1 : B0;
            // unfold with the conjugate chirp
#pragma unroll
            for (int k = 0; k < kTilePoints2 / kThreads; ++k) {
                const int e = t + k * kThreads;
                const int r = e >> LM, m = e & (M - 1);
                const int q = g.qb + min(i0 + r, g.qn - 1);
                Yb[px<T>(e)] = cmulc<T>(Z[px<T>(r * M + (m & (P - 1)))], TB[q * M + m]);
            }
            __syncthreads();
            const C<T>* Y = P2Run<T, LM, 0, true>::run(Yb, Z, tr, nullptr);
#pragma unroll
            for (int r = 0; r < TS; ++r) {
                if (i0 + r < g.qn) {
                    const int q = g.qb + i0 + r;
#pragma unroll
                    for (int j = 0; j < ACC; ++j) {
                        const int n = t + j * kThreads;
                        acc[j] = cfmac<T>(acc[j], Y[px<T>(r * M + n)], TA[q * M + n]);
                    }
                }
            }
            __syncthreads();  // the next round overwrites both buffers
        }
#pragma unroll
        for (int j = 0; j < ACC; ++j) {
            const int n = t + j * kThreads;
            const int64_t off = ((qo * g.A + a) * M + n) * S + s;
            C<T> v = cscale<T>(acc[j], scale);
            if (accumulate) v = cadd<T>(v, out[off]);
            out[off] = v;
        }
    }
}

// ------------------------------------------------------------------------------------
// EA for M = 2^LM: the 1-D prescription on every line, q loop inside the workgroup.
// ------------------------------------------------------------------------------------
template <typename T, int LM>
__global__ __launch_bounds__(kThreads) void k_EA2(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g, int accumulate, T* __restrict__ rho, int LP) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int M = 1 << LM;
    constexpr int TS = kTilePoints2 / M;
    constexpr int ACC = kTilePoints2 / kThreads;
    constexpr int PT = padded_tile(sizeof(T) == 8);
    const int P = ax.P;
    const FDiv fP(P);
    C<T>* RAW = (C<T>*)smem;
    C<T>* B0 = RAW + PT;
    C<T>* B1 = B0 + PT;
    const C<T>* tw = stage_roots_p2<T, LM>(B1 + PT, (const C<T>*)ax.tw);
    C<T>* Wsc = B1 + PT + M;
    TwReg<T, LM> tr;
    tr.load(tw);
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
        int en[ACC], er[ACC];
        int64_t eoff[ACC];
        C<T> acc[ACC];
#pragma unroll
        for (int k = 0; k < ACC; ++k) {
            const int e = threadIdx.x + k * kThreads;
            en[k] = 0;
            er[k] = 0;
            eoff[k] = 0;
            acc[k] = mk<T>(0, 0);
            if (e < cnt) {
                int l, n;
                eoff[k] = tile_elem(g, tl, qi, M, fdM, e, l, n);
                RAW[px<T>(l * M + n)] = in[eoff[k]];
                en[k] = n;
                er[k] = px<T>(l * M + fP.mod(n * ax.lg));  // LDS slot of the element's n'' sample
            }
        }
        __syncthreads();
        for (int i = 0; i < g.qn; ++i) {
            const int q = g.qb + i;
            const C<T>* ta = TA + q * M;
#pragma unroll
            for (int k = 0; k < ACC; ++k) {
                const int e = threadIdx.x + k * kThreads;  // every slot of the tile; unused lines are ignored
                B0[px<T>(e)] = cmul<T>(RAW[px<T>(e)], ta[e & (M - 1)]);
            }
            __syncthreads();
            C<T>* Y = P2Run<T, LM, 0, false>::run(B0, B1, tr, TB + q * M);
            C<T>* Z = (Y == B0) ? B1 : B0;
            fold2<T>(Y, Z, Wsc, TS, M, LP, ax.g);
            C<T>* Rz = p2_fft_rt<T>(Z, Y, TS, M, LP, tw, ax.g, true);
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
hipError_t prep_lds2(K kernel, size_t bytes) {
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

int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

template <typename T, int LM>
hipError_t launch_lm(Kind kind, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                     void* rho, hipStream_t st) {
    const int LP = ilog2(ax.P);
    const size_t lds = p2_lds_bytes(kind, sizeof(T) == 8, ax.M);
    if (kind == Kind::E) {
        auto k = k_E2<T, LM>;
        hipError_t e = prep_lds2(k, lds);
        if (e != hipSuccess) return e;
        int64_t blocks = g.Qin * g.qn * g.ntiles;
        if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = g.max_blocks;
        if (blocks > (1 << 22)) blocks = 1 << 22;
        hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kThreads), lds, st,
                           (const C<T>*)in, (C<T>*)out, ax, g, LP);
    } else {
        auto k = k_EA2<T, LM>;
        hipError_t e = prep_lds2(k, lds);
        if (e != hipSuccess) return e;
        int64_t blocks = g.Qin * g.ntiles;
        if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = g.max_blocks;
        if (blocks > (1 << 22)) blocks = 1 << 22;
        hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kThreads), lds, st,
                           (const C<T>*)in, (C<T>*)out, ax, g, accumulate, (T*)rho, LP);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_p2_T(Kind kind, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                       void* rho, hipStream_t st) {
    switch (ilog2(ax.M)) {
        case 3: return launch_lm<T, 3>(kind, in, out, ax, g, accumulate, rho, st);
        case 4: return launch_lm<T, 4>(kind, in, out, ax, g, accumulate, rho, st);
        case 5: return launch_lm<T, 5>(kind, in, out, ax, g, accumulate, rho, st);
        case 6: return launch_lm<T, 6>(kind, in, out, ax, g, accumulate, rho, st);
        case 7: return launch_lm<T, 7>(kind, in, out, ax, g, accumulate, rho, st);
        case 8: return launch_lm<T, 8>(kind, in, out, ax, g, accumulate, rho, st);
        case 9: return launch_lm<T, 9>(kind, in, out, ax, g, accumulate, rho, st);
        case 10: return launch_lm<T, 10>(kind, in, out, ax, g, accumulate, rho, st);
        case 11: return launch_lm<T, 11>(kind, in, out, ax, g, accumulate, rho, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int LM>
hipError_t launch_eh2_lm(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                         hipStream_t st) {
    const int LP = ilog2(ax.P);
    const size_t lds = eh2_lds_bytes(sizeof(T) == 8, ax.M);
    auto k = k_EH2<T, LM>;
    hipError_t e = prep_lds2(k, lds);
    if (e != hipSuccess) return e;
    int64_t blocks = (g.Qin * g.A * g.S + 7) / 8 * 8;  // the kernel's XCD-aware order
    if (blocks > (1 << 22)) blocks = 1 << 22;
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kThreads), lds, st, (const C<T>*)in,
                       (C<T>*)out, ax, g, accumulate, LP);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_eh2_T(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                        hipStream_t st) {
    switch (ilog2(ax.M)) {
        case 8: return launch_eh2_lm<T, 8>(in, out, ax, g, accumulate, st);
        case 9: return launch_eh2_lm<T, 9>(in, out, ax, g, accumulate, st);
        case 10: return launch_eh2_lm<T, 10>(in, out, ax, g, accumulate, st);
        case 11: return launch_eh2_lm<T, 11>(in, out, ax, g, accumulate, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool eh2_applicable(int M, int P) {
    return M >= kThreads && M <= kTilePoints2 && (M & (M - 1)) == 0 && P >= 1 && M % P == 0;
}

size_t eh2_lds_bytes(bool dbl, int M) {
    return (2 * (size_t)padded_tile(dbl) + (size_t)M) * (dbl ? 16 : 8);
}

hipError_t launch_pass_eh2(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                           int accumulate, hipStream_t st) {
    if (!eh2_applicable(ax.M, ax.P)) return hipErrorInvalidValue;
    return dbl ? launch_eh2_T<double>(in, out, ax, g, accumulate, st)
               : launch_eh2_T<float>(in, out, ax, g, accumulate, st);
}

bool p2_applicable(Kind kind, int M) {
    if (kind != Kind::E && kind != Kind::EA) return false;
    if (M < 8 || M > kTilePoints2 || (M & (M - 1)) != 0) return false;
    return true;
}

int p2_tile_lines(int M) { return kTilePoints2 / M; }

size_t p2_lds_bytes(Kind kind, bool dbl, int M) {
    const size_t c = dbl ? 16 : 8;
    const size_t nbuf = (kind == Kind::EA) ? 3 : 2;
    return (nbuf * (size_t)padded_tile(dbl) + (size_t)M + kThreads) * c;
}

hipError_t launch_pass_p2(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                          int accumulate, void* rho, hipStream_t st) {
    if (!p2_applicable(kind, ax.M) || g.TS != p2_tile_lines(ax.M)) return hipErrorInvalidValue;
    return dbl ? launch_p2_T<double>(kind, in, out, ax, g, accumulate, rho, st)
               : launch_p2_T<float>(kind, in, out, ax, g, accumulate, rho, st);
}

}  // namespace fx
