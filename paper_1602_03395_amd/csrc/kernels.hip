// HIP kernels of the free-flight expansion (gfx950).
//
// The prescription (FF) of section 5.2 is a sum over q = (q_0..q_{d-1}) of
// products of per-axis factors: the premultiply (presA), the forward DFT, the
// chirp (presB), the inverse DFT read at n'' (FFaux) and the twiddle f (presf)
// all act on one axis at a time. Every kernel here therefore works on "lines"
// along one axis of a tensor laid out as [slices][A][L][S] (L the axis
// length, S the product of the lengths after it), with a tile of TS lines
// staged in LDS:
//
//   E   : line of M -> TA_q -> FFT_M -> TB_q -> fold to P = M/g -> inverse DFT_P
//         (the output-pruned form of the inverse FFT: only the P distinct
//         n'' = g * r are computed, section 7.2) -> one slice per q.
//   A   : for each output point nb: sum over q of Tf_q[nb] * line_q[r(nb)],
//         r(nb) = (nb lam/g) mod P -- the gather/accumulate of (FFpsi).
//   EA  : E followed by A on the same line, the q loop inside the workgroup
//         (the 1-D prescription applied to each line).
//   EH, AH, EAH : Hermitian adjoints of the three (conjugated tables, forward
//         and inverse transforms exchanged, fold <-> unfold, gather <-> preimage
//         gather), used for U^H.
//
// Transforms are mixed-radix Stockham passes in LDS (radix 2, 3, 4, 8 with
// register butterflies; any other radix by a direct small DFT), ping-ponging
// between two LDS buffers with one barrier per stage. Roots come from the
// FP64-built table tw[k] = exp(-2 pi i k / M) of the axis; a length-P
// transform reads it with stride g.
//
// Global loads and stores of a tile are coalesced: for contiguous lines
// (S == 1) consecutive threads walk along the line, for strided lines
// (S > 1) they walk across the TS adjacent lines.
#include <hip/hip_runtime.h>

#include <mutex>
#include <set>

#include "fx_internal.h"

namespace fx {

template <typename T> struct CT;
template <> struct CT<float> { using type = float2; };
template <> struct CT<double> { using type = double2; };
template <typename T> using C = typename CT<T>::type;

template <typename T> __device__ __forceinline__ C<T> mk(T x, T y) { C<T> r; r.x = x; r.y = y; return r; }
template <typename T> __device__ __forceinline__ C<T> cadd(C<T> a, C<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ C<T> csub(C<T> a, C<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ C<T> cmul(C<T> a, C<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T> __device__ __forceinline__ C<T> cmulc(C<T> a, C<T> b) {
    return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// acc + a * b
template <typename T> __device__ __forceinline__ C<T> cfma(C<T> acc, C<T> a, C<T> b) {
    return mk<T>(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);
}
// acc + a * conj(b)
template <typename T> __device__ __forceinline__ C<T> cfmac(C<T> acc, C<T> a, C<T> b) {
    return mk<T>(acc.x + a.x * b.x + a.y * b.y, acc.y + a.y * b.x - a.x * b.y);
}
template <typename T> __device__ __forceinline__ C<T> cscale(C<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <typename T> __device__ __forceinline__ C<T> rot(C<T> a, bool inv) {
    return inv ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// ------------------------------------------------------------------------------------
// Register butterflies: v <- DFT_R(v), sign - (forward) or + (inverse), unnormalised.
// ------------------------------------------------------------------------------------
template <typename T, int R> struct Bfly;

template <typename T> struct Bfly<T, 2> {
    static __device__ __forceinline__ void run(C<T>* v, bool) {
        C<T> a = v[0], b = v[1];
        v[0] = cadd<T>(a, b);
        v[1] = csub<T>(a, b);
    }
};

template <typename T> struct Bfly<T, 3> {
    static __device__ __forceinline__ void run(C<T>* v, bool inv) {
        const T h = (T)0.86602540378443864676372317075294;  // sin(pi/3)
        C<T> s = cadd<T>(v[1], v[2]);
        C<T> d = csub<T>(v[1], v[2]);
        C<T> m = mk<T>(v[0].x - (T)0.5 * s.x, v[0].y - (T)0.5 * s.y);
        C<T> r = rot<T>(cscale<T>(d, h), inv);  // -i h d (forward)
        v[0] = cadd<T>(v[0], s);
        v[1] = cadd<T>(m, r);
        v[2] = csub<T>(m, r);
    }
};

template <typename T> struct Bfly<T, 4> {
    static __device__ __forceinline__ void run(C<T>* v, bool inv) {
        C<T> t0 = cadd<T>(v[0], v[2]);
        C<T> t1 = csub<T>(v[0], v[2]);
        C<T> t2 = cadd<T>(v[1], v[3]);
        C<T> t3 = rot<T>(csub<T>(v[1], v[3]), inv);
        v[0] = cadd<T>(t0, t2);
        v[2] = csub<T>(t0, t2);
        v[1] = cadd<T>(t1, t3);
        v[3] = csub<T>(t1, t3);
    }
};

template <typename T> struct Bfly<T, 8> {
    static __device__ __forceinline__ void run(C<T>* v, bool inv) {
        const T r2 = (T)0.70710678118654752440084436210485;  // sqrt(1/2)
        C<T> e[4] = {v[0], v[2], v[4], v[6]};
        C<T> o[4] = {v[1], v[3], v[5], v[7]};
        Bfly<T, 4>::run(e, inv);
        Bfly<T, 4>::run(o, inv);
        // o[u] *= exp(-+ 2 pi i u / 8)
        C<T> o1 = o[1];
        o[1] = inv ? mk<T>(r2 * (o1.x - o1.y), r2 * (o1.x + o1.y)) : mk<T>(r2 * (o1.x + o1.y), r2 * (o1.y - o1.x));
        o[2] = rot<T>(o[2], inv);
        C<T> o3 = o[3];
        o[3] = inv ? mk<T>(-r2 * (o3.x + o3.y), r2 * (o3.x - o3.y)) : mk<T>(r2 * (o3.y - o3.x), -r2 * (o3.x + o3.y));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[u] = cadd<T>(e[u], o[u]);
            v[u + 4] = csub<T>(e[u], o[u]);
        }
    }
};

// Division by a workgroup-uniform divisor: shifts for powers of two, otherwise a
// float-reciprocal quotient corrected to the exact one (x < 2^22), else the
// integer divide.
struct FDiv {
    int d;
    int sh;
    float inv;
    bool p2;
    __device__ __forceinline__ explicit FDiv(int dd) : d(dd) {
        p2 = (dd & (dd - 1)) == 0;
        sh = p2 ? (__ffs(dd) - 1) : 0;
        inv = 1.0f / (float)dd;
    }
    __device__ __forceinline__ int div(int x) const {
        if (p2) return x >> sh;
        if (x >= (1 << 22)) return x / d;
        int q = (int)((float)x * inv);
        int r = x - q * d;
        if (r < 0) { q -= 1; r += d; }
        if (r >= d) { q += 1; }
        return q;
    }
    __device__ __forceinline__ int mod(int x) const { return x - div(x) * d; }
};

template <typename T> __device__ __forceinline__ C<T> root(const C<T>* __restrict__ tw, int idx, bool inv) {
    C<T> w = tw[idx];
    if (inv) w.y = -w.y;
    return w;
}

// One Stockham stage with a compile-time radix over nl lines of length N at LDS stride ls.
template <typename T, int R>
__device__ void stage_r(const C<T>* __restrict__ X, C<T>* __restrict__ Y, int nl, int ls, int N, int Ns,
                        const C<T>* __restrict__ tw, int tws, bool inv, const C<T>* __restrict__ post) {
    const int nb = N / R;
    const int total = nl * nb;
    const int tstep = (N / (Ns * R)) * tws;
    const FDiv fnb(nb), fns(Ns);
    for (int j = threadIdx.x; j < total; j += blockDim.x) {
        const int l = fnb.div(j);
        const int jj = j - l * nb;
        const C<T>* x = X + l * ls;
        C<T>* y = Y + l * ls;
        const int k = fns.mod(jj);
        C<T> v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) v[t] = x[jj + t * nb];
        if (Ns > 1) {
#pragma unroll
            for (int t = 1; t < R; ++t) v[t] = cmul<T>(v[t], root<T>(tw, t * k * tstep, inv));
        }
        Bfly<T, R>::run(v, inv);
        const int base = (jj - k) * R + k;
        if (post) {
#pragma unroll
            for (int t = 0; t < R; ++t) y[base + t * Ns] = cmul<T>(v[t], post[base + t * Ns]);
        } else {
#pragma unroll
            for (int t = 0; t < R; ++t) y[base + t * Ns] = v[t];
        }
    }
}

// Any radix: direct R-point DFT per butterfly, roots from the same table.
template <typename T>
__device__ void stage_gen(const C<T>* __restrict__ X, C<T>* __restrict__ Y, int nl, int ls, int N, int Ns,
                          int R, const C<T>* __restrict__ tw, int tws, bool inv, const C<T>* __restrict__ post) {
    const int nb = N / R;
    const int total = nl * nb;
    const int tstep = (N / (Ns * R)) * tws;
    const int rstep = nb * tws;
    for (int j = threadIdx.x; j < total; j += blockDim.x) {
        const int l = j / nb;
        const int jj = j - l * nb;
        const C<T>* x = X + l * ls;
        C<T>* y = Y + l * ls;
        const int k = jj % Ns;
        const int base = (jj / Ns) * Ns * R + k;
        for (int u = 0; u < R; ++u) {
            C<T> acc = mk<T>(0, 0);
            for (int t = 0; t < R; ++t) {
                C<T> v = x[jj + t * nb];
                if (Ns > 1 && t > 0) v = cmul<T>(v, root<T>(tw, t * k * tstep, inv));
                acc = cfma<T>(acc, v, root<T>(tw, ((t * u) % R) * rstep, inv));
            }
            y[base + u * Ns] = post ? cmul<T>(acc, post[base + u * Ns]) : acc;
        }
    }
}

// Transform nl lines of length pl.n held in X (stride ls); returns the buffer holding the result.
// With `post` (a global row of pl.n values) the output is multiplied by it elementwise in the
// last stage (the chirp of (presB) fused into the forward transform).
template <typename T>
__device__ C<T>* lds_fft(C<T>* X, C<T>* Y, int nl, int ls, const RadixPlan& pl, const C<T>* __restrict__ tw,
                         int tws, bool inv, const C<T>* __restrict__ post = nullptr) {
    int Ns = 1;
    const int N = pl.n;
    if (pl.nst == 0 && post) {
        for (int e = threadIdx.x; e < nl * N; e += blockDim.x) {
            const int l = e / N;
            const int n = e - l * N;
            X[l * ls + n] = cmul<T>(X[l * ls + n], post[n]);
        }
        __syncthreads();
    }
    for (int s = 0; s < pl.nst; ++s) {
        const int R = pl.rad[s];
        const C<T>* pp = (s + 1 == pl.nst) ? post : nullptr;
        switch (R) {
            case 2: stage_r<T, 2>(X, Y, nl, ls, N, Ns, tw, tws, inv, pp); break;
            case 3: stage_r<T, 3>(X, Y, nl, ls, N, Ns, tw, tws, inv, pp); break;
            case 4: stage_r<T, 4>(X, Y, nl, ls, N, Ns, tw, tws, inv, pp); break;
            case 8: stage_r<T, 8>(X, Y, nl, ls, N, Ns, tw, tws, inv, pp); break;
            default: stage_gen<T>(X, Y, nl, ls, N, Ns, R, tw, tws, inv, pp); break;
        }
        __syncthreads();
        C<T>* t = X;
        X = Y;
        Y = t;
        Ns *= R;
    }
    return X;
}

// Z[l][u] = sum_{c<g} Y[l][u + c P] for nl lines (line stride ls). Several threads share an
// output when there are few outputs; their partial sums meet in the scratch W (blockDim entries).
template <typename T>
__device__ void fold_lines(const C<T>* __restrict__ Y, C<T>* __restrict__ Z, C<T>* __restrict__ W, int nl, int ls,
                           int P, int g, const FDiv& fP) {
    const int outs = nl * P;
    int K = 1;
    while (K * 2 <= g && outs * K * 2 <= (int)blockDim.x) K *= 2;
    if (K == 1) {
        for (int e = threadIdx.x; e < outs; e += blockDim.x) {
            const int l = fP.div(e);
            const int u = e - l * P;
            const C<T>* y = Y + l * ls + u;
            C<T> acc = mk<T>(0, 0);
            for (int c = 0; c < g; ++c) acc = cadd<T>(acc, y[c * P]);
            Z[l * ls + u] = acc;
        }
        __syncthreads();
        return;
    }
    const int kb = __ffs(K) - 1;
    const int t = threadIdx.x;
    if (t < outs * K) {
        const int o = t >> kb;
        const int kk = t & (K - 1);
        const int l = fP.div(o);
        const int u = o - l * P;
        const C<T>* y = Y + l * ls + u;
        C<T> acc = mk<T>(0, 0);
        for (int c = kk; c < g; c += K) acc = cadd<T>(acc, y[c * P]);
        W[t] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < outs; e += blockDim.x) {
        const int l = fP.div(e);
        const int u = e - l * P;
        C<T> acc = W[e << kb];
        for (int kk = 1; kk < K; ++kk) acc = cadd<T>(acc, W[(e << kb) + kk]);
        Z[l * ls + u] = acc;
    }
    __syncthreads();
}

// ------------------------------------------------------------------------------------
// Tile geometry
// ------------------------------------------------------------------------------------
struct Tile {
    int64_t a0;
    int64_t s0;
    int nl;
};

__device__ __forceinline__ Tile decode_tile(const PassGeom& g, int64_t t) {
    Tile r;
    if (g.S == 1) {
        r.a0 = t * g.TS;
        r.s0 = 0;
        r.nl = (int)min((int64_t)g.TS, g.A - r.a0);
    } else {
        const int64_t nsc = (g.S + g.TS - 1) / g.TS;
        r.a0 = t / nsc;
        r.s0 = (t - r.a0 * nsc) * g.TS;
        r.nl = (int)min((int64_t)g.TS, g.S - r.s0);
    }
    return r;
}

// Element e of a tile of nl lines of length L -> (line l, position n) and global offset in slice `slice`.
// `fd` divides by L when the lines are contiguous (S == 1) and by nl otherwise.
__device__ __forceinline__ int64_t tile_elem(const PassGeom& g, const Tile& tl, int64_t slice, int L,
                                             const FDiv& fd, int e, int& l, int& n) {
    if (g.S == 1) {
        l = fd.div(e);
        n = e - l * L;
        return (slice * g.A + tl.a0 + l) * L + n;
    }
    n = fd.div(e);
    l = e - n * tl.nl;
    return ((slice * g.A + tl.a0) * L + n) * g.S + tl.s0 + l;
}

__device__ __forceinline__ FDiv tile_div(const PassGeom& g, const Tile& tl, int L) {
    return FDiv(g.S == 1 ? L : tl.nl);
}

template <typename T> __device__ __forceinline__ const C<T>* tab(const void* p) { return (const C<T>*)p; }

// Copies the axis' FFT roots into LDS (after the tile buffers) once per workgroup.
template <typename T>
__device__ const C<T>* stage_roots(C<T>* dst, const AxisDev& ax) {
    const C<T>* src = (const C<T>*)ax.tw;
    for (int i = threadIdx.x; i < ax.M; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    return dst;
}

// ------------------------------------------------------------------------------------
// E: per q, line of M -> P values of B^(q) along this axis (times 1/M).
// in [Qin][A][M][S] -> out [Qin*qn][A][P][S], slice index qi*qn + (q - qb).
// ------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_E(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                PassGeom g) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int M = ax.M, P = ax.P;
    const FDiv fM(M), fP(P);
    C<T>* B0 = (C<T>*)smem;
    C<T>* B1 = B0 + g.TS * M;
    const C<T>* TA = tab<T>(ax.TA);
    const C<T>* TB = tab<T>(ax.TB);
    const C<T>* tw = stage_roots<T>(B1 + g.TS * M, ax);
    C<T>* Wsc = B1 + g.TS * M + M;  // fold scratch, kThreads entries
    const T scale = (T)ax.scale;
    const int64_t total = g.Qin * g.qn * g.ntiles;
    for (int64_t bid = blockIdx.x; bid < total; bid += gridDim.x) {
        const int64_t tt = bid % g.ntiles;
        const int64_t rest = bid / g.ntiles;
        const int qq = (int)(rest % g.qn);
        const int64_t qi = rest / g.qn;
        const int q = g.qb + qq;
        const Tile tl = decode_tile(g, tt);
        const FDiv fdM = tile_div(g, tl, M), fdP = tile_div(g, tl, P);
        const int nl = tl.nl;
        for (int e = threadIdx.x; e < nl * M; e += blockDim.x) {
            int l, n;
            const int64_t off = tile_elem(g, tl, qi, M, fdM, e, l, n);
            B0[l * M + n] = cmul<T>(in[off], TA[q * M + n]);
        }
        __syncthreads();
        C<T>* Y = lds_fft<T>(B0, B1, nl, M, ax.fm, tw, 1, false, TB + q * M);
        C<T>* Z = (Y == B0) ? B1 : B0;
        fold_lines<T>(Y, Z, Wsc, nl, M, P, ax.g, fP);
        C<T>* Rz = lds_fft<T>(Z, Y, nl, M, ax.fp, tw, ax.g, true);
        const int64_t qo = qi * g.qn + qq;
        for (int e = threadIdx.x; e < nl * P; e += blockDim.x) {
            int l, u;
            const int64_t off = tile_elem(g, tl, qo, P, fdP, e, l, u);
            out[off] = cscale<T>(Rz[l * M + u], scale);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// A: out[qo][a][nb][s] (+)= sum_i Tf[qb+i][nb] * in[qo*qn+i][a][r(nb)][s]   (one thread per output)
// ------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_A(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                PassGeom g, int accumulate, T* __restrict__ rho) {
    // grid: x over the (nb, s) plane of one (qo, a) row, y over rows
    const int M = ax.M, P = ax.P;
    const int S = (int)g.S;
    const int MS = M * S;
    const FDiv fS(S), fP(P);
    const C<T>* Tf = tab<T>(ax.Tf);
    const int64_t rows = g.Qin * g.A;
    const int64_t step = g.A * (int64_t)P * S;  // one magnification slice of the input
    for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
        const int64_t qo = row / g.A;
        const int64_t a = row - qo * g.A;
        const C<T>* src0 = in + ((qo * g.qn) * g.A + a) * (int64_t)P * S;
        C<T>* dst = out + row * (int64_t)MS;
        T* rdst = rho ? rho + row * (int64_t)MS : nullptr;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < MS; e += gridDim.x * blockDim.x) {
            const int n = fS.div(e);
            const int s = e - n * S;
            const int r = fP.mod(n * ax.lg);
            const C<T>* src = src0 + r * S + s;
            const C<T>* tf = Tf + g.qb * M + n;
            C<T> acc = mk<T>(0, 0);
            for (int i = 0; i < g.qn; ++i) acc = cfma<T>(acc, tf[i * M], src[i * step]);
            if (accumulate) acc = cadd<T>(acc, dst[e]);
            dst[e] = acc;
            if (rdst) rdst[e] = acc.x * acc.x + acc.y * acc.y;
        }
    }
}

// ------------------------------------------------------------------------------------
// EA: the 1-D prescription on each line: out = sum_q Tf_q * gather_r(E_q(line)).
// in [Qin][A][M][S] -> out [Qin][A][M][S]. LDS: raw tile + two transform buffers.
// ------------------------------------------------------------------------------------
template <typename T, int ACCN>
__global__ __launch_bounds__(kThreads) void k_EA(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                 PassGeom g, int accumulate, T* __restrict__ rho) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int M = ax.M, P = ax.P;
    const FDiv fM(M), fP(P);
    C<T>* RAW = (C<T>*)smem;
    C<T>* B0 = RAW + g.TS * M;
    C<T>* B1 = B0 + g.TS * M;
    const C<T>* TA = tab<T>(ax.TA);
    const C<T>* TB = tab<T>(ax.TB);
    const C<T>* Tf = tab<T>(ax.Tf);
    const C<T>* tw = stage_roots<T>(B1 + g.TS * M, ax);
    C<T>* Wsc = B1 + g.TS * M + M;  // fold scratch, kThreads entries
    const T scale = (T)ax.scale;
    const int64_t total = g.Qin * g.ntiles;
    for (int64_t bid = blockIdx.x; bid < total; bid += gridDim.x) {
        const int64_t tt = bid % g.ntiles;
        const int64_t qi = bid / g.ntiles;
        const Tile tl = decode_tile(g, tt);
        const FDiv fdM = tile_div(g, tl, M), fdP = tile_div(g, tl, P);
        const int nl = tl.nl;
        const int cnt = nl * M;
        int el[ACCN], en[ACCN];
        int64_t eoff[ACCN];
        C<T> acc[ACCN];
#pragma unroll
        for (int k = 0; k < ACCN; ++k) {
            const int e = threadIdx.x + k * kThreads;
            el[k] = 0;
            en[k] = 0;
            eoff[k] = 0;
            acc[k] = mk<T>(0, 0);
            if (e < cnt) {
                eoff[k] = tile_elem(g, tl, qi, M, fdM, e, el[k], en[k]);
                RAW[el[k] * M + en[k]] = in[eoff[k]];
            }
        }
        __syncthreads();
        for (int i = 0; i < g.qn; ++i) {
            const int q = g.qb + i;
            for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
                const int n = fM.mod(e);
                B0[e] = cmul<T>(RAW[e], TA[q * M + n]);
            }
            __syncthreads();
            C<T>* Y = lds_fft<T>(B0, B1, nl, M, ax.fm, tw, 1, false, TB + q * M);
            C<T>* Z = (Y == B0) ? B1 : B0;
            fold_lines<T>(Y, Z, Wsc, nl, M, P, ax.g, fP);
            C<T>* Rz = lds_fft<T>(Z, Y, nl, M, ax.fp, tw, ax.g, true);
#pragma unroll
            for (int k = 0; k < ACCN; ++k) {
                const int e = threadIdx.x + k * kThreads;
                if (e < cnt) {
                    const int r = fP.mod(en[k] * ax.lg);
                    acc[k] = cfma<T>(acc[k], Tf[q * M + en[k]], Rz[el[k] * M + r]);
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < ACCN; ++k) {
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

// ------------------------------------------------------------------------------------
// EH: adjoint of E, summed over the qn magnification indices:
// in [Qo*qn][A][P][S] -> out [Qo][A][M][S]:
//   out = (1/M) sum_i conj(TA_q) * IFFT_M( conj(TB_q) * unfold( DFT_P(in_i) ) )
// ------------------------------------------------------------------------------------
template <typename T, int ACCN>
__global__ __launch_bounds__(kThreads) void k_EH(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                 PassGeom g, int accumulate) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int M = ax.M, P = ax.P;
    const FDiv fM(M), fP(P);
    C<T>* B0 = (C<T>*)smem;
    C<T>* B1 = B0 + g.TS * M;
    const C<T>* TA = tab<T>(ax.TA);
    const C<T>* TB = tab<T>(ax.TB);
    const C<T>* tw = stage_roots<T>(B1 + g.TS * M, ax);
    C<T>* Wsc = B1 + g.TS * M + M;  // fold scratch, kThreads entries
    const T scale = (T)ax.scale;
    const int64_t total = g.Qin * g.ntiles;  // Qin = output slices here
    for (int64_t bid = blockIdx.x; bid < total; bid += gridDim.x) {
        const int64_t tt = bid % g.ntiles;
        const int64_t qo = bid / g.ntiles;
        const Tile tl = decode_tile(g, tt);
        const FDiv fdM = tile_div(g, tl, M), fdP = tile_div(g, tl, P);
        const int nl = tl.nl;
        const int cnt = nl * M;
        int el[ACCN], en[ACCN];
        int64_t eoff[ACCN];
        C<T> acc[ACCN];
#pragma unroll
        for (int k = 0; k < ACCN; ++k) {
            const int e = threadIdx.x + k * kThreads;
            el[k] = en[k] = 0;
            eoff[k] = 0;
            acc[k] = mk<T>(0, 0);
            if (e < cnt) eoff[k] = tile_elem(g, tl, qo, M, fdM, e, el[k], en[k]);
        }
        for (int i = 0; i < g.qn; ++i) {
            const int q = g.qb + i;
            const int64_t si = qo * g.qn + i;
            for (int e = threadIdx.x; e < nl * P; e += blockDim.x) {
                int l, u;
                const int64_t off = tile_elem(g, tl, si, P, fdP, e, l, u);
                B0[l * M + u] = in[off];
            }
            __syncthreads();
            C<T>* Z = lds_fft<T>(B0, B1, nl, M, ax.fp, tw, ax.g, false);
            C<T>* Yb = (Z == B0) ? B1 : B0;
            for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
                const int l = fM.div(e);
                const int m = e - l * M;
                Yb[e] = cmulc<T>(Z[l * M + fP.mod(m)], TB[q * M + m]);
            }
            __syncthreads();
            C<T>* Y = lds_fft<T>(Yb, Z, nl, M, ax.fm, tw, 1, true);
#pragma unroll
            for (int k = 0; k < ACCN; ++k) {
                const int e = threadIdx.x + k * kThreads;
                if (e < cnt) acc[k] = cfmac<T>(acc[k], Y[el[k] * M + en[k]], TA[q * M + en[k]]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < ACCN; ++k) {
            const int e = threadIdx.x + k * kThreads;
            if (e < cnt) {
                C<T> v = cscale<T>(acc[k], scale);
                if (accumulate) v = cadd<T>(v, out[eoff[k]]);
                out[eoff[k]] = v;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// AH: adjoint of A (preimage gather, no atomics):
// out[qo*qn+i][a][r][s] = sum_{c<g} conj(Tf[qb+i][n(r,c)]) * in[qo][a][n(r,c)][s],
// n(r,c) = (r * lg_inv mod P) + c P are exactly the nb with r(nb) = r.
// ------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_AH(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                 PassGeom g) {
    // grid: x over the (r, s) plane of one output slice row, y over rows (qo, i, a)
    const int M = ax.M, P = ax.P;
    const int S = (int)g.S;
    const int PS = P * S;
    const FDiv fS(S), fP(P);
    const C<T>* Tf = tab<T>(ax.Tf);
    const int64_t rows = g.Qin * g.qn * g.A;  // Qin = input slices (Qo)
    for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
        const int64_t a = row % g.A;
        const int64_t t = row / g.A;
        const int i = (int)(t % g.qn);
        const int64_t qo = t / g.qn;
        const int q = g.qb + i;
        const C<T>* src0 = in + (qo * g.A + a) * (int64_t)M * S;
        C<T>* dst = out + row * (int64_t)PS;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < PS; e += gridDim.x * blockDim.x) {
            const int r = fS.div(e);
            const int s = e - r * S;
            const int n0 = fP.mod(r * ax.lg_inv);
            C<T> acc = mk<T>(0, 0);
            for (int c = 0; c < ax.g; ++c) {
                const int n = n0 + c * P;
                acc = cfmac<T>(acc, src0[n * S + s], Tf[q * M + n]);
            }
            dst[e] = acc;
        }
    }
}

// ------------------------------------------------------------------------------------
// EAH: adjoint of EA on each line.
// ------------------------------------------------------------------------------------
template <typename T, int ACCN>
__global__ __launch_bounds__(kThreads) void k_EAH(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g, int accumulate) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int M = ax.M, P = ax.P;
    const FDiv fM(M), fP(P);
    C<T>* RAW = (C<T>*)smem;
    C<T>* B0 = RAW + g.TS * M;
    C<T>* B1 = B0 + g.TS * M;
    const C<T>* TA = tab<T>(ax.TA);
    const C<T>* TB = tab<T>(ax.TB);
    const C<T>* Tf = tab<T>(ax.Tf);
    const C<T>* tw = stage_roots<T>(B1 + g.TS * M, ax);
    C<T>* Wsc = B1 + g.TS * M + M;  // fold scratch, kThreads entries
    const T scale = (T)ax.scale;
    const int64_t total = g.Qin * g.ntiles;
    for (int64_t bid = blockIdx.x; bid < total; bid += gridDim.x) {
        const int64_t tt = bid % g.ntiles;
        const int64_t qi = bid / g.ntiles;
        const Tile tl = decode_tile(g, tt);
        const FDiv fdM = tile_div(g, tl, M), fdP = tile_div(g, tl, P);
        const int nl = tl.nl;
        const int cnt = nl * M;
        int el[ACCN], en[ACCN];
        int64_t eoff[ACCN];
        C<T> acc[ACCN];
#pragma unroll
        for (int k = 0; k < ACCN; ++k) {
            const int e = threadIdx.x + k * kThreads;
            el[k] = en[k] = 0;
            eoff[k] = 0;
            acc[k] = mk<T>(0, 0);
            if (e < cnt) {
                eoff[k] = tile_elem(g, tl, qi, M, fdM, e, el[k], en[k]);
                RAW[el[k] * M + en[k]] = in[eoff[k]];
            }
        }
        __syncthreads();
        for (int i = 0; i < g.qn; ++i) {
            const int q = g.qb + i;
            for (int e = threadIdx.x; e < nl * P; e += blockDim.x) {
                const int l = fP.div(e);
                const int r = e - l * P;
                const int n0 = fP.mod(r * ax.lg_inv);
                C<T> a2 = mk<T>(0, 0);
                for (int c = 0; c < ax.g; ++c) {
                    const int n = n0 + c * P;
                    a2 = cfmac<T>(a2, RAW[l * M + n], Tf[q * M + n]);
                }
                B0[l * M + r] = a2;
            }
            __syncthreads();
            C<T>* Z = lds_fft<T>(B0, B1, nl, M, ax.fp, tw, ax.g, false);
            C<T>* Yb = (Z == B0) ? B1 : B0;
            for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
                const int l = fM.div(e);
                const int m = e - l * M;
                Yb[e] = cmulc<T>(Z[l * M + fP.mod(m)], TB[q * M + m]);
            }
            __syncthreads();
            C<T>* Y = lds_fft<T>(Yb, Z, nl, M, ax.fm, tw, 1, true);
#pragma unroll
            for (int k = 0; k < ACCN; ++k) {
                const int e = threadIdx.x + k * kThreads;
                if (e < cnt) acc[k] = cfmac<T>(acc[k], Y[el[k] * M + en[k]], TA[q * M + en[k]]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < ACCN; ++k) {
            const int e = threadIdx.x + k * kThreads;
            if (e < cnt) {
                C<T> v = cscale<T>(acc[k], scale);
                if (accumulate) v = cadd<T>(v, out[eoff[k]]);
                out[eoff[k]] = v;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// Small elementwise kernels
// ------------------------------------------------------------------------------------
template <typename T>
__global__ void k_density(const C<T>* __restrict__ psi, T* __restrict__ rho, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const C<T> v = psi[i];
        rho[i] = v.x * v.x + v.y * v.y;
    }
}

// img[a][s] = w * sum_l rho[a][l][s]
template <typename T>
__global__ void k_column(const T* __restrict__ rho, T* __restrict__ img, int64_t A, int64_t L, int64_t S, T w) {
    const int64_t total = A * S;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = i / S;
        const int64_t s = i - a * S;
        T acc = 0;
        for (int64_t l = 0; l < L; ++l) acc += rho[(a * L + l) * S + s];
        img[i] = acc * w;
    }
}

struct PtrArr {
    const void* p[64];
};
struct PtrArrW {
    void* p[64];
    void* r[64];
};

template <typename T>
__global__ void k_gather(PtrArr src, C<T>* __restrict__ dst, int64_t n_each, int count) {
    const int64_t total = n_each * count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / n_each);
        dst[i] = ((const C<T>*)src.p[b])[i - (int64_t)b * n_each];
    }
}

template <typename T>
__global__ void k_scatter(const C<T>* __restrict__ src, PtrArrW dst, int64_t n_each, int count, int want_rho) {
    const int64_t total = n_each * count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / n_each);
        const int64_t j = i - (int64_t)b * n_each;
        const C<T> v = src[i];
        if (dst.p[b]) ((C<T>*)dst.p[b])[j] = v;
        if (want_rho && dst.r[b]) ((T*)dst.r[b])[j] = v.x * v.x + v.y * v.y;
    }
}

// ------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------
namespace {

int elem_blocks(int64_t total) {
    int64_t b = (total + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > (1 << 20)) b = 1 << 20;
    return (int)b;
}

dim3 plane_grid(int64_t plane, int64_t rows) {
    int64_t bx = (plane + kThreads - 1) / kThreads;
    if (bx < 1) bx = 1;
    if (bx > 65535) bx = 65535;
    int64_t by = rows < 1 ? 1 : rows;
    if (by > 65535) by = 65535;
    return dim3((unsigned)bx, (unsigned)by);
}

int tile_blocks(int64_t total, int cap = 0) {
    if (total < 1) total = 1;
    if (total > (1 << 22)) total = 1 << 22;
    if (cap > 0 && total > cap) total = cap;
    return (int)total;
}

// Raises a kernel's dynamic-LDS limit to the device maximum once (before any graph capture
// that launches it: the plan and batch set-up runs every kernel eagerly first).
template <typename K>
hipError_t prep_lds(K kernel, size_t bytes) {
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

template <typename T, int ACCN>
hipError_t launch_acc_kind(Kind kind, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                           int accumulate, void* rho, hipStream_t st) {
    const size_t lds = pass_lds_bytes(kind, sizeof(T) == 8, g.TS, ax.M);
    const int blocks = tile_blocks(g.Qin * g.ntiles, g.max_blocks);
    hipError_t err = hipSuccess;
    switch (kind) {
        case Kind::EA: {
            auto k = k_EA<T, ACCN>;
            if ((err = prep_lds(k, lds)) != hipSuccess) return err;
            hipLaunchKernelGGL(k, dim3(blocks), dim3(kThreads), lds, st, (const C<T>*)in, (C<T>*)out, ax, g,
                               accumulate, (T*)rho);
            break;
        }
        case Kind::EH: {
            auto k = k_EH<T, ACCN>;
            if ((err = prep_lds(k, lds)) != hipSuccess) return err;
            hipLaunchKernelGGL(k, dim3(blocks), dim3(kThreads), lds, st, (const C<T>*)in, (C<T>*)out, ax, g,
                               accumulate);
            break;
        }
        case Kind::EAH: {
            auto k = k_EAH<T, ACCN>;
            if ((err = prep_lds(k, lds)) != hipSuccess) return err;
            hipLaunchKernelGGL(k, dim3(blocks), dim3(kThreads), lds, st, (const C<T>*)in, (C<T>*)out, ax, g,
                               accumulate);
            break;
        }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_T(Kind kind, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                    void* rho, hipStream_t st) {
    switch (kind) {
        case Kind::E: {
            const size_t lds = pass_lds_bytes(kind, sizeof(T) == 8, g.TS, ax.M);
            auto k = k_E<T>;
            hipError_t err = prep_lds(k, lds);
            if (err != hipSuccess) return err;
            hipLaunchKernelGGL(k, dim3(tile_blocks(g.Qin * g.qn * g.ntiles, g.max_blocks)), dim3(kThreads), lds, st,
                               (const C<T>*)in, (C<T>*)out, ax, g);
            return hipGetLastError();
        }
        case Kind::A: {
            const dim3 grid = plane_grid((int64_t)ax.M * g.S, g.Qin * g.A);
            hipLaunchKernelGGL(k_A<T>, grid, dim3(kThreads), 0, st, (const C<T>*)in, (C<T>*)out, ax, g,
                               accumulate, (T*)rho);
            return hipGetLastError();
        }
        case Kind::AH: {
            const dim3 grid = plane_grid((int64_t)ax.P * g.S, g.Qin * g.qn * g.A);
            hipLaunchKernelGGL(k_AH<T>, grid, dim3(kThreads), 0, st, (const C<T>*)in, (C<T>*)out, ax, g);
            return hipGetLastError();
        }
        default: break;
    }
    const int pts = g.TS * ax.M;
    const int need = (pts + kThreads - 1) / kThreads;
    if (need <= 1) return launch_acc_kind<T, 1>(kind, in, out, ax, g, accumulate, rho, st);
    if (need <= 2) return launch_acc_kind<T, 2>(kind, in, out, ax, g, accumulate, rho, st);
    if (need <= 4) return launch_acc_kind<T, 4>(kind, in, out, ax, g, accumulate, rho, st);
    if (need <= 8) return launch_acc_kind<T, 8>(kind, in, out, ax, g, accumulate, rho, st);
    if (need <= 16) return launch_acc_kind<T, 16>(kind, in, out, ax, g, accumulate, rho, st);
    return hipErrorInvalidValue;
}

}  // namespace

size_t pass_lds_bytes(Kind kind, bool dbl, int TS, int M) {
    const size_t c = dbl ? 16 : 8;
    switch (kind) {
        case Kind::E:
        case Kind::EH: return ((2 * (size_t)TS + 1) * M + kThreads) * c;
        case Kind::EA:
        case Kind::EAH: return ((3 * (size_t)TS + 1) * M + kThreads) * c;
        default: return 0;
    }
}

hipError_t launch_pass(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                       int accumulate, void* rho, hipStream_t st) {
    return dbl ? launch_T<double>(kind, in, out, ax, g, accumulate, rho, st)
               : launch_T<float>(kind, in, out, ax, g, accumulate, rho, st);
}

hipError_t launch_density(bool dbl, const void* psi, void* rho, int64_t n, hipStream_t st) {
    if (dbl)
        hipLaunchKernelGGL(k_density<double>, dim3(elem_blocks(n)), dim3(kThreads), 0, st, (const double2*)psi,
                           (double*)rho, n);
    else
        hipLaunchKernelGGL(k_density<float>, dim3(elem_blocks(n)), dim3(kThreads), 0, st, (const float2*)psi,
                           (float*)rho, n);
    return hipGetLastError();
}

hipError_t launch_column(bool dbl, const void* rho, void* img, int64_t A, int64_t L, int64_t S, double w,
                         hipStream_t st) {
    if (dbl)
        hipLaunchKernelGGL(k_column<double>, dim3(elem_blocks(A * S)), dim3(kThreads), 0, st, (const double*)rho,
                           (double*)img, A, L, S, w);
    else
        hipLaunchKernelGGL(k_column<float>, dim3(elem_blocks(A * S)), dim3(kThreads), 0, st, (const float*)rho,
                           (float*)img, A, L, S, (float)w);
    return hipGetLastError();
}

hipError_t launch_gather(bool dbl, const void* const* srcs, void* dst, int64_t n_each, int count, hipStream_t st) {
    if (count > 64) return hipErrorInvalidValue;
    PtrArr a;
    for (int i = 0; i < count; ++i) a.p[i] = srcs[i];
    const int64_t total = n_each * count;
    if (dbl)
        hipLaunchKernelGGL(k_gather<double>, dim3(elem_blocks(total)), dim3(kThreads), 0, st, a, (double2*)dst,
                           n_each, count);
    else
        hipLaunchKernelGGL(k_gather<float>, dim3(elem_blocks(total)), dim3(kThreads), 0, st, a, (float2*)dst,
                           n_each, count);
    return hipGetLastError();
}

hipError_t launch_scatter(bool dbl, const void* src, void* const* dsts, int64_t n_each, int count, int want_rho,
                          void* const* rhos, hipStream_t st) {
    if (count > 64) return hipErrorInvalidValue;
    PtrArrW a;
    for (int i = 0; i < count; ++i) {
        a.p[i] = dsts ? dsts[i] : nullptr;
        a.r[i] = rhos ? rhos[i] : nullptr;
    }
    const int64_t total = n_each * count;
    if (dbl)
        hipLaunchKernelGGL(k_scatter<double>, dim3(elem_blocks(total)), dim3(kThreads), 0, st, (const double2*)src,
                           a, n_each, count, want_rho);
    else
        hipLaunchKernelGGL(k_scatter<float>, dim3(elem_blocks(total)), dim3(kThreads), 0, st, (const float2*)src,
                           a, n_each, count, want_rho);
    return hipGetLastError();
}

}  // namespace fx
