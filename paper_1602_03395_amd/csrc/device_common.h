// Device helpers shared by the pass kernels (kernels.hip, kernels_p2.hip): complex arithmetic,
// register butterflies, the runtime mixed-radix Stockham engine, folds and tile addressing.
#pragma once

#include <hip/hip_runtime.h>

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

// Synchronisation of one wavefront's LDS traffic (lines owned by a single wave).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work distribution of a transform stage: in block mode the whole workgroup walks all
// (line, butterfly) pairs; in wave mode wave w owns lines w, w + nwaves, ... and its 64 lanes
// walk the butterflies of those lines only, so a stage needs no workgroup barrier.
struct Walk {
    bool wave;
    int start, step;  // over the flattened (line, butterfly) index
    __device__ __forceinline__ Walk(bool w) : wave(w) {
        start = threadIdx.x;
        step = blockDim.x;
    }
};

__device__ __forceinline__ void stage_sync(bool wave) {
    if (wave) wave_sync();
    else __syncthreads();
}

// One Stockham stage with a compile-time radix over nl lines of length N at LDS stride ls.
template <typename T, int R>
__device__ void stage_r(const C<T>* __restrict__ X, C<T>* __restrict__ Y, int nl, int ls, int N, int Ns,
                        const C<T>* __restrict__ tw, int tws, bool inv, const C<T>* __restrict__ post,
                        bool wave) {
    const int nb = N / R;
    const int tstep = (N / (Ns * R)) * tws;
    const FDiv fnb(nb), fns(Ns);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int total = wave ? ((nl - w + nw - 1) / nw) * nb : nl * nb;
    for (int j = wave ? lane : threadIdx.x; j < total; j += wave ? 64 : blockDim.x) {
        int l = fnb.div(j);
        const int jj = j - l * nb;
        if (wave) l = w + l * nw;
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
                          int R, const C<T>* __restrict__ tw, int tws, bool inv, const C<T>* __restrict__ post,
                          bool wave) {
    const int nb = N / R;
    const int tstep = (N / (Ns * R)) * tws;
    const int rstep = nb * tws;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int total = wave ? ((nl - w + nw - 1) / nw) * nb : nl * nb;
    for (int j = wave ? lane : threadIdx.x; j < total; j += wave ? 64 : blockDim.x) {
        int l = j / nb;
        const int jj = j - l * nb;
        if (wave) l = w + l * nw;
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
                         int tws, bool inv, const C<T>* __restrict__ post = nullptr, bool wave = false) {
    int Ns = 1;
    const int N = pl.n;
    if (pl.nst == 0 && post) {
        const int w = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
        for (int l = wave ? w : 0; l < nl; l += wave ? nw : 1)
            for (int n = wave ? lane : threadIdx.x; n < N; n += wave ? 64 : blockDim.x)
                X[l * ls + n] = cmul<T>(X[l * ls + n], post[n]);
        stage_sync(wave);
    }
    for (int s = 0; s < pl.nst; ++s) {
        const int R = pl.rad[s];
        const C<T>* pp = (s + 1 == pl.nst) ? post : nullptr;
        switch (R) {
            case 2: stage_r<T, 2>(X, Y, nl, ls, N, Ns, tw, tws, inv, pp, wave); break;
            case 3: stage_r<T, 3>(X, Y, nl, ls, N, Ns, tw, tws, inv, pp, wave); break;
            case 4: stage_r<T, 4>(X, Y, nl, ls, N, Ns, tw, tws, inv, pp, wave); break;
            case 8: stage_r<T, 8>(X, Y, nl, ls, N, Ns, tw, tws, inv, pp, wave); break;
            default: stage_gen<T>(X, Y, nl, ls, N, Ns, R, tw, tws, inv, pp, wave); break;
        }
        stage_sync(wave);
        C<T>* t = X;
        X = Y;
        Y = t;
        Ns *= R;
    }
    return X;
}

// Z[l][u] = sum_{c<g} Y[l][u + c P] for nl lines (line stride ls). Several threads share an
// output when there are few outputs; their partial sums meet in the scratch W (blockDim entries).
template <typename T> __device__ __forceinline__ C<T> shfl_xor(C<T> v, int m) {
    return mk<T>(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}

// Wave mode: each wave folds its own lines; up to 64/P lanes share an output and combine their
// partial sums with lane shuffles.
template <typename T>
__device__ void fold_lines_wave(const C<T>* __restrict__ Y, C<T>* __restrict__ Z, int nl, int ls, int P, int g) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int K = 1;
    while (K * 2 <= g && P * K * 2 <= 64) K *= 2;
    for (int l = w; l < nl; l += nw) {
        const C<T>* y = Y + l * ls;
        if (K == 1) {
            for (int u = lane; u < P; u += 64) {
                C<T> acc = mk<T>(0, 0);
                for (int c = 0; c < g; ++c) acc = cadd<T>(acc, y[u + c * P]);
                Z[l * ls + u] = acc;
            }
        } else {
            const int u = lane / K;   // K is a power of two; all 64 lanes take part in the shuffles
            const int kk = lane & (K - 1);
            C<T> acc = mk<T>(0, 0);
            if (u < P)
                for (int c = kk; c < g; c += K) acc = cadd<T>(acc, y[u + c * P]);
            for (int m = K >> 1; m > 0; m >>= 1) acc = cadd<T>(acc, shfl_xor<T>(acc, m));
            if (u < P && kk == 0) Z[l * ls + u] = acc;
        }
    }
    wave_sync();
}

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
        const int nsc = (int)((g.S + g.TS - 1) / g.TS);
        const FDiv fd(nsc);
        const int a0 = fd.div((int)t);  // tiles per slice < 2^31 (checked on the host)
        r.a0 = a0;
        r.s0 = (int64_t)((int)t - a0 * nsc) * g.TS;
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

}  // namespace fx
