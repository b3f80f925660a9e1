// Register form of the E and EA passes for short pruned lengths (P = M / g in {1, 2, 3, 4, 6, 8, 12,
// 16}, g a power of two <= 64).
//
// The E pass of one axis maps a line x[0..M) to, for every magnification index q, the P values
//   E_q[u] = (1/M) sum_r exp(2 pi i r u / P) sum_c (TB_q FFT_M(TA_q x))[r + P c]      (FF), (FFaux)
// With n = g n1 + n2 the forward transform splits into P-point transforms of the g stride-g
// subsequences, and the chirp, the alias fold over c and the remaining g-point stage fold into
// one table HT_q[n2][r] (built on the host in FP64, see tables.cpp):
//   E_q[u] = sum_n2 IDFT_P( HT_q[n2] * DFT_P( x[g n1 + n2] * TA_q[g n1] ) )[u].
// One thread owns one (line, n2): its P inputs stay in registers for every q of the workgroup,
// the two P-point transforms run in registers with constant twiddles, and the sum over n2 is a
// butterfly reduction across the g lanes of the line (a line never straddles a wavefront).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <set>

#include "fx_internal.h"
#include "device_common.h"

namespace fx {
namespace {

constexpr int kWave = 64;
constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// cos(2 pi e / 32) for e = 0..8; the other 32nd roots follow by symmetry
constexpr double kQ32[9] = {1.0,
                            0.980785280403230449126182236134,
                            0.923879532511286756128183189397,
                            0.831469612302545237078788377618,
                            0.707106781186547524400844362105,
                            0.555570233019602224742830813949,
                            0.382683432365089771728459984030,
                            0.195090322016128267848284868477,
                            0.0};
constexpr double cos32(int e) {
    e &= 31;
    return e <= 8 ? kQ32[e] : e <= 16 ? -kQ32[16 - e] : e <= 24 ? -kQ32[e - 16] : kQ32[32 - e];
}
constexpr double sin32(int e) { return cos32(e + 24); }  // sin x = cos(x - pi/2)

// a * exp(-+2 pi i e / 32) (forward sign -, inverse +), e a compile-time constant
template <typename T, bool INV, int E>
__device__ __forceinline__ C<T> tw32(C<T> a) {
    constexpr int e = E & 31;
    if constexpr (e == 0) return a;
    else if constexpr (e == 8) return rot<T>(a, INV);
    else if constexpr (e == 16) return mk<T>(-a.x, -a.y);
    else if constexpr (e == 24) return rot<T>(a, !INV);
    else {
        constexpr double cd = cos32(e), sd = sin32(e);
        const T c = (T)cd;
        const T s = INV ? (T)sd : (T)-sd;
        return mk<T>(a.x * c - a.y * s, a.x * s + a.y * c);
    }
}
template <typename T, bool INV, int E>
__device__ __forceinline__ C<T> tw16(C<T> a) { return tw32<T, INV, 2 * E>(a); }

template <typename T, bool INV>
__device__ __forceinline__ void dft2(C<T>& a, C<T>& b) {
    const C<T> t = a;
    a = cadd<T>(t, b);
    b = csub<T>(t, b);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(C<T>& a0, C<T>& a1, C<T>& a2, C<T>& a3) {
    const C<T> t0 = cadd<T>(a0, a2), t1 = csub<T>(a0, a2);
    const C<T> t2 = cadd<T>(a1, a3), t3 = rot<T>(csub<T>(a1, a3), INV);
    a0 = cadd<T>(t0, t2);
    a2 = csub<T>(t0, t2);
    a1 = cadd<T>(t1, t3);
    a3 = csub<T>(t1, t3);
}

// In-register DFT of N points, natural order in and out.
template <typename T, int N, bool INV> struct RegDFT;

template <typename T, bool INV> struct RegDFT<T, 1, INV> {
    __device__ __forceinline__ static void run(C<T>*) {}
};
template <typename T, bool INV> struct RegDFT<T, 2, INV> {
    __device__ __forceinline__ static void run(C<T>* v) { dft2<T, INV>(v[0], v[1]); }
};
template <typename T, bool INV> struct RegDFT<T, 4, INV> {
    __device__ __forceinline__ static void run(C<T>* v) { dft4<T, INV>(v[0], v[1], v[2], v[3]); }
};
template <typename T, bool INV> struct RegDFT<T, 8, INV> {
    // radix 2 over two 4-point transforms of the even and odd samples
    __device__ __forceinline__ static void run(C<T>* v) {
        C<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        C<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4<T, INV>(e0, e1, e2, e3);
        dft4<T, INV>(o0, o1, o2, o3);
        o1 = tw16<T, INV, 2>(o1);
        o2 = tw16<T, INV, 4>(o2);
        o3 = tw16<T, INV, 6>(o3);
        v[0] = cadd<T>(e0, o0); v[4] = csub<T>(e0, o0);
        v[1] = cadd<T>(e1, o1); v[5] = csub<T>(e1, o1);
        v[2] = cadd<T>(e2, o2); v[6] = csub<T>(e2, o2);
        v[3] = cadd<T>(e3, o3); v[7] = csub<T>(e3, o3);
    }
};
template <typename T, bool INV> struct RegDFT<T, 16, INV> {
    // 4 x 4: B[k1][j2] = DFT4 over n2 of v[k1 + 4 n2], times w16^(k1 j2), then DFT4 over k1.
    __device__ __forceinline__ static void run(C<T>* v) {
        dft4<T, INV>(v[0], v[4], v[8], v[12]);
        dft4<T, INV>(v[1], v[5], v[9], v[13]);
        dft4<T, INV>(v[2], v[6], v[10], v[14]);
        dft4<T, INV>(v[3], v[7], v[11], v[15]);
        v[5] = tw16<T, INV, 1>(v[5]);
        v[9] = tw16<T, INV, 2>(v[9]);
        v[13] = tw16<T, INV, 3>(v[13]);
        v[6] = tw16<T, INV, 2>(v[6]);
        v[10] = tw16<T, INV, 4>(v[10]);
        v[14] = tw16<T, INV, 6>(v[14]);
        v[7] = tw16<T, INV, 3>(v[7]);
        v[11] = tw16<T, INV, 6>(v[11]);
        v[15] = tw16<T, INV, 9>(v[15]);
        // after the first pass v[k1 + 4 j2] holds B[k1][j2]; y[j2 + 4 j1] = DFT4 over k1
        C<T> y[16];
#pragma unroll
        for (int j2 = 0; j2 < 4; ++j2) {
            C<T> b0 = v[0 + 4 * j2], b1 = v[1 + 4 * j2], b2 = v[2 + 4 * j2], b3 = v[3 + 4 * j2];
            dft4<T, INV>(b0, b1, b2, b3);
            y[j2] = b0;
            y[j2 + 4] = b1;
            y[j2 + 8] = b2;
            y[j2 + 12] = b3;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = y[i];
    }
};

template <typename T, bool INV> struct RegDFT<T, 32, INV> {
    // radix 2 over two 16-point transforms of the even and odd samples
    __device__ __forceinline__ static void run(C<T>* v) {
        C<T> e[16], o[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        RegDFT<T, 16, INV>::run(e);
        RegDFT<T, 16, INV>::run(o);
        twiddle_odd<0>(o);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            v[k] = cadd<T>(e[k], o[k]);
            v[k + 16] = csub<T>(e[k], o[k]);
        }
    }
    template <int K>
    __device__ __forceinline__ static void twiddle_odd(C<T>* o) {
        if constexpr (K < 16) {
            o[K] = tw32<T, INV, K>(o[K]);
            twiddle_odd<K + 1>(o);
        }
    }
};

constexpr double kH3 = 0.866025403784438646763723170753;  // sin(pi/3)

// a * exp(-+2 pi i k / 12) (forward sign -, inverse +), k a compile-time constant
template <typename T, bool INV, int K>
__device__ __forceinline__ C<T> tw12(C<T> a) {
    constexpr int k = K % 12;
    constexpr double ct[12] = {1.0, kH3, 0.5, 0.0, -0.5, -kH3, -1.0, -kH3, -0.5, 0.0, 0.5, kH3};
    constexpr double st[12] = {0.0, 0.5, kH3, 1.0, kH3, 0.5, 0.0, -0.5, -kH3, -1.0, -kH3, -0.5};
    if constexpr (k == 0) return a;
    else if constexpr (k == 3) return rot<T>(a, INV);
    else if constexpr (k == 6) return mk<T>(-a.x, -a.y);
    else if constexpr (k == 9) return rot<T>(a, !INV);
    else {
        const T c = (T)ct[k];
        const T sn = INV ? (T)st[k] : (T)-st[k];
        return mk<T>(a.x * c - a.y * sn, a.x * sn + a.y * c);
    }
}

template <typename T, bool INV> struct RegDFT<T, 3, INV> {
    __device__ __forceinline__ static void run(C<T>* v) {
        const C<T> t1 = cadd<T>(v[1], v[2]);
        const C<T> t2 = csub<T>(v[1], v[2]);
        const C<T> m = mk<T>(v[0].x - (T)0.5 * t1.x, v[0].y - (T)0.5 * t1.y);
        const C<T> n = rot<T>(mk<T>((T)kH3 * t2.x, (T)kH3 * t2.y), INV);
        v[0] = cadd<T>(v[0], t1);
        v[1] = cadd<T>(m, n);
        v[2] = csub<T>(m, n);
    }
};

// radix 2 over two N/2-point transforms of the even and odd samples, N = 6 or 12
template <typename T, bool INV, int N>
struct RegDFT2x {
    __device__ __forceinline__ static void run(C<T>* v) {
        constexpr int H = N / 2;
        C<T> e[H], o[H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        RegDFT<T, H, INV>::run(e);
        RegDFT<T, H, INV>::run(o);
        twiddle<1>(o);
#pragma unroll
        for (int k = 0; k < H; ++k) {
            v[k] = cadd<T>(e[k], o[k]);
            v[k + H] = csub<T>(e[k], o[k]);
        }
    }
    template <int K>
    __device__ __forceinline__ static void twiddle(C<T>* o) {
        if constexpr (K < N / 2) {
            o[K] = tw12<T, INV, K * (12 / N)>(o[K]);
            twiddle<K + 1>(o);
        }
    }
};
template <typename T, bool INV> struct RegDFT<T, 6, INV> {
    __device__ __forceinline__ static void run(C<T>* v) { RegDFT2x<T, INV, 6>::run(v); }
};
template <typename T, bool INV> struct RegDFT<T, 12, INV> {
    __device__ __forceinline__ static void run(C<T>* v) { RegDFT2x<T, INV, 12>::run(v); }
};

// a(lane ^ m) within a wavefront. Masks 1 and 2 stay inside a quad of lanes and use a DPP
// quad permutation (a VALU move without a trip through the LDS crossbar); other masks use
// ds_bpermute through __shfl_xor. m is uniform over the wavefront. The moves set bound_ctrl
// (a disabled source lane reads 0; every call site runs with the whole quad active, so the
// values are those of the plain move), which lets the compiler fold the move into the VOP2
// add or subtract that consumes it as a DPP operand: one VALU instruction instead of two.
__device__ __forceinline__ int dpp_quad_xor(int v, int m) {
    return (m == 1) ? __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true)   // quad_perm [1, 0, 3, 2]
                    : __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad_perm [2, 3, 0, 1]
}
__device__ __forceinline__ float xor_lane(float v, int m) {
    if (m == 1 || m == 2) return __int_as_float(dpp_quad_xor(__float_as_int(v), m));
    return __shfl_xor(v, m, kWave);
}
__device__ __forceinline__ double xor_lane(double v, int m) {
    if (m == 1 || m == 2) {
        const long long b = __double_as_longlong(v);
        const int lo = dpp_quad_xor((int)(b & 0xffffffffLL), m);
        const int hi = dpp_quad_xor((int)(b >> 32), m);
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
    return __shfl_xor(v, m, kWave);
}

template <typename T>
__device__ __forceinline__ C<T> shfl_xor_c(C<T> a, int m) {
    return mk<T>(xor_lane(a.x, m), xor_lane(a.y, m));
}

// Sum over the G = 2^lgG lanes of a line of each lane's P values. Reduce-scatter over the low
// log2 P lane bits (each step keeps half of the values: the upper half when the lane bit is set),
// then all-reduce over the remaining lane bits. Afterwards the lane holds P >> min(lgP, lgG)
// consecutive values starting at base(n2) = sum_s bit_s(n2) * (P >> (s + 1)).
template <typename T, int P, int S>
__device__ __forceinline__ void reduce_step(C<T>* v, int n2, int lgG) {
    if constexpr ((1 << S) < P) {
        if (S < lgG) {
            constexpr int half = (P >> S) >> 1;
            const bool hi = (n2 >> S) & 1;
#pragma unroll
            for (int i = 0; i < half; ++i) {
                const C<T> keep = hi ? v[i + half] : v[i];
                const C<T> send = hi ? v[i] : v[i + half];
                v[i] = cadd<T>(keep, shfl_xor_c<T>(send, 1 << S));
            }
            reduce_step<T, P, S + 1>(v, n2, lgG);
        }
    }
}

// The same reduce-scatter when the odd lane of every pair (n2, n2 ^ 1) holds its P values with
// the two halves exchanged (its input or its table row arranged for it): in the first step both
// lanes keep v[0, P/2) and send v[P/2, P), with no per-lane select; the remaining steps follow
// reduce_step. The result is the one reduce_step leaves.
template <typename T, int P>
__device__ __forceinline__ void reduce_scatter_x(C<T>* v, int n2, int lgG) {
    if constexpr (P >= 2) {
        if (lgG >= 1) {
            constexpr int half = P / 2;
#pragma unroll
            for (int i = 0; i < half; ++i) v[i] = cadd<T>(v[i], shfl_xor_c<T>(v[i + half], 1));
            reduce_step<T, P, 1>(v, n2, lgG);
        }
    }
}

// reduce_scatter_x for G >= P (every lane bit below log2 P is a line lane bit): all steps run,
// with no runtime step test, so the steps of independent calls can be interleaved.
template <typename T, int P, int S>
__device__ __forceinline__ void reduce_step_full(C<T>* v, int n2) {
    if constexpr ((1 << S) < P) {
        constexpr int half = (P >> S) >> 1;
        const bool hi = (n2 >> S) & 1;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const C<T> keep = hi ? v[i + half] : v[i];
            const C<T> send = hi ? v[i] : v[i + half];
            v[i] = cadd<T>(keep, shfl_xor_c<T>(send, 1 << S));
        }
        reduce_step_full<T, P, S + 1>(v, n2);
    }
}
template <typename T, int P>
__device__ __forceinline__ void reduce_scatter_full(C<T>* v, int n2) {
    if constexpr (P >= 2) {
        constexpr int half = P / 2;
#pragma unroll
        for (int i = 0; i < half; ++i) v[i] = cadd<T>(v[i], shfl_xor_c<T>(v[i + half], 1));
        reduce_step_full<T, P, 1>(v, n2);
    }
}

// a(lane ^ x) within each quad with x = 3 for quad lanes 0, 1 and x = 2 for lanes 2, 3: the quad
// permutation [3, 2, 0, 1] (step 1 of reduce_scatter_rot)
__device__ __forceinline__ int dpp_quad_3201(int v) { return __builtin_amdgcn_mov_dpp(v, 0x4B, 0xF, 0xF, true); }
__device__ __forceinline__ float quad_3201(float v) { return __int_as_float(dpp_quad_3201(__float_as_int(v))); }
__device__ __forceinline__ double quad_3201(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_quad_3201((int)(b & 0xffffffffLL));
    const int hi = dpp_quad_3201((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// a(source lane) with the source given as a byte address (4 x lane index) for ds_bpermute
__device__ __forceinline__ float bperm_lane(float v, int addr) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double bperm_lane(double v, int addr) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane spectral shifts of reduce_scatter_rot: s(n2) = bitrev(n2 mod P) over log2 P bits, and the part
// s'(n2) = s(n2) - (n2 mod 2) P / 2 that a table arranged for reduce_scatter_x (odd rows already
// turned by P / 2) still needs.
template <int P>
__device__ __forceinline__ int rot_shift(int n2) {
    constexpr int L = ilog2c(P);
    int s = 0;
#pragma unroll
    for (int b = 0; b < L; ++b) s |= ((n2 >> b) & 1) << (L - 1 - b);
    return s;
}
template <int P>
__device__ __forceinline__ int rot_shift_rest(int n2) { return rot_shift<P>(n2) - (n2 & 1) * (P / 2); }

// ds_bpermute byte addresses of steps 2 .. log2 P - 1 of reduce_scatter_rot for the lane at wave
// position lane (n2 = lane mod G, G >= P): partner n2 ^ x_j with x_1 = 2 or 3 (bit 1 of n2 set or
// not) and x_j = 2^j | (bit j of n2 ? 0 : x_(j-1)).
template <int P>
__device__ __forceinline__ void rot_addrs(int* addr, int lane, int n2) {
    constexpr int L = ilog2c(P);
    int x = ((n2 >> 1) & 1) ? 2 : 3;
#pragma unroll
    for (int j = 2; j < L; ++j) {
        x = (1 << j) | (((n2 >> j) & 1) ? 0 : x);
        addr[j - 2] = (lane ^ x) * 4;
    }
}

// Select-free reduce-scatter over the low log2 P lane bits for lanes whose P values come shifted by
// s(n2) = bitrev(n2 mod P), i.e. position p holds spectral index (p + s) mod P (the lane's input
// times exp(-2 pi i s n1 / P), its table row turned to match). Every step keeps positions [0, h)
// and adds positions [h, 2h) of one partner lane: the lane pairs of each step hold equal indices
// there and disjoint partial sums. Partners: step 0 n2 ^ 1, step 1 the quad permutation
// [3, 2, 0, 1], later steps ds_bpermute at addr (rot_addrs). Lane n2 ends with the sum of index
// bitrev(n2 mod P), the value reduce_step leaves it.
template <typename T, int P>
__device__ __forceinline__ void reduce_scatter_rot(C<T>* v, const int* addr) {
    constexpr int L = ilog2c(P);
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const int h = P >> (j + 1);
#pragma unroll
        for (int i = 0; i < h; ++i) {
            const C<T> b = v[i + h];
            C<T> r;
            if (j == 0) r = shfl_xor_c<T>(b, 1);
            else if (j == 1) r = mk<T>(quad_3201(b.x), quad_3201(b.y));
            else r = mk<T>(bperm_lane(b.x, addr[j - 2]), bperm_lane(b.y, addr[j - 2]));
            v[i] = cadd<T>(v[i], r);
        }
    }
}

// Every lane of a line ends with all P sums over the G = 2^lgG lanes (any P).
template <typename T, int P>
__device__ __forceinline__ void reduce_all(C<T>* v, int lgG) {
    for (int s = 0; s < lgG; ++s) {
#pragma unroll
        for (int i = 0; i < P; ++i) v[i] = cadd<T>(v[i], shfl_xor_c<T>(v[i], 1 << s));
    }
}

template <int P> constexpr bool kPow2 = (P & (P - 1)) == 0;

// The tile of TS = kThreads / g lines of M = g P points into LDS: exactly P elements per thread,
// loaded in chunks of CH whose loads are all issued before their stores, so that CH latencies
// overlap (CH trades the overlap against the registers the loads hold).
// Rows of the LDS tile are kTilePad elements longer than a line: with the line index fastest over
// the threads of a strided tile, rows M apart would put every line on the same LDS banks.
constexpr int kTilePad = 8;

template <typename T, int P, int CH>
__device__ __forceinline__ void load_tile(const C<T>* __restrict__ in, C<T>* B, const PassGeom& g, const Tile& tl,
                                          int64_t qi, int M, const FDiv& fdM, int ldb) {
    const int cnt = tl.nl * M;
    if (g.S != 1 && (kThreads % tl.nl) == 0) {
        // strided lines, nl | kThreads (every full tile): the thread's line l = tid mod nl is fixed
        // and its points advance by kThreads / nl, so the offsets are one base plus a stride
        const int tid = (int)threadIdx.x;
        const int l = tid % tl.nl;
        const int dn = kThreads / tl.nl;
        const int n0 = tid / tl.nl;
        const C<T>* src = in + ((qi * g.A + tl.a0) * M + n0) * g.S + tl.s0 + l;
        const int64_t stride = (int64_t)dn * g.S;
        C<T>* dst = B + l * ldb + n0;
#pragma unroll
        for (int k0 = 0; k0 < P; k0 += CH) {
            C<T> v[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k)
                if (k0 + k < P && n0 + (k0 + k) * dn < M) v[k] = src[(k0 + k) * stride];
#pragma unroll
            for (int k = 0; k < CH; ++k)
                if (k0 + k < P && n0 + (k0 + k) * dn < M) dst[(k0 + k) * dn] = v[k];
        }
        return;
    }
#pragma unroll
    for (int k0 = 0; k0 < P; k0 += CH) {
        C<T> v[CH];
        int dst[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int e = (int)threadIdx.x + (k0 + k) * kThreads;
            dst[k] = -1;
            if (k0 + k < P && e < cnt) {
                int ll, n;
                const int64_t off = tile_elem(g, tl, qi, M, fdM, e, ll, n);
                v[k] = in[off];
                dst[k] = ll * ldb + n;
            }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k)
            if (dst[k] >= 0) B[dst[k]] = v[k];
    }
}

// Twiddles of lane_idft_x: stage s uses wst[s] = w (lower lane) or -conj(w) (upper lane), with
// w = exp(2 pi i (n2 mod 2^s) / 2^(s+1)). Returns the lane's final rescale (see lane_idft_x).
// With INV = false the same for the forward transform, w = exp(-2 pi i (n2 mod 2^s) / 2^(s+1)).
template <typename T, int LP, bool INV = true>
__device__ __forceinline__ C<T> lane_twiddles_x(C<T>* wst, int n2, const C<T>* tw, int M) {
    C<T> c = mk<T>(1, 0);
#pragma unroll
    for (int s = 0; s < LP; ++s) {
        // exp(-2 pi i (n2 mod 2^s) / 2^(s+1)); exactly 1 at stage 0, whose factor is then the real
        // sign +-1 (lane_bfly relies on it)
        const C<T> t = (s == 0) ? mk<T>(1, 0) : tw[(n2 & ((1 << s) - 1)) * (M >> (s + 1))];
        const C<T> w = INV ? mk<T>(t.x, -t.y) : t;
        if ((n2 >> s) & 1) {
            wst[s] = mk<T>(-w.x, w.y);  // -conj(w)
            c = cmul<T>(c, wst[s]);
        } else {
            wst[s] = w;
        }
    }
    return mk<T>(c.x, -c.y);
}

// Inverse P-point DFT across the first P lanes of a line (power-of-two P <= G). On entry lane n2
// holds W[bitrev(n2 mod P)], the order the reduce-scatter leaves; radix-2 decimation in time on
// bit-reversed input yields natural order, so on exit lane n2 holds sum_r W[r] exp(2 pi i r u / P)
// for u = n2 mod P. No per-lane selects: both lanes of a butterfly form own + k * partner: the
// lower lane with k = w gives a_lo + w a_up exactly; the upper lane with k = -conj(w) gives
// a_up - conj(w) a_lo = -conj(w) (a_lo - w a_up), its true output times the unit factor
// -conj(w). The factors of the stages where the lane is the upper one multiply up to c; the
// result is multiplied by conj(c) = 1 / c at the end (fin from lane_twiddles_x).
// One butterfly stage of these lane transforms: own + w * partner, the partner d lanes away. At
// stage 0 (s = 0) lane_twiddles_x gives the real factor w = +-1, which takes two FMAs, not four.
template <typename T>
__device__ __forceinline__ C<T> lane_bfly(C<T> a, C<T> w, int d, int s) {
    const C<T> b = shfl_xor_c<T>(a, d);
    if (s == 0) return mk<T>(a.x + w.x * b.x, a.y + w.x * b.y);
    return cfma<T>(a, w, b);
}

template <typename T, int LP>
__device__ __forceinline__ C<T> lane_idft_x(C<T> a, const C<T>* wst, C<T> fin) {
#pragma unroll
    for (int s = 0; s < LP; ++s) a = lane_bfly<T>(a, wst[s], 1 << s, s);
    return cmul<T>(a, fin);
}
// The same without the final rescale: the lane's output times c, for callers that apply conj(c)
// (fin) once to a sum of many such outputs.
template <typename T, int LP>
__device__ __forceinline__ C<T> lane_idft_nofin(C<T> a, const C<T>* wst) {
#pragma unroll
    for (int s = 0; s < LP; ++s) a = lane_bfly<T>(a, wst[s], 1 << s, s);
    return a;
}

// Terms whose chirp-folded table rows (M values each) are staged in LDS at a time.
constexpr int kErStage = 4;

// Copies elements e0 <= e < cnt of a block of rows of P values into LDS with a row stride of P + 1, the
// loads of every chunk of 8 per thread issued before their stores: element e goes to
// (e / P)(P + 1) + e mod P. A lane then reads its own row with immediate
// offsets, and with the odd stride the g lanes of a line hit distinct banks.
template <typename T, int P>
__device__ __forceinline__ void copy_rows_to_lds(C<T>* dst, const C<T>* __restrict__ src, int e0, int cnt) {
    for (int b = e0; b < cnt; b += 8 * kThreads) {
        const int t = b + (int)threadIdx.x;
        C<T> v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (t + k * kThreads < cnt) ? src[t + k * kThreads] : mk<T>(0, 0);
        if constexpr (kThreads % P == 0) {
            // element t + k kThreads sits in row t / P + k kThreads / P, column t mod P
            C<T>* d = dst + (t / P) * (P + 1) + t % P;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (t + k * kThreads < cnt) d[k * (kThreads / P) * (P + 1)] = v[k];
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int e = t + k * kThreads;
                if (e < cnt) dst[(e / P) * (P + 1) + e % P] = v[k];
            }
        }
    }
}

// FP32 with P <= 8: at most 128 registers (four waves per SIMD)
template <typename T, int P, bool LANEINV>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && P <= 8) ? 4 : 1)))
void k_ER(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax, PassGeom g, int lgG,
          const C<T>* __restrict__ TA, const C<T>* __restrict__ HT) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int LP = (P >= 32) ? 5 : (P >= 16) ? 4 : (P >= 8) ? 3 : (P >= 4) ? 2 : (P >= 2) ? 1 : 0;
    const int M = ax.M;
    const int ldb = M + kTilePad;
    C<T>* B = (C<T>*)smem;          // tile of strided lines: TS rows of ldb (M points each)
    C<T>* TAs = B + (kThreads >> lgG) * ldb;  // TA_q[g i] of the workgroup's qc terms, [q - qlo][i]
    C<T>* Hs = TAs + g.qc * P;       // table rows of kErStage terms, [q - q0][n2][P + 1]
    const int G = 1 << lgG;
    const int l = (int)threadIdx.x >> lgG;
    const int n2 = (int)threadIdx.x & (G - 1);
    const int qc = g.qc;
    const int nqc = (g.qn + qc - 1) / qc;
    // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs (id mod 8); XCD x
    // takes the contiguous tile range [x T8, (x + 1) T8) with all nqc workgroups of each tile, so
    // a tile is read into one L2, and so are the neighbouring tiles that share its cache lines
    const int64_t ntl = g.Qin * g.ntiles;
    const int64_t T8 = (ntl + 7) / 8;
    const int64_t total = T8 * 8 * nqc;
    const int lk = (lgG < LP) ? lgG : LP;     // reduce-scatter steps
    const int cnt = P >> lk;                  // values a lane holds afterwards
    int base = 0;
    for (int s = 0; s < lk; ++s) base += ((n2 >> s) & 1) * ((P >> s) >> 1);
    const bool writer = (n2 >> lk) == 0 || lgG <= LP;
    // With the lane transform (power-of-two P <= G) and P <= 8 the lane's input is modulated by
    // exp(-2 pi i s n1 / P), s = bitrev(n2 mod P), once per tile below, and its table row (HT,
    // [q][n2][r]) is turned by s to match, so the sum over the lanes is reduce_scatter_rot. For
    // P >= 16 (where the modulation of P values per tile costs more than the selects it saves over
    // the few terms of a tile) HT is the table arranged for reduce_scatter_x, and the odd lane's
    // input is modulated by (-1)^n1, which exchanges the halves of its spectrum.
    constexpr bool ROT = LANEINV && P <= 8;
    int raddr[LP > 2 ? LP - 2 : 1];
    if constexpr (ROT) rot_addrs<P>(raddr, (int)threadIdx.x & (kWave - 1), n2);
    const int rsh = ROT ? rot_shift<P>(n2) : 0;
    const bool odd_flip = LANEINV && !ROT && (n2 & 1) && lgG >= 1;
    // P = 6 with g = 8: the odd lane's input times (-1)^i moves its spectrum by 3, and it reads its
    // table row rotated by 3 to match (see the sum over the lanes below)
    const bool six = (P == 6) && lgG == 3;
    const bool flip6 = six && (n2 & 1);
    int hrot[P];
#pragma unroll
    for (int r = 0; r < P; ++r) hrot[r] = flip6 ? (r + 3) % P : r;
    // the inverse 6-point transform of the summed values, output u = n2 (n2 < 6): with W[3 b0 + j] in the
    // lane and W[3 (1 - b0) + j] in its partner, E[u] = sum_j exp(2 pi i j u / 6) (W[j] + (-1)^u W[j + 3])
    T s_own = 1, s_par = 1;
    C<T> c6[2];
    if constexpr (P == 6) {
        const T sg = (n2 & 1) ? (T)-1 : (T)1;  // (-1)^u, u = n2
        s_own = (n2 & 1) ? sg : (T)1;
        s_par = (n2 & 1) ? (T)1 : sg;
        const C<T>* twp = (const C<T>*)ax.tw;
#pragma unroll
        for (int j = 1; j < 3; ++j) {
            const C<T> c = twp[((j * n2) % 6) * (M / 6)];
            c6[j - 1] = mk<T>(c.x, -c.y);
        }
    }
    C<T> wst[LP > 0 ? LP : 1];
    const C<T> fin = lane_twiddles_x<T, LP>(wst, n2, (const C<T>*)ax.tw, M);
    for (int64_t bid = blockIdx.x; bid < total; bid += gridDim.x) {
        // every id and index here is below 2^31 (checked on the host): 32-bit division
        const unsigned rr = (unsigned)bid >> 3;
        const int ci = (int)(rr % (unsigned)nqc);
        const int64_t tile = ((int64_t)bid & 7) * T8 + (int64_t)(rr / (unsigned)nqc);
        if (tile >= ntl) continue;  // uniform over the workgroup
        const int64_t qi = (int64_t)((unsigned)tile / (unsigned)g.ntiles);
        const int64_t tt = tile - qi * g.ntiles;
        const Tile tl = decode_tile(g, tt);
        const bool live = l < tl.nl;
        const int qlo = g.qb + ci * qc;
        const int qhi = min(qlo + qc, g.qb + g.qn);
        // the chunk's premultiply values go through LDS: issued first, stored after the tile
        const int nta = (qhi - qlo) * P;
        const int ti = (int)threadIdx.x;
        C<T> tav = mk<T>(0, 0);
        if (ti < nta) tav = TA[(int64_t)(qlo + ti / P) * M + ((ti % P) << lgG)];
        // the first round's table rows: their loads go out with the tile's
        const int nq0 = min(kErStage, qhi - qlo);
        const int hcnt = nq0 * M;
        const C<T>* hsrc = HT + (int64_t)qlo * M;
        C<T> hv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = ti + k * kThreads;
            hv[k] = (e < hcnt) ? hsrc[e] : mk<T>(0, 0);
        }
        C<T> x[P];
        if (g.S == 1) {
            // contiguous lines: lane n2 reads x[g i + n2] directly (G consecutive lanes per i)
            const C<T>* src = in + (qi * g.A + tl.a0 + (live ? l : 0)) * M + n2;
#pragma unroll
            for (int i = 0; i < P; ++i) x[i] = live ? src[i << lgG] : mk<T>(0, 0);
        } else {
            const FDiv fdM = tile_div(g, tl, M);
            load_tile<T, P, (sizeof(T) == 4 ? P : 1)>(in, B, g, tl, qi, M, fdM, ldb);
        }
        if (ti < nta) TAs[ti] = tav;
        for (int e = ti + kThreads; e < nta; e += kThreads) TAs[e] = TA[(int64_t)(qlo + e / P) * M + ((e % P) << lgG)];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = ti + k * kThreads;
            if (e < hcnt) {
                if constexpr (kThreads % P == 0) Hs[(ti / P + k * (kThreads / P)) * (P + 1) + ti % P] = hv[k];
                else Hs[(e / P) * (P + 1) + e % P] = hv[k];
            }
        }
        if (hcnt > 8 * kThreads) copy_rows_to_lds<T, P>(Hs, hsrc, 8 * kThreads, hcnt);
        __syncthreads();
        if (g.S != 1) {
#pragma unroll
            for (int i = 0; i < P; ++i) x[i] = live ? B[l * ldb + (i << lgG) + n2] : mk<T>(0, 0);
        }
        if (odd_flip || flip6) {
#pragma unroll
            for (int i = 1; i < P; i += 2) x[i] = mk<T>(-x[i].x, -x[i].y);
        }
        if constexpr (ROT) {
            // x[i] exp(-2 pi i s i / P): position p of the lane's spectrum holds index p + s
            const C<T>* twp = (const C<T>*)ax.tw;
#pragma unroll
            for (int i = 1; i < P; ++i) x[i] = cmul<T>(x[i], twp[((rsh * i) & (P - 1)) << lgG]);
        }
        for (int q = qlo; q < qhi; ++q) {
            if (q > qlo && (q - qlo) % kErStage == 0) {
                // next round of table rows (the previous round's reads are done first)
                __syncthreads();
                copy_rows_to_lds<T, P>(Hs, HT + (int64_t)q * M, 0, min(kErStage, qhi - q) * M);
                __syncthreads();
            }
            if constexpr (LANEINV) {
                // two terms at once (q - qlo even, so both rows are in the staged round): their
                // lane reductions are independent chains of shuffles the scheduler interleaves
                if (q + 1 < qhi) {
                    const C<T>* ta0 = TAs + (q - qlo) * P;
                    const C<T>* h0 = Hs + (((q - qlo) % kErStage) * G + n2) * (P + 1);
                    const C<T>* h1 = h0 + G * (P + 1);
                    C<T> va[P], vb[P];
#pragma unroll
                    for (int i = 0; i < P; ++i) {
                        va[i] = cmul<T>(x[i], ta0[i]);
                        vb[i] = cmul<T>(x[i], ta0[P + i]);
                    }
                    RegDFT<T, P, false>::run(va);
                    RegDFT<T, P, false>::run(vb);
#pragma unroll
                    for (int r = 0; r < P; ++r) {
                        va[r] = cmul<T>(va[r], h0[r]);
                        vb[r] = cmul<T>(vb[r], h1[r]);
                    }
                    if constexpr (ROT) {
                        reduce_scatter_rot<T, P>(va, raddr);
                        reduce_scatter_rot<T, P>(vb, raddr);
                    } else {
                        reduce_scatter_full<T, P>(va, n2);
                        reduce_scatter_full<T, P>(vb, n2);
                    }
                    C<T> sa = va[0], sb = vb[0];
                    for (int s = LP; s < lgG; ++s) {
                        sa = cadd<T>(sa, shfl_xor_c<T>(sa, 1 << s));
                        sb = cadd<T>(sb, shfl_xor_c<T>(sb, 1 << s));
                    }
                    sa = lane_idft_x<T, LP>(sa, wst, fin);
                    sb = lane_idft_x<T, LP>(sb, wst, fin);
                    if (live && n2 < P) {
                        const int64_t qo = qi * g.qn + (q - g.qb);
                        const int64_t off = (g.S == 1) ? ((qo * g.A + tl.a0 + l) * P + n2)
                                                       : (((qo * g.A + tl.a0) * P + n2) * g.S + tl.s0 + l);
                        const int64_t dq = g.A * P * g.S;  // the next term's slice
                        out[off] = sa;
                        out[off + dq] = sb;
                    }
                    ++q;
                    continue;
                }
            }
            const C<T>* ta = TAs + (q - qlo) * P;
            const C<T>* h = Hs + (((q - qlo) % kErStage) * G + n2) * (P + 1);
            C<T> v[P];
#pragma unroll
            for (int i = 0; i < P; ++i) v[i] = cmul<T>(x[i], ta[i]);
            RegDFT<T, P, false>::run(v);
#pragma unroll
            for (int r = 0; r < P; ++r) v[r] = cmul<T>(v[r], h[hrot[r]]);
            if constexpr (P == 6) {
                if (six) {
                    // sum over the 8 lanes: one select-free step (values 0..2 kept), the other two
                    // lane bits in full; lane n2 < 6 then forms E[n2] from its and its partner's values
#pragma unroll
                    for (int j = 0; j < 3; ++j) v[j] = cadd<T>(v[j], shfl_xor_c<T>(v[j + 3], 1));
#pragma unroll
                    for (int s2 = 1; s2 < 3; ++s2) {
#pragma unroll
                        for (int j = 0; j < 3; ++j) v[j] = cadd<T>(v[j], shfl_xor_c<T>(v[j], 1 << s2));
                    }
                    C<T> aj[3];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const C<T> pj = shfl_xor_c<T>(v[j], 1);
                        aj[j] = mk<T>(s_own * v[j].x + s_par * pj.x, s_own * v[j].y + s_par * pj.y);
                    }
                    const C<T> e = cfma<T>(cfma<T>(aj[0], c6[0], aj[1]), c6[1], aj[2]);
                    if (live && n2 < P) {
                        const int64_t qo = qi * g.qn + (q - g.qb);
                        const int64_t off = (g.S == 1) ? ((qo * g.A + tl.a0 + l) * P + n2)
                                                       : (((qo * g.A + tl.a0) * P + n2) * g.S + tl.s0 + l);
                        out[off] = e;
                    }
                    continue;
                }
            }
            if constexpr (LANEINV) {
                // sum over the lanes first, then one inverse transform across the P lanes
                if constexpr (ROT) reduce_scatter_rot<T, P>(v, raddr);
                else reduce_scatter_full<T, P>(v, n2);
                C<T> s0 = v[0];
                for (int s = LP; s < lgG; ++s) s0 = cadd<T>(s0, shfl_xor_c<T>(s0, 1 << s));
                s0 = lane_idft_x<T, LP>(s0, wst, fin);
                if (live && n2 < P) {
                    const int64_t qo = qi * g.qn + (q - g.qb);
                    const int64_t off = (g.S == 1) ? ((qo * g.A + tl.a0 + l) * P + n2)
                                                   : (((qo * g.A + tl.a0) * P + n2) * g.S + tl.s0 + l);
                    out[off] = s0;
                }
            } else {
                RegDFT<T, P, true>::run(v);
                if constexpr (!kPow2<P> && P < 8) {
                    if (lgG == 3) {
                        // g = 8 (P = 3): the values padded to 8 and summed by the select form of the
                        // reduce-scatter; lane n2 ends with value bitrev3(n2) and writes it
                        C<T> w8[8];
#pragma unroll
                        for (int k = 0; k < 8; ++k) w8[k] = k < P ? v[k] : mk<T>(0, 0);
                        reduce_step<T, 8, 0>(w8, n2, 3);
                        const int uu = ((n2 & 1) << 2) | (n2 & 2) | ((n2 >> 2) & 1);
                        if (live && uu < P) {
                            const int64_t qo = qi * g.qn + (q - g.qb);
                            const int64_t off = (g.S == 1) ? ((qo * g.A + tl.a0 + l) * P + uu)
                                                           : (((qo * g.A + tl.a0) * P + uu) * g.S + tl.s0 + l);
                            out[off] = w8[0];
                        }
                        continue;
                    }
                }
                if constexpr (!kPow2<P>) {
                    // all-reduce; lane n2 writes the values u = n2 mod G
                    reduce_all<T, P>(v, lgG);
                    if (live) {
                        const int64_t qo = qi * g.qn + (q - g.qb);
#pragma unroll
                        for (int u = 0; u < P; ++u) {
                            if ((u & (G - 1)) == n2) {
                                const int64_t off = (g.S == 1) ? ((qo * g.A + tl.a0 + l) * P + u)
                                                               : (((qo * g.A + tl.a0) * P + u) * g.S + tl.s0 + l);
                                out[off] = v[u];
                            }
                        }
                    }
                } else {
                    // G < P: the odd lane's table row carries (-1)^r, which exchanges the halves
                    // of its inverse output
                    reduce_scatter_x<T, P>(v, n2, lgG);
                    C<T> s0 = v[0];
                    for (int s = LP; s < lgG; ++s) s0 = cadd<T>(s0, shfl_xor_c<T>(s0, 1 << s));
                    v[0] = s0;
                    if (live && writer) {
                        const int64_t qo = qi * g.qn + (q - g.qb);
#pragma unroll
                        for (int i = 0; i < P; ++i) {
                            if (i < cnt) {
                                const int u = base + i;
                                const int64_t off = (g.S == 1) ? ((qo * g.A + tl.a0 + l) * P + u)
                                                               : (((qo * g.A + tl.a0) * P + u) * g.S + tl.s0 + l);
                                out[off] = v[i];
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();  // the next tile overwrites the buffers the q loop reads
    }
}

// Register E for longer pruned lengths (g = 8; P = 16, 32, 64 and 48: axes of 128 to 512 points),
// contiguous lines. With V = 8 values per lane (V = 6 for P = 48) and NL = P / V, a line takes
// L = 8 NL lanes; lane lam = lo + NL n2 (lo < NL, n2 < 8) keeps the V inputs x[8 n1 + n2] with
// n1 = NL i + lo (i < V) in registers for every term. With k = k1 + V k2 (k1 < V, k2 < NL) the
// P-point transform of the n2 subsequence splits as
//   V[n2][k1 + V k2] = sum_lo w_NL^(lo k2) w_P^(lo k1) sum_i w_V^(i k1) y[8 (NL i + lo) + n2],
// a V-point transform in the lane, a twiddle, and an NL-point transform across the lo lanes
// (decimation in frequency: natural input, lane lo ends with k2 = bitrev(lo)). The table multiply
// and the sum over n2 follow, and the inverse P-point transform splits the same way with
// u = u1 + NL u2:
//   E[u1 + NL u2] = sum_k1 w_V^(-k1 u2) w_P^(-k1 u1) sum_k2 w_NL^(-k2 u1) W[k1 + V k2].
// V = 8: the sum over n2 is a reduce-scatter over the n2 lane bits (lane (lo, n2) keeps
// k1 = bitrev3(n2)), and both inverse stages run across lanes on bit-reversed input (each lane
// forms own + c partner with one scale at the end, as in lane_idft_x), so lane lam ends with
// E[lam] and the writes of a line are contiguous. V = 6: one reduce-scatter step leaves each lane
// three values of k1, the other two n2 bits are summed in full, the inverse over k2 runs across
// lanes for the three values, and each lane n2 < 6 forms its output u2 = n2 as a 6-term sum over
// its own values and its partner's. The odd n2 lanes take their input times (-1)^i, which moves
// their k1 by V / 2, so the first reduce step needs no selects; the table rows are staged in LDS in
// the order each lane consumes them (row of lane lam: its V values, padded by one).
template <int P> constexpr int erw_values() { return (P % 3 == 0) ? 6 : 8; }

template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_ERW(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g, const C<T>* __restrict__ TA, const C<T>* __restrict__ HT) {
    constexpr int G = 8;
    constexpr int V = erw_values<P>();
    constexpr int NL = P / V;
    constexpr int LNL = ilog2c(NL);
    constexpr int L = NL * G;          // lanes per line
    constexpr int TL = kThreads / L;   // lines per tile
    constexpr int HR = V + 1;          // LDS row of one lane's table values
    constexpr int HV = V / 2;
    static_assert(NL >= 2 && (NL & (NL - 1)) == 0 && L <= kWave, "P = 16, 32, 48 or 64");
    extern __shared__ __align__(16) unsigned char smem[];
    C<T>* TAs = (C<T>*)smem;         // [q - qlo][n1]: TA_q[8 n1] of the workgroup's terms
    C<T>* Hs = TAs + g.qc * P;       // [q - q0][lam][HR]: table values of kErStage terms
    const int M = ax.M;
    const int lam = (int)threadIdx.x & (L - 1);
    const int l = (int)threadIdx.x / L;
    const int lo = lam & (NL - 1);
    const int n2 = lam >> LNL;
    const int b0 = n2 & 1;
    const C<T>* tw = (const C<T>*)ax.tw;  // exp(-2 pi i k / M); w_P^a = tw[8 a mod M]
    C<T> t1[V];
#pragma unroll
    for (int j = 0; j < V; ++j) t1[j] = tw[(lo * ((j + HV * b0) % V) * G) % M];
    // decimation-in-frequency stages across lo (top bit first): lower lane a + b, upper (a - b) w
    T dsg[LNL];
    C<T> dmul[LNL];
#pragma unroll
    for (int s = 0; s < LNL; ++s) {
        const bool up = (lo >> s) & 1;
        dsg[s] = up ? (T)-1 : (T)1;
        dmul[s] = up ? tw[(lo & ((1 << s) - 1)) * (M >> (s + 1))] : mk<T>(1, 0);
    }
    C<T> w1[LNL];
    const C<T> fin1 = lane_twiddles_x<T, LNL, true>(w1, lo, tw, M);
    // after the inverse over k2: undo its scale and apply w_P^(-k1 u1) (u1 = lo)
    constexpr int NM = (V == 8) ? 1 : HV;
    C<T> m2[NM];
    C<T> w3[3], fin3 = mk<T>(1, 0);
    C<T> cown[HV], cpar[HV];  // V = 6: w_6^(-k1 n2) for the lane's own k1 and its partner's
    if constexpr (V == 8) {
        fin3 = lane_twiddles_x<T, 3, true>(w3, n2, tw, M);
        const int k1 = ((n2 & 1) << 2) | (n2 & 2) | ((n2 >> 2) & 1);
        const C<T> e = tw[(k1 * lo * G) % M];
        m2[0] = cmul<T>(fin1, mk<T>(e.x, -e.y));
    } else {
#pragma unroll
        for (int j = 0; j < HV; ++j) {
            const C<T> e = tw[((HV * b0 + j) * lo * G) % M];
            m2[j] = cmul<T>(fin1, mk<T>(e.x, -e.y));
            const C<T> co = tw[(((HV * b0 + j) * n2) % 6) * (M / 6)];
            const C<T> cp = tw[(((HV * (1 - b0) + j) * n2) % 6) * (M / 6)];
            cown[j] = mk<T>(co.x, -co.y);
            cpar[j] = mk<T>(cp.x, -cp.y);
        }
    }
    const int qc = g.qc;
    const int nqc = (g.qn + qc - 1) / qc;
    // XCD-aware order as in k_ER: the nqc workgroups of a tile run on one XCD
    const int64_t ntl = g.Qin * g.ntiles;
    const int64_t T8 = (ntl + 7) / 8;
    const int64_t total = T8 * 8 * nqc;
    for (int64_t bid = blockIdx.x; bid < total; bid += gridDim.x) {
        const unsigned rr = (unsigned)bid >> 3;
        const int ci = (int)(rr % (unsigned)nqc);
        const int64_t tile = ((int64_t)bid & 7) * T8 + (int64_t)(rr / (unsigned)nqc);
        if (tile >= ntl) continue;  // uniform over the workgroup
        const int64_t qi = (int64_t)((unsigned)tile / (unsigned)g.ntiles);
        const int64_t a0 = (tile - qi * g.ntiles) * TL;
        const bool live = a0 + l < g.A;
        const int qlo = g.qb + ci * qc;
        const int qhi = min(qlo + qc, g.qb + g.qn);
        const int ti = (int)threadIdx.x;
        const int nta = (qhi - qlo) * P;
        for (int e = ti; e < nta; e += kThreads) TAs[e] = TA[(int64_t)(qlo + e / P) * M + (e % P) * G];
        C<T> x[V];
        {
            const C<T>* src = in + (qi * g.A + a0 + (live ? l : 0)) * M + G * lo + n2;
#pragma unroll
            for (int i = 0; i < V; ++i) x[i] = live ? src[i * G * NL] : mk<T>(0, 0);
        }
        if (b0) {
#pragma unroll
            for (int i = 1; i < V; i += 2) x[i] = mk<T>(-x[i].x, -x[i].y);
        }
        for (int q = qlo; q < qhi; ++q) {
            const int ql = (q - qlo) % kErStage;
            if (ql == 0) {
                // the next round of table rows, rearranged for the lanes: HT[q][r][n2] with
                // r = k1 + V k2 goes to lane bitrev(k2) + NL n2, slot k1 + V/2 (mod V) for odd n2
                __syncthreads();
                const int cnt = min(kErStage, qhi - q) * M;
                const C<T>* src = HT + (int64_t)q * M;
                for (int e = ti; e < cnt; e += kThreads) {
                    const int qq = e / M, rem = e - qq * M;
                    const int r = rem >> 3, m2i = rem & 7;
                    const int kk2 = r / V, kk1 = r - kk2 * V;
                    int br = 0;
#pragma unroll
                    for (int b = 0; b < LNL; ++b) br |= ((kk2 >> b) & 1) << (LNL - 1 - b);
                    Hs[(qq * L + br + NL * m2i) * HR + (kk1 + HV * (m2i & 1)) % V] = src[e];
                }
                __syncthreads();
            }
            const C<T>* ta = TAs + (q - qlo) * P + lo;
            C<T> v[V];
#pragma unroll
            for (int i = 0; i < V; ++i) v[i] = cmul<T>(x[i], ta[i * NL]);
            RegDFT<T, V, false>::run(v);
#pragma unroll
            for (int j = 0; j < V; ++j) v[j] = cmul<T>(v[j], t1[j]);
#pragma unroll
            for (int s = LNL - 1; s >= 0; --s) {
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    const C<T> pj = shfl_xor_c<T>(v[j], 1 << s);
                    v[j] = cmul<T>(mk<T>(pj.x + dsg[s] * v[j].x, pj.y + dsg[s] * v[j].y), dmul[s]);
                }
            }
            const C<T>* h = Hs + (ql * L + lam) * HR;
#pragma unroll
            for (int j = 0; j < V; ++j) v[j] = cmul<T>(v[j], h[j]);
            // sum over n2: both lanes of the first pair keep slots 0 .. V/2 - 1
#pragma unroll
            for (int j = 0; j < HV; ++j) v[j] = cadd<T>(v[j], shfl_xor_c<T>(v[j + HV], NL));
            C<T> a;
            if constexpr (V == 8) {
                {
                    const bool hi = (n2 >> 1) & 1;
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const C<T> keep = hi ? v[j + 2] : v[j];
                        const C<T> send = hi ? v[j] : v[j + 2];
                        v[j] = cadd<T>(keep, shfl_xor_c<T>(send, 2 * NL));
                    }
                }
                {
                    const bool hi = (n2 >> 2) & 1;
                    const C<T> keep = hi ? v[1] : v[0];
                    const C<T> send = hi ? v[0] : v[1];
                    a = cadd<T>(keep, shfl_xor_c<T>(send, 4 * NL));
                }
                // inverse: over k2 (lo lanes), twiddle, over k1 (n2 lanes)
#pragma unroll
                for (int s = 0; s < LNL; ++s) a = lane_bfly<T>(a, w1[s], 1 << s, s);
                a = cmul<T>(a, m2[0]);
#pragma unroll
                for (int s = 0; s < 3; ++s) a = lane_bfly<T>(a, w3[s], NL << s, s);
                a = cmul<T>(a, fin3);
            } else {
                // the other two n2 bits summed in full: the lane holds k1 = V/2 b0 + j, j < V/2
#pragma unroll
                for (int s = 1; s < 3; ++s) {
#pragma unroll
                    for (int j = 0; j < HV; ++j) v[j] = cadd<T>(v[j], shfl_xor_c<T>(v[j], NL << s));
                }
#pragma unroll
                for (int j = 0; j < HV; ++j) {
#pragma unroll
                    for (int s = 0; s < LNL; ++s) v[j] = lane_bfly<T>(v[j], w1[s], 1 << s, s);
                    v[j] = cmul<T>(v[j], m2[j]);
                }
                a = mk<T>(0, 0);
#pragma unroll
                for (int j = 0; j < HV; ++j) {
                    a = cfma<T>(a, cown[j], v[j]);
                    a = cfma<T>(a, cpar[j], shfl_xor_c<T>(v[j], NL));
                }
            }
            if (live && (V == 8 || n2 < V)) {
                const int64_t qo = qi * g.qn + (q - g.qb);
                out[(qo * g.A + a0 + l) * P + lo + NL * n2] = a;
            }
        }
        __syncthreads();  // the next tile overwrites the buffers the q loop reads
    }
}

// The same lane layout for g = 2, 4, 8 (G lanes of n2) and P = 16, 32, 64 with V = 8 values per
// lane, for E and for EA, contiguous or strided lines (strided tiles go through LDS). A line takes
// L = G NL lanes (NL = P / 8). After the table multiply the sum over the G lanes of n2 is a
// reduce-scatter that leaves VG = 8 / G values per lane, k1 = VG bitrev(n2) + t (t < VG), and the
// inverse splits once more: with k1 = t + VG j and u2 = u2a + G u2b,
//   sum_k1 w_8^(-k1 u2) Z[k1] = sum_t w_VG^(-t u2b) w_8^(-t u2a) sum_j w_G^(-j u2a) Z[t + VG j],
// the sum over j across the n2 lanes (bit-reversed input, lane n2 ends with u2a = n2), a twiddle,
// and a VG-point transform in the lane, so lane lam holds E[lam + L u2b] for u2b < VG. The EA form
// adds Tf_q[n0] E_q[u] into the residue (q - qb) mod g of the output group n0 of each held u (the
// term loop unrolled by g, so every residue is a fixed register) and ends each tile with the
// g-point inverse over the residues (the structured accumulate).
template <typename T, int P, int LG, bool EAF>
__global__ __launch_bounds__(kThreads) void k_ERG(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g, int accumulate, T* __restrict__ rho,
                                                  const C<T>* __restrict__ TA, const C<T>* __restrict__ HT) {
    constexpr int G = 1 << LG;
    constexpr int V = 8;
    constexpr int NL = P / V;
    constexpr int LNL = ilog2c(NL);
    constexpr int L = NL * G;          // lanes per line
    constexpr int TL = kThreads / L;   // lines per tile
    constexpr int HR = V + 1;
    constexpr int VG = V >> LG;        // values per lane after the sum over n2
    constexpr int M = G * P;
    static_assert(NL >= 2 && (NL & (NL - 1)) == 0 && L <= kWave && LG >= 1 && LG <= 3, "P = 16, 32, 64; g = 2, 4, 8");
    extern __shared__ __align__(16) unsigned char smem[];
    const int qcap = EAF ? g.qn : g.qc;
    C<T>* TAs = (C<T>*)smem;                    // [q - qlo][n1] = TA_q[g n1]
    C<T>* Tfs = TAs + qcap * P;                 // EA: [q - qb][n0] = Tf_q[n0]
    C<T>* Hs = Tfs + (EAF ? g.qn * P : 0);      // [q - q0][lam][HR]: table values of kErStage terms
    C<T>* B = Hs + kErStage * L * HR;           // strided tile: TL rows of M + kTilePad
    const int ldb = M + kTilePad;
    const int lam = (int)threadIdx.x & (L - 1);
    const int l = (int)threadIdx.x / L;
    const int lo = lam & (NL - 1);
    const int n2 = lam >> LNL;
    const int f = (n2 & 1) ? 4 : 0;
    const int ti = (int)threadIdx.x;
    const C<T>* tw = (const C<T>*)ax.tw;  // exp(-2 pi i k / M); w_P^a = tw[G a mod M]
    C<T> t1[V];
#pragma unroll
    for (int j = 0; j < V; ++j) t1[j] = tw[(lo * (j ^ f) * G) % M];
    T dsg[LNL];
    C<T> dmul[LNL];
#pragma unroll
    for (int s = 0; s < LNL; ++s) {
        const bool up = (lo >> s) & 1;
        dsg[s] = up ? (T)-1 : (T)1;
        dmul[s] = up ? tw[(lo & ((1 << s) - 1)) * (M >> (s + 1))] : mk<T>(1, 0);
    }
    C<T> w1[LNL], w3[LG];
    const C<T> fin1 = lane_twiddles_x<T, LNL, true>(w1, lo, tw, M);
    const C<T> fin3 = lane_twiddles_x<T, LG, true>(w3, n2, tw, M);
    int brn = 0;  // bitrev of n2 over LG bits
#pragma unroll
    for (int b = 0; b < LG; ++b) brn |= ((n2 >> b) & 1) << (LG - 1 - b);
    C<T> m2[VG], m3[VG];
#pragma unroll
    for (int t = 0; t < VG; ++t) {
        const int k1 = VG * brn + t;
        const C<T> e = tw[(k1 * lo * G) % M];
        m2[t] = cmul<T>(fin1, mk<T>(e.x, -e.y));           // undo step 1's scale, w_P^(-k1 u1)
        const C<T> e3 = tw[((t * n2) % V) * (M / V)];
        m3[t] = cmul<T>(fin3, mk<T>(e3.x, -e3.y));         // undo step 3's scale, w_8^(-t u2a)
    }
    // EA: output group of every held value u = lam + L u2b, and exp(2 pi i qb c / g)
    int n0u[EAF ? VG : 1];
    C<T> ctw[EAF ? G : 1];
    if constexpr (EAF) {
#pragma unroll
        for (int t = 0; t < VG; ++t) n0u[t] = (int)(((lam + L * t) * ax.lg_inv) % P);
        const int qbr = g.qb % G;
#pragma unroll
        for (int c = 0; c < G; ++c) {
            const C<T> e = tw[((qbr * c) % G) * P];
            ctw[c] = mk<T>(e.x, -e.y);
        }
        // the pass's premultiply and twiddle values, once per workgroup
        const C<T>* Tf = (const C<T>*)ax.Tf;
        for (int e = ti; e < g.qn * P; e += kThreads) {
            const int qq = e / P, i = e - qq * P;
            TAs[e] = TA[(int64_t)(g.qb + qq) * M + G * i];
            Tfs[e] = Tf[(int64_t)(g.qb + qq) * M + i];
        }
    }
    const int qc = EAF ? g.qn : g.qc;
    const int nqc = (g.qn + qc - 1) / qc;
    const int64_t ntl = g.Qin * g.ntiles;
    const int64_t T8 = (ntl + 7) / 8;
    const int64_t total = T8 * 8 * nqc;
    for (int64_t bid = blockIdx.x; bid < total; bid += gridDim.x) {
        // every id and index here is below 2^31 (checked on the host): 32-bit division
        const unsigned rr = (unsigned)bid >> 3;
        const int ci = (int)(rr % (unsigned)nqc);
        const int64_t tile = ((int64_t)bid & 7) * T8 + (int64_t)(rr / (unsigned)nqc);
        if (tile >= ntl) continue;  // uniform over the workgroup
        const int64_t qi = (int64_t)((unsigned)tile / (unsigned)g.ntiles);
        const Tile tl = decode_tile(g, tile - qi * g.ntiles);
        const bool live = l < tl.nl;
        const int qlo = g.qb + ci * qc;
        const int qhi = min(qlo + qc, g.qb + g.qn);
        if constexpr (!EAF) {
            const int nta = (qhi - qlo) * P;
            for (int e = ti; e < nta; e += kThreads) TAs[e] = TA[(int64_t)(qlo + e / P) * M + (e % P) * G];
        }
        C<T> x[V];
        if (g.S == 1) {
            const C<T>* src = in + (qi * g.A + tl.a0 + (live ? l : 0)) * M + G * lo + n2;
#pragma unroll
            for (int i = 0; i < V; ++i) x[i] = live ? src[i * L] : mk<T>(0, 0);
        } else {
            const FDiv fdM = tile_div(g, tl, M);
            load_tile<T, V, (sizeof(T) == 4 ? V : 1)>(in, B, g, tl, qi, M, fdM, ldb);
            __syncthreads();
#pragma unroll
            for (int i = 0; i < V; ++i) x[i] = live ? B[l * ldb + G * (NL * i + lo) + n2] : mk<T>(0, 0);
        }
        if (f) {
#pragma unroll
            for (int i = 1; i < V; i += 2) x[i] = mk<T>(-x[i].x, -x[i].y);
        }
        // E_q of the tile's lines for term q (q - qlo < the staged round): a[u2b] = E_q[lam + L u2b]
        auto term = [&](int q, C<T>* a) {
            const int ql = (q - qlo) % kErStage;
            const C<T>* ta = TAs + (q - qlo) * P + lo;
            C<T> v[V];
#pragma unroll
            for (int i = 0; i < V; ++i) v[i] = cmul<T>(x[i], ta[i * NL]);
            RegDFT<T, V, false>::run(v);
#pragma unroll
            for (int j = 0; j < V; ++j) v[j] = cmul<T>(v[j], t1[j]);
#pragma unroll
            for (int s = LNL - 1; s >= 0; --s) {
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    const C<T> pj = shfl_xor_c<T>(v[j], 1 << s);
                    v[j] = cmul<T>(mk<T>(pj.x + dsg[s] * v[j].x, pj.y + dsg[s] * v[j].y), dmul[s]);
                }
            }
            const C<T>* h = Hs + (ql * L + lam) * HR;
#pragma unroll
            for (int j = 0; j < V; ++j) v[j] = cmul<T>(v[j], h[j]);
            // sum over n2: the first step select-free (odd lanes hold k1 ^ 4), then the select form
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = cadd<T>(v[j], shfl_xor_c<T>(v[j + 4], NL));
#pragma unroll
            for (int s = 1; s < LG; ++s) {
                const int half = 4 >> s;
                const bool hi = (n2 >> s) & 1;
#pragma unroll
                for (int j = 0; j < half; ++j) {
                    const C<T> keep = hi ? v[j + half] : v[j];
                    const C<T> send = hi ? v[j] : v[j + half];
                    v[j] = cadd<T>(keep, shfl_xor_c<T>(send, NL << s));
                }
            }
#pragma unroll
            for (int t = 0; t < VG; ++t) {
                C<T> b = v[t];
#pragma unroll
                for (int s = 0; s < LNL; ++s) b = lane_bfly<T>(b, w1[s], 1 << s, s);
                b = cmul<T>(b, m2[t]);
#pragma unroll
                for (int s = 0; s < LG; ++s) b = lane_bfly<T>(b, w3[s], NL << s, s);
                a[t] = cmul<T>(b, m3[t]);
            }
            RegDFT<T, VG, true>::run(a);
        };
        // the table rows of the terms [q, q + kErStage), rearranged for the lanes: HT[q][r][n2] with
        // r = k1 + 8 k2 goes to lane bitrev(k2) + NL n2, slot k1 ^ 4 (n2 odd)
        auto stage_rows = [&](int q) {
            __syncthreads();
            const int cnt = min(kErStage, qhi - q) * M;
            const C<T>* src = HT + (int64_t)q * M;
            for (int e = ti; e < cnt; e += kThreads) {
                const int qq = e / M, rem = e - qq * M;
                const int r = rem >> LG, m2i = rem & (G - 1);
                const int kk2 = r >> 3, kk1 = r & 7;
                int br = 0;
#pragma unroll
                for (int b = 0; b < LNL; ++b) br |= ((kk2 >> b) & 1) << (LNL - 1 - b);
                Hs[(qq * L + br + NL * m2i) * HR + (kk1 ^ ((m2i & 1) << 2))] = src[e];
            }
            __syncthreads();
        };
        if constexpr (!EAF) {
            for (int q = qlo; q < qhi; ++q) {
                if ((q - qlo) % kErStage == 0) stage_rows(q);
                C<T> a[VG];
                term(q, a);
                if (live) {
                    const int64_t qo = qi * g.qn + (q - g.qb);
#pragma unroll
                    for (int t = 0; t < VG; ++t) {
                        const int u = lam + L * t;
                        const int64_t off = (g.S == 1) ? ((qo * g.A + tl.a0 + l) * P + u)
                                                       : (((qo * g.A + tl.a0) * P + u) * g.S + tl.s0 + l);
                        out[off] = a[t];
                    }
                }
            }
        } else {
            // term loop unrolled by g: residue jj of every output group is a fixed register
            C<T> H[VG][G];
#pragma unroll
            for (int t = 0; t < VG; ++t)
#pragma unroll
                for (int c = 0; c < G; ++c) H[t][c] = mk<T>(0, 0);
            for (int q0 = qlo; q0 < qhi; q0 += G) {
#pragma unroll
                for (int jj = 0; jj < G; ++jj) {
                    const int q = q0 + jj;
                    if (q < qhi) {  // uniform
                        if ((q - qlo) % kErStage == 0) stage_rows(q);
                        C<T> a[VG];
                        term(q, a);
#pragma unroll
                        for (int t = 0; t < VG; ++t) H[t][jj] = cfma<T>(H[t][jj], Tfs[(q - g.qb) * P + n0u[t]], a[t]);
                    }
                }
            }
            // the g-point inverse over the residues of each output group: outputs n0 + P c
#pragma unroll
            for (int t = 0; t < VG; ++t) {
                RegDFT<T, G, true>::run(H[t]);
                if (live) {
#pragma unroll
                    for (int c = 0; c < G; ++c) {
                        C<T> v = cmul<T>(H[t][c], ctw[c]);
                        const int nb = n0u[t] + P * c;
                        const int64_t off = (g.S == 1) ? ((qi * g.A + tl.a0 + l) * M + nb)
                                                       : (((qi * g.A + tl.a0) * M + nb) * g.S + tl.s0 + l);
                        if (accumulate) v = cadd<T>(v, out[off]);
                        out[off] = v;
                        if (rho) rho[off] = v.x * v.x + v.y * v.y;
                    }
                }
            }
        }
        __syncthreads();  // the next tile overwrites the buffers the term loop reads
    }
}

// Adjoint of E in the layout of k_ERG (g = 2, 4, 8; P = 16, 32, 64): the output line x (M points)
// collects, over the terms q of the pass, conj(TA_q) * IDFT_P(conj(HT_q[n2]) * DFT_P(y_q)) with both
// transforms unnormalised (the adjoint of E_q = IDFT_P(sum_n2 HT_q[n2] DFT_P(TA_q x_n2))). Lane lam =
// lo + NL n2 reads y_q[lam + L u2b] (u2b < VG) and runs the transpose of the forward pipeline: a
// VG-point forward transform in the lane, the twiddle w_8^(t n2), a g-point forward transform
// across the n2 lanes and the twiddle w_P^(lo k1), an NL-point forward transform across the lo
// lanes (both decimation in frequency: natural input, bit-reversed output), which leaves
// DFT_P(y)[k1 + 8 k2] with k1 = VG bitrev(n2) + t and k2 = bitrev(lo), the layout after the
// forward reduce-scatter; then the transpose of that reduce-scatter (an all-gather over the n2
// lanes, the odd lanes ending with their slots in k1 ^ 4 order), the table multiply, the inverse
// NL-point transform across the lo lanes (bit-reversed input), the twiddle w_P^(-lo k1) and an
// 8-point inverse transform in the lane, times conj(TA_q), summed over the terms in registers. The
// odd lanes' (-1)^i (from their k1 ^ 4 slots) is applied once per tile, when the line is written.
template <typename T, int P, int LG>
__global__ __launch_bounds__(kThreads) void k_EHG(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g, int accumulate, const C<T>* __restrict__ TA,
                                                  const C<T>* __restrict__ HT) {
    constexpr int G = 1 << LG;
    constexpr int V = 8;
    constexpr int NL = P / V;
    constexpr int LNL = ilog2c(NL);
    constexpr int L = NL * G;
    constexpr int TL = kThreads / L;
    constexpr int HR = V + 1;
    constexpr int VG = V >> LG;
    constexpr int M = G * P;
    static_assert(NL >= 2 && (NL & (NL - 1)) == 0 && L <= kWave && LG >= 1 && LG <= 3, "P = 16, 32, 64; g = 2, 4, 8");
    extern __shared__ __align__(16) unsigned char smem[];
    C<T>* TAs = (C<T>*)smem;                  // [q - qb][n1] = TA_q[g n1]
    C<T>* Hs = TAs + g.qn * P;                // [q - q0][lam][HR]
    C<T>* Ys = Hs + kErStage * L * HR;        // strided input: [q - q0][line][P]
    const int lam = (int)threadIdx.x & (L - 1);
    const int l = (int)threadIdx.x / L;
    const int lo = lam & (NL - 1);
    const int n2 = lam >> LNL;
    const int f = (n2 & 1) ? 4 : 0;
    const int ti = (int)threadIdx.x;
    const C<T>* tw = (const C<T>*)ax.tw;
    int brn = 0;
#pragma unroll
    for (int b = 0; b < LG; ++b) brn |= ((n2 >> b) & 1) << (LG - 1 - b);
    // forward part: w_8^(t n2) after the lane transform, w_P^(lo k1) between the two lane transforms
    C<T> b8[VG], dlo[VG];
#pragma unroll
    for (int t = 0; t < VG; ++t) {
        b8[t] = tw[((t * n2) % V) * (M / V)];
        dlo[t] = tw[(lo * (VG * brn + t) * G) % M];
    }
    // decimation-in-frequency stages across n2 (masks NL << s) and across lo (masks 1 << s)
    T sgn2[LG], sgn1[LNL];
    C<T> mul2[LG], mul1[LNL];
#pragma unroll
    for (int s = 0; s < LG; ++s) {
        const bool up = (n2 >> s) & 1;
        sgn2[s] = up ? (T)-1 : (T)1;
        mul2[s] = up ? tw[(n2 & ((1 << s) - 1)) * (M >> (s + 1))] : mk<T>(1, 0);
    }
#pragma unroll
    for (int s = 0; s < LNL; ++s) {
        const bool up = (lo >> s) & 1;
        sgn1[s] = up ? (T)-1 : (T)1;
        mul1[s] = up ? tw[(lo & ((1 << s) - 1)) * (M >> (s + 1))] : mk<T>(1, 0);
    }
    // inverse part: across lo on bit-reversed input, then w_P^(-lo k1) (k1 = j ^ f in slot j) with
    // the scale of the lane butterflies
    C<T> w1[LNL];
    const C<T> fin1 = lane_twiddles_x<T, LNL, true>(w1, lo, tw, M);
    C<T> it1[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        const C<T> e = tw[(lo * (j ^ f) * G) % M];
        it1[j] = cmul<T>(fin1, mk<T>(e.x, -e.y));
    }
    for (int e = ti; e < g.qn * P; e += kThreads) {
        const int qq = e / P, i = e - qq * P;
        TAs[e] = TA[(int64_t)(g.qb + qq) * M + G * i];
    }
    const int64_t ntl = g.Qin * g.ntiles;  // output lines' tiles, < 2^31 (host check)
    const int64_t T8 = (ntl + 7) / 8;
    for (int64_t bid = blockIdx.x; bid < 8 * T8; bid += gridDim.x) {
        const int64_t tile = (bid & 7) * T8 + (bid >> 3);
        if (tile >= ntl) continue;  // uniform over the workgroup
        const int64_t qo = (int64_t)((unsigned)tile / (unsigned)g.ntiles);
        const Tile tl = decode_tile(g, tile - qo * g.ntiles);
        const bool live = l < tl.nl;
        C<T> acc[V];
#pragma unroll
        for (int i = 0; i < V; ++i) acc[i] = mk<T>(0, 0);
        for (int qq = 0; qq < g.qn; ++qq) {
            const int ql = qq % kErStage;
            if (ql == 0) {
                // the next round: table rows in lane order (as k_ERG) and, for strided lines, the
                // inputs of the round's terms with the lines fastest (coalesced)
                __syncthreads();
                const int nq = min(kErStage, g.qn - qq);
                const C<T>* src = HT + (int64_t)(g.qb + qq) * M;
                for (int e = ti; e < nq * M; e += kThreads) {
                    const int q4 = e / M, rem = e - q4 * M;
                    const int r = rem >> LG, m2i = rem & (G - 1);
                    const int kk2 = r >> 3, kk1 = r & 7;
                    int br = 0;
#pragma unroll
                    for (int b = 0; b < LNL; ++b) br |= ((kk2 >> b) & 1) << (LNL - 1 - b);
                    Hs[(q4 * L + br + NL * m2i) * HR + (kk1 ^ ((m2i & 1) << 2))] = src[e];
                }
                if (g.S != 1) {
                    const int per = tl.nl * P;
                    for (int e = ti; e < nq * per; e += kThreads) {
                        const int q4 = e / per, rem = e - q4 * per;
                        const int u = rem / tl.nl, ll = rem - u * tl.nl;
                        const int64_t si = qo * g.qn + qq + q4;
                        Ys[(q4 * TL + ll) * P + u] = in[((si * g.A + tl.a0) * P + u) * g.S + tl.s0 + ll];
                    }
                }
                __syncthreads();
            }
            C<T> v[V];
            // y_q[lam + L u2b]
            if (g.S == 1) {
                const int64_t si = qo * g.qn + qq;
                const C<T>* src = in + (si * g.A + tl.a0 + (live ? l : 0)) * P + lam;
#pragma unroll
                for (int t = 0; t < VG; ++t) v[t] = live ? src[L * t] : mk<T>(0, 0);
            } else {
#pragma unroll
                for (int t = 0; t < VG; ++t) v[t] = live ? Ys[(ql * TL + l) * P + lam + L * t] : mk<T>(0, 0);
            }
            RegDFT<T, VG, false>::run(v);
#pragma unroll
            for (int t = 0; t < VG; ++t) v[t] = cmul<T>(v[t], b8[t]);
#pragma unroll
            for (int s = LG - 1; s >= 0; --s) {
#pragma unroll
                for (int t = 0; t < VG; ++t) {
                    const C<T> pj = shfl_xor_c<T>(v[t], NL << s);
                    v[t] = cmul<T>(mk<T>(pj.x + sgn2[s] * v[t].x, pj.y + sgn2[s] * v[t].y), mul2[s]);
                }
            }
#pragma unroll
            for (int t = 0; t < VG; ++t) v[t] = cmul<T>(v[t], dlo[t]);
#pragma unroll
            for (int s = LNL - 1; s >= 0; --s) {
#pragma unroll
                for (int t = 0; t < VG; ++t) {
                    const C<T> pj = shfl_xor_c<T>(v[t], 1 << s);
                    v[t] = cmul<T>(mk<T>(pj.x + sgn1[s] * v[t].x, pj.y + sgn1[s] * v[t].y), mul1[s]);
                }
            }
            // the transpose of the reduce-scatter: all-gather over the n2 lanes
#pragma unroll
            for (int s = LG - 1; s >= 1; --s) {
                const int half = 4 >> s;
                const bool hi = (n2 >> s) & 1;
#pragma unroll
                for (int j = 0; j < half; ++j) {
                    const C<T> pj = shfl_xor_c<T>(v[j], NL << s);
                    v[j + half] = hi ? v[j] : pj;
                    v[j] = hi ? pj : v[j];
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j + 4] = shfl_xor_c<T>(v[j], NL);
            const C<T>* h = Hs + (ql * L + lam) * HR;
#pragma unroll
            for (int j = 0; j < V; ++j) v[j] = cmulc<T>(v[j], h[j]);
#pragma unroll
            for (int j = 0; j < V; ++j) {
#pragma unroll
                for (int s = 0; s < LNL; ++s) v[j] = lane_bfly<T>(v[j], w1[s], 1 << s, s);
                v[j] = cmul<T>(v[j], it1[j]);
            }
            RegDFT<T, V, true>::run(v);
            const C<T>* ta = TAs + qq * P + lo;
#pragma unroll
            for (int i = 0; i < V; ++i) acc[i] = cfmac<T>(acc[i], v[i], ta[i * NL]);
        }
        if (live) {
#pragma unroll
            for (int i = 0; i < V; ++i) {
                C<T> v = (f && (i & 1)) ? mk<T>(-acc[i].x, -acc[i].y) : acc[i];
                const int n = G * (NL * i + lo) + n2;
                const int64_t off = (g.S == 1) ? ((qo * g.A + tl.a0 + l) * M + n)
                                               : (((qo * g.A + tl.a0) * M + n) * g.S + tl.s0 + l);
                if (accumulate) v = cadd<T>(v, out[off]);
                out[off] = v;
            }
        }
        __syncthreads();  // the next tile overwrites the staged rounds
    }
}

// EA in register form: the E values of every q are combined at once into the lane's M / G = P
// outputs nbar = n2 + G k (the accumulate of (FFpsi) along this axis):
//   out[nbar] = sum_q Tf_q[nbar] E_q[r(nbar)],  r(nbar) = (nbar lg) mod P.
// For a power-of-two P with G >= P, r(nbar) = (n2 lg) mod P is one value per lane, read with one
// cross-lane shuffle from the lane that holds it after the reduce-scatter; otherwise every lane
// keeps all P sums and picks r(nbar) per output.
template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_EAR(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g, int accumulate, T* __restrict__ rho, int lgG,
                                                  const C<T>* __restrict__ TA, const C<T>* __restrict__ Tf,
                                                  const C<T>* __restrict__ HT) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int LP = (P >= 32) ? 5 : (P >= 16) ? 4 : (P >= 8) ? 3 : (P >= 4) ? 2 : (P >= 2) ? 1 : 0;
    const int M = ax.M;
    const int ldb = M + kTilePad;
    C<T>* B = (C<T>*)smem;         // tile: TS rows of ldb (M points each)
    C<T>* TAs = B + (kThreads / ax.g) * ldb;  // TA_q[g i] of every term of the pass, [q - qb][i]
    const int G = 1 << lgG;
    const int l = (int)threadIdx.x >> lgG;
    const int n2 = (int)threadIdx.x & (G - 1);
    const int64_t total = g.Qin * g.ntiles;
    // after the reduction and the cross-lane inverse transform lane u holds E[u]; this lane
    // needs u = (n2 lg) mod P
    const int u_need = (int)(((int64_t)n2 * ax.lg) % P);
    const int lane = (int)threadIdx.x & (kWave - 1);
    const int src_lane = lane - n2 + u_need;
    C<T> wst[LP > 0 ? LP : 1];
    const C<T> fin = lane_twiddles_x<T, LP>(wst, n2, (const C<T>*)ax.tw, M);
    // power-of-two P with G >= P: reduce-scatter and one shuffle; otherwise all-reduce and pick
    const bool scatter = kPow2<P> && G >= P;
    // on the scatter path with P <= 8 the lane's input is modulated by exp(-2 pi i s n1 / P),
    // s = bitrev(n2 mod P), once per tile, its table row comes turned by s, and the lanes are summed
    // by reduce_scatter_rot; for P >= 16 the odd lane's input is modulated by (-1)^n1 and HT is the
    // table arranged for reduce_scatter_x (as for G < P)
    constexpr bool ROT = kPow2<P> && P <= 8;
    int raddr[LP > 2 ? LP - 2 : 1];
    if constexpr (ROT) rot_addrs<P>(raddr, lane, n2);
    const int rsh = ROT ? rot_shift<P>(n2) : 0;
    const bool odd_flip = scatter && !ROT && (n2 & 1) && lgG >= 1;
    const int nta = g.qn * P;
    // r(nbar) of the lane's outputs nbar = n2 + G k is r0 + k d (mod P)
    const int r0 = (int)(((int64_t)n2 * ax.lg) % P);
    const int rd = (int)(((int64_t)G * ax.lg) % P);
    // power-of-two P with G < P: after the reduce-scatter the lane holds cnt values from base
    const int lk = (lgG < LP) ? lgG : LP;
    const int cnt = P >> lk;
    int base = 0;
    for (int s = 0; s < lk; ++s) base += ((n2 >> s) & 1) * ((P >> s) >> 1);
    for (int64_t bid = blockIdx.x; bid < total; bid += gridDim.x) {
        const int64_t qi = (int64_t)((unsigned)bid / (unsigned)g.ntiles);  // total < 2^31 (host check)
        const int64_t tt = bid - qi * g.ntiles;
        const Tile tl = decode_tile(g, tt);
        const FDiv fdM = tile_div(g, tl, M);
        const int ti = (int)threadIdx.x;
        C<T> tav = mk<T>(0, 0);
        if (ti < nta) tav = TA[(int64_t)(g.qb + ti / P) * M + ((ti % P) << lgG)];
        load_tile<T, P, 1>(in, B, g, tl, qi, M, fdM, ldb);  // x stays in registers: keep the load phase lean
        if (ti < nta) TAs[ti] = tav;
        for (int e = ti + kThreads; e < nta; e += kThreads)
            TAs[e] = TA[(int64_t)(g.qb + e / P) * M + ((e % P) << lgG)];
        __syncthreads();
        const bool live = l < tl.nl;
        C<T> x[P], acc[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            x[i] = live ? B[l * ldb + (i << lgG) + n2] : mk<T>(0, 0);
            acc[i] = mk<T>(0, 0);
        }
        if (odd_flip) {
#pragma unroll
            for (int i = 1; i < P; i += 2) x[i] = mk<T>(-x[i].x, -x[i].y);
        }
        if (ROT && scatter) {
            const C<T>* twp = (const C<T>*)ax.tw;
#pragma unroll
            for (int i = 1; i < P; ++i) x[i] = cmul<T>(x[i], twp[((rsh * i) & (P - 1)) << lgG]);
        }
        __syncthreads();
        for (int q = g.qb; q < g.qb + g.qn; ++q) {
            const C<T>* ta = TAs + (q - g.qb) * P;
            const C<T>* h = HT + ((int64_t)q * G + n2) * P;  // [q][n2][r]: the lane's P values contiguous
            const C<T>* tf = Tf + (int64_t)q * M + n2;
            C<T> v[P];
#pragma unroll
            for (int i = 0; i < P; ++i) v[i] = cmul<T>(x[i], ta[i]);
            RegDFT<T, P, false>::run(v);
#pragma unroll
            for (int r = 0; r < P; ++r) v[r] = cmul<T>(v[r], h[r]);
            if (scatter) {
                if constexpr (ROT) reduce_scatter_rot<T, P>(v, raddr);
                else reduce_scatter_x<T, P>(v, n2, lgG);
                C<T> s0 = v[0];
                for (int s = LP; s < lgG; ++s) s0 = cadd<T>(s0, shfl_xor_c<T>(s0, 1 << s));
                s0 = lane_idft_x<T, LP>(s0, wst, fin);  // lane n2 < P now holds E[n2]
                const C<T> e = mk<T>(__shfl(s0.x, src_lane, kWave), __shfl(s0.y, src_lane, kWave));
#pragma unroll
                for (int k = 0; k < P; ++k) acc[k] = cfma<T>(acc[k], tf[k << lgG], e);
            } else {
                RegDFT<T, P, true>::run(v);
                // the line's P sums go through LDS (the tile buffer is free during the q loop)
                C<T>* El = B + l * P;
                if constexpr (kPow2<P>) {
                    reduce_scatter_x<T, P>(v, n2, lgG);  // G < P: the lane holds P / G values from base
#pragma unroll
                    for (int i = 0; i < P; ++i)
                        if (i < cnt) El[base + i] = v[i];
                } else {
                    reduce_all<T, P>(v, lgG);
#pragma unroll
                    for (int u = 0; u < P; ++u)
                        if ((u & (G - 1)) == n2) El[u] = v[u];
                }
                wave_sync();
                int rk = r0;
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    acc[k] = cfma<T>(acc[k], tf[k << lgG], El[rk]);
                    rk += rd;
                    if (rk >= P) rk -= P;
                }
                wave_sync();
            }
        }
        if (live) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int nb = n2 + (k << lgG);
                const int64_t off = (g.S == 1) ? ((qi * g.A + tl.a0 + l) * M + nb)
                                               : (((qi * g.A + tl.a0) * M + nb) * g.S + tl.s0 + l);
                C<T> v = acc[k];
                if (accumulate) v = cadd<T>(v, out[off]);
                out[off] = v;
                if (rho) rho[off] = v.x * v.x + v.y * v.y;
            }
        }
        __syncthreads();  // the next tile overwrites the buffer the q loop used
    }
}

// EA with the structured accumulate, power-of-two P <= g, g = 8, 16, 32 or 64. A workgroup holds
// the TS = 64 / g lines of one wavefront kEaWaves times; wave w takes the terms q with
// q - qb = w (mod kEaWaves). For each term the wave forms E_q of its lines as the register E
// kernel does (lane u < P ends with E_q[u]) and adds Tf_q[n0] E_q[u] into H[line][n0][j],
// n0 = (u lg_inv) mod P (the n0 with r(n0) = u), j = (q - qb) mod g: the waves own disjoint j
// (g is a multiple of kEaWaves). Then, as the structured accumulate (presf),
//   out[n0 + P c] = exp(2 pi i qb c / g) sum_j exp(2 pi i j c / g) H[line][n0][j],
// one g-point inverse per (line, n0), computed by K = g / 8 lanes as in k_ASK.
constexpr int kEaWaves = 8;

// The table rows HT_q of the pass's terms (qn M values) are staged in LDS once per workgroup when
// they fit kEasStageBytes (HST); the grid is then persistent, so every workgroup reuses them over
// many tiles and each term reads its row from LDS instead of global memory.
constexpr size_t kEasStageBytes = 32768;

template <typename T, int P, int K, bool HST>
__global__ __launch_bounds__(kEaWaves * kWave) void k_EAS(const C<T>* __restrict__ in, C<T>* __restrict__ out,
                                                         AxisDev ax, PassGeom g, int accumulate, T* __restrict__ rho,
                                                         int lgG, const C<T>* __restrict__ TA,
                                                         const C<T>* __restrict__ HT) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int LP = (P >= 16) ? 4 : (P >= 8) ? 3 : (P >= 4) ? 2 : (P >= 2) ? 1 : 0;
    constexpr int G = 8 * K;  // g
    constexpr int LK = (K == 8) ? 3 : (K == 4) ? 2 : (K == 2) ? 1 : 0;
    constexpr int TS = kWave / G;
    const int M = ax.M;
    C<T>* B = (C<T>*)smem;              // [TS][M] the tile's lines
    C<T>* H = B + TS * M;               // [TS][P][G]
    C<T>* TAs = H + TS * P * G;         // [q - qb][i]
    const C<T>* Tf = (const C<T>*)ax.Tf;
    const C<T>* twg = (const C<T>*)ax.tw;
    const int tid = (int)threadIdx.x;
    const int w = tid / kWave;
    const int lane = tid % kWave;
    const int l = lane / G;
    const int n2 = lane % G;
    for (int e = tid; e < g.qn * P; e += kEaWaves * kWave)
        TAs[e] = TA[(int64_t)(g.qb + e / P) * M + ((e % P) << lgG)];
    C<T>* Hst = TAs + g.qn * P;  // [q - qb][M] table rows (HST)
    if constexpr (HST) {
        const C<T>* hsrc = HT + (int64_t)g.qb * M;
        for (int e = tid; e < g.qn * M; e += kEaWaves * kWave) Hst[e] = hsrc[e];
    }
    // E part: lane twiddles, the odd lane's spectrum exchange, the lane's accumulate target
    const bool odd_flip = (n2 & 1) && lgG >= 1;
    C<T> wst[LP > 0 ? LP : 1];
    const C<T> fin = lane_twiddles_x<T, LP>(wst, n2, twg, M);
    const int n0u = (int)(((int64_t)(n2 % P) * ax.lg_inv) % P);
    // accumulate part: thread t < TS P K is lane k of group (l, n0)
    const int ak = tid % K;
    const int agrp = tid / K;
    const bool acc_thread = agrp < TS * P;
    int kr = 0;
    for (int b = 0; b < LK; ++b) kr |= ((ak >> b) & 1) << (LK - 1 - b);
    C<T> w1[8];  // exp(2 pi i k c1 / g)
#pragma unroll
    for (int c1 = 0; c1 < 8; ++c1) {
        const C<T> t = twg[((ak * c1) % G) * P];
        w1[c1] = mk<T>(t.x, -t.y);
    }
    C<T> om[LK > 0 ? LK : 1];  // cross-lane stage twiddles exp(2 pi i (k mod h) / (2 h))
#pragma unroll
    for (int st = 0; st < LK; ++st) {
        const int hh = 1 << st;
        const C<T> t = twg[(int64_t)(ak & (hh - 1)) * (M / (2 * hh))];
        om[st] = mk<T>(t.x, -t.y);
    }
    const int qbr = g.qb % G;
    // XCD-contiguous order: workgroups are dispatched round-robin over the 8 XCDs (id mod 8), so
    // tile (id mod 8) T8 + id / 8 gives each XCD a contiguous range of tiles, and the neighbouring
    // tiles that share the cache lines of a strided row meet in one L2
    const int64_t ntl = g.Qin * g.ntiles;  // < 2^31 (host check)
    const int64_t T8 = (ntl + 7) / 8;
    for (int64_t bid = blockIdx.x; bid < 8 * T8; bid += gridDim.x) {
        const int64_t tile = (bid & 7) * T8 + (bid >> 3);
        if (tile >= ntl) continue;  // uniform over the workgroup
        const int64_t qi = (int64_t)((unsigned)tile / (unsigned)g.ntiles);
        const int64_t tt = tile - qi * g.ntiles;
        const Tile tl = decode_tile(g, tt);
        const bool live = l < tl.nl;
        // the tile's lines into LDS (TS M = 64 P <= 2 kEaWaves kWave values: two per thread, both
        // loads issued first), H cleared
        C<T> bv[2];
        int bd[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int e = tid + k * kEaWaves * kWave;
            const int ll = (g.S == 1) ? e / M : e % TS;
            const int n = (g.S == 1) ? e % M : e / TS;
            bd[k] = -1;
            bv[k] = mk<T>(0, 0);
            if (e < TS * M && ll < tl.nl) {
                const int64_t off = (g.S == 1) ? ((qi * g.A + tl.a0 + ll) * M + n)
                                               : (((qi * g.A + tl.a0) * M + n) * g.S + tl.s0 + ll);
                bv[k] = in[off];
                bd[k] = ll * M + n;
            }
        }
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (bd[k] >= 0) B[bd[k]] = bv[k];
        for (int e = tid; e < TS * P * G; e += kEaWaves * kWave) H[e] = mk<T>(0, 0);
        __syncthreads();
        C<T> x[P];
#pragma unroll
        for (int i = 0; i < P; ++i) x[i] = live ? B[l * M + (i << lgG) + n2] : mk<T>(0, 0);
        if (odd_flip) {
#pragma unroll
            for (int i = 1; i < P; i += 2) x[i] = mk<T>(-x[i].x, -x[i].y);
        }
        for (int qq = w; qq < g.qn; qq += kEaWaves) {
            const int q = g.qb + qq;
            const C<T>* ta = TAs + qq * P;
            C<T> v[P];
#pragma unroll
            for (int i = 0; i < P; ++i) v[i] = cmul<T>(x[i], ta[i]);
            RegDFT<T, P, false>::run(v);
            if constexpr (HST) {
                const C<T>* h = Hst + qq * M + n2;
#pragma unroll
                for (int r = 0; r < P; ++r) v[r] = cmul<T>(v[r], h[r << lgG]);
            } else {
                const C<T>* h = HT + (int64_t)q * M + n2;
#pragma unroll
                for (int r = 0; r < P; ++r) v[r] = cmul<T>(v[r], h[r << lgG]);
            }
            reduce_scatter_x<T, P>(v, n2, lgG);
            C<T> s0 = v[0];
            for (int s = LP; s < lgG; ++s) s0 = cadd<T>(s0, shfl_xor_c<T>(s0, 1 << s));
            s0 = lane_idft_x<T, LP>(s0, wst, fin);  // lane n2 < P holds E_q[n2]
            if (live && n2 < P) {
                C<T>* hp = H + (l * P + n0u) * G + (qq % G);
                *hp = cfma<T>(*hp, Tf[(int64_t)q * M + n0u], s0);
            }
        }
        __syncthreads();
        if (acc_thread) {
            const int al = agrp / P;
            const int n0 = agrp % P;
            if (al < tl.nl) {
                const C<T>* hs = H + (al * P + n0) * G;
                C<T> hv[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) hv[m] = hs[ak + K * m];
                RegDFT<T, 8, true>::run(hv);
#pragma unroll
                for (int c1 = 1; c1 < 8; ++c1) hv[c1] = cmul<T>(hv[c1], w1[c1]);
                // K-point inverse transform across the lanes, decimation in frequency
#pragma unroll
                for (int st = LK - 1; st >= 0; --st) {
                    const int hh = 1 << st;
                    const bool upper = (ak & hh) != 0;
#pragma unroll
                    for (int c1 = 0; c1 < 8; ++c1) {
                        const C<T> b = shfl_xor_c<T>(hv[c1], hh);
                        hv[c1] = upper ? cmul<T>(csub<T>(b, hv[c1]), om[st]) : cadd<T>(hv[c1], b);
                    }
                }
#pragma unroll
                for (int c1 = 0; c1 < 8; ++c1) {
                    const int c = c1 + 8 * kr;
                    C<T> v = hv[c1];
                    if (qbr != 0) v = cmulc<T>(v, twg[((qbr * c) % G) * P]);  // exp(+2 pi i qb c / g)
                    const int nb = n0 + P * c;
                    const int64_t off = (g.S == 1) ? ((qi * g.A + tl.a0 + al) * M + nb)
                                                   : (((qi * g.A + tl.a0) * M + nb) * g.S + tl.s0 + al);
                    if (accumulate) v = cadd<T>(v, out[off]);
                    out[off] = v;
                    if (rho) rho[off] = v.x * v.x + v.y * v.y;
                }
            }
        }
        __syncthreads();  // the next tile overwrites B and H
    }
}

// Group decode of the structured accumulates: group index gi -> (qo, a, n0, s, r) with
// gi = ((qo A + a) P + n0) S + s and r = (n0 lg) mod P. Every group index is below 2^31
// (checked on the host), so the divisions are 32-bit.
struct AccGroup {
    int64_t row, qo, a, s;
    int n0, r;
};
__device__ __forceinline__ AccGroup acc_group(unsigned gi, unsigned PS, unsigned S, unsigned A, int P, int lg) {
    AccGroup o;
    const unsigned row = gi / PS;
    const unsigned rem = gi - row * PS;
    const unsigned n0 = rem / S;
    const unsigned qo = row / A;
    o.row = row;
    o.qo = qo;
    o.a = row - qo * A;
    o.s = rem - n0 * S;
    o.n0 = (int)n0;
    o.r = (P < 46341) ? (int)((n0 * (unsigned)lg) % (unsigned)P) : (int)(((int64_t)n0 * lg) % P);
    return o;
}

// Structured accumulate in registers: one thread per group (qo, a, n0, s). For the outputs
// nbar = n0 + P c (c < g) every term reads the same input sample r(n0), and the twiddle (presf)
// satisfies Tf_q[n0 + P c] = Tf_q[n0] exp(2 pi i q c / g), so with j = (q - qb) mod g
//   out[n0 + P c] = exp(2 pi i qb c / g) sum_j exp(2 pi i j c / g) H[j],
//   H[j] = sum_{q - qb = j mod g} Tf_q[n0] in_q[r(n0)],
// a g-point inverse transform of register accumulators per group.
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_ASR(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g, int accumulate, T* __restrict__ rho) {
    const int M = ax.M, P = ax.P;
    const int64_t S = g.S;
    const int64_t PS = (int64_t)P * S;
    const int64_t ngroups = g.Qin * g.A * PS;
    const int64_t step = g.A * PS;  // one magnification slice of the input
    const C<T>* Tf = (const C<T>*)ax.Tf;
    const C<T>* twg = (const C<T>*)ax.tw;
    const int qbr = g.qb % G;
    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < ngroups;
         gi += (int64_t)gridDim.x * blockDim.x) {
        const AccGroup grp = acc_group((unsigned)gi, (unsigned)PS, (unsigned)S, (unsigned)g.A, P, ax.lg);
        const int64_t row = grp.row, qo = grp.qo, a = grp.a, s = grp.s;
        const int n0 = grp.n0, r = grp.r;
        const C<T>* src = in + (qo * g.qn * g.A + a) * PS + (int64_t)r * S + s;
        const C<T>* tf = Tf + (int64_t)g.qb * M + n0;
        C<T> h[G];
#pragma unroll
        for (int j = 0; j < G; ++j) h[j] = mk<T>(0, 0);
        // whole blocks of G terms: every load of a block is issued before the first product
        int i0 = 0;
        for (; i0 + G <= g.qn; i0 += G) {
            C<T> a[G], b[G];
#pragma unroll
            for (int j = 0; j < G; ++j) {
                a[j] = tf[(int64_t)(i0 + j) * M];
                b[j] = src[(int64_t)(i0 + j) * step];
            }
#pragma unroll
            for (int j = 0; j < G; ++j) h[j] = cfma<T>(h[j], a[j], b[j]);
        }
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (i0 + j < g.qn) h[j] = cfma<T>(h[j], tf[(int64_t)(i0 + j) * M], src[(int64_t)(i0 + j) * step]);
        RegDFT<T, G, true>::run(h);
#pragma unroll
        for (int c = 0; c < G; ++c) {
            C<T> v = h[c];
            if (qbr != 0) v = cmulc<T>(v, twg[((qbr * c) % G) * P]);  // exp(+2 pi i qb c / g)
            const int64_t o = (row * M + n0 + (int64_t)P * c) * S + s;
            if (accumulate) v = cadd<T>(v, out[o]);
            out[o] = v;
            if (rho) rho[o] = v.x * v.x + v.y * v.y;
        }
    }
}

// The last two accumulate passes (axes u < v) in one: for the group (o, x, n0_u, y, n0_v, z) the
// outputs nbar_u = n0_u + P_u c_u, nbar_v = n0_v + P_v c_v read one input sample per (q_u, q_v),
// and the twiddles (presf) of both axes advance by q c / g per step P, so
//   out[.., nbar_u, .., nbar_v, ..] = sum_{j_u, j_v} exp(2 pi i (q_u c_u / g_u + q_v c_v / g_v)) H[j_u][j_v],
//   H[j_u][j_v] = sum_{q_u = j_u, q_v = j_v mod g} Tf_u[q_u][n0_u] Tf_v[q_v][n0_v] in[q_v][q_u][r_u][r_v],
// a g_u x g_v inverse transform per group, done in LDS: rows over j_u, a transpose, rows over j_v.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_AA(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev au,
                                                 AxisDev av, AAGeom g, int accumulate, T* __restrict__ rho) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int gu = au.g, gv = av.g, Pu = au.P, Pv = av.P, Mu = au.M, Mv = av.M;
    const int GG = gu * gv;
    const int TSG = g.tsg;
    C<T>* H0 = (C<T>*)smem;
    C<T>* H1 = H0 + TSG * GG;
    C<T>* twu = H1 + TSG * GG;  // exp(-2 pi i k / g_u)
    C<T>* twv = twu + gu;       // exp(-2 pi i k / g_v)
    const C<T>* tu = (const C<T>*)au.tw;
    const C<T>* tv = (const C<T>*)av.tw;
    for (int k = threadIdx.x; k < gu; k += blockDim.x) twu[k] = tu[k * Pu];
    for (int k = threadIdx.x; k < gv; k += blockDim.x) twv[k] = tv[k * Pv];
    __syncthreads();
    const C<T>* Tfu = (const C<T>*)au.Tf;
    const C<T>* Tfv = (const C<T>*)av.Tf;
    const int64_t X = g.X, Y = g.Y, Z = g.Z;
    const int64_t ngroups = g.O * X * Pu * Y * Pv * Z;
    const int64_t ntiles = (ngroups + TSG - 1) / TSG;
    const int qru = g.qb_u % gu, qrv = g.qb_v % gv;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t base = t * TSG;
        const int nt = (int)min((int64_t)TSG, ngroups - base);
        for (int it = threadIdx.x; it < nt * GG; it += blockDim.x) {
            const int p = it % nt;
            const int rest = it / nt;
            const int ju = rest % gu, jv = rest / gu;
            int64_t gi = base + p;
            const int64_t z = gi % Z; gi /= Z;
            const int n0v = (int)(gi % Pv); gi /= Pv;
            const int64_t y = gi % Y; gi /= Y;
            const int n0u = (int)(gi % Pu); gi /= Pu;
            const int64_t x = gi % X;
            const int64_t o = gi / X;
            const int ru = (int)(((int64_t)n0u * au.lg) % Pu);
            const int rv = (int)(((int64_t)n0v * av.lg) % Pv);
            C<T> acc = mk<T>(0, 0);
            for (int iv = jv; iv < g.qn_v; iv += gv) {
                const int qv = g.qb_v + iv;
                const C<T> fv = Tfv[(int64_t)qv * Mv + n0v];
                C<T> su = mk<T>(0, 0);
                for (int iu = ju; iu < g.qn_u; iu += gu) {
                    const int qu = g.qb_u + iu;
                    const int64_t slice = (o * g.qn_v + iv) * g.qn_u + iu;
                    const int64_t a = ((((slice * X + x) * Pu + ru) * Y + y) * Pv + rv) * Z + z;
                    su = cfma<T>(su, Tfu[(int64_t)qu * Mu + n0u], in[a]);
                }
                acc = cfma<T>(acc, fv, su);
            }
            H0[(p * gv + jv) * gu + ju] = acc;
        }
        __syncthreads();
        C<T>* R1 = lds_fft<T>(H0, H1, nt * gv, gu, au.fg, twu, 1, true);  // rows over j_u
        C<T>* Tb = (R1 == H0) ? H1 : H0;
        for (int e = threadIdx.x; e < nt * GG; e += blockDim.x) {
            const int cu = e % gu, r = e / gu;  // r = p * gv + jv
            const int jv = r % gv, p = r / gv;
            Tb[(p * gu + cu) * gv + jv] = R1[e];
        }
        __syncthreads();
        C<T>* R2 = lds_fft<T>(Tb, R1, nt * gu, gv, av.fg, twv, 1, true);  // rows over j_v
        for (int e = threadIdx.x; e < nt * GG; e += blockDim.x) {
            const int p = e % nt;
            const int rest = e / nt;
            const int cv = rest % gv, cu = rest / gv;
            int64_t gi = base + p;
            const int64_t z = gi % Z; gi /= Z;
            const int n0v = (int)(gi % Pv); gi /= Pv;
            const int64_t y = gi % Y; gi /= Y;
            const int n0u = (int)(gi % Pu); gi /= Pu;
            const int64_t x = gi % X;
            const int64_t o = gi / X;
            C<T> v = R2[(p * gu + cu) * gv + cv];
            if (qru != 0) v = cmulc<T>(v, tu[((qru * cu) % gu) * Pu]);  // exp(+2 pi i qb_u c_u / g_u)
            if (qrv != 0) v = cmulc<T>(v, tv[((qrv * cv) % gv) * Pv]);  // exp(+2 pi i qb_v c_v / g_v)
            const int64_t oa = ((((o * X + x) * Mu + n0u + (int64_t)Pu * cu) * Y + y) * Mv + n0v + (int64_t)Pv * cv) * Z + z;
            if (accumulate) v = cadd<T>(v, out[oa]);
            out[oa] = v;
            if (rho) rho[oa] = v.x * v.x + v.y * v.y;
        }
        __syncthreads();
    }
}

// The last two accumulate passes (axes u < v, the last two axes: Y = Z = 1) in registers for
// g_u = g_v = G (16 or 32). The G x G inverse transform of a group (the one k_AA does in LDS) runs
// as two structured accumulates: G K threads per group (K = G / R), thread (j_v, k) first holds
// H[k + K m][j_v] (m < R), transforms over j_u as the one-axis register accumulate does (an
// R-point transform in registers, a twiddle, a K-point transform across the K lanes), passes its
// values through LDS so that thread (c_u, k) holds j_v = k + K m of row c_u, and transforms over
// j_v the same way. Workgroups take the groups in XCD-contiguous ranges: the groups of one output line
// (all n0_v of an n0_u) write the same cache lines.
constexpr int aar_threads(int G, int R) { return (G * G / R > kThreads) ? G * G / R : kThreads; }

template <typename T, int G, int R>
__global__ __launch_bounds__(2 * kThreads) void k_AAR(const C<T>* __restrict__ in, C<T>* __restrict__ out,
                                                      AxisDev au, AxisDev av, AAGeom g, int accumulate,
                                                      T* __restrict__ rho) {
    constexpr int K = G / R;
    constexpr int LK = ilog2c(K);
    constexpr int TPG = G * K;                 // threads per group
    constexpr int WG = aar_threads(G, R);      // threads per workgroup
    constexpr int NG = WG / TPG;               // groups per workgroup
    constexpr int LDR = G + 1;                 // LDS row stride
    static_assert(TPG * NG == WG && WG <= 2 * kThreads, "group size must divide the workgroup");
    __shared__ __align__(16) unsigned char smem_aar[NG * G * LDR * sizeof(C<T>)];
    const int Pu = au.P, Pv = av.P, Mu = au.M, Mv = av.M;
    const int slot = (int)threadIdx.x / TPG;
    const int tt = (int)threadIdx.x % TPG;
    const int row = tt / K;  // j_v in the first transform, c_u in the second
    const int k = tt % K;
    C<T>* Sg = (C<T>*)smem_aar + slot * G * LDR;
    int kr = 0;  // bitrev_LK(k)
    for (int b = 0; b < LK; ++b) kr |= ((k >> b) & 1) << (LK - 1 - b);
    const C<T>* tu = (const C<T>*)au.tw;
    const C<T>* tv = (const C<T>*)av.tw;
    C<T> w1u[R], w1v[R];  // exp(2 pi i k c1 / G) of each axis
#pragma unroll
    for (int c1 = 0; c1 < R; ++c1) {
        const C<T> a = tu[((k * c1) % G) * Pu];
        const C<T> b = tv[((k * c1) % G) * Pv];
        w1u[c1] = mk<T>(a.x, -a.y);
        w1v[c1] = mk<T>(b.x, -b.y);
    }
    const C<T>* Tfu = (const C<T>*)au.Tf;
    const C<T>* Tfv = (const C<T>*)av.Tf;
    const int qnu = g.qn_u, qnv = g.qn_v;
    const int qru = g.qb_u % G, qrv = g.qb_v % G;
    // cross-lane stage twiddles exp(2 pi i (k mod h) / (2 h)), h = 2^st (M / 2h = P G / 2h)
    C<T> omu[LK], omv[LK];
#pragma unroll
    for (int st = 0; st < LK; ++st) {
        const int hh = 1 << st;
        const C<T> a = tu[(k & (hh - 1)) * (Pu * (G / (2 * hh)))];
        const C<T> b = tv[(k & (hh - 1)) * (Pv * (G / (2 * hh)))];
        omu[st] = mk<T>(a.x, -a.y);
        omv[st] = mk<T>(b.x, -b.y);
    }
    const int64_t X = g.X;
    const int64_t PP = (int64_t)Pu * Pv;
    const int64_t step_u = X * PP;              // input stride of one term along u
    const int64_t step_v = (int64_t)qnu * step_u;  // input stride of one term along v
    // group indices are below 2^31 (aar_applicable): 32-bit decode
    const unsigned ngroups = (unsigned)(g.O * X * PP);
    const unsigned ntl = (ngroups + NG - 1) / NG;
    const unsigned T8 = (ntl + 7) / 8;
    const unsigned total = T8 * 8;
    for (unsigned bid = blockIdx.x; bid < total; bid += gridDim.x) {
        const unsigned tile = (bid & 7) * T8 + (bid >> 3);
        if (tile >= ntl) continue;  // uniform over the workgroup
        const unsigned gid = tile * NG + slot;
        const bool live = gid < ngroups;
        const unsigned gq = live ? gid : 0;
        const unsigned t1 = gq / (unsigned)Pv;
        const int n0v = (int)(gq - t1 * (unsigned)Pv);
        const unsigned ox = t1 / (unsigned)Pu;
        const int n0u = (int)(t1 - ox * (unsigned)Pu);
        const unsigned o32 = ox / (unsigned)X;
        const int64_t x = (int64_t)(ox - o32 * (unsigned)X), o = o32;
        const int ru = (n0u * au.lg) % Pu;  // n0 lg < P^2 <= 2^16
        const int rv = (n0v * av.lg) % Pv;
        const C<T>* src = in + ((o * qnv * qnu) * X + x) * PP + (int64_t)(ru * Pv + rv);
        const C<T>* tfu = Tfu + (g.qb_u * Mu + n0u);  // lambda M <= 2^26
        const C<T>* tfv = Tfv + (g.qb_v * Mv + n0v);
        // H[k + K m][row]: the terms i_u = j_u (mod G), i_v = row (mod G)
        C<T> h[R];
#pragma unroll
        for (int m = 0; m < R; ++m) h[m] = mk<T>(0, 0);
        if (live) {
            for (int iv = row; iv < qnv; iv += G) {
                const C<T> fv = tfv[iv * Mv];
                const C<T>* sv = src + (int64_t)iv * step_v;
                C<T> su[R];
#pragma unroll
                for (int m = 0; m < R; ++m) su[m] = mk<T>(0, 0);
                int i0 = 0;
                for (; i0 + G <= qnu; i0 += G) {
                    C<T> a[R], b[R];
#pragma unroll
                    for (int m = 0; m < R; ++m) {
                        const int i = i0 + k + K * m;
                        a[m] = tfu[i * Mu];
                        b[m] = sv[(int64_t)i * step_u];
                    }
#pragma unroll
                    for (int m = 0; m < R; ++m) su[m] = cfma<T>(su[m], a[m], b[m]);
                }
#pragma unroll
                for (int m = 0; m < R; ++m) {
                    const int i = i0 + k + K * m;
                    if (i < qnu) su[m] = cfma<T>(su[m], tfu[i * Mu], sv[(int64_t)i * step_u]);
                }
#pragma unroll
                for (int m = 0; m < R; ++m) h[m] = cfma<T>(h[m], fv, su[m]);
            }
        }
        // transform over j_u; lane k ends with c_u = c1 + R bitrev(k)
        RegDFT<T, R, true>::run(h);
#pragma unroll
        for (int c1 = 1; c1 < R; ++c1) h[c1] = cmul<T>(h[c1], w1u[c1]);
#pragma unroll
        for (int st = LK - 1; st >= 0; --st) {
            const int hh = 1 << st;
            const bool upper = (k & hh) != 0;
#pragma unroll
            for (int c1 = 0; c1 < R; ++c1) {
                const C<T> b = shfl_xor_c<T>(h[c1], hh);
                h[c1] = upper ? cmul<T>(csub<T>(b, h[c1]), omu[st]) : cadd<T>(h[c1], b);
            }
        }
#pragma unroll
        for (int c1 = 0; c1 < R; ++c1) Sg[(c1 + R * kr) * LDR + row] = h[c1];
        __syncthreads();
        // row c_u = row: j_v = k + K m
#pragma unroll
        for (int m = 0; m < R; ++m) h[m] = Sg[row * LDR + k + K * m];
        RegDFT<T, R, true>::run(h);
#pragma unroll
        for (int c1 = 1; c1 < R; ++c1) h[c1] = cmul<T>(h[c1], w1v[c1]);
#pragma unroll
        for (int st = LK - 1; st >= 0; --st) {
            const int hh = 1 << st;
            const bool upper = (k & hh) != 0;
#pragma unroll
            for (int c1 = 0; c1 < R; ++c1) {
                const C<T> b = shfl_xor_c<T>(h[c1], hh);
                h[c1] = upper ? cmul<T>(csub<T>(b, h[c1]), omv[st]) : cadd<T>(h[c1], b);
            }
        }
        if (live) {
            const int cu = row;
            C<T> fu = mk<T>(1, 0);
            if (qru != 0) {  // exp(+2 pi i qb_u c_u / G)
                const C<T> t = tu[((qru * cu) % G) * Pu];
                fu = mk<T>(t.x, -t.y);
            }
            C<T>* dst = out + ((o * X + x) * Mu + n0u + (int64_t)Pu * cu) * Mv + n0v;
            T* drho = rho ? rho + ((o * X + x) * Mu + n0u + (int64_t)Pu * cu) * Mv + n0v : nullptr;
#pragma unroll
            for (int c1 = 0; c1 < R; ++c1) {
                const int cv = c1 + R * kr;
                C<T> v = cmul<T>(h[c1], fu);
                if (qrv != 0) v = cmulc<T>(v, tv[((qrv * cv) % G) * Pv]);  // exp(+2 pi i qb_v c_v / G)
                const int64_t oi = (int64_t)Pv * cv;
                if (accumulate) v = cadd<T>(v, dst[oi]);
                dst[oi] = v;
                if (drho) drho[oi] = v.x * v.x + v.y * v.y;
            }
        }
        __syncthreads();  // the next tile overwrites the LDS rows
    }
}

// Adjoint of k_AAR (the first two AH passes of the adjoint schedule, axes v then u, fused). For
// the group (n0_u, n0_v) the inputs y[c_u][c_v] = in[.., n0_u + P_u c_u, n0_v + P_v c_v] give every
// term pair's output sample through one G x G forward transform,
//   out[q_v][q_u][.., r_u, r_v] = conj(Tf_u[q_u][n0_u] Tf_v[q_v][n0_v]) Yh[(q_u - qb_u) mod G][(q_v - qb_v) mod G],
// done as the one-axis register adjoint (k_AHK) twice: thread (c_u, k) transforms its row over c_v
// (reading c_v = c1 + 4 bitrev(k)), the values pass through LDS to thread (j_v, k), which holds
// c_u = c1 + 4 bitrev(k) of column j_v, and transforms over c_u, leaving Yh[k + K m][j_v].
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_AAHR(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev au,
                                                   AxisDev av, AAGeom g, int accumulate) {
    constexpr int R = 4;
    constexpr int K = G / R;
    constexpr int LK = (K == 8) ? 3 : (K == 4) ? 2 : 1;
    constexpr int TPG = G * K;
    constexpr int NG = kThreads / TPG;
    constexpr int LDR = G + 1;
    static_assert(TPG * NG == kThreads, "group size must divide the workgroup");
    __shared__ __align__(16) unsigned char smem_aahr[NG * G * LDR * sizeof(C<T>)];
    const int Pu = au.P, Pv = av.P, Mu = au.M, Mv = av.M;
    const int slot = (int)threadIdx.x / TPG;
    const int tt = (int)threadIdx.x % TPG;
    const int row = tt / K;  // c_u in the first transform, j_v in the second
    const int k = tt % K;
    C<T>* Sg = (C<T>*)smem_aahr + slot * G * LDR;
    int kr = 0;  // bitrev_LK(k)
    for (int b = 0; b < LK; ++b) kr |= ((k >> b) & 1) << (LK - 1 - b);
    const C<T>* tu = (const C<T>*)au.tw;
    const C<T>* tv = (const C<T>*)av.tw;
    // cross-lane stage twiddles of each axis (select-free form; the rescale goes into w1)
    C<T> wsu[LK], wsv[LK];
    const C<T> finu = lane_twiddles_x<T, LK, false>(wsu, k, tu, Mu);
    const C<T> finv = lane_twiddles_x<T, LK, false>(wsv, k, tv, Mv);
    C<T> w1u[R], w1v[R];  // exp(-2 pi i k c1 / G) times the rescale
#pragma unroll
    for (int c1 = 0; c1 < R; ++c1) {
        w1u[c1] = cmul<T>(tu[((k * c1) % G) * Pu], finu);
        w1v[c1] = cmul<T>(tv[((k * c1) % G) * Pv], finv);
    }
    const C<T>* Tfu = (const C<T>*)au.Tf;
    const C<T>* Tfv = (const C<T>*)av.Tf;
    const int qnu = g.qn_u, qnv = g.qn_v;
    const int qru = g.qb_u % G, qrv = g.qb_v % G;
    const int64_t X = g.X;
    const int64_t PP = (int64_t)Pu * Pv;
    const int64_t step_u = X * PP;
    const int64_t step_v = (int64_t)qnu * step_u;
    // group indices are below 2^31 (aar_applicable): 32-bit decode
    const unsigned ngroups = (unsigned)(g.O * X * PP);
    const unsigned ntl = (ngroups + NG - 1) / NG;
    const unsigned T8 = (ntl + 7) / 8;
    const unsigned total = T8 * 8;
    for (unsigned bid = blockIdx.x; bid < total; bid += gridDim.x) {
        const unsigned tile = (bid & 7) * T8 + (bid >> 3);
        if (tile >= ntl) continue;  // uniform over the workgroup
        const unsigned gid = tile * NG + slot;
        const bool live = gid < ngroups;
        const unsigned gq = live ? gid : 0;
        const unsigned t1 = gq / (unsigned)Pv;
        const int n0v = (int)(gq - t1 * (unsigned)Pv);
        const unsigned ox = t1 / (unsigned)Pu;
        const int n0u = (int)(t1 - ox * (unsigned)Pu);
        const unsigned o32 = ox / (unsigned)X;
        const int64_t x = (int64_t)(ox - o32 * (unsigned)X), o = o32;
        const int ru = (n0u * au.lg) % Pu;  // n0 lg < P^2 <= 2^16
        const int rv = (n0v * av.lg) % Pv;
        // row c_u of the group, c_v = c1 + R bitrev(k)
        C<T> h[R];
        {
            const C<T>* src = in + ((o * X + x) * Mu + n0u + (int64_t)Pu * row) * Mv + n0v;
#pragma unroll
            for (int c1 = 0; c1 < R; ++c1) h[c1] = live ? src[(int64_t)Pv * (c1 + R * kr)] : mk<T>(0, 0);
        }
        if (qrv != 0) {  // exp(-2 pi i qb_v c_v / G)
#pragma unroll
            for (int c1 = 0; c1 < R; ++c1) h[c1] = cmul<T>(h[c1], tv[((qrv * (c1 + R * kr)) % G) * Pv]);
        }
#pragma unroll
        for (int st = 0; st < LK; ++st) {
#pragma unroll
            for (int c1 = 0; c1 < R; ++c1) h[c1] = lane_bfly<T>(h[c1], wsv[st], 1 << st, st);
        }
#pragma unroll
        for (int c1 = 0; c1 < R; ++c1) h[c1] = cmul<T>(h[c1], w1v[c1]);
        RegDFT<T, R, false>::run(h);  // h[m] = Z[c_u = row][j_v = k + K m]
#pragma unroll
        for (int m = 0; m < R; ++m) Sg[(k + K * m) * LDR + row] = h[m];
        __syncthreads();
        // column j_v = row: c_u = c1 + R bitrev(k)
#pragma unroll
        for (int c1 = 0; c1 < R; ++c1) h[c1] = Sg[row * LDR + c1 + R * kr];
        if (qru != 0) {  // exp(-2 pi i qb_u c_u / G)
#pragma unroll
            for (int c1 = 0; c1 < R; ++c1) h[c1] = cmul<T>(h[c1], tu[((qru * (c1 + R * kr)) % G) * Pu]);
        }
#pragma unroll
        for (int st = 0; st < LK; ++st) {
#pragma unroll
            for (int c1 = 0; c1 < R; ++c1) h[c1] = lane_bfly<T>(h[c1], wsu[st], 1 << st, st);
        }
#pragma unroll
        for (int c1 = 0; c1 < R; ++c1) h[c1] = cmul<T>(h[c1], w1u[c1]);
        RegDFT<T, R, false>::run(h);  // h[m] = Yh[j_u = k + K m][j_v = row]
        if (live) {
            C<T>* dst = out + ((o * qnv * qnu) * X + x) * PP + (int64_t)(ru * Pv + rv);
            const C<T>* tfu = Tfu + (g.qb_u * Mu + n0u);  // lambda M <= 2^26
            const C<T>* tfv = Tfv + (g.qb_v * Mv + n0v);
            for (int iv = row; iv < qnv; iv += G) {
                const C<T> fv = tfv[iv * Mv];
                C<T>* dv = dst + (int64_t)iv * step_v;
                for (int i0 = 0; i0 < qnu; i0 += G) {
                    C<T> t[R];
#pragma unroll
                    for (int m = 0; m < R; ++m) {
                        const int i = i0 + k + K * m;
                        t[m] = (i < qnu) ? tfu[i * Mu] : mk<T>(1, 0);
                    }
#pragma unroll
                    for (int m = 0; m < R; ++m) {
                        const int i = i0 + k + K * m;
                        if (i < qnu) {
                            C<T>* po = dv + (int64_t)i * step_u;
                            C<T> v = cmulc<T>(cmulc<T>(h[m], t[m]), fv);
                            if (accumulate) v = cadd<T>(v, *po);
                            *po = v;
                        }
                    }
                }
            }
        }
        __syncthreads();  // the next tile overwrites the LDS rows
    }
}

// Structured accumulate for g = R K (K lanes per group, R = 8 or 4 residues per lane): lane k of a
// group keeps the residues j = k + K m (m < R). With c = c1 + R c2 the g-point inverse transform
// splits as
//   out[c1 + R c2] = sum_k exp(2 pi i k c2 / K) exp(2 pi i k c1 / g) sum_m exp(2 pi i m c1 / R) H[k + K m],
// an R-point transform in registers, a twiddle, and a K-point transform across the K lanes
// (radix-2 decimation in frequency; lane k ends with c2 = bitrev(k)).
template <typename T, int K, int R>
__global__ __launch_bounds__(kThreads) void k_ASK(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g, int accumulate, T* __restrict__ rho) {
    constexpr int G = R * K;
    constexpr int LK = (K == 16) ? 4 : (K == 8) ? 3 : (K == 4) ? 2 : (K == 2) ? 1 : 0;
    const int M = ax.M, P = ax.P;
    const int64_t S = g.S;
    const int64_t PS = (int64_t)P * S;
    const int64_t ngroups = g.Qin * g.A * PS;
    const int64_t step = g.A * PS;
    const C<T>* Tf = (const C<T>*)ax.Tf;
    const C<T>* twg = (const C<T>*)ax.tw;
    const int k = (int)(threadIdx.x & (K - 1));  // the grid stride is a multiple of K
    int kr = 0;                                  // bitrev_LK(k)
    for (int b = 0; b < LK; ++b) kr |= ((k >> b) & 1) << (LK - 1 - b);
    C<T> w1[R];  // exp(2 pi i k c1 / g)
#pragma unroll
    for (int c1 = 0; c1 < R; ++c1) {
        const C<T> t = twg[((k * c1) % G) * P];
        w1[c1] = mk<T>(t.x, -t.y);
    }
    const int qbr = g.qb % G;
    const int64_t nthreads = ngroups * K;
    for (int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gt < nthreads;
         gt += (int64_t)gridDim.x * blockDim.x) {
        const AccGroup grp = acc_group((unsigned)(gt / K), (unsigned)PS, (unsigned)S, (unsigned)g.A, P, ax.lg);
        const int64_t row = grp.row, qo = grp.qo, a = grp.a, s = grp.s;
        const int n0 = grp.n0, r = grp.r;
        const C<T>* src = in + (qo * g.qn * g.A + a) * PS + (int64_t)r * S + s;
        const C<T>* tf = Tf + (int64_t)g.qb * M + n0;
        C<T> h[R];
#pragma unroll
        for (int m = 0; m < R; ++m) h[m] = mk<T>(0, 0);
        int i0 = 0;
        for (; i0 + G <= g.qn; i0 += G) {
            C<T> av[R], bv[R];
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int i = i0 + k + K * m;
                av[m] = tf[(int64_t)i * M];
                bv[m] = src[(int64_t)i * step];
            }
#pragma unroll
            for (int m = 0; m < R; ++m) h[m] = cfma<T>(h[m], av[m], bv[m]);
        }
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int i = i0 + k + K * m;
            if (i < g.qn) h[m] = cfma<T>(h[m], tf[(int64_t)i * M], src[(int64_t)i * step]);
        }
        RegDFT<T, R, true>::run(h);
#pragma unroll
        for (int c1 = 1; c1 < R; ++c1) h[c1] = cmul<T>(h[c1], w1[c1]);
        // K-point inverse transform across the lanes, decimation in frequency
#pragma unroll
        for (int st = LK - 1; st >= 0; --st) {
            const int hh = 1 << st;
            const bool upper = (k & hh) != 0;
            const int jj = k & (hh - 1);
            // exp(+2 pi i jj / (2 hh)) = conj(tw[jj * M / (2 hh)])
            const C<T> t = twg[(int64_t)jj * (M / (2 * hh))];
            const C<T> om = mk<T>(t.x, -t.y);
#pragma unroll
            for (int c1 = 0; c1 < R; ++c1) {
                const C<T> b = shfl_xor_c<T>(h[c1], hh);
                h[c1] = upper ? cmul<T>(csub<T>(b, h[c1]), om) : cadd<T>(h[c1], b);
            }
        }
#pragma unroll
        for (int c1 = 0; c1 < R; ++c1) {
            const int c = c1 + R * kr;
            C<T> v = h[c1];
            if (qbr != 0) v = cmulc<T>(v, twg[((qbr * c) % G) * P]);  // exp(+2 pi i qb c / g)
            const int64_t o = (row * M + n0 + (int64_t)P * c) * S + s;
            if (accumulate) v = cadd<T>(v, out[o]);
            out[o] = v;
            if (rho) rho[o] = v.x * v.x + v.y * v.y;
        }
    }
}

// AH (adjoint of A) in register form. For the group (qo, a, n0, s) of the forward structured
// accumulate, the inputs y[c] = in[.., n0 + P c, ..] (c < g) give every term's output sample
//   out_q[r(n0)] = conj(Tf_q[n0]) sum_c exp(-2 pi i q c / g) y[c] = conj(Tf_q[n0]) Yh[(q - qb) mod g],
//   Yh[j] = sum_c exp(-2 pi i j c / g) exp(-2 pi i qb c / g) y[c],
// the conjugate transpose of the forward group: one g-point forward transform per group, read
// by every term. One thread per group (g <= 8).
template <typename T, int G>
__global__ __launch_bounds__(kThreads) void k_AHR(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g, int accumulate) {
    const int M = ax.M, P = ax.P;
    const int64_t S = g.S;
    const int64_t PS = (int64_t)P * S;
    const int64_t ngroups = g.Qin * g.A * PS;
    const int64_t step = g.A * PS;  // one magnification slice of the output
    const C<T>* Tf = (const C<T>*)ax.Tf;
    const C<T>* twg = (const C<T>*)ax.tw;
    const int qbr = g.qb % G;
    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < ngroups;
         gi += (int64_t)gridDim.x * blockDim.x) {
        const AccGroup grp = acc_group((unsigned)gi, (unsigned)PS, (unsigned)S, (unsigned)g.A, P, ax.lg);
        const C<T>* src = in + (grp.row * M + grp.n0) * S + grp.s;
        C<T>* dst = out + (grp.qo * g.qn * g.A + grp.a) * PS + (int64_t)grp.r * S + grp.s;
        const C<T>* tf = Tf + (int64_t)g.qb * M + grp.n0;
        C<T> y[G];
#pragma unroll
        for (int c = 0; c < G; ++c) y[c] = src[(int64_t)c * PS];
        if (qbr != 0) {
#pragma unroll
            for (int c = 1; c < G; ++c) y[c] = cmul<T>(y[c], twg[((qbr * c) % G) * P]);  // exp(-2 pi i qb c / g)
        }
        RegDFT<T, G, false>::run(y);
        for (int i0 = 0; i0 < g.qn; i0 += G) {
            C<T> t[G];
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (i0 + j < g.qn) t[j] = tf[(int64_t)(i0 + j) * M];
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (i0 + j < g.qn) {
                    C<T>* o = dst + (int64_t)(i0 + j) * step;
                    C<T> v = cmulc<T>(y[j], t[j]);
                    if (accumulate) v = cadd<T>(v, *o);
                    *o = v;
                }
            }
        }
    }
}

// AH in register form for g = R K (K lanes per group, R = 8 or 4 residues per lane), the transpose
// of k_ASK: lane k reads y[c1 + R bitrev(k)] (c1 < R), a K-point forward transform across the lanes
// (decimation in time on bit-reversed input) gives Z[c1] = sum_c2 exp(-2 pi i k c2 / K) y[c1 + R c2],
// the twiddle exp(-2 pi i k c1 / g), and an R-point transform over c1 leaves Yh[k + K m] (m < R).
template <typename T, int K, int R>
__global__ __launch_bounds__(kThreads) void k_AHK(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                  PassGeom g, int accumulate) {
    constexpr int G = R * K;
    constexpr int LK = (K == 16) ? 4 : (K == 8) ? 3 : (K == 4) ? 2 : (K == 2) ? 1 : 0;
    const int M = ax.M, P = ax.P;
    const int64_t S = g.S;
    const int64_t PS = (int64_t)P * S;
    const int64_t ngroups = g.Qin * g.A * PS;
    const int64_t step = g.A * PS;
    const C<T>* Tf = (const C<T>*)ax.Tf;
    const C<T>* twg = (const C<T>*)ax.tw;
    const int k = (int)(threadIdx.x & (K - 1));  // the grid stride is a multiple of K
    int kr = 0;                                  // bitrev_LK(k)
    for (int b = 0; b < LK; ++b) kr |= ((k >> b) & 1) << (LK - 1 - b);
    // cross-lane stage twiddles (select-free form; its rescale goes into w1)
    C<T> wst[LK > 0 ? LK : 1];
    const C<T> fin = lane_twiddles_x<T, LK, false>(wst, k, twg, M);
    C<T> w1[R];  // exp(-2 pi i k c1 / g) times the rescale
#pragma unroll
    for (int c1 = 0; c1 < R; ++c1) w1[c1] = cmul<T>(twg[((k * c1) % G) * P], fin);
    const int qbr = g.qb % G;
    const int64_t nthreads = ngroups * K;
    for (int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gt < nthreads;
         gt += (int64_t)gridDim.x * blockDim.x) {
        const AccGroup grp = acc_group((unsigned)(gt / K), (unsigned)PS, (unsigned)S, (unsigned)g.A, P, ax.lg);
        const C<T>* src = in + (grp.row * M + grp.n0) * S + grp.s;
        C<T>* dst = out + (grp.qo * g.qn * g.A + grp.a) * PS + (int64_t)grp.r * S + grp.s;
        const C<T>* tf = Tf + (int64_t)g.qb * M + grp.n0;
        C<T> h[R];
#pragma unroll
        for (int c1 = 0; c1 < R; ++c1) h[c1] = src[(int64_t)(c1 + R * kr) * PS];
        if (qbr != 0) {
#pragma unroll
            for (int c1 = 0; c1 < R; ++c1) h[c1] = cmul<T>(h[c1], twg[((qbr * (c1 + R * kr)) % G) * P]);
        }
#pragma unroll
        for (int st = 0; st < LK; ++st) {
#pragma unroll
            for (int c1 = 0; c1 < R; ++c1) h[c1] = lane_bfly<T>(h[c1], wst[st], 1 << st, st);
        }
#pragma unroll
        for (int c1 = 0; c1 < R; ++c1) h[c1] = cmul<T>(h[c1], w1[c1]);
        RegDFT<T, R, false>::run(h);
        for (int i0 = 0; i0 < g.qn; i0 += G) {
            C<T> t[R];
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int i = i0 + k + K * m;
                if (i < g.qn) t[m] = tf[(int64_t)i * M];
            }
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int i = i0 + k + K * m;
                if (i < g.qn) {
                    C<T>* o = dst + (int64_t)i * step;
                    C<T> v = cmulc<T>(h[m], t[m]);
                    if (accumulate) v = cadd<T>(v, *o);
                    *o = v;
                }
            }
        }
    }
}

// EH (adjoint of E, summed over q) in register form, power-of-two P <= g. For lane (line, n2):
//   x[g n1 + n2] = sum_q conj(TA_q[g n1]) sum_r exp(2 pi i n1 r / P) conj(HT_q[n2][r]) Y_q[r],
//   Y_q[r] = sum_u exp(-2 pi i r u / P) y_q[u],
// the conjugate transpose of every step of the register E, in reverse order. Each lane forms the
// P-point transform of the line's P inputs itself (the G lanes of a line read the same values).
// A workgroup holds the 64 / g lines of one wavefront kEhWaves times: wave w sums the terms
// q = qb + w (mod kEhWaves), and the partial sums of the waves are added through LDS, so every
// output is written once (no atomics, no clearing pass).
constexpr int kEhWaves = 8;

template <typename T, int P>
__global__ __launch_bounds__(kEhWaves * kWave) void k_EHR(const C<T>* __restrict__ in, C<T>* __restrict__ out,
                                                         AxisDev ax, PassGeom g, int accumulate, int lgG,
                                                         const C<T>* __restrict__ TA, const C<T>* __restrict__ HT) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int M = ax.M;
    const int G = 1 << lgG;
    C<T>* Red = (C<T>*)smem;                    // [kEhWaves][P][kWave] partial sums
    C<T>* TAs = Red + kEhWaves * P * kWave;     // [q - qb][i] premultiply values of every term
    const int tid = (int)threadIdx.x;
    const int w = tid / kWave;
    const int lane = tid % kWave;
    const int l = lane >> lgG;
    const int n2 = lane & (G - 1);
    for (int e = tid; e < g.qn * P; e += kEhWaves * kWave)
        TAs[e] = TA[(int64_t)(g.qb + e / P) * M + ((e % P) << lgG)];
    __syncthreads();
    // XCD-contiguous tile order (as in k_EAS): neighbouring strided tiles meet in one L2
    const int64_t ntl = g.Qin * g.ntiles;  // < 2^31 (host check)
    const int64_t T8 = (ntl + 7) / 8;
    for (int64_t bid = blockIdx.x; bid < 8 * T8; bid += gridDim.x) {
        const int64_t tile = (bid & 7) * T8 + (bid >> 3);
        if (tile >= ntl) continue;  // uniform over the workgroup
        const int64_t qo = (int64_t)((unsigned)tile / (unsigned)g.ntiles);
        const int64_t tt = tile - qo * g.ntiles;
        const Tile tl = decode_tile(g, tt);
        const bool live = l < tl.nl;
        C<T> acc[P];
#pragma unroll
        for (int i = 0; i < P; ++i) acc[i] = mk<T>(0, 0);
        if (live) {
            for (int qq = w; qq < g.qn; qq += kEhWaves) {
                const int q = g.qb + qq;
                const int64_t si = qo * g.qn + qq;
                const C<T>* h = HT + (int64_t)q * M + n2;
                C<T> y[P], hv[P];
#pragma unroll
                for (int u = 0; u < P; ++u) {
                    const int64_t off = (g.S == 1) ? ((si * g.A + tl.a0 + l) * P + u)
                                                   : (((si * g.A + tl.a0) * P + u) * g.S + tl.s0 + l);
                    y[u] = in[off];
                    hv[u] = h[u << lgG];
                }
                RegDFT<T, P, false>::run(y);
#pragma unroll
                for (int r = 0; r < P; ++r) y[r] = cmulc<T>(y[r], hv[r]);
                RegDFT<T, P, true>::run(y);
                const C<T>* ta = TAs + qq * P;
#pragma unroll
                for (int i = 0; i < P; ++i) acc[i] = cfmac<T>(acc[i], y[i], ta[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < P; ++i) Red[(w * P + i) * kWave + lane] = acc[i];
        __syncthreads();
        // the kWave P outputs of the tile, (i, lane) pairs spread over the workgroup
        for (int o = tid; o < P * kWave; o += kEhWaves * kWave) {
            const int i = o / kWave;
            const int ln = o % kWave;
            const int ll = ln >> lgG;
            if (ll < tl.nl) {
                C<T> v = Red[i * kWave + ln];
#pragma unroll
                for (int ww = 1; ww < kEhWaves; ++ww) v = cadd<T>(v, Red[(ww * P + i) * kWave + ln]);
                const int n = (i << lgG) + (ln & (G - 1));
                const int64_t off = (g.S == 1) ? ((qo * g.A + tl.a0 + ll) * M + n)
                                               : (((qo * g.A + tl.a0) * M + n) * g.S + tl.s0 + ll);
                if (accumulate) v = cadd<T>(v, out[off]);
                out[off] = v;
            }
        }
        __syncthreads();  // the next tile overwrites the partial sums
    }
}

int cu_count() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cached = v;
        else
            cached = 256;
    }
    return cached;
}

hipError_t prep_lds(const void* k, size_t lds) {
    static std::mutex mu;
    static std::set<const void*> done;
    std::lock_guard<std::mutex> lk(mu);
    if (lds > 65536 && !done.count(k)) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        done.insert(k);
    }
    return hipSuccess;
}

int ilog2i(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

template <typename T, int P>
hipError_t launch_er(const void* in, void* out, const AxisDev& ax, const PassGeom& g, hipStream_t st) {
    // tile buffer (strided lines only; its size is fixed by the kernel's layout) + the chunk's TA values
    const size_t lds = cfp_lds_bytes(sizeof(T) == 8, ax.M, ax.g) +
                       ((size_t)g.qc * P + (size_t)kErStage * (ax.M + ax.g)) * sizeof(C<T>);
    // power-of-two P with at least P lanes per line: reduce first, inverse transform across lanes
    constexpr bool pow2 = kPow2<P>;
    auto k = (pow2 && ax.g >= P) ? k_ER<T, P, pow2> : k_ER<T, P, false>;
    hipError_t e = prep_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    const int nqc = (g.qn + g.qc - 1) / g.qc;
    int64_t blocks = ((g.Qin * g.ntiles + 7) / 8) * 8 * nqc;  // the kernel's XCD-aware order
    if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = (g.max_blocks + 7) / 8 * 8;
    if (blocks > (1 << 22)) blocks = 1 << 22;
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kThreads), lds, st, (const C<T>*)in,
                       (C<T>*)out, ax, g, ilog2i(ax.g), (const C<T>*)ax.TA, (const C<T>*)ax.HTl);
    return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_ear(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, void* rho,
                      hipStream_t st) {
    const size_t lds = cfp_lds_bytes(sizeof(T) == 8, ax.M, ax.g) + (size_t)g.qn * P * sizeof(C<T>);
    auto k = k_EAR<T, P>;
    hipError_t e = prep_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    int64_t blocks = g.Qin * g.ntiles;
    if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = g.max_blocks;
    if (blocks > (1 << 22)) blocks = 1 << 22;
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kThreads), lds, st, (const C<T>*)in,
                       (C<T>*)out, ax, g, accumulate, (T*)rho, ilog2i(ax.g), (const C<T>*)ax.TA,
                       (const C<T>*)ax.Tf, (const C<T>*)ax.HTl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_er_T(Kind kind, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                       void* rho, hipStream_t st) {
    if (kind == Kind::EA) {
        switch (ax.P) {
            case 1: return launch_ear<T, 1>(in, out, ax, g, accumulate, rho, st);
            case 2: return launch_ear<T, 2>(in, out, ax, g, accumulate, rho, st);
            case 4: return launch_ear<T, 4>(in, out, ax, g, accumulate, rho, st);
            case 8: return launch_ear<T, 8>(in, out, ax, g, accumulate, rho, st);
            case 16: return launch_ear<T, 16>(in, out, ax, g, accumulate, rho, st);
            case 3: return launch_ear<T, 3>(in, out, ax, g, accumulate, rho, st);
            case 6: return launch_ear<T, 6>(in, out, ax, g, accumulate, rho, st);
            case 12: return launch_ear<T, 12>(in, out, ax, g, accumulate, rho, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (ax.P) {
        case 1: return launch_er<T, 1>(in, out, ax, g, st);
        case 2: return launch_er<T, 2>(in, out, ax, g, st);
        case 4: return launch_er<T, 4>(in, out, ax, g, st);
        case 8: return launch_er<T, 8>(in, out, ax, g, st);
        case 16: return launch_er<T, 16>(in, out, ax, g, st);
        case 3: return launch_er<T, 3>(in, out, ax, g, st);
        case 6: return launch_er<T, 6>(in, out, ax, g, st);
        case 12: return launch_er<T, 12>(in, out, ax, g, st);
        default: return hipErrorInvalidValue;
    }
}

// Workgroup size of the accumulate kernels: one wavefront per workgroup when the launch is
// small, so that the work spreads over every CU (these passes are latency bound).
int acc_block(int64_t nthreads) { return nthreads < (int64_t)kThreads * 1024 ? 64 : kThreads; }

template <typename T, int G>
hipError_t launch_asr(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, void* rho,
                      hipStream_t st) {
    const int64_t ngroups = g.Qin * g.A * (int64_t)ax.P * g.S;
    const int bs = acc_block(ngroups);
    int64_t blocks = (ngroups + bs - 1) / bs;
    if (blocks > (1 << 20)) blocks = 1 << 20;
    hipLaunchKernelGGL((k_ASR<T, G>), dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(bs), 0, st,
                       (const C<T>*)in, (C<T>*)out, ax, g, accumulate, (T*)rho);
    return hipGetLastError();
}

template <typename T, int K, int R = 8>
hipError_t launch_ask(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, void* rho,
                      hipStream_t st) {
    const int64_t nthreads = g.Qin * g.A * (int64_t)ax.P * g.S * K;
    const int bs = acc_block(nthreads);
    int64_t blocks = (nthreads + bs - 1) / bs;
    if (blocks > (1 << 20)) blocks = 1 << 20;
    hipLaunchKernelGGL((k_ASK<T, K, R>), dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(bs), 0, st,
                       (const C<T>*)in, (C<T>*)out, ax, g, accumulate, (T*)rho);
    return hipGetLastError();
}

// Residues per lane of the lane-group accumulate: 4 (twice the lanes of 8 for the same g, more
// wavefronts for these latency-bound passes; C2 A passes 8.2 -> 7.6 us), FX_ASK_R=8 for 8.
int ask_residues() {
    static const int r = [] {
        const char* e = std::getenv("FX_ASK_R");
        return (e && std::atoi(e) == 8) ? 8 : 4;
    }();
    return r;
}

template <typename T, int G>
hipError_t launch_ahr(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                      hipStream_t st) {
    const int64_t ngroups = g.Qin * g.A * (int64_t)ax.P * g.S;
    const int bs = acc_block(ngroups);
    int64_t blocks = (ngroups + bs - 1) / bs;
    if (blocks > (1 << 20)) blocks = 1 << 20;
    hipLaunchKernelGGL((k_AHR<T, G>), dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(bs), 0, st,
                       (const C<T>*)in, (C<T>*)out, ax, g, accumulate);
    return hipGetLastError();
}

template <typename T, int K, int R>
hipError_t launch_ahk(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                      hipStream_t st) {
    const int64_t nthreads = g.Qin * g.A * (int64_t)ax.P * g.S * K;
    const int bs = acc_block(nthreads);
    int64_t blocks = (nthreads + bs - 1) / bs;
    if (blocks > (1 << 20)) blocks = 1 << 20;
    hipLaunchKernelGGL((k_AHK<T, K, R>), dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(bs), 0, st,
                       (const C<T>*)in, (C<T>*)out, ax, g, accumulate);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ahr_T(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                        hipStream_t st) {
    switch (ax.g) {
        case 64:
            return ask_residues() == 4 ? launch_ahk<T, 16, 4>(in, out, ax, g, accumulate, st)
                                       : launch_ahk<T, 8, 8>(in, out, ax, g, accumulate, st);
        case 1: return launch_ahr<T, 1>(in, out, ax, g, accumulate, st);
        case 2: return launch_ahr<T, 2>(in, out, ax, g, accumulate, st);
        case 4: return launch_ahr<T, 4>(in, out, ax, g, accumulate, st);
        case 8: return launch_ahr<T, 8>(in, out, ax, g, accumulate, st);
        case 16:
            return ask_residues() == 4 ? launch_ahk<T, 4, 4>(in, out, ax, g, accumulate, st)
                                       : launch_ahk<T, 2, 8>(in, out, ax, g, accumulate, st);
        case 32:
            return ask_residues() == 4 ? launch_ahk<T, 8, 4>(in, out, ax, g, accumulate, st)
                                       : launch_ahk<T, 4, 8>(in, out, ax, g, accumulate, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_asr_T(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, void* rho,
                        hipStream_t st) {
    switch (ax.g) {
        case 64:
            return ask_residues() == 4 ? launch_ask<T, 16, 4>(in, out, ax, g, accumulate, rho, st)
                                       : launch_ask<T, 8>(in, out, ax, g, accumulate, rho, st);
        case 1: return launch_asr<T, 1>(in, out, ax, g, accumulate, rho, st);
        case 2: return launch_asr<T, 2>(in, out, ax, g, accumulate, rho, st);
        case 4: return launch_asr<T, 4>(in, out, ax, g, accumulate, rho, st);
        case 8: return launch_asr<T, 8>(in, out, ax, g, accumulate, rho, st);
        case 16:
            return ask_residues() == 4 ? launch_ask<T, 4, 4>(in, out, ax, g, accumulate, rho, st)
                                       : launch_ask<T, 2>(in, out, ax, g, accumulate, rho, st);
        case 32:
            return ask_residues() == 4 ? launch_ask<T, 8, 4>(in, out, ax, g, accumulate, rho, st)
                                       : launch_ask<T, 4>(in, out, ax, g, accumulate, rho, st);
        default: return hipErrorInvalidValue;
    }
}

// EA with the structured accumulate for g = 8, one wavefront per tile of 8 lines (P = M / 8 in
// {2, 3, 4, 6, 8}). Each wave works alone on its tile and runs every term of the pass: lane
// (l, n2) keeps its P inputs x[8 i + n2] in registers, forms E_q for each term q as the register E
// kernel does and, as lane u = n2 < P holding E_q[u], adds Tf_q[n0] E_q[u] into the partial sum
// H[j], j = (q - qb) mod 8, of its output group n0 (r(n0) = u). The terms run j by j (q = qb + j,
// qb + j + 8, ...), so the running sum is one register and each finished H[j] goes to its slot (a
// register array in FP64, LDS in FP32) once per j. After the last term the lane applies the 8-point
// inverse transform of the structured accumulate (presf):
//   out[n0 + P c] = exp(2 pi i qb c / 8) sum_j exp(2 pi i j c / 8) H[j],   c < 8,
// and writes its 8 outputs. The sum over the 8 lanes of a line and the P-point inverse are, for a
// power-of-two P, a reduce-scatter (the rotated, select-free one when the rows are staged and
// P >= 4) and the cross-lane inverse of the register E kernel, whose final per-lane rescale is
// applied once to the H[j] instead of to every term; for P = 6 one select-free step over the lane
// pair, the other two lane bits summed in full, and a 6-term inverse for the lane's output; for
// P = 3 every lane applies the P-point inverse to its own HT-weighted values, pads them to 8 and
// the lanes' results are added by the select form of the reduce-scatter (lane n2 ends with value
// bitrev3(n2)). There is no workgroup barrier after the table rows of the pass (TA, HT, Tf) are
// staged in LDS, once per workgroup of a persistent grid.
constexpr int kEwWaves = 8;
constexpr size_t kEwStageBytes = 65536;  // HT rows of the pass staged when they fit

// FP32: at most 128 registers, so that the two resident workgroups of 8 waves (4 per SIMD) fit
template <typename T, int P, bool HST>
__global__ __launch_bounds__(kEwWaves * kWave) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
void k_EAW(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax, PassGeom g, int accumulate,
           T* __restrict__ rho, const C<T>* __restrict__ TA, const C<T>* __restrict__ HT) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int G = 8;
    constexpr int M = G * P;
    constexpr bool P2 = kPow2<P>;
    constexpr int LP = (P >= 8) ? 3 : (P >= 4) ? 2 : (P >= 2) ? 1 : 0;
    const int qn = g.qn;
    C<T>* TAs = (C<T>*)smem;         // [q - qb][i] = TA_q[8 i]
    C<T>* Tfs = TAs + qn * P;        // [q - qb][n0] = Tf_q[n0]
    C<T>* Hst = Tfs + qn * P;        // [q - qb][r][n2] (HST)
    // FP32: the eight accumulators of a tile wait in LDS, [wave][j][lane], not in registers, which
    // keeps the paired term loop within the registers of four waves per SIMD
    constexpr bool HJL = sizeof(T) == 4;
    C<T>* Hjs = Hst + (HST ? qn * M : 0);
    const int tid = (int)threadIdx.x;
    const int w = tid / kWave;
    const int lane = tid % kWave;
    const int l = lane / G;
    const int n2 = lane % G;
    const C<T>* Tf = (const C<T>*)ax.Tf;
    for (int e = tid; e < qn * P; e += kEwWaves * kWave) {
        const int qq = e / P, i = e % P;
        TAs[e] = TA[(int64_t)(g.qb + qq) * M + G * i];
        Tfs[e] = Tf[(int64_t)(g.qb + qq) * M + i];
    }
    // power-of-two P >= 4 with the rows staged: the lanes' spectra are shifted by bitrev(n2 mod P)
    // and summed by the select-free reduce_scatter_rot
    constexpr bool ROT = kPow2<P> && HST && P >= 4;
    if constexpr (HST) {
        // P = 6: the odd lanes' rows rotated by 3 (see below); ROT: lane m2's row turned by the
        // rest s'(m2) of its shift (HT comes with the odd rows turned by P / 2)
        const C<T>* hsrc = HT + (int64_t)g.qb * M;
        for (int e = tid; e < qn * M; e += kEwWaves * kWave) {
            int src = e;
            if constexpr (P == 6) {
                const int qq = e / M, rem = e - qq * M, r = rem / G, m2 = rem - r * G;
                src = qq * M + ((r + 3 * (m2 & 1)) % 6) * G + m2;
            } else if constexpr (ROT) {
                const int qq = e / M, rem = e - qq * M, r = rem / G, m2 = rem - r * G;
                src = qq * M + ((r + rot_shift_rest<P>(m2)) & (P - 1)) * G + m2;
            }
            Hst[e] = hsrc[src];
        }
    }
    __syncthreads();
    // lane constants: the cross-lane inverse (power-of-two P), the lane's output group, the
    // exp(2 pi i qb c / 8) of the final transform
    // P = 6: the odd lane's input times (-1)^i moves its spectrum by 3, and it reads its table row
    // rotated by 3 to match, so both lanes of the first reduce step keep values 0..2
    constexpr bool SIX = (P == 6);
    const bool odd_flip = !ROT && (P2 || SIX) && (n2 & 1);
    int raddr[LP > 2 ? LP - 2 : 1];
    if constexpr (ROT) rot_addrs<P>(raddr, lane, n2);
    const int rsh = ROT ? rot_shift<P>(n2) : 0;  // the lane's spectral shift s(n2)
    C<T> wst[LP > 0 ? LP : 1];
    C<T> fin = mk<T>(1, 0);
    if constexpr (P2) fin = lane_twiddles_x<T, LP>(wst, n2, (const C<T>*)ax.tw, M);
    // the value u of E_q the lane holds: n2 mod P after the cross-lane inverse (power-of-two P);
    // n2 for P = 6 (valid below 6); after the padded reduce-scatter (P = 3), bitrev3(n2), valid below P
    const int br = ((n2 & 1) << 2) | (n2 & 2) | ((n2 >> 2) & 1);
    const int u = P2 ? n2 % P : SIX ? (n2 < P ? n2 : 0) : (br < P ? br : 0);
    const bool holds = P2 ? n2 < P : SIX ? n2 < P : br < P;
    const int n0u = (int)((u * ax.lg_inv) % P);
    const C<T>* tw = (const C<T>*)ax.tw;  // exp(-2 pi i k / M); k = P m gives exp(-2 pi i m / 8)
    // table row offsets of the lane (P = 6 without staged rows: the odd lanes' rows rotated by 3)
    int hoff[P];
#pragma unroll
    for (int r = 0; r < P; ++r) hoff[r] = ((SIX && !HST) ? (r + 3 * (n2 & 1)) % 6 : r) * G;
    // P = 6: with the summed values W[3 b0 + j] in the lane and W[3 (1 - b0) + j] in its partner,
    // E[u] = sum_j exp(2 pi i j u / 6) (W[j] + (-1)^u W[j + 3]); the lane's factors: s_own on its own
    // value, s_par on its partner's, c_j = exp(2 pi i j u / 6) = conj(tw[8 j u mod M]) for j = 1, 2
    T s_own = 1, s_par = 1;
    C<T> c6[2];
    if constexpr (SIX) {
        const T sg = (u & 1) ? (T)-1 : (T)1;
        s_own = (n2 & 1) ? sg : (T)1;
        s_par = (n2 & 1) ? (T)1 : sg;
#pragma unroll
        for (int j = 1; j < 3; ++j) {
            const C<T> c = tw[((j * u) % 6) * (M / 6)];
            c6[j - 1] = mk<T>(c.x, -c.y);
        }
    }
    const int qbr = g.qb % G;
    // tiles: each wave is a worker; the waves of a workgroup take consecutive tiles and every XCD
    // (workgroup id mod 8) a contiguous range, so neighbouring strided tiles share one L2
    const int64_t ntl = g.Qin * g.ntiles;  // < 2^31 (host check)
    const int64_t units = (ntl + kEwWaves - 1) / kEwWaves;
    const int64_t U8 = (units + 7) / 8;
    for (int64_t bid = blockIdx.x; bid < 8 * U8; bid += gridDim.x) {
        const int64_t unit = (bid & 7) * U8 + (bid >> 3);
        const int64_t tile = unit * kEwWaves + w;
        if (unit >= units || tile >= ntl) continue;  // uniform over the wave
        const int64_t qi = (int64_t)((unsigned)tile / (unsigned)g.ntiles);
        const int64_t tt = tile - qi * g.ntiles;
        const Tile tl = decode_tile(g, tt);
        const bool live = l < tl.nl;
        C<T> x[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int n = G * i + n2;
            const int64_t off = (g.S == 1) ? ((qi * g.A + tl.a0 + l) * M + n)
                                           : (((qi * g.A + tl.a0) * M + n) * g.S + tl.s0 + l);
            x[i] = live ? in[off] : mk<T>(0, 0);
        }
        if (odd_flip) {
#pragma unroll
            for (int i = 1; i < P; i += 2) x[i] = mk<T>(-x[i].x, -x[i].y);
        }
        if constexpr (ROT) {
            // x[i] exp(-2 pi i s i / P) moves the lane's spectrum by s: position p holds index p + s
#pragma unroll
            for (int i = 1; i < P; ++i) x[i] = cmul<T>(x[i], tw[((rsh * i) & (P - 1)) * G]);
        }
        C<T> hj[HJL ? 1 : G];
        if constexpr (!HJL) {
#pragma unroll
            for (int j = 0; j < G; ++j) hj[j] = mk<T>(0, 0);
        }
        // FP32: the chains of slots j and j + 1 run together, two terms (q, q + 1) per iteration, so
        // their sequences of cross-lane steps are independent and interleave; FP64 keeps one term
        // per iteration, as two would not fit the registers of four waves per SIMD
        constexpr bool PAIR = sizeof(T) == 4;
        constexpr int JS = PAIR ? 2 : 1;
#pragma unroll 1
        for (int j = 0; j < G; j += JS) {
            C<T> acca = mk<T>(0, 0), accb = mk<T>(0, 0);
            for (int qq = j; qq < qn; qq += G) {
                const bool two = PAIR && qq + 1 < qn;
                const int qb2 = two ? qq + 1 : qq;
                C<T> va[P], vb[P];
                const C<T>* ta = TAs + qq * P;
                const C<T>* tb2 = TAs + qb2 * P;
                const C<T>* ha = (HST ? Hst + qq * M : HT + (int64_t)(g.qb + qq) * M) + n2;
                const C<T>* hb = (HST ? Hst + qb2 * M : HT + (int64_t)(g.qb + qb2) * M) + n2;
#pragma unroll
                for (int i = 0; i < P; ++i) va[i] = cmul<T>(x[i], ta[i]);
                RegDFT<T, P, false>::run(va);
#pragma unroll
                for (int r = 0; r < P; ++r) va[r] = cmul<T>(va[r], ha[hoff[r]]);
                if constexpr (PAIR) {
#pragma unroll
                    for (int i = 0; i < P; ++i) vb[i] = cmul<T>(x[i], tb2[i]);
                    RegDFT<T, P, false>::run(vb);
#pragma unroll
                    for (int r = 0; r < P; ++r) vb[r] = cmul<T>(vb[r], hb[hoff[r]]);
                }
                C<T> sa, sb = mk<T>(0, 0);
                if constexpr (SIX) {
                    // sum over the 8 lanes: one select-free step (values 0..2 kept), then the other
                    // two lane bits in full; then the 6-term inverse of the lane's output u
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        va[j] = cadd<T>(va[j], shfl_xor_c<T>(va[j + 3], 1));
                        if constexpr (PAIR) vb[j] = cadd<T>(vb[j], shfl_xor_c<T>(vb[j + 3], 1));
                    }
#pragma unroll
                    for (int s2 = 1; s2 < 3; ++s2) {
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            va[j] = cadd<T>(va[j], shfl_xor_c<T>(va[j], 1 << s2));
                            if constexpr (PAIR) vb[j] = cadd<T>(vb[j], shfl_xor_c<T>(vb[j], 1 << s2));
                        }
                    }
                    C<T> aa[3], ab[3];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const C<T> pa = shfl_xor_c<T>(va[j], 1);
                        aa[j] = mk<T>(s_own * va[j].x + s_par * pa.x, s_own * va[j].y + s_par * pa.y);
                        if constexpr (PAIR) {
                            const C<T> pb = shfl_xor_c<T>(vb[j], 1);
                            ab[j] = mk<T>(s_own * vb[j].x + s_par * pb.x, s_own * vb[j].y + s_par * pb.y);
                        }
                    }
                    sa = cfma<T>(cfma<T>(aa[0], c6[0], aa[1]), c6[1], aa[2]);
                    if constexpr (PAIR) sb = cfma<T>(cfma<T>(ab[0], c6[0], ab[1]), c6[1], ab[2]);
                } else if constexpr (P2) {
                    if constexpr (ROT) reduce_scatter_rot<T, P>(va, raddr);
                    else reduce_scatter_x<T, P>(va, n2, 3);
                    sa = va[0];
#pragma unroll
                    for (int s = LP; s < 3; ++s) sa = cadd<T>(sa, shfl_xor_c<T>(sa, 1 << s));
                    // lane n2 now holds E_q[n2 mod P] / fin; fin is applied to the accumulators
                    sa = lane_idft_nofin<T, LP>(sa, wst);
                    if constexpr (PAIR) {
                        if constexpr (ROT) reduce_scatter_rot<T, P>(vb, raddr);
                        else reduce_scatter_x<T, P>(vb, n2, 3);
                        sb = vb[0];
#pragma unroll
                        for (int s = LP; s < 3; ++s) sb = cadd<T>(sb, shfl_xor_c<T>(sb, 1 << s));
                        sb = lane_idft_nofin<T, LP>(sb, wst);
                    }
                } else {
                    // the P values padded to 8 and summed over the 8 lanes by the select form of the
                    // reduce-scatter: lane n2 ends with the sum of value bitrev3(n2)
                    RegDFT<T, P, true>::run(va);
                    C<T> wa[G];
#pragma unroll
                    for (int k = 0; k < G; ++k) wa[k] = k < P ? va[k] : mk<T>(0, 0);
                    reduce_step<T, G, 0>(wa, n2, 3);
                    sa = wa[0];
                    if constexpr (PAIR) {
                        RegDFT<T, P, true>::run(vb);
                        C<T> wb[G];
#pragma unroll
                        for (int k = 0; k < G; ++k) wb[k] = k < P ? vb[k] : mk<T>(0, 0);
                        reduce_step<T, G, 0>(wb, n2, 3);
                        sb = wb[0];
                    }
                }
                acca = cfma<T>(acca, Tfs[qq * P + n0u], sa);
                if (two) accb = cfma<T>(accb, Tfs[qb2 * P + n0u], sb);
            }
            if constexpr (HJL) {
                Hjs[(w * G + j) * kWave + lane] = acca;
                if constexpr (PAIR) Hjs[(w * G + j + 1) * kWave + lane] = accb;
            } else {
#pragma unroll
                for (int jj = 0; jj < G; jj += JS)
                    if (jj == j) {
                        hj[jj] = acca;
                        if constexpr (PAIR) hj[jj + 1] = accb;
                    }
            }
        }
        // the 8-point inverse over j of the output group (l, n0u); lanes n2 >= P hold copies
        C<T> hv[G];
#pragma unroll
        for (int j = 0; j < G; ++j) hv[j] = HJL ? Hjs[(w * G + j) * kWave + lane] : hj[HJL ? 0 : j];
        if constexpr (P2) {
            // the lane's rescale of the cross-lane inverse, once for the sums of all terms
#pragma unroll
            for (int j = 0; j < G; ++j) hv[j] = cmul<T>(hv[j], fin);
        }
        RegDFT<T, G, true>::run(hv);
        if (live && holds) {
#pragma unroll
            for (int c = 0; c < G; ++c) {
                // exp(2 pi i qb c / 8), read per tile rather than held in registers across it
                const C<T> t = tw[((qbr * c) % G) * P];
                C<T> v = cmulc<T>(hv[c], t);
                const int nb = n0u + P * c;
                const int64_t off = (g.S == 1) ? ((qi * g.A + tl.a0 + l) * M + nb)
                                               : (((qi * g.A + tl.a0) * M + nb) * g.S + tl.s0 + l);
                if (accumulate) v = cadd<T>(v, out[off]);
                out[off] = v;
                if (rho) rho[off] = v.x * v.x + v.y * v.y;
            }
        }
    }
}

template <typename T, int P>
hipError_t launch_eaw(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, void* rho,
                      hipStream_t st) {
    const size_t stage = (size_t)g.qn * ax.M * sizeof(C<T>);
    const bool hst = stage <= kEwStageBytes;
    // the pass's table rows staged in LDS once per workgroup when they fit kEwStageBytes; FP32 adds
    // the accumulators of the waves' tiles (8 per lane)
    const size_t hjl = sizeof(T) == 4 ? (size_t)kEwWaves * 8 * kWave : 0;
    const size_t lds = ((size_t)2 * g.qn * P + (hst ? (size_t)g.qn * ax.M : 0) + hjl) * sizeof(C<T>);
    const int64_t units = (g.Qin * g.ntiles + kEwWaves - 1) / kEwWaves;
    int64_t blocks = (units + 7) / 8 * 8;
    const int64_t cap = (int64_t)(2 * cu_count() + 7) / 8 * 8;  // persistent: the staged rows are reused
    if (blocks > cap) blocks = cap;
    if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = (g.max_blocks + 7) / 8 * 8;
    auto k = hst ? k_EAW<T, P, true> : k_EAW<T, P, false>;
    hipError_t e = prep_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kEwWaves * kWave), lds, st,
                       (const C<T>*)in, (C<T>*)out, ax, g, accumulate, (T*)rho, (const C<T>*)ax.TA,
                       (const C<T>*)ax.HTx);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_eaw_T(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, void* rho,
                        hipStream_t st) {
    switch (ax.P) {
        case 2: return launch_eaw<T, 2>(in, out, ax, g, accumulate, rho, st);
        case 3: return launch_eaw<T, 3>(in, out, ax, g, accumulate, rho, st);
        case 4: return launch_eaw<T, 4>(in, out, ax, g, accumulate, rho, st);
        case 6: return launch_eaw<T, 6>(in, out, ax, g, accumulate, rho, st);
        case 8: return launch_eaw<T, 8>(in, out, ax, g, accumulate, rho, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

// g <= 8: one thread per group (k_ASR); g = 16, 32, 64: K = g / 8 lanes per group (k_ASK).
bool asr_applicable(int g, int max_g) {
    return (g == 1 || g == 2 || g == 4 || g == 8 || g == 16 || g == 32 || g == 64) && g <= max_g;
}

hipError_t launch_pass_asr(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                           int accumulate, void* rho, hipStream_t st) {
    if (!asr_applicable(ax.g, 64) || (kind != Kind::A && kind != Kind::AH)) return hipErrorInvalidValue;
    if (kind == Kind::AH)
        return dbl ? launch_ahr_T<double>(in, out, ax, g, accumulate, st)
                   : launch_ahr_T<float>(in, out, ax, g, accumulate, st);
    return dbl ? launch_asr_T<double>(in, out, ax, g, accumulate, rho, st)
               : launch_asr_T<float>(in, out, ax, g, accumulate, rho, st);
}

template <typename T, int P>
hipError_t launch_ehr(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                      hipStream_t st) {
    int64_t blocks = (g.Qin * g.ntiles + 7) / 8 * 8;  // the kernel's XCD-contiguous order
    if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = (g.max_blocks + 7) / 8 * 8;
    if (blocks > (1 << 22)) blocks = 1 << 22;
    const size_t lds = ((size_t)kEhWaves * P * kWave + (size_t)g.qn * P) * sizeof(C<T>);
    hipError_t e = prep_lds((const void*)k_EHR<T, P>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_EHR<T, P>), dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kEhWaves * kWave), lds, st,
                       (const C<T>*)in, (C<T>*)out, ax, g, accumulate, ilog2i(ax.g), (const C<T>*)ax.TA,
                       (const C<T>*)ax.HT);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ehr_T(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                        hipStream_t st) {
    switch (ax.P) {
        case 1: return launch_ehr<T, 1>(in, out, ax, g, accumulate, st);
        case 2: return launch_ehr<T, 2>(in, out, ax, g, accumulate, st);
        case 4: return launch_ehr<T, 4>(in, out, ax, g, accumulate, st);
        case 8: return launch_ehr<T, 8>(in, out, ax, g, accumulate, st);
        case 16: return launch_ehr<T, 16>(in, out, ax, g, accumulate, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int P, int K>
hipError_t launch_eas(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, void* rho,
                      hipStream_t st) {
    constexpr int G = 8 * K;
    constexpr int TS = kWave / G;
    const size_t stage = (size_t)g.qn * ax.M * sizeof(C<T>);
    const bool hst = stage <= kEasStageBytes;
    int64_t blocks = (g.Qin * g.ntiles + 7) / 8 * 8;  // the kernel's XCD-contiguous order
    if (hst) blocks = std::min<int64_t>(blocks, (int64_t)(2 * cu_count() + 7) / 8 * 8);  // persistent
    if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = (g.max_blocks + 7) / 8 * 8;
    if (blocks > (1 << 22)) blocks = 1 << 22;
    const size_t lds = ((size_t)TS * ax.M + (size_t)TS * P * G + (size_t)g.qn * P) * sizeof(C<T>) + (hst ? stage : 0);
    auto k = hst ? k_EAS<T, P, K, true> : k_EAS<T, P, K, false>;
    hipError_t e = prep_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kEaWaves * kWave), lds, st,
                       (const C<T>*)in, (C<T>*)out, ax, g, accumulate, (T*)rho, ilog2i(ax.g), (const C<T>*)ax.TA,
                       (const C<T>*)ax.HTx);
    return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_eas_P(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, void* rho,
                        hipStream_t st) {
    if constexpr (sizeof(T) == 8 && P == 16) return hipErrorInvalidValue;  // excluded by eas_applicable
    else switch (ax.g) {
        case 8: if constexpr (P <= 8) return launch_eas<T, P, 1>(in, out, ax, g, accumulate, rho, st); break;
        case 16: return launch_eas<T, P, 2>(in, out, ax, g, accumulate, rho, st);
        case 32: return launch_eas<T, P, 4>(in, out, ax, g, accumulate, rho, st);
        case 64: return launch_eas<T, P, 8>(in, out, ax, g, accumulate, rho, st);
        default: break;
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_eas_T(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, void* rho,
                        hipStream_t st) {
    switch (ax.P) {
        case 1: return launch_eas_P<T, 1>(in, out, ax, g, accumulate, rho, st);
        case 2: return launch_eas_P<T, 2>(in, out, ax, g, accumulate, rho, st);
        case 4: return launch_eas_P<T, 4>(in, out, ax, g, accumulate, rho, st);
        case 8: return launch_eas_P<T, 8>(in, out, ax, g, accumulate, rho, st);
        case 16: return launch_eas_P<T, 16>(in, out, ax, g, accumulate, rho, st);
        default: return hipErrorInvalidValue;
    }
}

bool eas_applicable(bool dbl, int M, int g, int qn) {
    if (g < 8 || g > kWave || (g & (g - 1)) != 0 || M % g != 0 || qn < 1 || qn > 64) return false;
    const int P = M / g;
    if (!(P == 1 || P == 2 || P == 4 || P == 8 || P == 16) || P > g) return false;
    if (dbl && P == 16) return false;  // does not fit the registers of an eight-wave workgroup
    const size_t cs = dbl ? 16 : 8;
    const int TS = kWave / g;
    return ((size_t)TS * M + (size_t)TS * P * g + (size_t)qn * P) * cs <= (size_t)lds_limit_bytes();
}

int eas_tile_lines(int g) { return kWave / std::max(1, g); }

hipError_t launch_pass_eas(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                           void* rho, hipStream_t st) {
    if (!eas_applicable(dbl, ax.M, ax.g, g.qn) || !ax.HTx || g.TS != eas_tile_lines(ax.g)) return hipErrorInvalidValue;
    if (g.Qin * g.ntiles >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    return dbl ? launch_eas_T<double>(in, out, ax, g, accumulate, rho, st)
               : launch_eas_T<float>(in, out, ax, g, accumulate, rho, st);
}

bool eaw_applicable(bool dbl, int M, int g, int qn) {
    if (g != 8 || M % 8 != 0 || qn < 1) return false;
    const int P = M / 8;
    if (!(P == 2 || P == 3 || P == 4 || P == 6 || P == 8)) return false;
    const size_t cs = dbl ? 16 : 8;
    const size_t hjl = dbl ? 0 : (size_t)kEwWaves * 8 * kWave * cs;  // the FP32 accumulators
    return (size_t)2 * qn * P * cs + hjl <= (size_t)lds_limit_bytes();
}

int eaw_tile_lines() { return 8; }

hipError_t launch_pass_eaw(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                           void* rho, hipStream_t st) {
    if (!eaw_applicable(dbl, ax.M, ax.g, g.qn) || !ax.HTx || g.TS != eaw_tile_lines()) return hipErrorInvalidValue;
    if (g.Qin * g.ntiles >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    return dbl ? launch_eaw_T<double>(in, out, ax, g, accumulate, rho, st)
               : launch_eaw_T<float>(in, out, ax, g, accumulate, rho, st);
}

bool ehr_applicable(int M, int g) {
    if (g < 1 || g > kWave || (g & (g - 1)) != 0 || M % g != 0) return false;
    const int P = M / g;
    return (P == 1 || P == 2 || P == 4 || P == 8 || P == 16) && g >= P;
}

int ehr_tile_lines(int g) { return kWave / std::max(1, g); }

hipError_t launch_pass_ehr(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                           hipStream_t st) {
    if (!ehr_applicable(ax.M, ax.g) || !ax.HT || g.TS != ehr_tile_lines(ax.g) || g.qn > 64)
        return hipErrorInvalidValue;
    if (g.Qin * g.ntiles >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    return dbl ? launch_ehr_T<double>(in, out, ax, g, accumulate, st) : launch_ehr_T<float>(in, out, ax, g, accumulate, st);
}

bool aa_applicable(bool dbl, int gu, int gv) {
    (void)dbl;
    return gu >= 1 && gv >= 1 && gu * gv <= 1024;
}

int aa_tile_groups(int gu, int gv) { return std::max(1, 1024 / (gu * gv)); }

size_t aa_lds_bytes(bool dbl, int gu, int gv) {
    const size_t tsg = (size_t)aa_tile_groups(gu, gv);
    return (2 * tsg * gu * gv + gu + gv) * (dbl ? 16 : 8);
}

bool aar_applicable(int gu, int gv, int Pu, int Pv, const AAGeom& g) {
    return gu == gv && (gu == 16 || gu == 32) && g.Y == 1 && g.Z == 1 &&
           g.O * g.X * Pu * Pv + kThreads * 8 < (int64_t(1) << 31);
}

template <typename T, int G, int R>
static void launch_aar_r(const void* in, void* out, const AxisDev& au, const AxisDev& av, const AAGeom& g,
                         int accumulate, void* rho, hipStream_t st) {
    constexpr int WG = aar_threads(G, R);
    constexpr int NG = WG / (G * G / R);
    const int64_t ngroups = g.O * g.X * au.P * av.P;
    const int64_t ntl = (ngroups + NG - 1) / NG;
    const int64_t blocks = std::min<int64_t>(((ntl + 7) / 8) * 8, int64_t(1) << 24);
    hipLaunchKernelGGL((k_AAR<T, G, R>), dim3((unsigned)blocks), dim3(WG), 0, st, (const C<T>*)in, (C<T>*)out, au,
                       av, g, accumulate, (T*)rho);
}
template <typename T, int G>
static void launch_aar(const void* in, void* out, const AxisDev& au, const AxisDev& av, const AAGeom& g,
                       int accumulate, void* rho, hipStream_t st) {
    // two residues per lane: twice the waves of four per lane (one group per CU on the 512^2
    // workload), which hides more of the scattered loads' latency
    launch_aar_r<T, G, 2>(in, out, au, av, g, accumulate, rho, st);
}

template <typename T, int G>
static void launch_aahr(const void* in, void* out, const AxisDev& au, const AxisDev& av, const AAGeom& g,
                        int accumulate, hipStream_t st) {
    constexpr int NG = kThreads / (G * G / 4);
    const int64_t ngroups = g.O * g.X * au.P * av.P;
    const int64_t ntl = (ngroups + NG - 1) / NG;
    const int64_t blocks = std::min<int64_t>(((ntl + 7) / 8) * 8, int64_t(1) << 24);
    hipLaunchKernelGGL((k_AAHR<T, G>), dim3((unsigned)blocks), dim3(kThreads), 0, st, (const C<T>*)in, (C<T>*)out,
                       au, av, g, accumulate);
}

hipError_t launch_pass_aah(bool dbl, const void* in, void* out, const AxisDev& au, const AxisDev& av,
                           const AAGeom& g, int accumulate, hipStream_t st) {
    if (!aar_applicable(au.g, av.g, au.P, av.P, g)) return hipErrorInvalidValue;
    if (dbl) {
        if (au.g == 32) launch_aahr<double, 32>(in, out, au, av, g, accumulate, st);
        else launch_aahr<double, 16>(in, out, au, av, g, accumulate, st);
    } else {
        if (au.g == 32) launch_aahr<float, 32>(in, out, au, av, g, accumulate, st);
        else launch_aahr<float, 16>(in, out, au, av, g, accumulate, st);
    }
    return hipGetLastError();
}

hipError_t launch_pass_aa(bool dbl, const void* in, void* out, const AxisDev& au, const AxisDev& av, const AAGeom& g,
                          int accumulate, void* rho, hipStream_t st) {
    if (aar_applicable(au.g, av.g, au.P, av.P, g)) {
        if (dbl) {
            if (au.g == 32) launch_aar<double, 32>(in, out, au, av, g, accumulate, rho, st);
            else launch_aar<double, 16>(in, out, au, av, g, accumulate, rho, st);
        } else {
            if (au.g == 32) launch_aar<float, 32>(in, out, au, av, g, accumulate, rho, st);
            else launch_aar<float, 16>(in, out, au, av, g, accumulate, rho, st);
        }
        return hipGetLastError();
    }
    if (!aa_applicable(dbl, au.g, av.g) || g.tsg != aa_tile_groups(au.g, av.g)) return hipErrorInvalidValue;
    const int64_t ngroups = g.O * g.X * au.P * g.Y * av.P * g.Z;
    const int64_t tiles = (ngroups + g.tsg - 1) / g.tsg;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, 1 << 20));
    const size_t lds = aa_lds_bytes(dbl, au.g, av.g);
    if (dbl)
        hipLaunchKernelGGL(k_AA<double>, dim3(blocks), dim3(kThreads), lds, st, (const double2*)in, (double2*)out, au,
                           av, g, accumulate, (double*)rho);
    else
        hipLaunchKernelGGL(k_AA<float>, dim3(blocks), dim3(kThreads), lds, st, (const float2*)in, (float2*)out, au, av,
                           g, accumulate, (float*)rho);
    return hipGetLastError();
}

bool erg_applicable(bool dbl, int M, int g) {
    (void)dbl;
    if (!(g == 2 || g == 4 || g == 8) || M % g != 0) return false;
    const int P = M / g;
    return P == 16 || P == 32 || P == 64;
}

int erg_tile_lines(int M, int g) { return kThreads / std::max(1, g * (M / g) / 8); }

size_t erg_lds_bytes(bool dbl, Kind kind, int M, int g, int qc, int qn, bool strided) {
    const int P = M / g, L = g * P / 8, TL = kThreads / L;
    const size_t tab = (kind == Kind::EA) ? (size_t)2 * qn * P : (size_t)qc * P;
    return (tab + (size_t)kErStage * L * 9 + (strided ? (size_t)TL * (M + kTilePad) : 0)) * (dbl ? 16 : 8);
}

template <typename T, int P, int LG, bool EAF>
hipError_t launch_erg(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, void* rho,
                      hipStream_t st) {
    const size_t lds = erg_lds_bytes(sizeof(T) == 8, EAF ? Kind::EA : Kind::E, ax.M, ax.g, g.qc, g.qn, g.S != 1);
    auto k = k_ERG<T, P, LG, EAF>;
    hipError_t e = prep_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    const int nqc = EAF ? 1 : (g.qn + g.qc - 1) / g.qc;
    int64_t blocks = ((g.Qin * g.ntiles + 7) / 8) * 8 * nqc;
    if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = (g.max_blocks + 7) / 8 * 8;
    if (blocks > (1 << 22)) blocks = 1 << 22;
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kThreads), lds, st, (const C<T>*)in,
                       (C<T>*)out, ax, g, accumulate, (T*)rho, (const C<T>*)ax.TA, (const C<T>*)ax.HT);
    return hipGetLastError();
}

template <typename T, bool EAF>
hipError_t launch_erg_T(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, void* rho,
                        hipStream_t st) {
    const int key = ax.g * 100 + ax.P;
    switch (key) {
        case 216: return launch_erg<T, 16, 1, EAF>(in, out, ax, g, accumulate, rho, st);
        case 232: return launch_erg<T, 32, 1, EAF>(in, out, ax, g, accumulate, rho, st);
        case 264: return launch_erg<T, 64, 1, EAF>(in, out, ax, g, accumulate, rho, st);
        case 416: return launch_erg<T, 16, 2, EAF>(in, out, ax, g, accumulate, rho, st);
        case 432: return launch_erg<T, 32, 2, EAF>(in, out, ax, g, accumulate, rho, st);
        case 464: return launch_erg<T, 64, 2, EAF>(in, out, ax, g, accumulate, rho, st);
        case 816: return launch_erg<T, 16, 3, EAF>(in, out, ax, g, accumulate, rho, st);
        case 832: return launch_erg<T, 32, 3, EAF>(in, out, ax, g, accumulate, rho, st);
        case 864: return launch_erg<T, 64, 3, EAF>(in, out, ax, g, accumulate, rho, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass_erg(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                           int accumulate, void* rho, hipStream_t st) {
    if ((kind != Kind::E && kind != Kind::EA) || !erg_applicable(dbl, ax.M, ax.g) || !ax.HT || !ax.tw || !ax.Tf ||
        g.TS != erg_tile_lines(ax.M, ax.g) || g.qc < 1)
        return hipErrorInvalidValue;
    if ((int64_t)erg_lds_bytes(dbl, kind, ax.M, ax.g, g.qc, g.qn, g.S != 1) > lds_limit_bytes()) return hipErrorInvalidValue;
    const int nqc = kind == Kind::EA ? 1 : (g.qn + g.qc - 1) / g.qc;
    if (((g.Qin * g.ntiles + 7) / 8) * 8 * nqc >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    if (kind == Kind::EA)
        return dbl ? launch_erg_T<double, true>(in, out, ax, g, accumulate, rho, st)
                   : launch_erg_T<float, true>(in, out, ax, g, accumulate, rho, st);
    return dbl ? launch_erg_T<double, false>(in, out, ax, g, accumulate, rho, st)
               : launch_erg_T<float, false>(in, out, ax, g, accumulate, rho, st);
}

size_t ehg_lds_bytes(bool dbl, int M, int g, int qn, bool strided) {
    const int P = M / g, L = g * P / 8, TL = kThreads / L;
    return ((size_t)qn * P + (size_t)kErStage * L * 9 + (strided ? (size_t)kErStage * TL * P : 0)) * (dbl ? 16 : 8);
}

template <typename T, int P, int LG>
hipError_t launch_ehg(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, hipStream_t st) {
    const size_t lds = ehg_lds_bytes(sizeof(T) == 8, ax.M, ax.g, g.qn, g.S != 1);
    auto k = k_EHG<T, P, LG>;
    hipError_t e = prep_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    int64_t blocks = ((g.Qin * g.ntiles + 7) / 8) * 8;
    if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = (g.max_blocks + 7) / 8 * 8;
    if (blocks > (1 << 22)) blocks = 1 << 22;
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kThreads), lds, st, (const C<T>*)in,
                       (C<T>*)out, ax, g, accumulate, (const C<T>*)ax.TA, (const C<T>*)ax.HT);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ehg_T(const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate, hipStream_t st) {
    switch (ax.g * 100 + ax.P) {
        case 216: return launch_ehg<T, 16, 1>(in, out, ax, g, accumulate, st);
        case 232: return launch_ehg<T, 32, 1>(in, out, ax, g, accumulate, st);
        case 264: return launch_ehg<T, 64, 1>(in, out, ax, g, accumulate, st);
        case 416: return launch_ehg<T, 16, 2>(in, out, ax, g, accumulate, st);
        case 432: return launch_ehg<T, 32, 2>(in, out, ax, g, accumulate, st);
        case 464: return launch_ehg<T, 64, 2>(in, out, ax, g, accumulate, st);
        case 816: return launch_ehg<T, 16, 3>(in, out, ax, g, accumulate, st);
        case 832: return launch_ehg<T, 32, 3>(in, out, ax, g, accumulate, st);
        case 864: return launch_ehg<T, 64, 3>(in, out, ax, g, accumulate, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass_ehg(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g, int accumulate,
                           hipStream_t st) {
    if (!erg_applicable(dbl, ax.M, ax.g) || !ax.HT || !ax.tw || g.TS != erg_tile_lines(ax.M, ax.g)) return hipErrorInvalidValue;
    if ((int64_t)ehg_lds_bytes(dbl, ax.M, ax.g, g.qn, g.S != 1) > lds_limit_bytes()) return hipErrorInvalidValue;
    if (((g.Qin * g.ntiles + 7) / 8) * 8 >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    return dbl ? launch_ehg_T<double>(in, out, ax, g, accumulate, st) : launch_ehg_T<float>(in, out, ax, g, accumulate, st);
}

bool erw_applicable(bool dbl, int M, int g) {
    (void)dbl;
    if (g != 8 || M % 8 != 0) return false;
    const int P = M / 8;
    return P == 16 || P == 32 || P == 48 || P == 64;
}

// lanes per line of k_ERW: 8 P / V
static int erw_lanes(int P) { return (P % 3 == 0) ? 8 * (P / 6) : P; }

int erw_tile_lines(int P) { return kThreads / std::max(1, erw_lanes(P)); }

size_t erw_lds_bytes(bool dbl, int P, int qc) {
    const int V = (P % 3 == 0) ? 6 : 8;
    return ((size_t)qc * P + (size_t)kErStage * erw_lanes(P) * (V + 1)) * (dbl ? 16 : 8);
}

template <typename T, int P>
hipError_t launch_erw(const void* in, void* out, const AxisDev& ax, const PassGeom& g, hipStream_t st) {
    const size_t lds = erw_lds_bytes(sizeof(T) == 8, P, g.qc);
    auto k = k_ERW<T, P>;
    hipError_t e = prep_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    const int nqc = (g.qn + g.qc - 1) / g.qc;
    int64_t blocks = ((g.Qin * g.ntiles + 7) / 8) * 8 * nqc;
    if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = (g.max_blocks + 7) / 8 * 8;
    if (blocks > (1 << 22)) blocks = 1 << 22;
    hipLaunchKernelGGL(k, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kThreads), lds, st, (const C<T>*)in,
                       (C<T>*)out, ax, g, (const C<T>*)ax.TA, (const C<T>*)ax.HT);
    return hipGetLastError();
}

hipError_t launch_pass_erw(bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g, hipStream_t st) {
    if (!erw_applicable(dbl, ax.M, ax.g) || !ax.HT || !ax.tw || g.S != 1 || g.TS != erw_tile_lines(ax.P) || g.qc < 1)
        return hipErrorInvalidValue;
    if ((int64_t)erw_lds_bytes(dbl, ax.P, g.qc) > lds_limit_bytes()) return hipErrorInvalidValue;
    if (((g.Qin * g.ntiles + 7) / 8) * 8 * ((g.qn + g.qc - 1) / g.qc) >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    if ((g.Qin * g.A + 1) * (int64_t)ax.M >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    switch (ax.P) {
        case 16: return dbl ? launch_erw<double, 16>(in, out, ax, g, st) : launch_erw<float, 16>(in, out, ax, g, st);
        case 32: return dbl ? launch_erw<double, 32>(in, out, ax, g, st) : launch_erw<float, 32>(in, out, ax, g, st);
        case 48: return dbl ? launch_erw<double, 48>(in, out, ax, g, st) : launch_erw<float, 48>(in, out, ax, g, st);
        case 64: return dbl ? launch_erw<double, 64>(in, out, ax, g, st) : launch_erw<float, 64>(in, out, ax, g, st);
        default: return hipErrorInvalidValue;
    }
}

bool cfp_applicable(Kind kind, bool dbl, int M, int g) {
    if (kind != Kind::E && kind != Kind::EA) return false;
    if (g < 1 || g > kWave || (g & (g - 1)) != 0) return false;
    if (M % g != 0) return false;
    const int P = M / g;
    (void)dbl;
    return P == 1 || P == 2 || P == 4 || P == 8 || P == 16 || P == 3 || P == 6 || P == 12;
}

int cfp_tile_lines(int g) { return kThreads / std::max(1, g); }

size_t cfp_lds_bytes(bool dbl, int M, int g) {
    // TS rows of M + kTilePad points with TS = kThreads / g
    const size_t ts = (size_t)(kThreads / std::max(1, g));
    return ts * (size_t)(M + kTilePad) * (dbl ? 16 : 8);
}

hipError_t launch_pass_cfp(Kind kind, bool dbl, const void* in, void* out, const AxisDev& ax, const PassGeom& g,
                           int accumulate, void* rho, hipStream_t st) {
    if (!cfp_applicable(kind, dbl, ax.M, ax.g) || !ax.HTx || g.TS != cfp_tile_lines(ax.g) || g.qc < 1)
        return hipErrorInvalidValue;
    if (((g.Qin * g.ntiles + 7) / 8) * 8 * ((g.qn + g.qc - 1) / g.qc) >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    return dbl ? launch_er_T<double>(kind, in, out, ax, g, accumulate, rho, st)
               : launch_er_T<float>(kind, in, out, ax, g, accumulate, rho, st);
}

}  // namespace fx
