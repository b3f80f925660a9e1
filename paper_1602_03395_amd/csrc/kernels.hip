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

#include <algorithm>
#include <mutex>
#include <set>

#include "fx_internal.h"
#include "device_common.h"

namespace fx {

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
    const int total = (int)(g.Qin * g.qn * g.ntiles);  // < 2^31, checked on the host
    const FDiv fnt((int)g.ntiles), fqn(g.qn);
    const bool wm = g.TS >= (int)(blockDim.x >> 6);  // every wave owns at least one line of a full tile
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
        for (int e = threadIdx.x; e < nl * M; e += blockDim.x) {
            int l, n;
            const int64_t off = tile_elem(g, tl, qi, M, fdM, e, l, n);
            B0[l * M + n] = cmul<T>(in[off], TA[q * M + n]);
        }
        __syncthreads();
        C<T>* Y = lds_fft<T>(B0, B1, nl, M, ax.fm, tw, 1, false, TB + q * M, wm);
        C<T>* Z = (Y == B0) ? B1 : B0;
        if (wm) fold_lines_wave<T>(Y, Z, nl, M, P, ax.g);
        else fold_lines<T>(Y, Z, Wsc, nl, M, P, ax.g, fP);
        C<T>* Rz = lds_fft<T>(Z, Y, nl, M, ax.fp, tw, ax.g, true, nullptr, wm);
        if (wm) __syncthreads();
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
// AS: the same sum as A, organised by the n'' sample. The g output points nb = n0 + P c
// (c < g) read the same input value for every q, and Tf[q][n0 + P c] equals
// Tf[q][n0] exp(2 pi i q c / g) exactly (the twiddle (presf) advances by q/g cycles per step
// P), so
//   out[n0 + P c] = sum_{q' < g} exp(2 pi i q' c / g) H[q'],
//   H[q'] = sum_{q = q' mod g} Tf[q][n0] in_q[r(n0)],
// i.e. one pass over the inputs and a g-point inverse transform per (n0, s) group.
// Groups are numbered row-major over (qo, a, n0, s); a tile holds TSL groups.
// ------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_AS(const C<T>* __restrict__ in, C<T>* __restrict__ out, AxisDev ax,
                                                 PassGeom g, int accumulate, T* __restrict__ rho, int TSL) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int M = ax.M, P = ax.P, G = ax.g;
    const int S = (int)g.S;
    const int PS = P * S;
    C<T>* H0 = (C<T>*)smem;
    C<T>* H1 = H0 + TSL * G;
    C<T>* tw = H1 + TSL * G;  // exp(-2 pi i k / g), k < g
    const C<T>* twg = (const C<T>*)ax.tw;
    for (int i = threadIdx.x; i < G; i += blockDim.x) tw[i] = twg[(int64_t)i * P];
    __syncthreads();
    const C<T>* Tf = (const C<T>*)ax.Tf;
    const int ngroups = (int)(g.Qin * g.A * PS);  // < 2^31, checked on the host
    const int ntile = (ngroups + TSL - 1) / TSL;
    const FDiv fPS(PS), fS(S), fP(P), fA((int)g.A), fG(G);
    const int64_t step = g.A * (int64_t)PS;  // one magnification slice of the input
    const int q0r = fG.mod(g.qb);
    for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
        const int base = t * TSL;
        const int nt = min(TSL, ngroups - base);
        // work items (residue qr, group p): consecutive threads take consecutive groups
        const FDiv fnt(nt);
        // two work items per thread and step, their loads issued together
        for (int it0 = threadIdx.x; it0 < nt * G; it0 += 2 * blockDim.x) {
            const C<T>* src[2];
            const C<T>* tf[2];
            int i0[2], slot[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int it = it0 + h * (int)blockDim.x;
                slot[h] = -1;
                i0[h] = g.qn;  // no terms
                src[h] = in;
                tf[h] = Tf;
                if (it < nt * G) {
                    const int qr = fnt.div(it);
                    const int p = it - qr * nt;
                    const int gi = base + p;
                    const int row = fPS.div(gi);
                    const int rem = gi - row * PS;
                    const int n0 = fS.div(rem);
                    const int s = rem - n0 * S;
                    const int qo = fA.div(row);
                    const int a = row - qo * (int)g.A;
                    const int r = fP.mod(n0 * ax.lg);
                    src[h] = in + (((int64_t)qo * g.qn) * g.A + a) * (int64_t)PS + r * S + s;
                    tf[h] = Tf + g.qb * M + n0;
                    int f = qr - q0r;  // first i with (qb + i) mod G == qr
                    if (f < 0) f += G;
                    i0[h] = f;
                    slot[h] = p * G + qr;
                }
            }
            C<T> acc0 = mk<T>(0, 0), acc1 = mk<T>(0, 0);
            for (int d = 0; i0[0] + d < g.qn || i0[1] + d < g.qn; d += G) {
                const int ia = i0[0] + d, ib = i0[1] + d;
                if (ia < g.qn) acc0 = cfma<T>(acc0, tf[0][ia * M], src[0][ia * step]);
                if (ib < g.qn) acc1 = cfma<T>(acc1, tf[1][ib * M], src[1][ib * step]);
            }
            if (slot[0] >= 0) H0[slot[0]] = acc0;
            if (slot[1] >= 0) H0[slot[1]] = acc1;
        }
        for (int p = nt + threadIdx.x; p < TSL; p += blockDim.x)
            for (int qr = 0; qr < G; ++qr) H0[p * G + qr] = mk<T>(0, 0);
        __syncthreads();
        C<T>* R = lds_fft<T>(H0, H1, TSL, G, ax.fg, tw, 1, true);
        for (int e = threadIdx.x; e < nt * G; e += blockDim.x) {
            const int c = fnt.div(e);
            const int p = e - c * nt;
            const int gi = base + p;
            const int row = fPS.div(gi);
            const int rem = gi - row * PS;
            const int n0 = fS.div(rem);
            const int s = rem - n0 * S;
            const int64_t o = ((int64_t)row * M + n0 + P * c) * S + s;
            C<T> v = R[p * G + c];
            if (accumulate) v = cadd<T>(v, out[o]);
            out[o] = v;
            if (rho) rho[o] = v.x * v.x + v.y * v.y;
        }
        __syncthreads();
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
    const int total = (int)(g.Qin * g.ntiles);  // < 2^31, checked on the host
    const FDiv fnt((int)g.ntiles);
    const bool wm = g.TS >= (int)(blockDim.x >> 6);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    for (int bid = blockIdx.x; bid < total; bid += gridDim.x) {
        const int qi32 = fnt.div(bid);
        const int tt = bid - qi32 * (int)g.ntiles;
        const int64_t qi = qi32;
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
            if (wm) {
                for (int l = wv; l < nl; l += nwv)
                    for (int n = lane; n < M; n += 64) B0[l * M + n] = cmul<T>(RAW[l * M + n], TA[q * M + n]);
                wave_sync();
            } else {
                for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
                    const int n = fM.mod(e);
                    B0[e] = cmul<T>(RAW[e], TA[q * M + n]);
                }
                __syncthreads();
            }
            C<T>* Y = lds_fft<T>(B0, B1, nl, M, ax.fm, tw, 1, false, TB + q * M, wm);
            C<T>* Z = (Y == B0) ? B1 : B0;
            if (wm) fold_lines_wave<T>(Y, Z, nl, M, P, ax.g);
            else fold_lines<T>(Y, Z, Wsc, nl, M, P, ax.g, fP);
            C<T>* Rz = lds_fft<T>(Z, Y, nl, M, ax.fp, tw, ax.g, true, nullptr, wm);
            if (wm) __syncthreads();
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
            // four elements per thread and step, their loads issued before the stores
            for (int e0 = threadIdx.x; e0 < nl * P; e0 += 4 * blockDim.x) {
                C<T> v[4];
                int d[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int e = e0 + k * (int)blockDim.x;
                    d[k] = -1;
                    if (e < nl * P) {
                        int l, u;
                        const int64_t off = tile_elem(g, tl, si, P, fdP, e, l, u);
                        v[k] = in[off];
                        d[k] = l * M + u;
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (d[k] >= 0) B0[d[k]] = v[k];
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
            if (ax.g >= 4 && g.Qin * g.A * (int64_t)ax.P * g.S < (int64_t(1) << 31)) {
                const int TSL = as_tile_groups(ax.g);
                const size_t lds = as_lds_bytes(sizeof(T) == 8, ax.g, ax.M);
                auto k = k_AS<T>;
                hipError_t err = prep_lds(k, lds);
                if (err != hipSuccess) return err;
                const int64_t ngroups = g.Qin * g.A * (int64_t)ax.P * g.S;
                int64_t blocks = (ngroups + TSL - 1) / TSL;
                if (g.max_blocks > 0 && blocks > g.max_blocks) blocks = g.max_blocks;
                blocks = std::min<int64_t>(std::max<int64_t>(blocks, 1), 1 << 22);
                hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kThreads), lds, st, (const C<T>*)in, (C<T>*)out,
                                   ax, g, accumulate, (T*)rho, TSL);
                return hipGetLastError();
            }
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

int as_tile_groups(int g) { return std::max(1, 512 / std::max(1, g)); }

size_t as_lds_bytes(bool dbl, int g, int M) {
    const size_t c = dbl ? 16 : 8;
    return (2 * (size_t)as_tile_groups(g) * g + (size_t)M) * c;
}

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
    // tile kernels index their tiles with 32-bit integers (the count includes the padding of the
    // XCD-aware order of the register E kernel)
    if (((g.Qin * g.ntiles + 7) / 8) * 8 * g.qn >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    if (kind == Kind::E && g.erw) return launch_pass_erw(dbl, in, out, ax, g, st);
    if ((kind == Kind::E || kind == Kind::EA) && g.erg) return launch_pass_erg(kind, dbl, in, out, ax, g, accumulate, rho, st);
    if (kind == Kind::EH && g.erg) return launch_pass_ehg(dbl, in, out, ax, g, accumulate, st);
    if (kind == Kind::EA && g.eaw) return launch_pass_eaw(dbl, in, out, ax, g, accumulate, rho, st);
    if (kind == Kind::EA && g.eas) return launch_pass_eas(dbl, in, out, ax, g, accumulate, rho, st);
    if (g.qc > 0 && kind == Kind::EH) return launch_pass_ehr(dbl, in, out, ax, g, accumulate, st);
    if (kind == Kind::EH && g.eh2) return launch_pass_eh2(dbl, in, out, ax, g, accumulate, st);
    if (g.qc > 0) return launch_pass_cfp(kind, dbl, in, out, ax, g, accumulate, rho, st);
    // the register accumulates decode their groups (up to 8 lanes each) with 32-bit integers
    if ((kind == Kind::A || kind == Kind::AH) && g.reg_a && g.Qin * g.A * (int64_t)ax.P * g.S * 8 < (int64_t(1) << 31))
        return launch_pass_asr(kind, dbl, in, out, ax, g, accumulate, rho, st);
    if (p2_applicable(kind, ax.M) && g.TS == p2_tile_lines(ax.M))
        return launch_pass_p2(kind, dbl, in, out, ax, g, accumulate, rho, st);
    if (ct_applicable(kind, ax.M) && g.TS == ct_tile_lines(ax.M))
        return launch_pass_ct(kind, dbl, in, out, ax, g, accumulate, rho, st);
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
