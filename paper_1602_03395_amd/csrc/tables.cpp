// FP64 phase tables of the prescription (FF), section 5.2, one set per axis.
//
// Every phase is written in cycles (units of 2 pi) as a sum of
//   * an exact rational part (integer numerator reduced modulo its integer
//     denominator in int64),
//   * a small fractional-offset part (|value| <= 1/2 by construction), and
//   * a quadratic part beta * I with beta = pi hbar t / (m lam^2 L^2) and an
//     exact integer I; beta is carried as a double-double (computed in long
//     double) and beta_hi * I is split exactly with an FMA two-product, so the
//     product is reduced modulo 1 without losing the fractional digits that a
//     large chirp argument would otherwise swamp.
// Only the reduced phase (|c| <= 1/2 cycle) goes through sin/cos.
//
// With k = dk * l~ (eq. (kj)), alpha_q = q dk / lam, delta = (abar - a)/dx and
// ell = lam * l~ + q (the fine-lattice wave number of eq. (ulk)):
//   TA[q][n]   : -alpha_q (x_n - a)                      = -(q n) / (lam M)
//   TB[q][m~]  : k (abar - a) - k (k + 2 alpha_q) ht/2m  = l~ delta / M - beta (ell^2 - q^2)
//   Tf[q][nb]  : alpha_q (xbar - a) - alpha_q^2 ht/2m    = q (delta + lam nb) / (lam M) - beta q^2
// For odd M the largest positive coarse wave number is folded to the negative
// side when q >= lam/2 (the umklapp rule stated after (FF)).
//
// Other spectra (section 7.4): with exp(-i t omega_k) in place of the free-particle
// factor, the quadratic parts become -(phi(ell) - phi(q)) in TB and -phi(q) in Tf,
// phi = t omega / (2 pi) in cycles, read from a caller table over the fine wave numbers.
#include <cmath>
#include <cstdint>

#include "fx_internal.h"

namespace fx {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

inline double reduce_cycles(double c) { return c - std::nearbyint(c); }

// (num mod den) / den in [-1/2, 1/2], exact up to the final division.
inline double rational_cycles(int64_t num, int64_t den) {
    int64_t r = num % den;
    if (r < 0) r += den;
    if (2 * r > den) r -= den;
    return (double)r / (double)den;
}

struct DD { double hi, lo; };

// frac(beta * I) for the double-double beta and an integer I below 2^53.
inline double beta_cycles(DD beta, int64_t I) {
    const double x = (double)I;
    const double p = beta.hi * x;
    const double e = std::fma(beta.hi, x, -p);  // p + e == beta.hi * x exactly
    return reduce_cycles(reduce_cycles(p) + e + beta.lo * x);
}

inline void put(std::vector<double>& v, size_t i, double cycles, double amp) {
    const double ang = kTwoPi * reduce_cycles(cycles);
    v[2 * i] = amp * std::cos(ang);
    v[2 * i + 1] = amp * std::sin(ang);
}

// Chirp-folded table of the register E kernel. With g = gcd(lam, M), P = M / g, input index
// n = g n1 + n2 and spectral index m = r + P c (n1, r < P; n2, c < g), the forward DFT factors as
//   Y[r + P c] = sum_n2 w_g^(n2 c) w_M^(n2 r) V[n2][r],  V[n2][r] = sum_n1 w_P^(n1 r) y[g n1 + n2],
// so the chirp (presB) and the fold over c of the pruned inverse collapse into
//   W[r] = sum_c TB[r + P c] Y[r + P c] = sum_n2 HT[n2][r] V[n2][r],
//   HT[n2][r] = w_M^(n2 r) TA'[n2] sum_c TB[r + P c] w_g^(n2 c) / M,
// where the n2 part of (presA), TA'[n2] = exp(-2 pi i q n2 / (lam M)), and the 1/M of the inverse
// are folded in as well. Layout [q][r][n2] (the g lanes of a line read consecutive values, and the
// P g = M values of one q are contiguous), FP64 complex.
void build_ht(AxisTables& t, int64_t M, int64_t lam) {
    int64_t g = lam, b = M;
    while (b) { const int64_t r = g % b; g = b; b = r; }
    const int64_t P = M / g;
    const int64_t N = lam * M;
    t.HT.assign(2 * (size_t)(lam * M), 0.0);
    std::vector<double> rg(2 * (size_t)g);  // exp(-2 pi i k / g)
    for (int64_t k = 0; k < g; ++k) put(rg, (size_t)k, -rational_cycles(k, g), 1.0);
    auto at = [&](int64_t q, int64_t r, int64_t n2) { return 2 * (size_t)((q * P + r) * g + n2); };
    for (int64_t q = 0; q < lam; ++q) {
        const double* tb = &t.TB[2 * (size_t)(q * M)];
        for (int64_t n2 = 0; n2 < g; ++n2) {
            for (int64_t r = 0; r < P; ++r) {
                double sr = 0.0, si = 0.0;
                for (int64_t c = 0; c < g; ++c) {
                    const double* z = tb + 2 * (r + P * c);
                    const double* w = &rg[2 * (size_t)((n2 * c) % g)];
                    sr += z[0] * w[0] - z[1] * w[1];
                    si += z[0] * w[1] + z[1] * w[0];
                }
                // exp(-2 pi i (n2 r lam + q n2) / (lam M)) / M
                const double ang = -kTwoPi * rational_cycles(n2 * r * lam + q * n2, N);
                const double er = std::cos(ang) / (double)M, ei = std::sin(ang) / (double)M;
                const size_t i = at(q, r, n2);
                t.HT[i] = sr * er - si * ei;
                t.HT[i + 1] = sr * ei + si * er;
            }
        }
    }
    // Second copy for the forward register kernels. Their first cross-lane reduction step pairs
    // lanes n2 and n2 ^ 1; the odd lane keeps the upper half of the P sums. When the odd lane's
    // P values come with their halves exchanged, both lanes keep the lower half and send the upper
    // one, so no per-lane selects are needed:
    //   g >= P (transform, multiply, then reduce): the odd lane's input is modulated by (-1)^n1,
    //     which moves its spectrum by P/2, so its table row is HT[n2][r ^ P/2];
    //   g <  P (transform, multiply, inverse, then reduce): the odd lane's inverse output is moved
    //     by P/2 when its row is modulated by (-1)^r.
    t.HTx = t.HT;
    const bool p2 = (P & (P - 1)) == 0;
    if (p2 && P >= 2 && g >= 2) {
        for (int64_t q = 0; q < lam; ++q) {
            for (int64_t n2 = 1; n2 < g; n2 += 2) {
                for (int64_t r = 0; r < P; ++r) {
                    const size_t d = at(q, r, n2);
                    if (g >= P) {
                        const size_t s = at(q, r ^ (P / 2), n2);
                        t.HTx[d] = t.HT[s];
                        t.HTx[d + 1] = t.HT[s + 1];
                    } else if (r & 1) {
                        t.HTx[d] = -t.HT[d];
                        t.HTx[d + 1] = -t.HT[d + 1];
                    }
                }
            }
        }
    }
    // The table once more in [q][n2][r] order, for kernels whose lanes read their own P values of a
    // row contiguously. For power-of-two P <= min(g, 8) those kernels shift lane n2's spectrum by
    // s = bitrev(n2 mod P) (its input times exp(-2 pi i s n1 / P)), which makes every step of the
    // reduction over the lanes select-free, so the lane's row is turned by s: HTl[q][n2][r] =
    // HT[q][(r + s) mod P][n2] (for P = 2 this is HTx). Otherwise HTl is HTx reordered.
    t.HTl.assign(t.HTx.size(), 0.0);
    int lgp = 0;
    while ((int64_t(1) << lgp) < P) ++lgp;
    const bool rot = p2 && P >= 2 && P <= 8 && g >= P;
    for (int64_t q = 0; q < lam; ++q)
        for (int64_t n2 = 0; n2 < g; ++n2) {
            int64_t sh = 0;
            for (int b = 0; b < lgp; ++b) sh |= ((n2 >> b) & 1) << (lgp - 1 - b);
            for (int64_t r = 0; r < P; ++r) {
                const size_t d = 2 * (size_t)((q * g + n2) * P + r);
                const size_t src = rot ? at(q, (r + sh) % P, n2) : at(q, r, n2);
                const std::vector<double>& from = rot ? t.HT : t.HTx;
                t.HTl[d] = from[src];
                t.HTl[d + 1] = from[src + 1];
            }
        }
}

}  // namespace

AxisTables build_axis_tables(const AxisParams& p) {
    const int64_t M = p.M;
    const int64_t lam = p.lam;
    const int64_t N = lam * M;
    AxisTables t;
    t.TA.resize(2 * (size_t)(lam * M));
    t.TB.resize(2 * (size_t)(lam * M));
    t.Tf.resize(2 * (size_t)(lam * M));
    t.tw.resize(2 * (size_t)M);

    // beta = pi * (t / (m/hbar)) / (lam * M * dx)^2 in long double, split into hi + lo.
    const long double pi_l = 3.14159265358979323846264338327950288L;
    const long double Lb = (long double)N * (long double)p.dx;
    const long double beta_l = pi_l * ((long double)p.t / (long double)p.m_over_hbar) / (Lb * Lb);
    DD beta;
    beta.hi = (double)beta_l;
    beta.lo = (double)(beta_l - (long double)beta.hi);

    const double delta = (p.abar - p.a) / p.dx;
    const double di_d = std::nearbyint(delta);
    const int64_t di = (int64_t)di_d;
    const double df = delta - di_d;

    const double inv2pi = 1.0 / kTwoPi;
    const int64_t l0 = N / 2;  // table index of the fine wave number 0
    for (int64_t q = 0; q < lam; ++q) {
        const double phq = p.phase ? p.phase[l0 + q] * inv2pi : 0.0;
        for (int64_t n = 0; n < M; ++n) {
            const size_t i = (size_t)(q * M + n);
            // TA: -(q n)/(lam M)
            put(t.TA, i, -rational_cycles(q * n, N), 1.0);
            // TB: coarse wave number of eq. (kj) with the odd-M umklapp.
            int64_t lt = (2 * n < M) ? n : n - M;
            if ((M % 2 == 1) && (2 * n == M - 1) && (2 * q >= lam)) lt -= M;
            const int64_t ell = lam * lt + q;
            const int64_t I = ell * ell - q * q;
            const double chirp = p.phase ? reduce_cycles(p.phase[l0 + ell] * inv2pi - phq)
                                         : beta_cycles(beta, I);
            const double tb = rational_cycles(lt * di, M) + (double)lt * df / (double)M - chirp;
            put(t.TB, i, tb, 1.0);
            // Tf: q (delta + lam nb)/(lam M) - beta q^2, amplitude 1/lam.
            const double tf = rational_cycles(q * (di + lam * n), N) + (double)q * df / (double)N
                              - (p.phase ? reduce_cycles(phq) : beta_cycles(beta, q * q));
            put(t.Tf, i, tf, 1.0 / (double)lam);
        }
    }
    for (int64_t k = 0; k < M; ++k) put(t.tw, (size_t)k, -rational_cycles(k, M), 1.0);
    if (p.want_ht) build_ht(t, M, lam);
    return t;
}

}  // namespace fx
