/*
 * ORACLE -- test infrastructure only. Nothing in the product library links,
 * loads or calls this file; only the tests, the smoke check and the CPU
 * baseline of the benchmark do.
 *
 * Per-axis kernel of the discrete free propagator on the vacuum-padded,
 * lam-times-larger periodic lattice (section 5.1, eqs. (vacuum), (ex1), (ulk),
 * (ex2)-(ex5), (iDFTbar); the result that the prescription (FF) of section 5.2
 * reaches exactly):
 *
 *   G(s) = 1/(lam*M) * sum_{l in F} exp( 2 pi i [ l (s + delta) / (lam M) - beta l^2 ] )
 *
 * where F is the set of lam*M integer wave numbers centred on zero with the
 * Nyquist value negative (the ordering of eq. (kj) on the fine lattice),
 * delta = (abar - a)/dx, beta = pi hbar t / (m (lam L)^2) (cycles per l^2), and
 * s = lam*nbar - n is the integer distance between an output sample and an
 * input point in units of dx. The continuum wave number is
 * kappa_l = 2 pi l / (lam L), so l*(s+delta)/(lam M) is kappa_l * r / (2 pi) and
 * beta l^2 is hbar t kappa_l^2 / (2 m) / (2 pi).
 *
 * Plain direct sum: every term is evaluated, no FFT, no recurrences. The
 * phase is formed in cycles with the integer part l*(s + round(delta)) reduced
 * exactly modulo lam*M in 64-bit integers; the fractional offset and the
 * quadratic term are evaluated in long double (64-bit mantissa) and the sum is
 * accumulated in long double.
 */
#include <math.h>
#include <stdint.h>

static long double two_pi_l(void) { return 2.0L * acosl(-1.0L); }

/* Fills out_re/out_im[i] = G(s_min + i), i = 0..count-1. Returns 0 on success. */
int oracle_gtable(int64_t M, int64_t lam, double delta, double t, double m_over_hbar,
                  double dx, int64_t s_min, int64_t count, double* out_re, double* out_im)
{
    if (M < 1 || lam < 1 || count < 0 || !(dx > 0.0) || !(m_over_hbar > 0.0)) return -1;
    const int64_t N = lam * M;
    const long double pi = acosl(-1.0L);
    const long double L_big = (long double)N * (long double)dx;          /* lam * L */
    const long double beta = pi * ((long double)t / (long double)m_over_hbar) / (L_big * L_big);
    const long double tp = two_pi_l();
    const long double d_int = nearbyintl((long double)delta);
    const long double d_frac = (long double)delta - d_int;
    const int64_t di = (int64_t)d_int;
    /* F = { -floor(N/2), ..., ceil(N/2)-1 } */
    const int64_t l_lo = -(N / 2);
    const int64_t l_hi = l_lo + N;  /* exclusive */

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < count; ++i) {
        const int64_t s = s_min + i + di;
        long double re = 0.0L, im = 0.0L;
        for (int64_t l = l_lo; l < l_hi; ++l) {
            int64_t k = (l % N) * (s % N) % N;           /* l*s mod N, exact */
            if (k < 0) k += N;
            long double ph = (long double)k / (long double)N
                           + (long double)l * d_frac / (long double)N
                           - beta * (long double)l * (long double)l;
            ph -= nearbyintl(ph);
            long double ang = tp * ph;
            re += cosl(ang);
            im += sinl(ang);
        }
        out_re[i] = (double)(re / (long double)N);
        out_im[i] = (double)(im / (long double)N);
    }
    return 0;
}
