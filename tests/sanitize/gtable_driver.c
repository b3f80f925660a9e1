/* The oracle's kernel table (oracle/gtable.c) under AddressSanitizer and UndefinedBehaviorSanitizer:
 * a sweep of lengths, magnifications, offsets, flight times and index ranges, and the rejected
 * argument sets. Only the argument checks and finite values are asserted here; the values are
 * pinned by the oracle's own tests. Exit status 0 on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_gtable(int64_t M, int64_t lam, double delta, double t, double m_over_hbar, double dx, int64_t s_min,
                  int64_t count, double* out_re, double* out_im);

int main(void) {
    static const int64_t Ms[] = {1, 2, 3, 7, 16, 33};
    static const int64_t lams[] = {1, 2, 3, 5, 8};
    static const double deltas[] = {0.0, -19.5, 0.37, 1234.0};
    static const double ts[] = {0.0, 2.5, -7.0, 400.0};
    int fails = 0, calls = 0;
    for (size_t a = 0; a < sizeof Ms / sizeof Ms[0]; ++a)
        for (size_t b = 0; b < sizeof lams / sizeof lams[0]; ++b)
            for (size_t c = 0; c < sizeof deltas / sizeof deltas[0]; ++c)
                for (size_t d = 0; d < sizeof ts / sizeof ts[0]; ++d) {
                    const int64_t M = Ms[a], lam = lams[b];
                    const int64_t count = 2 * lam * M + 3;  /* the range of s = lam nbar - n and beyond */
                    const int64_t s_min = -(M - 1) - 1;
                    double* re = (double*)malloc(sizeof(double) * (size_t)count);
                    double* im = (double*)malloc(sizeof(double) * (size_t)count);
                    int rc = oracle_gtable(M, lam, deltas[c], ts[d], 1.0, 0.5, s_min, count, re, im);
                    ++calls;
                    if (rc != 0) { fprintf(stderr, "FAIL valid call rejected M=%lld lam=%lld\n", (long long)M, (long long)lam); ++fails; }
                    for (int64_t i = 0; rc == 0 && i < count; ++i)
                        if (!isfinite(re[i]) || !isfinite(im[i])) {
                            fprintf(stderr, "FAIL non-finite entry M=%lld lam=%lld i=%lld\n", (long long)M, (long long)lam, (long long)i);
                            ++fails;
                            break;
                        }
                    free(re);
                    free(im);
                }
    {  /* one table at the size of the 3-D ensemble's shortest axis */
        const int64_t M = 32, lam = 40, count = 2 * lam * M;
        double* re = (double*)malloc(sizeof(double) * (size_t)count);
        double* im = (double*)malloc(sizeof(double) * (size_t)count);
        if (oracle_gtable(M, lam, -623.5, 400.0, 1.0, 1.0, -(M - 1), count, re, im) != 0) ++fails;
        for (int64_t i = 0; i < count; ++i)
            if (!isfinite(re[i]) || !isfinite(im[i])) { ++fails; break; }
        free(re);
        free(im);
        ++calls;
    }
    double v[4];
    if (oracle_gtable(0, 3, 0.0, 1.0, 1.0, 1.0, 0, 2, v, v + 2) == 0) { fprintf(stderr, "FAIL M = 0 accepted\n"); ++fails; }
    if (oracle_gtable(4, 0, 0.0, 1.0, 1.0, 1.0, 0, 2, v, v + 2) == 0) { fprintf(stderr, "FAIL lam = 0 accepted\n"); ++fails; }
    if (oracle_gtable(4, 3, 0.0, 1.0, 1.0, -1.0, 0, 2, v, v + 2) == 0) { fprintf(stderr, "FAIL dx < 0 accepted\n"); ++fails; }
    if (oracle_gtable(4, 3, 0.0, 1.0, 0.0, 1.0, 0, 2, v, v + 2) == 0) { fprintf(stderr, "FAIL m/hbar = 0 accepted\n"); ++fails; }
    if (oracle_gtable(4, 3, 0.0, 1.0, 1.0, 1.0, 0, -1, v, v + 2) == 0) { fprintf(stderr, "FAIL count < 0 accepted\n"); ++fails; }
    printf("gtable driver: %d calls, %d failures\n", calls, fails);
    return fails ? 1 : 0;
}
