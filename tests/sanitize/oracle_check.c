/* The oracle's entry points on small and degenerate cases, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer: every buffer is exactly
 * the documented size, so an out-of-bounds access is reported.  Exit code 0 =
 * every call returned as documented. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_dft(int n, const double *s, double *X);
int oracle_idft(int n, const double *Y, double *z);
int oracle_hfso_coeffs(int n, int hop, int k1, int lv, const double *v, double *H);
int oracle_blocks_hfso(const double *x, int64_t len, int n, int hop, int lv, const double *v, int n_sched,
                       const int64_t *sched_from, const int32_t *sched_k1, const int64_t *blocks, int64_t n_sel,
                       double *out);
int oracle_channel_hfso(const double *x, int64_t len, int n, int hop, int lv, const double *v, int n_sched,
                        const int64_t *sched_from, const int32_t *sched_k1, double *y);

int main(void)
{
    int bad = 0;
    double v[8] = {0.9, 0.8, 0.6, 0.5, 0.3, 0.2, 0.1, 0.05};
    for (int n = 4; n <= 64; n *= 2) {
        double *s = malloc(sizeof(double) * 2 * n), *X = malloc(sizeof(double) * 2 * n);
        for (int i = 0; i < 2 * n; ++i) s[i] = (double)((i * 37) % 11) - 5.0;
        bad |= oracle_dft(n, s, X) != 0;
        bad |= oracle_idft(n, X, s) != 0;
        bad |= oracle_hfso_coeffs(n, n / 2, 1, 1, v, X) != 0;
        free(s);
        free(X);
    }
    int64_t lens[] = {0, 1, 5, 47, 48, 49, 300};
    for (unsigned li = 0; li < sizeof(lens) / sizeof(lens[0]); ++li) {
        int64_t len = lens[li];
        int n = 16, hop = 12;
        double *x = len ? malloc(sizeof(double) * 2 * len) : NULL;
        double *y = len ? malloc(sizeof(double) * 2 * len) : NULL;
        for (int64_t i = 0; i < 2 * len; ++i) x[i] = (double)(i % 7) - 3.0;
        int64_t from[2] = {0, 3};
        int32_t k1s[2] = {2, 5};
        bad |= oracle_channel_hfso(x, len, n, hop, 2, v, 2, from, k1s, y) != 0;
        int64_t nb = (len + hop - 1) / hop;
        if (nb > 0) {
            int64_t blocks[2] = {0, nb - 1};
            double *out = malloc(sizeof(double) * 2 * hop * 2);
            bad |= oracle_blocks_hfso(x, len, n, hop, 2, v, 2, from, k1s, blocks, 2, out) != 0;
            int64_t outside[1] = {nb};
            bad |= oracle_blocks_hfso(x, len, n, hop, 2, v, 2, from, k1s, outside, 1, out) == 0;
            free(out);
        }
        free(x);
        free(y);
    }
    printf("oracle checks: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
