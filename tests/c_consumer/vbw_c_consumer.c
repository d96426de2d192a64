/* A plain C consumer of the library: device buffers from the HIP runtime, a
 * plan with a band change, one vbw_filter call, and the result checked
 * against the FP64 oracle (test infrastructure) -- no Python, no PyTorch.
 * Prints the error in dB; exit code 0 when it is within the float32 bar. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "vbw.h"

int oracle_channel_hfso(const double *x, int64_t len, int n, int hop, int lv, const double *v, int n_sched,
                        const int64_t *sched_from, const int32_t *sched_k1, double *y);

#define CHECK_HIP(e)                                                   \
    do {                                                               \
        hipError_t err_ = (e);                                         \
        if (err_ != hipSuccess) {                                      \
            fprintf(stderr, "HIP error %d at line %d\n", err_, __LINE__); \
            return 2;                                                  \
        }                                                              \
    } while (0)

int main(void)
{
    enum { N = 256, HOP = 192, LV = 8, K1 = 24, LEN = 50 * HOP + 37 };
    double v[LV];
    for (int r = 0; r < LV; ++r) v[r] = (double)(float)(1.0 - (r + 0.5) / LV);   /* float32-exact */
    vbw_channel ch = {N, HOP, LV, 0, K1, 0, LEN};
    vbw_plan_desc desc = {1, LV, &ch, v, VBW_C64, VBW_ENGINE_FFT, 0, 0};
    vbw_plan_t plan = NULL;
    vbw_status st = vbw_plan(&desc, &plan);
    if (st != VBW_OK) {
        fprintf(stderr, "vbw_plan: %s\n", vbw_strerror(st));
        return 2;
    }
    st = vbw_set_bandwidth(plan, 0, 60, 20);      /* wider band from block 20 on */
    if (st != VBW_OK) return 2;

    float *hx = malloc(sizeof(float) * 2 * LEN), *hy = malloc(sizeof(float) * 2 * LEN);
    double *x64 = malloc(sizeof(double) * 2 * LEN), *ref = malloc(sizeof(double) * 2 * LEN);
    uint32_t s = 12345u;
    for (int i = 0; i < 2 * LEN; ++i) {            /* uniform in [-1, 1), exact in float32 */
        s = s * 1664525u + 1013904223u;
        hx[i] = (float)((int32_t)(s >> 8) - (1 << 23)) / (float)(1 << 23);
        x64[i] = hx[i];
    }
    void *dx = NULL, *dy = NULL;
    CHECK_HIP(hipMalloc(&dx, sizeof(float) * 2 * LEN));
    CHECK_HIP(hipMalloc(&dy, sizeof(float) * 2 * LEN));
    CHECK_HIP(hipMemcpy(dx, hx, sizeof(float) * 2 * LEN, hipMemcpyHostToDevice));
    const void *xs[1] = {dx};
    void *ys[1] = {dy};
    st = vbw_filter(plan, xs, ys, NULL);
    if (st != VBW_OK) {
        fprintf(stderr, "vbw_filter: %s\n", vbw_strerror(st));
        return 2;
    }
    CHECK_HIP(hipDeviceSynchronize());
    CHECK_HIP(hipMemcpy(hy, dy, sizeof(float) * 2 * LEN, hipMemcpyDeviceToHost));

    int64_t from[2] = {0, 20};
    int32_t k1s[2] = {K1, 60};
    if (oracle_channel_hfso(x64, LEN, N, HOP, LV, v, 2, from, k1s, ref) != 0) return 2;
    double num = 0.0, den = 0.0;
    for (int i = 0; i < 2 * LEN; ++i) {
        num += (hy[i] - ref[i]) * (hy[i] - ref[i]);
        den += ref[i] * ref[i];
    }
    const double db = 10.0 * log10(num / den);
    printf("C consumer: %d samples, error %.1f dB against the oracle\n", LEN, db);
    vbw_destroy(plan);
    CHECK_HIP(hipFree(dx));
    CHECK_HIP(hipFree(dy));
    free(hx);
    free(hy);
    free(x64);
    free(ref);
    return db <= -110.0 ? 0 : 1;
}
