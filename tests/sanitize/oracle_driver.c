/* Sanitizer driver for the C oracle: adversarial values (NaN, signed zeros,
 * infinities, ties), every tolerance and direction, masks and depths. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_evaluate(const float *a, int64_t N, int32_t M, int64_t ld, const int32_t *offsets,
                    const int32_t *cols, int32_t P, int32_t sigma, int32_t k, int32_t negative,
                    uint64_t *masks, int32_t *counts, double *fitness, int64_t *reads,
                    int32_t *depth, int32_t nthreads);

int main(void) {
    const int64_t N = 131;
    const int32_t M = 7, P = 5;
    float *a = malloc(sizeof(float) * N * M);
    for (int64_t i = 0; i < N * M; ++i) {
        const int r = (int)(i % 11);
        a[i] = r == 0 ? NAN : r == 1 ? -0.0f : r == 2 ? INFINITY : (float)((i * 37) % 13) - 6.0f;
    }
    const int32_t off[] = {0, 1, 3, 6, 10, 17};
    const int32_t cols[] = {2, 0, 1, 3, 4, 5, 6, 5, 4, 3, 0, 1, 2, 3, 4, 5, 6};
    const int64_t W = (N + 63) / 64;
    uint64_t *masks = calloc((size_t)(P * 2 * W), sizeof(uint64_t));
    int32_t counts[5], *depth = calloc((size_t)(P * N), sizeof(int32_t));
    double fit[5];
    int64_t reads[5];
    for (int k = 0; k <= 3; ++k)
        for (int neg = 0; neg <= 1; ++neg)
            if (oracle_evaluate(a, N, M, M, off, cols, P, 3, k, neg, masks, counts, fit, reads,
                                depth, 2) != 0)
                return 1;
    free(a);
    free(masks);
    free(depth);
    printf("oracle driver ok\n");
    return 0;
}
