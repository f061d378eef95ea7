/*
 * EBIC population evaluation -- the CPU oracle.
 *
 * TEST INFRASTRUCTURE.  This file is the plain, slow, obviously correct
 * definition that the GPU path is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header or table with the HIP library.
 *
 * What it computes (EBIC, Orzechowski et al. 2018):
 *   - a bicluster is an ordered series of column indices (Methods, the
 *     representation paragraph after Eq. 1; CBF in Fig. 2);
 *   - a row follows the series when its values rise strictly from each
 *     column of the series to the next (Motivation: the comparison is the
 *     strict "a_kp < a_kq");
 *   - with negative trends on, a row that falls strictly along the series
 *     also counts, and with an approximate tolerance k a row may break the
 *     rule on at most k consecutive pairs (Step 7 names approximate and
 *     negative trends without defining a tolerance; the reading used here
 *     is "at most k violating consecutive pairs per direction", a row being
 *     counted once if either direction accepts it);
 *   - |I| is the number of matching rows (Step 4) and the fitness is
 *     Eq. (1): f = 2^min(|I|-sigma, 0) * |J| * log(|I| - 1) when |I| > 1,
 *     else 0, with |J| the series length and log the natural logarithm.
 *
 * Comparisons are IEEE single precision: NaN compares false both ways, so a
 * pair holding NaN violates both directions, as does a tie (+0 and -0 tie).
 * Build without fast-math: the NaN behaviour is part of the definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_E_ARG 1
#define ORACLE_E_RANGE 2

/* Eq. (1).  FP64, natural log, 2^x applied exactly with ldexp. */
double oracle_fitness(int64_t count, int64_t len, int64_t sigma)
{
    if (count <= 1)
        return 0.0;
    int64_t e = count - sigma;
    if (e > 0)
        e = 0;
    return ldexp((double)len * log((double)(count - 1)), (int)e);
}

/* Validate a CBF population against an M-column matrix. */
int oracle_check_population(const int32_t *offsets, const int32_t *cols, int32_t P, int32_t M)
{
    if (P < 0)
        return ORACLE_E_ARG;
    if (P == 0)
        return ORACLE_OK;
    if (!offsets || !cols || offsets[0] != 0)
        return ORACLE_E_ARG;
    for (int32_t c = 0; c < P; ++c) {
        if (offsets[c + 1] <= offsets[c])
            return ORACLE_E_ARG;
        for (int32_t i = offsets[c]; i < offsets[c + 1]; ++i) {
            if (cols[i] < 0 || cols[i] >= M)
                return ORACLE_E_RANGE;
            for (int32_t j = offsets[c]; j < i; ++j)
                if (cols[j] == cols[i])
                    return ORACLE_E_ARG;
        }
    }
    return ORACLE_OK;
}

/*
 * Evaluate a population.
 *
 *   a            row-major N x M matrix, row stride ld (elements)
 *   offsets/cols CBF population, P candidates, 0-based columns
 *   sigma, k     Eq. (1) sigma and the approximate tolerance
 *   negative     0/1: also accept strictly falling rows
 *   masks        NULL, or P*2*W words: masks[(c*2+dir)*W + w], dir 0 = rising,
 *                dir 1 = falling, bit (r % 64) of word r / 64, W = ceil(N/64)
 *   counts       P: number of rows accepted by either direction
 *   fitness      P: Eq. (1)
 *   values_read  NULL, or P: sum over rows of d(c,r), the number of series
 *                values row r must be read, left to right, before its
 *                decision is fixed (L if accepted; otherwise 2 + the 0-based
 *                index of the pair after which every enabled direction has
 *                more than k violations)
 *   depth        NULL, or P*N: d(c,r) itself, at depth[c*N + r]
 *   nthreads     OpenMP threads over candidates (<= 0: runtime default)
 */
int oracle_evaluate(const float *a, int64_t N, int32_t M, int64_t ld,
                    const int32_t *offsets, const int32_t *cols, int32_t P,
                    int32_t sigma, int32_t k, int32_t negative,
                    uint64_t *masks, int32_t *counts, double *fitness,
                    int64_t *values_read, int32_t *depth, int32_t nthreads)
{
    if (!a || N < 1 || M < 1 || ld < M || !counts || !fitness)
        return ORACLE_E_ARG;
    if (sigma < 0 || k < 0)
        return ORACLE_E_RANGE;
    int rc = oracle_check_population(offsets, cols, P, M);
    if (rc != ORACLE_OK)
        return rc;
    const int64_t W = (N + 63) / 64;
    if (masks)
        memset(masks, 0, sizeof(uint64_t) * (size_t)P * 2 * (size_t)W);

#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic)
#endif
    for (int32_t c = 0; c < P; ++c) {
        const int32_t *s = cols + offsets[c];
        const int32_t L = offsets[c + 1] - offsets[c];
        int64_t count = 0;
        int64_t read = 0;
        for (int64_t r = 0; r < N; ++r) {
            const float *row = a + r * ld;
            int32_t vu = 0, vd = 0;
            int64_t d = L;
            int decided_early = 0;
            for (int32_t t = 0; t + 1 < L; ++t) {
                float x = row[s[t]];
                float y = row[s[t + 1]];
                if (!(x < y))
                    vu++;
                if (!(x > y))
                    vd++;
                if (!decided_early && vu > k && (!negative || vd > k)) {
                    decided_early = 1;
                    d = (int64_t)t + 2;
                }
            }
            int pos = vu <= k;
            int neg = negative && vd <= k;
            if (pos || neg)
                count++;
            read += d;
            if (depth)
                depth[(size_t)c * (size_t)N + (size_t)r] = (int32_t)d;
            if (masks) {
                if (pos)
                    masks[((size_t)c * 2 + 0) * W + (size_t)(r / 64)] |= (uint64_t)1 << (r % 64);
                if (neg)
                    masks[((size_t)c * 2 + 1) * W + (size_t)(r / 64)] |= (uint64_t)1 << (r % 64);
            }
        }
        counts[c] = (int32_t)count;
        fitness[c] = oracle_fitness(count, L, sigma);
        if (values_read)
            values_read[c] = read;
    }
    return ORACLE_OK;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int32_t oracle_max_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
