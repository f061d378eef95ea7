// Sanitizer driver for the host side of libebic (evolution steps, screened
// pools, stateful runs and checkpoints) with a deterministic fake evaluator
// in place of the GPU.  Built with AddressSanitizer and UBSan by
// tests/test_sanitizers_cpu.py; exits non-zero on any mismatch.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ebic.h"

namespace ebic {
void set_thread_error(const char *) {}
}
extern "C" ebic_status ebic_evaluate(ebic_ctx *, const int32_t *, const int32_t *, int32_t,
                                     const ebic_params *, uint64_t *, int32_t *, double *) {
    return EBIC_E_STATE;
}
extern "C" ebic_status ebic_get_info(const ebic_ctx *, ebic_ctx_info *) { return EBIC_E_STATE; }

static const int64_t kRows = 300;

// Count: a hash of the ordered series, so that fitness depends on order.
static ebic_status fake_eval(void *, const int32_t *off, const int32_t *cols, int32_t P,
                             const ebic_params *p, uint64_t *masks, int32_t *counts,
                             double *fit) {
    const int64_t W = (kRows + 63) / 64;
    for (int32_t i = 0; i < P; ++i) {
        uint64_t h = 1469598103934665603ull;
        for (int32_t t = off[i]; t < off[i + 1]; ++t) h = (h ^ (uint64_t)cols[t]) * 1099511628211ull;
        const int32_t c = (int32_t)(h % (uint64_t)kRows);
        const int32_t L = off[i + 1] - off[i];
        counts[i] = c;
        fit[i] = c > 1 ? std::ldexp(L * std::log((double)(c - 1)), std::min(c - p->sigma, 0)) : 0.0;
        if (p->want_masks)
            for (int64_t w = 0; w < 2 * W; ++w) masks[(int64_t)i * 2 * W + w] = h >> (w % 64);
    }
    return EBIC_OK;
}

static ebic_status fake_score(void *, const int32_t *off, const int32_t *cols, int32_t B,
                              double *s) {
    for (int32_t i = 0; i < B; ++i) s[i] = (double)((off[i + 1] - off[i]) * 7 % 13) + cols[off[i]] * 1e-3;
    return EBIC_OK;
}

static bool same(ebic_result *a, ebic_result *b) {
    if (ebic_result_size(a) != ebic_result_size(b)) return false;
    for (int32_t i = 0; i < ebic_result_size(a); ++i) {
        const int32_t *ca, *cb;
        int32_t la, lb, na, nb;
        double fa, fb;
        const uint64_t *ma, *mb;
        ebic_result_get(a, i, &ca, &la, &na, &fa, &ma);
        ebic_result_get(b, i, &cb, &lb, &nb, &fb, &mb);
        if (la != lb || na != nb || fa != fb || std::memcmp(ca, cb, sizeof(int32_t) * la) != 0)
            return false;
        if (std::memcmp(ma, mb, sizeof(uint64_t) * ((kRows + 63) / 64)) != 0) return false;
    }
    return true;
}

int main() {
    ebic_evolve_params p;
    ebic_evolve_defaults(&p, 120, 2, 9, 20);
    p.eval.max_violations = 1;
    p.eval.negative_trends = 1;
    const int32_t M = 30, G = 25;
    ebic_result *ref = nullptr, *res = nullptr, *scr = nullptr;
    if (ebic_evolve_with(fake_eval, nullptr, kRows, M, 7, G, &p, &ref) != EBIC_OK) return 2;

    ebic_run *run = nullptr;
    if (ebic_run_create_with(fake_eval, nullptr, kRows, M, 7, G, &p, &run) != EBIC_OK) return 3;
    int32_t done = 0;
    if (ebic_run_advance(run, 9, &done) != EBIC_OK) return 4;
    int64_t n = 0;
    ebic_run_save(run, nullptr, 0, &n);
    std::vector<uint8_t> buf((size_t)n);
    if (ebic_run_save(run, buf.data(), n, &n) != EBIC_OK) return 5;
    ebic_run_destroy(run);
    // truncated and corrupted checkpoints are refused or run safely
    for (int64_t cut : {n - 1, n / 2, (int64_t)12}) {
        ebic_run *bad = nullptr;
        if (ebic_run_load_with(fake_eval, nullptr, kRows, M, &p, buf.data(), cut, &bad) == EBIC_OK)
            return 6;
    }
    std::vector<uint8_t> flip = buf;
    for (size_t i = 60; i < flip.size(); i += 97) flip[i] ^= 0x5A;
    ebic_run *odd = nullptr;
    if (ebic_run_load_with(fake_eval, nullptr, kRows, M, &p, flip.data(), n, &odd) == EBIC_OK) {
        ebic_run_advance(odd, 50, &done);
        ebic_run_destroy(odd);
    }
    if (ebic_run_load_with(fake_eval, nullptr, kRows, M, &p, buf.data(), n, &run) != EBIC_OK)
        return 7;
    if (ebic_run_advance(run, 1000, &done) != EBIC_OK || !done) return 8;
    if (ebic_run_result(run, &res) != EBIC_OK) return 9;
    ebic_run_destroy(run);
    if (!same(ref, res)) return 10;

    if (ebic_evolve_screened_with(fake_eval, nullptr, fake_score, nullptr, kRows, M, 3, 12, 4, 2,
                                  4, &p, &scr) != EBIC_OK)
        return 11;
    ebic_result_free(ref);
    ebic_result_free(res);
    ebic_result_free(scr);
    std::printf("host driver ok\n");
    return 0;
}
