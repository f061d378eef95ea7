// EBIC's evolutionary run on the host (Steps 1-7), driving the GPU
// evaluator once per generation.
//
// The paper fixes the structure of the run (Section 2.2, Steps 1-7), the
// crowding penalty 1.2^theta with theta the mean per-column penalty of a
// series (Section 2.1), the five genetic operations (Fig. 1), the tabu list
// with its hit-count stop rule (Step 3) and the top-rank list with its
// overlap rule (Step 5).  The constants and operator details it leaves open
// are fixed as documented in include/ebic.h next to ebic_evolve, so that a
// run is a deterministic function of (matrix, seed, parameters).
//
// Populations are kept in CBF form (offsets + concatenated columns, Fig. 2),
// the form the evaluator consumes.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "ebic_run.h"

namespace {

using namespace ebic::host;

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

struct Evaluator {
    ebic_eval_fn fn;
    void *user;
    double ms = 0.0;
    int64_t evaluated = 0;
    ebic_status operator()(const Pop &p, int32_t first, const ebic_params *prm, uint64_t *masks,
                           int32_t *counts, double *fit) {
        const int32_t P = p.size() - first;
        if (P <= 0) return EBIC_OK;
        // Re-base the CBF offsets of members [first, size) to start at 0.
        std::vector<int32_t> off((size_t)P + 1);
        const int32_t base = p.off[(size_t)first];
        for (int32_t i = 0; i <= P; ++i) off[(size_t)i] = p.off[(size_t)(first + i)] - base;
        auto t0 = Clock::now();
        ebic_status st = fn(user, off.data(), p.cols.data() + base, P, prm, masks, counts, fit);
        ms += ms_since(t0);
        evaluated += P;
        return st;
    }
};



}  // namespace

namespace {

ebic_status run(Evaluator &ev, int64_t n_rows, int32_t M, uint64_t seed, int32_t generations,
                const ebic_evolve_params &p, ebic_result **out) {
    const auto t_start = Clock::now();
    const int64_t W = (n_rows + 63) / 64;
    Run run(M, seed, generations, p);
    std::vector<int32_t> cnt;
    std::vector<double> fit;
    while (run.next()) {
        const Pop &pop = run.pending();
        const int32_t first = run.first_new();
        cnt.resize((size_t)(pop.size() - first));
        fit.resize(cnt.size());
        ebic_status st = ev(pop, first, &run.eval_params(), nullptr, cnt.data(), fit.data());
        if (st != EBIC_OK) return st;
        run.accept(cnt.data(), fit.data());
    }
    // Steps 6-7: rows of the listed series with the expansion parameters.
    const std::vector<TopEntry> &top = run.top();
    const int32_t K = (int32_t)top.size();
    std::vector<uint64_t> masks((size_t)K * 2 * (size_t)W);
    std::vector<int32_t> rc((size_t)K);
    std::vector<double> rf((size_t)K);
    if (K > 0) {
        Pop tp;
        for (const TopEntry &e : top) tp.push(e.s.data(), (int32_t)e.s.size());
        ebic_params ex = p.expand;
        ex.want_masks = 1;
        ebic_status st = ev(tp, 0, &ex, masks.data(), rc.data(), rf.data());
        if (st != EBIC_OK) return st;
    }
    ebic_result *r = make_result(top, W, masks, std::move(rc), std::move(rf));
    if (!r) return evolve_error(EBIC_E_NOMEM, "cannot allocate result");
    r->stats.struct_size = sizeof(ebic_run_stats);
    r->stats.generations_run = run.generations_run();
    r->stats.stopped_by_tabu = run.stopped() ? 1 : 0;
    r->stats.candidates_evaluated = ev.evaluated;
    r->stats.wall_ms = ms_since(t_start);
    r->stats.eval_ms = ev.ms;
    r->stats.host_ms = r->stats.wall_ms - ev.ms;
    *out = r;
    return EBIC_OK;
}

// Screened run (offspring screening; not in the paper).  Generations after
// `warmup` draw an oversampled pool and keep the children `scorer` ranks
// highest; `scorer(pool, &status)` returns one float or double per child.
template <typename Scorer>
ebic_status run_screened(Evaluator &ev, Scorer &&score_pool, int64_t n_rows, int32_t M,
                         uint64_t seed, int32_t generations, int32_t oversample, int32_t warmup,
                         int32_t threads, const ebic_evolve_params &p, ebic_result **out) {
    const auto t_start = Clock::now();
    const int64_t W = (n_rows + 63) / 64;
    Run run(M, seed, generations, p);
    std::vector<int32_t> cnt, po;
    std::vector<double> fit;
    ebic_status score_st = EBIC_OK;
    auto scorer = [&](const Pop &pool) { return score_pool(pool, &score_st); };
    for (;;) {
        const bool screen = run.generation() > warmup;
        const bool more = screen ? run.next_screened(oversample, scorer, threads) : run.next();
        if (score_st != EBIC_OK) return score_st;
        if (!more) break;
        const Pop &pop = run.pending();
        const int32_t first = run.first_new();
        cnt.resize((size_t)(pop.size() - first));
        fit.resize(cnt.size());
        ebic_status st = ev(pop, first, &run.eval_params(), nullptr, cnt.data(), fit.data());
        if (st != EBIC_OK) return st;
        run.accept(cnt.data(), fit.data());
    }
    const std::vector<TopEntry> &top = run.top();
    const int32_t K = (int32_t)top.size();
    std::vector<uint64_t> masks((size_t)K * 2 * (size_t)W);
    std::vector<int32_t> rc((size_t)K);
    std::vector<double> rf((size_t)K);
    if (K > 0) {
        Pop tp;
        for (const TopEntry &e : top) tp.push(e.s.data(), (int32_t)e.s.size());
        ebic_params ex = p.expand;
        ex.want_masks = 1;
        ebic_status st = ev(tp, 0, &ex, masks.data(), rc.data(), rf.data());
        if (st != EBIC_OK) return st;
    }
    ebic_result *r = make_result(top, W, masks, std::move(rc), std::move(rf));
    if (!r) return evolve_error(EBIC_E_NOMEM, "cannot allocate result");
    r->stats.struct_size = sizeof(ebic_run_stats);
    r->stats.generations_run = run.generations_run();
    r->stats.stopped_by_tabu = run.stopped() ? 1 : 0;
    r->stats.candidates_evaluated = ev.evaluated;
    r->stats.wall_ms = ms_since(t_start);
    r->stats.eval_ms = ev.ms;
    r->stats.host_ms = r->stats.wall_ms - ev.ms;
    *out = r;
    return EBIC_OK;
}

ebic_status ctx_eval(void *user, const int32_t *offsets, const int32_t *cols, int32_t P,
                     const ebic_params *p, uint64_t *masks, int32_t *counts, double *fitness) {
    return ebic_evaluate(static_cast<ebic_ctx *>(user), offsets, cols, P, p, masks, counts,
                         fitness);
}

}  // namespace

extern "C" {

void ebic_evolve_defaults(ebic_evolve_params *p, int32_t population, int32_t len_min,
                          int32_t len_max, int32_t sigma) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(ebic_evolve_params);
    p->population = population;
    p->len_min = len_min;
    p->len_max = len_max;
    p->tournament = 3;
    for (int i = 0; i < 5; ++i) p->op_weight[i] = 1;
    p->elite_num = 1;
    p->elite_den = 4;
    p->penalty_base = 1.2;
    p->overlap = 0.5;
    p->toplist_size = 100;
    p->tabu_limit = -1;
    p->eval = ebic_params{sizeof(ebic_params), sigma, 0, 0, 0};
    p->expand = ebic_params{sizeof(ebic_params), sigma, 0, 1, 1};
}

ebic_status ebic_evolve_with(ebic_eval_fn eval, void *eval_user, int64_t n_rows, int32_t n_cols,
                             uint64_t seed, int32_t generations, const ebic_evolve_params *params,
                             ebic_result **out) {
    if (!eval || !out) return evolve_error(EBIC_E_ARG, "eval and out must not be null");
    if (generations < 0) return evolve_error(EBIC_E_ARG, "generations must be >= 0");
    ebic_status st = check_params(params, n_rows, n_cols);
    if (st != EBIC_OK) return st;
    *out = nullptr;
    Evaluator ev{eval, eval_user};
    try {
        return run(ev, n_rows, n_cols, seed, generations, *params, out);
    } catch (const std::bad_alloc &) {
        return evolve_error(EBIC_E_NOMEM, "out of host memory");
    }
}

ebic_status ebic_evolve(ebic_ctx *ctx, uint64_t seed, int32_t generations,
                        const ebic_evolve_params *params, ebic_result **out) {
    if (!ctx) return evolve_error(EBIC_E_ARG, "ctx is null");
    ebic_ctx_info info;
    info.struct_size = sizeof(info);
    ebic_status st = ebic_get_info(ctx, &info);
    if (st != EBIC_OK) return st;
    return ebic_evolve_with(ctx_eval, ctx, info.n_rows, info.n_cols, seed, generations, params,
                            out);
}

int32_t ebic_result_size(const ebic_result *r) { return r ? (int32_t)r->cols.size() : 0; }

ebic_status ebic_result_get(const ebic_result *r, int32_t i, const int32_t **cols, int32_t *len,
                            int32_t *count, double *fitness, const uint64_t **row_mask) {
    if (!r || i < 0 || i >= (int32_t)r->cols.size())
        return evolve_error(EBIC_E_ARG, "no such result entry");
    if (cols) *cols = r->cols[(size_t)i].data();
    if (len) *len = (int32_t)r->cols[(size_t)i].size();
    if (count) *count = r->counts[(size_t)i];
    if (fitness) *fitness = r->fit[(size_t)i];
    if (row_mask) *row_mask = r->masks[(size_t)i].data();
    return EBIC_OK;
}

ebic_status ebic_result_stats(const ebic_result *r, ebic_run_stats *stats) {
    if (!r || !stats || stats->struct_size < sizeof(ebic_run_stats))
        return evolve_error(EBIC_E_ARG, "null argument or struct_size too small");
    *stats = r->stats;
    return EBIC_OK;
}

void ebic_result_free(ebic_result *r) { delete r; }

}  // extern "C"

extern "C" ebic_status ebic_evolve_screened_with(ebic_eval_fn eval, void *eval_user,
                                                 ebic_score_fn score, void *score_user,
                                                 int64_t n_rows, int32_t n_cols, uint64_t seed,
                                                 int32_t generations, int32_t oversample,
                                                 int32_t warmup_generations, int32_t host_threads,
                                                 const ebic_evolve_params *params,
                                                 ebic_result **out) {
    if (!eval || !score || !out) return evolve_error(EBIC_E_ARG, "eval, score and out must not be null");
    if (generations < 0 || oversample < 1 || warmup_generations < 0)
        return evolve_error(EBIC_E_ARG, "need generations >= 0, oversample >= 1, warmup >= 0");
    ebic_status st = check_params(params, n_rows, n_cols);
    if (st != EBIC_OK) return st;
    *out = nullptr;
    Evaluator ev{eval, eval_user};
    auto scorer = [&](const Pop &pool, ebic_status *st) {
        std::vector<double> sc((size_t)pool.size(), -INFINITY);
        ebic_status e = score(score_user, pool.off.data(), pool.cols.data(), pool.size(), sc.data());
        if (e != EBIC_OK) *st = e;
        return sc;
    };
    return run_screened(ev, scorer, n_rows, n_cols, seed, generations, oversample,
                        warmup_generations, host_threads, *params, out);
}

extern "C" ebic_status ebic_evolve_oversampled(ebic_ctx *ctx, uint64_t seed, int32_t generations,
                                               int32_t oversample, int32_t warmup_generations,
                                               const ebic_evolve_params *params,
                                               ebic_result **out) {
    if (!ctx || !out) return evolve_error(EBIC_E_ARG, "ctx and out must not be null");
    if (generations < 0 || oversample < 1 || warmup_generations < 0)
        return evolve_error(EBIC_E_ARG, "need generations >= 0, oversample >= 1, warmup >= 0");
    ebic_ctx_info info{};
    info.struct_size = sizeof(info);
    ebic_status st = ebic_get_info(ctx, &info);
    if (st != EBIC_OK) return st;
    if ((st = check_params(params, info.n_rows, info.n_cols)) != EBIC_OK) return st;
    *out = nullptr;
    Evaluator ev{ctx_eval, ctx};
    // The pool is ranked by its exact fitness (evaluation-time parameters),
    // evaluated on the GPU like any population.
    ebic_params ep = params->eval;
    ep.want_masks = 0;
    std::vector<int32_t> cnt;
    auto scorer = [&](const Pop &pool, ebic_status *sst) {
        std::vector<double> sc((size_t)pool.size(), -INFINITY);
        cnt.resize((size_t)pool.size());
        const auto t0 = Clock::now();
        ebic_status e = pool.size() > 0
                            ? ebic_evaluate(ctx, pool.off.data(), pool.cols.data(), pool.size(),
                                            &ep, nullptr, cnt.data(), sc.data())
                            : EBIC_OK;
        ev.ms += ms_since(t0);
        ev.evaluated += pool.size();
        if (e != EBIC_OK) *sst = e;
        return sc;
    };
    return run_screened(ev, scorer, info.n_rows, info.n_cols, seed, generations, oversample,
                        warmup_generations, 0, *params, out);
}
