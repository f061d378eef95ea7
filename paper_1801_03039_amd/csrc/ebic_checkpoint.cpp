// Stateful EBIC runs with checkpoints: the run of ebic_evolve advanced a
// few generations at a time, saved between generations to bytes and
// resumed from them with the same result as an uninterrupted run.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "ebic_run.h"

using namespace ebic::host;

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

constexpr char kMagic[8] = {'E', 'B', 'I', 'C', 'R', 'U', 'N', '1'};
constexpr uint32_t kVersion = 1;

ebic_status ctx_eval(void *user, const int32_t *offsets, const int32_t *cols, int32_t P,
                     const ebic_params *p, uint64_t *masks, int32_t *counts, double *fitness) {
    return ebic_evaluate(static_cast<ebic_ctx *>(user), offsets, cols, P, p, masks, counts,
                         fitness);
}

// The parameters that decide a run's draws, written into the checkpoint so
// that a resume under other parameters is refused.
void put_params(Writer &w, const ebic_evolve_params &p) {
    w.put(p.population);
    w.put(p.len_min);
    w.put(p.len_max);
    w.put(p.tournament);
    for (int i = 0; i < 5; ++i) w.put(p.op_weight[i]);
    w.put(p.elite_num);
    w.put(p.elite_den);
    w.put(p.penalty_base);
    w.put(p.overlap);
    w.put(p.toplist_size);
    w.put(p.tabu_limit);
    for (const ebic_params *t : {&p.eval, &p.expand}) {
        w.put(t->sigma);
        w.put(t->max_violations);
        w.put(t->negative_trends);
    }
}

}  // namespace

struct ebic_run {
    ebic_eval_fn fn = nullptr;
    void *user = nullptr;
    ebic_ctx *ctx = nullptr;
    ebic_evolve_params p{};
    int64_t n_rows = 0;
    int32_t M = 0;
    std::unique_ptr<Run> run;
    double eval_ms = 0.0, wall_ms = 0.0;
    int64_t evaluated = 0;
    std::vector<int32_t> off, cnt;
    std::vector<double> fit;

    // Scores members [first, size) of `pop` (offsets re-based to 0).
    ebic_status eval(const Pop &pop, int32_t first, const ebic_params *prm, uint64_t *masks,
                     int32_t *counts, double *fitness) {
        const int32_t P = pop.size() - first;
        if (P <= 0) return EBIC_OK;
        off.resize((size_t)P + 1);
        const int32_t base = pop.off[(size_t)first];
        for (int32_t i = 0; i <= P; ++i) off[(size_t)i] = pop.off[(size_t)(first + i)] - base;
        const auto t0 = Clock::now();
        ebic_status st = fn(user, off.data(), pop.cols.data() + base, P, prm, masks, counts,
                            fitness);
        eval_ms += ms_since(t0);
        evaluated += P;
        return st;
    }
};

namespace {

ebic_status new_run(ebic_eval_fn fn, void *user, ebic_ctx *ctx, int64_t n_rows, int32_t n_cols,
                    uint64_t seed, int32_t generations, const ebic_evolve_params *params,
                    ebic_run **out) {
    if (!fn || !out) return evolve_error(EBIC_E_ARG, "evaluator and out must not be null");
    if (generations < 0) return evolve_error(EBIC_E_ARG, "generations must be >= 0");
    ebic_status st = check_params(params, n_rows, n_cols);
    if (st != EBIC_OK) return st;
    *out = nullptr;
    std::unique_ptr<ebic_run> r(new (std::nothrow) ebic_run());
    if (!r) return evolve_error(EBIC_E_NOMEM, "cannot allocate run");
    r->fn = fn;
    r->user = user;
    r->ctx = ctx;
    r->p = *params;
    r->n_rows = n_rows;
    r->M = n_cols;
    r->run.reset(new (std::nothrow) Run(n_cols, seed, generations, r->p));
    if (!r->run) return evolve_error(EBIC_E_NOMEM, "cannot allocate run");
    *out = r.release();
    return EBIC_OK;
}

ebic_status ctx_shape(ebic_ctx *ctx, int64_t *n_rows, int32_t *n_cols) {
    if (!ctx) return evolve_error(EBIC_E_ARG, "ctx is null");
    ebic_ctx_info info{};
    info.struct_size = sizeof(info);
    ebic_status st = ebic_get_info(ctx, &info);
    if (st != EBIC_OK) return st;
    *n_rows = info.n_rows;
    *n_cols = info.n_cols;
    return EBIC_OK;
}

}  // namespace

extern "C" {

ebic_status ebic_run_create(ebic_ctx *ctx, uint64_t seed, int32_t generations,
                            const ebic_evolve_params *params, ebic_run **out) {
    int64_t n = 0;
    int32_t m = 0;
    ebic_status st = ctx_shape(ctx, &n, &m);
    if (st != EBIC_OK) return st;
    return new_run(ctx_eval, ctx, ctx, n, m, seed, generations, params, out);
}

ebic_status ebic_run_create_with(ebic_eval_fn eval, void *eval_user, int64_t n_rows,
                                 int32_t n_cols, uint64_t seed, int32_t generations,
                                 const ebic_evolve_params *params, ebic_run **out) {
    return new_run(eval, eval_user, nullptr, n_rows, n_cols, seed, generations, params, out);
}

ebic_status ebic_run_advance(ebic_run *r, int32_t max_generations, int32_t *finished) {
    if (!r || max_generations < 0) return evolve_error(EBIC_E_ARG, "null run or negative count");
    const auto t0 = Clock::now();
    Run &run = *r->run;
    bool done = false;
    for (int32_t g = 0; g < max_generations; ++g) {
        if (!run.next()) {
            done = true;
            break;
        }
        const Pop &pop = run.pending();
        const int32_t first = run.first_new();
        r->cnt.resize((size_t)(pop.size() - first));
        r->fit.resize(r->cnt.size());
        ebic_status st = r->eval(pop, first, &run.eval_params(), nullptr, r->cnt.data(),
                                 r->fit.data());
        if (st != EBIC_OK) return st;
        run.accept(r->cnt.data(), r->fit.data());
    }
    if (!done) done = run.stopped() || run.generation() > run.generations();
    r->wall_ms += ms_since(t0);
    if (finished) *finished = done ? 1 : 0;
    return EBIC_OK;
}

ebic_status ebic_run_get_progress(const ebic_run *r, ebic_run_progress *out) {
    if (!r || !out || out->struct_size < sizeof(ebic_run_progress))
        return evolve_error(EBIC_E_ARG, "null argument or struct_size too small");
    const Run &run = *r->run;
    out->next_generation = run.generation();
    out->generations_run = run.generations_run();
    out->stopped_by_tabu = run.stopped() ? 1 : 0;
    out->toplist = (int32_t)run.top().size();
    out->best_fitness = run.top().empty() ? 0.0 : run.top()[0].fit;
    out->tabu_size = (int64_t)run.tabu_size();
    out->candidates_evaluated = r->evaluated;
    out->eval_ms = r->eval_ms;
    out->wall_ms = r->wall_ms;
    return EBIC_OK;
}

ebic_status ebic_run_save(const ebic_run *r, void *buf, int64_t capacity, int64_t *size) {
    if (!r || !size || capacity < 0) return evolve_error(EBIC_E_ARG, "null argument");
    std::vector<uint8_t> b;
    Writer w{b};
    for (char c : kMagic) w.put(c);
    w.put(kVersion);
    w.put(r->n_rows);
    w.put(r->M);
    w.put(r->run->generations());
    put_params(w, r->p);
    r->run->save(w);
    *size = (int64_t)b.size();
    if (!buf) return EBIC_OK;
    if (capacity < (int64_t)b.size()) return evolve_error(EBIC_E_RANGE, "buffer too small");
    std::memcpy(buf, b.data(), b.size());
    return EBIC_OK;
}

static ebic_status load_run(ebic_eval_fn fn, void *user, ebic_ctx *ctx, int64_t n_rows,
                            int32_t n_cols, const ebic_evolve_params *params, const void *buf,
                            int64_t size, ebic_run **out) {
    if (!buf || size < 0 || !out) return evolve_error(EBIC_E_ARG, "null argument");
    *out = nullptr;
    Reader rd{static_cast<const uint8_t *>(buf), (size_t)size};
    for (char c : kMagic)
        if (rd.get<char>() != c) return evolve_error(EBIC_E_ARG, "not a run checkpoint");
    if (rd.get<uint32_t>() != kVersion) return evolve_error(EBIC_E_ARG, "unknown checkpoint version");
    const int64_t n = rd.get<int64_t>();
    const int32_t m = rd.get<int32_t>();
    const int32_t generations = rd.get<int32_t>();
    if (!rd.ok || n != n_rows || m != n_cols)
        return evolve_error(EBIC_E_ARG, "checkpoint of a matrix of another shape");
    ebic_run *r = nullptr;
    ebic_status st = new_run(fn, user, ctx, n_rows, n_cols, 0, generations, params, &r);
    if (st != EBIC_OK) return st;
    std::unique_ptr<ebic_run> hold(r);
    std::vector<uint8_t> mine;
    Writer w{mine};
    put_params(w, *params);
    if (size - (int64_t)rd.at < (int64_t)mine.size() ||
        std::memcmp(rd.p + rd.at, mine.data(), mine.size()) != 0)
        return evolve_error(EBIC_E_ARG, "checkpoint was made with other run parameters");
    rd.at += mine.size();
    if (!r->run->load(rd) || rd.at != rd.n)
        return evolve_error(EBIC_E_ARG, "corrupt run checkpoint");
    *out = hold.release();
    return EBIC_OK;
}

ebic_status ebic_run_load(ebic_ctx *ctx, const ebic_evolve_params *params, const void *buf,
                          int64_t size, ebic_run **out) {
    int64_t n = 0;
    int32_t m = 0;
    ebic_status st = ctx_shape(ctx, &n, &m);
    if (st != EBIC_OK) return st;
    return load_run(ctx_eval, ctx, ctx, n, m, params, buf, size, out);
}

ebic_status ebic_run_load_with(ebic_eval_fn eval, void *eval_user, int64_t n_rows,
                               int32_t n_cols, const ebic_evolve_params *params, const void *buf,
                               int64_t size, ebic_run **out) {
    if (!eval) return evolve_error(EBIC_E_ARG, "eval must not be null");
    return load_run(eval, eval_user, nullptr, n_rows, n_cols, params, buf, size, out);
}

ebic_status ebic_run_result(ebic_run *r, ebic_result **out) {
    if (!r || !out) return evolve_error(EBIC_E_ARG, "null argument");
    *out = nullptr;
    const auto t0 = Clock::now();
    const Run &run = *r->run;
    const int64_t W = (r->n_rows + 63) / 64;
    const std::vector<TopEntry> &top = run.top();
    const int32_t K = (int32_t)top.size();
    std::vector<uint64_t> masks((size_t)K * 2 * (size_t)W);
    std::vector<int32_t> rc((size_t)K);
    std::vector<double> rf((size_t)K);
    if (K > 0) {
        Pop tp;
        for (const TopEntry &e : top) tp.push(e.s.data(), (int32_t)e.s.size());
        ebic_params ex = r->p.expand;
        ex.want_masks = 1;
        ebic_status st = r->eval(tp, 0, &ex, masks.data(), rc.data(), rf.data());
        if (st != EBIC_OK) return st;
    }
    ebic_result *res = make_result(top, W, masks, std::move(rc), std::move(rf));
    if (!res) return evolve_error(EBIC_E_NOMEM, "cannot allocate result");
    r->wall_ms += ms_since(t0);
    res->stats.struct_size = sizeof(ebic_run_stats);
    res->stats.generations_run = run.generations_run();
    res->stats.stopped_by_tabu = run.stopped() ? 1 : 0;
    res->stats.candidates_evaluated = r->evaluated;
    res->stats.wall_ms = r->wall_ms;
    res->stats.eval_ms = r->eval_ms;
    res->stats.host_ms = r->wall_ms - r->eval_ms;
    *out = res;
    return EBIC_OK;
}

void ebic_run_destroy(ebic_run *r) { delete r; }

}  // extern "C"
