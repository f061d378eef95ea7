// Surrogate-screened evolutionary run (not part of the paper's method): the
// MLP of ebic_mlp.cpp ranks oversampled offspring; kept children are scored
// exactly on the GPU evaluator, and the plain run is the fallback whenever
// the model's rank correlation with the exact scores is too low.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <numeric>
#include <vector>

#include "ebic_mlp.h"
#include "ebic_run.h"

using namespace ebic::host;

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Members [first, size) of a population as a CBF starting at offset 0.
void rebase(const Pop &p, int32_t first, std::vector<int32_t> &off, std::vector<int32_t> &cols) {
    const int32_t n = p.size() - first;
    const int32_t base = p.off[(size_t)first];
    off.resize((size_t)n + 1);
    for (int32_t i = 0; i <= n; ++i) off[(size_t)i] = p.off[(size_t)(first + i)] - base;
    cols.assign(p.cols.begin() + base, p.cols.begin() + p.off.back());
}

// Ranks 1..n with ties given their average rank.
std::vector<double> ranks(const std::vector<double> &v) {
    const size_t n = v.size();
    std::vector<size_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return v[a] < v[b]; });
    std::vector<double> r(n);
    for (size_t i = 0; i < n;) {
        size_t j = i;
        while (j + 1 < n && v[idx[j + 1]] == v[idx[i]]) ++j;
        const double avg = 0.5 * (double)(i + j) + 1.0;
        for (size_t k = i; k <= j; ++k) r[idx[k]] = avg;
        i = j + 1;
    }
    return r;
}

double spearman(const std::vector<double> &a, const std::vector<double> &b) {
    const size_t n = a.size();
    if (n < 3) return 0.0;
    const std::vector<double> ra = ranks(a), rb = ranks(b);
    const double ma = std::accumulate(ra.begin(), ra.end(), 0.0) / n;
    const double mb = std::accumulate(rb.begin(), rb.end(), 0.0) / n;
    double sab = 0, saa = 0, sbb = 0;
    for (size_t i = 0; i < n; ++i) {
        sab += (ra[i] - ma) * (rb[i] - mb);
        saa += (ra[i] - ma) * (ra[i] - ma);
        sbb += (rb[i] - mb) * (rb[i] - mb);
    }
    return (saa > 0 && sbb > 0) ? sab / std::sqrt(saa * sbb) : 0.0;
}

struct Batch {
    std::vector<int32_t> off, cols;
    std::vector<float> target;
};

}  // namespace

extern "C" {

void ebic_surrogate_defaults(ebic_surrogate_params *s) {
    if (!s) return;
    *s = ebic_surrogate_params{};
    s->struct_size = sizeof(ebic_surrogate_params);
    s->oversample = 8;
    s->warmup_generations = 3;
    s->train_steps = 16;
    s->replay_generations = 4;
    s->min_rank_corr = 0.1;
    s->check_sample = 512;
    s->exact_rerank = 0;
    s->mlp_seed = 0x5EED;
    ebic_mlp_defaults(&s->mlp);
    s->mlp.lr = 3e-3f;
}

ebic_status ebic_evolve_surrogate(ebic_ctx *ctx, uint64_t seed, int32_t generations,
                                  const ebic_evolve_params *params,
                                  const ebic_surrogate_params *sp, ebic_result **out) {
    if (!ctx || !out || !sp || sp->struct_size < sizeof(ebic_surrogate_params))
        return evolve_error(EBIC_E_ARG, "null argument or struct_size too small");
    if (generations < 0 || sp->oversample < 1 || sp->warmup_generations < 0 ||
        sp->train_steps < 0 || sp->replay_generations < 1)
        return evolve_error(EBIC_E_ARG, "bad surrogate parameters");
    ebic_ctx_info info;
    info.struct_size = sizeof(info);
    ebic_status st = ebic_get_info(ctx, &info);
    if (st != EBIC_OK) return st;
    if ((st = check_params(params, info.n_rows, info.n_cols)) != EBIC_OK) return st;
    *out = nullptr;
    const auto t_start = Clock::now();
    ebic_mlp *net = nullptr;
    if ((st = ebic_mlp_create(info.n_cols, &sp->mlp, sp->mlp_seed, info.device, &net)) != EBIC_OK)
        return st;
    struct NetGuard {
        ebic_mlp *m;
        ~NetGuard() { ebic_mlp_destroy(m); }
    } guard{net};

    double eval_ms = 0.0;
    int64_t evaluated = 0;
    Run run(info.n_cols, seed, generations, *params);
    std::deque<Batch> replay;
    std::vector<int32_t> off, cols, cnt;
    std::vector<double> fit;
    std::vector<float> pred;
    double last_corr = -1.0;
    bool have_corr = false;
    ebic_status score_st = EBIC_OK;
    // The rank check's own stream (the run's stream is not touched).
    SplitMix64 check_rng(seed ^ 0xA5A5A5A5D1B54A32ull);
    std::vector<int32_t> pool_off, pool_cols;   // the last screened pool
    std::vector<float> pool_pred;

    // The report of a generation waits for its training loss, which is read
    // once the next generation has drawn its pool (the training runs on the
    // GPU meanwhile) or after the last generation.
    struct Report {
        bool due = false, trained = false;
        int32_t gen = 0, screened = 0, pool = 0;
        double corr = NAN;
    } report;
    auto flush = [&]() -> ebic_status {
        if (!report.due) return EBIC_OK;
        report.due = false;
        double loss = 0.0;
        if (report.trained) {
            float l = 0.f;
            const ebic_status e = ebic::mlp_last_loss(net, &l);
            if (e != EBIC_OK) return e;
            loss = l;
        }
        if (sp->on_surrogate)
            sp->on_surrogate(sp->user, report.gen, report.screened, report.corr, loss, report.pool);
        return EBIC_OK;
    };

    for (;;) {
        const int32_t gen = run.generation();
        const bool screen = gen > sp->warmup_generations && have_corr && last_corr >= sp->min_rank_corr;
        int32_t pool = 0;
        bool more;
        if (screen) {
            const int32_t need = params->population - run.elites();
            more = run.next_screened(sp->oversample, [&](const Pop &pl) {
                rebase(pl, 0, pool_off, pool_cols);
                if ((score_st = flush()) != EBIC_OK) return std::vector<float>((size_t)pl.size());
                std::vector<float> s((size_t)pl.size(), -INFINITY);
                pool = pl.size();
                ebic_status e = ebic_mlp_predict(net, pool_off.data(), pool_cols.data(),
                                                 pl.size(), s.data());
                if (e != EBIC_OK) score_st = e;
                pool_pred = s;
                const int64_t keep = (int64_t)sp->exact_rerank * need;
                if (e != EBIC_OK || sp->exact_rerank <= 0 || keep >= pl.size()) return s;
                // Two-stage screen: the network's top `keep` children are
                // scored exactly and ranked by that score; the rest rank
                // below them.
                std::vector<int32_t> order((size_t)pl.size());
                std::iota(order.begin(), order.end(), 0);
                // the `keep` best predictions, ties to the earlier child
                std::nth_element(order.begin(), order.begin() + keep, order.end(),
                                 [&](int32_t a, int32_t b) {
                                     return s[(size_t)a] > s[(size_t)b] ||
                                            (s[(size_t)a] == s[(size_t)b] && a < b);
                                 });
                order.resize((size_t)keep);
                std::sort(order.begin(), order.end());
                std::vector<int32_t> ro(1, 0), rc, rcnt((size_t)keep);
                std::vector<double> rfit((size_t)keep);
                for (int32_t k : order) {
                    rc.insert(rc.end(), pool_cols.begin() + pool_off[(size_t)k],
                              pool_cols.begin() + pool_off[(size_t)k + 1]);
                    ro.push_back((int32_t)rc.size());
                }
                const auto r0 = Clock::now();
                e = ebic_evaluate(ctx, ro.data(), rc.data(), (int32_t)keep, &run.eval_params(),
                                  nullptr, rcnt.data(), rfit.data());
                eval_ms += ms_since(r0);
                evaluated += keep;
                if (e != EBIC_OK) {
                    score_st = e;
                    return s;
                }
                std::vector<float> r((size_t)pl.size(), -INFINITY);
                for (size_t i = 0; i < order.size(); ++i) r[(size_t)order[i]] = (float)rfit[i];
                return r;
            });
            if (score_st != EBIC_OK) return score_st;
        } else {
            more = run.next();
        }
        if (!more) break;
        if ((st = flush()) != EBIC_OK) return st;
        const Pop &pop = run.pending();
        const int32_t first = run.first_new();
        const int32_t n = pop.size() - first;
        rebase(pop, first, off, cols);
        // The model's view of the new members before their exact scores
        // (the rank check of a plainly bred generation; a screened one is
        // checked on a sample of its pool).
        double corr = 0.0;
        bool checked = false;
        if (gen > 0 && n > 0 && !(screen && pool > 0 && sp->check_sample > 0)) {
            pred.assign((size_t)n, 0.f);
            if ((st = ebic_mlp_predict(net, off.data(), cols.data(), n, pred.data())) != EBIC_OK)
                return st;
        }
        cnt.resize((size_t)n);
        fit.resize((size_t)n);
        const auto e0 = Clock::now();
        if (n > 0 && (st = ebic_evaluate(ctx, off.data(), cols.data(), n, &run.eval_params(),
                                         nullptr, cnt.data(), fit.data())) != EBIC_OK)
            return st;
        eval_ms += ms_since(e0);
        evaluated += n;
        if (screen && pool > 0 && sp->check_sample > 0) {
            // Judge on a uniform sample of the whole pool, scored exactly: the
            // admitted children alone are a truncated sample whose rank
            // correlation says little about the ranking of the pool.
            const int32_t S = std::min(sp->check_sample, pool);
            std::vector<int32_t> pick((size_t)pool);
            for (int32_t i = 0; i < pool; ++i) pick[(size_t)i] = i;
            for (int32_t i = 0; i < S; ++i) {        // partial Fisher-Yates
                const int32_t j = i + (int32_t)check_rng.below((uint64_t)(pool - i));
                std::swap(pick[(size_t)i], pick[(size_t)j]);
            }
            std::vector<int32_t> so(1, 0), sc, scnt((size_t)S);
            std::vector<double> sfit((size_t)S), spd((size_t)S);
            for (int32_t i = 0; i < S; ++i) {
                const int32_t k = pick[(size_t)i];
                sc.insert(sc.end(), pool_cols.begin() + pool_off[(size_t)k],
                          pool_cols.begin() + pool_off[(size_t)k + 1]);
                so.push_back((int32_t)sc.size());
                spd[(size_t)i] = pool_pred[(size_t)k];
            }
            const auto j0 = Clock::now();
            if ((st = ebic_evaluate(ctx, so.data(), sc.data(), S, &run.eval_params(), nullptr,
                                    scnt.data(), sfit.data())) != EBIC_OK)
                return st;
            eval_ms += ms_since(j0);
            evaluated += S;
            corr = spearman(spd, sfit);
            checked = true;
        } else if (gen > 0 && n > 0) {
            std::vector<double> pd(pred.begin(), pred.end());
            corr = spearman(pd, fit);
            checked = true;
        }
        run.accept(cnt.data(), fit.data());
        // Train on the exact pairs of the latest generations.
        Batch bt{off, cols, std::vector<float>((size_t)n)};
        for (int32_t i = 0; i < n; ++i) bt.target[(size_t)i] = (float)std::log1p(fit[(size_t)i]);
        if (n > 0) replay.push_back(std::move(bt));
        while ((int32_t)replay.size() > sp->replay_generations) replay.pop_front();
        bool trained = false;
        if (!replay.empty() && sp->train_steps > 0) {
            Batch all;
            all.off.push_back(0);
            for (const Batch &b : replay) {
                const int32_t base = all.off.back();
                for (size_t i = 1; i < b.off.size(); ++i) all.off.push_back(base + b.off[i]);
                all.cols.insert(all.cols.end(), b.cols.begin(), b.cols.end());
                all.target.insert(all.target.end(), b.target.begin(), b.target.end());
            }
            const int32_t B = (int32_t)all.target.size();
            if ((st = ebic_mlp_train(net, all.off.data(), all.cols.data(), B, all.target.data(),
                                     sp->train_steps, nullptr)) != EBIC_OK)
                return st;
            trained = true;
        }
        if (checked) {
            last_corr = corr;
            have_corr = true;
        }
        report = Report{true, trained, gen, screen ? 1 : 0, pool, checked ? corr : NAN};
    }
    if ((st = flush()) != EBIC_OK) return st;

    // Steps 6-7 with the expansion parameters.
    const int64_t W = ebic_mask_words(info.n_rows);
    const std::vector<TopEntry> &top = run.top();
    const int32_t K = (int32_t)top.size();
    std::vector<uint64_t> masks((size_t)K * 2 * (size_t)W);
    std::vector<int32_t> rc((size_t)K);
    std::vector<double> rf((size_t)K);
    if (K > 0) {
        Pop tp;
        for (const TopEntry &e : top) tp.push(e.s.data(), (int32_t)e.s.size());
        ebic_params ex = params->expand;
        ex.want_masks = 1;
        const auto e0 = Clock::now();
        if ((st = ebic_evaluate(ctx, tp.off.data(), tp.cols.data(), K, &ex, masks.data(), rc.data(),
                                rf.data())) != EBIC_OK)
            return st;
        eval_ms += ms_since(e0);
        evaluated += K;
    }
    ebic_result *r = make_result(top, W, masks, std::move(rc), std::move(rf));
    if (!r) return evolve_error(EBIC_E_NOMEM, "cannot allocate result");
    r->stats.struct_size = sizeof(ebic_run_stats);
    r->stats.generations_run = run.generations_run();
    r->stats.stopped_by_tabu = run.stopped() ? 1 : 0;
    r->stats.candidates_evaluated = evaluated;
    r->stats.wall_ms = ms_since(t_start);
    r->stats.eval_ms = eval_ms;
    r->stats.host_ms = r->stats.wall_ms - eval_ms;
    *out = r;
    return EBIC_OK;
}

}  // extern "C"
