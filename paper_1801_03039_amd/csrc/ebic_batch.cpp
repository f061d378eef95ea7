// Batched EBIC: many independent runs, one GPU launch per generation.
//
// Each run owns a context (its matrix, pairwise order index and ln table).
// Per generation every active run builds its population on a host thread
// (Steps 1-3); the new members of all runs are packed into one CBF with
// global offsets, a run table describes where each run's candidates,
// matrix index and outputs are, and one kernel covers the (run, candidate,
// 64-row word) tiles (Step 4).  The run table lives in device memory and is
// rewritten by one copy per generation; the kernel is launched directly or
// as a captured one-node HIP graph replayed each generation (use_graph),
// with the CBF and results moving by stream-ordered copies around it.
// Step 5 then runs per
// run on host threads.  Every run is exactly ebic_evolve on its own
// context: same seed, same draws, same scores.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ebic_internal.h"
#include "ebic_run.h"

using namespace ebic;
using namespace ebic::host;

struct ebic_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<ebic_ctx *> ctx;
    // 1: the run's matrix has no order index (over its budget, or no device
    // memory for it); it is evaluated by the direct kernel
    std::vector<uint8_t> direct;
    // device buffers
    IndexRun *d_runs = nullptr;          // run table, then the tile bases (one allocation)
    uint32_t *d_tile_base = nullptr;     // inside the d_runs allocation
    unsigned int *d_work = nullptr;
    int32_t *d_off = nullptr, *d_cols = nullptr, *d_counts = nullptr;
    double *d_fit = nullptr;
    unsigned long long *d_acc = nullptr;
    uint64_t *d_masks = nullptr;
    int64_t cap_cand = 0, cap_cols = 0, cap_masks = 0;
    // pinned host staging
    IndexRun *h_runs = nullptr;          // same layout as d_runs
    uint32_t *h_tile_base = nullptr;
    int32_t *h_off = nullptr, *h_cols = nullptr, *h_counts = nullptr;
    double *h_fit = nullptr;
    int64_t hcap_cand = 0, hcap_cols = 0;
    // launch shape and its graph
    int32_t resident_wgs = 0;       // workgroups resident at once (occupancy x CUs)
    int32_t workgroups = 0, unroll = 4, words = 1, whole = 0, use_graph = 0;
    uint64_t static_grid = 0;   // grid of the queue-free mode (largest tile count so far)
    double tuned_ms = 0.0;
    bool tuned = false;
    hipGraphExec_t exec = nullptr;
    BatchLaunch graph_key{};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // around the last graph launch
    double last_ms = 0.0;
    BatchLaunch last_launch{};   // the last launch (replayed by ebic_batch_time_replays)
    bool has_last = false;
};

namespace {

// Host-array calls check and pack the runs' columns on up to kPackThreads
// threads once they hold kPackParallelCols columns or more.
constexpr int32_t kPackThreads = 8;
constexpr int64_t kPackParallelCols = int64_t(1) << 17;

ebic_status bfail(ebic_status st, const std::string &msg) {
    set_thread_error(msg.c_str());
    return st;
}

ebic_status bhip(hipError_t e, const char *what) {
    return bfail(e == hipErrorOutOfMemory ? EBIC_E_NOMEM : EBIC_E_DEVICE,
                 std::string(what) + ": " + hipGetErrorString(e));
}

#define BHIP(expr)                                     \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return bhip(_e, #expr);  \
    } while (0)

void drop_graph(ebic_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
}

template <typename T>
ebic_status dgrow(ebic_batch *b, T *&p, int64_t need, int64_t &cap, bool zero) {
    if (need <= cap) return EBIC_OK;
    const int64_t ncap = std::max<int64_t>(need, cap * 2);
    BHIP(hipStreamSynchronize(b->stream));
    drop_graph(b);  // the graph holds the old pointers
    if (p) BHIP(hipFree(p));
    p = nullptr;
    cap = 0;
    BHIP(hipMalloc((void **)&p, sizeof(T) * (size_t)ncap));
    if (zero) BHIP(hipMemset(p, 0, sizeof(T) * (size_t)ncap));
    cap = ncap;
    return EBIC_OK;
}

template <typename T>
ebic_status hgrow(ebic_batch *b, T *&p, int64_t need, int64_t &cap) {
    if (need <= cap) return EBIC_OK;
    const int64_t ncap = std::max<int64_t>(need, cap * 2);
    BHIP(hipStreamSynchronize(b->stream));
    if (p) BHIP(hipHostFree(p));
    p = nullptr;
    cap = 0;
    BHIP(hipHostMalloc((void **)&p, sizeof(T) * (size_t)ncap, hipHostMallocDefault));
    cap = ncap;
    return EBIC_OK;
}

// One batched evaluation request: run r evaluates P[r] candidates whose CBF
// is already packed (global offsets) in the pinned staging buffers.
struct Request {
    std::vector<int32_t> P;   // per run
    int64_t n_cand = 0, n_cols = 0;
    const ebic_params *params = nullptr;
    bool masks = false;
};

// Capacity for n candidates / n column entries / mask words.
ebic_status reserve(ebic_batch *b, int64_t n_cand, int64_t n_cols, int64_t n_mask_words) {
    int64_t c1 = b->cap_cand, c2 = b->cap_cand, c3 = b->cap_cand, c4 = b->cap_cand;
    ebic_status st;
    if ((st = dgrow(b, b->d_off, n_cand + 1, c1, false)) != EBIC_OK) return st;
    if ((st = dgrow(b, b->d_counts, n_cand, c2, false)) != EBIC_OK) return st;
    if ((st = dgrow(b, b->d_fit, n_cand, c3, false)) != EBIC_OK) return st;
    if ((st = dgrow(b, b->d_acc, n_cand, c4, true)) != EBIC_OK) return st;
    b->cap_cand = std::min(std::min(c1, c2), std::min(c3, c4));
    if ((st = dgrow(b, b->d_cols, std::max<int64_t>(n_cols, 1), b->cap_cols, false)) != EBIC_OK)
        return st;
    if (n_mask_words &&
        (st = dgrow(b, b->d_masks, n_mask_words, b->cap_masks, false)) != EBIC_OK)
        return st;
    int64_t h1 = b->hcap_cand, h2 = b->hcap_cand, h3 = b->hcap_cand;
    if ((st = hgrow(b, b->h_off, n_cand + 1, h1)) != EBIC_OK) return st;
    if ((st = hgrow(b, b->h_counts, n_cand, h2)) != EBIC_OK) return st;
    if ((st = hgrow(b, b->h_fit, n_cand, h3)) != EBIC_OK) return st;
    b->hcap_cand = std::min(h1, std::min(h2, h3));
    return hgrow(b, b->h_cols, std::max<int64_t>(n_cols, 1), b->hcap_cols);
}

// Bytes of the run table of n runs followed by its n + 1 tile bases.
size_t run_table_bytes(int32_t n_runs) {
    return sizeof(IndexRun) * (size_t)n_runs + sizeof(uint32_t) * ((size_t)n_runs + 1);
}

// Whether run r of request q is evaluated by the batched index kernel (else
// by the direct kernel after it).
bool via_index(const ebic_batch *b, const Request &q, int32_t r) {
    return !b->direct[(size_t)r] && q.params->max_violations <= kIndexMaxViolations;
}

// Fills the run table for a request (tiles of 256 lanes with `words` 64-row
// words each); returns the total number of tiles.  With `whole`, a run
// whose candidates take at most 256 lanes each gets tiles of whole
// candidates (as many as fit); other runs, or all without it, get tiles of
// 256 consecutive (candidate, word-group) items.  Table entries are in tile
// order, which is not run order.
uint64_t fill_runs(ebic_batch *b, const Request &q, int32_t words, int32_t whole) {
    const int32_t R = (int32_t)b->ctx.size();
    std::vector<int64_t> cand((size_t)R), maskw((size_t)R);
    std::vector<int32_t> cpw((size_t)R), order((size_t)R);
    int64_t c0 = 0, m0 = 0;
    for (int32_t r = 0; r < R; ++r) {
        const ebic_ctx *c = b->ctx[(size_t)r];
        cand[(size_t)r] = c0;
        maskw[(size_t)r] = m0;
        c0 += q.P[(size_t)r];
        if (q.masks) m0 += (int64_t)q.P[(size_t)r] * 2 * c->W;
        const uint64_t items = (uint64_t)((c->W + words - 1) / words);
        cpw[(size_t)r] = (whole && items <= 256) ? (int32_t)(256 / items) : 0;
        order[(size_t)r] = r;
    }
    // Runs with more candidates per tile first: such a tile lasts as long as
    // the longest series among its candidates, so these tiles are the long
    // ones, and the launch ends on the short tiles of tall runs (measured
    // 0.1056-0.1077 ms per launch against 0.1093-0.1095 in run order and
    // 0.1104-0.1107 in the reverse order).  Each run's outputs stay where
    // its first candidate and mask word say.
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return std::max(cpw[(size_t)x], 1) > std::max(cpw[(size_t)y], 1);
    });
    uint64_t tiles = 0;
    for (int32_t i = 0; i < R; ++i) {
        const int32_t r = order[(size_t)i];
        ebic_ctx *c = b->ctx[(size_t)r];
        // a directly evaluated run keeps its place in the launch but gets no tiles
        const int32_t P = via_index(b, q, r) ? q.P[(size_t)r] : 0;
        const uint64_t items = (uint64_t)((c->W + words - 1) / words);
        const int32_t k = cpw[(size_t)r];
        b->h_runs[i] = IndexRun{c->d_idx, c->d_tie, c->d_log, c->n, c->W, c->wpad, c->m, P,
                                cand[(size_t)r], maskw[(size_t)r], k, 0};
        b->h_tile_base[i] = (uint32_t)tiles;
        tiles += k ? ((uint64_t)P + k - 1) / k : ((uint64_t)P * items + 255) / 256;
    }
    b->h_tile_base[R] = (uint32_t)tiles;
    return tiles;
}

// workgroups < 0: one workgroup per tile, no queue.  A direct launch has
// exactly one workgroup per tile; a graph launch uses the largest tile count
// seen since the shape was set (the kernel reads the current count, and
// surplus workgroups return at once), so that the captured graph stays valid
// from one generation to the next.
BatchLaunch make_launch(ebic_batch *b, const Request &q, int32_t workgroups, int32_t unroll,
                        int32_t words, uint64_t tiles) {
    BatchLaunch L{};
    L.runs = b->d_runs;
    L.tile_base = b->d_tile_base;
    L.n_runs = (int32_t)b->ctx.size();
    L.work = workgroups < 0 ? nullptr : b->d_work;
    L.offsets = b->d_off;
    L.cols = b->d_cols;
    // Bound for offsets checks: the allocated column buffer (stable across
    // generations, so the captured graph stays valid; the host validated
    // every CBF).
    L.n_entries = b->cap_cols;
    L.sigma = q.params->sigma;
    L.k = q.params->max_violations;
    L.negative = q.params->negative_trends ? 1 : 0;
    L.masks = q.masks ? b->d_masks : nullptr;
    L.acc = b->d_acc;
    L.counts = b->d_counts;
    L.fitness = b->d_fit;
    if (workgroups < 0 && b->use_graph) {
        b->static_grid = std::max<uint64_t>(b->static_grid, tiles);
        L.grid = (uint32_t)b->static_grid;
    } else if (workgroups < 0) {
        L.grid = (uint32_t)tiles;
    } else {
        L.grid = (uint32_t)workgroups;
    }
    L.unroll = unroll;
    L.words = words;
    return L;
}

bool same_graph(const BatchLaunch &a, const BatchLaunch &x) {
    // n_entries is a kernel argument too: the graph is re-made when it changes.
    return a.runs == x.runs && a.tile_base == x.tile_base && a.work == x.work &&
           a.offsets == x.offsets && a.cols == x.cols && a.n_entries == x.n_entries &&
           a.sigma == x.sigma && a.k == x.k && a.negative == x.negative && a.masks == x.masks &&
           a.acc == x.acc && a.counts == x.counts && a.fitness == x.fitness && a.grid == x.grid &&
           a.unroll == x.unroll && a.words == x.words;
}

// Graph = [kernel]; the run table is copied before it on the same stream.
ebic_status launch_graph(ebic_batch *b, const BatchLaunch &L) {
    if (!b->exec || !same_graph(b->graph_key, L)) {
        drop_graph(b);
        hipGraph_t g = nullptr;
        BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_eval_index_batch(L, b->stream);
        hipError_t e2 = hipStreamEndCapture(b->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bhip(e != hipSuccess ? e : e2, "graph capture");
        }
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->exec = nullptr;
            return bhip(e, "hipGraphInstantiate");
        }
        b->graph_key = L;
    }
    BHIP(hipGraphLaunch(b->exec, b->stream));
    return EBIC_OK;
}

ebic_status launch(ebic_batch *b, const BatchLaunch &L) {
    if (b->use_graph) return launch_graph(b, L);
    BHIP(launch_eval_index_batch(L, b->stream));
    return EBIC_OK;
}

// Mean device time of `reps` back-to-back launches of the last request
// (same inputs and outputs; the kernel leaves its queue and accumulators
// as it found them).
ebic_status time_replays(ebic_batch *b, int32_t reps, double *ms_per_launch) {
    if (!b->has_last) return bfail(EBIC_E_ARG, "no batched launch to replay");
    BHIP(hipEventRecord(b->ev0, b->stream));
    for (int32_t i = 0; i < reps; ++i) {
        ebic_status st = launch(b, b->last_launch);
        if (st != EBIC_OK) return st;
    }
    BHIP(hipEventRecord(b->ev1, b->stream));
    BHIP(hipEventSynchronize(b->ev1));
    float ms = 0.f;
    BHIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    *ms_per_launch = (double)ms / reps;
    return EBIC_OK;
}

// Runs one packed request (CBF already in h_off/h_cols, P per run set).
// Results land in h_counts/h_fit (and d_masks when asked).
// Runs evaluated directly (no index, or k above the index kernel's limit)
// get one direct-kernel launch each after the batched launch, on the same
// stream, over their slice of the packed CBF and outputs.
ebic_status run_request(ebic_batch *b, const Request &q, int32_t workgroups, int32_t unroll,
                        int32_t words, int32_t whole, bool copy_back = true) {
    b->has_last = false;
    const uint64_t tiles = fill_runs(b, q, words, whole);
    const int32_t R = (int32_t)b->ctx.size();
    bool any_direct = false;
    for (int32_t r = 0; r < R; ++r) any_direct |= q.P[(size_t)r] > 0 && !via_index(b, q, r);
    if (tiles == 0 && !any_direct) return EBIC_OK;
    if (tiles > 0x7FFFFFFFull)
        return bfail(EBIC_E_ARG, "batched populations too large for one launch; split them");
    BHIP(hipMemcpyAsync(b->d_off, b->h_off, sizeof(int32_t) * (size_t)(q.n_cand + 1),
                        hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->d_cols, b->h_cols, sizeof(int32_t) * (size_t)std::max<int64_t>(q.n_cols, 1),
                        hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->d_runs, b->h_runs, run_table_bytes((int32_t)b->ctx.size()),
                        hipMemcpyHostToDevice, b->stream));
    BHIP(hipEventRecord(b->ev0, b->stream));
    if (tiles > 0) {
        const BatchLaunch L =
            make_launch(b, q, workgroups < 0 ? -1 : std::max(1, workgroups), unroll, words, tiles);
        ebic_status st = launch(b, L);
        if (st != EBIC_OK) return st;
        b->last_launch = L;
        b->has_last = true;
    }
    int64_t cand = 0, maskw = 0;
    for (int32_t r = 0; r < R; ++r) {
        ebic_ctx *c = b->ctx[(size_t)r];
        const int32_t P = q.P[(size_t)r];
        if (P > 0 && !via_index(b, q, r)) {
            EvalArgs e{};
            e.offsets = b->d_off + cand;   // global column positions
            e.cols = b->d_cols;
            e.P = P;
            e.n_entries = b->cap_cols;
            e.sigma = q.params->sigma;
            e.k = q.params->max_violations;
            e.negative = q.params->negative_trends ? 1 : 0;
            e.masks = q.masks ? b->d_masks + maskw : nullptr;
            e.counts = b->d_counts + cand;
            e.fitness = b->d_fit + cand;
            e.logt = c->d_log;
            e.acc = b->d_acc + cand;
            BHIP(launch_eval_direct(c->d_a, c->n, c->npad, c->m, c->W, e, b->stream));
        }
        cand += P;
        if (q.masks) maskw += (int64_t)P * 2 * c->W;
    }
    BHIP(hipEventRecord(b->ev1, b->stream));
    if (copy_back) {
        BHIP(hipMemcpyAsync(b->h_counts, b->d_counts, sizeof(int32_t) * (size_t)q.n_cand,
                            hipMemcpyDeviceToHost, b->stream));
        BHIP(hipMemcpyAsync(b->h_fit, b->d_fit, sizeof(double) * (size_t)q.n_cand,
                            hipMemcpyDeviceToHost, b->stream));
    }
    BHIP(hipStreamSynchronize(b->stream));
    float ms = 0.f;
    BHIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    b->last_ms = ms;
    return EBIC_OK;
}

// Autotuner: times candidate launch shapes on this very request and keeps
// the fastest (mean of back-to-back replays of each shape after one
// launch that uploads its run table).  Shapes differ only in speed: every
// shape computes the same results.
constexpr int32_t kTuneReplays = 5;

ebic_status tune(ebic_batch *b, const Request &q) {
    const uint64_t tiles = fill_runs(b, q, 1, 0);
    if (tiles == 0) return EBIC_OK;
    const int32_t full = b->resident_wgs;
    // persistent grids, and one workgroup per tile without a queue (-1)
    std::vector<int32_t> grids = {std::max(1, full / 2), full, 2 * full, -1};
    const int32_t unrolls[] = {1, 2, 4, 8};
    const int32_t word_counts[] = {1, 2, 4, 8};
    double best = 1e300;
    int32_t best_g = full, best_u = 4, best_v = 1, best_w = 0;
    for (int32_t w = 0; w <= 1; ++w)
    for (int32_t v : word_counts)
    for (int32_t u : unrolls)
        for (int32_t g : grids) {
            if (u * v > kMaxUnrollWords) continue;
            ebic_status st = run_request(b, q, g, u, v, w, false);
            double med = 0.0;
            if (st == EBIC_OK) st = time_replays(b, kTuneReplays, &med);
            if (st != EBIC_OK) return st;
            if (med < best) {
                best = med;
                best_g = g;
                best_u = u;
                best_v = v;
                best_w = w;
            }
        }
    b->workgroups = best_g;
    b->unroll = best_u;
    b->words = best_v;
    b->whole = best_w;
    b->static_grid = 0;
    b->tuned_ms = best;
    b->tuned = true;
    return EBIC_OK;
}

// Packs per-run CBF pieces (offsets local to each piece) into the staging
// buffers with global offsets.
struct Packer {
    ebic_batch *b;
    int64_t cand = 0, cols = 0;
    void add(const int32_t *off, const int32_t *c, int32_t P) {
        const int32_t base = off[0];
        for (int32_t i = 0; i < P; ++i) b->h_off[cand + i] = (int32_t)(cols + off[i] - base);
        const int64_t n = off[P] - base;
        std::copy(c + base, c + base + n, b->h_cols + cols);
        cand += P;
        cols += n;
        b->h_off[cand] = (int32_t)cols;
    }
};

// f(0) .. f(n - 1) on up to `threads` threads; the calling thread takes
// items too, so the loop drains even if a helper thread cannot be started.
template <typename F>
void parallel_for(int32_t n, int32_t threads, F &&f) {
    threads = std::max(1, std::min(threads, n));
    std::atomic<int32_t> next{0};
    auto drain = [&] {
        for (int32_t i; (i = next.fetch_add(1)) < n;) f(i);
    };
    std::vector<std::thread> pool;
    for (int32_t t = 1; t < threads; ++t) {
        try {
            pool.emplace_back(drain);
        } catch (...) {
            break;
        }
    }
    drain();
    for (auto &th : pool) th.join();
}

// Steps 6-7 for every run in one launch (the listed series evaluated with
// the expansion parameters and their row masks), then the runs' results.
ebic_status finish_runs(ebic_batch *b, const ebic_evolve_params *params,
                        const std::vector<std::vector<TopEntry>> &top,
                        const std::vector<int32_t> &gens_run, const std::vector<int32_t> &stopped,
                        int64_t evaluated, double eval_ms,
                        std::chrono::steady_clock::time_point t0, ebic_result **results) {
    const int32_t R = (int32_t)b->ctx.size();
    ebic_params ex = params->expand;
    ex.want_masks = 1;
    Request q;
    q.params = &ex;
    q.masks = true;
    q.P.assign((size_t)R, 0);
    int64_t n_cols = 0, n_mask = 0;
    std::vector<Pop> tops((size_t)R);
    for (int32_t r = 0; r < R; ++r) {
        for (const TopEntry &e : top[(size_t)r]) tops[(size_t)r].push(e.s.data(), (int32_t)e.s.size());
        q.P[(size_t)r] = tops[(size_t)r].size();
        q.n_cand += q.P[(size_t)r];
        n_cols += tops[(size_t)r].off.back();
        n_mask += (int64_t)q.P[(size_t)r] * 2 * b->ctx[(size_t)r]->W;
    }
    q.n_cols = n_cols;
    ebic_status st = reserve(b, std::max<int64_t>(q.n_cand, 1), n_cols, std::max<int64_t>(n_mask, 1));
    if (st != EBIC_OK) return st;
    Packer pk{b};
    b->h_off[0] = 0;
    for (int32_t r = 0; r < R; ++r)
        if (q.P[(size_t)r]) pk.add(tops[(size_t)r].off.data(), tops[(size_t)r].cols.data(), q.P[(size_t)r]);
    const auto e0 = std::chrono::steady_clock::now();
    if (q.n_cand && (st = run_request(b, q, b->workgroups, b->unroll, b->words, b->whole)) != EBIC_OK) return st;
    std::vector<uint64_t> all_masks((size_t)std::max<int64_t>(n_mask, 1));
    if (n_mask)
        BHIP(hipMemcpy(all_masks.data(), b->d_masks, sizeof(uint64_t) * (size_t)n_mask,
                       hipMemcpyDeviceToHost));
    eval_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - e0).count();
    evaluated += q.n_cand;
    const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int64_t cand = 0, mw = 0;
    std::vector<ebic_result *> out((size_t)R, nullptr);
    for (int32_t r = 0; r < R; ++r) {
        const int32_t K = q.P[(size_t)r];
        const int64_t W = b->ctx[(size_t)r]->W;
        std::vector<uint64_t> m(all_masks.begin() + mw, all_masks.begin() + mw + (int64_t)K * 2 * W);
        std::vector<int32_t> rc(b->h_counts + cand, b->h_counts + cand + K);
        std::vector<double> rf(b->h_fit + cand, b->h_fit + cand + K);
        out[(size_t)r] = make_result(top[(size_t)r], W, m, std::move(rc), std::move(rf));
        if (!out[(size_t)r]) {
            for (ebic_result *x : out) ebic_result_free(x);
            return bfail(EBIC_E_NOMEM, "cannot allocate results");
        }
        ebic_run_stats &s = out[(size_t)r]->stats;
        s.struct_size = sizeof(ebic_run_stats);
        s.generations_run = gens_run[(size_t)r];
        s.stopped_by_tabu = stopped[(size_t)r];
        s.candidates_evaluated = evaluated;     // whole batch
        s.wall_ms = wall;                       // whole batch
        s.eval_ms = eval_ms;
        s.host_ms = wall - eval_ms;
        cand += K;
        mw += (int64_t)K * 2 * W;
    }
    for (int32_t r = 0; r < R; ++r) results[r] = out[(size_t)r];
    return EBIC_OK;
}

}  // namespace

extern "C" {

ebic_status ebic_batch_create(int32_t n_runs, const float *const *matrices, const int64_t *n_rows,
                              const int32_t *n_cols, int32_t device, ebic_batch **out) {
    if (!out || n_runs < 1 || !matrices || !n_rows || !n_cols)
        return bfail(EBIC_E_ARG, "need n_runs >= 1 and non-null arrays");
    *out = nullptr;
    std::unique_ptr<ebic_batch> b(new (std::nothrow) ebic_batch());
    if (!b) return bfail(EBIC_E_NOMEM, "cannot allocate batch");
    b->device = device;
    auto cleanup = [&](ebic_status st) {
        ebic_batch_destroy(b.release());
        return st;
    };
    for (int32_t r = 0; r < n_runs; ++r) {
        ebic_ctx *c = nullptr;
        ebic_status st = ebic_create(matrices[r], n_rows[r], n_cols[r], n_cols[r], EBIC_ROW_MAJOR,
                                     device, &c);
        if (st != EBIC_OK) return cleanup(st);
        b->ctx.push_back(c);
        // A matrix whose index exceeds its context's budget, or does not fit
        // in device memory, is evaluated by the direct kernel instead.
        uint8_t direct = c->idx_bytes > c->idx_budget ? 1 : 0;
        if (!direct) {
            st = ensure_index(c);
            if (st == EBIC_E_NOMEM) {
                direct = 1;
            } else if (st != EBIC_OK) {
                set_thread_error(c->err.c_str());
                return cleanup(st);
            }
        }
        b->direct.push_back(direct);
    }
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&b->ev0);
    if (e == hipSuccess) e = hipEventCreate(&b->ev1);
    if (e != hipSuccess) return cleanup(bhip(e, "batch stream"));
    // The run table and the tile bases share one allocation on each side,
    // so that one copy node per launch carries both.
    const size_t table = run_table_bytes(n_runs);
    if ((e = hipMalloc((void **)&b->d_runs, table)) != hipSuccess ||
        (e = hipMalloc((void **)&b->d_work, sizeof(unsigned int) * 2)) != hipSuccess ||
        (e = hipMemset(b->d_work, 0, sizeof(unsigned int) * 2)) != hipSuccess ||
        (e = hipHostMalloc((void **)&b->h_runs, table, hipHostMallocDefault)) != hipSuccess)
        return cleanup(bhip(e, "batch buffers"));
    b->d_tile_base = reinterpret_cast<uint32_t *>(b->d_runs + n_runs);
    b->h_tile_base = reinterpret_cast<uint32_t *>(b->h_runs + n_runs);
    int cus = 0;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)) !=
        hipSuccess)
        return cleanup(bhip(e, "hipDeviceGetAttribute"));
    b->resident_wgs = std::max(1, cus * batch_wgs_per_cu());
    b->workgroups = b->resident_wgs;
    *out = b.release();
    return EBIC_OK;
}

ebic_status ebic_batch_destroy(ebic_batch *b) {
    if (!b) return EBIC_OK;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    void *dev[] = {b->d_runs, b->d_work, b->d_off, b->d_cols, b->d_counts,
                   b->d_fit, b->d_acc, b->d_masks};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    void *host[] = {b->h_runs, b->h_off, b->h_cols, b->h_counts, b->h_fit};
    for (void *p : host)
        if (p) (void)hipHostFree(p);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    for (ebic_ctx *c : b->ctx) ebic_destroy(c);
    delete b;
    return EBIC_OK;
}

double ebic_batch_last_ms(const ebic_batch *b) { return b ? b->last_ms : 0.0; }

double ebic_batch_index_build_ms(const ebic_batch *b) {
    double ms = 0.0;
    if (b)
        for (const ebic_ctx *c : b->ctx) ms += c->idx_ms;
    return ms;
}

ebic_status ebic_batch_time_replays(ebic_batch *b, int32_t reps, double *ms_per_launch) {
    if (!b || !ms_per_launch || reps < 1) return bfail(EBIC_E_ARG, "null argument or reps < 1");
    BHIP(hipSetDevice(b->device));
    return time_replays(b, reps, ms_per_launch);
}

ebic_status ebic_batch_get_tuning(const ebic_batch *b, ebic_batch_tuning *t) {
    if (!b || !t || t->struct_size < sizeof(ebic_batch_tuning))
        return bfail(EBIC_E_ARG, "null argument or struct_size too small");
    t->workgroups = b->workgroups;
    t->unroll = b->unroll;
    t->best_ms = b->tuned ? b->tuned_ms : 0.0;
    t->words_per_lane = b->words;
    t->whole_candidates = b->whole;
    t->use_graph = b->use_graph;
    return EBIC_OK;
}

ebic_status ebic_batch_set_tuning(ebic_batch *b, const ebic_batch_tuning *t) {
    if (!b || !t || t->struct_size < sizeof(ebic_batch_tuning))
        return bfail(EBIC_E_ARG, "null argument or struct_size too small");
    if (t->workgroups < -1 || (t->unroll != 1 && t->unroll != 2 && t->unroll != 4 && t->unroll != 8) ||
        (t->words_per_lane != 1 && t->words_per_lane != 2 && t->words_per_lane != 4 &&
         t->words_per_lane != 8) ||
        t->unroll * t->words_per_lane > kMaxUnrollWords ||
        (t->whole_candidates != 0 && t->whole_candidates != 1) ||
        (t->use_graph != 0 && t->use_graph != 1))
        return bfail(EBIC_E_ARG, "workgroups must be >= -1, unroll 1, 2, 4 or 8, words_per_lane "
                                 "1, 2, 4 or 8 with unroll x words_per_lane <= 16, "
                                 "whole_candidates and use_graph 0 or 1");
    b->workgroups = t->workgroups ? t->workgroups : b->resident_wgs;
    b->unroll = t->unroll;
    b->words = t->words_per_lane;
    b->whole = t->whole_candidates;
    b->use_graph = t->use_graph;
    b->static_grid = 0;
    b->tuned = true;
    b->tuned_ms = 0.0;
    return EBIC_OK;
}

ebic_status ebic_batch_evaluate(ebic_batch *b, const int32_t *const *offsets,
                                const int32_t *const *cols, const int32_t *P,
                                const ebic_params *params, uint64_t *const *masks,
                                int32_t *const *counts, double *const *fitness, int32_t tune_now) {
    if (!b || !offsets || !cols || !P || !params || !counts || !fitness)
        return bfail(EBIC_E_ARG, "null argument");
    if (params->struct_size < sizeof(ebic_params)) return bfail(EBIC_E_ARG, "params struct_size");
    if (params->sigma < 0 || params->max_violations < 0)
        return bfail(EBIC_E_RANGE, "sigma and max_violations must be >= 0");
    if (params->want_masks && !masks) return bfail(EBIC_E_ARG, "want_masks needs masks");
    const int32_t R = (int32_t)b->ctx.size();
    Request q;
    q.params = params;
    q.masks = params->want_masks != 0;
    q.P.assign((size_t)R, 0);
    std::vector<int64_t> cand_base((size_t)R, 0), col_base((size_t)R, 0);
    int64_t n_cols = 0, n_mask = 0;
    // Pass 1: counts, pointers and offsets (which size the staging buffers).
    for (int32_t r = 0; r < R; ++r) {
        if (P[r] < 0) return bfail(EBIC_E_ARG, "P must be >= 0");
        if (P[r] == 0) continue;
        ebic_ctx *c = b->ctx[(size_t)r];
        if (!offsets[r] || !cols[r] || !counts[r] || !fitness[r] || (q.masks && !masks[r]))
            return bfail(EBIC_E_ARG, "null per-run array");
        const int32_t *o = offsets[r];
        if (o[0] != 0)
            return bfail(EBIC_E_ARG, "run " + std::to_string(r) + ": offsets[0] must be 0");
        for (int32_t i = 0; i < P[r]; ++i)
            if (o[i + 1] <= o[i])
                return bfail(EBIC_E_ARG, "run " + std::to_string(r) +
                                             ": offsets must increase (every series has L >= 1); "
                                             "candidate " + std::to_string(i));
        if ((int64_t)P[r] * c->W > (int64_t(1) << 32) - 256)
            return bfail(EBIC_E_ARG, "population too large for one launch");
        q.P[(size_t)r] = P[r];
        cand_base[(size_t)r] = q.n_cand;
        col_base[(size_t)r] = n_cols;
        q.n_cand += P[r];
        n_cols += o[P[r]];
        if (q.masks) n_mask += (int64_t)P[r] * 2 * c->W;
    }
    if (n_cols > INT32_MAX || q.n_cand > INT32_MAX)
        return bfail(EBIC_E_ARG, "batched populations hold more than 2^31 - 1 columns; split them");
    q.n_cols = n_cols;
    if (q.n_cand == 0) return EBIC_OK;
    BHIP(hipSetDevice(b->device));
    ebic_status st = reserve(b, q.n_cand, n_cols, n_mask);
    if (st != EBIC_OK) return st;
    // Pass 2: every run's columns checked (range, distinct within a series)
    // and packed into the staging buffers in one pass, runs spread over host
    // threads when there is enough to share; the first failing run (in run
    // order) is reported.
    std::vector<ebic_status> run_st((size_t)R, EBIC_OK);
    auto pack = [&](int32_t r) {
        if (!q.P[(size_t)r]) return;
        ebic_status s = EBIC_OK;
        if (!pack_valid_cbf(b->ctx[(size_t)r], offsets[r], cols[r], q.P[(size_t)r],
                            (int32_t)col_base[(size_t)r], b->h_off + cand_base[(size_t)r],
                            b->h_cols + col_base[(size_t)r], &s))
            run_st[(size_t)r] = s;
    };
    const int32_t threads =
        n_cols < kPackParallelCols
            ? 1
            : std::min<int32_t>({R, kPackThreads,
                                 (int32_t)std::max(1u, std::thread::hardware_concurrency())});
    parallel_for(R, threads, pack);
    for (int32_t r = 0; r < R; ++r)
        if (run_st[(size_t)r] != EBIC_OK) {
            set_thread_error(("run " + std::to_string(r) + ": " + b->ctx[(size_t)r]->err).c_str());
            return run_st[(size_t)r];
        }
    b->h_off[q.n_cand] = (int32_t)n_cols;
    if (tune_now && (st = tune(b, q)) != EBIC_OK) return st;
    if ((st = run_request(b, q, b->workgroups, b->unroll, b->words, b->whole)) != EBIC_OK) return st;
    int64_t cand = 0, mw = 0;
    for (int32_t r = 0; r < R; ++r) {
        const int32_t n = q.P[(size_t)r];
        if (!n) continue;
        std::copy(b->h_counts + cand, b->h_counts + cand + n, counts[r]);
        std::copy(b->h_fit + cand, b->h_fit + cand + n, fitness[r]);
        if (q.masks) {
            const int64_t words = (int64_t)n * 2 * b->ctx[(size_t)r]->W;
            BHIP(hipMemcpy(masks[r], b->d_masks + mw, sizeof(uint64_t) * (size_t)words,
                           hipMemcpyDeviceToHost));
            mw += words;
        }
        cand += n;
    }
    return EBIC_OK;
}

ebic_status ebic_batch_evolve(ebic_batch *b, const uint64_t *seeds, int32_t generations,
                              const ebic_evolve_params *params,
                              ebic_batch_generation_fn on_generation, void *user,
                              int32_t host_threads, ebic_result **results) {
    if (!b || !seeds || !params || !results) return bfail(EBIC_E_ARG, "null argument");
    if (generations < 0) return bfail(EBIC_E_ARG, "generations must be >= 0");
    const int32_t R = (int32_t)b->ctx.size();
    for (int32_t r = 0; r < R; ++r) {
        ebic_status st = check_params(params, b->ctx[(size_t)r]->n, b->ctx[(size_t)r]->m);
        if (st != EBIC_OK) return st;
    }
    if (host_threads <= 0) host_threads = (int32_t)std::max(1u, std::thread::hardware_concurrency());
    BHIP(hipSetDevice(b->device));
    const auto t0 = std::chrono::steady_clock::now();
    double eval_ms = 0.0;
    int64_t evaluated = 0;

    // Per-run parameters: the library calls each run's on_generation with a
    // trampoline that adds the run index and serialises the user callback.
    struct Tramp {
        ebic_batch_generation_fn fn;
        void *user;
        int32_t run;
        std::mutex *mu;
    };
    std::mutex mu;
    std::vector<Tramp> tramps((size_t)R);
    std::vector<ebic_evolve_params> rp((size_t)R, *params);
    std::vector<std::unique_ptr<Run>> runs;
    for (int32_t r = 0; r < R; ++r) {
        tramps[(size_t)r] = Tramp{on_generation, user, r, &mu};
        rp[(size_t)r].on_generation =
            on_generation ? +[](void *u, int32_t gen, const int32_t *off, const int32_t *cols,
                                int32_t P, const int32_t *cnt, const double *fit) {
                auto *t = static_cast<Tramp *>(u);
                std::lock_guard<std::mutex> lk(*t->mu);
                t->fn(t->user, t->run, gen, off, cols, P, cnt, fit);
            }
                          : nullptr;
        rp[(size_t)r].user = &tramps[(size_t)r];
        runs.emplace_back(new Run(b->ctx[(size_t)r]->m, seeds[r], generations, rp[(size_t)r]));
    }
    std::vector<uint8_t> active((size_t)R, 1);
    bool first = true;
    for (;;) {
        parallel_for(R, host_threads, [&](int32_t r) {
            if (active[(size_t)r]) active[(size_t)r] = runs[(size_t)r]->next() ? 1 : 0;
        });
        Request q;
        q.params = &runs[0]->eval_params();
        q.P.assign((size_t)R, 0);
        int64_t n_cols = 0;
        for (int32_t r = 0; r < R; ++r)
            if (active[(size_t)r]) {
                const Pop &pop = runs[(size_t)r]->pending();
                const int32_t f = runs[(size_t)r]->first_new();
                q.P[(size_t)r] = pop.size() - f;
                q.n_cand += q.P[(size_t)r];
                n_cols += pop.off.back() - pop.off[(size_t)f];
            }
        if (q.n_cand == 0) break;
        q.n_cols = n_cols;
        ebic_status st = reserve(b, q.n_cand, n_cols, 0);
        if (st != EBIC_OK) return st;
        Packer pk{b};
        b->h_off[0] = 0;
        for (int32_t r = 0; r < R; ++r)
            if (q.P[(size_t)r]) {
                const Pop &pop = runs[(size_t)r]->pending();
                const int32_t f = runs[(size_t)r]->first_new();
                pk.add(pop.off.data() + f, pop.cols.data(), q.P[(size_t)r]);
            }
        if (first && !b->tuned && (st = tune(b, q)) != EBIC_OK) return st;
        first = false;
        const auto e0 = std::chrono::steady_clock::now();
        if ((st = run_request(b, q, b->workgroups, b->unroll, b->words, b->whole)) != EBIC_OK) return st;
        eval_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - e0).count();
        evaluated += q.n_cand;
        std::vector<int64_t> base((size_t)R + 1, 0);
        for (int32_t r = 0; r < R; ++r) base[(size_t)r + 1] = base[(size_t)r] + q.P[(size_t)r];
        parallel_for(R, host_threads, [&](int32_t r) {
            if (q.P[(size_t)r])
                runs[(size_t)r]->accept(b->h_counts + base[(size_t)r], b->h_fit + base[(size_t)r]);
        });
    }

    std::vector<std::vector<TopEntry>> tops((size_t)R);
    std::vector<int32_t> gens((size_t)R), stopped((size_t)R);
    for (int32_t r = 0; r < R; ++r) {
        tops[(size_t)r] = runs[(size_t)r]->top();
        gens[(size_t)r] = runs[(size_t)r]->generations_run();
        stopped[(size_t)r] = runs[(size_t)r]->stopped() ? 1 : 0;
    }
    return finish_runs(b, params, tops, gens, stopped, evaluated, eval_ms, t0, results);
}

// Device-resident runs (Steps 1-3 and 5 in evolve_steps_kernel): each run
// owns fixed slots -- candidates [r (P + 1), r (P + 1) + P) of the batched
// launch and P * len_max column entries -- so that the run table, tile bases
// and launch arguments stay the same from one generation to the next.
ebic_status ebic_batch_evolve_device(ebic_batch *b, const uint64_t *seeds, int32_t generations,
                                     const ebic_evolve_params *params,
                                     ebic_batch_generation_fn on_generation, void *user,
                                     ebic_result **results) {
    if (!b || !seeds || !params || !results) return bfail(EBIC_E_ARG, "null argument");
    if (generations < 0) return bfail(EBIC_E_ARG, "generations must be >= 0");
    const int32_t R = (int32_t)b->ctx.size();
    int32_t max_m = 0;
    for (int32_t r = 0; r < R; ++r) {
        ebic_status st = check_params(params, b->ctx[(size_t)r]->n, b->ctx[(size_t)r]->m);
        if (st != EBIC_OK) return st;
        max_m = std::max(max_m, b->ctx[(size_t)r]->m);
    }
    if (params->eval.max_violations > kIndexMaxViolations ||
        params->expand.max_violations > kIndexMaxViolations)
        return bfail(EBIC_E_ARG, "device-side steps support max_violations <= 3");
    for (int32_t r = 0; r < R; ++r)
        if (b->direct[(size_t)r])
            return bfail(EBIC_E_ARG, "device-side steps need every run's order index (run " +
                                         std::to_string(r) + " has none)");
    const int32_t P = params->population, slot = params->len_max, K = params->toplist_size;
    int64_t wsum = 0;
    for (int i = 0; i < 5; ++i) wsum += params->op_weight[i];
    if (P > 65535 || slot > 58 || params->tournament > 31 || max_m > 65535 || K > 32767 ||
        wsum > INT32_MAX)
        return bfail(EBIC_E_ARG, "device steps need P <= 65535, len_max <= 58, tournament <= 31, "
                                 "n_cols <= 65535, toplist_size <= 32767, operation weights "
                                 "summing below 2^31");
    const int64_t lds = steps_lds_bytes(P, slot, max_m, K);
    if (lds > 160 * 1024)
        return bfail(EBIC_E_ARG, "device steps: the run's state does not fit in LDS (" +
                                     std::to_string(lds) + " bytes)");
    BHIP(hipSetDevice(b->device));
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t stride = (int64_t)P + 1;          // candidate slots per run
    const int64_t cslots = (int64_t)P * slot;       // column slots per run
    const int64_t entries = (int64_t)P * (generations + 1);
    uint64_t cap = 1024;
    while (cap < 2ull * (uint64_t)entries) cap <<= 1;
    const int64_t arena_cap = entries * slot;
    const int64_t tab_n = (int64_t)P * slot * (slot + 1) / 2 + slot;

    // device buffers, freed on every exit
    std::vector<void *> bufs;
    auto alloc = [&](void **p, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) bufs.push_back(*p);
        return e;
    };
    struct Free {
        std::vector<void *> &v;
        ~Free() {
            for (void *p : v) (void)hipFree(p);
        }
    } free_all{bufs};
    int32_t *d_off = nullptr, *d_cols = nullptr, *d_counts = nullptr, *d_top_cols = nullptr,
            *d_top_len = nullptr, *d_top_cnt = nullptr;
    double *d_fit = nullptr, *d_top_fit = nullptr, *d_pow = nullptr;
    unsigned long long *d_acc = nullptr;
    uint32_t *d_tabu = nullptr, *d_tile_base = nullptr;
    uint16_t *d_arena = nullptr;
    StepsState *d_state = nullptr;
    StepsRun *d_sruns = nullptr;
    IndexRun *d_iruns = nullptr;
    BHIP(alloc((void **)&d_off, sizeof(int32_t) * (size_t)(R * stride)));
    BHIP(alloc((void **)&d_cols, sizeof(int32_t) * (size_t)(R * cslots)));
    BHIP(alloc((void **)&d_counts, sizeof(int32_t) * (size_t)(R * stride)));
    BHIP(alloc((void **)&d_fit, sizeof(double) * (size_t)(R * stride)));
    BHIP(alloc((void **)&d_acc, sizeof(unsigned long long) * (size_t)(R * stride)));
    BHIP(alloc((void **)&d_top_cols, sizeof(int32_t) * (size_t)R * K * slot));
    BHIP(alloc((void **)&d_top_len, sizeof(int32_t) * (size_t)R * K));
    BHIP(alloc((void **)&d_top_cnt, sizeof(int32_t) * (size_t)R * K));
    BHIP(alloc((void **)&d_top_fit, sizeof(double) * (size_t)R * K));
    BHIP(alloc((void **)&d_tabu, sizeof(uint32_t) * 4 * (size_t)cap * R));
    BHIP(alloc((void **)&d_arena, sizeof(uint16_t) * (size_t)arena_cap * R));
    BHIP(alloc((void **)&d_state, sizeof(StepsState) * (size_t)R));
    BHIP(alloc((void **)&d_sruns, sizeof(StepsRun) * (size_t)R));
    BHIP(alloc((void **)&d_pow, sizeof(double) * (size_t)tab_n));
    BHIP(alloc((void **)&d_iruns, sizeof(IndexRun) * (size_t)R));
    BHIP(alloc((void **)&d_tile_base, sizeof(uint32_t) * (size_t)(R + 1)));
    BHIP(hipMemsetAsync(d_acc, 0, sizeof(unsigned long long) * (size_t)(R * stride), b->stream));
    BHIP(hipMemsetAsync(d_tabu, 0, sizeof(uint32_t) * 4 * (size_t)cap * R, b->stream));
    BHIP(hipMemsetAsync(d_off, 0, sizeof(int32_t) * (size_t)(R * stride), b->stream));

    // base^(s / L) for 1 <= L <= len_max, 0 <= s <= L P: the doubles the
    // host path computes with std::pow
    std::vector<double> powtab((size_t)tab_n);
    for (int32_t L = 1; L <= slot; ++L)
        for (int64_t sum = 0; sum <= (int64_t)L * P; ++sum)
            powtab[(size_t)((int64_t)P * L * (L - 1) / 2 + (L - 1) + sum)] =
                std::pow(params->penalty_base, (double)sum / (double)L);
    BHIP(hipMemcpyAsync(d_pow, powtab.data(), sizeof(double) * powtab.size(),
                        hipMemcpyHostToDevice, b->stream));
    std::vector<StepsState> states((size_t)R);
    std::vector<StepsRun> sruns((size_t)R);
    for (int32_t r = 0; r < R; ++r) {
        states[(size_t)r] = StepsState{seeds[r], 0, 0, 0, 0, 0, 0, 0};
        sruns[(size_t)r] = StepsRun{d_off + r * stride, d_cols + r * cslots, r * cslots,
                                    d_counts + r * stride, d_fit + r * stride,
                                    d_top_cols + (int64_t)r * K * slot, d_top_len + (int64_t)r * K,
                                    d_top_cnt + (int64_t)r * K, d_top_fit + (int64_t)r * K,
                                    d_tabu + (size_t)r * cap * 4, cap,
                                    d_arena + (size_t)r * arena_cap, arena_cap, d_state + r,
                                    b->ctx[(size_t)r]->m, 0};
    }
    BHIP(hipMemcpyAsync(d_state, states.data(), sizeof(StepsState) * (size_t)R,
                        hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(d_sruns, sruns.data(), sizeof(StepsRun) * (size_t)R,
                        hipMemcpyHostToDevice, b->stream));

    // the evaluation's run table: P candidates per run at stride P + 1
    const int32_t words = b->tuned ? b->words : 8;
    const int32_t unroll = b->tuned ? b->unroll : 2;
    const int32_t whole = b->tuned ? b->whole : 1;
    std::vector<IndexRun> iruns((size_t)R);
    std::vector<uint32_t> tile_base((size_t)R + 1);
    uint64_t tiles = 0;
    for (int32_t r = 0; r < R; ++r) {
        ebic_ctx *c = b->ctx[(size_t)r];
        const uint64_t items = (uint64_t)((c->W + words - 1) / words);
        const int32_t cpw = (whole && items <= 256) ? (int32_t)(256 / items) : 0;
        iruns[(size_t)r] = IndexRun{c->d_idx, c->d_tie, c->d_log, c->n, c->W, c->wpad, c->m, P,
                                    r * stride, 0, cpw, 0};
        tile_base[(size_t)r] = (uint32_t)tiles;
        tiles += cpw ? ((uint64_t)P + cpw - 1) / cpw : ((uint64_t)P * items + 255) / 256;
    }
    tile_base[(size_t)R] = (uint32_t)tiles;
    if (tiles > 0x7FFFFFFFull) return bfail(EBIC_E_ARG, "batched populations too large for one launch");
    BHIP(hipMemcpyAsync(d_iruns, iruns.data(), sizeof(IndexRun) * (size_t)R, hipMemcpyHostToDevice,
                        b->stream));
    BHIP(hipMemcpyAsync(d_tile_base, tile_base.data(), sizeof(uint32_t) * (size_t)(R + 1),
                        hipMemcpyHostToDevice, b->stream));
    BatchLaunch L{};
    L.runs = d_iruns;
    L.tile_base = d_tile_base;
    L.n_runs = R;
    L.work = nullptr;
    L.offsets = d_off;
    L.cols = d_cols;
    L.n_entries = R * cslots;
    L.sigma = params->eval.sigma;
    L.k = params->eval.max_violations;
    L.negative = params->eval.negative_trends ? 1 : 0;
    L.masks = nullptr;
    L.acc = d_acc;
    L.counts = d_counts;
    L.fitness = d_fit;
    L.grid = (uint32_t)tiles;
    L.unroll = unroll;
    L.words = words;

    StepsArgs A{};
    A.runs = d_sruns;
    A.powtab = d_pow;
    A.n_runs = R;
    A.P = P;
    A.len_min = params->len_min;
    A.len_max = params->len_max;
    A.slot = slot;
    A.tournament = params->tournament;
    A.wsum = 0;
    for (int i = 0; i < 5; ++i) {
        A.op_weight[i] = params->op_weight[i];
        A.wsum += params->op_weight[i];
    }
    A.elite_num = params->elite_num;
    A.elite_den = params->elite_den;
    A.K = K;
    A.tabu_limit = params->tabu_limit < 0 ? P : params->tabu_limit;
    A.theta = params->overlap;
    A.lds_bytes = (int32_t)lds;

    // host copies for on_generation
    std::vector<int32_t> h_off, h_cols, h_cnt;
    std::vector<double> h_fit;
    auto report = [&](int32_t gen) -> ebic_status {
        if (!on_generation) return EBIC_OK;
        BHIP(hipMemcpyAsync(states.data(), d_state, sizeof(StepsState) * (size_t)R,
                            hipMemcpyDeviceToHost, b->stream));
        h_off.resize((size_t)(R * stride));
        h_cols.resize((size_t)(R * cslots));
        h_cnt.resize((size_t)(R * stride));
        h_fit.resize((size_t)(R * stride));
        BHIP(hipMemcpyAsync(h_off.data(), d_off, sizeof(int32_t) * h_off.size(), hipMemcpyDeviceToHost, b->stream));
        BHIP(hipMemcpyAsync(h_cols.data(), d_cols, sizeof(int32_t) * h_cols.size(), hipMemcpyDeviceToHost, b->stream));
        BHIP(hipMemcpyAsync(h_cnt.data(), d_counts, sizeof(int32_t) * h_cnt.size(), hipMemcpyDeviceToHost, b->stream));
        BHIP(hipMemcpyAsync(h_fit.data(), d_fit, sizeof(double) * h_fit.size(), hipMemcpyDeviceToHost, b->stream));
        BHIP(hipStreamSynchronize(b->stream));
        std::vector<int32_t> off((size_t)P + 1);
        for (int32_t r = 0; r < R; ++r) {
            const StepsState &s = states[(size_t)r];
            if (s.stopped || s.error || s.gen != gen) continue;
            for (int32_t i = 0; i <= P; ++i)
                off[(size_t)i] = h_off[(size_t)(r * stride + i)] - (int32_t)(r * cslots);
            on_generation(user, r, gen, off.data(), h_cols.data() + r * cslots, P,
                          h_cnt.data() + r * stride, h_fit.data() + r * stride);
        }
        return EBIC_OK;
    };

    hipEvent_t e0 = nullptr, e1 = nullptr;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t &a, &b;
        ~Ev() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev_guard{e0, e1};
    BHIP(hipEventRecord(e0, b->stream));
    ebic_status st;
    for (int32_t g = 0; g <= generations; ++g) {
        A.mode = g == 0 ? 0 : 1;
        BHIP(launch_steps(A, b->stream));
        BHIP(launch_eval_index_batch(L, b->stream));
        if ((st = report(g)) != EBIC_OK) return st;
    }
    A.mode = 2;
    BHIP(launch_steps(A, b->stream));
    BHIP(hipEventRecord(e1, b->stream));
    BHIP(hipEventSynchronize(e1));
    float dev_ms = 0.f;
    BHIP(hipEventElapsedTime(&dev_ms, e0, e1));

    // the runs' top-rank lists
    BHIP(hipMemcpy(states.data(), d_state, sizeof(StepsState) * (size_t)R, hipMemcpyDeviceToHost));
    std::vector<int32_t> t_cols((size_t)R * K * slot), t_len((size_t)R * K), t_cnt((size_t)R * K);
    std::vector<double> t_fit((size_t)R * K);
    BHIP(hipMemcpy(t_cols.data(), d_top_cols, sizeof(int32_t) * t_cols.size(), hipMemcpyDeviceToHost));
    BHIP(hipMemcpy(t_len.data(), d_top_len, sizeof(int32_t) * t_len.size(), hipMemcpyDeviceToHost));
    BHIP(hipMemcpy(t_cnt.data(), d_top_cnt, sizeof(int32_t) * t_cnt.size(), hipMemcpyDeviceToHost));
    BHIP(hipMemcpy(t_fit.data(), d_top_fit, sizeof(double) * t_fit.size(), hipMemcpyDeviceToHost));
    std::vector<std::vector<TopEntry>> tops((size_t)R);
    std::vector<int32_t> gens((size_t)R), stopped((size_t)R);
    for (int32_t r = 0; r < R; ++r) {
        const StepsState &s = states[(size_t)r];
        if (s.error) return bfail(EBIC_E_STATE, "device steps: tabu table or arena full in run " + std::to_string(r));
        for (int32_t e = 0; e < s.n_top; ++e) {
            const size_t at = (size_t)r * K + e;
            const int32_t *c = t_cols.data() + at * slot;
            tops[(size_t)r].push_back(TopEntry{std::vector<int32_t>(c, c + t_len[at]), t_cnt[at], t_fit[at]});
        }
        gens[(size_t)r] = s.gens_run;
        stopped[(size_t)r] = s.stopped;
    }
    return finish_runs(b, params, tops, gens, stopped, (int64_t)R * P * (generations + 1),
                       (double)dev_ms, t0, results);
}

}  // extern "C"
