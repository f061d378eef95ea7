// Host-side building blocks of EBIC's evolutionary run (Steps 1-3, 5-7):
// random numbers, populations in CBF form, the tabu list, the top-rank list,
// the genetic operations and one run as a state machine.  Shared by the
// single-run driver (ebic_evolve.cpp) and the multi-run driver
// (ebic_batch.cpp).  Internal; not part of the public ABI.
#pragma once

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ebic.h"

namespace ebic {
// Message for ebic_last_error(NULL) (defined with the runtime).
void set_thread_error(const char *msg);
}  // namespace ebic

struct ebic_result {
    std::vector<std::vector<int32_t>> cols;
    std::vector<int32_t> counts;
    std::vector<double> fit;
    std::vector<std::vector<uint64_t>> masks;
    ebic_run_stats stats{};
};


namespace ebic {
namespace host {

inline ebic_status evolve_error(ebic_status st, const char *msg) {
    ebic::set_thread_error(msg);
    return st;
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): Weyl step
// 0x9E3779B97F4A7C15 and the 64-bit mixing finalizer.
struct SplitMix64 {
    uint64_t s;
    explicit SplitMix64(uint64_t seed) : s(seed) {}
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    // Draw in [0, n): plain modulo (the documented reading).
    uint32_t below(uint64_t n) { return (uint32_t)(next() % n); }
};

// Checkpoint bytes: little-endian PODs and vectors (length first).
struct Writer {
    std::vector<uint8_t> &b;
    template <typename T>
    void put(const T &v) {
        const uint8_t *p = reinterpret_cast<const uint8_t *>(&v);
        b.insert(b.end(), p, p + sizeof(T));
    }
    template <typename T>
    void vec(const std::vector<T> &v) {
        put<uint64_t>(v.size());
        const uint8_t *p = reinterpret_cast<const uint8_t *>(v.data());
        b.insert(b.end(), p, p + sizeof(T) * v.size());
    }
};

struct Reader {
    const uint8_t *p;
    size_t n, at = 0;
    bool ok = true;
    template <typename T>
    T get() {
        T v{};
        if (!ok || n - at < sizeof(T)) {
            ok = false;
            return v;
        }
        std::memcpy(&v, p + at, sizeof(T));
        at += sizeof(T);
        return v;
    }
    template <typename T>
    std::vector<T> vec(size_t max_elems) {
        const uint64_t k = get<uint64_t>();
        std::vector<T> v;
        if (!ok || k > max_elems || (n - at) / sizeof(T) < k) {
            ok = false;
            return v;
        }
        v.resize((size_t)k);
        std::memcpy(v.data(), p + at, sizeof(T) * (size_t)k);
        at += sizeof(T) * (size_t)k;
        return v;
    }
};

// A population in CBF form.
struct Pop {
    std::vector<int32_t> off{0};
    std::vector<int32_t> cols;
    std::vector<int32_t> counts;
    std::vector<double> fit;
    int32_t size() const { return (int32_t)off.size() - 1; }
    const int32_t *series(int32_t i) const { return cols.data() + off[(size_t)i]; }
    int32_t len(int32_t i) const { return off[(size_t)i + 1] - off[(size_t)i]; }
    void clear() {
        off.assign(1, 0);
        cols.clear();
        counts.clear();
        fit.clear();
    }
    void push(const int32_t *s, int32_t L) {
        cols.insert(cols.end(), s, s + L);
        off.push_back((int32_t)cols.size());
    }
    void save(Writer &w) const {
        w.vec(off);
        w.vec(cols);
        w.vec(counts);
        w.vec(fit);
    }
    // Loads and checks the CBF shape (offsets from 0, increasing, columns
    // in [0, M), scores for every member).
    bool load(Reader &r, int32_t M) {
        const size_t cap = (size_t)1 << 31;
        off = r.vec<int32_t>(cap);
        cols = r.vec<int32_t>(cap);
        counts = r.vec<int32_t>(cap);
        fit = r.vec<double>(cap);
        if (!r.ok || off.empty() || off[0] != 0 || (size_t)off.back() != cols.size()) return false;
        for (size_t i = 1; i < off.size(); ++i)
            if (off[i] <= off[i - 1]) return false;
        for (int32_t c : cols)
            if (c < 0 || c >= M) return false;
        return counts.size() == off.size() - 1 && fit.size() == counts.size();
    }
};

// Helper threads kept for the whole run: run(n, f) calls f(0) .. f(n - 1)
// on them and on the calling thread, and returns once every call has
// finished.  A helper that cannot be started is left out (the calling
// thread drains whatever remains).
class Helpers {
  public:
    explicit Helpers(int32_t threads) {
        for (int32_t t = 1; t < threads; ++t) {
            try {
                th_.emplace_back([this] { loop(); });
            } catch (...) {
                break;
            }
        }
    }
    ~Helpers() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (std::thread &t : th_) t.join();
    }
    Helpers(const Helpers &) = delete;
    Helpers &operator=(const Helpers &) = delete;

    void run(int32_t n, const std::function<void(int32_t)> &f) {
        {
            std::lock_guard<std::mutex> g(mu_);
            job_ = &f;
            n_ = n;
            next_.store(0);
            busy_ = (int32_t)th_.size();
            ++epoch_;
        }
        cv_.notify_all();
        drain(f, n);
        std::unique_lock<std::mutex> g(mu_);
        done_.wait(g, [this] { return busy_ == 0; });
        job_ = nullptr;
    }

  private:
    void drain(const std::function<void(int32_t)> &f, int32_t n) {
        for (int32_t i; (i = next_.fetch_add(1)) < n;) f(i);
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int32_t)> *f;
            int32_t n;
            {
                std::unique_lock<std::mutex> g(mu_);
                cv_.wait(g, [&] { return stop_ || epoch_ != seen; });
                if (stop_) return;
                seen = epoch_;
                f = job_;
                n = n_;
            }
            drain(*f, n);
            {
                std::lock_guard<std::mutex> g(mu_);
                if (--busy_ == 0) done_.notify_one();
            }
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    const std::function<void(int32_t)> *job_ = nullptr;
    int32_t n_ = 0, busy_ = 0;
    std::atomic<int32_t> next_{0};
    uint64_t epoch_ = 0;
    bool stop_ = false;
};

// Tabu list: every series ever analysed, exact and ordered.  Series live in
// an append-only arena; the set holds (offset, length) keys into it.
class Tabu {
  public:
    Tabu() : slots_(1024) {}
    bool contains(const int32_t *s, int32_t L) const {
        const uint64_t h = hash(s, L);
        return slots_[find(s, L, h)].len >= 0;
    }
    // Inserts; returns false when already present.
    bool insert(const int32_t *s, int32_t L) {
        const uint64_t h = hash(s, L);
        size_t i = find(s, L, h);
        if (slots_[i].len >= 0) return false;
        if (2 * (used_ + 1) > slots_.size()) {
            grow();
            i = find(s, L, h);
        }
        slots_[i] = Slot{h, arena_.size(), L};
        arena_.insert(arena_.end(), s, s + L);
        ++used_;
        return true;
    }

    size_t size() const { return used_; }
    static uint64_t hash(const int32_t *p, int32_t L) {
        uint64_t h = 0x84222325cbf29ce4ull ^ (uint64_t)L;
        for (int32_t i = 0; i < L; ++i) {
            h ^= (uint32_t)p[i];
            h *= 0x100000001b3ull;
            h ^= h >> 29;
        }
        return h ^ (h >> 32);
    }
    // The set as its series in insertion order (the arena and each entry's
    // length); loading re-inserts them.
    void save(Writer &w) const {
        std::vector<int32_t> lens(used_);
        std::vector<std::pair<size_t, int32_t>> at;
        at.reserve(used_);
        for (const Slot &e : slots_)
            if (e.len >= 0) at.emplace_back(e.at, e.len);
        std::sort(at.begin(), at.end());
        for (size_t i = 0; i < at.size(); ++i) lens[i] = at[i].second;
        w.vec(arena_);
        w.vec(lens);
    }
    bool load(Reader &r) {
        const std::vector<int32_t> arena = r.vec<int32_t>((size_t)1 << 40);
        const std::vector<int32_t> lens = r.vec<int32_t>((size_t)1 << 40);
        if (!r.ok) return false;
        *this = Tabu();
        size_t at = 0;
        for (int32_t L : lens) {
            if (L < 1 || arena.size() - at < (size_t)L) return false;
            if (!insert(arena.data() + at, L)) return false;
            at += (size_t)L;
        }
        return at == arena.size();
    }

  private:
    // Open addressing with linear probing over a power-of-two table kept at
    // most half full; series live in one arena.
    struct Slot {
        uint64_t h = 0;
        size_t at = 0;
        int32_t len = -1;   // -1: empty
    };
    // Slot holding the series, or the empty slot where it would go.
    size_t find(const int32_t *s, int32_t L, uint64_t h) const {
        const size_t mask = slots_.size() - 1;
        for (size_t i = (size_t)h & mask;; i = (i + 1) & mask) {
            const Slot &e = slots_[i];
            if (e.len < 0) return i;
            if (e.h == h && e.len == L &&
                std::memcmp(arena_.data() + e.at, s, sizeof(int32_t) * (size_t)L) == 0)
                return i;
        }
    }
    void grow() {
        std::vector<Slot> old((size_t)2 * slots_.size());
        old.swap(slots_);
        const size_t mask = slots_.size() - 1;
        for (const Slot &e : old) {
            if (e.len < 0) continue;
            size_t i = (size_t)e.h & mask;
            while (slots_[i].len >= 0) i = (i + 1) & mask;
            slots_[i] = e;
        }
    }
    std::vector<int32_t> arena_;
    std::vector<Slot> slots_;
    size_t used_ = 0;
};

struct TopEntry {
    std::vector<int32_t> s;
    int32_t count;
    double fit;
};

// Step 5: the top-rank list update.
//
// Members are visited by decreasing fitness (stable).  A member is skipped
// when its fitness is not positive or its series is already listed; it is
// rejected when a listed entry of at least its fitness overlaps it by more
// than theta (|x & e| / min(|x|, |e|) on column sets); otherwise it evicts
// the weaker entries it overlaps by more than theta and joins the list.  The
// list is then sorted by fitness (stable) and cut to K.
//
// Only entries sharing a column with x can overlap it (or equal it), so the
// intersections are accumulated through a column -> entries index instead of
// comparing x with every entry; the decisions are the same.
//
// The pass also stops as soon as its outcome is fixed.  An entry can only be
// evicted by a strictly fitter member, and members come by decreasing
// fitness; so when x is reached, every live entry with fitness >= f(x) stays
// live to the end and precedes x (and everything after x) in the final
// stable order.  Once there are K of them, no later member can enter the
// final K or remove one of them, and whatever it evicts has fitness < f(x)
// and falls beyond the cut anyway.
class TopRank {
  public:
    explicit TopRank(int32_t n_cols) : by_col_((size_t)n_cols) {}

    const std::vector<TopEntry> &entries() const { return top_; }

    void update(const Pop &pop, double theta, int32_t K) {
        const int32_t P = pop.size();
        order_.resize((size_t)P);
        for (int32_t i = 0; i < P; ++i) order_[(size_t)i] = i;
        std::stable_sort(order_.begin(), order_.end(), [&](int32_t a, int32_t b) {
            return pop.fit[(size_t)a] > pop.fit[(size_t)b];
        });
        // working list: top_ in insertion order, plus liveness and the index
        alive_.assign(top_.size(), 1);
        for (auto &v : by_col_) v.clear();
        for (size_t e = 0; e < top_.size(); ++e)
            for (int32_t c : top_[e].s) by_col_[(size_t)c].push_back((int32_t)e);

        const size_t n_old = top_.size();  // sorted by decreasing fitness
        size_t old_ptr = 0;
        int32_t settled = 0;                // live entries with fitness >= f(x)
        for (int32_t i : order_) {
            const double fx = pop.fit[(size_t)i];
            if (!(fx > 0.0)) break;         // the rest are not positive either
            for (; old_ptr < n_old && top_[old_ptr].fit >= fx; ++old_ptr)
                settled += alive_[old_ptr];
            if (settled >= K) break;
            const int32_t *x = pop.series(i);
            const int32_t lx = pop.len(i);
            // intersections with every entry sharing a column with x
            touched_.clear();
            if (inter_.size() < top_.size()) inter_.resize(top_.size(), 0);
            for (int32_t t = 0; t < lx; ++t)
                for (int32_t e : by_col_[(size_t)x[t]]) {
                    if (!alive_[(size_t)e]) continue;
                    if (inter_[(size_t)e]++ == 0) touched_.push_back(e);
                }
            bool listed = false, blocked = false;
            for (int32_t e : touched_) {
                const TopEntry &te = top_[(size_t)e];
                const int32_t le = (int32_t)te.s.size();
                if (inter_[(size_t)e] == lx && le == lx && std::equal(te.s.begin(), te.s.end(), x))
                    listed = true;
            }
            if (!listed)
                for (int32_t e : touched_) {
                    const TopEntry &te = top_[(size_t)e];
                    const double ov = (double)inter_[(size_t)e] /
                                      (double)std::min(lx, (int32_t)te.s.size());
                    if (te.fit >= fx && ov > theta) {
                        blocked = true;
                        break;
                    }
                }
            if (!listed && !blocked) {
                for (int32_t e : touched_) {
                    const TopEntry &te = top_[(size_t)e];
                    const double ov = (double)inter_[(size_t)e] /
                                      (double)std::min(lx, (int32_t)te.s.size());
                    if (te.fit < fx && ov > theta) alive_[(size_t)e] = 0;
                }
                const int32_t id = (int32_t)top_.size();
                top_.push_back(TopEntry{std::vector<int32_t>(x, x + lx), pop.counts[(size_t)i], fx});
                alive_.push_back(1);
                ++settled;                  // f(x) >= the fitness of every later member
                for (int32_t t = 0; t < lx; ++t) by_col_[(size_t)x[t]].push_back(id);
            }
            for (int32_t e : touched_) inter_[(size_t)e] = 0;
        }
        // compact (insertion order kept), stable sort by fitness, cut to K
        size_t k = 0;
        for (size_t e = 0; e < top_.size(); ++e)
            if (alive_[e]) {
                if (k != e) top_[k] = std::move(top_[e]);
                ++k;
            }
        top_.resize(k);
        std::stable_sort(top_.begin(), top_.end(),
                         [](const TopEntry &a, const TopEntry &b) { return a.fit > b.fit; });
        if ((int32_t)top_.size() > K) top_.resize((size_t)K);
    }

    void save(Writer &w) const {
        w.put<uint64_t>(top_.size());
        for (const TopEntry &e : top_) {
            w.vec(e.s);
            w.put(e.count);
            w.put(e.fit);
        }
    }
    bool load(Reader &r, int32_t M) {
        const uint64_t k = r.get<uint64_t>();
        if (!r.ok || k > ((uint64_t)1 << 31)) return false;
        top_.clear();
        for (uint64_t i = 0; i < k; ++i) {
            TopEntry e;
            e.s = r.vec<int32_t>((size_t)M);
            e.count = r.get<int32_t>();
            e.fit = r.get<double>();
            if (!r.ok || e.s.empty()) return false;
            for (int32_t c : e.s)
                if (c < 0 || c >= M) return false;
            top_.push_back(std::move(e));
        }
        return true;
    }

  private:
    std::vector<TopEntry> top_;
    std::vector<std::vector<int32_t>> by_col_;
    std::vector<uint8_t> alive_;
    std::vector<int32_t> inter_, touched_, order_;
};

inline bool contains(const std::vector<int32_t> &s, int32_t c) {
    return std::find(s.begin(), s.end(), c) != s.end();
}

inline int32_t new_column(SplitMix64 &rng, const std::vector<int32_t> &s, int32_t M) {
    for (;;) {
        const int32_t c = (int32_t)rng.below((uint64_t)M);
        if (!contains(s, c)) return c;
    }
}

enum { OP_INSERT = 0, OP_DELETE, OP_SWAP, OP_SUBSTITUTE, OP_CROSSOVER };

// Mutations of Fig. 1a-d; inapplicable ones leave s unchanged and draw nothing.
inline void mutate(SplitMix64 &rng, std::vector<int32_t> &s, int op, const ebic_evolve_params &p,
            int32_t M) {
    const int32_t L = (int32_t)s.size();
    switch (op) {
    case OP_INSERT:
        if (L < p.len_max) {
            const int32_t pos = (int32_t)rng.below((uint64_t)L + 1);
            const int32_t c = new_column(rng, s, M);
            s.insert(s.begin() + pos, c);
        }
        break;
    case OP_DELETE:
        if (L > p.len_min) s.erase(s.begin() + rng.below((uint64_t)L));
        break;
    case OP_SWAP:
        if (L >= 2) {
            const int32_t i = (int32_t)rng.below((uint64_t)L);
            int32_t j = (int32_t)rng.below((uint64_t)L - 1);
            if (j >= i) ++j;
            std::swap(s[(size_t)i], s[(size_t)j]);
        }
        break;
    case OP_SUBSTITUTE:
        if (L < M) {
            const int32_t pos = (int32_t)rng.below((uint64_t)L);
            s[(size_t)pos] = new_column(rng, s, M);
        }
        break;
    default:
        break;
    }
}

// One-point crossover of Fig. 1e with duplicate removal and clamping.
inline void crossover(SplitMix64 &rng, const int32_t *a, int32_t la, const int32_t *b, int32_t lb,
               const ebic_evolve_params &p, std::vector<int32_t> &child) {
    const int32_t i = 1 + (int32_t)rng.below((uint64_t)la);
    const int32_t j = (int32_t)rng.below((uint64_t)lb);
    child.assign(a, a + i);
    for (int32_t t = j; t < lb; ++t) {
        const int32_t c = b[t];
        if (std::find(a, a + i, c) == a + i) child.push_back(c);
    }
    if ((int32_t)child.size() > p.len_max) child.resize((size_t)p.len_max);
    if ((int32_t)child.size() < p.len_min) child.assign(a, a + la);
}

// Number of ordered series of distinct columns with lengths in
// [lmin, lmax], saturated at 2^62.
inline int64_t search_space(int32_t M, int32_t lmin, int32_t lmax) {
    const int64_t cap = int64_t(1) << 62;
    int64_t total = 0;
    for (int32_t L = lmin; L <= lmax; ++L) {
        int64_t t = 1;
        for (int32_t i = 0; i < L && t < cap; ++i) {
            const int64_t f = (int64_t)M - i;
            t = (f > 0 && t > cap / f) ? cap : t * f;
        }
        total = (t >= cap - total) ? cap : total + t;
    }
    return total;
}

inline ebic_status check_params(const ebic_evolve_params *p, int64_t n_rows, int32_t M) {
    if (!p || p->struct_size < sizeof(ebic_evolve_params))
        return evolve_error(EBIC_E_ARG, "params is null or struct_size too small");
    if (n_rows < 1 || M < 1) return evolve_error(EBIC_E_ARG, "empty matrix");
    if (p->population < 1 || p->len_min < 1 || p->len_min > p->len_max || p->len_max > M)
        return evolve_error(EBIC_E_ARG, "need P >= 1 and 1 <= len_min <= len_max <= n_cols");
    if (p->tournament < 1) return evolve_error(EBIC_E_ARG, "tournament must be >= 1");
    int64_t wsum = 0;
    for (int i = 0; i < 5; ++i) {
        if (p->op_weight[i] < 0) return evolve_error(EBIC_E_ARG, "negative operation weight");
        wsum += p->op_weight[i];
    }
    if (wsum <= 0) return evolve_error(EBIC_E_ARG, "operation weights sum to 0");
    if (p->elite_den < 1 || p->elite_num < 0 || p->elite_num > p->elite_den)
        return evolve_error(EBIC_E_ARG, "need 0 <= elite_num <= elite_den, elite_den >= 1");
    if (p->toplist_size < 1) return evolve_error(EBIC_E_ARG, "toplist_size must be >= 1");
    if (!(p->penalty_base > 0.0) || !(p->overlap >= 0.0 && p->overlap <= 1.0))
        return evolve_error(EBIC_E_ARG, "need penalty_base > 0 and 0 <= overlap <= 1");
    if (p->eval.struct_size < sizeof(ebic_params) || p->expand.struct_size < sizeof(ebic_params))
        return evolve_error(EBIC_E_ARG, "eval/expand struct_size too small");
    if (p->eval.sigma < 0 || p->eval.max_violations < 0 || p->expand.sigma < 0 ||
        p->expand.max_violations < 0)
        return evolve_error(EBIC_E_RANGE, "sigma and max_violations must be >= 0");
    if ((int64_t)p->population > search_space(M, p->len_min, p->len_max))
        return evolve_error(EBIC_E_ARG, "population exceeds the number of distinct series");
    return EBIC_OK;
}

// Step 3 draws: tournament selection with the crowding penalty, then one
// genetic operation.  Holds its own random stream, penalty counts and child
// buffer, so that several can draw in parallel from one population.
class Breeder {
  public:
    Breeder(const ebic_evolve_params &p, int32_t M, uint64_t seed)
        : p_(&p), M_(M), rng(seed), penalty((size_t)M) {
        for (int i = 0; i < 5; ++i) wsum_ += p.op_weight[i];
    }

    // Tournament over `prev` with the crowding penalty.
    int32_t tournament(const Pop &prev) {
        int32_t best = -1;
        double best_adj = -INFINITY;
        for (int32_t r = 0; r < p_->tournament; ++r) {
            const int32_t i = (int32_t)rng.below((uint64_t)prev.size());
            const int32_t *si = prev.series(i);
            const int32_t L = prev.len(i);
            int64_t sum = 0;
            for (int32_t t = 0; t < L; ++t) sum += penalty[(size_t)si[t]];
            const double adj = prev.fit[(size_t)i] / penalty_pow(sum, L);
            if (adj > best_adj) {
                best = i;
                best_adj = adj;
            }
        }
        return best;
    }

    // One Step 3 draw into `child`: tournament winner(s) and one operation.
    void make_child(const Pop &prev) {
        const int32_t ia = tournament(prev);
        const uint64_t u = rng.below((uint64_t)wsum_);
        int op = 0;
        int64_t acc = 0;
        for (op = 0; op < 5; ++op) {
            acc += p_->op_weight[op];
            if ((int64_t)u < acc) break;
        }
        if (op == OP_CROSSOVER) {
            const int32_t ib = tournament(prev);
            crossover(rng, prev.series(ia), prev.len(ia), prev.series(ib), prev.len(ib), *p_,
                      child);
        } else {
            child.assign(prev.series(ia), prev.series(ia) + prev.len(ia));
            mutate(rng, child, op, *p_, M_);
        }
    }

    void add_penalty(const int32_t *s, int32_t L) {
        for (int32_t t = 0; t < L; ++t) ++penalty[(size_t)s[t]];
    }

  private:
    // base^(sum / L), the crowding penalty of a series of length L whose
    // columns hold `sum` penalty points, memoised per (L, sum): the value is
    // the same double std::pow returns for those arguments.
    double penalty_pow(int64_t sum, int32_t L) {
        if ((size_t)L >= memo_.size()) memo_.resize((size_t)L + 1);
        std::vector<double> &t = memo_[(size_t)L];
        if ((size_t)sum >= t.size()) t.resize(std::max<size_t>((size_t)sum + 1, 2 * t.size()), -1.0);
        double &v = t[(size_t)sum];
        if (!(v >= 0.0)) v = std::pow(p_->penalty_base, (double)sum / (double)L);
        return v;
    }

    const ebic_evolve_params *p_;
    int32_t M_;
    int64_t wsum_ = 0;
    std::vector<std::vector<double>> memo_;

  public:
    SplitMix64 rng;
    std::vector<int32_t> penalty, child;
};

// One seeded run as a state machine, so that a driver can evaluate many
// runs' populations together: next() builds the population of the next
// generation (Step 1, or Steps 2-3) and says which members need scores;
// accept() takes their scores (Step 4) and applies Step 5.
class Run {
  public:
    Run(int32_t M, uint64_t seed, int32_t generations, const ebic_evolve_params &p)
        : p_(p), M_(M), generations_(generations), br_(p_, M, seed), toprank_(M) {
        tabu_limit_ = p.tabu_limit < 0 ? p.population : p.tabu_limit;
        evalp_ = p.eval;
        evalp_.want_masks = 0;
    }

    // Builds the next population to score.  Returns false when the run is
    // over (all generations done, or the tabu rule stopped it).
    bool next() {
        if (gen_ == 0) {
            initial();
            return true;
        }
        if (gen_ > generations_ || stopped_) return false;
        breed();
        return !stopped_;
    }
    const Pop &pending() const { return cur_; }
    int32_t first_new() const { return first_; }
    // Elites the next Steps 2-3 will carry over: min(|top|, P * num / den).
    int32_t elites() const {
        return (int32_t)std::min<int64_t>((int64_t)toprank_.entries().size(),
                                          (int64_t)p_.population * p_.elite_num / p_.elite_den);
    }
    int32_t generation() const { return gen_; }
    const ebic_params &eval_params() const { return evalp_; }
    // Scores of members [first_new(), P) of pending().
    void accept(const int32_t *counts, const double *fit) {
        const int32_t P = cur_.size();
        cur_.counts.resize((size_t)P);
        cur_.fit.resize((size_t)P);
        std::copy(counts, counts + (P - first_), cur_.counts.begin() + first_);
        std::copy(fit, fit + (P - first_), cur_.fit.begin() + first_);
        if (p_.on_generation)
            p_.on_generation(p_.user, gen_, cur_.off.data(), cur_.cols.data(), P,
                             cur_.counts.data(), cur_.fit.data());
        if (gen_ > 0) gens_run_ = gen_;
        toprank_.update(cur_, p_.overlap, p_.toplist_size);  // Step 5
        std::swap(prev_, cur_);
        ++gen_;
    }
    const std::vector<TopEntry> &top() const { return toprank_.entries(); }
    int32_t generations_run() const { return gens_run_; }
    bool stopped() const { return stopped_; }
    size_t tabu_size() const { return tabu_.size(); }
    int32_t generations() const { return generations_; }

    // Checkpoint of the run between generations (after accept()): the
    // random stream, counters, the last scored population, the tabu list and
    // the top-rank list.  The parameters are the caller's to supply again.
    void save(Writer &w) const {
        w.put(br_.rng.s);
        w.put(gen_);
        w.put(first_);
        w.put(gens_run_);
        w.put<uint8_t>(stopped_ ? 1 : 0);
        prev_.save(w);
        tabu_.save(w);
        toprank_.save(w);
    }
    bool load(Reader &r) {
        br_.rng.s = r.get<uint64_t>();
        gen_ = r.get<int32_t>();
        first_ = r.get<int32_t>();
        gens_run_ = r.get<int32_t>();
        stopped_ = r.get<uint8_t>() != 0;
        if (!r.ok || gen_ < 0 || gens_run_ < 0 || first_ < 0) return false;
        if (!prev_.load(r, M_) || !tabu_.load(r) || !toprank_.load(r, M_)) return false;
        cur_.clear();
        return gen_ == 0 || prev_.size() > 0;
    }

  private:
    // Step 1: P distinct random series.
    void initial() {
        const int32_t P = p_.population;
        cur_.clear();
        while (cur_.size() < P) {
            const int32_t L =
                p_.len_min + (int32_t)br_.rng.below((uint64_t)(p_.len_max - p_.len_min + 1));
            s_.clear();
            while ((int32_t)s_.size() < L) {
                const int32_t c = (int32_t)br_.rng.below((uint64_t)M_);
                if (!contains(s_, c)) s_.push_back(c);
            }
            if (!tabu_.insert(s_.data(), L)) continue;
            cur_.push(s_.data(), L);
        }
        first_ = 0;
    }

    // Step 2: elites from the top-rank list, penalties of their columns.
    void elitism() {
        const int32_t P = p_.population;
        const std::vector<TopEntry> &top = toprank_.entries();
        std::fill(br_.penalty.begin(), br_.penalty.end(), 0);
        cur_.clear();
        const int32_t n_e = (int32_t)std::min<int64_t>(
            (int64_t)top.size(), (int64_t)P * p_.elite_num / p_.elite_den);
        for (int32_t e = 0; e < n_e; ++e) {
            const TopEntry &te = top[(size_t)e];
            cur_.push(te.s.data(), (int32_t)te.s.size());
            cur_.counts.push_back(te.count);
            cur_.fit.push_back(te.fit);
            br_.add_penalty(te.s.data(), (int32_t)te.s.size());
        }
        first_ = n_e;
    }

    // Steps 2-3: elitism, penalties and novel children.
    void breed() {
        elitism();
        int32_t hits = 0;
        const std::vector<int32_t> &child = br_.child;
        while (cur_.size() < p_.population) {
            br_.make_child(prev_);
            const int32_t L = (int32_t)child.size();
            if (!tabu_.insert(child.data(), L)) {
                if (++hits > tabu_limit_) {
                    stopped_ = true;
                    return;
                }
                continue;
            }
            cur_.push(child.data(), L);
            br_.add_penalty(child.data(), L);
        }
    }

  public:
    // Screened Steps 2-3 (offspring screening by a surrogate; not in the
    // paper).  After elitism, kScreenShares breeders draw a pool of
    // oversample x (P - elites) children in parallel.  Breeder j draws an
    // equal share with a stream seeded by the j-th of kScreenShares draws
    // from the run's stream, starting from the elites' penalties and adding
    // its own children's (Step 3 within the share); it keeps children novel
    // with respect to the tabu list and to its share.  The shares are joined
    // in breeder order, dropping series an earlier share holds; should the
    // pool fall short of P - elites, the run's own breeder tops it up.  The
    // P - elites children that `score` ranks highest (ties: earlier child
    // first) are kept and enter the tabu list.  A draw that repeats a known
    // or pooled series is a hit; more than tabu_limit x oversample hits in a
    // generation stop the run.  `score(pool)` returns one value per pooled
    // child.  The outcome depends on neither the thread count nor timing.
    static constexpr int32_t kScreenShares = 16;

    template <typename Scorer>
    bool next_screened(int32_t oversample, Scorer &&score, int32_t threads = 0) {
        if (gen_ == 0) {
            initial();
            return true;
        }
        if (gen_ > generations_ || stopped_) return false;
        elitism();
        const int32_t need = p_.population - first_;
        const int64_t target = (int64_t)need * oversample;
        const int64_t limit = (int64_t)tabu_limit_ * oversample;
        struct Share {
            uint64_t seed = 0;
            Pop pop;
            Tabu mine;                   // the share's own series
            std::vector<uint64_t> hash;  // hash of each of its series
            int64_t hits = 0;
        };
        std::vector<Share> shares((size_t)kScreenShares);
        for (Share &sh : shares) sh.seed = br_.rng.next();
        if (!helpers_) {
            if (threads <= 0) threads = (int32_t)std::max(1u, std::thread::hardware_concurrency());
            helpers_ = std::make_unique<Helpers>(std::max(1, std::min(threads, kScreenShares)));
        }
        helpers_->run(kScreenShares, [&](int32_t j) {
            Share &sh = shares[(size_t)j];
            const int64_t quota = target / kScreenShares + (j < target % kScreenShares ? 1 : 0);
            Breeder b(p_, M_, sh.seed);
            b.penalty = br_.penalty;
            while (sh.pop.size() < quota) {
                b.make_child(prev_);
                const int32_t L = (int32_t)b.child.size();
                if (tabu_.contains(b.child.data(), L) || !sh.mine.insert(b.child.data(), L)) {
                    if (++sh.hits > limit) return;
                    continue;
                }
                sh.pop.push(b.child.data(), L);
                b.add_penalty(b.child.data(), L);
            }
        });
        // Join in share order; a series that an earlier share holds is a
        // repeat.  Hashes are taken in parallel, then one pass over a flat
        // table of (hash, share, index) keeps each series' first copy.
        helpers_->run(kScreenShares, [&](int32_t j) {
            Share &sh = shares[(size_t)j];
            sh.hash.resize((size_t)sh.pop.size());
            for (int32_t i = 0; i < sh.pop.size(); ++i)
                sh.hash[(size_t)i] = Tabu::hash(sh.pop.series(i), sh.pop.len(i));
        });
        struct Ref {
            uint64_t h;
            int32_t share, i;   // share -1: empty
        };
        int64_t total = 0;
        for (const Share &sh : shares) total += sh.pop.size();
        size_t cap = 1024;
        while (cap < (size_t)(2 * total + 2 * need)) cap *= 2;
        std::vector<Ref> table(cap, Ref{0, -1, 0});
        // share kScreenShares: a child of the top-up, by its index in the pool
        auto series_of = [&](const Ref &r) -> std::pair<const int32_t *, int32_t> {
            const Pop &pp = r.share == kScreenShares ? pool_ : shares[(size_t)r.share].pop;
            return {pp.series(r.i), pp.len(r.i)};
        };
        // Inserts (h, share, i) unless the series is present; false if present.
        auto insert = [&](uint64_t h, const int32_t *c, int32_t L, int32_t share, int32_t i) {
            for (size_t k = (size_t)h & (cap - 1);; k = (k + 1) & (cap - 1)) {
                Ref &r = table[k];
                if (r.share < 0) {
                    r = Ref{h, share, i};
                    return true;
                }
                if (r.h != h) continue;
                const auto o = series_of(r);
                if (o.second == L && std::memcmp(o.first, c, sizeof(int32_t) * (size_t)L) == 0)
                    return false;
            }
        };
        int64_t hits = 0;
        pool_.clear();
        for (int32_t j = 0; j < kScreenShares; ++j) {
            const Share &sh = shares[(size_t)j];
            hits += sh.hits;
            for (int32_t i = 0; i < sh.pop.size(); ++i) {
                if (insert(sh.hash[(size_t)i], sh.pop.series(i), sh.pop.len(i), j, i))
                    pool_.push(sh.pop.series(i), sh.pop.len(i));
                else
                    ++hits;
            }
        }
        const std::vector<int32_t> &child = br_.child;
        while (hits <= limit && pool_.size() < need) {
            br_.make_child(prev_);
            const int32_t L = (int32_t)child.size();
            if (tabu_.contains(child.data(), L)) {
                ++hits;
                continue;
            }
            pool_.push(child.data(), L);
            const int32_t at = pool_.size() - 1;
            if (!insert(Tabu::hash(child.data(), L), pool_.series(at), L, kScreenShares, at)) {
                pool_.cols.resize((size_t)pool_.off[(size_t)at]);   // a repeat: drop it
                pool_.off.pop_back();
                ++hits;
            }
        }
        if (hits > limit) {
            stopped_ = true;
            return false;
        }
        auto sc = score(pool_);      // one float or double per pooled child
        // The `need` highest scores, ties to the earlier child, kept in pool
        // order (NaN ranks last).
        std::vector<int32_t> order((size_t)pool_.size());
        for (int32_t i = 0; i < pool_.size(); ++i) {
            order[(size_t)i] = i;
            if (sc[(size_t)i] != sc[(size_t)i]) sc[(size_t)i] = -INFINITY;
        }
        auto before = [&](int32_t a, int32_t b) {
            return sc[(size_t)a] > sc[(size_t)b] || (sc[(size_t)a] == sc[(size_t)b] && a < b);
        };
        if ((size_t)need < order.size())
            std::nth_element(order.begin(), order.begin() + need, order.end(), before);
        order.resize((size_t)need);
        std::sort(order.begin(), order.end());
        for (int32_t i : order) {
            cur_.push(pool_.series(i), pool_.len(i));
            tabu_.insert(pool_.series(i), pool_.len(i));
        }
        return true;
    }

    Run(const Run &) = delete;
    Run &operator=(const Run &) = delete;

  private:
    const ebic_evolve_params p_;
    const int32_t M_;
    const int32_t generations_;
    Breeder br_;
    Tabu tabu_;
    TopRank toprank_;
    std::vector<int32_t> s_;
    Pop prev_, cur_, pool_;
    std::unique_ptr<Helpers> helpers_;   // pool drawing threads, started on first use
    ebic_params evalp_{};
    int32_t tabu_limit_ = 0;
    int32_t gen_ = 0, first_ = 0, gens_run_ = 0;
    bool stopped_ = false;
};

// Steps 6-7 output from the listed series' expansion evaluation.
inline ebic_result *make_result(const std::vector<TopEntry> &top, int64_t W,
                         const std::vector<uint64_t> &masks, std::vector<int32_t> &&counts,
                         std::vector<double> &&fit) {
    ebic_result *r = new (std::nothrow) ebic_result();
    if (!r) return nullptr;
    r->counts = std::move(counts);
    r->fit = std::move(fit);
    for (size_t i = 0; i < top.size(); ++i) {
        r->cols.push_back(top[i].s);
        std::vector<uint64_t> m((size_t)W);
        for (int64_t w = 0; w < W; ++w)
            m[(size_t)w] = masks[(i * 2 + 0) * W + w] | masks[(i * 2 + 1) * W + w];
        r->masks.push_back(std::move(m));
    }
    return r;
}

}  // namespace host
}  // namespace ebic
