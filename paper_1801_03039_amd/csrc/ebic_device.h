// Device code shared by the single-run and batched evaluation kernels
// (gfx950, wave64): helpers, the Eq. (1) fitness write, and one tile of the
// index evaluator (strict, negative and approximate trend tests over the
// pairwise order index).  Included by the .hip files only.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "ebic_internal.h"

namespace ebic {
namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kAlignedThreads = 320;   // largest single-run whole-candidate workgroup
constexpr int kXcds = 8;

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Pointers read from device memory (a run table) are generic to the
// compiler; declaring them global lets it emit global (not flat) loads.
template <typename T>
using global_ptr = const __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ global_ptr<T> as_global(const T *p) {
    return (global_ptr<T>)p;
}

__device__ __forceinline__ uint64_t tail_bits(int64_t n, int64_t w, int64_t W) {
    if (w < W - 1) return ~0ull;
    const int rem = (int)(n - (W - 1) * 64);  // 1..64
    return rem == 64 ? ~0ull : ((1ull << rem) - 1ull);
}

// --------------------------------------------------------- fitness (Eq. 1) --
//
// Each part of a candidate (a workgroup's row slice, or a run of 64-row
// words) reports with ONE 64-bit atomic add on acc[c]:
//   bits  0..31  rows it accepted (|I| <= n < 2^31)
//   bit  32      set by the part that found the candidate malformed
//   bits 33..63  its share of the candidate's `parts`
// The part whose add completes the shares owns the total: a single
// read-modify-write orders everything, so no memory fence is needed.  It
// resets acc[c] for the next call and writes the count and Eq. (1).
// ln(count-1) comes from a table built on the host with the C library's
// log; L * ln is one rounded FP64 product and 2^e an exact scaling, so the
// result equals the host formula bit for bit.
constexpr int kShareShift = 33;
constexpr uint64_t kBadBit = 1ull << 32;

// Count and Eq. (1) fitness of candidate c (count -1 and NaN fitness for a
// malformed candidate).
template <typename LogPtr>
__device__ __forceinline__ void write_result(int64_t c, int32_t total, bool bad, int32_t L,
                                             int32_t sigma, LogPtr logt,
                                             int32_t *__restrict__ counts,
                                             double *__restrict__ fitness) {
    if (bad) {
        counts[c] = -1;
        fitness[c] = __builtin_nan("");
        return;
    }
    counts[c] = total;
    double f = 0.0;
    if (total > 1) {
        const int32_t e = total - sigma < 0 ? total - sigma : 0;
        f = ldexp((double)L * logt[total - 1], e);
    }
    fitness[c] = f;
}

template <typename LogPtr>
__device__ __forceinline__ void finish_part(int64_t c, uint32_t cnt, bool bad, int64_t share,
                                            int64_t parts, int32_t L, int32_t sigma,
                                            LogPtr logt,
                                            unsigned long long *__restrict__ acc,
                                            int32_t *__restrict__ counts,
                                            double *__restrict__ fitness) {
    const unsigned long long add =
        ((unsigned long long)share << kShareShift) | (bad ? kBadBit : 0ull) | cnt;
    const unsigned long long before = atomicAdd(acc + c, add);
    const unsigned long long now = before + add;
    if ((int64_t)(now >> kShareShift) != parts) return;
    atomicExch(acc + c, 0ull);
    write_result(c, (int32_t)(uint32_t)now, (now & kBadBit) != 0, L, sigma, logt, counts, fitness);
}

// -------------------------------------------------------- index evaluator --
//
// Thread = (candidate c, V consecutive 64-row words), c-major, so every
// lane has work whatever W is; the V words share the lane's column reads and
// loop, and are read with 16-byte loads when V > 1 (fewer waves, more loads
// in flight per lane, the same bytes).  The workgroup first stages the CBF
// columns of the candidates it covers in LDS.  Per consecutive pair (p, q) a
// lane reads lt(p,q) -- and lt(q,p) for the falling direction -- from the
// pairwise order index and folds the violation words (complements) into K+1
// saturating bit-sliced counters per direction: c[i] has bit b set when row
// b has more than i violations.  lt(q,p) is read only for pairs that may
// tie (a set tie flag, or a set bit of the tie-pair bitmap); otherwise it is
// ~lt(p,q) (lt(p,p) itself for a repeated column).  Single-run workgroups
// look every staged pair up in the bitmap while staging, and run a loop
// without any tie test when none is set.  Loads for kUnroll pairs are issued
// before any is consumed (the lane's latency chain is one order-word round
// trip per kUnroll pairs), and a lane stops once every row of its word is
// rejected in every enabled direction.
constexpr int kIdxLds = 4096;   // staged column entries per workgroup
constexpr int kUnroll = 4;   // pairs per batch of loads (single-run default)
constexpr int kWordsPerLane = 2;   // 64-row words per lane (flattened single-run tiling)

template <int K, bool NEG>
__device__ __forceinline__ void fold(uint64_t (&cu)[K + 1], uint64_t (&cd)[K + 1], uint64_t lt_pq,
                                     uint64_t lt_qp) {
    const uint64_t vu = ~lt_pq;
#pragma unroll
    for (int i = K; i > 0; --i) cu[i] |= cu[i - 1] & vu;
    cu[0] |= vu;
    if (NEG) {
        const uint64_t vd = ~lt_qp;
#pragma unroll
        for (int i = K; i > 0; --i) cd[i] |= cd[i - 1] & vd;
        cd[0] |= vd;
    }
}

// LDS of one tile: the staged CBF columns, for whole-candidate tiles the
// per-candidate row counts and malformed flags, and the tie-pair bitmap.
struct TileLds {
    int32_t cols[kIdxLds];
    int32_t rows[kBlock];
    int32_t bad[kBlock];
    uint32_t tbits[kTieWords];
    int32_t any_tied;        // a staged consecutive pair is in the tie-pair bitmap
};

// How the falling test learns that a pair has a tied row (lt(q,p) is then
// read from the index instead of taken as ~lt(p,q)): never (the matrix has
// no tied pair), from the m*m byte flags (one load per pair), or from the
// tie-pair bitmap staged in LDS.
enum TieMode { kTieNone = 0, kTieFlags = 1, kTieBitmap = 2 };

// V consecutive order words of one pair, read with 16-byte loads when V > 1
// (the caller keeps the address 16-byte aligned).
template <int V>
__device__ __forceinline__ void load_words(global_ptr<uint64_t> p, uint64_t (&o)[V]) {
    if constexpr (V == 1) {
        o[0] = p[0];
    } else {
        typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int i = 0; i < V; i += 2) {
            const u64x2 x = *(global_ptr<u64x2>)(p + i);
            o[i] = x.x;
            o[i + 1] = x.y;
        }
    }
}

// Calls f(integral_constant<int, r>) for the run-time count r in [1, N]
// (nothing for r = 0): the last, shorter batch of a series' pairs.
template <int N>
struct ShortBatch {
    template <class F>
    __device__ __forceinline__ static void run(int32_t r, F &&f) {
        if (r == N)
            f(std::integral_constant<int, N>{});
        else
            ShortBatch<N - 1>::run(r, f);
    }
};
template <>
struct ShortBatch<0> {
    template <class F>
    __device__ __forceinline__ static void run(int32_t, F &&) {}
};

// One tile of one run.  An item is a candidate and V consecutive 64-row
// words of it (V words per lane share the lane's column reads and loop).
// Two tilings:
//   ALIGNED = false: kBlock consecutive items of the flattened (candidate,
//     item) order; a candidate may span workgroups, so each workgroup adds
//     its share of a candidate's count with one packed global atomic and the
//     last share writes the result (finish_part).  Shared by the single-run
//     kernel and the persistent multi-run kernel.
//   ALIGNED = true: the workgroup holds `cpw` whole candidates (requires
//     ceil(W / V) <= kBlock and cpw <= kBlock; the workgroup may have up to
//     kAlignedThreads lanes); counts are summed with LDS atomics and the
//     first lane of each candidate writes its result after a workgroup
//     barrier -- no global atomics and no accumulator scratch.
template <int K, bool NEG, int U, int V, bool ALIGNED, int TIES = kTieFlags, bool OFF32 = false,
          bool TAIL = false>
__device__ __forceinline__ void index_tile(const IndexRun &R, uint32_t tile, uint32_t cpw,
                                           const int32_t *__restrict__ offsets,
                                           const int32_t *__restrict__ cols, int64_t n_entries,
                                           int32_t sigma, uint64_t *__restrict__ masks,
                                           unsigned long long *__restrict__ acc,
                                           int32_t *__restrict__ counts,
                                           double *__restrict__ fitness, TileLds &lds) {
    // (V <= 8 keeps a wave's per-candidate row count within 16 bits below)
    static_assert(V == 1 || V == 2 || V == 4 || V == 8, "words per lane");
    int32_t *const s_cols = lds.cols;
    const auto idx = as_global(R.idx);
    const auto tie = as_global(R.tie);
    const auto logt = as_global(R.logt);
    const int64_t n = R.n, W = R.W, wpad = R.wpad;
    const int32_t m = R.m, P = R.P;
    const int tid = threadIdx.x, lane = tid & 63;
    // The launcher guarantees P * ceil(W / V) < 2^32.
    const uint32_t Wg = (uint32_t)((W + V - 1) / V);   // items per candidate
    uint32_t cl, g, c_lo, c_hi, slot = 0;
    bool active;
    if constexpr (ALIGNED) {
        slot = (uint32_t)tid / Wg;                                // candidate slot in the tile
        c_lo = tile * cpw;
        c_hi = min(c_lo + cpw, (uint32_t)P) - 1;
        active = slot < cpw && c_lo + slot < (uint32_t)P;
        cl = active ? c_lo + slot : c_hi;
        g = active ? (uint32_t)tid - slot * Wg : 0;
    } else {
        const uint32_t item = tile * (uint32_t)kBlock + (uint32_t)tid;
        active = item < (uint32_t)P * Wg;
        cl = active ? item / Wg : (uint32_t)P - 1;               // candidate within the run
        g = active ? item - cl * Wg : 0;
        const uint32_t i0 = tile * (uint32_t)kBlock;
        c_lo = i0 / Wg;
        c_hi = min((i0 + kBlock - 1) / Wg, (uint32_t)P - 1);
    }
    const int64_t w0 = (int64_t)g * V;                           // first word of the item
    const int64_t c = R.cand_base + cl;                          // candidate in the launch

    // the tie-pair bitmap, ordered before its first use by the barrier below
    if constexpr (NEG && TIES == kTieBitmap) {
        const auto tb = as_global(R.tbits);
        for (int i = tid; i < kTieWords; i += (int)blockDim.x) lds.tbits[i] = tb[i];
    }
    auto in_bitmap = [&](int64_t pq) -> bool {
        const uint32_t h = tie_hash((uint32_t)pq);
        return ((lds.tbits[h >> 5] >> (h & 31)) & 1u) != 0;
    };

    const int64_t start = offsets[c], end = offsets[c + 1];
    const bool ok_range = start >= 0 && end <= n_entries && end > start;
    const int32_t L = ok_range ? (int32_t)(end - start) : 0;

    // Stage the columns of candidates [c_lo, c_hi] in LDS when they fit and
    // every lane's series lies inside the staged span (always, for a
    // well-formed CBF); otherwise the whole workgroup reads them from global
    // memory.  The choice is uniform over the workgroup.
    const int64_t b0 = offsets[R.cand_base + c_lo], b1 = offsets[R.cand_base + c_hi + 1];
    int32_t *const s_rows = lds.rows;
    int32_t *const s_bad = lds.bad;
    if (ALIGNED && (uint32_t)tid < cpw) {
        s_rows[tid] = 0;
        s_bad[tid] = 0;
    }
    if (tid == 0) lds.any_tied = 0;
    const bool span_ok = b0 >= 0 && b1 <= n_entries && b1 >= b0 && b1 - b0 <= kIdxLds;
    const bool lane_ok = !ok_range || (start >= b0 && end <= b1);
    const bool use_lds = __syncthreads_and(span_ok && lane_ok) != 0;
    // Staging also checks every staged column: when none is out of range
    // (the common case) the per-candidate validation below is skipped.  With
    // the tie-pair bitmap it also looks up every staged consecutive pair
    // (pairs that straddle two candidates included): a workgroup none of
    // whose pairs is in the bitmap runs the tie-free loop.
    bool staged_bad = true;
    [[maybe_unused]] bool staged_tie = true;
    if (use_lds) {
        bool inval = false, any_tied = false;
        for (int32_t e = tid; e < (int32_t)(b1 - b0); e += (int32_t)blockDim.x) {
            const int32_t x = cols[b0 + e];
            inval |= x < 0 || x >= m;
            s_cols[e] = x;
            if constexpr (NEG && TIES == kTieBitmap) {
                if (e > 0) {
                    const int32_t xp = cols[b0 + e - 1];
                    if (x >= 0 && x < m && xp >= 0 && xp < m && x != xp)
                        any_tied |= in_bitmap((int64_t)xp * m + x);
                }
            }
        }
        if (any_tied) lds.any_tied = 1;
        staged_bad = __syncthreads_or(inval) != 0;
        staged_tie = lds.any_tied != 0;
    }
    const int32_t lds0 = (int32_t)(start - b0);

    uint64_t valid[V];
    uint64_t any_valid = 0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        valid[v] = (active && ok_range && w0 + v < W) ? tail_bits(n, w0 + v, W) : 0ull;
        any_valid |= valid[v];
    }
    uint64_t cu[V][K + 1], cd[V][K + 1];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int i = 0; i <= K; ++i) cu[v][i] = cd[v][i] = 0ull;
    bool bad = false;

    // Per-lane work, instantiated for columns in LDS or in global memory and
    // for a tie mode (TIES, or kTieNone for a workgroup without tied pairs).
    auto lane_work = [&](auto from_lds, auto tie_mode, auto unroll) {
        constexpr bool kLds = decltype(from_lds)::value;
        constexpr int TM = decltype(tie_mode)::value;
        constexpr int UU = decltype(unroll)::value;
        auto tied = [&](int64_t pq) -> uint8_t {
            if constexpr (TM == kTieFlags) return tie[pq];
            if constexpr (TM == kTieBitmap) return in_bitmap(pq) ? 1 : 0;
            return 0;
        };
        auto col = [&](int32_t t) -> int32_t {
            if constexpr (kLds) return s_cols[lds0 + t];
            else return cols[start + t];
        };
        // The lane of the first word validates every column (batched,
        // branch-free reads; skipped when staging found every staged column
        // in range) and reports the outcome with its part; other lanes only
        // clamp column indices so that no read leaves the index.
        if (active && g == 0) bad = !ok_range;
        if (active && g == 0 && (!kLds || staged_bad)) {
            for (int32_t t = 0; t < L; t += UU) {
                int32_t x[UU];
#pragma unroll
                for (int u = 0; u < UU; ++u) x[u] = col(min(t + u, L - 1));
#pragma unroll
                for (int u = 0; u < UU; ++u) bad |= (x[u] < 0 || x[u] >= m);
            }
        }
        if (!any_valid) return;
        // Address of the words of pair row `pq`: with OFF32 (index < 4 GiB)
        // a 32-bit byte offset from the uniform base, which the compiler
        // forms as a scalar base plus one offset register per load.
        auto words_at = [&](int64_t pq) {
            if constexpr (OFF32) {
                typedef const __attribute__((address_space(1))) char *gchar;
                const uint32_t off = ((uint32_t)pq * (uint32_t)wpad + (uint32_t)w0) * 8u;
                return (global_ptr<uint64_t>)((gchar)idx + off);
            } else {
                return idx + w0 + pq * wpad;
            }
        };
        if constexpr (TAIL) {
            int32_t p = col(0);
            p = (p < 0 || p >= m) ? 0 : p;
            // One batch of N consecutive pairs from pair t (t + N <= L): the
            // column reads and order-word loads are all issued before any is
            // consumed.  Returns whether a row of the lane's words is still
            // undecided.
            auto batch = [&](auto n, int32_t t) -> bool {
                constexpr int N = decltype(n)::value;
                int32_t q[N];
#pragma unroll
                for (int u = 0; u < N; ++u) {
                    const int32_t x = col(t + u);
                    q[u] = (x < 0 || x >= m) ? 0 : x;
                }
                uint64_t lu[N][V], ld[N][V];
                uint8_t tf[N];
                int32_t pp = p;
#pragma unroll
                for (int u = 0; u < N; ++u) {
                    const int64_t pq = (int64_t)pp * m + q[u];
                    load_words<V>(words_at(pq), lu[u]);
                    if (NEG) tf[u] = tied(pq);
                    pp = q[u];
                }
                if (NEG) {
                    // lt(q,p) is the complement of lt(p,q) unless the pair ties
                    pp = p;
#pragma unroll
                    for (int u = 0; u < N; ++u) {
                        if (TM != kTieNone && tf[u]) {
                            load_words<V>(words_at((int64_t)q[u] * m + pp), ld[u]);
                        } else {
                            // a repeated column is its own reverse: lt(p,p) = 0
                            // (the byte flags mark it as tied instead)
                            const bool self = TM != kTieFlags && q[u] == pp;
#pragma unroll
                            for (int v = 0; v < V; ++v) ld[u][v] = self ? lu[u][v] : ~lu[u][v];
                        }
                        pp = q[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < N; ++u)
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        fold<K, NEG>(cu[v], cd[v], lu[u][v], NEG ? ld[u][v] : 0ull);
                p = q[N - 1];
                uint64_t live = 0;
#pragma unroll
                for (int v = 0; v < V; ++v)
                    live |= valid[v] & ~(NEG ? (cu[v][K] & cd[v][K]) : cu[v][K]);
                return live != 0ull;
            };
            // Whole batches of UU pairs, then the last L - t < UU pairs as one
            // shorter batch: no load reads past the end of the series.
            int32_t t = 1;
            bool undecided = true;
            for (; t + UU <= L; t += UU)
                if (!(undecided = batch(std::integral_constant<int, UU>{}, t))) break;
            if (undecided)
                ShortBatch<UU - 1>::run(L - t, [&](auto n) { (void)batch(n, t); });
        } else {
            const int32_t last = L - 1;
            int32_t p = col(0);
            p = (p < 0 || p >= m) ? 0 : p;
            for (int32_t t = 1; t < L; t += UU) {
                // Column reads and order-word loads of the batch are issued
                // unconditionally (slots past the end repeat the last pair, a
                // harmless in-bounds read whose words are then ignored).
                int32_t q[UU];
#pragma unroll
                for (int u = 0; u < UU; ++u) {
                    const int32_t x = col(min(t + u, last));
                    q[u] = (x < 0 || x >= m) ? 0 : x;
                }
                uint64_t lu[UU][V], ld[UU][V];
                uint8_t tf[UU];
                int32_t pp = p;
                int64_t pq_prev = 0;
#pragma unroll
                for (int u = 0; u < UU; ++u) {
                    // a slot past the end re-reads the words of the last
                    // pair (just fetched) rather than a diagonal row
                    int64_t pq = (int64_t)pp * m + q[u];
                    if (u > 0) pq = t + u < L ? pq : pq_prev;
                    pq_prev = pq;
                    load_words<V>(words_at(pq), lu[u]);
                    if (NEG) tf[u] = tied(pq);
                    pp = q[u];
                }
#pragma unroll
                for (int u = 0; u < UU; ++u) {
                    const bool in = t + u < L;
#pragma unroll
                    for (int v = 0; v < V; ++v) lu[u][v] = in ? lu[u][v] : ~0ull;
                    if (NEG) tf[u] = in ? tf[u] : 0;
                }
                if (NEG) {
                    // lt(q,p) is the complement of lt(p,q) unless the pair ties;
                    // slots past the end of the series break nothing.
                    pp = p;
#pragma unroll
                    for (int u = 0; u < UU; ++u) {
                        if (TM != kTieNone && tf[u]) {
                            load_words<V>(words_at((int64_t)q[u] * m + pp), ld[u]);
                        } else {
                            // a repeated column is its own reverse: lt(p,p) = 0
                            // (the byte flags mark it as tied instead)
                            const bool self = TM != kTieFlags && q[u] == pp;
#pragma unroll
                            for (int v = 0; v < V; ++v) ld[u][v] = self ? lu[u][v] : ~lu[u][v];
                        }
#pragma unroll
                        for (int v = 0; v < V; ++v) ld[u][v] = t + u < L ? ld[u][v] : ~0ull;
                        pp = q[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < UU; ++u)
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        fold<K, NEG>(cu[v], cd[v], lu[u][v], NEG ? ld[u][v] : 0ull);
                p = pp;
                uint64_t live = 0;
#pragma unroll
                for (int v = 0; v < V; ++v)
                    live |= valid[v] & ~(NEG ? (cu[v][K] & cd[v][K]) : cu[v][K]);
                if (live == 0ull) break;
            }
        }
    };
    using tie_none = std::integral_constant<int, kTieNone>;
    using tie_mode = std::integral_constant<int, TIES>;
    using unroll = std::integral_constant<int, U>;
    if constexpr (NEG && TIES == kTieBitmap) {
        // Workgroups with a tied pair (rare) take batches of at most 2
        // pairs: the reverse words then never hold the kernel's register
        // count above that of the tie-free loop.
        using unroll_tied = std::integral_constant<int, (U < 2 ? U : 2)>;
        if (use_lds && !staged_bad && !staged_tie)
            lane_work(std::true_type{}, tie_none{}, unroll{});
        else if (use_lds)
            lane_work(std::true_type{}, tie_mode{}, unroll_tied{});
        else
            lane_work(std::false_type{}, tie_mode{}, unroll_tied{});
    } else {
        if (use_lds)
            lane_work(std::true_type{}, tie_mode{}, unroll{});
        else
            lane_work(std::false_type{}, tie_mode{}, unroll{});
    }

    int32_t rows = 0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const uint64_t pos = valid[v] & ~cu[v][K];
        const uint64_t neg = NEG ? (valid[v] & ~cd[v][K]) : 0ull;
        rows += __popcll(pos | neg);
        if (masks && active && w0 + v < W) {
            masks[R.mask_base + ((int64_t)cl * 2 + 0) * W + w0 + v] = pos;
            masks[R.mask_base + ((int64_t)cl * 2 + 1) * W + w0 + v] = neg;
        }
    }

    if constexpr (ALIGNED) {
        // The staging barrier above ordered the zeroing of s_rows/s_bad
        // before these updates.
        if (active) {
            atomicAdd(&s_rows[slot], rows);
            if (bad) s_bad[slot] = 1;
        }
        __syncthreads();
        if (active && g == 0)
            write_result(c, s_rows[slot], s_bad[slot] != 0, L, sigma, logt, counts, fitness);
        return;
    }

    // Segmented sum over lanes of the same candidate (lanes hold consecutive
    // items, so each candidate is one contiguous run of lanes): the run's
    // head gets the run's row count (low 16 bits, <= 64*64*V) and its number
    // of words (high bits), then reports them once.
    const int32_t words = active ? (int32_t)min<int64_t>(V, W - w0) : 0;
    int32_t packed = active ? (rows | (words << 16)) : 0;
    const int32_t cc = (int32_t)cl;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t x = __shfl_down(packed, off);
        const int32_t oc = __shfl_down(cc, off);
        if (lane + off < kWave && oc == cc) packed += x;
    }
    const int32_t prev_c = __shfl_up(cc, 1);
    const bool head = lane == 0 || prev_c != cc;
    // the first item of a candidate is always the first lane of its run,
    // hence a head itself.
    if (active && head)
        finish_part(c, (uint32_t)(packed & 0xFFFF), bad, packed >> 16, W, L, sigma, logt, acc,
                    counts, fitness);
}

}  // namespace
}  // namespace ebic
