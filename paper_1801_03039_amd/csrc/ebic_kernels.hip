// EBIC population evaluation kernels for gfx950 (CDNA4, wave64).
//
// The trend test (Motivation: row k follows the series p, q, r when
// a_kp < a_kq < a_kr, a strict comparison), its negative and approximate
// variants (Step 7), the row count |I| (Step 4), the row masks (Step 6) and
// the fitness of Eq. (1) are all computed here.  Nothing in this file is a
// dense contraction, so nothing uses MFMA: the work is gathers, compares and
// bit operations, bound by memory and VALU issue.
//
// Layouts
//   matrix  column-major FP32 a[j*npad + r], npad = 64*ceil(n/64), pad rows 0
//   index   idx[(p*m + q)*wpad + w]: bit b set when row 64w+b < n has
//           a[r,p] < a[r,q]; wpad = W rounded up to 8 words (64 bytes)
//   masks   masks[(c*2 + dir)*W + w], dir 0 rising, dir 1 falling
//
// One evaluation is one kernel launch: the part of each candidate that
// finishes last writes its count and fitness.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "ebic_internal.h"

namespace ebic {
namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
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

// ---------------------------------------------------------------- ingest --

// Row-major -> padded column-major through a 64x64 LDS tile.
__global__ __launch_bounds__(kBlock) void ingest_rows_kernel(const float *__restrict__ src,
                                                             int64_t n, int32_t m, int64_t ld,
                                                             int64_t npad, int64_t tiles_r,
                                                             float *__restrict__ dst) {
    __shared__ float tile[64][65];
    const int64_t tr = blockIdx.x % tiles_r;
    const int64_t tj = blockIdx.x / tiles_r;
    const int64_t r0 = tr * 64;
    const int32_t j0 = (int32_t)(tj * 64);
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i;
        const int32_t j = j0 + tx;
        tile[i][tx] = (r < n && j < m) ? src[r * ld + j] : 0.0f;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int32_t j = j0 + i;
        if (j < m) dst[(int64_t)j * npad + r0 + tx] = tile[tx][i];
    }
}

__global__ __launch_bounds__(kBlock) void ingest_cols_kernel(const float *__restrict__ src,
                                                             int64_t n, int32_t m, int64_t ld,
                                                             int64_t npad,
                                                             float *__restrict__ dst) {
    const int64_t total = (int64_t)m * npad;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t j = i / npad, r = i - j * npad;
        dst[i] = r < n ? src[j * ld + r] : 0.0f;
    }
}

// ----------------------------------------------------------- index build --
//
// One wave per (64-row word w, block of kPB columns p).  Lane = row.  The
// kPB values a[r,p] stay in registers while the wave streams every column q
// once: each compare is one ballot giving 64 rows of lt(p,q) at once.
constexpr int kPB = 16;

__global__ __launch_bounds__(kBlock) void index_build_kernel(const float *__restrict__ a,
                                                             int64_t n, int64_t npad, int32_t m,
                                                             int64_t W, int64_t wpad,
                                                             int64_t wblocks,
                                                             uint64_t *__restrict__ idx) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t wb = blockIdx.x % wblocks;
    const int32_t p0 = (int32_t)(blockIdx.x / wblocks) * kPB;
    const int64_t w = wb * 4 + wv;
    if (w >= W) return;  // uniform per wave
    const int64_t r = w * 64 + lane;
    const bool valid = r < n;
    float vp[kPB];
#pragma unroll
    for (int i = 0; i < kPB; ++i) vp[i] = (p0 + i < m) ? a[(int64_t)(p0 + i) * npad + r] : 0.0f;
    const bool writer = lane < kPB && p0 + lane < m;
    uint64_t *out = idx + ((int64_t)(p0 + lane) * m) * wpad + w;
    for (int32_t q = 0; q < m; ++q) {
        const float vq = a[(int64_t)q * npad + r];
        uint64_t mine = 0;
#pragma unroll
        for (int i = 0; i < kPB; ++i) {
            const uint64_t bits = ballot(valid && vp[i] < vq);
            mine = (lane == i) ? bits : mine;
        }
        if (writer) out[(int64_t)q * wpad] = mine;
    }
}

// Tie flags: tie[p*m + q] = 1 when some row r < n has a[r,p] and a[r,q]
// equal or unordered (NaN), i.e. when neither lt(p,q) nor lt(q,p) holds.
// For a pair without such a row the falling test needs no second order
// word: lt(q,p) = ~lt(p,q) on every row.  One wave per ordered pair, lanes
// over words.
__global__ __launch_bounds__(kBlock) void tie_flags_kernel(const uint64_t *__restrict__ idx,
                                                           int64_t n, int32_t m, int64_t W,
                                                           int64_t wpad,
                                                           uint8_t *__restrict__ tie) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t pair = (int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6);
         pair < (int64_t)m * m; pair += waves) {  // uniform per wave
        const int64_t p = pair / m, q = pair - p * m;
        const uint64_t *pq = idx + pair * wpad;
        const uint64_t *qp = idx + (q * m + p) * wpad;
        bool any = false;
        for (int64_t w = lane; w < W; w += kWave)
            any |= (~(pq[w] | qp[w]) & tail_bits(n, w, W)) != 0ull;
        const uint64_t hit = ballot(any);
        if (lane == 0) tie[pair] = hit ? 1 : 0;
    }
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

// ------------------------------------------------------- direct evaluator --
//
// Workgroup = (candidate c, row slice s); 4 waves, lane = row.  The
// candidate's column offsets (col * npad) are staged in LDS once; each wave
// walks 64-row blocks of its slice, reading the row's values along the
// series (coalesced 256-byte loads of the column-major matrix), counting
// violating pairs per lane and leaving the block as soon as every row of the
// wave is decided.  With 8 slices, slice s runs on XCD s (workgroups are
// dealt to the 8 XCDs round-robin), so each XCD's L2 holds one eighth of
// the matrix.
template <bool NEG>
__global__ __launch_bounds__(kBlock) void eval_direct_kernel(
    const float *__restrict__ a, int64_t n, int64_t npad, int32_t m, int64_t W, int32_t S,
    const int32_t *__restrict__ offsets, const int32_t *__restrict__ cols, int64_t n_entries,
    int32_t k, int32_t sigma, const double *__restrict__ logt, uint64_t *__restrict__ masks,
    unsigned long long *__restrict__ acc, int32_t *__restrict__ counts,
    double *__restrict__ fitness) {
    __shared__ int64_t s_off[kDirectLdsCols];
    __shared__ int32_t s_bad;
    __shared__ int32_t s_cnt[kBlock / kWave];
    const int c = (int)(blockIdx.x / S);
    const int s = (int)(blockIdx.x % S);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    const int64_t start = offsets[c], end = offsets[c + 1];
    const bool ok_range = start >= 0 && end <= n_entries && end > start;
    if (tid == 0) s_bad = ok_range ? 0 : 1;
    __syncthreads();
    const int32_t L = ok_range ? (int32_t)(end - start) : 0;
    for (int32_t t = tid; t < L; t += kBlock) {
        const int32_t col = cols[start + t];
        if (col < 0 || col >= m) s_bad = 1;
        if (t < kDirectLdsCols) s_off[t] = (int64_t)(col < 0 || col >= m ? 0 : col) * npad;
    }
    __syncthreads();
    const bool bad = s_bad != 0;
    if (bad) {  // uniform per workgroup
        if (s == 0 && tid == 0) {
            counts[c] = -1;
            fitness[c] = __builtin_nan("");
        }
        return;
    }

    const int64_t rb0 = (W * s) / S, rb1 = (W * (s + 1)) / S;
    int32_t cnt = 0;
    for (int64_t rb = rb0 + wv; rb < rb1; rb += kBlock / kWave) {
        const int64_t r = rb * 64 + lane;
        const bool valid = r < n;
        const float *base = a + r;
        float prev = base[s_off[0]];
        int32_t vu = 0, vd = 0;
        for (int32_t t0 = 1; t0 < L; t0 += 4) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t t = t0 + u;
                if (t < L) {
                    const int64_t off =
                        t < kDirectLdsCols ? s_off[t] : (int64_t)cols[start + t] * npad;
                    v[u] = base[off];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (t0 + u < L) {
                    vu += !(prev < v[u]);
                    if (NEG) vd += !(prev > v[u]);
                    prev = v[u];
                }
            }
            const bool alive = (vu <= k) || (NEG && vd <= k);
            if (ballot(alive && valid) == 0) break;
        }
        const uint64_t bp = ballot(valid && vu <= k);
        const uint64_t bn = NEG ? ballot(valid && vd <= k) : 0ull;
        cnt += __popcll(bp | bn);
        if (masks && lane == 0) {
            masks[((int64_t)c * 2 + 0) * W + rb] = bp;
            masks[((int64_t)c * 2 + 1) * W + rb] = bn;
        }
    }
    if (lane == 0) s_cnt[wv] = cnt;
    __syncthreads();
    if (tid == 0) {
        int32_t sum = 0;
        for (int i = 0; i < kBlock / kWave; ++i) sum += s_cnt[i];
        finish_part(c, (uint32_t)sum, false, 1, S, L, sigma, logt, acc, counts, fitness);
    }
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
// b has more than i violations.  lt(q,p) is read only for pairs whose tie
// flag is set; otherwise it is ~lt(p,q).  Loads for kUnroll pairs are issued before
// any is consumed (the lane's latency chain is one order-word round trip per
// kUnroll pairs), and a lane stops once every row of its word is rejected in
// every enabled direction.
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

// One tile of one run.  An item is a candidate and V consecutive 64-row
// words of it (V words per lane share the lane's column reads and loop).
// Two tilings:
//   ALIGNED = false: kBlock consecutive items of the flattened (candidate,
//     item) order; a candidate may span workgroups, so each workgroup adds
//     its share of a candidate's count with one packed global atomic and the
//     last share writes the result (finish_part).  Shared by the single-run
//     kernel and the persistent multi-run kernel.
//   ALIGNED = true: the workgroup holds `cpw` whole candidates (requires
//     ceil(W / V) <= kBlock); counts are summed with LDS atomics and the
//     first lane of each candidate writes its result after a workgroup
//     barrier -- no global atomics and no accumulator scratch.
template <int K, bool NEG, int U, int V, bool ALIGNED, bool TIES = true, bool OFF32 = false>
__device__ __forceinline__ void index_tile(const IndexRun &R, uint32_t tile, uint32_t cpw,
                                           const int32_t *__restrict__ offsets,
                                           const int32_t *__restrict__ cols, int64_t n_entries,
                                           int32_t sigma, uint64_t *__restrict__ masks,
                                           unsigned long long *__restrict__ acc,
                                           int32_t *__restrict__ counts,
                                           double *__restrict__ fitness) {
    static_assert(V == 1 || V == 2 || V == 4, "words per lane");
    __shared__ int32_t s_cols[kIdxLds];
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

    const int64_t start = offsets[c], end = offsets[c + 1];
    const bool ok_range = start >= 0 && end <= n_entries && end > start;
    const int32_t L = ok_range ? (int32_t)(end - start) : 0;

    // Stage the columns of candidates [c_lo, c_hi] in LDS when they fit and
    // every lane's series lies inside the staged span (always, for a
    // well-formed CBF); otherwise the whole workgroup reads them from global
    // memory.  The choice is uniform over the workgroup.
    const int64_t b0 = offsets[R.cand_base + c_lo], b1 = offsets[R.cand_base + c_hi + 1];
    __shared__ int32_t s_rows[ALIGNED ? kBlock : 1];
    __shared__ int32_t s_bad[ALIGNED ? kBlock : 1];
    if (ALIGNED && (uint32_t)tid < cpw) {
        s_rows[tid] = 0;
        s_bad[tid] = 0;
    }
    const bool span_ok = b0 >= 0 && b1 <= n_entries && b1 >= b0 && b1 - b0 <= kIdxLds;
    const bool lane_ok = !ok_range || (start >= b0 && end <= b1);
    const bool use_lds = __syncthreads_and(span_ok && lane_ok) != 0;
    // Staging also checks every staged column: when none is out of range
    // (the common case) the per-candidate validation below is skipped.
    bool staged_bad = true;
    if (use_lds) {
        bool inval = false;
        for (int32_t e = tid; e < (int32_t)(b1 - b0); e += (int32_t)blockDim.x) {
            const int32_t x = cols[b0 + e];
            inval |= x < 0 || x >= m;
            s_cols[e] = x;
        }
        staged_bad = __syncthreads_or(inval) != 0;
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

    // Per-lane work, instantiated for columns in LDS or in global memory.
    auto lane_work = [&](auto from_lds) {
        constexpr bool kLds = decltype(from_lds)::value;
        auto col = [&](int32_t t) -> int32_t {
            if constexpr (kLds) return s_cols[lds0 + t];
            else return cols[start + t];
        };
        // The lane of the first word validates every column (batched,
        // branch-free reads; skipped when staging found every staged column
        // in range) and reports the verdict with its part; other lanes only
        // clamp column indices so that no read leaves the index.
        if (active && g == 0) bad = !ok_range;
        if (active && g == 0 && (!kLds || staged_bad)) {
            for (int32_t t = 0; t < L; t += U) {
                int32_t x[U];
#pragma unroll
                for (int u = 0; u < U; ++u) x[u] = col(min(t + u, L - 1));
#pragma unroll
                for (int u = 0; u < U; ++u) bad |= (x[u] < 0 || x[u] >= m);
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
        const int32_t last = L - 1;
        int32_t p = col(0);
        p = (p < 0 || p >= m) ? 0 : p;
        for (int32_t t = 1; t < L; t += U) {
            // Column reads and order-word loads of the batch are issued
            // unconditionally (indices past the end repeat the last column,
            // a harmless in-bounds read whose words are then ignored).
            int32_t q[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t x = col(min(t + u, last));
                q[u] = (x < 0 || x >= m) ? 0 : x;
            }
            uint64_t lu[U][V], ld[U][V];
            uint8_t tf[U];
            int32_t pp = p;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t pq = (int64_t)pp * m + q[u];
                load_words<V>(words_at(pq), lu[u]);
                if (NEG) tf[u] = TIES ? tie[pq] : 0;
                pp = q[u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
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
                for (int u = 0; u < U; ++u) {
                    if (TIES && tf[u]) {
                        load_words<V>(words_at((int64_t)q[u] * m + pp), ld[u]);
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v) ld[u][v] = ~lu[u][v];
                    }
#pragma unroll
                    for (int v = 0; v < V; ++v) ld[u][v] = t + u < L ? ld[u][v] : ~0ull;
                    pp = q[u];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
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
    };
    if (use_lds)
        lane_work(std::true_type{});
    else
        lane_work(std::false_type{});

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

template <int K, bool NEG, int U, int V, bool ALIGNED, bool TIES, bool OFF32>
__global__ __launch_bounds__(kBlock) void eval_index_kernel(
    IndexRun R, uint32_t cpw, const int32_t *__restrict__ offsets,
    const int32_t *__restrict__ cols, int64_t n_entries, int32_t sigma,
    uint64_t *__restrict__ masks, unsigned long long *__restrict__ acc,
    int32_t *__restrict__ counts, double *__restrict__ fitness) {
    index_tile<K, NEG, U, V, ALIGNED, TIES, OFF32>(R, blockIdx.x, cpw, offsets, cols, n_entries,
                                                   sigma, masks, acc, counts, fitness);
}

// --------------------------------------------------- batched (many runs) --
//
// One persistent launch evaluates one population per run for many runs with
// matrices of different shapes.  The work is a queue of tiles (kBlock
// consecutive (candidate, word) items of one run), run after run; each
// workgroup takes the next tile with an atomic until the queue is empty.
// The last workgroup to leave resets the queue, so the launch can be
// replayed (a captured graph) without any clearing step.  work[0] is the
// next tile, work[1] the number of workgroups that have left.
constexpr int kRunsLds = 1024;   // tile bases kept in LDS (more runs: read from memory)
static_assert(sizeof(IndexRun) % 8 == 0, "run descriptor copied as 8-byte words");

template <int K, bool NEG, int U, int V>
__global__ __launch_bounds__(kBlock) void eval_index_batch_kernel(
    const IndexRun *__restrict__ runs, const uint32_t *__restrict__ tile_base, int32_t n_runs,
    unsigned int *__restrict__ work, const int32_t *__restrict__ offsets,
    const int32_t *__restrict__ cols, int64_t n_entries, int32_t sigma,
    uint64_t *__restrict__ masks, unsigned long long *__restrict__ acc,
    int32_t *__restrict__ counts, double *__restrict__ fitness) {
    __shared__ uint32_t s_tb[kRunsLds + 1];
    __shared__ IndexRun s_R;
    __shared__ uint32_t s_tile, s_local;
    __shared__ int32_t s_run;
    const int tid = threadIdx.x;
    const bool tb_lds = n_runs <= kRunsLds;
    if (tb_lds)
        for (int32_t i = tid; i <= n_runs; i += kBlock) s_tb[i] = tile_base[i];
    const uint32_t total_tiles = tile_base[n_runs];
    if (work == nullptr) {
        // One tile per workgroup (grid = total tiles): no queue.
        __syncthreads();  // s_tb filled
        const uint32_t t = blockIdx.x;
        if (t >= total_tiles) return;  // uniform
        int32_t lo = 0, hi = n_runs - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            const uint32_t base = tb_lds ? s_tb[mid] : tile_base[mid];
            if (base <= t) lo = mid; else hi = mid - 1;
        }
        const uint32_t local = t - (tb_lds ? s_tb[lo] : tile_base[lo]);
        index_tile<K, NEG, U, V, false>(runs[lo], local, 0, offsets, cols, n_entries, sigma, masks,
                                        acc, counts, fitness);
        return;
    }
    // Thread 0 claims the next tile one iteration ahead, so the queue's
    // atomic round trip overlaps the current tile's work.
    uint32_t next = 0;
    if (tid == 0) next = atomicAdd(work, 1u);
    __syncthreads();  // s_tb filled
    for (;;) {
        if (tid == 0) {
            const uint32_t t = next;
            int32_t r = 0;
            if (t < total_tiles) {
                // last run whose first tile is <= t
                int32_t lo = 0, hi = n_runs - 1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    const uint32_t base = tb_lds ? s_tb[mid] : tile_base[mid];
                    if (base <= t) lo = mid; else hi = mid - 1;
                }
                r = lo;
                s_local = t - (tb_lds ? s_tb[r] : tile_base[r]);
            }
            s_tile = t;
            s_run = r;
        }
        __syncthreads();
        const uint32_t t = s_tile;
        if (t >= total_tiles) break;  // uniform
        // the tile's run descriptor into LDS, one 8-byte word per thread
        constexpr int kWords = (int)(sizeof(IndexRun) / 8);
        if (tid < kWords)
            reinterpret_cast<uint64_t *>(&s_R)[tid] =
                reinterpret_cast<const uint64_t *>(runs + s_run)[tid];
        if (tid == 0) next = atomicAdd(work, 1u);
        __syncthreads();
        index_tile<K, NEG, U, V, false>(s_R, s_local, 0, offsets, cols, n_entries, sigma, masks,
                                        acc, counts, fitness);
        __syncthreads();  // every wave is done with s_R, s_local and s_cols
    }
    if (tid == 0) {
        const unsigned left = atomicAdd(work + 1, 1u);
        if (left == gridDim.x - 1) {
            atomicExch(work, 0u);
            atomicExch(work + 1, 0u);
        }
    }
}

}  // namespace

// ----------------------------------------------------------- launchers --

hipError_t launch_ingest(const float *src, int64_t n, int32_t m, int64_t ld, int32_t layout,
                         int64_t npad, float *dst, hipStream_t stream) {
    if (layout == EBIC_ROW_MAJOR) {
        const int64_t tiles_r = npad / 64, tiles_j = (m + 63) / 64;
        hipLaunchKernelGGL(ingest_rows_kernel, dim3((unsigned)(tiles_r * tiles_j)), dim3(kBlock),
                           0, stream, src, n, m, ld, npad, tiles_r, dst);
    } else {
        const int64_t total = (int64_t)m * npad;
        int64_t blocks = (total + kBlock - 1) / kBlock;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(ingest_cols_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream,
                           src, n, m, ld, npad, dst);
    }
    return hipGetLastError();
}

hipError_t launch_index_build(const float *a, int64_t n, int64_t npad, int32_t m, int64_t W,
                              int64_t wpad, uint64_t *idx, uint8_t *tie, hipStream_t stream) {
    const int64_t wblocks = (W + 3) / 4;
    const int64_t pblocks = (m + kPB - 1) / kPB;
    hipLaunchKernelGGL(index_build_kernel, dim3((unsigned)(wblocks * pblocks)), dim3(kBlock), 0,
                       stream, a, n, npad, m, W, wpad, wblocks, idx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t pairs = (int64_t)m * m;
    const int64_t waves_per_block = kBlock / kWave;
    int64_t blocks = (pairs + waves_per_block - 1) / waves_per_block;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(tie_flags_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, idx, n, m,
                       W, wpad, tie);
    return hipGetLastError();
}

hipError_t launch_eval_direct(const float *a, int64_t n, int64_t npad, int32_t m, int64_t W,
                              const EvalArgs &e, hipStream_t stream) {
    const int32_t S = W >= 32 ? kXcds : 1;
    const dim3 grid((unsigned)((int64_t)e.P * S));
    if (e.negative)
        hipLaunchKernelGGL(eval_direct_kernel<true>, grid, dim3(kBlock), 0, stream, a, n, npad, m,
                           W, S, e.offsets, e.cols, e.n_entries, e.k, e.sigma, e.logt, e.masks,
                           e.acc, e.counts, e.fitness);
    else
        hipLaunchKernelGGL(eval_direct_kernel<false>, grid, dim3(kBlock), 0, stream, a, n, npad,
                           m, W, S, e.offsets, e.cols, e.n_entries, e.k, e.sigma, e.logt, e.masks,
                           e.acc, e.counts, e.fitness);
    return hipGetLastError();
}

// Falling trends read tie flags (and reverse words) only when the matrix
// has a tied or unordered pair somewhere (`ties`); otherwise lt(q,p) is
// ~lt(p,q) for every pair and the flags are not loaded.
template <int K, int U, int V, bool ALIGNED, bool OFF32>
static void launch_index_o(const IndexRun &R, uint32_t cpw, dim3 grid, dim3 block,
                           const EvalArgs &e, bool ties, hipStream_t stream) {
    if (e.negative && ties)
        hipLaunchKernelGGL((eval_index_kernel<K, true, U, V, ALIGNED, true, OFF32>), grid, block,
                           0, stream, R, cpw, e.offsets, e.cols, e.n_entries, e.sigma, e.masks,
                           e.acc, e.counts, e.fitness);
    else if (e.negative)
        hipLaunchKernelGGL((eval_index_kernel<K, true, U, V, ALIGNED, false, OFF32>), grid, block,
                           0, stream, R, cpw, e.offsets, e.cols, e.n_entries, e.sigma, e.masks,
                           e.acc, e.counts, e.fitness);
    else
        hipLaunchKernelGGL((eval_index_kernel<K, false, U, V, ALIGNED, false, OFF32>), grid, block,
                           0, stream, R, cpw, e.offsets, e.cols, e.n_entries, e.sigma, e.masks,
                           e.acc, e.counts, e.fitness);
}

// 32-bit index offsets when the whole index is below 4 GiB.
template <int K, int U, int V, bool ALIGNED>
static void launch_index_t(const IndexRun &R, uint32_t cpw, dim3 grid, dim3 block,
                           const EvalArgs &e, bool ties, hipStream_t stream) {
    const uint64_t bytes = (uint64_t)R.m * (uint64_t)R.m * (uint64_t)R.wpad * 8ull;
    if (bytes <= 0xFFFFFFFFull)
        launch_index_o<K, U, V, ALIGNED, true>(R, cpw, grid, block, e, ties, stream);
    else
        launch_index_o<K, U, V, ALIGNED, false>(R, cpw, grid, block, e, ties, stream);
}

template <int K, int U, int V>
static void launch_aligned(const IndexRun &R, const EvalArgs &e, bool ties, hipStream_t stream) {
    const int64_t Wg = (R.W + V - 1) / V;
    const int64_t cpw = kBlock / Wg;
    const int64_t threads = (cpw * Wg + kWave - 1) / kWave * kWave;
    const dim3 grid((unsigned)((R.P + cpw - 1) / cpw));
    launch_index_t<K, U, V, true>(R, (uint32_t)cpw, grid, dim3((unsigned)threads), e, ties,
                                  stream);
}

// Tiling by matrix height.  Up to 1024 words (65536 rows) a workgroup holds
// whole candidates: 1 word per lane up to 128 words, 2 up to 512 (measured
// faster than 1 from 128 words on: half the lanes, twice the loads in
// flight), 4 up to 1024; as many candidates per workgroup as fit, and a
// workgroup just large enough (whole waves) to hold them.  Taller matrices
// use the flattened tiling with 2 words per lane.
template <int K, int U>
static void launch_index_k(const IndexRun &R, const EvalArgs &e, bool ties, hipStream_t stream) {
    if (R.W <= kBlock / 2)
        launch_aligned<K, U, 1>(R, e, ties, stream);
    else if (R.W <= 2 * kBlock)
        launch_aligned<K, U, 2>(R, e, ties, stream);
    else if (R.W <= 4 * kBlock)
        launch_aligned<K, U, 4>(R, e, ties, stream);
    else {
        constexpr int V = kWordsPerLane;
        const int64_t total = (int64_t)R.P * ((R.W + V - 1) / V);
        const dim3 grid((unsigned)((total + kBlock - 1) / kBlock));
        launch_index_t<K, U, V, false>(R, 0, grid, dim3(kBlock), e, ties, stream);
    }
}

hipError_t launch_eval_index(const uint64_t *idx, const uint8_t *tie, bool ties, int64_t n,
                             int32_t m, int64_t W, int64_t wpad, const EvalArgs &e,
                             hipStream_t stream) {
    const IndexRun R{idx, tie, e.logt, n, W, wpad, m, e.P, 0, 0};
    switch (e.k) {
    case 0: launch_index_k<0, kUnroll>(R, e, ties, stream); break;
    case 1: launch_index_k<1, kUnroll>(R, e, ties, stream); break;
    case 2: launch_index_k<2, kUnroll>(R, e, ties, stream); break;
    case 3: launch_index_k<3, kUnroll>(R, e, ties, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int K, int U, int V>
static void launch_batch_k(const BatchLaunch &b, hipStream_t stream) {
    if (b.negative)
        hipLaunchKernelGGL((eval_index_batch_kernel<K, true, U, V>), dim3(b.grid), dim3(kBlock), 0,
                           stream, b.runs, b.tile_base, b.n_runs, b.work, b.offsets, b.cols,
                           b.n_entries, b.sigma, b.masks, b.acc, b.counts, b.fitness);
    else
        hipLaunchKernelGGL((eval_index_batch_kernel<K, false, U, V>), dim3(b.grid), dim3(kBlock),
                           0, stream, b.runs, b.tile_base, b.n_runs, b.work, b.offsets, b.cols,
                           b.n_entries, b.sigma, b.masks, b.acc, b.counts, b.fitness);
}

template <int U, int V>
static hipError_t launch_batch_uv(const BatchLaunch &b, hipStream_t stream) {
    switch (b.k) {
    case 0: launch_batch_k<0, U, V>(b, stream); break;
    case 1: launch_batch_k<1, U, V>(b, stream); break;
    case 2: launch_batch_k<2, U, V>(b, stream); break;
    case 3: launch_batch_k<3, U, V>(b, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int V>
static hipError_t launch_batch_v(const BatchLaunch &b, hipStream_t stream) {
    switch (b.unroll) {
    case 2: return launch_batch_uv<2, V>(b, stream);
    case 4: return launch_batch_uv<4, V>(b, stream);
    case 8: return launch_batch_uv<8, V>(b, stream);
    default: return hipErrorInvalidValue;
    }
}

int batch_wgs_per_cu() {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks,
                                                     eval_index_batch_kernel<1, true, 4, 1>,
                                                     kBlock, 0) != hipSuccess || blocks < 1)
        blocks = 1;
    return blocks;
}

hipError_t launch_eval_index_batch(const BatchLaunch &b, hipStream_t stream) {
    switch (b.words) {
    case 1: return launch_batch_v<1>(b, stream);
    case 2: return launch_batch_v<2>(b, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ebic
