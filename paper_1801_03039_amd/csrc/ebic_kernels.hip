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
//           a[r,p] < a[r,q]; wpad = W rounded up to 16 words (128 bytes)
//   masks   masks[(c*2 + dir)*W + w], dir 0 rising, dir 1 falling
//
// One evaluation is one kernel launch: the part of each candidate that
// finishes last writes its count and fitness.
#include "ebic_device.h"

namespace ebic {
namespace {

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
// Workgroup = 4 waves over one block of kRW consecutive 64-row words (lane =
// row within each word), one group of kPG columns p (kPW per wave, their
// values for the block's rows held in registers) and one chunk of kQC
// columns q.  Each unordered pair {p, q} is built by one wave: the wave
// whose p columns hold the smaller column (q < p0 is skipped; in a diagonal
// block some words are written twice, with equal values).  Per q and word
// the wave takes two ballots, lt = (a[r,p] < a[r,q]) and gt = (a[r,q] <
// a[r,p]); lt is word w of order row (p,q), and a valid row in neither
// (equal values, or a NaN) ties the pair.  Only lt is moved into the lane
// that stores it (lane kRW*i + j holds column p0+i and word j, two
// v_writelane); order row (q,p) is then ~lt restricted to the valid rows,
// minus the tied rows, which are moved into the lanes only for the rare
// (pair, q) that has one.  One store instruction writes kRW contiguous
// words (128 bytes) of each of kPW order rows, and one more the kPW
// reverse rows.
//
// Tie flags: tie[p*m + q] = tie[q*m + p] = 1 for a tied pair (zeroed before
// the launch; every writer stores 1), and any_tie[0] = 1 when a pair of
// distinct columns ties (a column always ties with itself: lt(p,p) = 0);
// a tied pair of distinct columns also sets its two bits of the tie-pair
// bitmap (atomic OR; zeroed before the launch).
//
// A ballot of an ordered not-equal compare is avoided: the compiler lowers
// it to the unordered form (true for NaN); lt and gt are ordered less-than
// compares.
constexpr int kRW = 16;               // 64-row words per row block
constexpr int kPW = 4;                // columns p per wave
constexpr int kPG = kPW * kBlock / kWave;   // columns p per workgroup (16)
constexpr int kQC = 16;               // columns q per workgroup
static_assert(kPW * kRW == kWave, "one stored word per lane");
static_assert(kQC == kPG, "a column group and a column chunk cover the same columns");

// v_writelane_b32 through its LLVM intrinsic (clang has no builtin for it):
// lane `lane` of the result takes the uniform value `src`, the other lanes
// keep `old`.  It moves a ballot (two SGPRs) into the lane that stores it.
__device__ int32_t amdgcn_writelane(int32_t src, int32_t lane, int32_t old)
    __asm("llvm.amdgcn.writelane.i32");

__global__ __launch_bounds__(kBlock) void index_fill_kernel(uint8_t *__restrict__ tie,
                                                            int64_t n_bytes,
                                                            int32_t *__restrict__ any_tie,
                                                            uint32_t *__restrict__ tbits) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n_bytes) tie[i] = 0;
    if (i < kTieWords) tbits[i] = 0;
    if (i == 0) any_tie[0] = 0;
}

__global__ __launch_bounds__(kBlock) void index_build_kernel(
    const float *__restrict__ a, int64_t n, int64_t npad, int32_t m, int64_t W, int64_t wpad,
    int32_t G, int64_t pairs, int64_t tiles, int64_t per_xcd, uint64_t *__restrict__ idx,
    uint8_t *__restrict__ tie, int32_t *__restrict__ any_tie, uint32_t *__restrict__ tbits) {
    // Tiles in (row block, column-group pair) order; XCD x (workgroups are
    // dealt round-robin to the 8 XCDs) takes the x-th contiguous range, so
    // the workgroups of a row block share one L2.
    const int64_t t = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    if (t >= tiles) return;
    const int64_t rb = t / pairs;
    int64_t k = t - rb * pairs;
    // k-th pair (g, h), g <= h < G, in row-major order of the upper triangle
    int32_t g = 0;
    {
        int32_t lo = 0, hi = G - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            const int64_t first = (int64_t)mid * G - (int64_t)mid * (mid - 1) / 2;
            if (first <= k) lo = mid; else hi = mid - 1;
        }
        g = lo;
        k -= (int64_t)g * G - (int64_t)g * (g - 1) / 2;
    }
    const int32_t h = g + (int32_t)k;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t p0 = g * kPG + wv * kPW;
    if (p0 >= m) return;                                    // uniform per wave
    const int32_t q_lo = max(h * kQC, p0), q_hi = min(h * kQC + kQC, m);
    if (q_lo >= q_hi) return;                               // uniform per wave
    const int64_t w0 = rb * kRW;
    const int32_t jn = (int32_t)min<int64_t>(kRW, W - w0);   // words of the block in the matrix
    const uint64_t last = tail_bits(n, w0 + jn - 1, W);      // rows of its last word
    // Word j of the block: rows r = 64*(w0 + j) + lane.  Loads past the
    // matrix (j >= jn, or a column past m) read a clamped, valid address and
    // their results are masked off.
    auto row_of = [&](int j) { return min<int64_t>(w0 + j, W - 1) * 64 + lane; };

    float vp[kPW][kRW];
#pragma unroll
    for (int i = 0; i < kPW; ++i) {
        const float *col = a + (int64_t)min(p0 + i, m - 1) * npad;
#pragma unroll
        for (int j = 0; j < kRW; ++j) vp[i][j] = col[row_of(j)];
    }
    // the (column, word) this lane stores, and the valid rows of that word
    const int32_t sp = p0 + lane / kRW;
    const int64_t sw = w0 + lane % kRW;
    const bool store = sp < m && sw < W;
    const uint64_t sw_valid = sw < W ? tail_bits(n, sw, W) : 0ull;

    // FULL: every row of the block's kRW words is in the matrix (all but
    // the last block), so no valid-row masks are needed.
    auto run = [&](auto full) {
        constexpr bool FULL = decltype(full)::value;
        auto valid = [&](int j) -> uint64_t {
            if constexpr (FULL) return ~0ull;
            else return j + 1 < jn ? ~0ull : (j + 1 == jn ? last : 0ull);
        };
        for (int32_t q = q_lo; q < q_hi; ++q) {
            float vq[kRW];
            const float *col = a + (int64_t)q * npad;
#pragma unroll
            for (int j = 0; j < kRW; ++j) vq[j] = col[row_of(j)];
            int32_t lt_lo = 0, lt_hi = 0, tie_lo = 0, tie_hi = 0;
            uint64_t tied = 0;   // some valid row of the block ties the pair (p0+i, q)
#pragma unroll
            for (int i = 0; i < kPW; ++i) {
                uint64_t ti = 0;
#pragma unroll
                for (int j = 0; j < kRW; ++j) {
                    // pad rows hold 0 in every column, so lt is 0 there
                    const uint64_t lt = ballot(vp[i][j] < vq[j]);
                    const uint64_t gt = ballot(vq[j] < vp[i][j]);
                    ti |= valid(j) & ~(lt | gt);
                    lt_lo = amdgcn_writelane((int32_t)(uint32_t)lt, i * kRW + j, lt_lo);
                    lt_hi = amdgcn_writelane((int32_t)(uint32_t)(lt >> 32), i * kRW + j, lt_hi);
                }
                tied |= (ti != 0ull ? 1ull : 0ull) << i;
            }
            if (tied != 0ull) {   // rare (always for q in [p0, p0 + kPW))
                // the tied rows of each tied pair, word by word: equal values or a NaN
#pragma unroll
                for (int i = 0; i < kPW; ++i) {
                    if (!((tied >> i) & 1ull) || p0 + i >= m) continue;
#pragma unroll
                    for (int j = 0; j < kRW; ++j) {
                        const uint64_t t = (ballot(vp[i][j] == vq[j]) | ballot(vp[i][j] != vp[i][j]) |
                                            ballot(vq[j] != vq[j])) & valid(j);
                        tie_lo = amdgcn_writelane((int32_t)(uint32_t)t, i * kRW + j, tie_lo);
                        tie_hi = amdgcn_writelane((int32_t)(uint32_t)(t >> 32), i * kRW + j,
                                                  tie_hi);
                    }
                    if (lane == 0) {
                        const int32_t p = p0 + i;
                        tie[(int64_t)p * m + q] = 1;
                        tie[(int64_t)q * m + p] = 1;
                        if (p != q) {
                            any_tie[0] = 1;
                            const uint32_t h0 = tie_hash((uint32_t)p * (uint32_t)m + (uint32_t)q);
                            const uint32_t h1 = tie_hash((uint32_t)q * (uint32_t)m + (uint32_t)p);
                            atomicOr(tbits + (h0 >> 5), 1u << (h0 & 31));
                            atomicOr(tbits + (h1 >> 5), 1u << (h1 & 31));
                        }
                    }
                }
            }
            if (store) {
                const uint64_t lt = ((uint64_t)(uint32_t)lt_hi << 32) | (uint32_t)lt_lo;
                const uint64_t tw = ((uint64_t)(uint32_t)tie_hi << 32) | (uint32_t)tie_lo;
                idx[((int64_t)sp * m + q) * wpad + sw] = lt;
                idx[((int64_t)q * m + sp) * wpad + sw] = ~lt & sw_valid & ~tw;
            }
        }
    };
    if (jn == kRW && last == ~0ull)
        run(std::true_type{});
    else
        run(std::false_type{});
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

template <int K, bool NEG, int U, int V, bool ALIGNED, int TIES, bool OFF32, bool TAIL>
__global__ __launch_bounds__(kAlignedThreads) void eval_index_kernel(
    IndexRun R, uint32_t cpw, const int32_t *__restrict__ offsets,
    const int32_t *__restrict__ cols, int64_t n_entries, int32_t sigma,
    uint64_t *__restrict__ masks, unsigned long long *__restrict__ acc,
    int32_t *__restrict__ counts, double *__restrict__ fitness) {
    __shared__ TileLds lds;
    index_tile<K, NEG, U, V, ALIGNED, TIES, OFF32, TAIL>(R, blockIdx.x, cpw, offsets, cols,
                                                         n_entries, sigma, masks, acc, counts,
                                                         fitness, lds);
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
                              int64_t wpad, uint64_t *idx, uint8_t *tie, int32_t *any_tie,
                              uint32_t *tbits, hipStream_t stream) {
    const int64_t flags = (int64_t)m * m;
    const int64_t fill = flags > kTieWords ? flags : kTieWords;
    hipLaunchKernelGGL(index_fill_kernel, dim3((unsigned)((fill + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, stream, tie, flags, any_tie, tbits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int32_t G = (m + kPG - 1) / kPG;
    const int64_t pairs = (int64_t)G * (G + 1) / 2;
    const int64_t rblocks = (W + kRW - 1) / kRW;
    const int64_t tiles = rblocks * pairs;
    const int64_t per_xcd = (tiles + kXcds - 1) / kXcds;
    const int64_t grid = per_xcd * kXcds;
    if (grid > 0x7FFFFFFFll) return hipErrorInvalidValue;
    hipLaunchKernelGGL(index_build_kernel, dim3((unsigned)grid), dim3(kBlock), 0, stream, a, n,
                       npad, m, W, wpad, G, pairs, tiles, per_xcd, idx, tie, any_tie, tbits);
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

// Falling trends consult the tie-pair bitmap (and read reverse words) only
// when two distinct columns of the matrix tie somewhere (`ties`); otherwise
// lt(q,p) is ~lt(p,q) for every pair of distinct columns.  The bitmap is
// staged in LDS, so a pair's test is an LDS read rather than a load of its
// byte flag (measured 10.6 -> 9.6 us per launch for the expression
// workload, whose matrix has 10 tied pairs).
template <int K, int U, int V, bool ALIGNED, bool OFF32, bool TAIL>
static void launch_index_o(const IndexRun &R, uint32_t cpw, dim3 grid, dim3 block,
                           const EvalArgs &e, bool ties, hipStream_t stream) {
    if (e.negative && ties)
        hipLaunchKernelGGL((eval_index_kernel<K, true, U, V, ALIGNED, kTieBitmap, OFF32, TAIL>), grid, block,
                           0, stream, R, cpw, e.offsets, e.cols, e.n_entries, e.sigma, e.masks,
                           e.acc, e.counts, e.fitness);
    else if (e.negative)
        hipLaunchKernelGGL((eval_index_kernel<K, true, U, V, ALIGNED, kTieNone, OFF32, TAIL>), grid, block,
                           0, stream, R, cpw, e.offsets, e.cols, e.n_entries, e.sigma, e.masks,
                           e.acc, e.counts, e.fitness);
    else
        hipLaunchKernelGGL((eval_index_kernel<K, false, U, V, ALIGNED, kTieNone, OFF32, TAIL>), grid, block,
                           0, stream, R, cpw, e.offsets, e.cols, e.n_entries, e.sigma, e.masks,
                           e.acc, e.counts, e.fitness);
}

// 32-bit index offsets when the whole index is below 4 GiB.
template <int K, int U, int V, bool ALIGNED, bool TAIL = false>
static void launch_index_t(const IndexRun &R, uint32_t cpw, dim3 grid, dim3 block,
                           const EvalArgs &e, bool ties, hipStream_t stream) {
    const uint64_t bytes = (uint64_t)R.m * (uint64_t)R.m * (uint64_t)R.wpad * 8ull;
    if (bytes <= 0xFFFFFFFFull)
        launch_index_o<K, U, V, ALIGNED, true, TAIL>(R, cpw, grid, block, e, ties, stream);
    else
        launch_index_o<K, U, V, ALIGNED, false, TAIL>(R, cpw, grid, block, e, ties, stream);
}

// Whole-candidate workgroups.  With 4 words per lane, as many candidates as
// fit in 256 lanes.  With 1 or 2, the candidate count (up to 320 lanes) that
// leaves the fewest idle lanes in the workgroup's whole waves: e.g. 2
// candidates of 157 lanes in 5 waves instead of 1 in 3 waves with 35 idle
// lanes (measured 6% faster at 20000 rows, 7% at 5000; with 4 words per
// lane the same rule was slower).
template <int K, int U, int V, bool TAIL = false>
static void launch_aligned(const IndexRun &R, const EvalArgs &e, bool ties, hipStream_t stream) {
    const int64_t Wg = (R.W + V - 1) / V;
    int64_t cpw = kBlock / Wg;
    if (V <= 2) {
        int64_t best = INT64_MAX;
        for (int64_t c = 1; c <= kBlock && c * Wg <= kAlignedThreads; ++c) {
            const int64_t th = (c * Wg + kWave - 1) / kWave * kWave;
            const int64_t idle = (th - c * Wg) * 4096 / th;   // idle share, 1/4096 units
            if (idle < best) {
                best = idle;
                cpw = c;
            }
        }
    }
    const int64_t threads = (cpw * Wg + kWave - 1) / kWave * kWave;
    const dim3 grid((unsigned)((R.P + cpw - 1) / cpw));
    launch_index_t<K, U, V, true, TAIL>(R, (uint32_t)cpw, grid, dim3((unsigned)threads), e,
                                        ties, stream);
}

// Tiling by matrix height.  Up to 1024 words (65536 rows) a workgroup holds
// whole candidates: 1 word per lane up to 128 words, 2 up to 320 (measured
// faster than 1 from 128 words on: half the lanes, twice the loads in
// flight), 4 with 2 pairs per batch of loads up to 1024 (measured 7-13%
// faster than 2 words from 391 to 1016 words, equal at 344); as many
// candidates per workgroup as fit, and a workgroup just large enough (whole
// waves) to hold them.  Taller matrices use the flattened tiling with 2
// words per lane.  With 2 words per lane up to 256 words, the last batch of
// each series is cut to its remaining pairs (no loads past the series end:
// 8.25 -> 7.53 us at 10000 rows, 9.33 -> 8.51 at 15000); above 256 words the
// extra registers of that form cost resident waves and it is slower (10.8
// -> 14.1 us at 20000 rows).
constexpr int64_t kTwoWordsMax = 320;
constexpr int64_t kTailMax = 256;

template <int K, int U>
static void launch_index_k(const IndexRun &R, const EvalArgs &e, bool ties, hipStream_t stream) {
    if (R.W <= kBlock / 2)
        launch_aligned<K, U, 1>(R, e, ties, stream);
    else if (R.W <= kTailMax)
        launch_aligned<K, U, 2, true>(R, e, ties, stream);
    else if (R.W <= kTwoWordsMax)
        launch_aligned<K, U, 2>(R, e, ties, stream);
    else if (R.W <= 4 * kBlock)
        launch_aligned<K, 2, 4>(R, e, ties, stream);
    else {
        constexpr int V = kWordsPerLane;
        const int64_t total = (int64_t)R.P * ((R.W + V - 1) / V);
        const dim3 grid((unsigned)((total + kBlock - 1) / kBlock));
        launch_index_t<K, U, V, false>(R, 0, grid, dim3(kBlock), e, ties, stream);
    }
}

hipError_t launch_eval_index(const uint64_t *idx, const uint32_t *tbits, bool ties, int64_t n,
                             int32_t m, int64_t W, int64_t wpad, const EvalArgs &e,
                             hipStream_t stream) {
    const IndexRun R{idx, nullptr, e.logt, n, W, wpad, m, e.P, 0, 0, 0, 0, tbits};
    switch (e.k) {
    case 0: launch_index_k<0, kUnroll>(R, e, ties, stream); break;
    case 1: launch_index_k<1, kUnroll>(R, e, ties, stream); break;
    case 2: launch_index_k<2, kUnroll>(R, e, ties, stream); break;
    case 3: launch_index_k<3, kUnroll>(R, e, ties, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


}  // namespace ebic
