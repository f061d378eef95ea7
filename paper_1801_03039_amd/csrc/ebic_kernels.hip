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

template <int K, bool NEG, int U, int V, bool ALIGNED, bool TIES, bool OFF32, bool TAIL>
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
template <int K, int U, int V, bool ALIGNED, bool OFF32, bool TAIL>
static void launch_index_o(const IndexRun &R, uint32_t cpw, dim3 grid, dim3 block,
                           const EvalArgs &e, bool ties, hipStream_t stream) {
    if (e.negative && ties)
        hipLaunchKernelGGL((eval_index_kernel<K, true, U, V, ALIGNED, true, OFF32, TAIL>), grid, block,
                           0, stream, R, cpw, e.offsets, e.cols, e.n_entries, e.sigma, e.masks,
                           e.acc, e.counts, e.fitness);
    else if (e.negative)
        hipLaunchKernelGGL((eval_index_kernel<K, true, U, V, ALIGNED, false, OFF32, TAIL>), grid, block,
                           0, stream, R, cpw, e.offsets, e.cols, e.n_entries, e.sigma, e.masks,
                           e.acc, e.counts, e.fitness);
    else
        hipLaunchKernelGGL((eval_index_kernel<K, false, U, V, ALIGNED, false, OFF32, TAIL>), grid, block,
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


}  // namespace ebic
