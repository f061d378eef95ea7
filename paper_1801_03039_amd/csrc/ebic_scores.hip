// Step 6 output and the accuracy scores of Section 3 on the device:
//   * row-index lists from 64-row masks (prefix sums of popcounts, then a
//     scatter in increasing row order);
//   * the cell Jaccard index of every (found, expected) bicluster pair and
//     the recovery / relevance scores of Eqs. (2)-(3).
// Integer work throughout; the only floating point is one FP64 division per
// Jaccard index, the max over a row or column of the index matrix and two
// sums taken in index order, so results are bit-exact and deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "ebic_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ inline uint64_t tail_word(uint64_t v, int64_t w, int64_t W, uint64_t tail) {
    return w == W - 1 ? v & tail : v;
}

// Union of a bicluster's mask planes for word w.
__device__ inline uint64_t plane_or(const uint64_t *m, int32_t planes, int64_t W, int64_t w) {
    uint64_t v = 0;
    for (int32_t p = 0; p < planes; ++p) v |= m[(int64_t)p * W + w];
    return v;
}

template <typename T>
__device__ inline T wave_sum(T v) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Exclusive prefix sum of v over the 256 threads of the block; *total gets
// the block's sum.  s_wave holds kWaves partial sums.
template <typename T>
__device__ inline T block_exclusive_scan(T v, T *s_wave, T *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wave[wid] = x;
    __syncthreads();
    T base = 0, tot = 0;
    for (int i = 0; i < kWaves; ++i) {
        const T t = s_wave[i];
        if (i < wid) base += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// offsets[k + 1] = number of rows in bicluster k.  One block per bicluster.
__global__ __launch_bounds__(kBlock) void mask_count_kernel(const uint64_t *masks, int32_t planes,
                                                            int64_t W, uint64_t tail,
                                                            int64_t *offsets) {
    const int64_t k = blockIdx.x;
    const uint64_t *m = masks + k * planes * W;
    int64_t c = 0;
    for (int64_t w = threadIdx.x; w < W; w += kBlock)
        c += __popcll(tail_word(plane_or(m, planes, W, w), w, W, tail));
    c = wave_sum(c);
    __shared__ int64_t s[kWaves];
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int i = 0; i < kWaves; ++i) t += s[i];
        offsets[k + 1] = t;
    }
}

// In-place inclusive scan of offsets[1..K]; offsets[0] = 0.  One block.
__global__ __launch_bounds__(kBlock) void offsets_scan_kernel(int64_t *offsets, int32_t K) {
    __shared__ int64_t s_wave[kWaves];
    int64_t carry = 0;
    for (int32_t base = 0; base < K; base += kBlock) {
        const int32_t i = base + (int32_t)threadIdx.x;
        const int64_t v = i < K ? offsets[i + 1] : 0;
        int64_t total;
        const int64_t ex = block_exclusive_scan(v, s_wave, &total);
        if (i < K) offsets[i + 1] = carry + ex + v;
        carry += total;
    }
    if (threadIdx.x == 0) offsets[0] = 0;
}

// Row indices of bicluster k at rows[offsets[k] ...], increasing; entries at
// or beyond `capacity` are not written.  One block per bicluster.
__global__ __launch_bounds__(kBlock) void mask_scatter_kernel(const uint64_t *masks, int32_t planes,
                                                              int64_t W, uint64_t tail,
                                                              const int64_t *offsets, int32_t *rows,
                                                              int64_t capacity) {
    const int64_t k = blockIdx.x;
    const uint64_t *m = masks + k * planes * W;
    __shared__ int64_t s_wave[kWaves];
    int64_t pos0 = offsets[k];
    for (int64_t base = 0; base < W; base += kBlock) {
        const int64_t w = base + threadIdx.x;
        uint64_t v = w < W ? tail_word(plane_or(m, planes, W, w), w, W, tail) : 0;
        int64_t total;
        int64_t pos = pos0 + block_exclusive_scan((int64_t)__popcll(v), s_wave, &total);
        while (v) {
            const int b = __builtin_ctzll(v);
            if (pos < capacity) rows[pos] = (int32_t)(w * 64 + b);
            ++pos;
            v &= v - 1;
        }
        pos0 += total;
    }
}

struct SetView {
    const uint64_t *masks;
    int32_t planes;
    const int32_t *off;
    const int32_t *cols;
};

// Number of distinct columns of list a[0..la) and how many of them occur in
// b[0..lb), summed over the wave.
__device__ inline void column_counts(const int32_t *a, int32_t la, const int32_t *b, int32_t lb,
                                     int64_t *distinct, int64_t *shared) {
    const int lane = threadIdx.x & 63;
    int64_t d = 0, s = 0;
    for (int32_t i = lane; i < la; i += 64) {
        const int32_t c = a[i];
        bool first = true;
        for (int32_t j = 0; j < i; ++j) first = first && a[j] != c;
        if (!first) continue;
        ++d;
        bool in = false;
        for (int32_t j = 0; j < lb; ++j) in = in || b[j] == c;
        s += in ? 1 : 0;
    }
    *distinct = wave_sum(d);
    *shared = wave_sum(s);
}

// J[f * E + e] for every pair; one wave per pair.
__global__ __launch_bounds__(kBlock) void jaccard_kernel(SetView fs, int32_t F, SetView es,
                                                         int32_t E, int64_t W, uint64_t tail,
                                                         double *J) {
    const int64_t pair = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (pair >= (int64_t)F * E) return;     // whole waves leave; no block barrier follows
    const int32_t f = (int32_t)(pair / E), e = (int32_t)(pair % E);
    const uint64_t *a = fs.masks + (int64_t)f * fs.planes * W;
    const uint64_t *b = es.masks + (int64_t)e * es.planes * W;
    const int lane = threadIdx.x & 63;
    int64_t na = 0, nb = 0, ni = 0;
    for (int64_t w = lane; w < W; w += 64) {
        const uint64_t x = tail_word(plane_or(a, fs.planes, W, w), w, W, tail);
        const uint64_t y = tail_word(plane_or(b, es.planes, W, w), w, W, tail);
        na += __popcll(x);
        nb += __popcll(y);
        ni += __popcll(x & y);
    }
    na = wave_sum(na);
    nb = wave_sum(nb);
    ni = wave_sum(ni);
    const int32_t *ca = fs.cols + fs.off[f], *cb = es.cols + es.off[e];
    const int32_t la = fs.off[f + 1] - fs.off[f], lb = es.off[e + 1] - es.off[e];
    int64_t da, sa, db, sb;
    column_counts(ca, la, cb, lb, &da, &sa);
    column_counts(cb, lb, ca, la, &db, &sb);   // sb == sa: shared columns counted from B's side
    if (lane == 0) {
        const int64_t inter = ni * (sa < sb ? sa : sb);
        const int64_t uni = na * da + nb * db - inter;
        J[pair] = uni > 0 ? (double)inter / (double)uni : 0.0;
    }
}

// scores[0] = recovery, scores[1] = relevance.  One block: the maxima of a
// chunk of columns (rows) of J are formed in parallel, then added in index
// order by one thread.
__global__ __launch_bounds__(kBlock) void scores_kernel(const double *J, int32_t F, int32_t E,
                                                        double *scores) {
    __shared__ double s_max[kBlock];
    double sums[2] = {0.0, 0.0};
    for (int which = 0; which < 2; ++which) {
        const int32_t outer = which == 0 ? E : F, inner = which == 0 ? F : E;
        for (int32_t base = 0; base < outer; base += kBlock) {
            const int32_t i = base + (int32_t)threadIdx.x;
            if (i < outer) {
                double mx = 0.0;
                for (int32_t j = 0; j < inner; ++j) {
                    const double v = which == 0 ? J[(int64_t)j * E + i] : J[(int64_t)i * E + j];
                    mx = v > mx ? v : mx;
                }
                s_max[threadIdx.x] = mx;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                const int32_t n = outer - base < kBlock ? outer - base : kBlock;
                for (int32_t t = 0; t < n; ++t) sums[which] += s_max[t];
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        const bool none = F == 0 || E == 0;
        scores[0] = none ? 0.0 : sums[0] / (double)E;
        scores[1] = none ? 0.0 : sums[1] / (double)F;
    }
}

ebic_status arg_error(const std::string &msg) {
    ebic::set_thread_error(msg.c_str());
    return EBIC_E_ARG;
}

ebic_status hip_error(hipError_t e, const char *what) {
    ebic::set_thread_error((std::string(what) + ": " + hipGetErrorString(e)).c_str());
    return EBIC_E_DEVICE;
}

uint64_t tail_mask(int64_t n_rows) {
    const int r = (int)(n_rows % 64);
    return r == 0 ? ~0ull : ((1ull << r) - 1);
}

bool set_ok(const ebic_bicluster_set *s, const char *name, std::string *msg) {
    if (!s || s->struct_size < sizeof(ebic_bicluster_set)) {
        *msg = std::string(name) + ": null or struct_size too small";
        return false;
    }
    if (s->count < 0 || (s->count > 0 && (s->planes < 1 || !s->row_masks || !s->col_offsets ||
                                          !s->cols))) {
        *msg = std::string(name) + ": count < 0, planes < 1 or a null device pointer";
        return false;
    }
    return true;
}

}  // namespace

extern "C" {

ebic_status ebic_mask_rows(const uint64_t *d_masks, int32_t K, int32_t planes, int64_t n_rows,
                           int64_t *d_offsets, int32_t *d_rows, int64_t rows_capacity,
                           void *hip_stream) {
    if (K < 0 || n_rows < 0 || rows_capacity < 0) return arg_error("K, n_rows, capacity >= 0");
    if (n_rows > INT32_MAX) return arg_error("n_rows must fit int32 row indices");
    if (!d_offsets) return arg_error("d_offsets is null");
    if (K > 0 && planes < 1) return arg_error("planes must be >= 1");
    if (K > 0 && n_rows > 0 && !d_masks) return arg_error("d_masks is null");
    if (rows_capacity > 0 && !d_rows) return arg_error("d_rows is null");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t W = n_rows == 0 ? 0 : (n_rows + 63) / 64;
    hipError_t e;
    if (K > 0) {
        // With no rows (W = 0) every count is 0 and the masks are not read.
        hipLaunchKernelGGL(mask_count_kernel, dim3((unsigned)K), dim3(kBlock), 0, s, d_masks,
                           planes, W, tail_mask(n_rows), d_offsets);
        if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "mask_count_kernel");
    }
    hipLaunchKernelGGL(offsets_scan_kernel, dim3(1), dim3(kBlock), 0, s, d_offsets, K);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "offsets_scan_kernel");
    if (K > 0 && W > 0) {
        hipLaunchKernelGGL(mask_scatter_kernel, dim3((unsigned)K), dim3(kBlock), 0, s, d_masks,
                           planes, W, tail_mask(n_rows), d_offsets, d_rows, rows_capacity);
        if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "mask_scatter_kernel");
    }
    return EBIC_OK;
}

ebic_status ebic_match_scores(const ebic_bicluster_set *found, const ebic_bicluster_set *expected,
                              int64_t n_rows, double *d_jaccard, double *d_scores,
                              void *hip_stream) {
    std::string msg;
    if (!set_ok(found, "found", &msg) || !set_ok(expected, "expected", &msg))
        return arg_error(msg);
    if (n_rows < 0) return arg_error("n_rows must be >= 0");
    if (!d_scores) return arg_error("d_scores is null");
    const int64_t F = found->count, E = expected->count;
    if (F * E > 0 && !d_jaccard) return arg_error("d_jaccard is null");
    if (F * E > (int64_t)INT32_MAX * kWaves) return arg_error("too many bicluster pairs");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t W = (n_rows + 63) / 64;
    hipError_t e;
    if (F * E > 0) {
        SetView fs{found->row_masks, found->planes, found->col_offsets, found->cols};
        SetView es{expected->row_masks, expected->planes, expected->col_offsets, expected->cols};
        const int64_t blocks = (F * E + kWaves - 1) / kWaves;
        hipLaunchKernelGGL(jaccard_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, fs,
                           (int32_t)F, es, (int32_t)E, W, tail_mask(n_rows), d_jaccard);
        if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "jaccard_kernel");
    }
    hipLaunchKernelGGL(scores_kernel, dim3(1), dim3(kBlock), 0, s, d_jaccard, (int32_t)F,
                       (int32_t)E, d_scores);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "scores_kernel");
    return EBIC_OK;
}

}  // extern "C"
