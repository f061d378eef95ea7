// libebic runtime: contexts, matrix ingest, the pairwise order index, and
// the evaluation entry points of include/ebic.h.
//
// Every step of an evaluation runs in the kernels of ebic_kernels.hip; this
// file validates arguments, owns device memory and orders launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ebic_internal.h"

using namespace ebic;

namespace {

thread_local std::string g_tls_error;

ebic_status fail(ebic_ctx *ctx, ebic_status st, const std::string &msg) {
    if (ctx)
        ctx->err = msg;
    else
        g_tls_error = msg;
    return st;
}

ebic_status hip_fail(ebic_ctx *ctx, hipError_t e, const char *what) {
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? EBIC_E_NOMEM : EBIC_E_DEVICE, msg);
}

#define HIP_TRY(ctx, expr)                                  \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
    } while (0)

constexpr int64_t kDefaultIndexBudget = int64_t(8) << 30;
constexpr int64_t kMaxLaunchThreads = (int64_t(1) << 32) - 256;

int64_t words_of(int64_t n) { return (n + 63) / 64; }

template <typename T>
ebic_status grow(ebic_ctx *ctx, T *&ptr, int64_t &cap, int64_t need, bool zero) {
    if (need <= cap) return EBIC_OK;
    int64_t ncap = std::max<int64_t>(need, cap * 2);
    if (ptr) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, hipDeviceSynchronize());
        HIP_TRY(ctx, hipFree(ptr));
        ptr = nullptr;
        cap = 0;
    }
    void *p = nullptr;
    HIP_TRY(ctx, hipMalloc(&p, sizeof(T) * (size_t)ncap));
    if (zero) {
        hipError_t e = hipMemset(p, 0, sizeof(T) * (size_t)ncap);
        if (e != hipSuccess) {
            (void)hipFree(p);
            return hip_fail(ctx, e, "hipMemset");
        }
    }
    ptr = static_cast<T *>(p);
    cap = ncap;
    return EBIC_OK;
}

// Pinned host staging (grown on demand; the caller has synchronised the
// stream, so no copy is reading the old buffer).
template <typename T>
ebic_status grow_pinned(ebic_ctx *ctx, T *&ptr, int64_t &cap, int64_t need) {
    if (need <= cap) return EBIC_OK;
    const int64_t ncap = std::max<int64_t>(need, cap * 2);
    if (ptr) {
        HIP_TRY(ctx, hipHostFree(ptr));
        ptr = nullptr;
        cap = 0;
    }
    void *p = nullptr;
    HIP_TRY(ctx, hipHostMalloc(&p, sizeof(T) * (size_t)ncap, hipHostMallocDefault));
    ptr = static_cast<T *>(p);
    cap = ncap;
    return EBIC_OK;
}

ebic_status ensure_scratch(ebic_ctx *ctx, int64_t P) {
    return grow(ctx, ctx->d_acc, ctx->cap_P, P, true);
}

// The any-tie flag follows the m*m tie flags, 8-byte aligned; the tie-pair
// bitmap follows it, 16-byte aligned.
size_t tie_flag_offset(int32_t m) { return ((size_t)m * (size_t)m + 7) / 8 * 8; }
size_t tie_bits_offset(int32_t m) { return tie_flag_offset(m) + 16; }

int64_t index_bytes_for(int32_t m, int64_t wpad) {
    return (int64_t)m * (int64_t)m * (wpad * 8 + 1);  // order words + tie flags
}

struct BuildScratch {
    std::mutex mu;
    void *ptr = nullptr;
    size_t bytes = 0;
};

BuildScratch &build_scratch(int device) {
    constexpr int kDevices = 64;
    static BuildScratch per_device[kDevices];
    return per_device[device < 0 || device >= kDevices ? 0 : device];
}

ebic_status build_index(ebic_ctx *ctx) {
    if (ctx->idx_built) return EBIC_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (!ctx->d_idx) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, (size_t)ctx->m * (size_t)ctx->m * (size_t)ctx->wpad * 8);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, EBIC_E_NOMEM, "cannot allocate the pairwise order index (" +
                                               std::to_string(ctx->idx_bytes) + " bytes)");
        }
        ctx->d_idx = static_cast<uint64_t *>(p);
        e = hipMalloc(&p, tie_bits_offset(ctx->m) + kTieWords * sizeof(uint32_t));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(ctx->d_idx);
            ctx->d_idx = nullptr;
            return fail(ctx, EBIC_E_NOMEM, "cannot allocate the index tie flags");
        }
        ctx->d_tie = static_cast<uint8_t *>(p);
    }
    // The rank-based build needs a scratch (ranks and bit-planes), shared by
    // every build on the device and held until the process ends; a build
    // holds it until its launches have completed.  Without it (a matrix
    // wider than the ranked build takes, or no memory) the direct build runs.
    BuildScratch &bs = build_scratch(ctx->device);
    std::lock_guard<std::mutex> lock(bs.mu);
    const size_t need = index_ranked_scratch_bytes(ctx->n, ctx->m, ctx->W);
    if (need > bs.bytes) {
        if (bs.ptr) {
            (void)hipFree(bs.ptr);
            bs.ptr = nullptr;
            bs.bytes = 0;
        }
        void *p = nullptr;
        if (hipMalloc(&p, need) == hipSuccess) {
            bs.ptr = p;
            bs.bytes = need;
        } else {
            (void)hipGetLastError();
        }
    }
    const bool ranked = need > 0 && need <= bs.bytes;
    if (ranked) HIP_TRY(ctx, index_ranked_prepare(ctx->m));
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
    int32_t *d_any = reinterpret_cast<int32_t *>(ctx->d_tie + tie_flag_offset(ctx->m));
    uint32_t *d_bits = reinterpret_cast<uint32_t *>(ctx->d_tie + tie_bits_offset(ctx->m));
    if (ranked)
        HIP_TRY(ctx, launch_index_build_ranked(ctx->d_a, ctx->n, ctx->npad, ctx->m, ctx->W,
                                               ctx->wpad, ctx->d_idx, ctx->d_tie, d_any, d_bits,
                                               bs.ptr, ctx->stream));
    else
        HIP_TRY(ctx, launch_index_build(ctx->d_a, ctx->n, ctx->npad, ctx->m, ctx->W, ctx->wpad,
                                        ctx->d_idx, ctx->d_tie, d_any, d_bits, ctx->stream));
    HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
    HIP_TRY(ctx, hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // Whether two distinct columns have a tied or unordered row.
    int32_t any = 1;
    HIP_TRY(ctx, hipMemcpy(&any, d_any, sizeof(any), hipMemcpyDeviceToHost));
    ctx->any_tie = any != 0;
    ctx->idx_ms = ms;
    ctx->idx_built = true;
    return EBIC_OK;
}

bool params_ok(ebic_ctx *ctx, const ebic_params *p, ebic_status *st) {
    if (!p || p->struct_size < sizeof(ebic_params)) {
        *st = fail(ctx, EBIC_E_ARG, "params is null or struct_size too small");
        return false;
    }
    if (p->sigma < 0 || p->max_violations < 0) {
        *st = fail(ctx, EBIC_E_RANGE, "sigma and max_violations must be >= 0");
        return false;
    }
    return true;
}

// Decide the evaluator for this call; builds the index on first need.
ebic_status choose_path(ebic_ctx *ctx, const ebic_params *p, bool *use_index) {
    const bool k_ok = p->max_violations <= kIndexMaxViolations;
    *use_index = false;
    if (ctx->path == EBIC_PATH_DIRECT || !k_ok) return EBIC_OK;
    if (ctx->path == EBIC_PATH_AUTO && ctx->idx_bytes > ctx->idx_budget) return EBIC_OK;
    ebic_status st = build_index(ctx);
    if (st != EBIC_OK) {
        if (ctx->path == EBIC_PATH_INDEX) return st;
        return EBIC_OK;  // AUTO: fall back to the direct kernel on the GPU
    }
    *use_index = true;
    return EBIC_OK;
}

ebic_status launch_all(ebic_ctx *ctx, const EvalArgs &e, bool use_index, hipStream_t s) {
    const int64_t items = use_index ? (int64_t)e.P * ctx->W : (int64_t)e.P * 8 * 256;
    if (items > kMaxLaunchThreads)
        return fail(ctx, EBIC_E_ARG, "population too large for one launch; split it");
    if (use_index)
        HIP_TRY(ctx, launch_eval_index(
                         ctx->d_idx,
                         reinterpret_cast<const uint32_t *>(ctx->d_tie + tie_bits_offset(ctx->m)),
                         ctx->any_tie, ctx->n, ctx->m, ctx->W, ctx->wpad, e, s));
    else
        HIP_TRY(ctx, launch_eval_direct(ctx->d_a, ctx->n, ctx->npad, ctx->m, ctx->W, e, s));
    return EBIC_OK;
}

ebic_status create_common(const float *a, bool on_device, int64_t n_rows, int32_t n_cols,
                          int64_t ld, int32_t layout, int32_t device, ebic_ctx **out) {
    if (!out) return fail(nullptr, EBIC_E_ARG, "out is null");
    *out = nullptr;
    if (!a) return fail(nullptr, EBIC_E_ARG, "matrix pointer is null");
    if (n_rows < 1 || n_cols < 1) return fail(nullptr, EBIC_E_ARG, "n_rows and n_cols must be >= 1");
    if (layout != EBIC_ROW_MAJOR && layout != EBIC_COL_MAJOR)
        return fail(nullptr, EBIC_E_ARG, "layout must be EBIC_ROW_MAJOR or EBIC_COL_MAJOR");
    if ((layout == EBIC_ROW_MAJOR && ld < n_cols) || (layout == EBIC_COL_MAJOR && ld < n_rows))
        return fail(nullptr, EBIC_E_ARG, "leading dimension too small");
    if (n_rows > (int64_t(1) << 31) - 64)
        return fail(nullptr, EBIC_E_ARG, "n_rows must fit a 32-bit row count");

    ebic_ctx *ctx = new (std::nothrow) ebic_ctx();
    if (!ctx) return fail(nullptr, EBIC_E_NOMEM, "cannot allocate context");
    auto bail = [&](ebic_status st) {
        std::string msg = ctx->err;
        ebic_destroy(ctx);
        return fail(nullptr, st, msg);
    };
    ctx->device = device;
    ctx->n = n_rows;
    ctx->m = n_cols;
    ctx->W = words_of(n_rows);
    ctx->npad = ctx->W * 64;
    ctx->wpad = (ctx->W + 15) / 16 * 16;   // order rows start on 128-byte lines
    ctx->idx_bytes = index_bytes_for(n_cols, ctx->wpad);

    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipSetDevice"));
    e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipStreamCreate"));
    // Once per device: the address of its no-allocation scratch array.  A
    // failure is kept and reported by the entry point that needs it.
    (void)noalloc_setup(device);

    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    ctx->idx_budget = std::min<int64_t>(kDefaultIndexBudget, (int64_t)(free_b / 4));

    const size_t abytes = sizeof(float) * (size_t)ctx->npad * (size_t)n_cols;
    e = hipMalloc(&ctx->d_a, abytes);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipMalloc(matrix)"));

    const float *src = a;
    float *staging = nullptr;
    const size_t src_elems = layout == EBIC_ROW_MAJOR
                                 ? (size_t)(n_rows - 1) * (size_t)ld + (size_t)n_cols
                                 : (size_t)(n_cols - 1) * (size_t)ld + (size_t)n_rows;
    if (on_device) {
        // The caller's writes to d_a may be pending on any stream.
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipDeviceSynchronize"));
    } else {
        e = hipMalloc(&staging, sizeof(float) * src_elems);
        if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipMalloc(staging)"));
        e = hipMemcpy(staging, a, sizeof(float) * src_elems, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(staging);
            return bail(hip_fail(ctx, e, "hipMemcpy(matrix)"));
        }
        src = staging;
    }
    e = launch_ingest(src, n_rows, n_cols, ld, layout, ctx->npad, ctx->d_a, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (staging) (void)hipFree(staging);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "matrix ingest"));

    // ln(i) for i = 0..n with the C library's log (Eq. (1)).
    std::vector<double> logt((size_t)n_rows + 1);
    for (int64_t i = 0; i <= n_rows; ++i) logt[(size_t)i] = std::log((double)i);
    e = hipMalloc(&ctx->d_log, sizeof(double) * logt.size());
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipMalloc(log table)"));
    e = hipMemcpy(ctx->d_log, logt.data(), sizeof(double) * logt.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipMemcpy(log table)"));

    *out = ctx;
    return EBIC_OK;
}

// Host CBF checks: offsets[0] = 0, increasing offsets, columns in range and
// distinct within a series.  With dst_cols, the columns are also copied to
// dst_cols and dst_off[c] = col_base + offsets[c] for c < P, in the same pass.
bool check_cbf(ebic_ctx *ctx, const int32_t *offsets, const int32_t *cols, int32_t P,
               ebic_status *st, int32_t *dst_off = nullptr, int32_t *dst_cols = nullptr,
               int32_t col_base = 0) {
    if (offsets[0] != 0) {
        *st = fail(ctx, EBIC_E_ARG, "offsets[0] must be 0");
        return false;
    }
    std::vector<int32_t> seen((size_t)ctx->m, -1);
    for (int32_t c = 0; c < P; ++c) {
        if (offsets[c + 1] <= offsets[c]) {
            *st = fail(ctx, EBIC_E_ARG, "offsets must increase (every series has L >= 1); candidate " +
                                            std::to_string(c));
            return false;
        }
        if (dst_off) dst_off[c] = col_base + offsets[c];
        for (int32_t i = offsets[c]; i < offsets[c + 1]; ++i) {
            const int32_t col = cols[i];
            if (col < 0 || col >= ctx->m) {
                *st = fail(ctx, EBIC_E_RANGE, "column out of range in candidate " + std::to_string(c));
                return false;
            }
            if (seen[(size_t)col] == c) {
                *st = fail(ctx, EBIC_E_ARG, "duplicate column in candidate " + std::to_string(c));
                return false;
            }
            seen[(size_t)col] = c;
            if (dst_cols) dst_cols[i] = col;
        }
    }
    return true;
}

}  // namespace

namespace ebic {
// Shared body of the device-pointer entry points.  acc == nullptr: the
// context's accumulators (grown on demand) and the index built on first
// need.  Otherwise `acc` holds >= P zeroed accumulators and nothing is
// allocated: the index is used only if it is already built.
ebic_status evaluate_device_impl(ebic_ctx *ctx, const int32_t *d_offsets, const int32_t *d_cols,
                                 int32_t P, int64_t n_entries, const ebic_params *params,
                                 uint64_t *d_masks, int32_t *d_counts, double *d_fitness,
                                 void *hip_stream, unsigned long long *acc) {
    if (!ctx) return fail(nullptr, EBIC_E_ARG, "ctx is null");
    ebic_status st;
    if (!params_ok(ctx, params, &st)) return st;
    if (P < 0 || n_entries < 0) return fail(ctx, EBIC_E_ARG, "P and n_entries must be >= 0");
    if (P == 0) return EBIC_OK;
    if (!d_offsets || !d_counts || !d_fitness || (n_entries > 0 && !d_cols))
        return fail(ctx, EBIC_E_ARG, "null device pointer");
    if (params->want_masks && !d_masks) return fail(ctx, EBIC_E_ARG, "want_masks needs masks");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    bool use_index = false;
    if (!acc) {
        st = ensure_scratch(ctx, P);
        if (st != EBIC_OK) return st;
        acc = ctx->d_acc;
        st = choose_path(ctx, params, &use_index);
        if (st != EBIC_OK) return st;
    } else {
        use_index = ctx->idx_built && ctx->path != EBIC_PATH_DIRECT &&
                    params->max_violations <= kIndexMaxViolations &&
                    !(ctx->path == EBIC_PATH_AUTO && ctx->idx_bytes > ctx->idx_budget);
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    EvalArgs e{d_offsets, d_cols, P, n_entries, params->sigma, params->max_violations,
               params->negative_trends ? 1 : 0, params->want_masks ? d_masks : nullptr,
               d_counts, d_fitness, ctx->d_log, acc};
    return launch_all(ctx, e, use_index, s);
}

ebic_status fail_status(ebic_ctx *ctx, ebic_status st, const char *msg) {
    return fail(ctx, st, msg);
}

void set_thread_error(const char *msg) { g_tls_error = msg; }
ebic_status ensure_index(ebic_ctx *ctx) { return build_index(ctx); }
bool valid_cbf(ebic_ctx *ctx, const int32_t *offsets, const int32_t *cols, int32_t P,
               ebic_status *st) {
    return check_cbf(ctx, offsets, cols, P, st);
}
bool pack_valid_cbf(ebic_ctx *ctx, const int32_t *offsets, const int32_t *cols, int32_t P,
                    int32_t col_base, int32_t *dst_off, int32_t *dst_cols, ebic_status *st) {
    return check_cbf(ctx, offsets, cols, P, st, dst_off, dst_cols, col_base);
}
}  // namespace ebic

extern "C" {

int64_t ebic_mask_words(int64_t n_rows) { return n_rows <= 0 ? 0 : words_of(n_rows); }

ebic_status ebic_create(const float *a, int64_t n_rows, int32_t n_cols, int64_t ld,
                        int32_t layout, int32_t device, ebic_ctx **out) {
    return create_common(a, false, n_rows, n_cols, ld, layout, device, out);
}

ebic_status ebic_create_device(const float *d_a, int64_t n_rows, int32_t n_cols, int64_t ld,
                               int32_t layout, int32_t device, ebic_ctx **out) {
    return create_common(d_a, true, n_rows, n_cols, ld, layout, device, out);
}

ebic_status ebic_destroy(ebic_ctx *ctx) {
    if (!ctx) return EBIC_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    void *bufs[] = {ctx->d_a, ctx->d_log, ctx->d_idx, ctx->d_tie, ctx->d_acc,
                    ctx->d_cbf, ctx->d_res, ctx->d_masks};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (ctx->h_cbf) (void)hipHostFree(ctx->h_cbf);
    if (ctx->h_res) (void)hipHostFree(ctx->h_res);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return EBIC_OK;
}

ebic_status ebic_set_path(ebic_ctx *ctx, int32_t path) {
    if (!ctx) return fail(nullptr, EBIC_E_ARG, "ctx is null");
    if (path != EBIC_PATH_AUTO && path != EBIC_PATH_DIRECT && path != EBIC_PATH_INDEX)
        return fail(ctx, EBIC_E_ARG, "unknown path");
    ctx->path = path;
    if (path == EBIC_PATH_INDEX) return build_index(ctx);
    return EBIC_OK;
}

ebic_status ebic_set_index_budget(ebic_ctx *ctx, int64_t bytes) {
    if (!ctx) return fail(nullptr, EBIC_E_ARG, "ctx is null");
    if (bytes < 0) return fail(ctx, EBIC_E_ARG, "budget must be >= 0");
    ctx->idx_budget = bytes;
    return EBIC_OK;
}

ebic_status ebic_get_info(const ebic_ctx *ctx, ebic_ctx_info *info) {
    if (!ctx || !info || info->struct_size < sizeof(ebic_ctx_info))
        return fail(const_cast<ebic_ctx *>(ctx), EBIC_E_ARG, "null argument or struct_size too small");
    info->device = ctx->device;
    info->n_rows = ctx->n;
    info->n_cols = ctx->m;
    info->rows_padded = ctx->npad;
    info->mask_words = ctx->W;
    info->path = ctx->path;
    info->index_built = ctx->idx_built ? 1 : 0;
    info->index_bytes = ctx->idx_bytes;
    info->index_budget = ctx->idx_budget;
    info->index_build_ms = ctx->idx_ms;
    info->index_ties = ctx->any_tie ? 1 : 0;
    return EBIC_OK;
}

ebic_status ebic_evaluate_device(ebic_ctx *ctx, const int32_t *d_offsets, const int32_t *d_cols,
                                 int32_t P, int64_t n_entries, const ebic_params *params,
                                 uint64_t *d_masks, int32_t *d_counts, double *d_fitness,
                                 void *hip_stream) {
    return ebic::evaluate_device_impl(ctx, d_offsets, d_cols, P, n_entries, params, d_masks,
                                      d_counts, d_fitness, hip_stream, nullptr);
}

ebic_status ebic_evaluate(ebic_ctx *ctx, const int32_t *offsets, const int32_t *cols, int32_t P,
                          const ebic_params *params, uint64_t *masks, int32_t *counts,
                          double *fitness) {
    if (!ctx) return fail(nullptr, EBIC_E_ARG, "ctx is null");
    ebic_status st;
    if (!params_ok(ctx, params, &st)) return st;
    if (P < 0) return fail(ctx, EBIC_E_ARG, "P must be >= 0");
    if (P == 0) return EBIC_OK;
    if (!offsets || !cols || !counts || !fitness)
        return fail(ctx, EBIC_E_ARG, "null pointer");
    if (params->want_masks && !masks) return fail(ctx, EBIC_E_ARG, "want_masks needs masks");
    if (!check_cbf(ctx, offsets, cols, P, &st)) return st;
    const int64_t n_entries = offsets[P];
    // One upload (offsets then columns) and one download (fitness then
    // counts), both through pinned staging buffers.
    const int64_t n_cbf = (int64_t)P + 1 + n_entries;      // int32
    const int64_t n_res = (int64_t)P + ((int64_t)P + 1) / 2;  // doubles: P fitness + P int32
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if ((st = ensure_scratch(ctx, P)) != EBIC_OK) return st;
    if ((st = grow(ctx, ctx->d_cbf, ctx->cap_cbf, n_cbf, false)) != EBIC_OK) return st;
    if ((st = grow(ctx, ctx->d_res, ctx->cap_res, n_res, false)) != EBIC_OK) return st;
    if ((st = grow_pinned(ctx, ctx->h_cbf, ctx->hcap_cbf, n_cbf)) != EBIC_OK) return st;
    if ((st = grow_pinned(ctx, ctx->h_res, ctx->hcap_res, n_res)) != EBIC_OK) return st;
    const int64_t mask_words = params->want_masks ? (int64_t)P * 2 * ctx->W : 0;
    if (mask_words && (st = grow(ctx, ctx->d_masks, ctx->cap_masks, mask_words, false)) != EBIC_OK)
        return st;
    bool use_index = false;
    if ((st = choose_path(ctx, params, &use_index)) != EBIC_OK) return st;

    hipStream_t s = ctx->stream;
    std::memcpy(ctx->h_cbf, offsets, sizeof(int32_t) * ((size_t)P + 1));
    std::memcpy(ctx->h_cbf + P + 1, cols, sizeof(int32_t) * (size_t)n_entries);
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_cbf, ctx->h_cbf, sizeof(int32_t) * (size_t)n_cbf,
                                hipMemcpyHostToDevice, s));
    int32_t *d_counts = reinterpret_cast<int32_t *>(ctx->d_res + P);
    EvalArgs e{ctx->d_cbf, ctx->d_cbf + P + 1, P, n_entries, params->sigma,
               params->max_violations, params->negative_trends ? 1 : 0,
               mask_words ? ctx->d_masks : nullptr, d_counts, ctx->d_res, ctx->d_log,
               ctx->d_acc};
    if ((st = launch_all(ctx, e, use_index, s)) != EBIC_OK) return st;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_res, ctx->d_res,
                                sizeof(double) * (size_t)P + sizeof(int32_t) * (size_t)P,
                                hipMemcpyDeviceToHost, s));
    if (mask_words)
        HIP_TRY(ctx, hipMemcpyAsync(masks, ctx->d_masks, sizeof(uint64_t) * (size_t)mask_words,
                                    hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    std::memcpy(fitness, ctx->h_res, sizeof(double) * (size_t)P);
    std::memcpy(counts, ctx->h_res + P, sizeof(int32_t) * (size_t)P);
    return EBIC_OK;
}

ebic_status ebic_synchronize(ebic_ctx *ctx) {
    if (!ctx) return fail(nullptr, EBIC_E_ARG, "ctx is null");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return EBIC_OK;
}

const char *ebic_last_error(const ebic_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_tls_error.c_str();
}

}  // extern "C"
