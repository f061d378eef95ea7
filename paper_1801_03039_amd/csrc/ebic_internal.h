// Internal declarations shared by the libebic runtime, kernels and evolution
// engine.  Not part of the public ABI (see include/ebic.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/ebic.h"

namespace ebic {

// Largest approximate tolerance the pairwise-index evaluator handles; it
// keeps k+1 saturating bit-sliced violation counters per direction.
constexpr int kIndexMaxViolations = 3;

// Candidate columns staged in LDS by the direct evaluator; longer series
// read their tail from global memory.
constexpr int kDirectLdsCols = 512;

struct DeviceBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// Launchers (ebic_kernels.hip).  All are asynchronous on `stream` and return
// the HIP status of the launch.
hipError_t launch_ingest(const float *src, int64_t n, int32_t m, int64_t ld, int32_t layout,
                         int64_t npad, float *dst, hipStream_t stream);

// Tie-pair filter of the falling test: a bitmap of kTieBits bits in which
// ordered pair id p*m + q (p != q) sets bit tie_hash(p*m + q) when columns
// p and q have a tied or unordered row.  Every tied pair sets its bit, so a
// clear bit proves lt(q,p) = ~lt(p,q) on the valid rows; a set bit of an
// untied pair (a hash collision) only costs a read of the true reverse word.
constexpr int kTieBitsLog2 = 13;
constexpr int kTieWords = (1 << kTieBitsLog2) / 32;   // 1 KiB
__host__ __device__ inline uint32_t tie_hash(uint32_t pq) {
    return (pq * 0x9E3779B1u) >> (32 - kTieBitsLog2);   // Fibonacci hashing
}

// Builds the pairwise order index, its per-pair tie flags (m*m bytes), the
// tie-pair bitmap (kTieWords words) and any_tie[0] = whether two distinct
// columns tie on some row.
hipError_t launch_index_build(const float *a, int64_t n, int64_t npad, int32_t m, int64_t W,
                              int64_t wpad, uint64_t *idx, uint8_t *tie, int32_t *any_tie,
                              uint32_t *tbits, hipStream_t stream);

// The same index built from per-row ranks (ebic_index.hip) for matrices of
// at most kRankMaxCols columns.  It needs a device scratch of
// index_ranked_scratch_bytes(n, m, W) bytes (0: the matrix is too wide),
// which the caller keeps alive until the launches have completed.
constexpr int32_t kRankMaxCols = 2048;
size_t index_ranked_scratch_bytes(int64_t n, int32_t m, int64_t W);
// Resolves the ranked build's kernels for m columns (their code is loaded on
// first use), so that a timed build measures the launches alone.
hipError_t index_ranked_prepare(int32_t m);
hipError_t launch_index_build_ranked(const float *a, int64_t n, int64_t npad, int32_t m,
                                     int64_t W, int64_t wpad, uint64_t *idx, uint8_t *tie,
                                     int32_t *any_tie, uint32_t *tbits, void *scratch,
                                     hipStream_t stream);

struct EvalArgs {
    const int32_t *offsets;
    const int32_t *cols;
    int32_t P;
    int64_t n_entries;
    int32_t sigma;
    int32_t k;
    int32_t negative;
    uint64_t *masks;      // nullptr: no masks
    int32_t *counts;
    double *fitness;
    const double *logt;          // ln(i), i = 0..n
    unsigned long long *acc;     // P zero-initialised packed accumulators; left zeroed
};

// One run's share of an index evaluation (device-visible POD).
struct IndexRun {
    const uint64_t *idx;     // pairwise order index of the run's matrix
    const uint8_t *tie;      // its tie flags
    const double *logt;      // ln table of the run's matrix
    int64_t n, W, wpad;      // rows, mask words, padded words
    int32_t m;               // columns
    int32_t P;               // candidates of the run in this launch
    int64_t cand_base;       // index of the run's first candidate in the launch
    int64_t mask_base;       // first mask word of the run (when masks are written)
    int32_t cpw;             // batched tiles: whole candidates per tile (0: flattened tiles)
    int32_t reserved;
    const uint32_t *tbits;   // tie-pair bitmap (single-run launches; batched runs read `tie`)
};

// Batched launch shapes: unroll x words per lane is at most this.
constexpr int kMaxUnrollWords = 16;

// A persistent multi-run launch.  runs/tile_base/work are device arrays;
// tile_base[r] is the first tile of run r (tile_base[n_runs] = total);
// work[2] is a zeroed queue state that the kernel leaves zeroed.
struct BatchLaunch {
    const IndexRun *runs;
    const uint32_t *tile_base;
    int32_t n_runs;
    unsigned int *work;
    const int32_t *offsets;
    const int32_t *cols;
    int64_t n_entries;
    int32_t sigma, k, negative;
    uint64_t *masks;
    unsigned long long *acc;
    int32_t *counts;
    double *fitness;
    uint32_t grid;     // persistent workgroups, or the tile count when work is null
    int32_t unroll;    // pairs per batch of loads: 2, 4 or 8
    int32_t words;     // 64-row words per lane: 1 or 2 (a tile is 256 lanes)
};
// work == nullptr selects one tile per workgroup (no queue, grid = tiles).

hipError_t launch_eval_index_batch(const BatchLaunch &b, hipStream_t stream);
// Workgroups of the batch kernel resident per compute unit.
int batch_wgs_per_cu();

// Device-side evolution steps of batched runs (ebic_steps.hip): one
// workgroup (one wave) per run carries Steps 1-3 and 5 of the run.
//
// Per-run state between launches, in device memory.
struct StepsState {
    uint64_t rng;        // SplitMix64 state
    int32_t gen;         // generation of the population in the run's CBF slots
    int32_t n_top;       // entries of the top-rank list
    int32_t first_new;   // elites at the head of the population
    int32_t stopped;     // the tabu rule ended the run
    int32_t gens_run;    // generations completed after Step 1
    int32_t error;       // 1: the tabu table or its arena is full (the run stops)
    int64_t arena_used;  // columns stored in the tabu arena
};

// One run's buffers (device pointers).
struct StepsRun {
    int32_t *off;          // P + 1 offsets: global indices into the batch's column array
    int32_t *cols;         // the run's P * slot column slots (cols[0] is global index col_base)
    int64_t col_base;
    const int32_t *counts; // evaluation outputs of the run's P members
    const double *fit;
    int32_t *top_cols;     // K * slot columns of the top-rank list
    int32_t *top_len;      // K
    int32_t *top_cnt;      // K
    double *top_fit;       // K
    uint32_t *tabu;        // tabu_cap slots of 4 dwords {tag lo, tag hi, arena offset, length}
    uint64_t tabu_cap;     // power of two
    uint16_t *arena;       // columns of the listed series
    int64_t arena_cap;
    StepsState *state;
    int32_t m;             // matrix columns
    int32_t pad;
};

struct StepsArgs {
    const StepsRun *runs;
    const double *powtab;  // penalty_base^(s/L) at P*L*(L-1)/2 + (L-1) + s, s <= L*P
    int32_t n_runs, mode;  // mode 0: Step 1; 1: Step 5 then Steps 2-3; 2: Step 5
    int32_t P, len_min, len_max, slot;   // slot >= len_max: column slots per series
    int32_t tournament, wsum, elite_num, elite_den, K, tabu_limit;
    int32_t op_weight[5];
    int32_t lds_bytes;
    double theta;
};

// Dynamic LDS bytes a steps launch needs for P members, `slot` column slots,
// m columns and a top-rank list of K.
int64_t steps_lds_bytes(int32_t P, int32_t slot, int32_t m, int32_t K);
hipError_t launch_steps(const StepsArgs &a, hipStream_t stream);

// Device-pointer evaluation (ebic_runtime.cpp).  acc == nullptr: the
// context's own accumulators, grown on demand, and the order index built on
// first need.  Otherwise acc holds >= P zeroed accumulators and nothing is
// allocated; the index is used only if it is already built.
ebic_status evaluate_device_impl(ebic_ctx *ctx, const int32_t *d_offsets, const int32_t *d_cols,
                                 int32_t P, int64_t n_entries, const ebic_params *params,
                                 uint64_t *d_masks, int32_t *d_counts, double *d_fitness,
                                 void *hip_stream, unsigned long long *acc);
// Records msg as the context's (or, for ctx == nullptr, the thread's) error.
ebic_status fail_status(ebic_ctx *ctx, ebic_status st, const char *msg);
// Looks up the current device's no-allocation scratch array once
// (ebic_noalloc.hip); called with `device` current.
hipError_t noalloc_setup(int device);

// Runtime helpers shared with the multi-run driver (ebic_runtime.cpp).
void set_thread_error(const char *msg);
ebic_status ensure_index(ebic_ctx *ctx);  // builds the order index if missing
bool valid_cbf(ebic_ctx *ctx, const int32_t *offsets, const int32_t *cols, int32_t P,
               ebic_status *st);          // host CBF checks of ebic_evaluate
// The same checks, copying the columns to dst_cols (column i of the CBF to
// dst_cols[i]) and dst_off[c] = col_base + offsets[c] for c < P in one pass.
bool pack_valid_cbf(ebic_ctx *ctx, const int32_t *offsets, const int32_t *cols, int32_t P,
                    int32_t col_base, int32_t *dst_off, int32_t *dst_cols, ebic_status *st);

hipError_t launch_eval_direct(const float *a, int64_t n, int64_t npad, int32_t m, int64_t W,
                              const EvalArgs &e, hipStream_t stream);

// `ties`: two distinct columns of the matrix have a tied or unordered row;
// when false the falling test never reads the tie-pair bitmap or reverse
// words.
hipError_t launch_eval_index(const uint64_t *idx, const uint32_t *tbits, bool ties, int64_t n,
                             int32_t m, int64_t W, int64_t wpad, const EvalArgs &e,
                             hipStream_t stream);

}  // namespace ebic

struct ebic_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n = 0, npad = 0, W = 0, wpad = 0;
    int32_t m = 0;
    float *d_a = nullptr;        // column-major [m][npad]
    double *d_log = nullptr;     // ln(i), i = 0..n
    // pairwise order index
    uint64_t *d_idx = nullptr;
    // m*m tie flags of the index, an int32 any-tie flag, then the tie-pair
    // bitmap (tie_bits_offset)
    uint8_t *d_tie = nullptr;
    bool any_tie = true;         // two distinct columns tie (known once the index is built)
    int64_t idx_bytes = 0;
    int64_t idx_budget = 0;
    bool idx_built = false;
    double idx_ms = 0.0;
    int32_t path = EBIC_PATH_AUTO;
    // per-call scratch
    unsigned long long *d_acc = nullptr;
    int64_t cap_P = 0;
    // staging for the host-pointer entry point: offsets then columns, and
    // fitness then counts, on the device and in pinned host memory
    int32_t *d_cbf = nullptr, *h_cbf = nullptr;
    double *d_res = nullptr, *h_res = nullptr;
    uint64_t *d_masks = nullptr;
    int64_t cap_cbf = 0, cap_res = 0, hcap_cbf = 0, hcap_res = 0, cap_masks = 0;
    std::string err;
};
