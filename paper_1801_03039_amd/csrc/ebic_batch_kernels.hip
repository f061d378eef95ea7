// Batched EBIC evaluation for gfx950: one launch evaluates one population
// per run for many runs (matrices of different shapes), each tile with the
// index evaluator's tile code (strict, negative and approximate trend
// tests, row counts, Eq. (1) fitness, optional row masks).
#include "ebic_device.h"

namespace ebic {
namespace {

// --------------------------------------------------- batched (many runs) --
//
// One launch evaluates one population per run for many runs with matrices
// of different shapes.  The work is a list of tiles, run after run: a tile
// is kBlock lanes of one run holding V words each, either whole candidates
// (the run's cpw > 0) or consecutive (candidate, word-group) items.  With
// `work`, persistent workgroups take the next tile with an atomic until the
// list is exhausted, and the last workgroup to leave resets the queue, so
// the launch can be replayed (a captured graph) without any clearing step;
// work[0] is the next tile, work[1] the number of workgroups that have
// left.  Without it, workgroup b takes tile b (surplus workgroups return).
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
    __shared__ TileLds lds;
    // A run's tiles hold whole candidates (cpw > 0) or flattened items.
    auto tile = [&](const IndexRun &R, uint32_t local) {
        if (R.cpw > 0)
            index_tile<K, NEG, U, V, true>(R, local, (uint32_t)R.cpw, offsets, cols, n_entries,
                                           sigma, masks, acc, counts, fitness, lds);
        else
            index_tile<K, NEG, U, V, false>(R, local, 0, offsets, cols, n_entries, sigma, masks,
                                            acc, counts, fitness, lds);
    };
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
        if (tid < (int)(sizeof(IndexRun) / 8))
            reinterpret_cast<uint64_t *>(&s_R)[tid] =
                reinterpret_cast<const uint64_t *>(runs + lo)[tid];
        __syncthreads();
        tile(s_R, local);
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
        tile(s_R, s_local);
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

// Shapes with unroll x words_per_lane above 16 hold more order words in
// flight per lane than the register file allows at useful occupancy; they
// are not built.
template <int U, int V>
static hipError_t launch_batch_uv_if(const BatchLaunch &b, hipStream_t stream) {
    if constexpr (U * V <= kMaxUnrollWords)
        return launch_batch_uv<U, V>(b, stream);
    else
        return hipErrorInvalidValue;
}

template <int V>
static hipError_t launch_batch_v(const BatchLaunch &b, hipStream_t stream) {
    switch (b.unroll) {
    case 1: return launch_batch_uv_if<1, V>(b, stream);
    case 2: return launch_batch_uv_if<2, V>(b, stream);
    case 4: return launch_batch_uv_if<4, V>(b, stream);
    case 8: return launch_batch_uv_if<8, V>(b, stream);
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
    case 4: return launch_batch_v<4>(b, stream);
    case 8: return launch_batch_v<8>(b, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ebic
