/*
 * ebic.h -- C ABI of libebic, an MI355X (gfx950) implementation of the
 * population evaluation at the heart of EBIC (Orzechowski, Sipper, Huang &
 * Moore, "EBIC: an evolutionary-based parallel biclustering algorithm for
 * pattern discovery", Bioinformatics 2018) and of the evolutionary run that
 * drives it.
 *
 * Conventions
 *   - Every entry point returns ebic_status; EBIC_OK (0) is success.  No
 *     exception crosses the ABI.  On error, outputs are left untouched and
 *     ebic_last_error(ctx) holds a message.
 *   - Pointers documented as "host" are read or written by the CPU; "device"
 *     pointers are HIP device allocations on the context's device.
 *   - A context is not thread-safe: serialise calls on one context.
 *     Distinct contexts are independent.
 *   - Matrix values are IEEE binary32.  Any value is legal: NaN compares
 *     false against everything and +0 equals -0, so pairs holding NaN or a
 *     tie break both directions.
 *
 * Population wire format -- CBF, the Compressed Bicluster Format of Fig. 2:
 *   offsets  int32[P+1]   offsets[0] = 0, offsets[c+1] > offsets[c],
 *                         offsets[P] = total number of column entries
 *   cols     int32[offsets[P]]  0-based column indices; candidate c is the
 *                         ordered series cols[offsets[c] .. offsets[c+1])
 *
 * Row masks: masks[(c*2 + dir)*W + w], W = ebic_mask_words(n_rows), dir 0 =
 * rows following the rising trend, dir 1 = rows following the falling trend,
 * bit (r % 64) of word r / 64 set when row r matches; bits of rows >= n_rows
 * are zero.
 */
#ifndef EBIC_H
#define EBIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ebic_ctx ebic_ctx;
typedef struct ebic_result ebic_result;

typedef enum {
    EBIC_OK = 0,
    EBIC_E_ARG = 1,     /* null pointer, bad size, malformed CBF, duplicate column */
    EBIC_E_RANGE = 2,   /* column outside [0, n_cols), sigma < 0, max_violations < 0 */
    EBIC_E_NOMEM = 3,   /* device or host allocation failed */
    EBIC_E_DEVICE = 4,  /* a HIP call failed; see ebic_last_error */
    EBIC_E_STATE = 5    /* call not valid in the context's current state */
} ebic_status;

enum { EBIC_ROW_MAJOR = 0, EBIC_COL_MAJOR = 1 };

/* Evaluation strategies (ebic_set_path).  Both give identical results.
 *   DIRECT: every (candidate, row) pair reads the row's values along the
 *           series from the column-major matrix.
 *   INDEX:  a per-context pairwise order index, built once on the device,
 *           holds for every ordered column pair (p, q) the 64-row bitmasks
 *           of rows with a[r,p] < a[r,q]; evaluation then combines one
 *           64-bit word per consecutive pair and 64 rows.  Uses
 *           n_cols^2 * (wpad * 8 + 1) bytes of device memory (wpad =
 *           ceil(n_rows/64) rounded up to 16), plus a build scratch of
 *           ranks and bit-planes (about n_rows * n_cols * 3.7 bytes for up
 *           to 2048 columns) that the library keeps per device and reuses,
 *           and supports max_violations <= 3 (larger tolerances use DIRECT).
 *   AUTO:   INDEX when it fits the context's index budget, else DIRECT. */
enum { EBIC_PATH_AUTO = 0, EBIC_PATH_DIRECT = 1, EBIC_PATH_INDEX = 2 };

/* Trend and fitness parameters of one evaluation. */
typedef struct {
    uint32_t struct_size;     /* sizeof(ebic_params) */
    int32_t sigma;            /* Eq. (1): expected minimal number of rows, >= 0 */
    int32_t max_violations;   /* k >= 0: consecutive pairs a row may break per
                                 direction (approximate trends, Step 7) */
    int32_t negative_trends;  /* 0/1: also accept rows falling along the series
                                 (negative trends, Step 7); a row is counted
                                 once if either direction accepts it */
    int32_t want_masks;       /* 0: counts and fitness only; 1: also row masks */
} ebic_params;

typedef struct {
    uint32_t struct_size;     /* sizeof(ebic_ctx_info) */
    int32_t device;
    int64_t n_rows;
    int32_t n_cols;
    int64_t rows_padded;      /* leading dimension of the device matrix */
    int64_t mask_words;       /* W */
    int32_t path;             /* requested path (EBIC_PATH_*) */
    int32_t index_built;      /* 1 once the pairwise order index exists */
    int64_t index_bytes;      /* size of the index (built or prospective) */
    int64_t index_budget;     /* AUTO builds the index only within this many bytes */
    double index_build_ms;    /* device time of the last index build */
    int32_t index_ties;       /* 1 if two distinct columns have a tied or unordered row
                                 (then the falling test reads tie flags); valid once
                                 built */
} ebic_ctx_info;

/*
 * Matrix ingest (Step 1: the data is sent to the GPU once).
 *
 * ebic_create copies the host matrix a (n_rows x n_cols, element (r, j) at
 * a[r*ld + j] for EBIC_ROW_MAJOR or a[j*ld + r] for EBIC_COL_MAJOR) to the
 * device `device` as a column-major FP32 matrix padded to a multiple of 64
 * rows, and builds the log table of Eq. (1) on the host.  The caller may
 * free `a` on return.  ebic_create_device does the same from a device
 * pointer on that device: it synchronises the device first, so writes to
 * d_a pending on any stream are seen, and the caller keeps ownership.  The
 * context owns every device buffer and one HIP stream.
 * Errors: E_ARG (null pointer, n_rows < 1, n_cols < 1, ld too small, bad
 * layout), E_NOMEM, E_DEVICE.
 */
ebic_status ebic_create(const float *a, int64_t n_rows, int32_t n_cols, int64_t ld,
                        int32_t layout, int32_t device, ebic_ctx **out);
ebic_status ebic_create_device(const float *d_a, int64_t n_rows, int32_t n_cols, int64_t ld,
                               int32_t layout, int32_t device, ebic_ctx **out);
ebic_status ebic_destroy(ebic_ctx *ctx);

/* W = ceil(n_rows / 64), the number of 64-bit words of one row mask. */
int64_t ebic_mask_words(int64_t n_rows);

/* Choose the evaluation path (EBIC_PATH_*).  INDEX builds the index now if
 * it is missing (E_NOMEM if it cannot be allocated).  AUTO defers the
 * decision to each evaluation. */
ebic_status ebic_set_path(ebic_ctx *ctx, int32_t path);
/* Bytes the index may take under AUTO (default: 8 GiB, capped at a quarter
 * of the device's free memory at creation). */
ebic_status ebic_set_index_budget(ebic_ctx *ctx, int64_t bytes);
ebic_status ebic_get_info(const ebic_ctx *ctx, ebic_ctx_info *info);

/*
 * Population evaluation -- Step 4 (counts and fitness, Eq. (1)) and, with
 * want_masks, Step 6 (the rows matching each series).
 *
 * For each candidate c = (j_0 .. j_{L-1}) and each row r:
 *   vu = #{t < L-1 : !(a[r,j_t] < a[r,j_{t+1}])}
 *   vd = #{t < L-1 : !(a[r,j_t] > a[r,j_{t+1}])}
 *   rising(r)  = vu <= k,  falling(r) = negative_trends && vd <= k
 *   count[c]   = #{r : rising(r) || falling(r)}
 *   fitness[c] = count <= 1 ? 0 : 2^min(count - sigma, 0) * L * ln(count - 1)
 * computed in FP64 with the natural log (Eq. (1); |J| = L).
 *
 * ebic_evaluate: host pointers, blocking.  The CBF is validated (E_ARG for
 * offsets[0] != 0, non-increasing offsets, duplicate columns within a
 * candidate; E_RANGE for a column outside [0, n_cols), sigma < 0 or k < 0).
 * masks may be NULL unless want_masks; counts and fitness must not be NULL.
 * P = 0 returns EBIC_OK and touches nothing.
 */
ebic_status ebic_evaluate(ebic_ctx *ctx, const int32_t *offsets, const int32_t *cols, int32_t P,
                          const ebic_params *params, uint64_t *masks, int32_t *counts,
                          double *fitness);

/*
 * ebic_evaluate_device: device pointers, ordered on `hip_stream` (a
 * hipStream_t; NULL is the HIP null stream), returns without waiting.
 * d_offsets holds P+1 int32, d_cols n_entries int32; d_counts P int32,
 * d_fitness P doubles, d_masks 2*P*W words when want_masks.  The CBF is not
 * validated on the host: the kernels never read outside [0, n_entries) of
 * d_cols or outside the matrix, and a candidate whose offsets or columns are
 * malformed gets count -1 and fitness NaN (its mask words are unspecified).
 * Calls on one context share its scratch buffers: calls issued on different
 * streams must not overlap in time.  Duplicate columns are evaluated
 * by the definition above.  Buffers must stay alive until the stream
 * reaches the end of the call's work.
 */
ebic_status ebic_evaluate_device(ebic_ctx *ctx, const int32_t *d_offsets, const int32_t *d_cols,
                                 int32_t P, int64_t n_entries, const ebic_params *params,
                                 uint64_t *d_masks, int32_t *d_counts, double *d_fitness,
                                 void *hip_stream);

/*
 * ebic_evaluate_device_noalloc: for callers that cannot allocate device
 * memory -- code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results, stream ordering and
 * validation as ebic_evaluate_device; the call itself allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).
 *   Scratch: the per-candidate accumulators of the evaluation live in a
 *   fixed device array of EBIC_NOALLOC_MAX_CANDIDATES 8-byte entries
 *   (512 KiB) that the library holds on every device it runs on until the
 *   process ends (its address is taken when the first context on the device
 *   is created).  Each call clears the P entries it uses, with a fill kernel
 *   on hip_stream, before evaluating.  All calls on one GPU share that array:
 *   calls that overlap in time on one GPU (other streams, other contexts,
 *   other threads) race and must be serialised by the caller.
 *   Path: the order index is used only if it is already built (after
 *   ebic_set_path(ctx, EBIC_PATH_INDEX), or after an evaluation that built
 *   it); otherwise the direct kernel runs (identical results).
 * Errors: as ebic_evaluate_device; E_RANGE for P >
 * EBIC_NOALLOC_MAX_CANDIDATES; E_DEVICE if the array's address could not be
 * obtained on the context's device.
 */
#define EBIC_NOALLOC_MAX_CANDIDATES 65536
ebic_status ebic_evaluate_device_noalloc(ebic_ctx *ctx, const int32_t *d_offsets,
                                         const int32_t *d_cols, int32_t P, int64_t n_entries,
                                         const ebic_params *params, uint64_t *d_masks,
                                         int32_t *d_counts, double *d_fitness,
                                         void *hip_stream);

/* Wait for all work on the context's stream. */
ebic_status ebic_synchronize(ebic_ctx *ctx);

/*
 * The evolutionary run, Steps 1-7.  The paper fixes the structure; the
 * constants and operator details below are this library's readings:
 *
 *   RNG          SplitMix64 seeded with `seed`; uint(n) = next() % n.
 *   Step 1       P series of length len_min + uint(len_max - len_min + 1),
 *                distinct columns by rejection in draw order, a repeated
 *                series redrawn whole; evaluate; seed the top-rank list.
 *   Step 2       per-column penalties reset to 0; the first
 *                min(|top|, floor(P*elite_num/elite_den)) top-rank entries
 *                join the new population with their scores, adding 1 to
 *                the penalty of each of their columns.
 *   Step 3       until P members: tournament of `tournament` draws with
 *                replacement, adjusted quality fitness / penalty_base^theta,
 *                theta = (sum of the series' column penalties) / L, first
 *                best draw wins ties; one operation chosen with weights
 *                op_weight = {insert, delete, swap, substitute, crossover}
 *                (crossover takes a second tournament winner); a child seen
 *                before is a tabu hit, and more than tabu_limit hits (-1: P)
 *                in one generation end the run (go to Step 6); a novel child
 *                joins the population and the tabu list and adds 1 to its
 *                columns' penalties.
 *   Step 4       the new members are evaluated on the GPU with `eval`.
 *   Step 5       members by decreasing fitness (ties by position), fitness
 *                > 0 and not yet listed, are admitted unless a listed entry
 *                of at least equal fitness overlaps them by more than
 *                `overlap` (|x & e| / min(|x|, |e|) on column sets); an
 *                admitted member evicts weaker entries it overlaps by more
 *                than `overlap`; the list is sorted by fitness (stable) and
 *                cut to toplist_size.
 *   Steps 6-7    the listed series are evaluated with `expand` and returned
 *                with their matching rows (rising | falling).
 *   Mutations    (Fig. 1a-d) are no-ops when inapplicable and then draw
 *                nothing: insert needs L < len_max (position uint(L+1), a
 *                new column by rejection), delete needs L > len_min
 *                (position uint(L)), swap needs L >= 2 (i = uint(L),
 *                j = uint(L-1), j += 1 if j >= i), substitute needs
 *                L < n_cols (position uint(L), a new column by rejection).
 *   Crossover    (Fig. 1e) i = 1 + uint(|a|), j = uint(|b|), child = a[:i]
 *                then the columns of b[j:] not in a[:i], cut to len_max; a
 *                child shorter than len_min is a.
 *
 * Generation 0 is Step 1; `generations` more are run unless the tabu rule
 * stops the run earlier.  on_generation (may be NULL) sees every evaluated
 * population in CBF with its counts and fitness (elites carry their stored
 * scores).  Errors: E_ARG for bad bounds (1 <= len_min <= len_max <= n_cols,
 * P >= 1, tournament >= 1, weights >= 0 with a positive sum, 1 <= elite_den,
 * 0 <= elite_num <= elite_den, toplist_size >= 1, 0 <= overlap <= 1,
 * penalty_base > 0) or when P exceeds the number of distinct series.
 */
typedef void (*ebic_generation_fn)(void *user, int32_t gen, const int32_t *offsets,
                                   const int32_t *cols, int32_t P, const int32_t *counts,
                                   const double *fitness);

typedef struct {
    uint32_t struct_size;       /* sizeof(ebic_evolve_params) */
    int32_t population;         /* P */
    int32_t len_min, len_max;   /* series length bounds */
    int32_t tournament;         /* tournament size */
    int32_t op_weight[5];       /* insert, delete, swap, substitute, crossover */
    int32_t elite_num, elite_den;  /* elite share of P (Step 2: 1/4) */
    double penalty_base;        /* crowding penalty base (1.2) */
    double overlap;             /* top-rank overlap threshold (0.5 or 0.75) */
    int32_t toplist_size;       /* number of biclusters kept and reported */
    int32_t tabu_limit;         /* -1: the population size */
    ebic_params eval;           /* evolution-time trend parameters */
    ebic_params expand;         /* Step 7 trend parameters */
    ebic_generation_fn on_generation;
    void *user;
} ebic_evolve_params;

/* Fill p with this library's defaults for population P and length bounds. */
void ebic_evolve_defaults(ebic_evolve_params *p, int32_t population, int32_t len_min,
                          int32_t len_max, int32_t sigma);

ebic_status ebic_evolve(ebic_ctx *ctx, uint64_t seed, int32_t generations,
                        const ebic_evolve_params *params, ebic_result **out);

/*
 * The same run with a caller-supplied evaluator in place of the GPU, for
 * callers that score candidates themselves (and to test the host steps in
 * isolation).  eval receives host CBF arrays and must fill counts and
 * fitness (and masks, W = ebic_mask_words(n_rows) words per direction, when
 * p->want_masks) and return EBIC_OK.
 */
typedef ebic_status (*ebic_eval_fn)(void *user, const int32_t *offsets, const int32_t *cols,
                                    int32_t P, const ebic_params *p, uint64_t *masks,
                                    int32_t *counts, double *fitness);
ebic_status ebic_evolve_with(ebic_eval_fn eval, void *eval_user, int64_t n_rows, int32_t n_cols,
                             uint64_t seed, int32_t generations,
                             const ebic_evolve_params *params, ebic_result **out);

/*
 * Offspring screening with a caller-supplied ranking (not in the paper; the
 * host side of ebic_evolve_surrogate with any scorer, e.g. exact fitness).
 * Generations after warmup_generations draw a pool of oversample x (P -
 * elites) novel children and keep the P - elites that score ranks highest;
 * see ebic_evolve_surrogate for the pool rules.  score receives the pool as
 * host CBF (B series) and fills scores[B] (FP64, so exact fitness values rank
 * as ebic_evolve_oversampled ranks them; higher is better; NaN ranks last)
 * and returns EBIC_OK.  host_threads (<= 0: the hardware's) draws the pool in
 * parallel; results do not depend on it.  eval as in ebic_evolve_with.
 */
typedef ebic_status (*ebic_score_fn)(void *user, const int32_t *offsets, const int32_t *cols,
                                     int32_t B, double *scores);
ebic_status ebic_evolve_screened_with(ebic_eval_fn eval, void *eval_user, ebic_score_fn score,
                                      void *score_user, int64_t n_rows, int32_t n_cols,
                                      uint64_t seed, int32_t generations, int32_t oversample,
                                      int32_t warmup_generations, int32_t host_threads,
                                      const ebic_evolve_params *params, ebic_result **out);

/*
 * Offspring screening by exact fitness on the GPU (not in the paper): the
 * screened run of ebic_evolve_screened_with, with the pool of oversample x
 * (P - elites) children ranked by its exact Eq. (1) fitness (params->eval),
 * evaluated on ctx like any population.  The kept children's scores are
 * those exact values.  stats.candidates_evaluated and eval_ms include the
 * pools.  Errors as ebic_evolve.
 */
ebic_status ebic_evolve_oversampled(ebic_ctx *ctx, uint64_t seed, int32_t generations,
                                    int32_t oversample, int32_t warmup_generations,
                                    const ebic_evolve_params *params, ebic_result **out);

/* Result of a run: the top-rank biclusters after Step 7, best first. */
typedef struct {
    uint32_t struct_size;       /* sizeof(ebic_run_stats) */
    int32_t generations_run;    /* generations completed after Step 1 */
    int32_t stopped_by_tabu;    /* 1 if the tabu-hit rule ended the run */
    int64_t candidates_evaluated;
    double wall_ms;             /* whole run */
    double eval_ms;             /* inside Step 4 / Step 6 evaluations */
    double host_ms;             /* Steps 1-3 and 5 on the host */
} ebic_run_stats;

int32_t ebic_result_size(const ebic_result *r);
ebic_status ebic_result_get(const ebic_result *r, int32_t i, const int32_t **cols, int32_t *len,
                            int32_t *count, double *fitness, const uint64_t **row_mask);
ebic_status ebic_result_stats(const ebic_result *r, ebic_run_stats *stats);
void ebic_result_free(ebic_result *r);

/*
 * Stateful runs and checkpoints.  An ebic_run is the run of ebic_evolve
 * (same draws, same result) advanced a few generations at a time; between
 * generations it can be saved to bytes and resumed from them, and the
 * resumed run continues exactly as the uninterrupted one would (the random
 * stream, the last scored population, the tabu list and the top-rank list
 * are saved; caches are rebuilt).  ebic_run_create evaluates on ctx;
 * ebic_run_create_with on a caller's evaluator (as ebic_evolve_with).
 * Generation 0 is Step 1; ebic_run_advance performs up to max_generations
 * more generations (each: build, evaluate, Step 5) and sets *finished when
 * the run is over (all generations done or stopped by the tabu rule).
 * params is copied; its on_generation is called as in ebic_evolve (its
 * `user` must stay valid while the run advances).  ebic_run_result performs Steps 6-7 on the current top-rank list
 * (the run may still be advanced afterwards).
 *
 * Checkpoint bytes (ebic_run_save: with buf NULL only *size is set; E_RANGE
 * when capacity < *size): a magic tag, a version, the matrix shape, the
 * generation count, the draw-deciding parameters, then the run state.
 * ebic_run_load refuses (E_ARG) bytes of another matrix shape, other
 * parameters, another version, or bytes that do not parse.  Timing and
 * evaluation counters restart at zero in a loaded run.  Errors: message via
 * ebic_last_error(NULL) (evaluation failures: on ctx).
 */
typedef struct ebic_run ebic_run;
typedef struct {
    uint32_t struct_size;         /* sizeof(ebic_run_progress) */
    int32_t next_generation;      /* index of the next generation to build */
    int32_t generations_run;      /* generations completed after Step 1 */
    int32_t stopped_by_tabu;
    int32_t toplist;              /* entries in the top-rank list */
    double best_fitness;          /* fitness of its first entry (0 if empty) */
    int64_t tabu_size;            /* distinct series seen */
    int64_t candidates_evaluated; /* since creation or load */
    double eval_ms, wall_ms;      /* since creation or load */
} ebic_run_progress;

ebic_status ebic_run_create(ebic_ctx *ctx, uint64_t seed, int32_t generations,
                            const ebic_evolve_params *params, ebic_run **out);
ebic_status ebic_run_create_with(ebic_eval_fn eval, void *eval_user, int64_t n_rows,
                                 int32_t n_cols, uint64_t seed, int32_t generations,
                                 const ebic_evolve_params *params, ebic_run **out);
ebic_status ebic_run_advance(ebic_run *r, int32_t max_generations, int32_t *finished);
ebic_status ebic_run_get_progress(const ebic_run *r, ebic_run_progress *out);
ebic_status ebic_run_save(const ebic_run *r, void *buf, int64_t capacity, int64_t *size);
ebic_status ebic_run_load(ebic_ctx *ctx, const ebic_evolve_params *params, const void *buf,
                          int64_t size, ebic_run **out);
ebic_status ebic_run_load_with(ebic_eval_fn eval, void *eval_user, int64_t n_rows,
                               int32_t n_cols, const ebic_evolve_params *params, const void *buf,
                               int64_t size, ebic_run **out);
ebic_status ebic_run_result(ebic_run *r, ebic_result **out);
void ebic_run_destroy(ebic_run *r);

/*
 * Batched EBIC: many independent runs, each on its own matrix (any shapes),
 * sharing one GPU launch per generation.  Each run behaves exactly as
 * ebic_evolve on its own context with its own seed; the runs' populations
 * are evaluated together by one kernel over tiles of (run, candidate,
 * 64-row words), either one workgroup per tile or persistent workgroups
 * draining a tile queue, launched directly or as a captured HIP graph; the
 * run table lives in device memory and is refreshed each generation.  The
 * host steps of the runs proceed on host threads.  Evaluation uses each run's
 * pairwise order index (built at creation) for max_violations <= 3.  A run
 * whose index exceeds its context's budget (ebic_set_index_budget's
 * default) or does not fit in device memory has none; such runs, and every
 * run when max_violations > 3, are evaluated by the direct kernel, one
 * launch per run after the batched launch on the batch's stream.  Results
 * are the same either way.
 */
typedef struct ebic_batch ebic_batch;

/* matrices[r]: host row-major n_rows[r] x n_cols[r] FP32 (copied; the
 * caller may free them on return).  Errors: E_ARG (n_runs < 1, null or bad
 * sizes), E_NOMEM (a matrix does not fit; an order index that does not fit
 * leaves its run to the direct kernel), E_DEVICE. */
ebic_status ebic_batch_create(int32_t n_runs, const float *const *matrices, const int64_t *n_rows,
                              const int32_t *n_cols, int32_t device, ebic_batch **out);
ebic_status ebic_batch_destroy(ebic_batch *b);

/* Launch shape of the batched kernel: `workgroups` persistent workgroups
 * draining the tile queue (0: one per resident slot; -1: one workgroup per
 * tile and no queue), `unroll` pairs per batch of loads
 * (1, 2, 4 or 8), `words_per_lane` 64-row words per lane (1, 2, 4 or 8; a tile
 * is 256 lanes; unroll x words_per_lane at most 16) and `whole_candidates` (0: a tile is 256 consecutive
 * (candidate, word-group) items, a candidate may span tiles; 1: a tile holds
 * as many whole candidates as fit in 256 lanes, for runs whose candidates
 * fit, and per-candidate counts are reduced inside the workgroup).
 * `use_graph` = 1 replays the kernel as a captured one-node HIP graph
 * (re-captured when a buffer or the shape changes); 0 (default) launches it
 * directly.  The autotuner sets the first four fields and keeps use_graph. */
typedef struct {
    uint32_t struct_size;       /* sizeof(ebic_batch_tuning) */
    int32_t workgroups;
    int32_t unroll;
    double best_ms;             /* time of the chosen shape in the last tuning (0: untuned) */
    int32_t words_per_lane;
    int32_t whole_candidates;
    int32_t use_graph;
} ebic_batch_tuning;
ebic_status ebic_batch_get_tuning(const ebic_batch *b, ebic_batch_tuning *t);
ebic_status ebic_batch_set_tuning(ebic_batch *b, const ebic_batch_tuning *t);

/*
 * One population per run, evaluated in one launch (host arrays, blocking).
 * offsets[r]/cols[r] is run r's CBF with P[r] candidates (P[r] = 0 skips
 * the run); counts[r], fitness[r] receive P[r] values; masks may be NULL,
 * else masks[r] receives 2*P[r]*ebic_mask_words(n_rows[r]) words when
 * params->want_masks.  Same semantics and validation as ebic_evaluate.
 * With tune = 1 the launch shape is first chosen by timing a set of
 * candidate shapes on exactly this input (the autotuner); the result is
 * kept for later calls.
 */
ebic_status ebic_batch_evaluate(ebic_batch *b, const int32_t *const *offsets,
                                const int32_t *const *cols, const int32_t *P,
                                const ebic_params *params, uint64_t *const *masks,
                                int32_t *const *counts, double *const *fitness, int32_t tune);

/* Runs ebic_evolve's algorithm for every run r with seeds[r]; results[r]
 * receives run r's result (free each with ebic_result_free).  params is
 * shared by all runs (its on_generation is ignored; use on_generation
 * here, called with the run index, one call at a time).  host_threads <= 0
 * picks the hardware concurrency.  The launch shape is tuned on the first
 * generation unless set before. */
/* Device time (ms) of the last batched launch: the kernel, from events on
 * the batch's stream around its launch (the run table is copied before). */
double ebic_batch_last_ms(const ebic_batch *b);
/* Device time (ms) spent building the runs' pairwise order indexes at
 * ebic_batch_create (sum over runs, from events around each build). */
double ebic_batch_index_build_ms(const ebic_batch *b);
/* Replays the last batched launch `reps` times back to back on the batch's
 * stream (same inputs, same results written again) and stores the mean
 * device time per launch in ms, from events around the replays: the
 * kernel's own duration without per-call copies and synchronisation, for
 * profiling and launch-shape comparisons (the autotuner uses it).  Errors:
 * E_ARG (null, reps < 1, or no launch since the batch was created or since
 * a request with no candidates), E_DEVICE. */
ebic_status ebic_batch_time_replays(ebic_batch *b, int32_t reps, double *ms_per_launch);

typedef void (*ebic_batch_generation_fn)(void *user, int32_t run, int32_t gen,
                                         const int32_t *offsets, const int32_t *cols, int32_t P,
                                         const int32_t *counts, const double *fitness);
ebic_status ebic_batch_evolve(ebic_batch *b, const uint64_t *seeds, int32_t generations,
                              const ebic_evolve_params *params,
                              ebic_batch_generation_fn on_generation, void *user,
                              int32_t host_threads, ebic_result **results);
/* The same runs with Steps 1-3 and 5 on the device (Section 2.2; the
 * steps themselves are documented at ebic_evolve): one workgroup per run
 * keeps the run's random stream, tabu list, top-rank list and penalties in
 * device memory, so each generation is two launches on the batch's stream
 * -- the steps, then the batched evaluation of all P members (elites are
 * evaluated again; their scores are the same) -- with no host round trip.
 * Results equal ebic_batch_evolve's run for run.  Limits (E_ARG beyond
 * them): population <= 65535, len_max <= 58, tournament <= 31, n_cols <=
 * 65535, and one run's state (previous population, penalties, top-rank
 * list and its column index) within 160 KiB of LDS, operation weights
 * summing below 2^31.  Device memory per run: a tabu table of 16-byte slots
 * (2 (generations + 1) P rounded up to a power of two) and an arena of
 * (generations + 1) P len_max 16-bit columns.  on_generation (optional; it copies every generation
 * back and synchronises) sees each running run's population after its
 * evaluation.  In the stats, eval_ms is the device time of the whole
 * generation loop (steps and evaluations) plus the Steps 6-7 evaluation.
 * Every run needs its order index and max_violations <= 3 (E_ARG
 * otherwise).  Errors: E_STATE if a run's tabu table fills up. */
ebic_status ebic_batch_evolve_device(ebic_batch *b, const uint64_t *seeds, int32_t generations,
                                     const ebic_evolve_params *params,
                                     ebic_batch_generation_fn on_generation, void *user,
                                     ebic_result **results);

/*
 * Surrogate fitness model for screening offspring: a 3-layer MLP over
 * learned per-column embeddings (not in the paper; it only ranks
 * candidates, every admitted candidate is still scored exactly).
 *
 *   x    = [ mean over the series of E[c_t] + Z[L] ;
 *            mean over consecutive pairs of F[c_t] * T[c_{t+1}] (0 if L = 1) ]
 *          (E, F, T, Z: embed_dim each; the pair term makes the model see
 *          order, Z the series length L)
 *   h1   = relu(W1 bf16(x) + b1)        W1: hidden x (2 embed_dim)
 *   h2   = relu(W2 bf16(h1) + b2)       W2: hidden x hidden
 *   y    = w3 . bf16(h2) + b3           w3: hidden
 * Products use BF16 copies of the FP32 master weights on MFMA units with
 * FP32 accumulation; training minimises (1/B) sum (y - target)^2 with Adam
 * on the masters (gradients pass through the BF16 casts unchanged).
 * Parameters, flattened FP32 in this order: E, F, T [n_cols][embed_dim]
 * each, Z [n_cols + 1][embed_dim], W1 [hidden][2 embed_dim], b1 [hidden], W2 [hidden][hidden],
 * b2 [hidden], w3 [hidden], b3 [1].  All reductions run in a fixed order, so results are
 * deterministic on a given device.  Errors: message via ebic_last_error(NULL).
 */
typedef struct ebic_mlp ebic_mlp;
typedef struct {
    uint32_t struct_size;       /* sizeof(ebic_mlp_config) */
    int32_t embed_dim;          /* 32 */
    int32_t hidden;             /* 256 */
    float lr, beta1, beta2, eps;/* Adam: 1e-3, 0.9, 0.999, 1e-8 */
} ebic_mlp_config;

void ebic_mlp_defaults(ebic_mlp_config *c);
/* Parameters initialised from SplitMix64(seed): E, F, T ~ U(-1,1), Z = 0, W1 ~
 * U(+-sqrt(6/(2 embed_dim))), W2 ~ U(+-sqrt(6/hidden)), w3 ~
 * U(+-sqrt(3/hidden)), biases 0. */
ebic_status ebic_mlp_create(int32_t n_cols, const ebic_mlp_config *cfg, uint64_t seed,
                            int32_t device, ebic_mlp **out);
ebic_status ebic_mlp_destroy(ebic_mlp *m);
int64_t ebic_mlp_param_count(const ebic_mlp *m);
ebic_status ebic_mlp_get_params(const ebic_mlp *m, float *params);
ebic_status ebic_mlp_set_params(ebic_mlp *m, const float *params);   /* also resets Adam */
/* Host CBF in, host outputs, blocking.  Columns must lie in [0, n_cols) and
 * series hold 1 to n_cols entries (E_RANGE otherwise). */
ebic_status ebic_mlp_predict(ebic_mlp *m, const int32_t *offsets, const int32_t *cols, int32_t B,
                             float *y);
ebic_status ebic_mlp_gradients(ebic_mlp *m, const int32_t *offsets, const int32_t *cols,
                               int32_t B, const float *target, float *grad, float *loss);
ebic_status ebic_mlp_train_step(ebic_mlp *m, const int32_t *offsets, const int32_t *cols,
                                int32_t B, const float *target, float *loss);
/* `steps` Adam steps on one batch (uploaded once); *loss (may be NULL)
 * receives the loss before the last step.  Same result as `steps` calls of
 * ebic_mlp_train_step on the batch. */
ebic_status ebic_mlp_train(ebic_mlp *m, const int32_t *offsets, const int32_t *cols, int32_t B,
                           const float *target, int32_t steps, float *loss);

/*
 * Surrogate-screened run (not in the paper).  As ebic_evolve, except that
 * after `warmup_generations` a generation draws oversample x (P - elites)
 * novel children and keeps the P - elites that the surrogate MLP ranks
 * highest.  The pool is drawn by 16 breeders in parallel: breeder j draws an
 * equal share by Step 3's rules (tournament with crowding penalties starting
 * from the elites' and adding its own children's, one operation, novel with
 * respect to the tabu list and its share) from a stream seeded by the j-th
 * of 16 draws of the run's stream; shares are joined in order without
 * repeats (the run's own breeder tops up a short pool).  The outcome does not
 * depend on the number of host threads.
 * Every kept child is scored exactly on the GPU; only kept children enter
 * the tabu list.  The model is trained each generation (train_steps Adam
 * steps) on the exact (candidate, log(1 + fitness)) pairs of the last
 * replay_generations generations.  The rank check: in a screened
 * generation, check_sample pool members drawn uniformly (from a stream of
 * the check's own) are also scored exactly and compared with the model's
 * predictions (Spearman rank correlation); in a plainly bred generation the
 * new members are.  A generation is screened only if the previous
 * generation's correlation reached min_rank_corr, otherwise it is bred
 * exactly as in ebic_evolve (the plain method is the fallback).  The
 * sample's evaluations count in the run's statistics.
 * on_surrogate (may be NULL) reports, per generation: whether it was
 * screened, the rank correlation, the training loss and the pool size.
 */
typedef void (*ebic_surrogate_fn)(void *user, int32_t gen, int32_t screened, double rank_corr,
                                  double train_loss, int32_t pool);
typedef struct {
    uint32_t struct_size;         /* sizeof(ebic_surrogate_params) */
    int32_t oversample;           /* 8 */
    int32_t warmup_generations;   /* 3 */
    int32_t train_steps;          /* 16 */
    int32_t replay_generations;   /* 4 */
    double min_rank_corr;         /* 0.1 */
    uint64_t mlp_seed;
    ebic_mlp_config mlp;          /* ebic_mlp_defaults with lr 3e-3 */
    ebic_surrogate_fn on_surrogate;
    void *user;
    int32_t check_sample;         /* 512: pool members scored exactly to check the ranking */
    int32_t exact_rerank;         /* 0; r > 0: the network keeps r x (P - elites) of the
                                     pool, those are scored exactly and the best kept */
} ebic_surrogate_params;

void ebic_surrogate_defaults(ebic_surrogate_params *s);
ebic_status ebic_evolve_surrogate(ebic_ctx *ctx, uint64_t seed, int32_t generations,
                                  const ebic_evolve_params *params,
                                  const ebic_surrogate_params *sp, ebic_result **out);

/*
 * Step 6 output on the device: the indices of the rows each bicluster
 * matches, from its 64-row masks (bit r mod 64 of word r / 64, as written by
 * ebic_evaluate*).  d_masks: [K][planes][W] words, W = ebic_mask_words(n_rows);
 * the planes of a bicluster are united (planes = 2 takes both trend
 * directions of ebic_evaluate's masks); bits at or beyond n_rows are not
 * rows.  Outputs (device, caller-owned): d_offsets [K + 1] int64 with
 * d_offsets[0] = 0 and bicluster k's rows at d_rows[d_offsets[k] ..
 * d_offsets[k + 1]), increasing; entries at or beyond rows_capacity are not
 * written, so a caller that sizes d_rows after reading d_offsets[K] (or
 * passes n_rows * K) gets every list.  Stream-ordered on hip_stream (NULL:
 * the HIP null stream); allocates nothing.  Errors: E_ARG (negative sizes,
 * null pointers, n_rows > INT32_MAX), E_DEVICE (launch), message via
 * ebic_last_error(NULL).
 */
ebic_status ebic_mask_rows(const uint64_t *d_masks, int32_t K, int32_t planes, int64_t n_rows,
                           int64_t *d_offsets, int32_t *d_rows, int64_t rows_capacity,
                           void *hip_stream);

/* A set of biclusters in device memory: rows as masks [count][planes][W]
 * (planes united, as in ebic_mask_rows), columns as CBF (col_offsets
 * [count + 1], cols).  Column order does not matter here; repeated columns
 * count once. */
typedef struct {
    uint32_t struct_size;        /* sizeof(ebic_bicluster_set) */
    int32_t count;
    int32_t planes;
    const uint64_t *row_masks;
    const int32_t *col_offsets;
    const int32_t *cols;
} ebic_bicluster_set;

/*
 * Accuracy of found biclusters against expected ones (Section 3, Eqs. 2-3)
 * on the device.  Each bicluster is the set of cells rows x columns; the
 * Jaccard index of two is |intersection| / |union| of their cells (0 when
 * both are empty).  d_jaccard [found->count][expected->count] (FP64,
 * row-major; may be NULL only if either count is 0) receives every index;
 * d_scores[0] = recovery = mean over expected e of max over found f of
 * J[f][e], d_scores[1] = relevance = mean over found f of max over expected
 * e of J[f][e] (both 0 when either set is empty).  The paper prints the two
 * as bare sums and reports shares; we divide by the set sizes.  Sums are
 * taken in index order, so results are deterministic.  Stream-ordered on
 * hip_stream; allocates nothing.  Errors: E_ARG (bad set descriptions, null
 * outputs, more than 2^33 pairs), E_DEVICE; message via ebic_last_error(NULL).
 */
ebic_status ebic_match_scores(const ebic_bicluster_set *found, const ebic_bicluster_set *expected,
                              int64_t n_rows, double *d_jaccard, double *d_scores,
                              void *hip_stream);

/* Message of the last error on ctx.  With ctx == NULL: the calling thread's
 * last error from a call that had no context (ebic_create*, argument errors
 * of ebic_evolve*, ebic_result_*); an evaluation failure inside
 * ebic_evolve is reported on its context. */
const char *ebic_last_error(const ebic_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* EBIC_H */
