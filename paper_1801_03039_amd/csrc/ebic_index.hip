// Pairwise order index from per-row ranks (gfx950, wave64).
//
// The index holds, for every ordered column pair (p, q) and 64-row word w,
// the bits of the rows r with a[r,p] < a[r,q]: the strict comparison of the
// trend test (Motivation: a row follows the series when its values increase
// strictly along it; Step 7 reverses or relaxes that test).  Row by row, the
// comparisons between columns depend only on the order of the row's values,
// so the build first replaces each row by its ranks and then compares ranks
// as bit-sliced integers, 64 rows per operation:
//
//   1. rank   each row's values become order-preserving 32-bit keys; a wave
//             sorts them (bitonic network, 16 keys per lane up to 1024
//             columns, 32 up to 2048) and every column's rank is the number
//             of smaller keys in the row (a binary search of the sorted
//             row).  Equal values share a rank.  A row with two equal values
//             or a NaN flags its 64-row word.
//   2. planes each (column, word) becomes b bit-planes of its rows' ranks
//             (b = rank bits) plus one plane of its NaN rows.
//   3. compare lane = word: lt(p,q) = the rows whose rank in p is below the
//             rank in q, from the b planes of p and q, least significant
//             first (at each plane the rows where the planes differ take q's
//             bit, the others keep what lower planes decided).  In a wave
//             with no flagged word the two orders are exact complements:
//             lt(q,p) = ~lt(p,q) on valid rows.  Otherwise lt(q,p) is formed
//             the same way, NaN rows are cleared from both, and tied pairs
//             are reported.
//
// The compare step stores 512 contiguous bytes per wave and order row, and
// issues about 2 ALU operations per plane and half-word, so the build is
// bound by its index writes rather than by its comparisons.  The order words
// are stored non-temporally: nothing reads them before the build ends, and
// streaming them past the caches keeps the planes there.  Matrices with
// more than kRankMaxCols columns keep the direct ballot build of
// ebic_kernels.hip.
#include "ebic_device.h"

namespace ebic {
namespace {

constexpr uint32_t kNanKey = 0xFFFFFFFFu;   // NaN and pad slots: above every real key
constexpr uint16_t kNanRank = 0xFFFFu;      // rank stored for a NaN value (bit 15 set)
constexpr int kNanBit = 15;

// Order-preserving image of an FP32 value: x < y exactly when
// key(x) < key(y), and x == y exactly when the keys are equal (-0 and +0
// share one key); every NaN maps to kNanKey.
__device__ __forceinline__ uint32_t order_key(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return kNanKey;
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// The value of lane (lane ^ X): DPP for the patterns that stay inside a
// row of 16 lanes and have one (quad permutations, row mirrors, the
// rotation by 8; for X = 4 two row shifts, each writing the banks of four
// lanes that read from its side), a swizzle for other patterns within 32
// lanes, a permute across the halves.
template <int X>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
    const int s = (int)v;
    if constexpr (X == 1) return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0xB1, 0xF, 0xF, false);
    else if constexpr (X == 2) return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x4E, 0xF, 0xF, false);
    else if constexpr (X == 3) return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x1B, 0xF, 0xF, false);
    else if constexpr (X == 4) {
        const int up = __builtin_amdgcn_update_dpp(0, s, 0x104, 0xF, 0x5, false);   // row_shl:4
        return (uint32_t)__builtin_amdgcn_update_dpp(up, s, 0x114, 0xF, 0xA, false);  // row_shr:4
    }
    else if constexpr (X == 7) return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x141, 0xF, 0xF, false);
    else if constexpr (X == 8) return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x128, 0xF, 0xF, false);
    else if constexpr (X == 15) return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x140, 0xF, 0xF, false);
    else if constexpr (X < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle(s, 0x1F | (X << 10));
    else return (uint32_t)__shfl_xor(s, X);
}
// The median of three: with c = 0 the smaller of a and b, with c = ~0 the
// larger (one v_med3_u32).
__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c) {
    return max(min(a, b), min(max(a, b), c));
}

// Bitonic sorting network over the E x (lanes) slots of a row, slot
// j = lg * E + e, ascending.  Merge form: the first stage of each merge of
// two sorted blocks of 2^(LK-1) slots pairs slot j with its mirror
// j ^ (2^LK - 1), later stages pair j with j ^ 2^LD; in every pair the
// lower slot keeps the smaller key, so no stage needs a per-lane direction.
// A pair in two lanes exchanges keys through a lane permutation (at
// distance 16 a swap of 16-lane rows that leaves both keys in each lane).
// The stages are template recursions, so every distance is a constant.
template <int E, int LD>
__device__ __forceinline__ void bitonic_halves(uint32_t (&x)[E], int lg) {
    if constexpr (LD >= 0) {
        constexpr int d = 1 << LD;
        if constexpr (d < E) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (e & d) continue;
                const uint32_t lo = min(x[e], x[e | d]), hi = max(x[e], x[e | d]);
                x[e] = lo;
                x[e | d] = hi;
            }
        } else {
            constexpr int dl = d / E;
            const uint32_t keep = (lg & dl) ? ~0u : 0u;   // upper lanes keep the larger
            if constexpr (dl == 16) {
                // rows of 16 lanes swap in pairs: each lane then holds both
                // keys of its pair, and min or max needs no order of the two
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const auto two = __builtin_amdgcn_permlane16_swap(x[e], x[e], false, false);
                    x[e] = med3_u32(two[0], two[1], keep);
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) x[e] = med3_u32(x[e], lane_xor<dl>(x[e]), keep);
            }
        }
        bitonic_halves<E, LD - 1>(x, lg);
    }
}
template <int E, int LK, int LOGM>
__device__ __forceinline__ void bitonic_merges(uint32_t (&x)[E], int lg) {
    if constexpr (LK <= LOGM) {
        constexpr int k = 1 << LK;
        if constexpr (k <= E) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (e & (k >> 1)) continue;
                const int f = e ^ (k - 1);
                const uint32_t lo = min(x[e], x[f]), hi = max(x[e], x[f]);
                x[e] = lo;
                x[f] = hi;
            }
        } else {
            constexpr int kl = k / E;   // lanes of the merged block
            const uint32_t keep = (lg & (kl >> 1)) ? ~0u : 0u;
            uint32_t y[E];
#pragma unroll
            for (int e = 0; e < E; ++e) y[e] = lane_xor<kl - 1>(x[E - 1 - e]);
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = med3_u32(x[e], y[e], keep);
        }
        bitonic_halves<E, LK - 2>(x, lg);
        bitonic_merges<E, LK + 1, LOGM>(x, lg);
    }
}

// Rows of a rank launch: 2^LOGM key slots per row (the columns padded to a
// power of two), E per lane, GL lanes per row.
template <int LOGM>
struct RankShape {
    static constexpr int M = 1 << LOGM;
    static constexpr int E = M <= 1024 ? 16 : M / kWave;
    static constexpr int GL = M / E;
    static constexpr int RPW = kWave / GL;     // rows per wave
    static constexpr int RPB = 4 * RPW;        // rows per workgroup (4 waves)
    static_assert(LOGM >= 4 && GL >= 1 && GL <= kWave, "rank shape");
};

// Step 1.  Workgroup = RPB consecutive rows; blocks are dealt to the XCDs in
// contiguous ranges so that neighbouring rows share an L2.
template <int LOGM>
__global__ __launch_bounds__(kBlock) void index_rank_kernel(const float *__restrict__ a, int64_t n,
                                                           int64_t npad, int32_t m,
                                                           int64_t blocks, int64_t per_xcd,
                                                           uint16_t *__restrict__ rank,
                                                           int64_t mr, uint32_t *__restrict__ wflag) {
    using S = RankShape<LOGM>;
    constexpr int M = S::M, E = S::E, GL = S::GL, RPW = S::RPW;
    __shared__ uint32_t s_sorted[4 * RPW * M];
    const int64_t b = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    if (b >= blocks) return;   // uniform per workgroup
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane / GL, lg = lane % GL;
    const int64_t r = b * S::RPB + wv * RPW + grp;
    const bool row_ok = r < n;

    // Every lane loads all its slots from clamped, in-bounds addresses (no
    // load waits on another); slots past the row's columns take kNanKey.
    const int64_t rc = row_ok ? r : n - 1;
    float v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = a[(int64_t)min(lg * E + e, m - 1) * npad + rc];
    uint32_t x[E];
    bool nan_seen = false;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const bool in = row_ok && lg * E + e < m;
        const uint32_t k = order_key(v[e]);
        nan_seen |= in && k == kNanKey;
        x[e] = in ? k : kNanKey;
    }
    uint32_t o[E];   // the row's keys, kept for the rank search
#pragma unroll
    for (int e = 0; e < E; ++e) o[e] = x[e];

    // Bitonic sort of the row's M slots, ascending; slot j = lg * E + e.
    bitonic_merges<E, 1, LOGM>(x, lg);

    // A tie: two equal real keys are neighbours in the sorted row.
    bool tie = false;
#pragma unroll
    for (int e = 0; e + 1 < E; ++e) tie |= x[e] == x[e + 1] && x[e] != kNanKey;
    const uint32_t next = (uint32_t)__shfl_down((int)x[0], 1);
    if (lg + 1 < GL) tie |= x[E - 1] == next && x[E - 1] != kNanKey;
    const uint64_t flagged = ballot(row_ok && (tie || nan_seen));
    const uint64_t gmask = (GL == kWave ? ~0ull : ((1ull << GL) - 1ull)) << (grp * GL);
    if (lg == 0 && (flagged & gmask) != 0ull) atomicOr(wflag + (r >> 6), 1u);

    uint32_t *row = s_sorted + (wv * RPW + grp) * M;
#pragma unroll
    for (int e = 0; e < E; ++e) row[lg * E + e] = x[e];
    __syncthreads();
    if (!row_ok) return;
    // Ranks of the lane's E columns, stored as 16-byte pieces (the row
    // stride mr is a multiple of 64, so every piece lies inside the row).
    uint32_t rk[E / 2];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t key = o[e];
        uint32_t pos = 0;   // number of sorted keys below `key`
#pragma unroll
        for (int ls = LOGM - 1; ls >= 0; --ls)
            if (row[pos + (1u << ls) - 1] < key) pos += 1u << ls;
        const uint32_t v = key == kNanKey ? kNanRank : pos;
        if (e & 1) rk[e / 2] |= v << 16;
        else rk[e / 2] = v;
    }
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int i = 0; i < E / 8; ++i) {
        const int32_t j = lg * E + 8 * i;
        if (j < m) {
            u32x4 v;
            v.x = rk[4 * i];
            v.y = rk[4 * i + 1];
            v.z = rk[4 * i + 2];
            v.w = rk[4 * i + 3];
            *(u32x4 *)(rank + r * mr + j) = v;
        }
    }
}

// Step 2.  Workgroup = 4 waves, wave = (16 columns, one 64-row word):
// lane = (column c, quarter u of the word's rows); the lane gathers the
// ranks of its 16 rows (pad rows: rank 0) into 16-bit slices of each plane,
// and the four quarters are joined with two lane exchanges.  Plane k < NB
// holds bit k of the rows' ranks, plane NB the NaN rows:
// planes[(p*(NB+1) + k)*wq + w].  Workgroups are dealt to the XCDs in
// contiguous word ranges, so the eight-byte stores of neighbouring words
// meet in one L2.
template <int NB>
__global__ __launch_bounds__(kBlock) void index_planes_kernel(const uint16_t *__restrict__ rank,
                                                             int64_t n, int32_t m, int64_t mr,
                                                             int64_t W, int64_t wq,
                                                             int64_t col_groups, int64_t items,
                                                             int64_t per_xcd,
                                                             uint64_t *__restrict__ planes) {
    constexpr int NB1 = NB + 1;
    const int64_t blk = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    const int lane = threadIdx.x & 63;
    const int64_t item = blk * (kBlock / kWave) + (threadIdx.x >> 6);
    if (item >= items) return;   // uniform per wave
    const int64_t w = item / col_groups, cg = item - w * col_groups;
    const int c = lane >> 2, u = lane & 3;
    const int32_t p = (int32_t)(cg * 16) + c;
    const bool col_ok = p < m;
    const int64_t r0 = w * 64 + u * 16;
    uint32_t v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t r = r0 + i;
        v[i] = (col_ok && r < n) ? (uint32_t)rank[r * mr + p] : 0u;
    }
    uint32_t pl[NB1];
#pragma unroll
    for (int k = 0; k < NB1; ++k) {
        const int bit = k < NB ? k : kNanBit;
        uint32_t x = 0u;
#pragma unroll
        for (int i = 0; i < 16; ++i) x |= ((v[i] >> bit) & 1u) << i;
        pl[k] = x;
    }
    // quarters u = 0..3 hold rows 16u..16u+15: lanes of a column exchange
    // their slices (lane ^ 1, then lane ^ 2)
    uint32_t lo[NB1], hi[NB1];
#pragma unroll
    for (int k = 0; k < NB1; ++k) {
        const uint32_t mine = pl[k] << (16 * (u & 1));
        const uint32_t half = mine | (uint32_t)__shfl_xor((int)mine, 1);   // 32 rows
        const uint32_t other = (uint32_t)__shfl_xor((int)half, 2);
        lo[k] = (u & 2) ? other : half;
        hi[k] = (u & 2) ? half : other;
    }
    if (!col_ok) return;
    // lane u stores planes u, u+4, u+8, ... of its column
#pragma unroll
    for (int k = 0; k < NB1; ++k)
        if ((k & 3) == u) planes[((int64_t)p * NB1 + k) * wq + w] = ((uint64_t)hi[k] << 32) | lo[k];
}

// Step 3.  Workgroup = (64-word block, column groups g <= h of 16 columns):
// wave v holds the planes of the four columns p = 16g + 4v + i and takes
// every q >= p of group h; lane = word.  Each q's planes are loaded once
// for four pairs, so the plane reads stay below the index writes.  Within
// a word block, tiles run through the groups h in order (all g <= h for
// each h), so the planes of group h are read from L2 by every tile that
// pairs with it; tiles are dealt to the XCDs in contiguous ranges.
constexpr int kComparePerWave = 4;
template <int NB>
__global__ __launch_bounds__(kBlock) void index_compare_kernel(
    const uint64_t *__restrict__ planes, const uint32_t *__restrict__ wflag, int64_t n,
    int32_t m, int64_t W, int64_t wq, int64_t wpad, int32_t G, int64_t pairs, int64_t tiles,
    int64_t per_xcd, uint64_t *__restrict__ idx, uint8_t *__restrict__ tie,
    int32_t *__restrict__ any_tie, uint32_t *__restrict__ tbits) {
    constexpr int NB1 = NB + 1;
    constexpr int PW = kComparePerWave;
    const int64_t t = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    if (t >= tiles) return;
    const int64_t wb = t / pairs;
    const int64_t k = t - wb * pairs;
    // k-th pair (g, h), g <= h < G, ordered by h then g: h is the largest
    // with h(h+1)/2 <= k
    int32_t h = (int32_t)((__builtin_sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
    while ((int64_t)(h + 1) * (h + 2) / 2 <= k) ++h;
    while ((int64_t)h * (h + 1) / 2 > k) --h;
    const int32_t g = (int32_t)(k - (int64_t)h * (h + 1) / 2);
    const int lane = threadIdx.x & 63;
    const int32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t p0 = 16 * g + PW * wv;
    if (p0 >= m) return;                                  // uniform per wave
    const int32_t q_lo = max(16 * h, p0), q_hi = min(16 * h + 16, m);
    if (q_lo >= q_hi) return;                             // uniform per wave
    const uint32_t lw = (uint32_t)(wb * kWave) + (uint32_t)lane;   // word of the lane (< wq)
    const bool word_ok = lw < (uint64_t)W;
    const uint64_t valid = word_ok ? tail_bits(n, lw, W) : 0ull;

    // planes of the wave's columns p0 + i (a column past m repeats the last
    // one; its pairs are skipped)
    uint32_t pp[PW][2][NB];
#pragma unroll
    for (int i = 0; i < PW; ++i) {
        const int32_t p = min(p0 + i, m - 1);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uint64_t v = (planes + ((int64_t)p * NB1 + b) * wq)[lw];
            pp[i][0][b] = (uint32_t)v;
            pp[i][1][b] = (uint32_t)(v >> 32);
        }
    }
    const bool flagged = ballot(word_ok && wflag[lw] != 0u) != 0ull;

    // lt (rows with rank_p < rank_q) and, with GT, gt (rank_p > rank_q) of
    // one half-word, least significant plane first.
    auto compare = [&](const uint32_t (&pb)[NB], const uint32_t (&qb)[NB], auto want_gt,
                       uint32_t &gt) {
        constexpr bool GT = decltype(want_gt)::value;
        uint32_t lt = ~pb[0] & qb[0];
        if constexpr (GT) gt = pb[0] & ~qb[0];
#pragma unroll
        for (int b = 1; b < NB; ++b) {
            const uint32_t d = pb[b] ^ qb[b];
            lt = (d & qb[b]) | (~d & lt);
            if constexpr (GT) gt = (d & pb[b]) | (~d & gt);
        }
        return lt;
    };
    auto store = [&](int32_t p, int32_t q, uint64_t lt, uint64_t rev) {
        if (word_ok) {
            __builtin_nontemporal_store(lt, idx + ((int64_t)p * m + q) * wpad + lw);
            if (q != p) __builtin_nontemporal_store(rev, idx + ((int64_t)q * m + p) * wpad + lw);
        }
    };
    uint64_t pnan[PW];
#pragma unroll
    for (int i = 0; i < PW; ++i)
        pnan[i] = flagged ? (planes + ((int64_t)min(p0 + i, m - 1) * NB1 + NB) * wq)[lw] : 0ull;

    for (int32_t q = q_lo; q < q_hi; ++q) {
        uint32_t qq[2][NB];
        const uint64_t *base = planes + (int64_t)q * NB1 * wq;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uint64_t v = (base + b * wq)[lw];
            qq[0][b] = (uint32_t)v;
            qq[1][b] = (uint32_t)(v >> 32);
        }
        if (!flagged) {
            // no tied or NaN row in any word of the wave: lt(q,p) = ~lt(p,q)
#pragma unroll
            for (int i = 0; i < PW; ++i) {
                const int32_t p = p0 + i;
                if (p >= m || q < p) continue;   // uniform
                uint32_t unused = 0;
                const uint64_t lt =
                    ((uint64_t)compare(pp[i][1], qq[1], std::false_type{}, unused) << 32) |
                    compare(pp[i][0], qq[0], std::false_type{}, unused);
                store(p, q, lt, ~lt & valid);
            }
            continue;
        }
        const uint64_t qnan = (base + NB * wq)[lw];
#pragma unroll
        for (int i = 0; i < PW; ++i) {
            const int32_t p = p0 + i;
            if (p >= m || q < p) continue;   // uniform
            uint32_t g0, g1;
            const uint32_t l0 = compare(pp[i][0], qq[0], std::true_type{}, g0);
            const uint32_t l1 = compare(pp[i][1], qq[1], std::true_type{}, g1);
            const uint64_t keep = ~(pnan[i] | qnan);   // a NaN row is ordered with nothing
            const uint64_t lt = (((uint64_t)l1 << 32) | l0) & keep;
            const uint64_t gt = (((uint64_t)g1 << 32) | g0) & keep;
            store(p, q, lt, gt);
            // tied rows: valid, in neither order (equal values or a NaN)
            const bool tied = word_ok && q != p && (valid & ~(lt | gt)) != 0ull;
            if (ballot(tied) != 0ull && lane == 0) {
                tie[(int64_t)p * m + q] = 1;
                tie[(int64_t)q * m + p] = 1;
                any_tie[0] = 1;
                const uint32_t h0 = tie_hash((uint32_t)p * (uint32_t)m + (uint32_t)q);
                const uint32_t h1 = tie_hash((uint32_t)q * (uint32_t)m + (uint32_t)p);
                atomicOr(tbits + (h0 >> 5), 1u << (h0 & 31));
                atomicOr(tbits + (h1 >> 5), 1u << (h1 & 31));
            }
        }
    }
}

// Clears the tie flags (a column is always tied with itself: lt(p,p) = 0
// both ways), the any-tie flag, the tie-pair bitmap and the word flags.
__global__ __launch_bounds__(kBlock) void index_init_kernel(uint8_t *__restrict__ tie, int32_t m,
                                                           int64_t n_flags,
                                                           int32_t *__restrict__ any_tie,
                                                           uint32_t *__restrict__ tbits,
                                                           uint32_t *__restrict__ wflag,
                                                           int64_t wq) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n_flags) tie[i] = (i % ((int64_t)m + 1)) == 0 ? 1 : 0;
    if (i < kTieWords) tbits[i] = 0;
    if (i < wq) wflag[i] = 0;
    if (i == 0) any_tie[0] = 0;
}

// Rank bits stored per column: enough for ranks up to m-1, rounded up to
// an even count (fewer kernel forms; extra planes are zero on both sides).
int rank_planes(int32_t m) {
    int b = 1;
    while ((1ll << b) < (int64_t)m) ++b;
    return b <= 4 ? 4 : (b + 1) / 2 * 2;
}

struct RankedLayout {
    int logm = 0, nb = 0;
    int64_t wq = 0, mr = 0;
    size_t off_rank = 0, off_planes = 0, bytes = 0;
};

RankedLayout ranked_layout(int64_t n, int32_t m, int64_t W) {
    RankedLayout L;
    int logm = 4;
    while ((1 << logm) < m) ++logm;
    L.logm = logm;
    L.nb = rank_planes(m);
    L.wq = (W + kWave - 1) / kWave * kWave;
    L.mr = ((int64_t)m + kWave - 1) / kWave * kWave;
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    L.off_rank = up((size_t)L.wq * sizeof(uint32_t));
    L.off_planes = L.off_rank + up((size_t)n * (size_t)L.mr * sizeof(uint16_t));
    L.bytes = L.off_planes + (size_t)m * (size_t)(L.nb + 1) * (size_t)L.wq * sizeof(uint64_t);
    return L;
}

template <int LOGM>
hipError_t launch_rank(const float *a, int64_t n, int64_t npad, int32_t m, uint16_t *rank,
                       int64_t mr, uint32_t *wflag, hipStream_t stream) {
    using S = RankShape<LOGM>;
    const int64_t blocks = (n + S::RPB - 1) / S::RPB;
    const int64_t per_xcd = (blocks + kXcds - 1) / kXcds;
    const int64_t grid = per_xcd * kXcds;
    if (grid > 0x7FFFFFFFll) return hipErrorInvalidValue;
    hipLaunchKernelGGL(index_rank_kernel<LOGM>, dim3((unsigned)grid), dim3(kBlock), 0, stream, a,
                       n, npad, m, blocks, per_xcd, rank, mr, wflag);
    return hipGetLastError();
}

template <int NB>
hipError_t launch_planes_compare(const uint16_t *rank, const uint32_t *wflag, int64_t n,
                                 int32_t m, int64_t mr, int64_t W, int64_t wq, int64_t wpad,
                                 uint64_t *planes, uint64_t *idx, uint8_t *tie, int32_t *any_tie,
                                 uint32_t *tbits, hipStream_t stream) {
    const int64_t col_groups = ((int64_t)m + 15) / 16;
    const int64_t items = col_groups * W;
    const int64_t pblocks = (items + 3) / 4;
    const int64_t pper = (pblocks + kXcds - 1) / kXcds;
    if (pper * kXcds > 0x7FFFFFFFll) return hipErrorInvalidValue;
    hipLaunchKernelGGL(index_planes_kernel<NB>, dim3((unsigned)(pper * kXcds)), dim3(kBlock), 0,
                       stream, rank, n, m, mr, W, wq, col_groups, items, pper, planes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int32_t G = (m + 15) / 16;
    const int64_t pairs = (int64_t)G * (G + 1) / 2;
    const int64_t tiles = (wq / kWave) * pairs;
    const int64_t per_xcd = (tiles + kXcds - 1) / kXcds;
    const int64_t grid = per_xcd * kXcds;
    if (grid > 0x7FFFFFFFll) return hipErrorInvalidValue;
    hipLaunchKernelGGL(index_compare_kernel<NB>, dim3((unsigned)grid), dim3(kBlock), 0, stream,
                       planes, wflag, n, m, W, wq, wpad, G, pairs, tiles, per_xcd, idx, tie,
                       any_tie, tbits);
    return hipGetLastError();
}

}  // namespace

namespace {
template <int LOGM>
hipError_t resolve_rank() {
    hipFuncAttributes fa;
    return hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&index_rank_kernel<LOGM>));
}
template <int NB>
hipError_t resolve_planes_compare() {
    hipFuncAttributes fa;
    hipError_t e =
        hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&index_planes_kernel<NB>));
    if (e != hipSuccess) return e;
    return hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&index_compare_kernel<NB>));
}
}  // namespace

hipError_t index_ranked_prepare(int32_t m) {
    if (m < 1 || m > kRankMaxCols) return hipErrorInvalidValue;
    const RankedLayout L = ranked_layout(1, m, 1);
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&index_init_kernel));
    if (e != hipSuccess) return e;
    switch (L.logm) {
    case 4: e = resolve_rank<4>(); break;
    case 5: e = resolve_rank<5>(); break;
    case 6: e = resolve_rank<6>(); break;
    case 7: e = resolve_rank<7>(); break;
    case 8: e = resolve_rank<8>(); break;
    case 9: e = resolve_rank<9>(); break;
    case 10: e = resolve_rank<10>(); break;
    case 11: e = resolve_rank<11>(); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    switch (L.nb) {
    case 4: return resolve_planes_compare<4>();
    case 6: return resolve_planes_compare<6>();
    case 8: return resolve_planes_compare<8>();
    case 10: return resolve_planes_compare<10>();
    case 12: return resolve_planes_compare<12>();
    default: return hipErrorInvalidValue;
    }
}

size_t index_ranked_scratch_bytes(int64_t n, int32_t m, int64_t W) {
    if (m < 1 || m > kRankMaxCols) return 0;
    return ranked_layout(n, m, W).bytes;
}

hipError_t launch_index_build_ranked(const float *a, int64_t n, int64_t npad, int32_t m,
                                     int64_t W, int64_t wpad, uint64_t *idx, uint8_t *tie,
                                     int32_t *any_tie, uint32_t *tbits, void *scratch,
                                     hipStream_t stream) {
    if (m < 1 || m > kRankMaxCols || !scratch) return hipErrorInvalidValue;
    const RankedLayout L = ranked_layout(n, m, W);
    char *base = static_cast<char *>(scratch);
    uint32_t *wflag = reinterpret_cast<uint32_t *>(base);
    uint16_t *rank = reinterpret_cast<uint16_t *>(base + L.off_rank);
    uint64_t *planes = reinterpret_cast<uint64_t *>(base + L.off_planes);

    const int64_t flags = (int64_t)m * m;
    int64_t fill = flags > kTieWords ? flags : kTieWords;
    fill = fill > L.wq ? fill : L.wq;
    hipLaunchKernelGGL(index_init_kernel, dim3((unsigned)((fill + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, stream, tie, m, flags, any_tie, tbits, wflag, L.wq);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (L.logm) {
    case 4: e = launch_rank<4>(a, n, npad, m, rank, L.mr, wflag, stream); break;
    case 5: e = launch_rank<5>(a, n, npad, m, rank, L.mr, wflag, stream); break;
    case 6: e = launch_rank<6>(a, n, npad, m, rank, L.mr, wflag, stream); break;
    case 7: e = launch_rank<7>(a, n, npad, m, rank, L.mr, wflag, stream); break;
    case 8: e = launch_rank<8>(a, n, npad, m, rank, L.mr, wflag, stream); break;
    case 9: e = launch_rank<9>(a, n, npad, m, rank, L.mr, wflag, stream); break;
    case 10: e = launch_rank<10>(a, n, npad, m, rank, L.mr, wflag, stream); break;
    case 11: e = launch_rank<11>(a, n, npad, m, rank, L.mr, wflag, stream); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    switch (L.nb) {
    case 4: return launch_planes_compare<4>(rank, wflag, n, m, L.mr, W, L.wq, wpad, planes, idx,
                                            tie, any_tie, tbits, stream);
    case 6: return launch_planes_compare<6>(rank, wflag, n, m, L.mr, W, L.wq, wpad, planes, idx,
                                            tie, any_tie, tbits, stream);
    case 8: return launch_planes_compare<8>(rank, wflag, n, m, L.mr, W, L.wq, wpad, planes, idx,
                                            tie, any_tie, tbits, stream);
    case 10: return launch_planes_compare<10>(rank, wflag, n, m, L.mr, W, L.wq, wpad, planes,
                                              idx, tie, any_tie, tbits, stream);
    case 12: return launch_planes_compare<12>(rank, wflag, n, m, L.mr, W, L.wq, wpad, planes,
                                              idx, tie, any_tie, tbits, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ebic
