// Device-side Steps 1-3 and 5 of EBIC's evolutionary run (Section 2.2), for
// batched runs: one workgroup of one wave per run keeps the run's random
// stream, tabu list, top-rank list and column penalties in device memory,
// so that a generation is two launches -- this kernel, then the batched
// evaluation (Step 4) -- with no host round trip.
//
// The readings are those of the host implementation (ebic_run.h) and give
// the same run draw for draw:
//   * SplitMix64; a draw in [0, n) is next() % n.  The wave holds a window
//     of the next 64 outputs, one per lane (output k of a window starting at
//     state s is mix(s + k * gamma)), so several draws are reduced modulo
//     their bounds in parallel and consumed in order.
//   * Step 3 tournament: T draws with replacement from the previous
//     population; adjusted quality fitness / base^(penalty sum / L), with
//     base^(s/L) read from a table the host fills with std::pow (the same
//     doubles the host path uses); the first strictly best draw wins.
//   * Step 5: members by decreasing fitness (stable), positive fitness and
//     not yet listed, admitted unless a listed entry of at least equal
//     fitness overlaps them by more than theta; an admitted member evicts
//     weaker entries it overlaps by more than theta; stable sort, cut to K.
//     The pass stops once K live entries have fitness >= f(x): no later
//     member can change the first K.
// The tabu list is an open-addressing hash table of 16-byte slots over an
// arena of the listed series (exact comparison).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ebic_internal.h"

namespace ebic {
namespace {

constexpr int kLanes = 64;
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
enum { OP_INSERT = 0, OP_DELETE, OP_SWAP, OP_SUBSTITUTE, OP_CROSSOVER };

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int lane_id() { return (int)threadIdx.x; }

// The workgroup is one wave: its LDS operations are performed in program
// order, so lanes only need the compiler not to move memory operations
// across this point (no s_barrier, and no wait for outstanding global
// stores as a workgroup barrier's fence would do).
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

__device__ __forceinline__ int32_t rl32(int32_t v, int lane) {
    return __builtin_amdgcn_readlane(v, lane);
}
__device__ __forceinline__ uint64_t rl64(uint64_t v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double rlf64(double v, int lane) {
    return __longlong_as_double((long long)rl64((uint64_t)__double_as_longlong(v), lane));
}

// x % n.  For n < 2^16 the 64-bit value is reduced Horner-style in 16-bit
// digits with three 32-bit remainders (each partial value stays below
// 2^32), much shorter than a 64-bit division.
__device__ __forceinline__ uint32_t mod_u64(uint64_t x, uint32_t n) {
    if (n <= 0xFFFFu) {
        uint32_t r = (uint32_t)(x >> 32) % n;
        r = ((r << 16) | (uint32_t)((x >> 16) & 0xFFFFu)) % n;
        return ((r << 16) | (uint32_t)(x & 0xFFFFu)) % n;
    }
    return (uint32_t)(x % (uint64_t)n);
}

// A window of the next 64 SplitMix64 outputs: lane i holds output used+1+i
// relative to `base` (which already excludes the consumed ones); uniform
// `used` counts the outputs consumed from the window.
struct Draws {
    uint64_t base;   // generator state at the window start
    uint64_t raw;    // this lane's output: mix(base + (lane + 1) * gamma)
    int used;
    // this lane's output reduced modulo the run's fixed bounds (the
    // population size, the operation weight sum and the column count),
    // computed once per window
    uint32_t nP, nW, nM;
    uint32_t modP, modW, modM;

    __device__ void fill() {
        raw = mix64(base + (uint64_t)(lane_id() + 1) * kGamma);
        modP = mod_u64(raw, nP);
        modW = mod_u64(raw, nW);
        modM = mod_u64(raw, nM);
    }
    __device__ void start(uint64_t state, uint32_t P, uint32_t W, uint32_t M) {
        base = state;
        used = 0;
        nP = P;
        nW = W;
        nM = M;
        fill();
    }
    // At least n (<= 64) unconsumed outputs in the window.
    __device__ void need(int n) {
        if (used + n > kLanes) {
            base += (uint64_t)used * kGamma;
            used = 0;
            fill();
        }
    }
    __device__ uint64_t state() const { return base + (uint64_t)used * kGamma; }
    // Unconsumed output k (uniform k, used + k < 64).
    __device__ uint64_t at(int k) const { return rl64(raw, used + k); }
    __device__ uint32_t below(uint32_t n) {
        need(1);
        const uint64_t r = at(0);
        ++used;
        return mod_u64(r, n);
    }
    // A draw in [0, M) (the column count).
    __device__ uint32_t below_m() {
        need(1);
        return (uint32_t)rl32((int32_t)modM, used++);
    }
};

// LDS layout of one run (byte offsets; every array 16-byte aligned).
struct Lds {
    uint16_t *pcols;    // previous population, P * slot
    uint8_t *plen;      // P
    double *pfit;       // P
    int32_t *pcnt;      // P
    uint32_t *pen;      // m column penalties
    uint16_t *order;    // P2 member indices by decreasing fitness
    uint16_t *ecols;    // E * slot top-rank entries (old list, then admitted members)
    uint8_t *elen;      // E
    uint8_t *ealive;    // E
    double *efit;       // E
    int32_t *ecnt;      // E
    uint16_t *erank;    // K: entry at each rank of the updated list
    uint64_t *colmask;  // m * EW: bit e of column c's words when entry e holds c
    int32_t *cbuf;      // 64: crossover scratch
    uint32_t *tsum;     // 64: tournament penalty sums
};

__host__ __device__ inline int64_t align16(int64_t x) { return (x + 15) & ~int64_t(15); }

struct LdsShape {
    int32_t P, P2, slot, pstride, m, K, E, EW;
    int64_t off[15];
    int64_t total;
};

__host__ __device__ inline LdsShape lds_shape(int32_t P, int32_t slot, int32_t m, int32_t K) {
    LdsShape s{};
    s.P = P;
    s.P2 = 1;
    while (s.P2 < P) s.P2 <<= 1;
    s.slot = slot;
    s.pstride = (slot + 1) & ~1;   // even: a series row is whole dwords
    s.m = m;
    s.K = K;
    s.E = 2 * K;
    s.EW = (s.E + 63) / 64;
    const int64_t sizes[15] = {
        (int64_t)P * s.pstride * 2, P, (int64_t)P * 8, (int64_t)P * 4, (int64_t)m * 4,
        (int64_t)s.P2 * 2, (int64_t)s.E * slot * 2, s.E, s.E, (int64_t)s.E * 8,
        (int64_t)s.E * 4, (int64_t)K * 2, (int64_t)m * s.EW * 8, 64 * 4, 64 * 4};
    int64_t at = 0;
    for (int i = 0; i < 15; ++i) {
        s.off[i] = at;
        at = align16(at + sizes[i]);
    }
    s.total = at;
    return s;
}

__device__ inline Lds lds_map(unsigned char *base, const LdsShape &s) {
    Lds L;
    L.pcols = (uint16_t *)(base + s.off[0]);
    L.plen = (uint8_t *)(base + s.off[1]);
    L.pfit = (double *)(base + s.off[2]);
    L.pcnt = (int32_t *)(base + s.off[3]);
    L.pen = (uint32_t *)(base + s.off[4]);
    L.order = (uint16_t *)(base + s.off[5]);
    L.ecols = (uint16_t *)(base + s.off[6]);
    L.elen = (uint8_t *)(base + s.off[7]);
    L.ealive = (uint8_t *)(base + s.off[8]);
    L.efit = (double *)(base + s.off[9]);
    L.ecnt = (int32_t *)(base + s.off[10]);
    L.erank = (uint16_t *)(base + s.off[11]);
    L.colmask = (uint64_t *)(base + s.off[12]);
    L.cbuf = (int32_t *)(base + s.off[13]);
    L.tsum = (uint32_t *)(base + s.off[14]);
    return L;
}

// Whether the series in lanes [0, L) (ch) holds column c, per lane's c.
__device__ __forceinline__ bool series_has(int32_t ch, int32_t L, int32_t c) {
    bool in = false;
    for (int32_t t = 0; t < L; ++t) in |= (c == rl32(ch, t));
    return in;
}

// A column not in the series ch[0, L): draws c = next() % M until one is
// new.  Usually the first draw is (L < M), so draws are tested one at a
// time, each against every lane of the series at once.
__device__ int32_t new_column(Draws &d, int32_t ch, int32_t L, int32_t M) {
    const int lane = lane_id();
    for (;;) {
        const int32_t c = (int32_t)d.below_m();
        if (__ballot(lane < L && ch == c) == 0ull) return c;
    }
}

// XOR of x over the wave's 64 lanes: DPP exchanges inside each row of 16
// lanes (adjacent lanes, lane pairs, half-row mirror, row mirror), then the
// four row values.
__device__ __forceinline__ uint32_t wave_xor(uint32_t x) {
    x ^= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xb1, 0xf, 0xf, false);   // quad_perm 1,0,3,2
    x ^= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4e, 0xf, 0xf, false);   // quad_perm 2,3,0,1
    x ^= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x141, 0xf, 0xf, false);  // row_half_mirror
    x ^= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x140, 0xf, 0xf, false);  // row_mirror
    return (uint32_t)(rl32((int32_t)x, 0) ^ rl32((int32_t)x, 16) ^ rl32((int32_t)x, 32) ^
                      rl32((int32_t)x, 48));
}

// Tabu list: open addressing with linear probing over 16-byte slots {tag
// (two dwords, never 0 when used), arena offset, length}; the series
// themselves are appended to the run's arena (16-bit columns).  A probe
// reads 8 consecutive slots at once (one lane each); a tag match is
// confirmed against the stored series, so membership is exact.  Inserts
// the series ch[0, L) and returns true, or returns false if it is already
// listed.  *full is set when the table or the arena has no room left.
__device__ bool tabu_insert(const StepsRun &R, int64_t &arena_used, int32_t ch, int32_t L,
                            bool *full) {
    const int lane = lane_id();
    const uint64_t v = lane < L ? mix64(((uint64_t)(uint32_t)ch << 8) ^ (uint64_t)lane ^
                                        ((uint64_t)L << 40) ^ 0x5851F42D4C957F2Dull)
                                : 0ull;
    const uint64_t h = ((uint64_t)wave_xor((uint32_t)(v >> 32)) << 32) | wave_xor((uint32_t)v);
    const uint64_t tag = mix64(h) | 1ull;
    const uint32_t tlo = (uint32_t)tag, thi = (uint32_t)(tag >> 32);
    const uint64_t mask = R.tabu_cap - 1;
    uint64_t s0 = (tag >> 1) & mask;
    for (uint64_t seen = 0; seen < R.tabu_cap;) {
        const uint64_t my = (s0 + (uint64_t)lane) & mask;
        uint4 w = make_uint4(0u, 0u, 0u, 0u);
        if (lane < 8) w = reinterpret_cast<const uint4 *>(R.tabu)[my];
        const bool empty = w.x == 0u;
        const bool match = w.x == tlo && w.y == thi && (int32_t)w.w == L;
        const uint64_t hit = __ballot(lane < 8 && (empty || match));
        if (hit == 0ull) {
            s0 = (s0 + 8) & mask;
            seen += 8;
            continue;
        }
        const int f = __ffsll((unsigned long long)hit) - 1;
        if (rl32((int32_t)w.x, f) == 0) {      // an empty slot first: the series is new
            if (arena_used + L > R.arena_cap) break;
            if (lane == f)
                reinterpret_cast<uint4 *>(R.tabu)[my] =
                    make_uint4(tlo, thi, (uint32_t)arena_used, (uint32_t)L);
            if (lane < L) R.arena[arena_used + lane] = (uint16_t)ch;
            arena_used += L;
            return true;
        }
        // tag and length match: compare the stored series
        const uint32_t at = (uint32_t)rl32((int32_t)w.z, f);
        const bool same = __ballot(lane < L && (int32_t)R.arena[at + lane] != ch) == 0ull;
        if (same) return false;
        s0 = (s0 + (uint64_t)f + 1) & mask;
        seen += (uint64_t)f + 1;
    }
    *full = true;
    return false;
}

// Tournament draws: lane t < nsets*T takes output used + set*(T+1) + j of
// the window (set = t / T, j = t % T) and computes its member and adjusted
// quality.  The penalty sums of all draws are gathered at once: lane g of
// a grid over (draw, dword of the draw's series row, two columns per
// dword) adds its columns' penalties into the draw's LDS sum.
__device__ void tournament_lanes(const Draws &d, int nsets, int T, int32_t P, const Lds &S,
                                 int32_t pstride, const double *__restrict__ powtab,
                                 int32_t &idx, double &adj) {
    const int lane = lane_id();
    const int set = lane / T, j = lane - set * T;
    const int nd = nsets * T;
    const bool act = set < nsets;
    const int32_t mp = __shfl((int32_t)d.modP, act ? d.used + set * (T + 1) + j : 0);
    idx = act ? mp : 0;
    const int32_t L = act ? (int32_t)S.plen[idx] : 0;
    if (lane < nd) S.tsum[lane] = 0u;
    wave_sync();
    const int dw = pstride / 2;                  // dwords per series row
    for (int base = 0; base < nd * dw; base += kLanes) {
        const int g = base + lane;
        const int dd = g / dw, q = g - dd * dw;
        const int32_t id = __shfl(idx, min(dd, kLanes - 1));
        const int32_t Ld = __shfl(L, min(dd, kLanes - 1));
        if (dd < nd && 2 * q < Ld) {
            const uint32_t w =
                reinterpret_cast<const uint32_t *>(S.pcols + (int64_t)id * pstride)[q];
            uint32_t sum = S.pen[w & 0xFFFFu];
            if (2 * q + 1 < Ld) sum += S.pen[w >> 16];
            atomicAdd(&S.tsum[dd], sum);
        }
    }
    wave_sync();
    adj = -INFINITY;
    if (act) {
        const int64_t sum = S.tsum[lane];
        const double pw = powtab[(int64_t)P * L * (L - 1) / 2 + (L - 1) + sum];
        adj = S.pfit[idx] / pw;
    }
}

// The first strictly best draw among lanes [first, first + T): the lane
// whose quality beats every earlier draw and is at least every later one
// (all lanes test this at once).
__device__ int32_t tournament_winner(int32_t idx, double adj, int first, int T) {
    const int lane = lane_id();
    const int t = lane - first;
    bool win = t >= 0 && t < T;
    for (int j = 0; j < T; ++j) {
        const double a = rlf64(adj, first + j);
        win &= j < t ? adj > a : (j > t ? adj >= a : true);
    }
    const uint64_t b = __ballot(win);
    return rl32(idx, __ffsll((unsigned long long)b) - 1);
}

// Appends the series ch[0, L) as member n of the run's new population.
__device__ __forceinline__ void put_member(const StepsRun &R, int32_t n, int64_t &cur, int32_t ch,
                                           int32_t L) {
    const int lane = lane_id();
    if (lane < L) R.cols[cur + lane] = ch;
    if (lane == 0) R.off[n] = (int32_t)(R.col_base + cur);
    cur += L;
}

// Step 5 over the population in LDS; leaves the updated list in global
// memory and its ranks in S.erank.  Returns the list size.
__device__ int32_t step5(const StepsArgs &A, const StepsRun &R, const Lds &S, const LdsShape &sh,
                         int32_t n_old) {
    const int lane = lane_id();
    const int32_t P = A.P, slot = A.slot, K = A.K, EW = sh.EW, m = R.m;
    // members by decreasing fitness, ties by position (bitonic sort)
    auto before = [&](int32_t a, int32_t b) -> bool {
        if (a >= P) return false;
        if (b >= P) return true;
        const double fa = S.pfit[a], fb = S.pfit[b];
        return fa > fb || (fa == fb && a < b);
    };
    for (int32_t i = lane; i < sh.P2; i += kLanes) S.order[i] = (uint16_t)i;
    wave_sync();
    for (int32_t k = 2; k <= sh.P2; k <<= 1)
        for (int32_t j = k >> 1; j > 0; j >>= 1) {
            for (int32_t i = lane; i < sh.P2; i += kLanes) {
                const int32_t ixj = i ^ j;
                if (ixj > i) {
                    const int32_t a = S.order[i], b = S.order[ixj];
                    const bool sw = (i & k) == 0 ? before(b, a) : before(a, b);
                    if (sw) {
                        S.order[i] = (uint16_t)b;
                        S.order[ixj] = (uint16_t)a;
                    }
                }
            }
            wave_sync();
        }
    // the old list (sorted by decreasing fitness) and its column index
    for (int64_t i = lane; i < (int64_t)m * EW; i += kLanes) S.colmask[i] = 0ull;
    for (int32_t e = lane; e < n_old; e += kLanes) {
        const int32_t le = R.top_len[e];
        S.elen[e] = (uint8_t)le;
        S.efit[e] = R.top_fit[e];
        S.ecnt[e] = R.top_cnt[e];
        S.ealive[e] = 1;
        for (int32_t t = 0; t < le; ++t) S.ecols[e * slot + t] = (uint16_t)R.top_cols[e * slot + t];
    }
    wave_sync();
    for (int32_t e = lane; e < n_old; e += kLanes)
        for (int32_t t = 0; t < S.elen[e]; ++t)
            atomicOr((unsigned long long *)&S.colmask[(int64_t)S.ecols[e * slot + t] * EW + e / 64],
                     1ull << (e % 64));
    wave_sync();

    int32_t n_ent = n_old, settled = 0, old_ptr = 0;
    for (int32_t ii = 0; ii < P; ++ii) {
        const int32_t i = S.order[ii];
        const double fx = S.pfit[i];
        if (!(fx > 0.0)) break;
        for (; old_ptr < n_old && S.efit[old_ptr] >= fx; ++old_ptr) settled += S.ealive[old_ptr];
        if (settled >= K) break;
        const int32_t lx = S.plen[i];
        const int32_t xc = lane < lx ? (int32_t)S.pcols[i * sh.pstride + lane] : -1;
        // per entry: intersection with x, listed (same series), overlap
        auto entry = [&](int32_t e, bool &listed, bool &over) -> bool {
            int32_t inter = 0;
#pragma unroll 8
            for (int32_t t = 0; t < lx; ++t) {
                const int32_t c = rl32(xc, t);
                inter += (int32_t)((S.colmask[(int64_t)c * EW + e / 64] >> (e % 64)) & 1ull);
            }
            const int32_t le = S.elen[e];
            listed = false;
            if (inter == lx && le == lx) {
                listed = true;
                for (int32_t t = 0; t < lx; ++t) listed &= (int32_t)S.ecols[e * slot + t] == rl32(xc, t);
            }
            const double ov = (double)inter / (double)min(lx, le);
            over = ov > A.theta;
            return true;
        };
        bool listed = false, blocked = false;
        for (int32_t e0 = 0; e0 < n_ent; e0 += kLanes) {
            const int32_t e = e0 + lane;
            bool l = false, blk = false;
            if (e < n_ent && S.ealive[e]) {
                bool o = false;
                entry(e, l, o);
                blk = o && S.efit[e] >= fx;
            }
            listed |= __ballot(l) != 0ull;
            blocked |= __ballot(blk) != 0ull;
        }
        if (!listed && !blocked) {
            for (int32_t e0 = 0; e0 < n_ent; e0 += kLanes) {
                const int32_t e = e0 + lane;
                if (e < n_ent && S.ealive[e]) {
                    bool l = false, o = false;
                    entry(e, l, o);
                    if (o && S.efit[e] < fx) S.ealive[e] = 0;
                }
            }
            const int32_t ne = n_ent++;
            if (lane < lx) {
                S.ecols[ne * slot + lane] = (uint16_t)xc;
                atomicOr((unsigned long long *)&S.colmask[(int64_t)xc * EW + ne / 64],
                         1ull << (ne % 64));
            }
            if (lane == 0) {
                S.elen[ne] = (uint8_t)lx;
                S.efit[ne] = fx;
                S.ecnt[ne] = S.pcnt[i];
                S.ealive[ne] = 1;
            }
            ++settled;
        }
        wave_sync();
    }
    // live entries in insertion order, stable by decreasing fitness, first K
    int32_t live = 0;
    for (int32_t e0 = 0; e0 < n_ent; e0 += kLanes) {
        const int32_t e = e0 + lane;
        bool act = false;
        if (e < n_ent) act = S.ealive[e] != 0;
        live += __popcll(__ballot(act));
        if (act) {
            const double f = S.efit[e];
            int32_t rank = 0;
            for (int32_t x = 0; x < n_ent; ++x)
                if (S.ealive[x] && (S.efit[x] > f || (S.efit[x] == f && x < e))) ++rank;
            if (rank < K) S.erank[rank] = (uint16_t)e;
        }
    }
    wave_sync();
    const int32_t n_top = min(live, K);
    for (int32_t r = lane; r < n_top; r += kLanes) {
        const int32_t e = S.erank[r];
        const int32_t le = S.elen[e];
        R.top_len[r] = le;
        R.top_fit[r] = S.efit[e];
        R.top_cnt[r] = S.ecnt[e];
        for (int32_t t = 0; t < le; ++t) R.top_cols[r * slot + t] = S.ecols[e * slot + t];
    }
    return n_top;
}

__global__ __launch_bounds__(kLanes) void evolve_steps_kernel(StepsArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = lane_id();
    const StepsRun R = A.runs[blockIdx.x];
    StepsState st = *R.state;
    if (st.stopped || st.error) return;
    const int32_t P = A.P, slot = A.slot, M = R.m;
    const LdsShape sh = lds_shape(P, slot, M, A.K);
    const Lds S = lds_map(smem, sh);
    Draws d;
    d.start(st.rng, (uint32_t)P, (uint32_t)A.wsum, (uint32_t)M);
    bool full = false;

    if (A.mode == 0) {
        // Step 1: P distinct random series
        int64_t cur = 0;
        for (int32_t n = 0; n < P;) {
            const int32_t L = A.len_min + (int32_t)d.below((uint32_t)(A.len_max - A.len_min + 1));
            int32_t ch = -1;
            for (int32_t k = 0; k < L; ++k) {
                const int32_t c = new_column(d, ch, k, M);
                if (lane == k) ch = c;
            }
            if (!tabu_insert(R, st.arena_used, ch, L, &full)) {
                if (full) break;
                continue;
            }
            put_member(R, n, cur, ch, L);
            ++n;
        }
        if (lane == 0) R.off[P] = (int32_t)(R.col_base + cur);
        st.first_new = 0;
        st.gen = 0;
    } else {
        // the evaluated population into LDS
        for (int32_t i = lane; i < P; i += kLanes) {
            const int32_t o = R.off[i];
            const int32_t L = R.off[i + 1] - o;
            S.plen[i] = (uint8_t)L;
            S.pfit[i] = R.fit[i];
            S.pcnt[i] = R.counts[i];
            const int32_t *src = R.cols + (o - R.col_base);
            for (int32_t t = 0; t < L; ++t) S.pcols[i * sh.pstride + t] = (uint16_t)src[t];
        }
        wave_sync();
        // Step 5 with the population of generation st.gen
        st.n_top = step5(A, R, S, sh, st.n_top);
        if (st.gen > 0) st.gens_run = st.gen;
        wave_sync();
        if (A.mode == 1) {
            // Step 2: elites and their penalties
            for (int32_t c = lane; c < M; c += kLanes) S.pen[c] = 0u;
            wave_sync();
            const int32_t n_e = (int32_t)min<int64_t>(
                (int64_t)st.n_top, (int64_t)P * A.elite_num / A.elite_den);
            int64_t cur = 0;
            for (int32_t e = 0; e < n_e; ++e) {
                const int32_t id = S.erank[e];
                const int32_t L = S.elen[id];
                const int32_t ch = lane < L ? (int32_t)S.ecols[id * slot + lane] : -1;
                if (lane < L) atomicAdd(&S.pen[ch], 1u);
                put_member(R, e, cur, ch, L);
            }
            wave_sync();
            // Step 3: novel children until the population is full
            const int T = A.tournament;
            int32_t n = n_e, hits = 0;
            while (n < P) {
                d.need(2 * T + 1);
                const uint32_t u = (uint32_t)rl32((int32_t)d.modW, d.used + T);
                int op = 0;
                int64_t acc = 0;
                for (op = 0; op < 5; ++op) {
                    acc += A.op_weight[op];
                    if ((int64_t)u < acc) break;
                }
                const int nsets = op == OP_CROSSOVER ? 2 : 1;
                int32_t idx;
                double adj;
                tournament_lanes(d, nsets, T, P, S, sh.pstride, A.powtab, idx, adj);
                const int32_t ia = tournament_winner(idx, adj, 0, T);
                const int32_t ib = nsets == 2 ? tournament_winner(idx, adj, T, T) : ia;
                d.used += nsets * (T + 1) - (nsets == 2 ? 1 : 0);
                const int32_t la = S.plen[ia];
                int32_t ch = lane < la ? (int32_t)S.pcols[ia * sh.pstride + lane] : -1;
                int32_t L = la;
                switch (op) {
                case OP_INSERT:
                    if (L < A.len_max) {
                        const int32_t pos = (int32_t)d.below((uint32_t)L + 1);
                        const int32_t c = new_column(d, ch, L, M);
                        const int32_t left = __shfl(ch, max(lane - 1, 0));
                        ch = lane < pos ? ch : (lane == pos ? c : left);
                        ++L;
                    }
                    break;
                case OP_DELETE:
                    if (L > A.len_min) {
                        const int32_t pos = (int32_t)d.below((uint32_t)L);
                        const int32_t right = __shfl(ch, min(lane + 1, kLanes - 1));
                        if (lane >= pos) ch = right;
                        --L;
                    }
                    break;
                case OP_SWAP:
                    if (L >= 2) {
                        const int32_t i = (int32_t)d.below((uint32_t)L);
                        int32_t j = (int32_t)d.below((uint32_t)L - 1);
                        if (j >= i) ++j;
                        const int32_t ci = rl32(ch, i), cj = rl32(ch, j);
                        if (lane == i) ch = cj;
                        if (lane == j) ch = ci;
                    }
                    break;
                case OP_SUBSTITUTE:
                    if (L < M) {
                        const int32_t pos = (int32_t)d.below((uint32_t)L);
                        const int32_t c = new_column(d, ch, L, M);
                        if (lane == pos) ch = c;
                    }
                    break;
                default: {   // one-point crossover of Fig. 1e
                    const int32_t lb = S.plen[ib];
                    const int32_t b = lane < lb ? (int32_t)S.pcols[ib * sh.pstride + lane] : -1;
                    const int32_t i = 1 + (int32_t)d.below((uint32_t)la);
                    const int32_t j = (int32_t)d.below((uint32_t)lb);
                    const bool keep = lane >= j && lane < lb && !series_has(ch, i, b);
                    const uint64_t km = __ballot(keep);
                    const int32_t rank = __popcll(km & ((1ull << lane) - 1ull));
                    const int32_t n_c = min(i + __popcll(km), A.len_max);
                    S.cbuf[lane] = lane < i ? ch : -1;
                    wave_sync();
                    if (keep && i + rank < A.len_max) S.cbuf[i + rank] = b;
                    wave_sync();
                    if (n_c >= A.len_min) {
                        ch = S.cbuf[lane];
                        L = n_c;
                    }
                    wave_sync();
                    break;
                }
                }
                if (lane >= L) ch = -1;
                if (!tabu_insert(R, st.arena_used, ch, L, &full)) {
                    if (full) break;
                    if (++hits > A.tabu_limit) {
                        st.stopped = 1;
                        break;
                    }
                    continue;
                }
                if (lane < L) atomicAdd(&S.pen[ch], 1u);
                put_member(R, n, cur, ch, L);
                ++n;
                wave_sync();
            }
            // a stopped run leaves empty members behind (never read)
            for (int32_t i = n + lane; i <= P; i += kLanes) R.off[i] = (int32_t)(R.col_base + cur);
            st.first_new = n_e;
            ++st.gen;
        }
    }
    if (full) st.error = 1;
    st.rng = d.state();
    if (lane == 0) *R.state = st;
}

}  // namespace

int64_t steps_lds_bytes(int32_t P, int32_t slot, int32_t m, int32_t K) {
    return lds_shape(P, slot, m, K).total;
}

hipError_t launch_steps(const StepsArgs &a, hipStream_t stream) {
    // (dynamic LDS above 64 KiB; a runtime without the attribute fails the
    // launch itself if the size is not allowed)
    if (hipFuncSetAttribute((const void *)evolve_steps_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, a.lds_bytes) != hipSuccess)
        (void)hipGetLastError();
    hipLaunchKernelGGL(evolve_steps_kernel, dim3((unsigned)a.n_runs), dim3(kLanes),
                       (unsigned)a.lds_bytes, stream, a);
    return hipGetLastError();
}

}  // namespace ebic
