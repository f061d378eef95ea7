// Fused training step of the surrogate MLP for embed_dim 32 and hidden 256
// (the configuration of the screened runs) on gfx950:
//
//   A  mlp_rows_kernel    per tile of 32 candidates: pooling, both layers,
//                         the output, the loss gradient and the whole
//                         per-candidate backward pass (dz2, dz1, dx), with
//                         the tile's activations kept in LDS; writes the
//                         BF16 operands of the weight gradients transposed
//                         (feature-major, candidates contiguous) and each
//                         tile's partial bias/output-weight gradient sums
//   B  mlp_grads_kernel   weight gradients as split-K products over the
//                         batch (one partial per 256 candidates), the bias
//                         and output-weight gradients from the tiles'
//                         partial sums, and the embedding gradients gathered
//                         by column occurrence and by series length
//   C  mlp_update_kernel  every parameter: its gradient (partials summed in
//                         a fixed order), then Adam, then the BF16 copies
//                         (row-major and transposed) of W1, W2 and w3
//
// Products run on v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32
// accumulation) with 16-byte operand fragments: A and B lane l holds row or
// column (l mod 16) and 8 consecutive k from 8 (l / 16); the 16 x 16 result
// gives lane l rows 4 (l / 16) + v, column l mod 16.  The rounding points
// are those of the layer-by-layer kernels: bf16(x), bf16(relu(z1)),
// bf16(relu(z2)), bf16(dz2), bf16(dz1), weights read as BF16 copies.  Every
// sum has a fixed order, so a step is deterministic on one device.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ebic_mlp.h"

namespace ebic {
namespace mlp {
namespace {

constexpr int kBlock = 256;
constexpr int kTB = 32;                // candidates per row tile
constexpr int kD = 32, kD2 = 64, kH = 256;
constexpr int kLdX = kD2 + 8, kLdH = kH + 8;   // LDS row strides (bf16), 16-byte aligned rows
constexpr int kChunk = 256;            // candidates per weight-gradient partial

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// 16 x 32 fragment of a row-major BF16 matrix (row stride ld elements):
// rows r0 + (lane mod 16), columns k0 + 8 (lane / 16) .. + 7.
__device__ __forceinline__ bf16x8 frag(const uint16_t *base, int64_t ld, int64_t r0, int64_t k0,
                                      int lane) {
    return *reinterpret_cast<const bf16x8 *>(base + (r0 + (lane & 15)) * ld + k0 + 8 * (lane >> 4));
}

// Sum over the four lane groups (l, l+16, l+32, l+48) in a fixed order.
__device__ __forceinline__ float sum_groups(float v) {
    const float a = v + __shfl_xor(v, 16);
    return a + __shfl_xor(a, 32);
}
// Sum over the 16 lanes of a group in a fixed order.
__device__ __forceinline__ float sum_row(float v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    return v + __shfl_xor(v, 8);
}

constexpr int kTileCols = 2048;        // series entries of a tile staged in LDS

struct RowsLds {
    int32_t off[kTB + 1];
    int32_t cols[kTileCols];
    uint16_t x[kTB][kLdX];
    uint16_t h1[kTB][kLdH];
    uint16_t dz2[kTB][kLdH];
    uint16_t dz1[kTB][kLdH];
    uint8_t m1[kTB][kH];
    float yp[4][kTB];
    float dy[kTB];
};

// Copies a [32][W] LDS tile to a feature-major global matrix dst[W][Bp]
// (columns b0 .. b0 + 31), 16 bytes per store.
template <int W, int LD>
__device__ __forceinline__ void store_transposed(const uint16_t (*src)[LD], uint16_t *dst,
                                                 int64_t Bp, int64_t b0) {
    for (int i = threadIdx.x; i < W * (kTB / 8); i += kBlock) {
        const int w = i / (kTB / 8), c = i % (kTB / 8);
        uint16_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = src[c * 8 + j][w];
        uint4 q;
        q.x = v[0] | ((uint32_t)v[1] << 16);
        q.y = v[2] | ((uint32_t)v[3] << 16);
        q.z = v[4] | ((uint32_t)v[5] << 16);
        q.w = v[6] | ((uint32_t)v[7] << 16);
        *reinterpret_cast<uint4 *>(dst + (int64_t)w * Bp + b0 + c * 8) = q;
    }
}

__global__ __launch_bounds__(kBlock) void mlp_rows_kernel(FusedRows a) {
    __shared__ RowsLds S;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t b0 = (int64_t)blockIdx.x * kTB;

    // pooling: x = [mean E + Z[L] ; mean of F[c_t] * T[c_{t+1}]], bf16(x).
    // The tile's series are staged in LDS.
    if (tid <= kTB) {
        const int64_t b = b0 + tid;
        S.off[tid] = b <= a.B ? a.off[b] : a.off[a.B];
    }
    __syncthreads();
    const int32_t base = S.off[0], n_cols = S.off[kTB] - base;
    for (int i = tid; i < n_cols && i < kTileCols; i += kBlock) S.cols[i] = a.cols[base + i];
    __syncthreads();
    {
        // thread = (candidate r, 8 consecutive dimensions 8q .. 8q + 7 of x):
        // q < 4 pools E, q >= 4 the pair products F * T; four series
        // positions' loads in flight at a time, sums in series order
        const int r = tid / 8, q = tid % 8;
        const bool pair = q >= kD / 8;
        const int d0 = 8 * (pair ? q - kD / 8 : q);
        const int32_t s = S.off[r], e = S.off[r + 1], L = e - s;
        const bool staged = n_cols <= kTileCols;
        auto col = [&](int32_t t) -> int32_t { return staged ? S.cols[t - base] : a.cols[t]; };
        float acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = 0.f;
        const int32_t n_terms = pair ? L - 1 : L;
        for (int32_t t0 = 0; t0 < n_terms; t0 += 4) {
            float4 v[4][2];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int32_t t = t0 + j;
                v[j][0] = v[j][1] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (t < n_terms) {
                    const int32_t c = col(s + t);
                    if (!pair) {
                        const float4 *er = reinterpret_cast<const float4 *>(a.E + (int64_t)c * kD + d0);
                        v[j][0] = er[0];
                        v[j][1] = er[1];
                    } else {
                        const int32_t c2 = col(s + t + 1);
                        const float4 *fr = reinterpret_cast<const float4 *>(a.F + (int64_t)c * kD + d0);
                        const float4 *tr = reinterpret_cast<const float4 *>(a.T + (int64_t)c2 * kD + d0);
                        const float4 f0 = fr[0], f1 = fr[1], u0 = tr[0], u1 = tr[1];
                        v[j][0] = make_float4(f0.x * u0.x, f0.y * u0.y, f0.z * u0.z, f0.w * u0.w);
                        v[j][1] = make_float4(f1.x * u1.x, f1.y * u1.y, f1.z * u1.z, f1.w * u1.w);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc[0] += v[j][0].x;
                acc[1] += v[j][0].y;
                acc[2] += v[j][0].z;
                acc[3] += v[j][0].w;
                acc[4] += v[j][1].x;
                acc[5] += v[j][1].y;
                acc[6] += v[j][1].z;
                acc[7] += v[j][1].w;
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            float x = 0.f;
            if (b0 + r < a.B) {
                if (!pair) x = acc[u] / (float)L + a.Zl[(int64_t)L * kD + d0 + u];
                else if (L > 1) x = acc[u] / (float)(L - 1);
            }
            S.x[r][(pair ? kD : 0) + d0 + u] = to_bf16(x);
        }
    }
    __syncthreads();

    // layer 1: z1 = bf16(x) W1^T + b1 (wave wv: columns 64 wv .. 64 wv + 63)
    {
        f32x4 acc[2][4] = {};
#pragma unroll
        for (int k0 = 0; k0 < kD2; k0 += 32) {
            bf16x8 fa[2], fb[4];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) fa[rb] = frag(&S.x[0][0], kLdX, 16 * rb, k0, lane);
#pragma unroll
            for (int c = 0; c < 4; ++c) fb[c] = frag(a.W1b, kD2, 64 * wv + 16 * c, k0, lane);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[rb][c] = mfma(fa[rb], fb[c], acc[rb][c]);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int n = 64 * wv + 16 * c + (lane & 15);
            const float bias = a.b1[n];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rb + 4 * (lane >> 4) + v;
                    const float z = acc[rb][c][v] + bias;
                    S.h1[r][n] = to_bf16(fmaxf(z, 0.f));
                    S.m1[r][n] = z > 0.f ? 1 : 0;
                }
        }
    }
    __syncthreads();

    // layer 2: z2 = bf16(h1) W2^T + b2; h2 = bf16(relu(z2)) kept in registers
    float h2[2][4][4], m2[2][4][4];
    {
        f32x4 acc[2][4] = {};
        bf16x8 fb[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) fb[c] = frag(a.W2b, kH, 64 * wv + 16 * c, 0, lane);
        for (int k0 = 0; k0 < kH; k0 += 32) {
            bf16x8 fa[2], nb[4];
            const int k1 = k0 + 32 < kH ? k0 + 32 : k0;   // next step's weights in flight
#pragma unroll
            for (int c = 0; c < 4; ++c) nb[c] = frag(a.W2b, kH, 64 * wv + 16 * c, k1, lane);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) fa[rb] = frag(&S.h1[0][0], kLdH, 16 * rb, k0, lane);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[rb][c] = mfma(fa[rb], fb[c], acc[rb][c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) fb[c] = nb[c];
        }
        float yp[2][4] = {};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int n = 64 * wv + 16 * c + (lane & 15);
            const float bias = a.b2[n], w3 = from_bf16(a.w3b[n]);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float z = acc[rb][c][v] + bias;
                    h2[rb][c][v] = from_bf16(to_bf16(fmaxf(z, 0.f)));
                    m2[rb][c][v] = z > 0.f ? 1.f : 0.f;
                    yp[rb][v] += h2[rb][c][v] * w3;
                }
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float s = sum_row(yp[rb][v]);
                if ((lane & 15) == 0) S.yp[wv][16 * rb + 4 * (lane >> 4) + v] = s;
            }
    }
    __syncthreads();
    if (tid < kTB) {
        const int64_t b = b0 + tid;
        const float y = ((S.yp[0][tid] + S.yp[1][tid]) + (S.yp[2][tid] + S.yp[3][tid])) + a.b3[0];
        float dy = 0.f;
        if (b < a.B) {
            a.y[b] = y;
            if (a.target) {
                const float r = y - a.target[b];
                dy = 2.f * r / (float)a.B;
                a.sq[b] = r * r;
            }
        }
        S.dy[tid] = dy;
    }
    if (!a.target) return;   // forward only (uniform)
    __syncthreads();

    // output layer backward: dz2 = dy w3 [z2 > 0]; per-tile sums of dz2
    // (b2), h2 dy (w3) and dy (b3); bf16(dz2) to LDS
    const int64_t tile = blockIdx.x;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int n = 64 * wv + 16 * c + (lane & 15);
        const float w3 = from_bf16(a.w3b[n]);
        float sb2 = 0.f, sw3 = 0.f;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * rb + 4 * (lane >> 4) + v;
                const float dy = S.dy[r];
                const float g = m2[rb][c][v] != 0.f ? dy * w3 : 0.f;
                sb2 += g;
                sw3 += h2[rb][c][v] * dy;
                S.dz2[r][n] = to_bf16(g);
            }
        sb2 = sum_groups(sb2);
        sw3 = sum_groups(sw3);
        if (lane < 16) {
            a.pb2[tile * kH + n] = sb2;
            a.pw3[tile * kH + n] = sw3;
        }
    }
    if (tid == 0) {
        float s = 0.f;
        for (int r = 0; r < kTB; ++r) s += S.dy[r];
        a.pb3[tile] = s;
    }
    __syncthreads();

    // dz1 = (bf16(dz2) W2) [z1 > 0]; per-tile sums (b1); bf16(dz1) to LDS
    {
        f32x4 acc[2][4] = {};
        bf16x8 fb[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) fb[c] = frag(a.W2bT, kH, 64 * wv + 16 * c, 0, lane);
        for (int k0 = 0; k0 < kH; k0 += 32) {
            bf16x8 fa[2], nb[4];
            const int k1 = k0 + 32 < kH ? k0 + 32 : k0;
#pragma unroll
            for (int c = 0; c < 4; ++c) nb[c] = frag(a.W2bT, kH, 64 * wv + 16 * c, k1, lane);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) fa[rb] = frag(&S.dz2[0][0], kLdH, 16 * rb, k0, lane);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[rb][c] = mfma(fa[rb], fb[c], acc[rb][c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) fb[c] = nb[c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int n = 64 * wv + 16 * c + (lane & 15);
            float sb1 = 0.f;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rb + 4 * (lane >> 4) + v;
                    const float g = S.m1[r][n] ? acc[rb][c][v] : 0.f;
                    sb1 += g;
                    S.dz1[r][n] = to_bf16(g);
                }
            sb1 = sum_groups(sb1);
            if (lane < 16) a.pb1[tile * kH + n] = sb1;
        }
    }
    __syncthreads();

    // dx = bf16(dz1) W1 (wave wv: columns 16 wv .. 16 wv + 15)
    {
        f32x4 acc[2] = {};
        bf16x8 fb[kH / 32];
#pragma unroll
        for (int k = 0; k < kH / 32; ++k) fb[k] = frag(a.W1bT, kH, 16 * wv, 32 * k, lane);
#pragma unroll
        for (int k = 0; k < kH / 32; ++k)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
                acc[rb] = mfma(frag(&S.dz1[0][0], kLdH, 16 * rb, 32 * k, lane), fb[k], acc[rb]);
        const int d = 16 * wv + (lane & 15);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t b = b0 + 16 * rb + 4 * (lane >> 4) + v;
                a.dX[b * kD2 + d] = acc[rb][v];
            }
    }
    // the weight-gradient operands, feature-major
    store_transposed<kD2, kLdX>(S.x, a.XrT, a.Bp, b0);
    store_transposed<kH, kLdH>(S.h1, a.H1rT, a.Bp, b0);
    store_transposed<kH, kLdH>(S.dz2, a.dZ2rT, a.Bp, b0);
    store_transposed<kH, kLdH>(S.dz1, a.dZ1rT, a.Bp, b0);
}

// ------------------------------------------------------------- kernel B --

// One 64 x 64 tile of a split-K product over a chunk of 256 candidates:
// out[m][n] = sum_b A[m][b] Bm[n][b], A and Bm feature-major (row stride
// Bp); four waves of 32 x 32.
__device__ void grad_tile(const uint16_t *A, const uint16_t *Bm, int64_t Bp, int64_t m0,
                          int64_t n0, int64_t kb, float *out, int64_t ldo) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t mw = m0 + 32 * (wv >> 1), nw = n0 + 32 * (wv & 1);
    f32x4 acc[2][2] = {};
    for (int64_t k0 = kb; k0 < kb + kChunk; k0 += 32) {
        bf16x8 fa[2], fb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            fa[i] = frag(A, Bp, mw + 16 * i, k0, lane);
            fb[i] = frag(Bm, Bp, nw + 16 * i, k0, lane);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma(fa[i], fb[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                out[(mw + 16 * i + 4 * (lane >> 4) + v) * ldo + nw + 16 * j + (lane & 15)] =
                    acc[i][j][v];
}

// Fixed-order sum of the kBlock threads' vectors v[0..kD) into out (thread
// c < kD writes out[c]): threads' rows of 32 are added in order, then the
// eight rows.  red holds kBlock x kD floats.
__device__ void block_sum(const float (&v)[kD], float *red, float *out) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int c = 0; c < kD; ++c) red[tid * kD + c] = v[c];
    __syncthreads();
    constexpr int kGroups = kBlock / kD;          // 8 groups of 32 threads' vectors
    const int r = tid / kD, c = tid % kD;         // thread: group r, dimension c
    float acc = 0.f;
    for (int k = 0; k < kBlock / kGroups; ++k) acc += red[(r * (kBlock / kGroups) + k) * kD + c];
    __syncthreads();
    red[r * kD + c] = acc;
    __syncthreads();
    if (tid < kD) {
        float s = 0.f;
        for (int k = 0; k < kGroups; ++k) s += red[k * kD + tid];
        out[tid] = s;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void mlp_grads_kernel(FusedGrads g) {
    __shared__ float red[kBlock * kD];
    const int tid = threadIdx.x;
    const int64_t nS = g.Bp / kChunk;
    const int64_t nT = g.Bp / kTB;
    int64_t job = blockIdx.x;
    // dW2 partials: 16 tiles per chunk
    if (job < 16 * nS) {
        const int64_t s = job / 16, t = job % 16;
        grad_tile(g.dZ2rT, g.H1rT, g.Bp, 64 * (t / 4), 64 * (t % 4), s * kChunk,
                  g.ws2 + s * (int64_t)kH * kH, kH);
        return;
    }
    job -= 16 * nS;
    // dW1 partials: 4 tiles per chunk
    if (job < 4 * nS) {
        const int64_t s = job / 4, t = job % 4;
        grad_tile(g.dZ1rT, g.XrT, g.Bp, 64 * t, 0, s * kChunk, g.ws1 + s * (int64_t)kH * kD2, kD2);
        return;
    }
    job -= 4 * nS;
    // b1, b2, w3: the row tiles' partial sums, 32 columns per job
    if (job < 3 * (kH / 32)) {
        const int v = (int)(job / (kH / 32));
        const int h = (int)(job % (kH / 32)) * 32 + tid % 32, r = tid / 32;
        const float *src = v == 0 ? g.pb1 : (v == 1 ? g.pb2 : g.pw3);
        float *dst = v == 0 ? g.gb1 : (v == 1 ? g.gb2 : g.gw3);
        float acc = 0.f;
        for (int64_t t = r; t < nT; t += kBlock / 32) acc += src[t * kH + h];
        red[r * 32 + tid % 32] = acc;
        __syncthreads();
        if (r == 0) {
            float sum = 0.f;
            for (int k = 0; k < kBlock / 32; ++k) sum += red[k * 32 + tid];
            dst[h] = sum;
        }
        return;
    }
    job -= 3 * (kH / 32);
    if (job == 0) {   // b3
        float acc = 0.f;
        for (int64_t t = tid; t < nT; t += kBlock) acc += g.pb3[t];
        red[tid] = acc;
        __syncthreads();
        if (tid == 0) {
            float sum = 0.f;
            for (int k = 0; k < kBlock; ++k) sum += red[k];
            g.gb3[0] = sum;
        }
        return;
    }
    job -= 1;
    if (job < g.M) {
        // embedding tables of column j: one occurrence per thread at a time
        // (occurrences in candidate-then-series order), then fixed-order sums
        const int32_t j = (int32_t)job;
        float ge[kD], gf[kD], gt[kD];
#pragma unroll
        for (int c = 0; c < kD; ++c) ge[c] = gf[c] = gt[c] = 0.f;
        const int32_t o1 = g.occ_start[j + 1];
        for (int32_t o = g.occ_start[j] + tid; o < o1; o += kBlock) {
            const int32_t pos = g.occ_pos[o], b = g.occ_b[o];
            const int32_t s = g.off[b], e = g.off[b + 1];
            const float4 *dx = reinterpret_cast<const float4 *>(g.dX + (int64_t)b * kD2);
            const float inv_l = 1.f / (float)(e - s);
#pragma unroll
            for (int q = 0; q < kD / 4; ++q) {
                const float4 x = dx[q];
                ge[4 * q] += x.x * inv_l;
                ge[4 * q + 1] += x.y * inv_l;
                ge[4 * q + 2] += x.z * inv_l;
                ge[4 * q + 3] += x.w * inv_l;
            }
            if (e - s > 1) {
                const float inv = 1.f / (float)(e - s - 1);
                const bool has_next = pos + 1 < e, has_prev = pos > s;
                const float4 *tn = reinterpret_cast<const float4 *>(
                    g.T + (int64_t)g.cols[has_next ? pos + 1 : pos] * kD);
                const float4 *fp = reinterpret_cast<const float4 *>(
                    g.F + (int64_t)g.cols[has_prev ? pos - 1 : pos] * kD);
#pragma unroll
                for (int q = 0; q < kD / 4; ++q) {
                    const float4 x = dx[kD / 4 + q];
                    const float xs[4] = {x.x, x.y, x.z, x.w};
                    const float4 tv = tn[q], fv = fp[q];
                    const float ts[4] = {tv.x, tv.y, tv.z, tv.w};
                    const float fs[4] = {fv.x, fv.y, fv.z, fv.w};
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (has_next) gf[4 * q + u] += xs[u] * ts[u] * inv;
                        if (has_prev) gt[4 * q + u] += xs[u] * fs[u] * inv;
                    }
                }
            }
        }
        block_sum(ge, red, g.gE + (int64_t)j * kD);
        block_sum(gf, red, g.gF + (int64_t)j * kD);
        block_sum(gt, red, g.gT + (int64_t)j * kD);
        return;
    }
    job -= g.M;
    if (job <= g.M) {
        // length embedding: candidates of length l, one per thread at a time
        const int32_t l = (int32_t)job;
        float gz[kD];
#pragma unroll
        for (int c = 0; c < kD; ++c) gz[c] = 0.f;
        const int32_t o1 = g.len_start[l + 1];
        for (int32_t o = g.len_start[l] + tid; o < o1; o += kBlock) {
            const float4 *dx = reinterpret_cast<const float4 *>(g.dX + (int64_t)g.len_b[o] * kD2);
#pragma unroll
            for (int q = 0; q < kD / 4; ++q) {
                const float4 x = dx[q];
                gz[4 * q] += x.x;
                gz[4 * q + 1] += x.y;
                gz[4 * q + 2] += x.z;
                gz[4 * q + 3] += x.w;
            }
        }
        block_sum(gz, red, g.gZ + (int64_t)l * kD);
    }
}

// ------------------------------------------------------------- kernel C --

__global__ __launch_bounds__(kBlock) void mlp_update_kernel(FusedUpdate u) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= u.n_params) return;
    float p = u.p[i];
    if (u.mode != kUpdateCast) {
        float g;
        if (i < u.oW1 || (i >= u.ob1 && i < u.oW2) || i >= u.ob2) {
            g = u.g[i];                        // embeddings, b1, b2, w3, b3 (kernel B)
        } else if (i < u.ob1) {
            const int64_t k = i - u.oW1;
            g = 0.f;
#pragma unroll 8
            for (int64_t s = 0; s < u.nS; ++s) g += u.ws1[s * (int64_t)kH * kD2 + k];
        } else {
            const int64_t k = i - u.oW2;
            g = 0.f;
#pragma unroll 8
            for (int64_t s = 0; s < u.nS; ++s) g += u.ws2[s * (int64_t)kH * kH + k];
        }
        u.g[i] = g;
        if (u.mode == kUpdateGradients) return;
        const float m1 = u.beta1 * u.m1[i] + (1.f - u.beta1) * g;
        const float m2 = u.beta2 * u.m2[i] + (1.f - u.beta2) * g * g;
        u.m1[i] = m1;
        u.m2[i] = m2;
        p -= u.lr * (m1 / u.c1) / (sqrtf(m2 / u.c2) + u.eps);
        u.p[i] = p;
    }
    // BF16 copies
    if (i >= u.oW1 && i < u.ob1) {
        const int64_t k = i - u.oW1, h = k / kD2, d = k % kD2;
        const uint16_t q = to_bf16(p);
        u.W1b[k] = q;
        u.W1bT[d * kH + h] = q;
    } else if (i >= u.oW2 && i < u.ob2) {
        const int64_t k = i - u.oW2, n = k / kH, c = k % kH;
        const uint16_t q = to_bf16(p);
        u.W2b[k] = q;
        u.W2bT[c * kH + n] = q;
    } else if (i >= u.ow3 && i < u.ob3) {
        u.w3b[i - u.ow3] = to_bf16(p);
    }
}

}  // namespace

bool fused_shape(int32_t D, int32_t H) { return D == kD && H == kH; }
int32_t fused_tile_rows() { return kTB; }
int32_t fused_chunk() { return kChunk; }

hipError_t fused_rows(const FusedRows &a, hipStream_t s) {
    hipLaunchKernelGGL(mlp_rows_kernel, dim3((unsigned)(a.Bp / kTB)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t fused_grads(const FusedGrads &g, hipStream_t s) {
    const int64_t nS = g.Bp / kChunk;
    const int64_t jobs = 20 * nS + 3 * (kH / 32) + 1 + g.M + (g.M + 1);
    hipLaunchKernelGGL(mlp_grads_kernel, dim3((unsigned)jobs), dim3(kBlock), 0, s, g);
    return hipGetLastError();
}

hipError_t fused_update(const FusedUpdate &u, hipStream_t s) {
    hipLaunchKernelGGL(mlp_update_kernel, dim3((unsigned)((u.n_params + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, u);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace ebic
