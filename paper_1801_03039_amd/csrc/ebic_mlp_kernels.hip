// Surrogate fitness model: a 3-layer MLP over learned column embeddings,
// trained and run on gfx950 with hand-written kernels.
//
//   x_b  = [ (1/L) sum_t E[c_t] ;                     node embeddings, mean pool
//            (1/(L-1)) sum_{t<L-1} F[c_t] * T[c_{t+1}] ]   ordered pairs (0 if L = 1)
//   z1   = W1 bf16(x_b) + b1,  h1 = relu(z1)          BF16 MFMA, FP32 accumulate
//   z2   = W2 bf16(h1) + b2,   h2 = relu(z2)          BF16 MFMA, FP32 accumulate
//   y_b  = w3 . bf16(h2) + b3                         FP32 accumulate
//   loss = (1/B) sum_b (y_b - t_b)^2
//
// Weights are FP32 masters with BF16 copies used by the products; gradients
// flow through the BF16 casts unchanged.  Every reduction has a fixed order
// (no floating-point atomics), so training is deterministic on one device.
// The network only ranks candidates; the evolutionary run still scores every
// admitted candidate exactly.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ebic_mlp.h"

namespace ebic {
namespace mlp {
namespace {

constexpr int kBlock = 256;
constexpr int kWave = 64;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------ embedding --

// X[b][d] for d < D: (sum_t E[c_t][d]) / L; for d = D + e:
// (sum_{t < L-1} F[c_t][e] * T[c_{t+1}][e]) / (L - 1), 0 when L = 1; sums in
// series order.  Xb = bf16(X).  X is B x 2D.
__global__ __launch_bounds__(kBlock) void pool_fwd_kernel(const float *__restrict__ E,
                                                          const float *__restrict__ F,
                                                          const float *__restrict__ T,
                                                          const float *__restrict__ Zl, int32_t D,
                                                          const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ cols,
                                                          int32_t B, float *__restrict__ X,
                                                          uint16_t *__restrict__ Xb) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int32_t D2 = 2 * D;
    if (i >= (int64_t)B * D2) return;
    const int32_t b = (int32_t)(i / D2), d = (int32_t)(i - (int64_t)b * D2);
    const int32_t s = off[b], e = off[b + 1];
    float x = 0.f;
    if (d < D) {
        float acc = 0.f;
        for (int32_t t = s; t < e; ++t) acc += E[(int64_t)cols[t] * D + d];
        x = acc / (float)(e - s) + Zl[(int64_t)(e - s) * D + d];
    } else if (e - s > 1) {
        const int32_t dd = d - D;
        float acc = 0.f;
        for (int32_t t = s; t + 1 < e; ++t)
            acc += F[(int64_t)cols[t] * D + dd] * T[(int64_t)cols[t + 1] * D + dd];
        x = acc / (float)(e - s - 1);
    }
    X[i] = x;
    Xb[i] = to_bf16(x);
}

// Gradients of the three embedding tables for column j, gathered over its
// occurrences (positions in cols, in candidate-then-series order, with their
// candidate in occ_b) so that every sum has a fixed order:
//   dE[j] += dX[b][0:D] / L
//   dF[j] += dX[b][D:2D] * T[next column] / (L-1)   (j not last)
//   dT[j] += dX[b][D:2D] * F[previous column] / (L-1) (j not first)
// Workgroup = (column j, slice of kLaneW embedding dims); its kRows rows of
// lanes take occurrences r, r + kRows, ... in order, and row 0 adds the
// rows' partial sums in row order.
constexpr int kLaneW = 32;
constexpr int kRows = kBlock / kLaneW;

__global__ __launch_bounds__(kBlock) void pool_bwd_kernel(const float *__restrict__ dX, int32_t D,
                                                          const float *__restrict__ F,
                                                          const float *__restrict__ T,
                                                          const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ cols,
                                                          const int32_t *__restrict__ occ_start,
                                                          const int32_t *__restrict__ occ_pos,
                                                          const int32_t *__restrict__ occ_b,
                                                          int32_t M, float *__restrict__ dE,
                                                          float *__restrict__ dF,
                                                          float *__restrict__ dT) {
    const int32_t j = blockIdx.x;
    const int32_t r = threadIdx.x / kLaneW;
    const int32_t d = blockIdx.y * kLaneW + (int32_t)(threadIdx.x % kLaneW);
    float ge = 0.f, gf = 0.f, gt = 0.f;
    if (d < D) {
        const int32_t o1 = occ_start[j + 1];
        for (int32_t o = occ_start[j] + r; o < o1; o += kRows) {
            const int32_t pos = occ_pos[o], b = occ_b[o];
            const int32_t s = off[b], e = off[b + 1];
            const float *dx = dX + (int64_t)b * 2 * D;
            ge += dx[d] / (float)(e - s);
            if (e - s > 1) {
                const float inv = 1.f / (float)(e - s - 1);
                if (pos + 1 < e) gf += dx[D + d] * T[(int64_t)cols[pos + 1] * D + d] * inv;
                if (pos > s) gt += dx[D + d] * F[(int64_t)cols[pos - 1] * D + d] * inv;
            }
        }
    }
    __shared__ float s_g[3][kRows][kLaneW];
    const int32_t c = threadIdx.x % kLaneW;
    s_g[0][r][c] = ge;
    s_g[1][r][c] = gf;
    s_g[2][r][c] = gt;
    __syncthreads();
    if (r == 0 && d < D) {
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
        for (int32_t k = 0; k < kRows; ++k) {
            a0 += s_g[0][k][c];
            a1 += s_g[1][k][c];
            a2 += s_g[2][k][c];
        }
        const int64_t i = (int64_t)j * D + d;
        dE[i] = a0;
        dF[i] = a1;
        dT[i] = a2;
    }
}

// Gradient of the length embedding: dZ[l] = sum of dX[b][0:D] over the
// candidates of length l (len_b[len_start[l] .. len_start[l+1]), in
// candidate order).  Workgroup = (length l, slice of kLaneW dims); rows of
// lanes take list entries r, r + kRows, ... and row 0 adds the partial sums
// in row order.
__global__ __launch_bounds__(kBlock) void len_bwd_kernel(const float *__restrict__ dX, int32_t D,
                                                         const int32_t *__restrict__ len_start,
                                                         const int32_t *__restrict__ len_b,
                                                         int32_t n_len, float *__restrict__ dZl) {
    const int32_t l = blockIdx.x;
    const int32_t r = threadIdx.x / kLaneW;
    const int32_t c = threadIdx.x % kLaneW;
    const int32_t d = blockIdx.y * kLaneW + c;
    float acc = 0.f;
    if (d < D) {
        const int32_t o1 = len_start[l + 1];
        int32_t o = len_start[l] + r;
        // four entries per step: their indices, then their values, then the
        // additions in list order
        for (; o + 3 * kRows < o1; o += 4 * kRows) {
            int32_t bb[4];
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) bb[k] = len_b[o + k * kRows];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = dX[(int64_t)bb[k] * 2 * D + d];
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += v[k];
        }
        for (; o < o1; o += kRows) acc += dX[(int64_t)len_b[o] * 2 * D + d];
    }
    __shared__ float s_p[kRows][kLaneW];
    s_p[r][c] = acc;
    __syncthreads();
    if (r == 0 && d < D) {
        float a = 0.f;
        for (int32_t k = 0; k < kRows; ++k) a += s_p[k][c];
        dZl[(int64_t)l * D + d] = a;
    }
}

// ----------------------------------------------------------------- GEMM --
//
// C[M x N] = sum_k A(m,k) B(k,n) with BF16 operands addressed by strides
// (A(m,k) = A[m*am + k*ak], B(k,n) = B[k*bk + n*bn]) and FP32 accumulation
// on v_mfma_f32_16x16x16_bf16.  Workgroup tile 64 x 64, four waves of
// 32 x 32 (2 x 2 MFMA blocks), K staged through LDS 32 at a time.
// blockIdx.z selects a K split: with splits > 1 each split writes its
// partial tile to ws[z][M][N] (summed later in a fixed order).
// Epilogue (splits == 1): v = C + bias[n]; out_f32 <- v; out_bf16 <-
// bf16(relu ? max(v, 0) : v).
constexpr int kT = 64, kK = 32, kPad = 4;

struct GemmArgs {
    const uint16_t *A;
    int64_t am, ak;
    const uint16_t *B;
    int64_t bk, bn;
    int32_t M, N, K;
    int32_t splits;
    const float *bias;
    int32_t relu;
    float *out_f32;
    uint16_t *out_bf16;
    float *ws;
};

__global__ __launch_bounds__(kBlock) void gemm_bf16_kernel(GemmArgs g) {
    __shared__ uint16_t As[kT][kK + kPad];   // [m][k]
    __shared__ uint16_t Bt[kT][kK + kPad];   // [n][k]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv >> 1, wn = wv & 1;
    const int64_t m0 = (int64_t)blockIdx.x * kT, n0 = (int64_t)blockIdx.y * kT;
    const int32_t split = blockIdx.z;
    const int64_t kchunk = ((int64_t)g.K + g.splits - 1) / g.splits;
    const int64_t kbeg = split * kchunk;
    const int64_t kend = kbeg + kchunk < g.K ? kbeg + kchunk : g.K;

    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    const bool a_kfast = g.ak == 1, b_kfast = g.bk == 1;
    for (int64_t k0 = kbeg; k0 < kend; k0 += kK) {
        // stage A[m0..m0+64) x [k0..k0+32) and B[k0..k0+32) x [n0..n0+64)
#pragma unroll
        for (int r = 0; r < (kT * kK) / kBlock; ++r) {
            const int e = r * kBlock + tid;
            const int mi = a_kfast ? e / kK : e % kT;
            const int ki = a_kfast ? e % kK : e / kT;
            const int64_t m = m0 + mi, k = k0 + ki;
            As[mi][ki] = (m < g.M && k < kend) ? g.A[m * g.am + k * g.ak] : (uint16_t)0;
            const int ni = b_kfast ? e / kK : e % kT;
            const int kj = b_kfast ? e % kK : e / kT;
            const int64_t n = n0 + ni, kk = k0 + kj;
            Bt[ni][kj] = (n < g.N && kk < kend) ? g.B[kk * g.bk + n * g.bn] : (uint16_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kK; ks += 16) {
            bf16x4 a[2], b[2];
            const int kq = ks + 4 * (lane >> 4);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = wm * 32 + i * 16 + (lane & 15);
#pragma unroll
                for (int v = 0; v < 4; ++v) a[i][v] = (short)As[row][kq + v];
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = wn * 32 + j * 16 + (lane & 15);
#pragma unroll
                for (int v = 0; v < 4; ++v) b[j][v] = (short)Bt[col][kq + v];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // acc[i][j][v] is C[row0 + 4*(lane/16) + v][col0 + lane%16]
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
                const int64_t n = n0 + wn * 32 + j * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float val = acc[i][j][v];
                if (g.splits > 1) {
                    g.ws[((int64_t)split * g.M + m) * g.N + n] = val;
                    continue;
                }
                if (g.bias) val += g.bias[n];
                if (g.out_f32) g.out_f32[m * g.N + n] = val;
                if (g.out_bf16) g.out_bf16[m * g.N + n] = to_bf16(g.relu ? fmaxf(val, 0.f) : val);
            }
}

// out[i] = sum_s ws[s][i], s in order.
__global__ __launch_bounds__(kBlock) void split_sum_kernel(const float *__restrict__ ws,
                                                           int32_t splits, int64_t n,
                                                           float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float acc = 0.f;
    for (int32_t s = 0; s < splits; ++s) acc += ws[(int64_t)s * n + i];
    out[i] = acc;
}

// Column sums of a B x N FP32 matrix, weighted per row when w != nullptr:
// ws[s][n] = sum over rows of chunk s of (w ? w[b] : 1) * X[b][n].
__global__ __launch_bounds__(kBlock) void colsum_kernel(const float *__restrict__ X,
                                                        const float *__restrict__ w, int32_t B,
                                                        int32_t N, int32_t splits,
                                                        float *__restrict__ ws) {
    const int32_t n = blockIdx.x * kBlock + threadIdx.x;
    const int32_t s = blockIdx.y;
    if (n >= N) return;
    const int32_t chunk = (B + splits - 1) / splits;
    const int32_t b0 = s * chunk, b1 = b0 + chunk < B ? b0 + chunk : B;
    float acc = 0.f;
    int32_t b = b0;
    for (; b + 7 < b1; b += 8) {   // eight loads in flight, additions in row order
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (w ? w[b + k] : 1.f) * X[(int64_t)(b + k) * N + n];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += v[k];
    }
    for (; b < b1; ++b) acc += (w ? w[b] : 1.f) * X[(int64_t)b * N + n];
    ws[(int64_t)s * N + n] = acc;
}

// --------------------------------------------------------- output layer --

// y[b] = sum_n w3b[n] * H2b[b][n] + b3: lanes take n = lane, lane+64, ...;
// the wave's partial sums are added by a fixed shuffle tree.
__global__ __launch_bounds__(kBlock) void out_fwd_kernel(const uint16_t *__restrict__ H2b,
                                                         const uint16_t *__restrict__ w3b,
                                                         const float *__restrict__ b3,
                                                         int32_t B, int32_t H,
                                                         float *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6);
    if (b >= B) return;  // uniform per wave
    float acc = 0.f;
    for (int32_t n = lane; n < H; n += kWave)
        acc += from_bf16(w3b[n]) * from_bf16(H2b[b * H + n]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if (lane == 0) y[b] = acc + b3[0];
}

// dy[b] = 2 (y[b] - t[b]) / B; sq[b] = (y[b] - t[b])^2 (summed later).
__global__ __launch_bounds__(kBlock) void loss_kernel(const float *__restrict__ y,
                                                      const float *__restrict__ t, int32_t B,
                                                      float *__restrict__ dy,
                                                      float *__restrict__ sq) {
    const int32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= B) return;
    const float r = y[b] - t[b];
    dy[b] = 2.f * r / (float)B;
    sq[b] = r * r;
}

// dZ2[b][n] = dy[b] * w3b[n] * [z2 > 0]  (FP32 and BF16 copies).
__global__ __launch_bounds__(kBlock) void out_bwd_kernel(const float *__restrict__ dy,
                                                         const uint16_t *__restrict__ w3b,
                                                         const float *__restrict__ Z2, int32_t B,
                                                         int32_t H, float *__restrict__ dZ2,
                                                         uint16_t *__restrict__ dZ2b) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)B * H) return;
    const int32_t b = (int32_t)(i / H), n = (int32_t)(i - (int64_t)b * H);
    const float g = Z2[i] > 0.f ? dy[b] * from_bf16(w3b[n]) : 0.f;
    dZ2[i] = g;
    dZ2b[i] = to_bf16(g);
}

// dZ1 = G * [z1 > 0]  (FP32 and BF16 copies).
__global__ __launch_bounds__(kBlock) void relu_bwd_kernel(const float *__restrict__ G,
                                                          const float *__restrict__ Z, int64_t n,
                                                          float *__restrict__ dZ,
                                                          uint16_t *__restrict__ dZb) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float g = Z[i] > 0.f ? G[i] : 0.f;
    dZ[i] = g;
    dZb[i] = to_bf16(g);
}

// Weighted column sum for dw3: dw3[n] = sum_b dy[b] * H2b[b][n], split
// over row chunks like colsum_kernel (H2 read as BF16).
__global__ __launch_bounds__(kBlock) void dw3_kernel(const uint16_t *__restrict__ H2b,
                                                     const float *__restrict__ dy, int32_t B,
                                                     int32_t N, int32_t splits,
                                                     float *__restrict__ ws) {
    const int32_t n = blockIdx.x * kBlock + threadIdx.x;
    const int32_t s = blockIdx.y;
    if (n >= N) return;
    const int32_t chunk = (B + splits - 1) / splits;
    const int32_t b0 = s * chunk, b1 = b0 + chunk < B ? b0 + chunk : B;
    float acc = 0.f;
    int32_t b = b0;
    for (; b + 7 < b1; b += 8) {   // eight loads in flight, additions in row order
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = dy[b + k] * from_bf16(H2b[(int64_t)(b + k) * N + n]);
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += v[k];
    }
    for (; b < b1; ++b) acc += dy[b] * from_bf16(H2b[(int64_t)b * N + n]);
    ws[(int64_t)s * N + n] = acc;
}

// ---------------------------------------------------------------- Adam --

__global__ __launch_bounds__(kBlock) void adam_kernel(float *__restrict__ p,
                                                      const float *__restrict__ g,
                                                      float *__restrict__ m1,
                                                      float *__restrict__ m2, int64_t n, float lr,
                                                      float beta1, float beta2, float eps,
                                                      float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = beta1 * m1[i] + (1.f - beta1) * gi;
    const float b = beta2 * m2[i] + (1.f - beta2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

__global__ __launch_bounds__(kBlock) void cast_kernel(const float *__restrict__ src, int64_t n,
                                                      uint16_t *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = to_bf16(src[i]);
}

inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

}  // namespace

// ----------------------------------------------------------- launchers --

hipError_t pool_fwd(const float *E, const float *F, const float *T, const float *Zl, int32_t D,
                    const int32_t *off, const int32_t *cols, int32_t B, float *X, uint16_t *Xb,
                    hipStream_t s) {
    hipLaunchKernelGGL(pool_fwd_kernel, grid1((int64_t)B * 2 * D), dim3(kBlock), 0, s, E, F, T, Zl,
                       D, off, cols, B, X, Xb);
    return hipGetLastError();
}

hipError_t len_bwd(const float *dX, int32_t D, const int32_t *len_start, const int32_t *len_b,
                   int32_t n_len, float *dZl, hipStream_t s) {
    const dim3 grid((unsigned)n_len, (unsigned)((D + kLaneW - 1) / kLaneW));
    hipLaunchKernelGGL(len_bwd_kernel, grid, dim3(kBlock), 0, s, dX, D, len_start, len_b, n_len,
                       dZl);
    return hipGetLastError();
}

hipError_t pool_bwd(const float *dX, int32_t D, const float *F, const float *T, const int32_t *off,
                    const int32_t *cols, const int32_t *occ_start, const int32_t *occ_pos,
                    const int32_t *occ_b, int32_t M, float *dE, float *dF, float *dT,
                    hipStream_t s) {
    const dim3 grid((unsigned)M, (unsigned)((D + kLaneW - 1) / kLaneW));
    hipLaunchKernelGGL(pool_bwd_kernel, grid, dim3(kBlock), 0, s, dX, D, F, T, off, cols,
                       occ_start, occ_pos, occ_b, M, dE, dF, dT);
    return hipGetLastError();
}

hipError_t gemm(const Gemm &q, hipStream_t s) {
    GemmArgs g{q.A, q.am, q.ak, q.B, q.bk, q.bn, q.M, q.N, q.K, q.splits < 1 ? 1 : q.splits,
               q.bias, q.relu, q.out_f32, q.out_bf16, q.ws};
    const dim3 grid((unsigned)((q.M + kT - 1) / kT), (unsigned)((q.N + kT - 1) / kT),
                    (unsigned)g.splits);
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(kBlock), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || g.splits == 1) return e;
    const int64_t n = (int64_t)q.M * q.N;
    hipLaunchKernelGGL(split_sum_kernel, grid1(n), dim3(kBlock), 0, s, q.ws, g.splits, n,
                       q.out_f32);
    return hipGetLastError();
}

hipError_t colsum(const float *X, const float *w, int32_t B, int32_t N, int32_t splits, float *ws,
                  float *out, hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((N + kBlock - 1) / kBlock), (unsigned)splits),
                       dim3(kBlock), 0, s, X, w, B, N, splits, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(split_sum_kernel, grid1(N), dim3(kBlock), 0, s, ws, splits, (int64_t)N, out);
    return hipGetLastError();
}

hipError_t dw3(const uint16_t *H2b, const float *dy, int32_t B, int32_t N, int32_t splits,
               float *ws, float *out, hipStream_t s) {
    hipLaunchKernelGGL(dw3_kernel, dim3((unsigned)((N + kBlock - 1) / kBlock), (unsigned)splits),
                       dim3(kBlock), 0, s, H2b, dy, B, N, splits, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(split_sum_kernel, grid1(N), dim3(kBlock), 0, s, ws, splits, (int64_t)N, out);
    return hipGetLastError();
}

hipError_t out_fwd(const uint16_t *H2b, const uint16_t *w3b, const float *b3, int32_t B, int32_t H,
                   float *y, hipStream_t s) {
    hipLaunchKernelGGL(out_fwd_kernel, dim3((unsigned)((B + 3) / 4)), dim3(kBlock), 0, s, H2b, w3b,
                       b3, B, H, y);
    return hipGetLastError();
}

hipError_t loss(const float *y, const float *t, int32_t B, float *dy, float *sq, hipStream_t s) {
    hipLaunchKernelGGL(loss_kernel, grid1(B), dim3(kBlock), 0, s, y, t, B, dy, sq);
    return hipGetLastError();
}

hipError_t out_bwd(const float *dy, const uint16_t *w3b, const float *Z2, int32_t B, int32_t H,
                   float *dZ2, uint16_t *dZ2b, hipStream_t s) {
    hipLaunchKernelGGL(out_bwd_kernel, grid1((int64_t)B * H), dim3(kBlock), 0, s, dy, w3b, Z2, B,
                       H, dZ2, dZ2b);
    return hipGetLastError();
}

hipError_t relu_bwd(const float *G, const float *Z, int64_t n, float *dZ, uint16_t *dZb,
                    hipStream_t s) {
    hipLaunchKernelGGL(relu_bwd_kernel, grid1(n), dim3(kBlock), 0, s, G, Z, n, dZ, dZb);
    return hipGetLastError();
}

hipError_t adam(float *p, const float *g, float *m1, float *m2, int64_t n, float lr, float beta1,
                float beta2, float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, grid1(n), dim3(kBlock), 0, s, p, g, m1, m2, n, lr, beta1, beta2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t cast_bf16(const float *src, int64_t n, uint16_t *dst, hipStream_t s) {
    hipLaunchKernelGGL(cast_kernel, grid1(n), dim3(kBlock), 0, s, src, n, dst);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace ebic
