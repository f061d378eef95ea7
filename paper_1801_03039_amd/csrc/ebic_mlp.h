// Internal launchers of the surrogate MLP kernels (ebic_mlp_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ebic.h"

struct ebic_mlp;

namespace ebic {

// Loss of the last ebic_mlp_train call before its last step (waits for the
// steps that call queued when it was made without a loss pointer).
ebic_status mlp_last_loss(ebic_mlp *m, float *loss);

namespace mlp {

// C[M x N] = sum_k A(m,k) B(k,n), BF16 operands by strides, FP32 result.
// splits > 1: K is cut into `splits` ranges whose partial products go to ws
// (splits*M*N floats) and are then summed in order into out_f32.
struct Gemm {
    const uint16_t *A;
    int64_t am, ak;
    const uint16_t *B;
    int64_t bk, bn;
    int32_t M, N, K;
    int32_t splits;
    const float *bias;     // per n, or nullptr (splits == 1 only)
    int32_t relu;          // out_bf16 holds relu(v) when set
    float *out_f32;        // or nullptr (splits == 1)
    uint16_t *out_bf16;    // or nullptr (splits == 1 only)
    float *ws;             // splits > 1
};

hipError_t pool_fwd(const float *E, const float *F, const float *T, const float *Zl, int32_t D,
                    const int32_t *off, const int32_t *cols, int32_t B, float *X, uint16_t *Xb,
                    hipStream_t s);
// dZl[l][d] = sum over the candidates b of length l (CSR len_start/len_b)
// of dX[b][d], for l < n_len.
hipError_t len_bwd(const float *dX, int32_t D, const int32_t *len_start, const int32_t *len_b,
                   int32_t n_len, float *dZl, hipStream_t s);
hipError_t pool_bwd(const float *dX, int32_t D, const float *F, const float *T, const int32_t *off,
                    const int32_t *cols, const int32_t *occ_start, const int32_t *occ_pos,
                    const int32_t *occ_b, int32_t M, float *dE, float *dF, float *dT,
                    hipStream_t s);
hipError_t gemm(const Gemm &g, hipStream_t s);
hipError_t colsum(const float *X, const float *w, int32_t B, int32_t N, int32_t splits, float *ws,
                  float *out, hipStream_t s);
hipError_t dw3(const uint16_t *H2b, const float *dy, int32_t B, int32_t N, int32_t splits,
               float *ws, float *out, hipStream_t s);
hipError_t out_fwd(const uint16_t *H2b, const uint16_t *w3b, const float *b3, int32_t B, int32_t H,
                   float *y, hipStream_t s);
hipError_t loss(const float *y, const float *t, int32_t B, float *dy, float *sq, hipStream_t s);
hipError_t out_bwd(const float *dy, const uint16_t *w3b, const float *Z2, int32_t B, int32_t H,
                   float *dZ2, uint16_t *dZ2b, hipStream_t s);
hipError_t relu_bwd(const float *G, const float *Z, int64_t n, float *dZ, uint16_t *dZb,
                    hipStream_t s);
hipError_t adam(float *p, const float *g, float *m1, float *m2, int64_t n, float lr, float beta1,
                float beta2, float eps, float c1, float c2, hipStream_t s);
hipError_t cast_bf16(const float *src, int64_t n, uint16_t *dst, hipStream_t s);

// ------------------------------------------------ fused step (D 32, H 256) --
// (ebic_mlp_fused.hip) Three launches per training step: rows (forward and
// per-candidate backward per tile of candidates), grads (weight and
// embedding gradients), update (gradient sums, Adam, BF16 copies).
bool fused_shape(int32_t D, int32_t H);
int32_t fused_tile_rows();   // candidates per rows workgroup
int32_t fused_chunk();       // candidates per weight-gradient partial; Bp is a multiple

struct FusedRows {
    const float *E, *F, *T, *Zl;
    const int32_t *off, *cols;
    int64_t B, Bp;                   // candidates, padded to a multiple of fused_chunk()
    const uint16_t *W1b, *W1bT, *W2b, *W2bT, *w3b;
    const float *b1, *b2, *b3;
    const float *target;             // nullptr: forward only (y)
    float *y, *sq;
    uint16_t *XrT, *H1rT, *dZ2rT, *dZ1rT;   // feature-major [features][Bp]
    float *dX;                       // [Bp][2D]
    float *pw3, *pb2, *pb1, *pb3;    // per row tile: [tiles][H] (pb3: [tiles])
};

struct FusedGrads {
    int64_t Bp;
    int32_t M;
    const uint16_t *XrT, *H1rT, *dZ2rT, *dZ1rT;
    const float *dX, *F, *T;
    const int32_t *off, *cols, *occ_start, *occ_pos, *occ_b, *len_start, *len_b;
    float *ws1, *ws2;                // [Bp / chunk][H][2D], [Bp / chunk][H][H]
    const float *pw3, *pb2, *pb1, *pb3;   // the rows kernel's per-tile sums
    float *gE, *gF, *gT, *gZ, *gb1, *gb2, *gw3, *gb3;
};

enum { kUpdateCast = 0, kUpdateGradients = 1, kUpdateAdam = 2 };
struct FusedUpdate {
    int32_t mode;
    int64_t n_params, oW1, ob1, oW2, ob2, ow3, ob3;
    int64_t nS, nTiles;
    float *p, *g, *m1, *m2;
    const float *ws1, *ws2;
    float lr, beta1, beta2, eps, c1, c2;
    uint16_t *W1b, *W1bT, *W2b, *W2bT, *w3b;
};

hipError_t fused_rows(const FusedRows &a, hipStream_t s);
hipError_t fused_grads(const FusedGrads &g, hipStream_t s);
hipError_t fused_update(const FusedUpdate &u, hipStream_t s);

}  // namespace mlp
}  // namespace ebic
