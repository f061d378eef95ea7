// Surrogate MLP runtime: parameters, buffers and the forward / backward /
// Adam sequences of the kernels in ebic_mlp_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/ebic.h"
#include "ebic_mlp.h"

namespace ebic {
void set_thread_error(const char *msg);
}

using namespace ebic;

struct ebic_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t M = 0, D = 0, H = 0;
    ebic_mlp_config cfg{};
    int64_t n_params = 0;
    int64_t oE = 0, oF = 0, oT = 0, oZ = 0, oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, ow3 = 0, ob3 = 0;
    float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    uint16_t *W1b = nullptr, *W2b = nullptr, *w3b = nullptr;
    int64_t step = 0;
    int32_t last_B = 0;   // batch of the last training call (its loss is in sq)
    // per-batch buffers (capacity cap_B candidates, cap_L column entries)
    int64_t cap_B = 0, cap_L = 0;
    int32_t *off = nullptr, *cols = nullptr, *occ_start = nullptr, *occ_pos = nullptr,
            *occ_b = nullptr, *len_start = nullptr, *len_b = nullptr;
    float *X = nullptr, *Z1 = nullptr, *Z2 = nullptr, *y = nullptr, *t = nullptr, *dy = nullptr,
          *sq = nullptr, *dZ2 = nullptr, *G1 = nullptr, *dZ1 = nullptr, *dX = nullptr;
    uint16_t *Xb = nullptr, *H1b = nullptr, *H2b = nullptr, *dZ2b = nullptr, *dZ1b = nullptr;
    float *ws = nullptr;
    int64_t cap_ws = 0;
    // fused step (embed_dim 32, hidden 256): transposed BF16 weights and
    // per-step buffers for up to cap_Bp (padded) candidates
    bool fused = false;
    uint16_t *W1bT = nullptr, *W2bT = nullptr;
    int64_t cap_Bp = 0;
    uint16_t *XrT = nullptr, *H1rT = nullptr, *dZ2rT = nullptr, *dZ1rT = nullptr;
    float *fdX = nullptr, *ws1 = nullptr, *ws2 = nullptr, *pw3 = nullptr, *pb2 = nullptr,
          *pb1 = nullptr, *pb3 = nullptr;
};

namespace {

constexpr int32_t kMaxSplits = 64;

ebic_status mfail(ebic_status st, const std::string &msg) {
    set_thread_error(msg.c_str());
    return st;
}

#define MHIP(expr)                                                                           \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess)                                                                \
            return mfail(_e == hipErrorOutOfMemory ? EBIC_E_NOMEM : EBIC_E_DEVICE,           \
                         std::string(#expr) + ": " + hipGetErrorString(_e));                 \
    } while (0)

template <typename T>
hipError_t dalloc(T *&p, int64_t n) {
    if (p) {
        hipError_t e = hipFree(p);
        p = nullptr;
        if (e != hipSuccess) return e;
    }
    return hipMalloc((void **)&p, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
}

ebic_status reserve(ebic_mlp *m, int64_t B, int64_t L) {
    const int64_t H = m->H, D = m->D;
    if (B > m->cap_B) {
        MHIP(hipStreamSynchronize(m->stream));
        const int64_t c = std::max<int64_t>(B, m->cap_B * 2);
        MHIP(dalloc(m->off, c + 1));
        MHIP(dalloc(m->X, c * 2 * D));
        MHIP(dalloc(m->Xb, c * 2 * D));
        MHIP(dalloc(m->Z1, c * H));
        MHIP(dalloc(m->H1b, c * H));
        MHIP(dalloc(m->Z2, c * H));
        MHIP(dalloc(m->H2b, c * H));
        MHIP(dalloc(m->y, c));
        MHIP(dalloc(m->t, c));
        MHIP(dalloc(m->dy, c));
        MHIP(dalloc(m->sq, c));
        MHIP(dalloc(m->dZ2, c * H));
        MHIP(dalloc(m->dZ2b, c * H));
        MHIP(dalloc(m->G1, c * H));
        MHIP(dalloc(m->dZ1, c * H));
        MHIP(dalloc(m->dZ1b, c * H));
        MHIP(dalloc(m->dX, c * 2 * D));
        MHIP(dalloc(m->len_b, c));
        m->cap_B = c;
    }
    if (L > m->cap_L) {
        MHIP(hipStreamSynchronize(m->stream));
        const int64_t c = std::max<int64_t>(L, m->cap_L * 2);
        MHIP(dalloc(m->cols, c));
        MHIP(dalloc(m->occ_pos, c));
        MHIP(dalloc(m->occ_b, c));
        m->cap_L = c;
    }
    const int64_t need_ws = (int64_t)kMaxSplits * std::max<int64_t>(H * H, H * 2 * D);
    if (need_ws > m->cap_ws) {
        MHIP(dalloc(m->ws, need_ws));
        m->cap_ws = need_ws;
    }
    return EBIC_OK;
}

int32_t splits_for(int32_t B) { return std::max(1, std::min(kMaxSplits, B / 256)); }

int64_t padded_batch(int64_t B) {
    const int64_t c = mlp::fused_chunk();
    return (B + c - 1) / c * c;
}

// Buffers of the fused step for a batch of B candidates.
ebic_status reserve_fused(ebic_mlp *m, int64_t B) {
    const int64_t Bp = padded_batch(B);
    if (Bp <= m->cap_Bp) return EBIC_OK;
    MHIP(hipStreamSynchronize(m->stream));
    const int64_t c = std::max<int64_t>(Bp, m->cap_Bp * 2);
    const int64_t H = m->H, D2 = 2 * m->D;
    const int64_t tiles = c / mlp::fused_tile_rows(), nS = c / mlp::fused_chunk();
    MHIP(dalloc(m->XrT, D2 * c));
    MHIP(dalloc(m->H1rT, H * c));
    MHIP(dalloc(m->dZ2rT, H * c));
    MHIP(dalloc(m->dZ1rT, H * c));
    MHIP(dalloc(m->fdX, c * D2));
    MHIP(dalloc(m->ws1, nS * H * D2));
    MHIP(dalloc(m->ws2, nS * H * H));
    MHIP(dalloc(m->pw3, tiles * H));
    MHIP(dalloc(m->pb2, tiles * H));
    MHIP(dalloc(m->pb1, tiles * H));
    MHIP(dalloc(m->pb3, tiles));
    m->cap_Bp = c;
    return EBIC_OK;
}

mlp::FusedRows fused_rows_args(ebic_mlp *m, int32_t B, bool train) {
    mlp::FusedRows a{};
    a.E = m->p + m->oE;
    a.F = m->p + m->oF;
    a.T = m->p + m->oT;
    a.Zl = m->p + m->oZ;
    a.off = m->off;
    a.cols = m->cols;
    a.B = B;
    a.Bp = padded_batch(B);
    a.W1b = m->W1b;
    a.W1bT = m->W1bT;
    a.W2b = m->W2b;
    a.W2bT = m->W2bT;
    a.w3b = m->w3b;
    a.b1 = m->p + m->ob1;
    a.b2 = m->p + m->ob2;
    a.b3 = m->p + m->ob3;
    a.target = train ? m->t : nullptr;
    a.y = m->y;
    a.sq = m->sq;
    a.XrT = m->XrT;
    a.H1rT = m->H1rT;
    a.dZ2rT = m->dZ2rT;
    a.dZ1rT = m->dZ1rT;
    a.dX = m->fdX;
    a.pw3 = m->pw3;
    a.pb2 = m->pb2;
    a.pb1 = m->pb1;
    a.pb3 = m->pb3;
    return a;
}

// One fused step: rows, gradients, then the update in `mode`
// (mlp::kUpdateGradients leaves the gradient in m->g; mlp::kUpdateAdam
// also applies Adam with bias corrections c1, c2).
ebic_status fused_step(ebic_mlp *m, int32_t B, int32_t mode, float c1, float c2) {
    const int64_t Bp = padded_batch(B);
    hipStream_t s = m->stream;
    MHIP(mlp::fused_rows(fused_rows_args(m, B, true), s));
    mlp::FusedGrads g{};
    g.Bp = Bp;
    g.M = m->M;
    g.XrT = m->XrT;
    g.H1rT = m->H1rT;
    g.dZ2rT = m->dZ2rT;
    g.dZ1rT = m->dZ1rT;
    g.dX = m->fdX;
    g.F = m->p + m->oF;
    g.T = m->p + m->oT;
    g.off = m->off;
    g.cols = m->cols;
    g.occ_start = m->occ_start;
    g.occ_pos = m->occ_pos;
    g.occ_b = m->occ_b;
    g.len_start = m->len_start;
    g.len_b = m->len_b;
    g.ws1 = m->ws1;
    g.ws2 = m->ws2;
    g.pw3 = m->pw3;
    g.pb2 = m->pb2;
    g.pb1 = m->pb1;
    g.pb3 = m->pb3;
    g.gE = m->g + m->oE;
    g.gF = m->g + m->oF;
    g.gT = m->g + m->oT;
    g.gZ = m->g + m->oZ;
    g.gb1 = m->g + m->ob1;
    g.gb2 = m->g + m->ob2;
    g.gw3 = m->g + m->ow3;
    g.gb3 = m->g + m->ob3;
    MHIP(mlp::fused_grads(g, s));
    mlp::FusedUpdate u{};
    u.mode = mode;
    u.n_params = m->n_params;
    u.oW1 = m->oW1;
    u.ob1 = m->ob1;
    u.oW2 = m->oW2;
    u.ob2 = m->ob2;
    u.ow3 = m->ow3;
    u.ob3 = m->ob3;
    u.nS = Bp / mlp::fused_chunk();
    u.nTiles = Bp / mlp::fused_tile_rows();
    u.p = m->p;
    u.g = m->g;
    u.m1 = m->m1;
    u.m2 = m->m2;
    u.ws1 = m->ws1;
    u.ws2 = m->ws2;
    u.lr = m->cfg.lr;
    u.beta1 = m->cfg.beta1;
    u.beta2 = m->cfg.beta2;
    u.eps = m->cfg.eps;
    u.c1 = c1;
    u.c2 = c2;
    u.W1b = m->W1b;
    u.W1bT = m->W1bT;
    u.W2b = m->W2b;
    u.W2bT = m->W2bT;
    u.w3b = m->w3b;
    MHIP(mlp::fused_update(u, s));
    return EBIC_OK;
}

bool check_cbf(const ebic_mlp *m, const int32_t *off, const int32_t *cols, int32_t B) {
    if (off[0] != 0) return false;
    for (int32_t b = 0; b < B; ++b) {
        if (off[b + 1] <= off[b] || off[b + 1] - off[b] > m->M) return false;
        for (int32_t i = off[b]; i < off[b + 1]; ++i)
            if (cols[i] < 0 || cols[i] >= m->M) return false;
    }
    return true;
}

// Uploads a batch (CBF, occurrence lists by column, optional targets).
ebic_status upload(ebic_mlp *m, const int32_t *off, const int32_t *cols, int32_t B,
                   const float *target, bool occurrences) {
    if (!off || !cols || B < 1) return mfail(EBIC_E_ARG, "need a non-empty CBF batch");
    if (!check_cbf(m, off, cols, B)) return mfail(EBIC_E_RANGE, "malformed CBF, a series longer than n_cols or a column out of range");
    const int64_t L = off[B];
    ebic_status st = reserve(m, B, L);
    if (st != EBIC_OK) return st;
    MHIP(hipMemcpyAsync(m->off, off, sizeof(int32_t) * ((size_t)B + 1), hipMemcpyHostToDevice,
                        m->stream));
    MHIP(hipMemcpyAsync(m->cols, cols, sizeof(int32_t) * (size_t)L, hipMemcpyHostToDevice,
                        m->stream));
    if (target)
        MHIP(hipMemcpyAsync(m->t, target, sizeof(float) * (size_t)B, hipMemcpyHostToDevice,
                            m->stream));
    if (occurrences) {
        // CSR by column: every occurrence (position in cols, and its
        // candidate) of column j, in candidate-then-series order.
        std::vector<int32_t> start((size_t)m->M + 1, 0), pos((size_t)L), occ((size_t)L);
        for (int64_t i = 0; i < L; ++i) ++start[(size_t)cols[i] + 1];
        for (int32_t j = 0; j < m->M; ++j) start[(size_t)j + 1] += start[(size_t)j];
        std::vector<int32_t> fill(start.begin(), start.end() - 1);
        for (int32_t b = 0; b < B; ++b)
            for (int32_t i = off[b]; i < off[b + 1]; ++i) {
                const int32_t k = fill[(size_t)cols[i]]++;
                pos[(size_t)k] = i;
                occ[(size_t)k] = b;
            }
        // CSR by series length: the candidates of length l, in order.
        std::vector<int32_t> lstart((size_t)m->M + 2, 0), lb((size_t)B);
        for (int32_t b = 0; b < B; ++b) ++lstart[(size_t)(off[b + 1] - off[b]) + 1];
        for (int32_t l = 0; l <= m->M; ++l) lstart[(size_t)l + 1] += lstart[(size_t)l];
        std::vector<int32_t> lfill(lstart.begin(), lstart.end() - 1);
        for (int32_t b = 0; b < B; ++b) lb[(size_t)lfill[(size_t)(off[b + 1] - off[b])]++] = b;
        if (!m->occ_start) MHIP(hipMalloc((void **)&m->occ_start, sizeof(int32_t) * ((size_t)m->M + 1)));
        if (!m->len_start) MHIP(hipMalloc((void **)&m->len_start, sizeof(int32_t) * ((size_t)m->M + 2)));
        MHIP(hipStreamSynchronize(m->stream));  // no kernel still reads the previous lists
        MHIP(hipMemcpy(m->occ_start, start.data(), sizeof(int32_t) * start.size(),
                       hipMemcpyHostToDevice));
        MHIP(hipMemcpy(m->occ_pos, pos.data(), sizeof(int32_t) * (size_t)L, hipMemcpyHostToDevice));
        MHIP(hipMemcpy(m->occ_b, occ.data(), sizeof(int32_t) * (size_t)L, hipMemcpyHostToDevice));
        MHIP(hipMemcpy(m->len_start, lstart.data(), sizeof(int32_t) * lstart.size(),
                       hipMemcpyHostToDevice));
        MHIP(hipMemcpy(m->len_b, lb.data(), sizeof(int32_t) * (size_t)B, hipMemcpyHostToDevice));
    }
    return EBIC_OK;
}

ebic_status forward(ebic_mlp *m, int32_t B) {
    const int32_t D = m->D, H = m->H;
    hipStream_t s = m->stream;
    if (m->fused) {
        ebic_status st = reserve_fused(m, B);
        if (st != EBIC_OK) return st;
        MHIP(mlp::fused_rows(fused_rows_args(m, B, false), s));
        return EBIC_OK;
    }
    const int32_t D2 = 2 * D;
    MHIP(mlp::pool_fwd(m->p + m->oE, m->p + m->oF, m->p + m->oT, m->p + m->oZ, D, m->off,
                       m->cols, B, m->X, m->Xb, s));
    mlp::Gemm l1{m->Xb, D2, 1, m->W1b, 1, D2, B, H, D2, 1, m->p + m->ob1, 1, m->Z1, m->H1b, nullptr};
    MHIP(mlp::gemm(l1, s));
    mlp::Gemm l2{m->H1b, H, 1, m->W2b, 1, H, B, H, H, 1, m->p + m->ob2, 1, m->Z2, m->H2b, nullptr};
    MHIP(mlp::gemm(l2, s));
    MHIP(mlp::out_fwd(m->H2b, m->w3b, m->p + m->ob3, B, H, m->y, s));
    return EBIC_OK;
}

// Gradients of the mean squared error into m->g (layout of the parameters).
ebic_status backward(ebic_mlp *m, int32_t B) {
    const int32_t D = m->D, D2 = 2 * m->D, H = m->H, S = splits_for(B);
    hipStream_t s = m->stream;
    float *g = m->g;
    MHIP(mlp::loss(m->y, m->t, B, m->dy, m->sq, s));
    MHIP(mlp::dw3(m->H2b, m->dy, B, H, S, m->ws, g + m->ow3, s));
    MHIP(mlp::colsum(m->dy, nullptr, B, 1, S, m->ws, g + m->ob3, s));
    MHIP(mlp::out_bwd(m->dy, m->w3b, m->Z2, B, H, m->dZ2, m->dZ2b, s));
    MHIP(mlp::colsum(m->dZ2, nullptr, B, H, S, m->ws, g + m->ob2, s));
    // dW2[n][k] = sum_b dZ2[b][n] h1[b][k]
    mlp::Gemm gw2{m->dZ2b, 1, H, m->H1b, H, 1, H, H, B, S, nullptr, 0, g + m->oW2, nullptr, m->ws};
    MHIP(mlp::gemm(gw2, s));
    // G1[b][k] = sum_n dZ2[b][n] W2[n][k]
    mlp::Gemm gh1{m->dZ2b, H, 1, m->W2b, H, 1, B, H, H, 1, nullptr, 0, m->G1, nullptr, nullptr};
    MHIP(mlp::gemm(gh1, s));
    MHIP(mlp::relu_bwd(m->G1, m->Z1, (int64_t)B * H, m->dZ1, m->dZ1b, s));
    MHIP(mlp::colsum(m->dZ1, nullptr, B, H, S, m->ws, g + m->ob1, s));
    // dW1[h][d] = sum_b dZ1[b][h] x[b][d]
    mlp::Gemm gw1{m->dZ1b, 1, H, m->Xb, D2, 1, H, D2, B, S, nullptr, 0, g + m->oW1, nullptr, m->ws};
    MHIP(mlp::gemm(gw1, s));
    // dX[b][d] = sum_h dZ1[b][h] W1[h][d]
    mlp::Gemm gx{m->dZ1b, H, 1, m->W1b, D2, 1, B, D2, H, 1, nullptr, 0, m->dX, nullptr, nullptr};
    MHIP(mlp::gemm(gx, s));
    MHIP(mlp::pool_bwd(m->dX, D, m->p + m->oF, m->p + m->oT, m->off, m->cols, m->occ_start,
                       m->occ_pos, m->occ_b, m->M, g + m->oE, g + m->oF, g + m->oT, s));
    MHIP(mlp::len_bwd(m->dX, D, m->len_start, m->len_b, m->M + 1, g + m->oZ, s));
    return EBIC_OK;
}

ebic_status refresh_bf16(ebic_mlp *m) {
    if (m->fused) {
        mlp::FusedUpdate u{};
        u.mode = mlp::kUpdateCast;
        u.n_params = m->n_params;
        u.oW1 = m->oW1;
        u.ob1 = m->ob1;
        u.oW2 = m->oW2;
        u.ob2 = m->ob2;
        u.ow3 = m->ow3;
        u.ob3 = m->ob3;
        u.p = m->p;
        u.W1b = m->W1b;
        u.W1bT = m->W1bT;
        u.W2b = m->W2b;
        u.W2bT = m->W2bT;
        u.w3b = m->w3b;
        MHIP(mlp::fused_update(u, m->stream));
        return EBIC_OK;
    }
    MHIP(mlp::cast_bf16(m->p + m->oW1, (int64_t)m->H * 2 * m->D, m->W1b, m->stream));
    MHIP(mlp::cast_bf16(m->p + m->oW2, (int64_t)m->H * m->H, m->W2b, m->stream));
    MHIP(mlp::cast_bf16(m->p + m->ow3, (int64_t)m->H, m->w3b, m->stream));
    return EBIC_OK;
}

float host_loss(ebic_mlp *m, int32_t B, ebic_status *st) {
    std::vector<float> sq((size_t)B);
    hipError_t e = hipMemcpyAsync(sq.data(), m->sq, sizeof(float) * (size_t)B,
                                  hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        *st = mfail(EBIC_E_DEVICE, std::string("loss copy: ") + hipGetErrorString(e));
        return 0.f;
    }
    double acc = 0.0;
    for (float v : sq) acc += v;
    *st = EBIC_OK;
    return (float)(acc / B);
}

struct SplitMix {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    float sym(float a) { return ((float)(next() >> 40) * (1.0f / 16777216.0f) * 2.f - 1.f) * a; }
};

}  // namespace

extern "C" {

void ebic_mlp_defaults(ebic_mlp_config *c) {
    if (!c) return;
    *c = ebic_mlp_config{sizeof(ebic_mlp_config), 32, 256, 1e-3f, 0.9f, 0.999f, 1e-8f};
}

ebic_status ebic_mlp_create(int32_t n_cols, const ebic_mlp_config *cfg, uint64_t seed,
                            int32_t device, ebic_mlp **out) {
    if (!out || n_cols < 1 || !cfg || cfg->struct_size < sizeof(ebic_mlp_config))
        return mfail(EBIC_E_ARG, "need n_cols >= 1, a config and out");
    if (cfg->embed_dim < 1 || cfg->hidden < 1 || cfg->embed_dim > 4096 || cfg->hidden > 4096)
        return mfail(EBIC_E_ARG, "embed_dim and hidden must be in [1, 4096]");
    *out = nullptr;
    std::unique_ptr<ebic_mlp> m(new (std::nothrow) ebic_mlp());
    if (!m) return mfail(EBIC_E_NOMEM, "cannot allocate model");
    m->device = device;
    m->M = n_cols;
    m->D = cfg->embed_dim;
    m->H = cfg->hidden;
    m->cfg = *cfg;
    const int64_t M = n_cols, D = m->D, H = m->H;
    m->oE = 0;
    m->oF = m->oE + M * D;
    m->oT = m->oF + M * D;
    m->oZ = m->oT + M * D;
    m->oW1 = m->oZ + (M + 1) * D;
    m->ob1 = m->oW1 + H * 2 * D;
    m->oW2 = m->ob1 + H;
    m->ob2 = m->oW2 + H * H;
    m->ow3 = m->ob2 + H;
    m->ob3 = m->ow3 + H;
    m->n_params = m->ob3 + 1;
    std::vector<float> init((size_t)m->n_params, 0.f);
    SplitMix rng{seed};
    for (int64_t i = 0; i < 3 * M * D; ++i) init[(size_t)(m->oE + i)] = rng.sym(1.f);
    for (int64_t i = 0; i < H * 2 * D; ++i)
        init[(size_t)(m->oW1 + i)] = rng.sym(std::sqrt(6.f / (2 * D)));
    for (int64_t i = 0; i < H * H; ++i) init[(size_t)(m->oW2 + i)] = rng.sym(std::sqrt(6.f / H));
    for (int64_t i = 0; i < H; ++i) init[(size_t)(m->ow3 + i)] = rng.sym(std::sqrt(3.f / H));
    auto fail = [&](hipError_t e, const char *w) {
        ebic_mlp_destroy(m.release());
        return mfail(e == hipErrorOutOfMemory ? EBIC_E_NOMEM : EBIC_E_DEVICE,
                     std::string(w) + ": " + hipGetErrorString(e));
    };
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = dalloc(m->p, m->n_params);
    if (e == hipSuccess) e = dalloc(m->g, m->n_params);
    if (e == hipSuccess) e = dalloc(m->m1, m->n_params);
    if (e == hipSuccess) e = dalloc(m->m2, m->n_params);
    if (e == hipSuccess) e = dalloc(m->W1b, H * 2 * D);
    if (e == hipSuccess) e = dalloc(m->W2b, H * H);
    if (e == hipSuccess) e = dalloc(m->w3b, H);
    m->fused = mlp::fused_shape(m->D, m->H);
    if (m->fused && e == hipSuccess) e = dalloc(m->W1bT, H * 2 * D);
    if (m->fused && e == hipSuccess) e = dalloc(m->W2bT, H * H);
    if (e != hipSuccess) return fail(e, "model buffers");
    ebic_status st = ebic_mlp_set_params(m.get(), init.data());
    if (st != EBIC_OK) {
        ebic_mlp_destroy(m.release());
        return st;
    }
    *out = m.release();
    return EBIC_OK;
}

ebic_status ebic_mlp_destroy(ebic_mlp *m) {
    if (!m) return EBIC_OK;
    (void)hipSetDevice(m->device);
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    void *bufs[] = {m->p, m->g, m->m1, m->m2, m->W1b, m->W2b, m->w3b, m->off, m->cols,
                    m->occ_start, m->occ_pos, m->occ_b, m->len_start, m->len_b, m->X, m->Z1, m->Z2, m->y, m->t, m->dy, m->sq,
                    m->dZ2, m->G1, m->dZ1, m->dX, m->Xb, m->H1b, m->H2b, m->dZ2b, m->dZ1b, m->ws,
                    m->W1bT, m->W2bT, m->XrT, m->H1rT, m->dZ2rT, m->dZ1rT, m->fdX, m->ws1,
                    m->ws2, m->pw3, m->pb2, m->pb1, m->pb3};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
    return EBIC_OK;
}

int64_t ebic_mlp_param_count(const ebic_mlp *m) { return m ? m->n_params : 0; }

ebic_status ebic_mlp_get_params(const ebic_mlp *m, float *params) {
    if (!m || !params) return mfail(EBIC_E_ARG, "null argument");
    MHIP(hipSetDevice(m->device));
    MHIP(hipStreamSynchronize(m->stream));
    MHIP(hipMemcpy(params, m->p, sizeof(float) * (size_t)m->n_params, hipMemcpyDeviceToHost));
    return EBIC_OK;
}

ebic_status ebic_mlp_set_params(ebic_mlp *m, const float *params) {
    if (!m || !params) return mfail(EBIC_E_ARG, "null argument");
    MHIP(hipSetDevice(m->device));
    MHIP(hipStreamSynchronize(m->stream));
    MHIP(hipMemcpy(m->p, params, sizeof(float) * (size_t)m->n_params, hipMemcpyHostToDevice));
    MHIP(hipMemset(m->m1, 0, sizeof(float) * (size_t)m->n_params));
    MHIP(hipMemset(m->m2, 0, sizeof(float) * (size_t)m->n_params));
    m->step = 0;
    ebic_status st = refresh_bf16(m);
    if (st != EBIC_OK) return st;
    MHIP(hipStreamSynchronize(m->stream));
    return EBIC_OK;
}

ebic_status ebic_mlp_predict(ebic_mlp *m, const int32_t *offsets, const int32_t *cols, int32_t B,
                             float *y) {
    if (!m || !y) return mfail(EBIC_E_ARG, "null argument");
    MHIP(hipSetDevice(m->device));
    ebic_status st = upload(m, offsets, cols, B, nullptr, false);
    if (st != EBIC_OK) return st;
    if ((st = forward(m, B)) != EBIC_OK) return st;
    MHIP(hipMemcpyAsync(y, m->y, sizeof(float) * (size_t)B, hipMemcpyDeviceToHost, m->stream));
    MHIP(hipStreamSynchronize(m->stream));
    return EBIC_OK;
}

ebic_status ebic_mlp_gradients(ebic_mlp *m, const int32_t *offsets, const int32_t *cols,
                               int32_t B, const float *target, float *grad, float *loss) {
    if (!m || !target || !grad) return mfail(EBIC_E_ARG, "null argument");
    MHIP(hipSetDevice(m->device));
    ebic_status st = upload(m, offsets, cols, B, target, true);
    if (st != EBIC_OK) return st;
    if (m->fused) {
        if ((st = reserve_fused(m, B)) != EBIC_OK ||
            (st = fused_step(m, B, mlp::kUpdateGradients, 1.f, 1.f)) != EBIC_OK)
            return st;
    } else if ((st = forward(m, B)) != EBIC_OK || (st = backward(m, B)) != EBIC_OK) {
        return st;
    }
    MHIP(hipMemcpyAsync(grad, m->g, sizeof(float) * (size_t)m->n_params, hipMemcpyDeviceToHost,
                        m->stream));
    const float l = host_loss(m, B, &st);
    if (st != EBIC_OK) return st;
    if (loss) *loss = l;
    return EBIC_OK;
}

ebic_status ebic_mlp_train(ebic_mlp *m, const int32_t *offsets, const int32_t *cols, int32_t B,
                           const float *target, int32_t steps, float *loss) {
    if (!m || !target) return mfail(EBIC_E_ARG, "null argument");
    if (steps < 1) return mfail(EBIC_E_ARG, "steps must be >= 1");
    MHIP(hipSetDevice(m->device));
    ebic_status st = upload(m, offsets, cols, B, target, true);
    if (st != EBIC_OK) return st;
    if (m->fused && (st = reserve_fused(m, B)) != EBIC_OK) return st;
    for (int32_t k = 0; k < steps; ++k) {
        if (m->fused) {
            m->step += 1;
            const float c1 = 1.f - std::pow(m->cfg.beta1, (float)m->step);
            const float c2 = 1.f - std::pow(m->cfg.beta2, (float)m->step);
            if ((st = fused_step(m, B, mlp::kUpdateAdam, c1, c2)) != EBIC_OK) return st;
            continue;
        }
        if ((st = forward(m, B)) != EBIC_OK || (st = backward(m, B)) != EBIC_OK) return st;
        m->step += 1;
        const float c1 = 1.f - std::pow(m->cfg.beta1, (float)m->step);
        const float c2 = 1.f - std::pow(m->cfg.beta2, (float)m->step);
        MHIP(mlp::adam(m->p, m->g, m->m1, m->m2, m->n_params, m->cfg.lr, m->cfg.beta1,
                       m->cfg.beta2, m->cfg.eps, c1, c2, m->stream));
        if ((st = refresh_bf16(m)) != EBIC_OK) return st;
    }
    m->last_B = B;
    if (!loss) return EBIC_OK;   // the steps stay queued on the network's stream
    const float l = host_loss(m, B, &st);  // loss before the last step
    if (st != EBIC_OK) return st;
    *loss = l;
    return EBIC_OK;
}

}  // extern "C"

namespace ebic {
ebic_status mlp_last_loss(ebic_mlp *m, float *loss) {
    if (!m || !loss || m->last_B < 1) return mfail(EBIC_E_STATE, "no training call to report");
    MHIP(hipSetDevice(m->device));
    ebic_status st = EBIC_OK;
    const float l = host_loss(m, m->last_B, &st);
    if (st == EBIC_OK) *loss = l;
    return st;
}
}  // namespace ebic

extern "C" {

ebic_status ebic_mlp_train_step(ebic_mlp *m, const int32_t *offsets, const int32_t *cols,
                                int32_t B, const float *target, float *loss) {
    return ebic_mlp_train(m, offsets, cols, B, target, 1, loss);
}

}  // extern "C"
