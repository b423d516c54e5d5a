// Learned sampling proposal: layout of the network's parameters and the
// kernel launchers.  Network (H = 64 hidden units, L = 3 rounds):
//   E     = diag(1/||a_j||) [A; B]
//   Fv_i  = [x_i, 4 x_i (1 - x_i), c~_i / max|c~|, 1]
//   Fc_j  = [y_j / (1 + |y_j|), r~_j / max|r~|, [row j is an equality], 1]
//   Hv = relu(Fv Uv + uv), Hc = relu(Fc Uc + uc)
//   repeat L times:  Hc = relu([Hc | E Hv] [Wcc; Wcv] + bc)
//                    Hv = relu([Hv | E^T Hc] [Wvv; Wvc] + bv)
//   logit = Hv wo + bo, p = sigmoid(logit), loss = mean BCE(logit, incumbent)
// Flat FP32 parameter vector, in this order: Uv[4][64], uv[64], Uc[4][64],
// uc[64], then per round {Wcc[64][64], Wcv[64][64], bc[64], Wvv[64][64],
// Wvc[64][64], bv[64]} (W[in][out]), then wo[64], bo.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace gfors {

constexpr int kGnnH = 64;
constexpr int kGnnL = 3;
constexpr int kGnnOffUv = 0;
constexpr int kGnnOffuv = 256;
constexpr int kGnnOffUc = 320;
constexpr int kGnnOffuc = 576;
constexpr int kGnnOffLayer = 640;
constexpr int kGnnLayerSize = 2 * (2 * 64 * 64 + 64);   // 16512
constexpr int kGnnOffwo = kGnnOffLayer + kGnnL * kGnnLayerSize;   // 50176
constexpr int kGnnOffbo = kGnnOffwo + 64;                          // 50240
constexpr int kGnnNumParams = kGnnOffbo + 1;                       // 50241
constexpr int kGnnMaxParts = 256;
constexpr int kGnnHeavyLen = 1024;   // SpMM node classes: heavy from this many entries
constexpr int kGnnShortLen = 16;     // short up to this many

void launch_gnn_embed(hipStream_t s, int64_t n, int64_t m, int m1, const float *x, const float *y,
                      const float *ct, const float *rt, float ictmax, float irtmax,
                      const float *theta, uint16_t *Hv, uint16_t *Hc);
// nodes in `order` (longest first): the first nheavy have >= 1024 entries, the
// next nmedium more than 16, the rest at most 16
void launch_gnn_spmm(hipStream_t s, bool rows, bool in_bf16, int out_mode, int64_t nrows,
                     const int *order, int nheavy, int nmedium, const int *rp, const int *ci,
                     const int *val, const float *rowinv, const void *in, void *out);
void launch_gnn_dense_fwd(hipStream_t s, int64_t N, const uint16_t *A1, const uint16_t *A2,
                          const uint16_t *BT, const float *bias, uint16_t *out);
void launch_gnn_dense_bwd_in(hipStream_t s, int64_t N, const uint16_t *dZ, const uint16_t *Wrm,
                             float *dA1, float *dA2, int accumulate);
void launch_gnn_wgrad(hipStream_t s, int64_t N, const uint16_t *A1, const uint16_t *A2,
                      const uint16_t *dZ, float *part, int max_parts, float *dW1, float *dW2);
void launch_gnn_mask(hipStream_t s, int64_t N, const float *dOut, const uint16_t *Out,
                     uint16_t *dZ, float *part, int max_parts, float *db);
void launch_gnn_out(hipStream_t s, int64_t n, const uint16_t *Hv, const float *theta, float *logit,
                    float *p, const float *target, float *dHv, float *part, int max_parts,
                    float *grad, float *loss_out);
void launch_gnn_embed_bwd(hipStream_t s, int64_t N, int is_var, int m1, const float *xy,
                          const float *crt, float iscale, const uint16_t *H0, const float *dH,
                          float *part, int max_parts, float *gU, float *gu);
void launch_gnn_pack(hipStream_t s, const float *theta, uint16_t *wf, uint16_t *wb);
void launch_gnn_adam(hipStream_t s, int np, float *theta, const float *g, float *m, float *v,
                     float lr, float b1, float b2, float eps, float c1, float c2);

}  // namespace gfors
