// mlp.h -- kernels of the learned gate (mlp.hip) and its host object.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chx_internal.h"

namespace chx {

constexpr int MLP_IN = 6;         // features
constexpr int MLP_INP = 16;       // padded input width
constexpr int MLP_H = 256;        // hidden width
constexpr int MLP_OUTP = 16;      // padded logits (2 used)
constexpr int MLP_STAT_BLOCKS = 256;
// flat parameter layout
constexpr int64_t MLP_W1 = 0;
constexpr int64_t MLP_B1 = MLP_W1 + (int64_t)MLP_INP * MLP_H;
constexpr int64_t MLP_W2 = MLP_B1 + MLP_H;
constexpr int64_t MLP_B2 = MLP_W2 + (int64_t)MLP_H * MLP_H;
constexpr int64_t MLP_W3 = MLP_B2 + MLP_H;
constexpr int64_t MLP_B3 = MLP_W3 + (int64_t)MLP_H * MLP_OUTP;
constexpr int64_t MLP_NPARAM = MLP_B3 + MLP_OUTP;
// columns of a training block's partial sums: b1 | b2 | b3 | loss, padded
// to a multiple of 16
constexpr int MLP_BIAS_LOSS = 2 * MLP_H + MLP_OUTP;
constexpr int MLP_BIAS_COLS = MLP_BIAS_LOSS + 16;
// regions of the training pass's BF16 weights in MFMA operand order (pbF)
constexpr int64_t MLP_F_W1 = 0;                                      // W1, forward
constexpr int64_t MLP_F_W2 = MLP_F_W1 + (int64_t)MLP_INP * MLP_H;    // W2, forward
constexpr int64_t MLP_F_W2T = MLP_F_W2 + (int64_t)MLP_H * MLP_H;     // W2, backward
constexpr int64_t MLP_F_W3 = MLP_F_W2T + (int64_t)MLP_H * MLP_H;     // W3, forward
constexpr int64_t MLP_F_W3T = MLP_F_W3 + (int64_t)MLP_H * MLP_OUTP;  // W3, backward
constexpr int64_t MLP_NFRAG = MLP_F_W3T + (int64_t)MLP_H * MLP_OUTP;

// C = A B (+ bias) (+ C): BF16 operands at any strides, FP32 result.
// work (work_len floats, may be null; needs parts) holds split-K partial
// products.
// Epilogue EPI_GELU (no accumulate): also stores GELU(C) in BF16 to Cb
// (C's row stride).
enum { EPI_NONE = 0, EPI_GELU = 1 };
hipError_t mlp_gemm(const uint16_t *A, int64_t a_r, int64_t a_c, const uint16_t *B, int64_t b_r,
                    int64_t b_c, float *C, int64_t ldc, int M, int N, int K, const float *bias,
                    int accumulate, hipStream_t s, float *work = nullptr, int64_t work_len = 0,
                    int epi = EPI_NONE, uint16_t *Cb = nullptr, int *parts = nullptr);
// With parts given (no bias, no accumulate, ldc == N): a product split over
// K leaves its parts in work[z][M][N] for the caller to add and *parts = S
// (the number of parts); with *parts == 1 the product is in C.
// Split-K workspaces of the training pass (floats): up to 32 parts of the
// 256 x 256 weight gradient, 64 of the 16 x 256 and 256 x 16 ones
constexpr int64_t MLP_SPLITK_WORK = (int64_t)32 * MLP_H * MLP_H;
constexpr int64_t MLP_SPLITK_WORK_SMALL = (int64_t)64 * MLP_H * MLP_OUTP;
// The row-local part of a training batch of B rows (multiple of 16): rows
// (a i + c) mod n of the batch positions start + i (-1 at or past n), their
// z-scored inputs, the forward pass, softmax cross-entropy against labels
// (gradient scaled by inv) and the activation
// gradients; X, A1, A2, dZ3, dZ2, dZ1 (BF16, feature-major: row r of
// feature j at j ld + r, ld >= B a multiple of 16) are left for the weight
// gradients and each 16-row block's column sums of dZ1 | dZ2 | dZ3 and its
// loss in bpart[B / 16][MLP_BIAS_COLS] for mlp_bias_grad.  pbF: the weights' BF16
// copy in MFMA operand order (mlp_weights_bf16).
struct MlpRowsArgs {
  int64_t n, start, ld;
  uint64_t a, c;
  const float *feat, *mean, *istd;
  const int8_t *labels;
  float inv;
  const float *p;
  const uint16_t *pb, *pbF;
  uint16_t *X, *A1b, *A2b, *dZ3b, *dZ2b, *dZ1b;
  float *bpart;
};
hipError_t mlp_train_rows(const MlpRowsArgs &r, int B, hipStream_t s);
// grad's b1, b2, b3 = the sums of the nblk blocks' partials (in order);
// their loss sum is added to *loss_sum (if not null)
hipError_t mlp_bias_grad(const float *bpart, int nblk, float *grad, float *loss_sum,
                         hipStream_t s);
hipError_t mlp_apply_mask(float *p, const uint8_t *mask, int64_t n, hipStream_t s);
hipError_t mlp_fill(float *p, int64_t n, float v, hipStream_t s);
hipError_t gate_select(int64_t n, const int *status, const int8_t *label1, const float *pc,
                       const float *conf, float conf_min, int8_t *label, uint8_t *source,
                       uint8_t *keep, float *conf_out, unsigned long long *counts,
                       hipStream_t s);
hipError_t gate_scatter(int64_t n2, const int64_t *orbit, const int8_t *label2, int8_t *label,
                        hipStream_t s);
// Split-K parts of the three weight gradients (sN parts at wN; sN <= 1:
// the gradient is already in g).
struct GradParts {
  const float *w1, *w2, *w3;
  int s1, s2, s3;
};
// g = the batch's gradient (adding the weight gradients' parts); with step
// set, AdamW on the FP32 masters p (entries with mask set), pb receiving
// their BF16 copies and pbF the weights' operand-order BF16 copies.
hipError_t mlp_grad_step(const GradParts &gp, float *p, uint16_t *pb, uint16_t *pbF, float *g,
                         float *m, float *v, const uint8_t *mask, int step, float lr, float b1,
                         float b2, float eps, float wd, float bc1, float bc2, hipStream_t s);
// pb = BF16 of all MLP_NPARAM parameters; pbF (MLP_NFRAG entries) = BF16
// of the weights in the training pass's MFMA operand order
hipError_t mlp_weights_bf16(const float *p, uint16_t *pb, uint16_t *pbF, hipStream_t s);
hipError_t mlp_batch_input(const float *feat, const int64_t *rows, int B, int64_t n_valid,
                           const float *mean, const float *istd, uint16_t *X, hipStream_t s);
hipError_t mlp_init_params(float *p, uint8_t *mask, uint64_t seed, hipStream_t s);
hipError_t mlp_feature_stats(const float *feat, int64_t n, float *mean, float *istd,
                             double *partials, hipStream_t s);
hipError_t mlp_infer_out(const float *Z3, int B, float *pc, float *conf, hipStream_t s);
hipError_t mlp_features(const double *x0, const double *ld, const double *lg, double t, int64_t n,
                        float *out, hipStream_t s);

}  // namespace chx
