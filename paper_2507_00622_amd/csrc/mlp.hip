// mlp.hip -- the learned gate: a 6 -> 256 -> 256 -> 2 perceptron with erf
// GELU activations, trained and evaluated on the GPU by these kernels.
//
// Layout.  Inputs are padded to 16 features and the two logits to 16
// columns so that every product is a whole number of 16x16x16 MFMA tiles;
// the padded weights start at zero and receive zero gradients, so they stay
// zero.  Master parameters are FP32 (flat: W1[16][256], b1[256],
// W2[256][256], b2[256], W3[256][16], b3[16]); the products read BF16 copies
// of weights and activations and accumulate in FP32
// (v_mfma_f32_16x16x16_bf16).  Training: softmax cross-entropy on the two
// logits, AdamW on the FP32 masters.
#include <math.h>

#include "mlp.h"

namespace chx {

namespace {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (finite inputs; NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// erf(z / sqrt 2) given e = exp(-z^2 / 2): Abramowitz and Stegun 7.1.26,
// erf(x) = 1 - (a1 t + ... + a5 t^5) exp(-x^2), t = 1 / (1 + p x) for x >= 0
// (absolute error at most 1.5e-7), odd in x.  Free of branches, so the 16
// activations of a lane in the product's epilogue interleave.
__device__ __forceinline__ float erf_scaled(float z, float e) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * x);
  const float poly =
      t * (0.254829592f +
           t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  return copysignf(1.0f - poly * e, z);
}
__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erf_scaled(z, __expf(-0.5f * z * z)));
}
__device__ __forceinline__ float gelu_grad(float z) {
  const float e = __expf(-0.5f * z * z);
  return 0.5f * (1.0f + erf_scaled(z, e)) + z * 0.39894228040143268f * e;
}

// C[M][N] (fp32, row stride ldc) = A B (+ bias[col]) (+ C if accumulate),
// A(i,k) = A[i*a_r + k*a_c], B(k,j) = B[k*b_r + j*b_c], both BF16; M, N, K
// multiples of 16.  A block of 4 wavefronts computes a BM x BN tile of C,
// (64, 64), (16, 64) or (64, 16) (rows past M are not stored).  K goes in
// chunks of 32: the block stages the chunk of A (BM x 32) and of B
// (32 x BN) in LDS with k contiguous (As[i][k], Bs[j][k], rows padded to
// 40 elements against bank conflicts), reading global memory along
// whichever index has unit stride, 8 elements (16 bytes) per load where VEC
// says the addresses allow it, the next chunk's loads in flight during this
// chunk's products; rows past M are staged as zeros, k past the end of the
// block's K range is neither staged nor multiplied.  Each
// wavefront takes its 16 x 16 tiles' fragments from LDS (4 consecutive k
// per lane, one 8-byte read) and issues v_mfma_f32_16x16x16bf16_1k per tile
// and 16 k: lane l holds A[l % 16][4 (l / 16) + e], B[4 (l / 16) + e][l % 16]
// and, after, D[4 (l / 16) + r][l % 16].  Split K: block z of gridDim.z
// takes chunks [z cpc, (z + 1) cpc) and, when gridDim.z > 1, writes its
// partial tile to work[z][M][N] for the caller to add in order of z.  Epilogue EPI_GELU
// (no split): Z = AB + bias to C and its activation GELU(Z) in BF16 to Cb
// (C's row stride).
constexpr int GBK = 32, GPAD = GBK + 8;

template <int BM, int BN, bool VEC, int EPI>
__global__ void __launch_bounds__(256) gemm_tile_kernel(const uint16_t *A, int64_t a_r,
                                                        int64_t a_c, const uint16_t *B,
                                                        int64_t b_r, int64_t b_c, float *C,
                                                        int64_t ldc, int M, int N, int K,
                                                        int cpc, const float *bias,
                                                        int accumulate, float *work,
                                                        uint16_t *Cb) {
  // wavefronts: (64, 64) 2 x 2 of 2 x 2 tiles; (64, 16) 4 x 1 and (16, 64)
  // 1 x 4 of one tile
  constexpr int WGM = BM == 64 && BN == 64 ? 2 : (BM == 64 ? 4 : 1);
  constexpr int WGN = 4 / WGM;
  constexpr int TM = BM / (16 * WGM), TN = BN / (16 * WGN);
  __shared__ __align__(16) uint16_t As[BM][GPAD];
  __shared__ __align__(16) uint16_t Bs[BN][GPAD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave / WGN, wn = wave % WGN;
  const int row0 = blockIdx.y * BM, col0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * cpc * GBK;
  const int kend = min(K, kbeg + cpc * GBK);
  const int li = lane & 15, lk = 4 * (lane >> 4);
  float4_t acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = (float4_t){0.f, 0.f, 0.f, 0.f};
  // Runs of 8 elements of the A chunk and of the B chunk, run t of A being
  // (i, kk) along k when a_c == 1, else along i (B alike: (j, kk) along k
  // when b_r == 1, else along j); thread tid takes runs tid, tid + 256, ...
  // M and K are multiples of 16 and runs start at multiples of 8, so a run
  // is wholly inside or wholly outside the matrix.
  constexpr int RA = BM * GBK / 8, RB = BN * GBK / 8;
  constexpr int NA = (RA + 255) / 256, NB = (RB + 255) / 256;
  const bool a_k = a_c == 1, b_k = b_r == 1;
  const int64_t a_step = a_k ? 1 : a_r, b_step = b_k ? 1 : b_c;
  auto run_a = [&](int q, int &i, int &k) {
    const int t = tid + 256 * q;
    i = a_k ? t / (GBK / 8) : (t % (BM / 8)) * 8;
    k = a_k ? (t % (GBK / 8)) * 8 : t / (BM / 8);
  };
  auto run_b = [&](int q, int &j, int &k) {
    const int t = tid + 256 * q;
    j = b_k ? t / (GBK / 8) : (t % (BN / 8)) * 8;
    k = b_k ? (t % (GBK / 8)) * 8 : t / (BN / 8);
  };
  auto load_run = [](const uint16_t *src, int64_t step, bool vec) {
    uint4 v;
    if (vec && step == 1) {
      v = *(const uint4 *)src;
    } else {
      uint16_t *h = (uint16_t *)&v;
#pragma unroll
      for (int e = 0; e < 8; ++e) h[e] = src[(int64_t)e * step];
    }
    return v;
  };
  uint4 va[NA], vb[NB];
  // every run of the chunk at k0 goes out before any is waited for
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int i, k;
      run_a(q, i, k);
      va[q] = (tid + 256 * q < RA && row0 + i < M && k0 + k < kend)
                  ? load_run(A + (int64_t)(row0 + i) * a_r + (int64_t)(k0 + k) * a_c, a_step, VEC)
                  : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int j, k;
      run_b(q, j, k);
      vb[q] = (tid + 256 * q < RB && k0 + k < kend)
                  ? load_run(B + (int64_t)(k0 + k) * b_r + (int64_t)(col0 + j) * b_c, b_step, VEC)
                  : make_uint4(0, 0, 0, 0);
    }
  };
  load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += GBK) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      if (tid + 256 * q >= RA) continue;
      int i, k;
      run_a(q, i, k);
      if (k0 + k >= kend) continue;
      if (a_k) {
        *(uint4 *)&As[i][k] = va[q];
      } else {
        const uint16_t *h = (const uint16_t *)&va[q];
#pragma unroll
        for (int e = 0; e < 8; ++e) As[i + e][k] = h[e];
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (tid + 256 * q >= RB) continue;
      int j, k;
      run_b(q, j, k);
      if (k0 + k >= kend) continue;
      if (b_k) {
        *(uint4 *)&Bs[j][k] = vb[q];
      } else {
        const uint16_t *h = (const uint16_t *)&vb[q];
#pragma unroll
        for (int e = 0; e < 8; ++e) Bs[j + e][k] = h[e];
      }
    }
    __syncthreads();
    // the next chunk's loads go out before this chunk's products
    if (k0 + GBK < kend) load(k0 + GBK);
    // the products stop at the end of the staged k (a multiple of 16)
    const int kn = min(GBK, kend - k0);
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 16) {
      if (kk >= kn) break;
      short4_t af[TM], bfr[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a)
        af[a] = *(const short4_t *)&As[(wm * TM + a) * 16 + li][kk + lk];
#pragma unroll
      for (int b = 0; b < TN; ++b)
        bfr[b] = *(const short4_t *)&Bs[(wn * TN + b) * 16 + li][kk + lk];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bfr[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  if (gridDim.z > 1) {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = row0 + (wm * TM + a) * 16 + lk + r, j = col0 + (wn * TN + b) * 16 + li;
          if (i < M) work[((int64_t)blockIdx.z * M + i) * N + j] = acc[a][b][r];
        }
    return;
  }
  // every load of the epilogue (bias, the C accumulated onto) goes out
  // before its first store, so one wait covers them all
  float x[TM][TN][4];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int j = col0 + (wn * TN + b) * 16 + li;
      const float bj = bias ? bias[j] : 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row0 + (wm * TM + a) * 16 + lk + r;
        const int64_t e = (int64_t)i * ldc + j;
        if (bias) acc[a][b][r] += bj;
        if constexpr (EPI == EPI_NONE) x[a][b][r] = (accumulate && i < M) ? C[e] : 0.f;
      }
    }
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row0 + (wm * TM + a) * 16 + lk + r, j = col0 + (wn * TN + b) * 16 + li;
        if (i >= M) continue;
        const float v = acc[a][b][r];
        const int64_t e = (int64_t)i * ldc + j;
        if constexpr (EPI == EPI_GELU) {
          C[e] = v;
          Cb[e] = f2bf(gelu(v));
        } else {
          C[e] = accumulate ? x[a][b][r] + v : v;
        }
      }
}

// t = t + p[0] + p[stride] + ... + p[(count - 1) stride], added in that
// order; the loads go out G at a time ahead of the additions.
template <int G = 8>
__device__ __forceinline__ float ordered_sum(float t, const float *p, int64_t stride, int count) {
  for (int c = 0; c < count; c += G) {
    float v[G];
#pragma unroll
    for (int e = 0; e < G; ++e) v[e] = c + e < count ? p[(int64_t)(c + e) * stride] : 0.f;
#pragma unroll
    for (int e = 0; e < G; ++e)
      if (c + e < count) t += v[e];
  }
  return t;
}

// four consecutive BF16 values as one 8-byte store (p 8-byte aligned)
__device__ __forceinline__ void store4(uint16_t *p, const uint16_t (&h)[4]) {
  *(uint2 *)p = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16),
                           (uint32_t)h[2] | ((uint32_t)h[3] << 16));
}

// Block barrier for LDS traffic only: waits for this wavefront's LDS
// accesses, not for its global loads in flight (which __syncthreads would
// drain); the memory clobber keeps the compiler from moving accesses across.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The training pass's BF16 weights in MFMA operand order: the B operand of
// 16-column tile jt and k-step ks of a product is 64 lanes x 4 consecutive k
// (lane l: column 16 jt + l % 16, k = 16 ks + 4 (l / 16) + e), one
// contiguous 512-byte run, so a wavefront's operand load is one coalesced
// read.  Entry (jt, ks, l, e) of a product with KS k-steps lies at
// ((jt KS + ks) 64 + l) 4 + e of its region.  Regions: layer 1 forward
// (B = W1), layer 2 forward (W2) and backward (W2^T), layer 3 forward (W3)
// and backward (W3^T).
__device__ __forceinline__ int64_t frag_at(int64_t base, int ks_count, int jt, int ks, int k4,
                                           int col16) {
  // k4 = k mod 16 within the k-step, col16 = column mod 16
  return base + ((int64_t)(jt * ks_count + ks) * 64 + (k4 >> 2) * 16 + col16) * 4 + (k4 & 3);
}
// Positions of weight entry i in the operand-order copy (second one for
// the weights used by both passes; -1 where there is none).
__device__ __forceinline__ void mlp_fpos(int64_t i, int64_t &f0, int64_t &f1) {
  f0 = f1 = -1;
  if (i < MLP_B1) {  // W1[k][j], k < 16
    const int k = (int)(i / MLP_H), j = (int)(i % MLP_H);
    f0 = frag_at(MLP_F_W1, 1, j >> 4, 0, k, j & 15);
  } else if (i >= MLP_W2 && i < MLP_B2) {  // W2[k][j]
    const int k = (int)((i - MLP_W2) / MLP_H), j = (int)((i - MLP_W2) % MLP_H);
    f0 = frag_at(MLP_F_W2, MLP_H / 16, j >> 4, k >> 4, k & 15, j & 15);
    f1 = frag_at(MLP_F_W2T, MLP_H / 16, k >> 4, j >> 4, j & 15, k & 15);
  } else if (i >= MLP_W3 && i < MLP_B3) {  // W3[k][j], j < 16
    const int k = (int)((i - MLP_W3) / MLP_OUTP), j = (int)((i - MLP_W3) % MLP_OUTP);
    f0 = frag_at(MLP_F_W3, MLP_H / 16, 0, k >> 4, k & 15, j);
    f1 = frag_at(MLP_F_W3T, 1, k >> 4, 0, j, k & 15);
  }
}

// The row-local part of one training batch, 16 rows per block of TR_W
// wavefronts (the weight gradients, sums over all rows, follow as products):
//   rows: batch position i -> (a i + c) mod n (-1 at or past n), z-scored
//     BF16 inputs X;
//   Z1 = X W1 + b1, A1 = GELU(Z1); Z2 = A1 W2 + b2, A2 = GELU(Z2);
//   Z3 = A2 W3 + b3; softmax cross-entropy on the two logits: dZ3 =
//     (softmax - onehot(label)) inv, the block's loss (rows without a
//     label 0 or 1 contribute nothing);
//   dZ2 = (dZ3 W3^T) GELU'(Z2); dZ1 = (dZ2 W2^T) GELU'(Z1).
// Wavefront w of TR_W computes columns 16 TR_T w .. 16 TR_T (w + 1) - 1 of
// the 256-wide layers (TR_T 16 x 16 tiles) and keeps Z1, Z2 in registers;
// the activation entering each product waits in LDS (16 x 256 BF16).  The
// weights come from the operand-order BF16 copy pbF, one coalesced 8-byte
// load per lane and operand; the MFMAs run over k in ascending order as in
// gemm_tile_kernel, so the products equal those of separate
// gemm_tile_kernel launches bit for bit.  Block barriers wait for LDS only.
// The logits and the softmax are the first wavefront's.  Outputs for
// the weight gradients: X, A1, A2, dZ3, dZ2, dZ1 (BF16) feature-major,
// element (row r, feature j) at j ld + r, so that the weight-gradient
// products A^T dZ read both operands along K (the rows); for the
// bias gradients the block's column sums of dZ1, dZ2, dZ3 (FP32: per lane
// its 4 rows in order, then the 4 lane groups in order; dZ3's 16 rows in
// order) and its loss to bpart[block][b1 256 | b2 256 | b3 16 | loss 1].
constexpr int TR_LD = MLP_H + 8;  // LDS row of a 256-wide BF16 activation
// wavefronts per block and 16-column tiles per wavefront of the 256-wide
// layers
constexpr int TR_W = 8, TR_T = 16 / TR_W;
__global__ void __launch_bounds__(64 * TR_W) train_rows_kernel(const MlpRowsArgs t) {
  __shared__ __align__(16) uint16_t Xs[16][24];
  __shared__ __align__(16) uint16_t Gs[16][24];
  __shared__ __align__(16) uint16_t As[16][TR_LD];
  __shared__ float Zs[16][17];
  __shared__ float Ps2[4][MLP_H], Ps1[4][MLP_H];  // column sums per lane group
  __shared__ int64_t srcs[16];
  float *bp = t.bpart + (int64_t)blockIdx.x * MLP_BIAS_COLS;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 16;
  const int cw = wave * 16 * TR_T;
  const float4_t zero = {0.f, 0.f, 0.f, 0.f};
  // the weight operands do not depend on the rows: W2's and W3's go out
  // first, W2's backward ones once the forward product is done, each in
  // flight under the work before its product
  short4_t wf[MLP_H / 16][TR_T], w3f[MLP_H / 16], w3b[TR_T];
#pragma unroll
  for (int b = 0; b < TR_T; ++b)
    w3b[b] = *(const short4_t *)&t.pbF[MLP_F_W3T + ((TR_T * wave + b) * 64 + lane) * 4];
#pragma unroll
  for (int ks = 0; ks < MLP_H / 16; ++ks) {
#pragma unroll
    for (int b = 0; b < TR_T; ++b)
      wf[ks][b] =
          *(const short4_t *)&t.pbF[MLP_F_W2 + (((TR_T * wave + b) * 16 + ks) * 64 + lane) * 4];
    w3f[ks] = *(const short4_t *)&t.pbF[MLP_F_W3 + (ks * 64 + lane) * 4];
  }
  if (tid < 256) {
    const int i = tid >> 4, k = tid & 15;
    const int64_t pos = t.start + r0 + i;
    const int64_t src =
        pos < t.n ? (int64_t)((t.a * (uint64_t)pos + t.c) % (uint64_t)t.n) : -1;
    if (k == 0) srcs[i] = src;
    const float v =
        (src >= 0 && k < MLP_IN) ? (t.feat[src * MLP_IN + k] - t.mean[k]) * t.istd[k] : 0.f;
    const uint16_t h = f2bf(v);
    Xs[i][k] = h;
    t.X[(int64_t)k * t.ld + r0 + i] = h;
  }
  lds_barrier();
  // layer 1 (one k-step)
  float4_t z1[TR_T], z2[TR_T];
  {
    const short4_t x = *(const short4_t *)&Xs[li][4 * lq];
#pragma unroll
    for (int b = 0; b < TR_T; ++b) {
      const short4_t w =
          *(const short4_t *)&t.pbF[MLP_F_W1 + ((TR_T * wave + b) * 64 + lane) * 4];
      z1[b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, w, zero, 0, 0, 0);
    }
  }
#pragma unroll
  for (int b = 0; b < TR_T; ++b) {
    const int j = cw + 16 * b + li;
    const float bj = t.p[MLP_B1 + j];
    uint16_t h[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      z1[b][r] += bj;
      h[r] = f2bf(gelu(z1[b][r]));
      As[4 * lq + r][j] = h[r];
    }
    store4(t.A1b + (int64_t)j * t.ld + r0 + 4 * lq, h);
  }
  lds_barrier();
  // layer 2
#pragma unroll
  for (int b = 0; b < TR_T; ++b) z2[b] = zero;
#pragma unroll
  for (int ks = 0; ks < MLP_H / 16; ++ks) {
    const short4_t x = *(const short4_t *)&As[li][16 * ks + 4 * lq];
#pragma unroll
    for (int b = 0; b < TR_T; ++b)
      z2[b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, wf[ks][b], z2[b], 0, 0, 0);
  }
#pragma unroll
  for (int ks = 0; ks < MLP_H / 16; ++ks)
#pragma unroll
    for (int b = 0; b < TR_T; ++b)
      wf[ks][b] =
          *(const short4_t *)&t.pbF[MLP_F_W2T + (((TR_T * wave + b) * 16 + ks) * 64 + lane) * 4];
  uint16_t h2[TR_T][4];
#pragma unroll
  for (int b = 0; b < TR_T; ++b) {
    const int j = cw + 16 * b + li;
    const float bj = t.p[MLP_B2 + j];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      z2[b][r] += bj;
      h2[b][r] = f2bf(gelu(z2[b][r]));
    }
    store4(t.A2b + (int64_t)j * t.ld + r0 + 4 * lq, h2[b]);
  }
  lds_barrier();  // every wavefront has read A1
#pragma unroll
  for (int b = 0; b < TR_T; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) As[4 * lq + r][cw + 16 * b + li] = h2[b][r];
  lds_barrier();
  // logits (first wavefront)
  if (wave == 0) {
    float4_t z3 = zero;
#pragma unroll
    for (int ks = 0; ks < MLP_H / 16; ++ks) {
      const short4_t x = *(const short4_t *)&As[li][16 * ks + 4 * lq];
      z3 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, w3f[ks], z3, 0, 0, 0);
    }
    const float bj = t.p[MLP_B3 + li];
#pragma unroll
    for (int r = 0; r < 4; ++r) Zs[4 * lq + r][li] = z3[r] + bj;
  }
  lds_barrier();
  // softmax cross-entropy, one lane per row (first wavefront)
  if (wave == 0) {
    float l = 0.f;
    if (lane < 16) {
      const int i = lane;
      const int64_t src = srcs[i];
      const int y = (src >= 0 && src < t.n) ? (int)t.labels[src] : -1;
      float g0 = 0.f, g1 = 0.f;
      if (y == 0 || y == 1) {
        const float za = Zs[i][0], zb = Zs[i][1];
        const float m = fmaxf(za, zb);
        const float ea = expf(za - m), eb = expf(zb - m), s = ea + eb;
        const float pa = ea / s, pb = eb / s;
        // -log softmax_y = log(s) - (z_y - m)
        l = logf(s) - ((y ? zb : za) - m);
        g0 = (pa - (y == 0 ? 1.f : 0.f)) * t.inv;
        g1 = (pb - (y == 1 ? 1.f : 0.f)) * t.inv;
      }
      for (int c = 0; c < MLP_OUTP; ++c) {
        const float g = c == 0 ? g0 : (c == 1 ? g1 : 0.f);
        const uint16_t h = f2bf(g);
        t.dZ3b[(int64_t)c * t.ld + r0 + i] = h;
        Gs[i][c] = h;
        Zs[i][c] = g;
      }
    }
    for (int off = 8; off > 0; off >>= 1) l += __shfl_down(l, off, 64);
    if (lane == 0) bp[MLP_BIAS_LOSS] = l;
  }
  lds_barrier();
  if (tid < MLP_OUTP) {
    float sum = 0.f;
    for (int i = 0; i < 16; ++i) sum += Zs[i][tid];
    bp[2 * MLP_H + tid] = sum;
  }
  // dZ2 = (dZ3 W3^T) GELU'(Z2) (one k-step); its BF16 copy replaces A2
  {
    const short4_t x = *(const short4_t *)&Gs[li][4 * lq];
#pragma unroll
    for (int b = 0; b < TR_T; ++b) {
      const int j = cw + 16 * b + li;
      const float4_t d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, w3b[b], zero, 0, 0, 0);
      float sum = 0.f;
      uint16_t h[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float g = d[r] * gelu_grad(z2[b][r]);
        h[r] = f2bf(g);
        sum += g;
        As[4 * lq + r][j] = h[r];
      }
      store4(t.dZ2b + (int64_t)j * t.ld + r0 + 4 * lq, h);
      Ps2[lq][j] = sum;
    }
  }
  lds_barrier();
  if (tid < MLP_H)
    bp[MLP_H + tid] = ((Ps2[0][tid] + Ps2[1][tid]) + Ps2[2][tid]) + Ps2[3][tid];
  // dZ1 = (dZ2 W2^T) GELU'(Z1)
  float4_t d1[TR_T];
#pragma unroll
  for (int b = 0; b < TR_T; ++b) d1[b] = zero;
#pragma unroll
  for (int ks = 0; ks < MLP_H / 16; ++ks) {
    const short4_t x = *(const short4_t *)&As[li][16 * ks + 4 * lq];
#pragma unroll
    for (int b = 0; b < TR_T; ++b)
      d1[b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, wf[ks][b], d1[b], 0, 0, 0);
  }
#pragma unroll
  for (int b = 0; b < TR_T; ++b) {
    const int j = cw + 16 * b + li;
    float sum = 0.f;
    uint16_t h[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float g = d1[b][r] * gelu_grad(z1[b][r]);
      sum += g;
      h[r] = f2bf(g);
    }
    store4(t.dZ1b + (int64_t)j * t.ld + r0 + 4 * lq, h);
    Ps1[lq][j] = sum;
  }
  lds_barrier();
  if (tid < MLP_H) bp[tid] = ((Ps1[0][tid] + Ps1[1][tid]) + Ps1[2][tid]) + Ps1[3][tid];
}

// Bias gradients and loss from the blocks' sums of train_rows_kernel:
// column col of bpart[nblk][MLP_BIAS_COLS] summed over the blocks; thread
// group g of a block of 256 adds blocks g, g + 16, g + 32, ... in order,
// then the 16 group sums are added in order.  Columns 0..255 go to b1,
// 256..511 to b2, 512..527 to b3, the loss column is added to *loss_sum.
__global__ void __launch_bounds__(256) bias_grad_kernel(const float *bpart, int nblk,
                                                        float *grad, float *loss_sum) {
  __shared__ float red[16][17];
  const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int col = blockIdx.x * 16 + c;
  const int cnt = g < nblk ? (nblk - g + 15) / 16 : 0;
  red[g][c] = ordered_sum<>(0.f, bpart + (int64_t)g * MLP_BIAS_COLS + col,
                          (int64_t)16 * MLP_BIAS_COLS, cnt);
  __syncthreads();
  if (g == 0) {
    float t = 0.f;
    for (int q = 0; q < 16; ++q) t += red[q][c];
    if (col < 2 * MLP_H + MLP_OUTP) {
      const int64_t dst = col < MLP_H ? MLP_B1 + col
                                      : (col < 2 * MLP_H ? MLP_B2 + (col - MLP_H)
                                                         : MLP_B3 + (col - 2 * MLP_H));
      grad[dst] = t;
    } else if (col == MLP_BIAS_LOSS && loss_sum) {
      *loss_sum += t;
    }
  }
}

__global__ void fill_f32_kernel(float *p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Gate selection per orbit from its status and label at the gate time and
// the gate's output: masked -> label -1, source 0; stopped -> its label,
// source 1; confident -> gate label, source 2; else keep for integration
// to T, source 3.  counts[0..3] += orbits per source.
__global__ void gate_select_kernel(int64_t n, const int *status, const int8_t *label1,
                                   const float *pc, const float *conf, float conf_min,
                                   int8_t *label, uint8_t *source, uint8_t *keep, float *conf_out,
                                   unsigned long long *counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int src = -1;
  if (i < n) {
    const int st = status[i];
    int8_t lb;
    float cf = __builtin_nanf("");
    uint8_t kp = 0;
    if (st == CHX_ORBIT_MASKED) {
      src = 0;
      lb = -1;
    } else if (st != CHX_ORBIT_OK) {
      src = 1;
      lb = label1[i];
    } else {
      cf = conf[i];
      if (cf >= conf_min) {
        src = 2;
        lb = pc[i] >= 0.5f ? 1 : 0;
      } else {
        src = 3;
        lb = -1;
        kp = 1;
      }
    }
    label[i] = lb;
    if (source) source[i] = (uint8_t)src;
    keep[i] = kp;
    if (conf_out) conf_out[i] = cf;
  }
  for (int c = 0; c < 4; ++c) {
    const uint64_t m = __ballot(src == c);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&counts[c], (unsigned long long)__popcll(m));
  }
}

// label[orbit[j]] = label2[j]
__global__ void gate_scatter_kernel(int64_t n2, const int64_t *orbit, const int8_t *label2,
                                    int8_t *label) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n2) label[orbit[j]] = label2[j];
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// The gradient of one batch, entry i of g: a weight whose product was split
// over K is the sum of its parts in order of the part (deterministic); the
// other entries (unsplit products, biases) are already in g.  With step set, AdamW then updates the FP32
// master (entries with mask set) and its BF16 copies pb and pbF.
__global__ void grad_step_kernel(GradParts gp, float *p, uint16_t *pb, uint16_t *pbF, float *g,
                                 float *m, float *v, const uint8_t *mask, int step, float lr,
                                 float b1, float b2, float eps, float wd, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  float gi;
  // (32 parts' loads in flight at a time: the 256 x 256 gradient has up to
  // 32 parts, the 16-wide ones up to 64)
  if (i < MLP_B1 && gp.s1 > 1)
    gi = ordered_sum<32>(0.f, gp.w1 + (i - MLP_W1), MLP_B1 - MLP_W1, gp.s1);
  else if (i >= MLP_W2 && i < MLP_B2 && gp.s2 > 1)
    gi = ordered_sum<32>(0.f, gp.w2 + (i - MLP_W2), MLP_B2 - MLP_W2, gp.s2);
  else if (i >= MLP_W3 && i < MLP_B3 && gp.s3 > 1)
    gi = ordered_sum<32>(0.f, gp.w3 + (i - MLP_W3), MLP_B3 - MLP_W3, gp.s3);
  else
    gi = g[i];
  g[i] = gi;
  if (!step || !mask[i]) return;
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1, vh = vi / bc2;
  const float pn = p[i] - lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
  p[i] = pn;
  const uint16_t h = f2bf(pn);
  pb[i] = h;
  int64_t f0, f1;
  mlp_fpos(i, f0, f1);
  if (f0 >= 0) pbF[f0] = h;
  if (f1 >= 0) pbF[f1] = h;
}

// BF16 copies of the parameters: pb in their own layout, pbF the weights in
// the training pass's operand order
__global__ void weights_bf16_kernel(const float *p, uint16_t *pb, uint16_t *pbF) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  const uint16_t h = f2bf(p[i]);
  pb[i] = h;
  int64_t f0, f1;
  mlp_fpos(i, f0, f1);
  if (f0 >= 0) pbF[f0] = h;
  if (f1 >= 0) pbF[f1] = h;
}

// X[r][0..15] = BF16 of the z-scored features of row rows[r] (zero pad;
// rows at or past n_valid are all zero)
__global__ void batch_input_kernel(const float *feat, const int64_t *rows, int B,
                                   int64_t n_valid, const float *mean, const float *istd,
                                   uint16_t *X) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= B) return;
  const int64_t src = rows ? rows[r] : r;
  const bool ok = src >= 0 && src < n_valid;
  for (int c = 0; c < 16; ++c) {
    const float v = (ok && c < MLP_IN) ? (feat[src * MLP_IN + c] - mean[c]) * istd[c] : 0.f;
    X[r * 16 + c] = f2bf(v);
  }
}

// Initial weights: N(0, 2/fan_in) on the real entries (SplitMix64 counters
// and the Box-Muller cosine branch), zero biases and padding; mask marks
// the real entries.
__device__ inline uint64_t mlp_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void init_params_kernel(float *p, uint8_t *mask, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  bool real;
  double fan = 1.0;
  bool bias = false;
  if (i < MLP_B1) {
    real = (i / MLP_H) < MLP_IN;
    fan = MLP_IN;
  } else if (i < MLP_W2) {
    real = true;
    bias = true;
  } else if (i < MLP_B2) {
    real = true;
    fan = MLP_H;
  } else if (i < MLP_W3) {
    real = true;
    bias = true;
  } else if (i < MLP_B3) {
    real = ((i - MLP_W3) % MLP_OUTP) < 2;
    fan = MLP_H;
  } else {
    real = (i - MLP_B3) < 2;
    bias = true;
  }
  mask[i] = real ? 1 : 0;
  float v = 0.f;
  if (real && !bias) {
    const uint64_t key = mlp_mix64(seed ^ mlp_mix64(3));
    const double u1 = (double)(mlp_mix64(key + (2 * i + 1) * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53;
    const double u2 = (double)(mlp_mix64(key + (2 * i + 2) * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53;
    const double z = sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * M_PI * u2);
    v = (float)(z * sqrt(2.0 / fan));
  }
  p[i] = v;
}

// Z-score statistics of the features, in two passes: per-block partial
// sums of v and v^2 (FP64), then mean and 1/std (population) per feature.
__global__ void feature_partials_kernel(const float *feat, int64_t n, double *part) {
  double a[MLP_IN], b[MLP_IN];
  for (int c = 0; c < MLP_IN; ++c) a[c] = b[c] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    for (int c = 0; c < MLP_IN; ++c) {
      const double v = feat[r * MLP_IN + c];
      a[c] += v;
      b[c] += v * v;
    }
  }
  __shared__ double sa[256][2 * MLP_IN];
  for (int c = 0; c < MLP_IN; ++c) {
    sa[threadIdx.x][c] = a[c];
    sa[threadIdx.x][MLP_IN + c] = b[c];
  }
  __syncthreads();
  if (threadIdx.x < 2 * MLP_IN) {
    double t = 0.0;
    for (int k = 0; k < (int)blockDim.x; ++k) t += sa[k][threadIdx.x];
    part[blockIdx.x * 2 * MLP_IN + threadIdx.x] = t;
  }
}
__global__ void feature_stats_kernel(const double *part, int nblocks, int64_t n, float *mean,
                                     float *istd) {
  const int c = threadIdx.x;
  if (c >= MLP_IN) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nblocks; ++k) {
    a += part[k * 2 * MLP_IN + c];
    b += part[k * 2 * MLP_IN + MLP_IN + c];
  }
  const double mu = a / (double)n;
  const double var = b / (double)n - mu * mu;
  mean[c] = (float)mu;
  istd[c] = var > 0.0 ? (float)(1.0 / sqrt(var)) : 1.0f;
}

// Inference output: p(chaotic) and the confidence max(p, 1 - p).
__global__ void infer_out_kernel(const float *Z3, int B, float *pc, float *conf) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= B) return;
  const float a = Z3[r * 16 + 0], b = Z3[r * 16 + 1];
  const float m = fmaxf(a, b);
  const float ea = expf(a - m), eb = expf(b - m);
  const float p1 = eb / (ea + eb);
  if (pc) pc[r] = p1;
  if (conf) conf[r] = fmaxf(p1, 1.f - p1);
}

// Gate features at time t: (y, p_y, p_x, LD/t, G1/t, G2/t) from the
// initial conditions [n][4], the LD [n] and the ln-growths [n][2].
__global__ void features_kernel(const double *x0, const double *ld, const double *lg, double t,
                                int64_t n, float *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i * 6 + 0] = (float)x0[i * 4 + 1];
  out[i * 6 + 1] = (float)x0[i * 4 + 3];
  out[i * 6 + 2] = (float)x0[i * 4 + 2];
  out[i * 6 + 3] = (float)(ld[i] / t);
  out[i * 6 + 4] = (float)(lg[i * 2 + 0] / t);
  out[i * 6 + 5] = (float)(lg[i * 2 + 1] / t);
}


// p[i] *= mask[i] (keeps padded entries at zero after a load)
__global__ void apply_mask_kernel(float *p, const uint8_t *mask, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !mask[i]) p[i] = 0.f;
}

inline unsigned nb(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t mlp_gemm(const uint16_t *A, int64_t a_r, int64_t a_c, const uint16_t *B, int64_t b_r,
                    int64_t b_c, float *C, int64_t ldc, int M, int N, int K, const float *bias,
                    int accumulate, hipStream_t s, float *work, int64_t work_len, int epi,
                    uint16_t *Cb, int *parts) {
  if (M <= 0 || N <= 0 || K <= 0 || M % 16 || N % 16 || K % 16) return hipErrorInvalidValue;
  // (64, 64) tiles where N allows, (16, 64) for a 16-row product, else
  // (64, 16)
  const int BN = N % 64 == 0 ? 64 : 16;
  const int BM = BN == 64 && M == 16 ? 16 : 64;
  const int64_t gm = (M + BM - 1) / BM, gn = N / BN;
  if (gm > 65535) return hipErrorInvalidValue;
  // split K (a workspace given) until about 512 blocks (two per CU), each
  // part at least two chunks
  const int chunks = (K + GBK - 1) / GBK;
  if (epi < EPI_NONE || epi > EPI_GELU || (epi == EPI_GELU && (!Cb || accumulate)) ||
      (work && !parts) || (parts && (bias || accumulate || ldc != N)))
    return hipErrorInvalidValue;
  int S = 1;
  while (epi == EPI_NONE && work && gm * gn * S < 512 && chunks >= 4 * S &&
         (int64_t)2 * S * M * N <= work_len)
    S *= 2;
  const int cpc = (chunks + S - 1) / S;
  // 16-byte loads when every run of 8 along the unit stride is aligned
  auto al = [](const void *p, int64_t s1, int64_t s2) {
    const int64_t st = s1 == 1 ? s2 : s1;
    return ((uintptr_t)p % 16 == 0) && (st % 8 == 0);
  };
  const bool vec = al(A, a_r, a_c) && al(B, b_c, b_r);
  const dim3 grid((unsigned)gn, (unsigned)gm, (unsigned)S);
#define CHX_GEMM_GO(bm, bn, v, ep)                                                               \
  hipLaunchKernelGGL((gemm_tile_kernel<bm, bn, v, ep>), grid, dim3(256), 0, s, A, a_r, a_c, B,   \
                     b_r, b_c, C, ldc, M, N, K, cpc, bias, accumulate, work, Cb)
#define CHX_GEMM_LAUNCH(bm, bn, ep)                                                              \
  do {                                                                                          \
    if (vec) CHX_GEMM_GO(bm, bn, true, ep);                                                     \
    else CHX_GEMM_GO(bm, bn, false, ep);                                                        \
  } while (0)
  // the activation epilogues exist for the 256-wide layers only
  if (BN == 16) {
    if (epi != EPI_NONE) return hipErrorInvalidValue;
    CHX_GEMM_LAUNCH(64, 16, EPI_NONE);
  } else if (BM == 16) {
    if (epi == EPI_GELU) CHX_GEMM_LAUNCH(16, 64, EPI_GELU);
    else CHX_GEMM_LAUNCH(16, 64, EPI_NONE);
  } else {
    if (epi == EPI_GELU) CHX_GEMM_LAUNCH(64, 64, EPI_GELU);
    else CHX_GEMM_LAUNCH(64, 64, EPI_NONE);
  }
#undef CHX_GEMM_LAUNCH
#undef CHX_GEMM_GO
  if (parts) *parts = S;
  return hipGetLastError();
}

hipError_t mlp_train_rows(const MlpRowsArgs &r, int B, hipStream_t s) {
  if (B <= 0 || B % 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(train_rows_kernel, dim3((unsigned)(B / 16)), dim3(64 * TR_W), 0, s, r);
  return hipGetLastError();
}
hipError_t mlp_bias_grad(const float *bpart, int nblk, float *grad, float *loss_sum,
                         hipStream_t s) {
  if (nblk <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bias_grad_kernel, dim3(MLP_BIAS_COLS / 16), dim3(256), 0, s, bpart, nblk,
                     grad, loss_sum);
  return hipGetLastError();
}
hipError_t mlp_fill(float *p, int64_t n, float v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f32_kernel, dim3(nb(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t gate_select(int64_t n, const int *status, const int8_t *label1, const float *pc,
                       const float *conf, float conf_min, int8_t *label, uint8_t *source,
                       uint8_t *keep, float *conf_out, unsigned long long *counts,
                       hipStream_t s) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, counts, 4);
  if (n > 0)
    hipLaunchKernelGGL(gate_select_kernel, dim3(nb(n)), dim3(256), 0, s, n, status, label1, pc,
                       conf, conf_min, label, source, keep, conf_out, counts);
  return hipGetLastError();
}
hipError_t gate_scatter(int64_t n2, const int64_t *orbit, const int8_t *label2, int8_t *label,
                        hipStream_t s) {
  if (n2 == 0) return hipSuccess;
  hipLaunchKernelGGL(gate_scatter_kernel, dim3(nb(n2)), dim3(256), 0, s, n2, orbit, label2, label);
  return hipGetLastError();
}
hipError_t mlp_grad_step(const GradParts &gp, float *p, uint16_t *pb, uint16_t *pbF, float *g,
                         float *m, float *v, const uint8_t *mask, int step, float lr, float b1,
                         float b2, float eps, float wd, float bc1, float bc2, hipStream_t s) {
  hipLaunchKernelGGL(grad_step_kernel, dim3(nb(MLP_NPARAM)), dim3(256), 0, s, gp, p, pb, pbF, g, m,
                     v, mask, step, lr, b1, b2, eps, wd, bc1, bc2);
  return hipGetLastError();
}
hipError_t mlp_weights_bf16(const float *p, uint16_t *pb, uint16_t *pbF, hipStream_t s) {
  hipLaunchKernelGGL(weights_bf16_kernel, dim3(nb(MLP_NPARAM)), dim3(256), 0, s, p, pb, pbF);
  return hipGetLastError();
}
hipError_t mlp_batch_input(const float *feat, const int64_t *rows, int B, int64_t n_valid,
                           const float *mean, const float *istd, uint16_t *X, hipStream_t s) {
  hipLaunchKernelGGL(batch_input_kernel, dim3(nb(B)), dim3(256), 0, s, feat, rows, B, n_valid,
                     mean, istd, X);
  return hipGetLastError();
}
hipError_t mlp_init_params(float *p, uint8_t *mask, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(init_params_kernel, dim3(nb(MLP_NPARAM)), dim3(256), 0, s, p, mask, seed);
  return hipGetLastError();
}
hipError_t mlp_feature_stats(const float *feat, int64_t n, float *mean, float *istd,
                             double *partials, hipStream_t s) {
  hipLaunchKernelGGL(feature_partials_kernel, dim3(MLP_STAT_BLOCKS), dim3(256), 0, s, feat, n,
                     partials);
  hipLaunchKernelGGL(feature_stats_kernel, dim3(1), dim3(64), 0, s, partials, MLP_STAT_BLOCKS, n,
                     mean, istd);
  return hipGetLastError();
}
hipError_t mlp_infer_out(const float *Z3, int B, float *pc, float *conf, hipStream_t s) {
  hipLaunchKernelGGL(infer_out_kernel, dim3(nb(B)), dim3(256), 0, s, Z3, B, pc, conf);
  return hipGetLastError();
}
hipError_t mlp_features(const double *x0, const double *ld, const double *lg, double t, int64_t n,
                        float *out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(features_kernel, dim3(nb(n)), dim3(256), 0, s, x0, ld, lg, t, n, out);
  return hipGetLastError();
}
hipError_t mlp_apply_mask(float *p, const uint8_t *mask, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(apply_mask_kernel, dim3(nb(n)), dim3(256), 0, s, p, mask, n);
  return hipGetLastError();
}

}  // namespace chx
