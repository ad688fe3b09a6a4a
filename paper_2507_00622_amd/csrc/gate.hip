// gate.hip -- host side of the learned gate (chx_gate_* in include/chx.h):
// the parameter object, the training loop (forward, backward, AdamW on the
// kernels of mlp.hip), inference, and the classify workflow that labels a
// Henon-Heiles ensemble from a short integration and resumes only the
// unconfident orbits.
#include <math.h>
#include <string.h>

#include <vector>

#include "ensemble.h"
#include "mlp.h"

using namespace chx;
using namespace chx::host;

struct chx_gate {
  int device = -1;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  uint8_t *mask = nullptr;
  uint16_t *pb = nullptr;   // BF16 copy of p
  uint16_t *pbF = nullptr;  // BF16 copy of the weights in MFMA operand order
  float *mean = nullptr;    // [16] z-score mean (first 6 used)
  float *istd = nullptr;    // [16] inverse standard deviation
  double *partials = nullptr;
  int64_t t = 0;            // AdamW steps taken
  bool have_stats = false;
};

namespace {

#define GCHK(expr, what)                             \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return dev_fail(e_, what); \
  } while (0)

constexpr int CHUNK = 65536;  // rows per forward pass (inference) / max batch

inline int64_t round16(int64_t n) { return (n + 15) / 16 * 16; }

chx_status check_device(const chx_gate *g) {
  if (!g) return fail(CHX_ERR_INVALID_ARG, "gate is NULL");
  int d = -1;
  GCHK(hipGetDevice(&d), "current device");
  if (d != g->device)
    return fail(CHX_ERR_INVALID_ARG, "gate lives on device %d, current device is %d", g->device, d);
  return CHX_OK;
}

chx_status stream_for(uint32_t flags, void *stream, hipStream_t *s) {
  if (flags & ~1u) return fail(CHX_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  if (!(flags & CHX_PTR_DEVICE) && stream)
    return fail(CHX_ERR_INVALID_ARG, "stream given without CHX_PTR_DEVICE");
  *s = (flags & CHX_PTR_DEVICE) ? (hipStream_t)stream : nullptr;
  return CHX_OK;
}

// Device allocations released together (stream-ordered).
struct Scratch {
  hipStream_t s;
  std::vector<void *> ptrs;
  hipError_t err = hipSuccess;
  explicit Scratch(hipStream_t st) : s(st) {}
  template <class T>
  T *get(size_t count) {
    if (err != hipSuccess || count == 0) return nullptr;
    T *p = nullptr;
    err = hipMallocAsync((void **)&p, sizeof(T) * count, s);
    if (err == hipSuccess) ptrs.push_back(p);
    else p = nullptr;
    return p;
  }
  template <class T>
  T *in(const T *src, size_t count, bool device) {
    if (device || !src || count == 0) return const_cast<T *>(src);
    T *p = get<T>(count);
    if (p && err == hipSuccess) err = hipMemcpyAsync(p, src, sizeof(T) * count, hipMemcpyHostToDevice, s);
    return p;
  }
  ~Scratch() {
    for (void *p : ptrs) (void)hipFreeAsync(p, s);
  }
};

// Activations of one pass over up to B rows: inference (the products'
// FP32 outputs Z) or training (the activation gradients).
struct Acts {
  uint16_t *X, *A1b, *A2b, *dZ3b, *dZ2b, *dZ1b;
  float *Z1, *Z2, *Z3;
  float *bpart;  // per 16-row block: column sums of dZ1 | dZ2 | dZ3
  float *work1, *work2, *work3;  // split-K parts of the weight gradients
};

bool alloc_acts(Scratch &S, int64_t B, bool backward, Acts *a) {
  memset(a, 0, sizeof *a);
  a->X = S.get<uint16_t>(B * MLP_INP);
  a->A1b = S.get<uint16_t>(B * MLP_H);
  a->A2b = S.get<uint16_t>(B * MLP_H);
  if (!backward) {
    a->Z1 = S.get<float>(B * MLP_H);
    a->Z2 = S.get<float>(B * MLP_H);
    a->Z3 = S.get<float>(B * MLP_OUTP);
  } else {
    a->dZ3b = S.get<uint16_t>(B * MLP_OUTP);
    a->dZ2b = S.get<uint16_t>(B * MLP_H);
    a->dZ1b = S.get<uint16_t>(B * MLP_H);
    a->bpart = S.get<float>((size_t)(B / 16) * MLP_BIAS_COLS);
    a->work1 = S.get<float>(MLP_SPLITK_WORK_SMALL);
    a->work2 = S.get<float>(MLP_SPLITK_WORK);
    a->work3 = S.get<float>(MLP_SPLITK_WORK_SMALL);
  }
  return S.err == hipSuccess;
}

// Forward pass of B rows (multiple of 16) whose z-scored BF16 inputs are in
// a.X: Z3 = logits.
hipError_t forward(const chx_gate *g, const Acts &a, int B, hipStream_t s) {
  const uint16_t *pb = g->pb;
  const float *p = g->p;
  hipError_t e;
  // Z = X W + b and its GELU in BF16, from the product's epilogue
  if ((e = mlp_gemm(a.X, MLP_INP, 1, pb + MLP_W1, MLP_H, 1, a.Z1, MLP_H, B, MLP_H, MLP_INP,
                    p + MLP_B1, 0, s, nullptr, 0, EPI_GELU, a.A1b)))
    return e;
  if ((e = mlp_gemm(a.A1b, MLP_H, 1, pb + MLP_W2, MLP_H, 1, a.Z2, MLP_H, B, MLP_H, MLP_H,
                    p + MLP_B2, 0, s, nullptr, 0, EPI_GELU, a.A2b)))
    return e;
  return mlp_gemm(a.A2b, MLP_H, 1, pb + MLP_W3, MLP_OUTP, 1, a.Z3, MLP_OUTP, B, MLP_OUTP, MLP_H,
                  p + MLP_B3, 0, s);
}

// Loss and gradient of one batch of B rows (multiple of 16) into g->g and
// the weight gradients' split-K parts (gp; mlp_grad_step adds them): the
// rows at positions start .. start + B - 1 of the permutation
// i -> (pa i + pc) mod n (padding at or past n) and their labels; inv = 1 /
// (rows in the batch mean).  One launch does the rows' forward and
// backward passes and their blocks' column sums; the weight gradients are
// products over the batch's rows, the bias gradients the sums of the
// blocks' column sums.
hipError_t batch_grad(chx_gate *g, const Acts &a, int B, const float *feat, const int8_t *labels,
                      int64_t n, int64_t start, uint64_t pa, uint64_t pc, float inv,
                      float *loss_sum, GradParts *gp, hipStream_t s) {
  MlpRowsArgs r;
  r.n = n;
  r.start = start;
  r.ld = B;
  r.a = pa;
  r.c = pc;
  r.feat = feat;
  r.mean = g->mean;
  r.istd = g->istd;
  r.labels = labels;
  r.inv = inv;
  r.p = g->p;
  r.pb = g->pb;
  r.pbF = g->pbF;
  r.X = a.X;
  r.A1b = a.A1b;
  r.A2b = a.A2b;
  r.dZ3b = a.dZ3b;
  r.dZ2b = a.dZ2b;
  r.dZ1b = a.dZ1b;
  r.bpart = a.bpart;
  float *gr = g->g;
  hipError_t e;
  if ((e = mlp_train_rows(r, B, s))) return e;
  if ((e = mlp_bias_grad(a.bpart, B / 16, gr, loss_sum, s))) return e;
  // weight gradients A^T dZ, layer 3, 2, 1, their parts left for mlp_grad_step
  gp->w1 = a.work1;
  gp->w2 = a.work2;
  gp->w3 = a.work3;
  // (the row kernel's outputs are feature-major with row stride B, so both
  // operands run along K = rows)
  if ((e = mlp_gemm(a.A2b, B, 1, a.dZ3b, 1, B, gr + MLP_W3, MLP_OUTP, MLP_H, MLP_OUTP, B, nullptr,
                    0, s, a.work3, MLP_SPLITK_WORK_SMALL, EPI_NONE, nullptr, &gp->s3)))
    return e;
  if ((e = mlp_gemm(a.A1b, B, 1, a.dZ2b, 1, B, gr + MLP_W2, MLP_H, MLP_H, MLP_H, B, nullptr, 0, s,
                    a.work2, MLP_SPLITK_WORK, EPI_NONE, nullptr, &gp->s2)))
    return e;
  return mlp_gemm(a.X, B, 1, a.dZ1b, 1, B, gr + MLP_W1, MLP_H, MLP_INP, MLP_H, B, nullptr, 0, s,
                  a.work1, MLP_SPLITK_WORK_SMALL, EPI_NONE, nullptr, &gp->s1);
}

// p(chaotic) and confidence of n rows of device features.
chx_status infer_dev(const chx_gate *g, const float *feat, int64_t n, float *pc, float *conf,
                     hipStream_t s) {
  if (n == 0) return CHX_OK;
  Scratch S(s);
  Acts a;
  const int64_t B = n < CHUNK ? round16(n) : CHUNK;
  if (!alloc_acts(S, B, false, &a)) return dev_fail(S.err, "allocate activations");
  for (int64_t r0 = 0; r0 < n; r0 += CHUNK) {
    const int64_t rows = (n - r0) < CHUNK ? (n - r0) : CHUNK;
    const int Bp = (int)round16(rows);
    GCHK(mlp_batch_input(feat + r0 * MLP_IN, nullptr, Bp, rows, g->mean, g->istd, a.X, s),
         "gate input");
    GCHK(forward(g, a, Bp, s), "gate forward");
    GCHK(mlp_infer_out(a.Z3, (int)rows, pc ? pc + r0 : nullptr, conf ? conf + r0 : nullptr, s),
         "gate output");
  }
  return CHX_OK;
}

uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace

extern "C" {

chx_status chx_gate_create(uint64_t seed, chx_gate **out) {
  g_err.clear();
  if (!out) return fail(CHX_ERR_INVALID_ARG, "output handle pointer is NULL");
  *out = nullptr;
  chx_gate *g = new chx_gate();
  hipError_t e = hipGetDevice(&g->device);
  auto al = [&](auto **p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc((void **)p, bytes);
  };
  al(&g->p, sizeof(float) * MLP_NPARAM);
  al(&g->m, sizeof(float) * MLP_NPARAM);
  al(&g->v, sizeof(float) * MLP_NPARAM);
  al(&g->g, sizeof(float) * MLP_NPARAM);
  al(&g->mask, MLP_NPARAM);
  al(&g->pb, sizeof(uint16_t) * MLP_NPARAM);
  al(&g->pbF, sizeof(uint16_t) * MLP_NFRAG);
  al(&g->mean, sizeof(float) * 16);
  al(&g->istd, sizeof(float) * 16);
  al(&g->partials, sizeof(double) * MLP_STAT_BLOCKS * 2 * MLP_IN);
  if (e == hipSuccess) e = mlp_init_params(g->p, g->mask, seed, nullptr);
  if (e == hipSuccess) e = mlp_fill(g->m, MLP_NPARAM, 0.f, nullptr);
  if (e == hipSuccess) e = mlp_fill(g->v, MLP_NPARAM, 0.f, nullptr);
  if (e == hipSuccess) e = mlp_fill(g->g, MLP_NPARAM, 0.f, nullptr);
  if (e == hipSuccess) e = mlp_fill(g->mean, 16, 0.f, nullptr);
  if (e == hipSuccess) e = mlp_fill(g->istd, 16, 1.f, nullptr);
  if (e == hipSuccess) e = mlp_weights_bf16(g->p, g->pb, g->pbF, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    chx_gate_destroy(g);
    return dev_fail(e, "create gate");
  }
  *out = g;
  return CHX_OK;
}

void chx_gate_destroy(chx_gate *g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  for (void *p : {(void *)g->p, (void *)g->m, (void *)g->v, (void *)g->g, (void *)g->mask,
                  (void *)g->pb, (void *)g->pbF, (void *)g->mean, (void *)g->istd,
                  (void *)g->partials})
    if (p) (void)hipFree(p);
  delete g;
}

chx_status chx_gate_train(chx_gate *g, const float *features, const int8_t *labels, int64_t n,
                          const chx_gate_train_cfg *cfg_in, int32_t reset_stats,
                          float *epoch_loss, uint32_t flags, void *stream) {
  g_err.clear();
  chx_status st = check_device(g);
  if (st) return st;
  hipStream_t s;
  if ((st = stream_for(flags, stream, &s))) return st;
  if (!cfg_in) return fail(CHX_ERR_INVALID_ARG, "cfg is NULL");
  if (n <= 0) return fail(CHX_ERR_INVALID_ARG, "n must be > 0");
  if (n > ((int64_t)1 << 40)) return fail(CHX_ERR_INVALID_ARG, "n too large");
  if (!features || !labels) return fail(CHX_ERR_INVALID_ARG, "features or labels is NULL");
  chx_gate_train_cfg c = *cfg_in;
  if (c.epochs == 0) c.epochs = 1;
  if (c.batch == 0) c.batch = 4096;
  if (c.lr == 0.f) c.lr = 1e-3f;
  if (c.beta1 == 0.f) c.beta1 = 0.9f;
  if (c.beta2 == 0.f) c.beta2 = 0.999f;
  if (c.eps == 0.f) c.eps = 1e-8f;
  if (c.epochs < 0) return fail(CHX_ERR_INVALID_ARG, "epochs must be >= 0");
  if (c.batch < 16 || c.batch > CHUNK || c.batch % 16)
    return fail(CHX_ERR_INVALID_ARG, "batch must be a multiple of 16 in 16..%d", CHUNK);
  if (!(c.lr > 0.f) || !(c.beta1 >= 0.f && c.beta1 < 1.f) || !(c.beta2 >= 0.f && c.beta2 < 1.f) ||
      !(c.eps > 0.f) || !(c.weight_decay >= 0.f))
    return fail(CHX_ERR_INVALID_ARG, "invalid optimiser settings");
  const bool dev = flags & CHX_PTR_DEVICE;
  Scratch S(s);
  const float *feat = S.in(features, (size_t)n * MLP_IN, dev);
  const int8_t *lab = S.in(labels, (size_t)n, dev);
  float *loss = S.get<float>((size_t)c.epochs);
  Acts a;
  const int B = c.batch;
  if (!alloc_acts(S, B, true, &a)) return dev_fail(S.err, "allocate training buffers");
  if (reset_stats || !g->have_stats) {
    GCHK(mlp_feature_stats(feat, n, g->mean, g->istd, g->partials, s), "feature statistics");
    g->have_stats = true;
  }
  GCHK(mlp_fill(loss, c.epochs, 0.f, s), "clear loss");
  const int64_t nbatch = (n + B - 1) / B;
  // the BF16 copy of the weights; each AdamW step refreshes it
  GCHK(mlp_weights_bf16(g->p, g->pb, g->pbF, s), "weights to bf16");
  for (int ep = 0; ep < c.epochs; ++ep) {
    // epoch permutation i -> (pa i + pc) mod n with pa coprime to n
    const uint64_t key = mix64(c.seed ^ mix64(0x6a7e0000ull + (uint64_t)ep));
    uint64_t pa = (uint64_t)n > 1 ? 1 + mix64(key) % ((uint64_t)n - 1) : 1;
    while (gcd64(pa, (uint64_t)n) != 1) pa = pa + 1 < (uint64_t)n ? pa + 1 : 1;
    const uint64_t pc = mix64(key + 1) % (uint64_t)n;
    for (int64_t b = 0; b < nbatch; ++b) {
      const int64_t start = b * B;
      const int64_t rows = (n - start) < B ? (n - start) : B;
      const int Bp = (int)round16(rows);
      GradParts gp;
      GCHK(batch_grad(g, a, Bp, feat, lab, n, start, pa, pc, 1.0f / (float)rows, loss + ep, &gp,
                      s),
           "batch gradient");
      g->t += 1;
      const double bc1 = 1.0 - pow((double)c.beta1, (double)g->t);
      const double bc2 = 1.0 - pow((double)c.beta2, (double)g->t);
      GCHK(mlp_grad_step(gp, g->p, g->pb, g->pbF, g->g, g->m, g->v, g->mask, 1, c.lr, c.beta1,
                         c.beta2, c.eps, c.weight_decay, (float)bc1, (float)bc2, s),
           "AdamW");
    }
  }
  std::vector<float> hl((size_t)c.epochs);
  if (c.epochs > 0) GCHK(hipMemcpyAsync(hl.data(), loss, sizeof(float) * c.epochs, hipMemcpyDeviceToHost, s), "read loss");
  GCHK(hipStreamSynchronize(s), "synchronise");
  if (epoch_loss)
    for (int ep = 0; ep < c.epochs; ++ep) epoch_loss[ep] = hl[ep] / (float)n;
  return CHX_OK;
}

chx_status chx_gate_grad(chx_gate *g, const float *features, const int8_t *labels, int64_t n,
                         float *grad_out, float *loss_out, uint32_t flags, void *stream) {
  g_err.clear();
  chx_status st = check_device(g);
  if (st) return st;
  hipStream_t s;
  if ((st = stream_for(flags, stream, &s))) return st;
  if (n <= 0 || n > CHUNK) return fail(CHX_ERR_INVALID_ARG, "n must be in 1..%d", CHUNK);
  if (!features || !labels) return fail(CHX_ERR_INVALID_ARG, "features or labels is NULL");
  const bool dev = flags & CHX_PTR_DEVICE;
  Scratch S(s);
  const float *feat = S.in(features, (size_t)n * MLP_IN, dev);
  const int8_t *lab = S.in(labels, (size_t)n, dev);
  float *loss = S.get<float>(1);
  Acts a;
  const int Bp = (int)round16(n);
  if (!alloc_acts(S, Bp, true, &a)) return dev_fail(S.err, "allocate buffers");
  GCHK(mlp_fill(loss, 1, 0.f, s), "clear loss");
  GCHK(mlp_fill(g->g, MLP_NPARAM, 0.f, s), "clear gradient");
  GradParts gp;
  GCHK(batch_grad(g, a, Bp, feat, lab, n, 0, 1, 0, 1.0f / (float)n, loss, &gp, s), "gradient");
  GCHK(mlp_grad_step(gp, g->p, g->pb, g->pbF, g->g, g->m, g->v, g->mask, 0, 0.f, 0.f, 0.f, 0.f,
                     0.f, 1.f, 1.f, s),
       "gradient parts");
  float hl = 0.f;
  GCHK(hipMemcpyAsync(&hl, loss, sizeof hl, hipMemcpyDeviceToHost, s), "read loss");
  if (grad_out)
    GCHK(hipMemcpyAsync(grad_out, g->g, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, s),
         "read gradient");
  GCHK(hipStreamSynchronize(s), "synchronise");
  if (loss_out) *loss_out = hl / (float)n;
  return CHX_OK;
}

chx_status chx_gate_infer(const chx_gate *g, const float *features, int64_t n, float *p_chaotic,
                          float *confidence, uint32_t flags, void *stream) {
  g_err.clear();
  chx_status st = check_device(g);
  if (st) return st;
  hipStream_t s;
  if ((st = stream_for(flags, stream, &s))) return st;
  if (n < 0) return fail(CHX_ERR_INVALID_ARG, "n must be >= 0");
  if (n == 0) return CHX_OK;
  if (!features) return fail(CHX_ERR_INVALID_ARG, "features is NULL");
  const bool dev = flags & CHX_PTR_DEVICE;
  Scratch S(s);
  const float *feat = S.in(features, (size_t)n * MLP_IN, dev);
  float *pc = dev ? p_chaotic : (p_chaotic ? S.get<float>(n) : nullptr);
  float *cf = dev ? confidence : (confidence ? S.get<float>(n) : nullptr);
  if (S.err != hipSuccess) return dev_fail(S.err, "stage inputs");
  if ((st = infer_dev(g, feat, n, pc, cf, s))) return st;
  if (!dev) {
    if (p_chaotic) GCHK(hipMemcpyAsync(p_chaotic, pc, sizeof(float) * n, hipMemcpyDeviceToHost, s), "read p");
    if (confidence) GCHK(hipMemcpyAsync(confidence, cf, sizeof(float) * n, hipMemcpyDeviceToHost, s), "read confidence");
    GCHK(hipStreamSynchronize(s), "synchronise");
  }
  return CHX_OK;
}

chx_status chx_gate_get(const chx_gate *g, float *params, float *mean, float *istd) {
  g_err.clear();
  chx_status st = check_device(g);
  if (st) return st;
  if (params) GCHK(hipMemcpy(params, g->p, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost), "read params");
  if (mean) GCHK(hipMemcpy(mean, g->mean, sizeof(float) * MLP_IN, hipMemcpyDeviceToHost), "read mean");
  if (istd) GCHK(hipMemcpy(istd, g->istd, sizeof(float) * MLP_IN, hipMemcpyDeviceToHost), "read istd");
  return CHX_OK;
}

chx_status chx_gate_set(chx_gate *g, const float *params, const float *mean, const float *istd) {
  g_err.clear();
  chx_status st = check_device(g);
  if (st) return st;
  if (params) {
    for (int64_t i = 0; i < MLP_NPARAM; ++i)
      if (!isfinite(params[i])) return fail(CHX_ERR_INVALID_ARG, "parameter %lld is not finite", (long long)i);
    GCHK(hipMemcpy(g->p, params, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice), "write params");
    GCHK(mlp_apply_mask(g->p, g->mask, MLP_NPARAM, nullptr), "mask params");
    GCHK(mlp_fill(g->m, MLP_NPARAM, 0.f, nullptr), "clear moments");
    GCHK(mlp_fill(g->v, MLP_NPARAM, 0.f, nullptr), "clear moments");
    GCHK(mlp_weights_bf16(g->p, g->pb, g->pbF, nullptr), "weights to bf16");
    g->t = 0;
  }
  if ((mean == nullptr) != (istd == nullptr))
    return fail(CHX_ERR_INVALID_ARG, "mean and istd must be given together");
  if (mean) {
    for (int c = 0; c < MLP_IN; ++c)
      if (!isfinite(mean[c]) || !isfinite(istd[c]) || !(istd[c] > 0.f))
        return fail(CHX_ERR_INVALID_ARG, "feature scaling %d is invalid", c);
    GCHK(hipMemcpy(g->mean, mean, sizeof(float) * MLP_IN, hipMemcpyHostToDevice), "write mean");
    GCHK(hipMemcpy(g->istd, istd, sizeof(float) * MLP_IN, hipMemcpyHostToDevice), "write istd");
    g->have_stats = true;
  }
  GCHK(hipStreamSynchronize(nullptr), "synchronise");
  return CHX_OK;
}

chx_status chx_gate_features(const double *x0, const double *ld, const double *ln_growth,
                             double t, int64_t n, float *features_out, uint32_t flags,
                             void *stream) {
  g_err.clear();
  hipStream_t s;
  chx_status st = stream_for(flags, stream, &s);
  if (st) return st;
  if (n < 0) return fail(CHX_ERR_INVALID_ARG, "n must be >= 0");
  if (!(t > 0.0) || !isfinite(t)) return fail(CHX_ERR_INVALID_ARG, "t must be finite and > 0");
  if (n == 0) return CHX_OK;
  if (!x0 || !ld || !ln_growth || !features_out) return fail(CHX_ERR_INVALID_ARG, "NULL pointer");
  const bool dev = flags & CHX_PTR_DEVICE;
  Scratch S(s);
  const double *dx = S.in(x0, (size_t)n * 4, dev);
  const double *dl = S.in(ld, (size_t)n, dev);
  const double *dg = S.in(ln_growth, (size_t)n * 2, dev);
  float *out = dev ? features_out : S.get<float>((size_t)n * MLP_IN);
  if (S.err != hipSuccess) return dev_fail(S.err, "stage inputs");
  GCHK(mlp_features(dx, dl, dg, t, n, out, s), "features");
  if (!dev) {
    GCHK(hipMemcpyAsync(features_out, out, sizeof(float) * n * MLP_IN, hipMemcpyDeviceToHost, s), "read features");
    GCHK(hipStreamSynchronize(s), "synchronise");
  }
  return CHX_OK;
}

chx_status chx_gate_classify(const chx_gate *g, const chx_system *sys, const double *x0,
                             const uint8_t *mask, int64_t n, const chx_options *opt,
                             double t_gate, float conf_min, int8_t *label_out,
                             uint8_t *source_out, float *confidence_out,
                             chx_gate_stats *stats) {
  g_err.clear();
  chx_status st = check_device(g);
  if (st) return st;
  if ((st = check_system(sys))) return st;
  if (sys->kind != CHX_SYS_HENON_HEILES)
    return fail(CHX_ERR_UNSUPPORTED, "the gate's features are defined for Henon-Heiles only");
  Plan pl;
  if ((st = make_plan(sys, opt, &pl))) return st;
  const uint32_t ind = pl.o.indicators;
  if (!(ind & CHX_IND_SALI) || !(ind & CHX_IND_LD))
    return fail(CHX_ERR_INVALID_ARG, "the gate needs the SALI and LD indicators");
  if (ind & (CHX_IND_GALI | CHX_IND_LYAP))
    return fail(CHX_ERR_INVALID_ARG, "GALI and Lyapunov indicators are not available with the gate");
  if (n < 0) return fail(CHX_ERR_INVALID_ARG, "n must be >= 0");
  if (!(conf_min >= 0.5f && conf_min <= 1.0f))
    return fail(CHX_ERR_INVALID_ARG, "conf_min must be in [0.5, 1]");
  if (!(t_gate > 0.0) || !isfinite(t_gate)) return fail(CHX_ERR_INVALID_ARG, "t_gate must be > 0");
  const double r = t_gate / pl.o.dt;
  const int64_t s_gate = (int64_t)nearbyint(r);
  if (fabs(r - (double)s_gate) > 1e-9 * (double)s_gate || s_gate % pl.K != 0 || s_gate <= 0 ||
      s_gate >= pl.n_total)
    return fail(CHX_ERR_INVALID_ARG, "t_gate must be a checkpoint time before T (t_gate/dt a multiple of %d below %lld)",
                pl.K, (long long)pl.n_total);
  if (stats) memset(stats, 0, sizeof *stats);
  if (n == 0) return CHX_OK;
  if (!x0 || !label_out) return fail(CHX_ERR_INVALID_ARG, "x0 or label_out is NULL");
  const bool dev = pl.o.flags & CHX_PTR_DEVICE;
  const hipStream_t s = dev ? (hipStream_t)pl.o.stream : nullptr;
  if (!dev && pl.o.stream) return fail(CHX_ERR_INVALID_ARG, "stream given without CHX_PTR_DEVICE");

  Scratch S(s);
  const double *dx0 = S.in(x0, (size_t)n * 4, dev);
  const uint8_t *dmask = S.in(mask, (size_t)n, dev);
  int *status1 = S.get<int>(n);
  int8_t *label1 = S.get<int8_t>(n);
  double *ld = S.get<double>(n);
  double *lg = S.get<double>((size_t)n * 2);
  float *feat = S.get<float>((size_t)n * MLP_IN);
  float *pc = S.get<float>(n);
  float *conf = S.get<float>(n);
  uint8_t *keep = S.get<uint8_t>(n);
  unsigned long long *counts = S.get<unsigned long long>(4);
  int8_t *lab = dev ? label_out : S.get<int8_t>(n);
  uint8_t *src = dev ? source_out : (source_out ? S.get<uint8_t>(n) : nullptr);
  float *cfo = dev ? confidence_out : (confidence_out ? S.get<float>(n) : nullptr);
  if (S.err != hipSuccess) return dev_fail(S.err, "allocate gate buffers");

  hipEvent_t ev[4] = {};
  for (auto &e : ev) GCHK(hipEventCreate(&e), "create event");
  struct EvGuard {
    hipEvent_t *ev;
    ~EvGuard() {
      for (int i = 0; i < 4; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    }
  } evg{ev};

  chx_options dopt = pl.o;
  dopt.flags = CHX_PTR_DEVICE;
  dopt.stream = s;
  dopt.w0 = opt->w0;
  if (opt->w0 && !dev) return fail(CHX_ERR_INVALID_ARG, "w0 with host pointers is not supported by the gate");
  chx_ensemble *e1 = nullptr, *e2 = nullptr;
  int64_t *orbit = nullptr;
  struct EnsGuard {
    chx_ensemble **a, **b;
    int64_t **orbit;
    hipStream_t s;
    ~EnsGuard() {
      if (*orbit) (void)hipFreeAsync(*orbit, s);
      release(*a);
      release(*b);
    }
  } eg{&e1, &e2, &orbit, s};

  GCHK(hipEventRecord(ev[0], s), "event");
  if ((st = create(sys, dx0, dmask, n, &dopt, &e1))) return st;
  if ((st = advance(e1, s_gate))) return st;
  GCHK(hipEventRecord(ev[1], s), "event");
  chx_result r1;
  memset(&r1, 0, sizeof r1);
  r1.status = status1;
  r1.label = label1;
  r1.ld = ld;
  r1.ln_growth = lg;
  if ((st = results(e1, &r1))) return st;
  GCHK(mlp_features(dx0, ld, lg, t_gate, n, feat, s), "features");
  if ((st = infer_dev(g, feat, n, pc, conf, s))) return st;
  GCHK(gate_select(n, status1, label1, pc, conf, conf_min, lab, src, keep, cfo, counts, s),
       "select");
  GCHK(hipEventRecord(ev[2], s), "event");
  if ((st = subset(e1, keep, &e2, &orbit))) return st;
  release(e1);
  e1 = nullptr;
  const int64_t n2 = e2->n_all;
  if (n2 > 0) {
    if ((st = advance(e2, pl.n_total))) return st;
    int8_t *label2 = S.get<int8_t>(n2);
    if (!label2) return dev_fail(S.err, "allocate labels");
    chx_result r2;
    memset(&r2, 0, sizeof r2);
    r2.label = label2;
    if ((st = results(e2, &r2))) return st;
    GCHK(gate_scatter(n2, orbit, label2, lab, s), "merge labels");
  }
  GCHK(hipEventRecord(ev[3], s), "event");
  unsigned long long hc[4] = {0, 0, 0, 0};
  GCHK(hipMemcpyAsync(hc, counts, sizeof hc, hipMemcpyDeviceToHost, s), "read counts");
  if (!dev) {
    GCHK(hipMemcpyAsync(label_out, lab, (size_t)n, hipMemcpyDeviceToHost, s), "read labels");
    if (source_out) GCHK(hipMemcpyAsync(source_out, src, (size_t)n, hipMemcpyDeviceToHost, s), "read sources");
    if (confidence_out)
      GCHK(hipMemcpyAsync(confidence_out, cfo, sizeof(float) * n, hipMemcpyDeviceToHost, s), "read confidence");
  }
  GCHK(hipStreamSynchronize(s), "synchronise");
  if (stats) {
    stats->n_active = (int64_t)(hc[1] + hc[2] + hc[3]);
    stats->n_early = (int64_t)hc[1];
    stats->n_accepted = (int64_t)hc[2];
    stats->n_fallback = (int64_t)hc[3];
    float a = 0.f, b = 0.f, c = 0.f;
    (void)hipEventElapsedTime(&a, ev[0], ev[1]);
    (void)hipEventElapsedTime(&b, ev[1], ev[2]);
    (void)hipEventElapsedTime(&c, ev[2], ev[3]);
    stats->ms_gate = a;
    stats->ms_infer = b;
    stats->ms_fallback = c;
  }
  return CHX_OK;
}

}  // extern "C"
