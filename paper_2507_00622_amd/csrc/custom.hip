// custom.hip -- user-supplied systems: separable (CHX_SYS_CUSTOM: the
// user's potential, gradient and Hessian) or general (CHX_SYS_CUSTOM_GENERAL:
// the user's field J grad H over a generic number type, and H), HIP device
// code compiled at run time with hipRTC together with the library's own
// lane-per-orbit kernel templates (lane_kernel.h, lane_rk.h), so a custom
// system runs the same Yoshida-4 (separable only), DOP853 and adaptive
// DOP8(5) kernels, checkpoints and indicators as the built-in ones.  The
// paper's package integrates any Hamiltonian system given by its user; this
// is that entry, for N <= CHX_CUSTOM_MAX_NDOF (8).  The DOP853 kernels keep
// their per-stage records in LDS: plans needing more than 1 KB per orbit are
// refused before any device work.
//
// The kernel headers are read from the csrc/ directory beside libchx.so
// (and include/chx.h from ../include), so the run-time compilation uses the
// same sources as the built library.  hipRTC has no host runtime headers:
// hip/hip_runtime.h, stddef.h and stdint.h are given as small stand-ins
// holding what the headers' host-side declarations name (never compiled
// into device code).  Compiled programs are cached per process, keyed by
// the source text, ndof and the kernel instantiation, and loaded on each
// device where they run.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "chx_internal.h"
#include "ensemble.h"

namespace chx {
namespace host {

namespace {

const char *kRuntimeStub =
    "#pragma once\n"
    "typedef int hipError_t;\n"
    "typedef struct ihipStream_t *hipStream_t;\n"
    "enum { hipSuccess = 0, hipErrorInvalidValue = 1 };\n"
    "static inline hipError_t hipGetLastError() { return 0; }\n"
    "#define hipLaunchKernelGGL(...) ((void)0)\n";
const char *kStdintStub =
    "#pragma once\n"
    "typedef signed char int8_t; typedef unsigned char uint8_t;\n"
    "typedef short int16_t; typedef unsigned short uint16_t;\n"
    "typedef int int32_t; typedef unsigned int uint32_t;\n"
    "typedef long int64_t; typedef unsigned long uint64_t;\n"
    "#define INT64_MAX 9223372036854775807L\n";
const char *kStddefStub = "#pragma once\n";

// The wrappers that turn the user's functions into a system of the lane
// kernels, and the kernel that sets H(0) and the LD integrand at t = 0
// (the built-in set-up kernel knows only the built-in systems).  Separable
// form: V, grad V, Hess V.
const char *kWrapper = R"(
namespace chx {
struct SysCustom {
  static constexpr int N = CHX_CUSTOM_NDOF;
  static constexpr int NH = N * (N + 1) / 2;
  static constexpr bool diag_only = false;
  __device__ static inline void force(const double *q, double *F, const double *prm) {
    ::chx_force(q, F, prm);
  }
  __device__ static inline void hess_scaled(const double *q, double h, double *Hs,
                                            const double *prm) {
    ::chx_hess(q, Hs, prm);
#pragma unroll
    for (int i = 0; i < NH; ++i) Hs[i] *= h;
  }
  __device__ static inline double potential(const double *q, const double *prm) {
    return ::chx_potential(q, prm);
  }
};
}  // namespace chx

extern "C" __global__ void chx_custom_init(const chx::StepArgs a) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n || a.st[i] != CHX_ORBIT_OK) return;
  constexpr int N = chx::SysCustom::N;
  const long P = a.pitch;
  double x[2 * N], F[N];
  for (int c = 0; c < 2 * N; ++c) x[c] = a.x[c * P + i];
  chx::SysCustom::force(x, F, a.prm);
  double kin = 0.0, g = 0.0;
  for (int r = 0; r < N; ++r) {
    kin += x[N + r] * x[N + r];
    g += (a.ld_p == 0.5) ? sqrt(fabs(x[N + r])) : pow(fabs(x[N + r]), a.ld_p);
    g += (a.ld_p == 0.5) ? sqrt(fabs(F[r])) : pow(fabs(F[r]), a.ld_p);
  }
  a.sc[chx::SC_H0 * P + i] = 0.5 * kin + chx::SysCustom::potential(x, a.prm);
  a.sc[chx::SC_GPREV * P + i] = (a.ind & CHX_IND_LD) ? g : 0.0;
}
)";

// General form (any Hamiltonian): the field f = J grad H written once over
// T = double and T = MDual<M> (value and M derivative parts), and H itself;
// the Runge-Kutta kernels take the field, the records and the tangents
// from it exactly as for the built-in double pendulum.
const char *kWrapperGeneral = R"(
namespace chx {
struct SysCustom {
  static constexpr int N = CHX_CUSTOM_NDOF;
  static constexpr int NREC = 2 * N;  // stage record: the stage state
  __device__ static inline void rhs_rec(const double *x, double *f, double *rec,
                                        const double *prm) {
#pragma unroll
    for (int c = 0; c < 2 * N; ++c) rec[c] = x[c];
    ::chx_field<double>(x, f, prm);
  }
  __device__ static inline void jvp(const double *rec, const double *dx, double *df,
                                    const double *prm) {
    MDual<1> X[2 * N], F[2 * N];
#pragma unroll
    for (int c = 0; c < 2 * N; ++c) {
      X[c].v = rec[c];
      X[c].d[0] = dx[c];
    }
    ::chx_field<MDual<1>>(X, F, prm);
#pragma unroll
    for (int c = 0; c < 2 * N; ++c) df[c] = F[c].d[0];
  }
  template <int M>
  __device__ static inline void rhs_multi(const double *x, const double (&dx)[M][2 * N],
                                          double *f, double (&df)[M][2 * N], const double *prm) {
    MDual<M> X[2 * N], F[2 * N];
#pragma unroll
    for (int c = 0; c < 2 * N; ++c) {
      X[c].v = x[c];
#pragma unroll
      for (int v = 0; v < M; ++v) X[c].d[v] = dx[v][c];
    }
    ::chx_field<MDual<M>>(X, F, prm);
#pragma unroll
    for (int c = 0; c < 2 * N; ++c) {
      f[c] = F[c].v;
#pragma unroll
      for (int v = 0; v < M; ++v) df[v][c] = F[c].d[v];
    }
  }
  __device__ static inline double hamiltonian(const double *x, const double *prm) {
    return ::chx_hamiltonian(x, prm);
  }
};
}  // namespace chx

extern "C" __global__ void chx_custom_init(const chx::StepArgs a) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n || a.st[i] != CHX_ORBIT_OK) return;
  constexpr int N = chx::SysCustom::N;
  const long P = a.pitch;
  double x[2 * N], f[2 * N];
  for (int c = 0; c < 2 * N; ++c) x[c] = a.x[c * P + i];
  ::chx_field<double>(x, f, a.prm);
  double g = 0.0;
  for (int c = 0; c < 2 * N; ++c)
    g += (a.ld_p == 0.5) ? sqrt(fabs(f[c])) : pow(fabs(f[c]), a.ld_p);
  a.sc[chx::SC_H0 * P + i] = chx::SysCustom::hamiltonian(x, a.prm);
  a.sc[chx::SC_GPREV * P + i] = (a.ind & CHX_IND_LD) ? g : 0.0;
}
)";

struct Loaded {
  hipModule_t mod = nullptr;
  hipFunction_t kernel = nullptr, init = nullptr;
};
struct Program {
  std::vector<char> code;
  std::string lowered;        // the integration kernel's symbol
  std::map<int, Loaded> dev;  // the code object loaded on each device used
};

std::mutex g_mu;
std::map<std::string, std::unique_ptr<Program>> g_progs;

std::string read_file(const std::string &p, bool *ok) {
  std::ifstream f(p);
  std::stringstream s;
  s << f.rdbuf();
  *ok = f.good() || f.eof();
  return s.str();
}

std::string lib_dir() {
  Dl_info info{};
  if (!dladdr((void *)&lib_dir, &info) || !info.dli_fname) return std::string();
  std::string p = info.dli_fname;
  const size_t k = p.rfind('/');
  return k == std::string::npos ? std::string(".") : p.substr(0, k);
}

// "chx::lane_kernel<chx::SysCustom, M, GP, MS>" and the like
std::string kernel_expr(int integrator, int M, bool gp, int m_s) {
  char b[128];
  if (integrator == CHX_INT_YOSHIDA4) {
    const int ms = (!gp && M >= 2 && m_s == 2) ? 2 : -1;
    snprintf(b, sizeof b, "chx::lane_kernel<chx::SysCustom, %d, %s, %d>", M, gp ? "true" : "false",
             ms);
  } else {
    snprintf(b, sizeof b, "chx::%s<chx::SysCustom, %d, %s>",
             integrator == CHX_INT_DOP853 ? "lane_rk_kernel" : "lane_rka_kernel", M,
             gp ? "true" : "false");
  }
  return b;
}

chx_status compile(const std::string &src, int ndof, bool general, const std::string &expr,
                   Program *pg) {
  const std::string dir = lib_dir();
  if (dir.empty()) return fail(CHX_ERR_INTERNAL, "custom system: cannot locate libchx.so");
  const char *hdr[] = {"chx_internal.h", "device_math.h", "systems.h", "lane_kernel.h",
                       "dop853.h", "systems_dp.h", "lane_rk.h"};
  std::vector<std::string> names, bodies;
  for (const char *h : hdr) {
    bool ok = false;
    bodies.push_back(read_file(dir + "/csrc/" + h, &ok));
    if (!ok || bodies.back().empty())
      return fail(CHX_ERR_INTERNAL, "custom system: kernel header %s/csrc/%s not found", dir.c_str(), h);
    names.push_back(h);
  }
  {
    bool ok = false;
    bodies.push_back(read_file(dir + "/../include/chx.h", &ok));
    if (!ok || bodies.back().empty())
      return fail(CHX_ERR_INTERNAL, "custom system: %s/../include/chx.h not found", dir.c_str());
    names.push_back("../../include/chx.h");
  }
  names.push_back("hip/hip_runtime.h");
  bodies.push_back(kRuntimeStub);
  names.push_back("stdint.h");
  bodies.push_back(kStdintStub);
  names.push_back("stddef.h");
  bodies.push_back(kStddefStub);
  std::vector<const char *> hn, hb;
  for (size_t i = 0; i < names.size(); ++i) {
    hn.push_back(names[i].c_str());
    hb.push_back(bodies[i].c_str());
  }
  const std::string full = "#include \"lane_rk.h\"\n#define CHX_CUSTOM_NDOF " +
                           std::to_string(ndof) + "\n#line 1 \"custom system\"\n" + src +
                           "\n#line 1 \"custom wrapper\"\n" +
                           (general ? kWrapperGeneral : kWrapper);
  hiprtcProgram p;
  if (hiprtcCreateProgram(&p, full.c_str(), "custom.hip", (int)hn.size(), hb.data(), hn.data()) !=
      HIPRTC_SUCCESS)
    return fail(CHX_ERR_INTERNAL, "custom system: hiprtcCreateProgram failed");
  if (hiprtcAddNameExpression(p, expr.c_str()) != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&p);
    return fail(CHX_ERR_INTERNAL, "custom system: cannot name kernel %s", expr.c_str());
  }
  const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                        "-Wno-cuda-compat", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(p, (int)(sizeof opts / sizeof opts[0]), opts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(p, &ls);
  std::string log(ls + 1, '\0');
  if (ls) hiprtcGetProgramLog(p, &log[0]);
  if (r != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&p);
    if (log.size() > 3000) log = log.substr(0, 3000) + " ...";
    return fail(CHX_ERR_INVALID_ARG, "custom system source does not compile: %s", log.c_str());
  }
  const char *low = nullptr;
  if (hiprtcGetLoweredName(p, expr.c_str(), &low) != HIPRTC_SUCCESS || !low) {
    hiprtcDestroyProgram(&p);
    return fail(CHX_ERR_INTERNAL, "custom system: kernel %s not instantiated", expr.c_str());
  }
  pg->lowered = low;
  size_t cs = 0;
  hiprtcResult rc = hiprtcGetCodeSize(p, &cs);
  if (rc == HIPRTC_SUCCESS && cs > 0) {
    pg->code.resize(cs);
    rc = hiprtcGetCode(p, pg->code.data());
  }
  hiprtcDestroyProgram(&p);
  if (rc != HIPRTC_SUCCESS || cs == 0)
    return fail(CHX_ERR_INTERNAL, "custom system: no code object from hipRTC");
  return CHX_OK;
}

}  // namespace

// Compile (or find) the program of the ensemble's custom system for its
// plan; no device work, so compile errors surface before any allocation.
chx_status custom_prepare(const std::string &src, int ndof, bool general, const Plan &pl,
                          void **handle) {
  const bool gp = (pl.o.indicators & CHX_IND_LD) && pl.o.ld_p != 0.5;
  const std::string expr = kernel_expr(pl.o.integrator, pl.M, gp, pl.m_s);
  const std::string key =
      std::to_string(ndof) + (general ? " general\n" : " separable\n") + expr + "\n" + src;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_progs.find(key);
  if (it == g_progs.end()) {
    auto pg = std::make_unique<Program>();
    const chx_status st = compile(src, ndof, general, expr, pg.get());
    if (st) return st;
    it = g_progs.emplace(key, std::move(pg)).first;
  }
  *handle = it->second.get();
  return CHX_OK;
}

// LDS bytes per lane of the DOP853 kernels for a custom system: per stage
// the positions (separable) or the stage state (general; none when one or
// two vectors go through the stages with the state), and for the adaptive
// solver the vectors' step-start values.
size_t custom_rk_lds_per_lane(bool general, bool adaptive, int N, int M) {
  if (M == 0) return 0;
  const int stage = general ? ((M <= 2) ? 0 : 2 * N) : N;
  return sizeof(double) * (size_t)(12 * stage + (adaptive ? M * 2 * N : 0));
}

namespace {
// the program's functions on the current device (loaded there at first use)
hipError_t load(Program *pg, Loaded **out) {
  int d = 0;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) return e;
  Loaded &l = pg->dev[d];
  if (!l.mod) {
    if ((e = hipModuleLoadData(&l.mod, pg->code.data())) != hipSuccess) {
      l = Loaded();
      return e;
    }
    if ((e = hipModuleGetFunction(&l.kernel, l.mod, pg->lowered.c_str())) != hipSuccess ||
        (e = hipModuleGetFunction(&l.init, l.mod, "chx_custom_init")) != hipSuccess) {
      (void)hipModuleUnload(l.mod);
      l = Loaded();
      return e;
    }
  }
  *out = &l;
  return hipSuccess;
}
}  // namespace

// Unloads every user-system code object from each device it was loaded on,
// after that device's work has finished; the compiled code stays cached
// and is loaded again on its next use.
hipError_t custom_unload_all() {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  hipError_t e = hipGetDevice(&cur), first = hipSuccess;
  if (e != hipSuccess) return e;
  for (auto &kv : g_progs) {
    for (auto &dl : kv.second->dev) {
      if (!dl.second.mod) continue;
      hipError_t u = hipSetDevice(dl.first);
      if (u == hipSuccess) u = hipDeviceSynchronize();
      if (u == hipSuccess) u = hipModuleUnload(dl.second.mod);
      if (u != hipSuccess && first == hipSuccess) first = u;
    }
    kv.second->dev.clear();
  }
  e = hipSetDevice(cur);
  return first != hipSuccess ? first : e;
}

// H(0) and the LD integrand at t = 0 of every active orbit (after the
// built-in set-up kernel).
hipError_t custom_init(void *handle, const StepArgs &a, hipStream_t s) {
  Program *pg = (Program *)handle;
  if (a.n == 0) return hipSuccess;
  hipError_t e;
  Loaded *l = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if ((e = load(pg, &l)) != hipSuccess) return e;
  }
  StepArgs arg = a;
  void *params[] = {&arg};
  const unsigned grid = (unsigned)((a.n + 255) / 256);
  return hipModuleLaunchKernel(l->init, grid, 1, 1, 256, 1, 1, 0, s, params, nullptr);
}

// One integration launch with the plan's kernel: lane per orbit, block
// threads per block; the Runge-Kutta kernels take their stage records and,
// adaptive, the attempted vectors in dynamic LDS, at most 64 KB per block.
hipError_t custom_launch(void *handle, bool general, const Plan &pl, const StepArgs &a,
                         int block, hipStream_t s) {
  Program *pg = (Program *)handle;
  if (a.n == 0) return hipSuccess;
  hipError_t e;
  Loaded *l = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if ((e = load(pg, &l)) != hipSuccess) return e;
  }
  size_t lds = 0;
  if (pl.o.integrator != CHX_INT_YOSHIDA4 && pl.M > 0) {
    const size_t per = custom_rk_lds_per_lane(general, pl.o.integrator == CHX_INT_DOP853_ADAPTIVE,
                                              pl.N, pl.M);
    while (block > 64 && per * (size_t)block > 65536) block /= 2;
    lds = per * (size_t)block;
    if (lds > 65536) return hipErrorInvalidValue;  // rejected by the plan already
  }
  StepArgs arg = a;
  void *params[] = {&arg};
  const unsigned grid = (unsigned)((a.n + block - 1) / block);
  return hipModuleLaunchKernel(l->kernel, grid, 1, 1, (unsigned)block, 1, 1, (unsigned)lds, s,
                               params, nullptr);
}

}  // namespace host
}  // namespace chx
