// batched_host.hip -- host side of the persistent batched launch:
// validation, one ensemble per item, the queues, the autotuner and the
// hipGraph replay loop (chx_integrate_batched in include/chx.h).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batched.h"
#include "chx_internal.h"
#include "ensemble.h"

using namespace chx;
using namespace chx::host;

namespace {

// ---- autotune cache: GPU time per orbit-step of one pool kind at one
// block size, for the whole device ---------------------------------------
std::mutex g_tune_mu;
std::map<std::string, double> g_tune;
std::string g_tune_path;  // cache file last read ("" = none)

std::string tune_key(int kind, int threads, uint32_t ind) {
  char b[96];
  snprintf(b, sizeof b, "gfx950/kind%d/threads%d/ind%u", kind, threads, ind);
  return b;
}

// Reads the cache file named by CHX_AUTOTUNE_CACHE whenever that name
// differs from the file read last (timings already known are kept).
void tune_load() {
  const char *path = getenv("CHX_AUTOTUNE_CACHE");
  const std::string now = path ? path : "";
  if (now == g_tune_path) return;
  g_tune_path = now;
  if (!path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char key[128];
  double v;
  while (fscanf(f, "%127s %lf", key, &v) == 2) g_tune[key] = v;
  fclose(f);
}

void tune_store(const std::string &key, double v) {
  g_tune[key] = v;
  const char *path = getenv("CHX_AUTOTUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %.6e\n", key.c_str(), v);
  fclose(f);
}

struct PoolBuf {
  int64_t *sdone = nullptr, *queue = nullptr;
};

// Probe: one short launch of the persistent kernel on a copy of up to `m`
// orbits of pool `src`; returns seconds per orbit-step.
chx_status probe_cost(const Pool &src, const Plan &pl, int threads, int blocks, hipStream_t s,
                      double *cost) {
  const int64_t m = src.a.n;
  const int64_t Pm = ((m + 63) / 64) * 64;
  const int D = pl.D, M = pl.M;
  const size_t nd = (size_t)Pm * (D + (size_t)M * D + M + NSC);
  const size_t ni = (size_t)Pm * (M + 1);
  double *st = nullptr;
  int *it = nullptr;
  int64_t *sdone = nullptr, *queue = nullptr;
  unsigned long long *ctr = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipSuccess;
  auto ok = [&](hipError_t e) {
    if (he == hipSuccess) he = e;
    return he == hipSuccess;
  };
  ok(hipMallocAsync((void **)&st, sizeof(double) * nd, s));
  ok(hipMallocAsync((void **)&it, sizeof(int) * ni, s));
  ok(hipMallocAsync((void **)&sdone, sizeof(int64_t) * Pm, s));
  ok(hipMallocAsync((void **)&queue, sizeof(int64_t) * m, s));
  ok(hipMallocAsync((void **)&ctr, sizeof(unsigned long long) * 4, s));
  ok(hipEventCreate(&e0));
  ok(hipEventCreate(&e1));
  Pool p = src;
  if (he == hipSuccess) {
    // rows of the structure-of-arrays layout, m columns each
    const size_t rows_d = D + (size_t)M * D + M + NSC, rows_i = M + 1;
    ok(hipMemcpy2DAsync(st, Pm * sizeof(double), src.a.x, src.a.pitch * sizeof(double),
                        m * sizeof(double), rows_d, hipMemcpyDeviceToDevice, s));
    ok(hipMemcpy2DAsync(it, Pm * sizeof(int), src.a.ge, src.a.pitch * sizeof(int),
                        m * sizeof(int), rows_i, hipMemcpyDeviceToDevice, s));
    p.a.x = st;
    p.a.w = st + (size_t)D * Pm;
    p.a.gm = p.a.w + (size_t)M * D * Pm;
    p.a.sc = p.a.gm + (size_t)M * Pm;
    p.a.ge = it;
    p.a.st = it + (size_t)M * Pm;
    p.a.pitch = Pm;
    p.sdone = sdone;
    p.queue = queue;
    p.ctr = ctr;
    p.qcap = m;
  }
  BatchArgs b{};
  b.pool[0] = p;
  b.npool = 1;
  b.split[0] = 0;
  b.split[1] = blocks * (threads / 64);
  const int K = pl.K;
  float ms = 0.f;
  if (he == hipSuccess) {
    // warm-up launch, then a timed one on fresh queues
    b.budget = 4 * (int64_t)K;
    ok(launch_queue_init(queue, m, ctr, sdone, Pm, s));
    ok(launch_batched(b, blocks, threads, s));
    b.budget = 40 * (int64_t)K;
    ok(launch_queue_init(queue, m, ctr, sdone, Pm, s));
    ok(hipEventRecord(e0, s));
    ok(launch_batched(b, blocks, threads, s));
    ok(hipEventRecord(e1, s));
    ok(hipEventSynchronize(e1));
    ok(hipEventElapsedTime(&ms, e0, e1));
  }
  if (st) (void)hipFreeAsync(st, s);
  if (it) (void)hipFreeAsync(it, s);
  if (sdone) (void)hipFreeAsync(sdone, s);
  if (queue) (void)hipFreeAsync(queue, s);
  if (ctr) (void)hipFreeAsync(ctr, s);
  (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (he != hipSuccess) return dev_fail(he, "autotune probe");
  *cost = (double)ms * 1e-3 / ((double)m * (double)b.budget);
  return CHX_OK;
}

}  // namespace

extern "C" chx_status chx_integrate_batched(const chx_batch_item *items, int32_t n_items,
                                            const chx_options *opt, chx_result *per_item,
                                            chx_batch_stats *stats) {
  g_err.clear();
  if (!items || !per_item) return fail(CHX_ERR_INVALID_ARG, "items or results is NULL");
  if (n_items < 1 || n_items > MAX_POOLS)
    return fail(CHX_ERR_INVALID_ARG, "n_items must be 1..%d", MAX_POOLS);
  if (!opt) return fail(CHX_ERR_INVALID_ARG, "options is NULL");
  if (!(opt->indicators & CHX_IND_SALI))
    return fail(CHX_ERR_INVALID_ARG, "the batched form needs the SALI indicator");
  if (opt->indicators & (CHX_IND_GALI | CHX_IND_LYAP))
    return fail(CHX_ERR_UNSUPPORTED, "the batched form carries two deviation vectors: no GALI or Lyapunov");
  if (opt->w0) return fail(CHX_ERR_INVALID_ARG, "the batched form draws its deviation vectors: w0 must be NULL");
  if (opt->integrator != CHX_INT_YOSHIDA4)
    return fail(CHX_ERR_UNSUPPORTED, "the batched form integrates with Yoshida-4 only");
  std::vector<Plan> plans(n_items);
  std::vector<int> kinds(n_items);
  for (int i = 0; i < n_items; ++i) {
    chx_status st = check_system(&items[i].sys);
    if (st) return st;
    chx_options o = *opt;
    o.dt = items[i].dt;
    o.T = items[i].T;
    st = make_plan(&items[i].sys, &o, &plans[i]);
    if (st) return st;
    if ((plans[i].o.indicators & CHX_IND_LD) && plans[i].o.ld_p != 0.5)
      return fail(CHX_ERR_UNSUPPORTED, "the batched form computes the LD with p = 1/2 only");
    if (!pool_kind_of(items[i].sys.kind, items[i].sys.ndof, plans[i].M, &kinds[i]))
      return fail(CHX_ERR_UNSUPPORTED, "item %d: system kind %d ndof %d is not supported in the batched form", i, items[i].sys.kind, items[i].sys.ndof);
    if (plans[i].n_total % plans[i].K != 0)
      return fail(CHX_ERR_INVALID_ARG, "item %d: T/dt must be a multiple of renorm_every", i);
    if (items[i].n < 0) return fail(CHX_ERR_INVALID_ARG, "item %d: n must be >= 0", i);
    if (items[i].n > 0 && !items[i].x0) return fail(CHX_ERR_INVALID_ARG, "item %d: x0 is NULL", i);
  }
  const bool device = opt->flags & CHX_PTR_DEVICE;
  const hipStream_t cs = device ? (hipStream_t)opt->stream : nullptr;

  std::vector<chx_ensemble *> ens(n_items, nullptr);
  std::vector<PoolBuf> bufs(n_items);
  unsigned long long *ctr = nullptr;
  hipStream_t bs = nullptr;
  hipEvent_t ev = nullptr, t0 = nullptr, t1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t he = hipSuccess;
  chx_status st = CHX_OK;
  auto ok = [&](hipError_t e) {
    if (he == hipSuccess) he = e;
    return he == hipSuccess;
  };
  auto cleanup = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (bs) {
      for (auto &b : bufs) {
        if (b.sdone) (void)hipFreeAsync(b.sdone, bs);
        if (b.queue) (void)hipFreeAsync(b.queue, bs);
      }
      if (ctr) (void)hipFreeAsync(ctr, bs);
      (void)hipStreamSynchronize(bs);
      (void)hipStreamDestroy(bs);
    }
    if (ev) (void)hipEventDestroy(ev);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    for (auto *e : ens) release(e);
  };

  for (int i = 0; i < n_items; ++i) {
    chx_options o = *opt;
    o.dt = items[i].dt;
    o.T = items[i].T;
    o.seed = opt->seed + (uint64_t)i;
    st = create(&items[i].sys, items[i].x0, items[i].mask, items[i].n, &o, &ens[i]);
    if (st) {
      cleanup();
      return st;
    }
  }
  // our own stream, ordered after the caller's
  ok(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
  ok(hipEventCreate(&ev));
  ok(hipEventCreate(&t0));
  ok(hipEventCreate(&t1));
  ok(hipEventRecord(ev, cs));
  ok(hipStreamWaitEvent(bs, ev, 0));
  ok(hipMallocAsync((void **)&ctr, sizeof(unsigned long long) * 4 * MAX_POOLS, bs));
  BatchArgs b{};
  b.npool = n_items;
  for (int i = 0; i < n_items && he == hipSuccess; ++i) {
    chx_ensemble *e = ens[i];
    const int64_t na = e->n_active;
    ok(hipMallocAsync((void **)&bufs[i].sdone, sizeof(int64_t) * e->pitch, bs));
    ok(hipMallocAsync((void **)&bufs[i].queue, sizeof(int64_t) * (na > 0 ? na : 1), bs));
    if (he != hipSuccess) break;
    ok(launch_queue_init(bufs[i].queue, na, ctr + 4 * i, bufs[i].sdone, e->pitch, bs));
    Pool &p = b.pool[i];
    p.a = e->args;
    p.sdone = bufs[i].sdone;
    p.queue = bufs[i].queue;
    p.ctr = ctr + 4 * i;
    p.qcap = na > 0 ? na : 1;
    p.kind = kinds[i];
  }
  if (he != hipSuccess) {
    cleanup();
    return dev_fail(he, "batched set-up");
  }

  // ---- autotune: block size, per-system cost, wave split, launch budget
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  std::vector<int> cands;
  if (opt->block_size) cands.push_back(opt->block_size);
  else cands = {64, 128, 256};
  double best_t = -1.0;
  int best_threads = cands[0];
  std::vector<double> best_cost(n_items, 0.0);
  int from_cache = 1;
  for (int threads : cands) {
    int bpc = 0;
    if (!ok(batched_occupancy(threads, &bpc)) || bpc < 1) {
      he = hipSuccess;
      continue;
    }
    const int blocks = ncu * bpc;
    const int64_t waves = (int64_t)blocks * (threads / 64);
    double total = 0.0;
    std::vector<double> cost(n_items, 0.0);
    for (int i = 0; i < n_items; ++i) {
      const std::string key = tune_key(kinds[i], threads, opt->indicators);
      double c = 0.0;
      {
        std::lock_guard<std::mutex> g(g_tune_mu);
        tune_load();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) c = it->second;
      }
      if (c <= 0.0 && ens[i]->n_active > 0) {
        from_cache = 0;
        const int64_t slots = waves * 64 / pool_slot_width(kinds[i]);
        Pool probe = b.pool[i];
        probe.a.n = ens[i]->n_active < slots ? ens[i]->n_active : slots;
        st = probe_cost(probe, plans[i], threads, blocks, bs, &c);
        if (st) {
          cleanup();
          return st;
        }
        std::lock_guard<std::mutex> g(g_tune_mu);
        tune_store(key, c);
      }
      cost[i] = c;
      total += c * (double)ens[i]->n_active * (double)plans[i].n_total;
    }
    if (best_t < 0.0 || total < best_t) {
      best_t = total;
      best_threads = threads;
      best_cost = cost;
    }
  }
  int bpc = 1;
  ok(batched_occupancy(best_threads, &bpc));
  if (bpc < 1) bpc = 1;
  const int blocks = ncu * bpc;
  const int waves = blocks * (best_threads / 64);
  // waves per pool in proportion to its estimated GPU time
  {
    std::vector<double> w(n_items);
    double tot = 0.0;
    for (int i = 0; i < n_items; ++i) {
      w[i] = best_cost[i] * (double)ens[i]->n_active * (double)plans[i].n_total;
      tot += w[i];
    }
    b.split[0] = 0;
    double acc = 0.0;
    for (int i = 0; i < n_items; ++i) {
      acc += (tot > 0.0) ? w[i] / tot : 1.0 / n_items;
      b.split[i + 1] = (int)llround(acc * waves);
    }
    b.split[n_items] = waves;
  }
  // steps per launch: about 200 ms of GPU time per launch
  const int K = plans[0].K;
  int64_t budget = opt->steps_per_launch;
  if (budget <= 0) {
    double worst = 0.0;
    for (int i = 0; i < n_items; ++i) {
      const double slots = (double)waves * 64.0 / pool_slot_width(kinds[i]);
      worst = fmax(worst, best_cost[i] * slots);
    }
    budget = worst > 0.0 ? (int64_t)(0.2 / worst) : 100000;
  }
  budget = (budget / K) * K;
  if (budget < K) budget = K;
  b.budget = budget;

  // ---- capture R launches in a graph, replay until every queue is empty
  const int R = 4;
  ok(hipStreamBeginCapture(bs, hipStreamCaptureModeThreadLocal));
  for (int r = 0; r < R; ++r) ok(launch_batched(b, blocks, best_threads, bs));
  ok(hipStreamEndCapture(bs, &graph));
  if (he == hipSuccess) ok(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  unsigned long long hc[4 * MAX_POOLS];
  int launches = 0;
  float ms_total = 0.f;
  // a bound on the replays: every launch finishes budget steps on every busy slot
  int64_t max_launches = 16;
  for (int i = 0; i < n_items; ++i) {
    const double slots = (double)waves * 64.0 / pool_slot_width(kinds[i]);
    const double rounds = ceil((double)ens[i]->n_active / slots) + 1.0;
    max_launches += (int64_t)(rounds * ((double)plans[i].n_total / (double)budget + 1.0)) * 2;
  }
  bool done = false;
  while (he == hipSuccess && !done) {
    ok(hipEventRecord(t0, bs));
    ok(hipGraphLaunch(exec, bs));
    ok(hipEventRecord(t1, bs));
    ok(hipMemcpyAsync(hc, ctr, sizeof hc, hipMemcpyDeviceToHost, bs));
    ok(hipStreamSynchronize(bs));
    float ms = 0.f;
    if (he == hipSuccess) ok(hipEventElapsedTime(&ms, t0, t1));
    ms_total += ms;
    launches += R;
    done = true;
    for (int i = 0; i < n_items; ++i) {
      const unsigned long long head = hc[4 * i], tail = hc[4 * i + 1], tl0 = hc[4 * i + 2];
      const unsigned long long h = head < tl0 ? head : tl0;
      if (!(h == tail && tl0 == tail)) done = false;
    }
    if (!done && launches > max_launches) {
      cleanup();
      return fail(CHX_ERR_INTERNAL, "batched queues did not drain after %d launches", launches);
    }
  }
  if (he != hipSuccess) {
    cleanup();
    return dev_fail(he, "batched launches");
  }
  // results: every orbit is final; the caller's stream waits for ours
  int64_t osteps[MAX_POOLS] = {0, 0, 0, 0};
  for (int i = 0; i < n_items; ++i) {
    chx_ensemble *e = ens[i];
    if (e->n_active > 0) {
      std::vector<int64_t> sd(e->n_active);
      ok(hipMemcpyAsync(sd.data(), bufs[i].sdone, sizeof(int64_t) * e->n_active,
                        hipMemcpyDeviceToHost, bs));
      ok(hipStreamSynchronize(bs));
      for (int64_t v : sd) osteps[i] += v;
    }
    e->s_done = e->pl.n_total;
  }
  ok(hipEventRecord(ev, bs));
  ok(hipStreamWaitEvent(cs, ev, 0));
  for (int i = 0; i < n_items && he == hipSuccess && st == CHX_OK; ++i)
    if (items[i].n > 0) st = results(ens[i], &per_item[i]);
  if (stats && he == hipSuccess && st == CHX_OK) {
    memset(stats, 0, sizeof *stats);
    stats->threads_per_block = best_threads;
    stats->blocks = blocks;
    stats->launches = launches;
    stats->from_cache = from_cache;
    stats->steps_per_launch = budget;
    stats->integrate_ms = ms_total;
    for (int i = 0; i < n_items; ++i) {
      stats->orbit_steps[i] = osteps[i];
      stats->cost_ps[i] = best_cost[i] * 1e12;
    }
  }
  const hipError_t h_end = he;
  cleanup();
  if (h_end != hipSuccess) return dev_fail(h_end, "batched results");
  return st;
}
