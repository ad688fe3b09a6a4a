// batched.hip -- one persistent launch for a mixed ensemble: Henon-Heiles
// and coupled-quartic orbits (one lane each) and FPU-16 / FPU-8 orbits (one
// 16-lane component row each), two deviation vectors per orbit, early exit
// at the first checkpoint with SALI below threshold.
//
// Work distribution.  Each system is a pool: its ensemble state (the same
// structure-of-arrays layout as the plain path), the steps done per orbit,
// and a circular queue of orbit indices with counters head / tail / tail0.
// A launch lets every wavefront integrate for a fixed budget of steps:
//   - a slot (lane or row) pops an orbit from its pool's queue (one
//     wave-aggregated atomicAdd per refill), integrates it in blocks of K
//     steps, and at every checkpoint an orbit that exited, stopped or
//     reached T is written back and the slot refills at once -- lanes are
//     never left idle while the queue has work;
//   - when its pool has nothing left to pop, the wavefront moves on to the
//     next pool (so one launch balances systems of different dimension);
//   - when the budget is spent, unfinished orbits are written back with
//     their step count and pushed to the queue's tail for the next launch.
// Pops only see [head, tail0), tail0 being the tail at launch start, so an
// orbit pushed in this launch is taken up by the next.  A one-thread flip
// kernel between launches clamps head and advances tail0; (flip, launch)
// pairs are captured once in a hipGraph and replayed until every queue is
// empty.  Because the per-orbit code is the same LaneOrbit / CRowOrbit as
// the plain kernels, an orbit's results do not depend on which slot or
// launch integrated it.
//
// Memory ordering.  Within one launch no orbit, step count or queue slot
// passes between wavefronts: an orbit is popped at most once per launch
// and what a launch pushes is popped only by a later one.  All hand-over
// goes from one kernel to a later one and across the XCDs, each with its
// own L2.  Plain accesses there would depend on the cache maintenance at
// the kernel boundary, and a plain store to a location that other kernels
// read or update with atomics (the counters) meets accesses that do not
// go through the writer's L2.  The protocol depends on neither:
//   - every access to data that changes hands (the orbit's state and step
//     count, queue slots, the counters) is an agent-scope atomic access,
//     which reads and writes the device-coherent copy, never a line one
//     XCD's L2 still holds from an earlier launch;
//   - push: the orbit's state and step count are stored, then the queue
//     slot is written with release semantics, so whoever reads the slot
//     finds the state it names already written;
//   - pop: the queue slot is read with acquire semantics before the state
//     it names is loaded;
//   - the counters move only by agent-scope atomics: the wave-aggregated
//     atomicAdd of pop and push, the loads of head and (acquire) tail0 when
//     a wavefront enters a pool, and the flip kernel's acquire load and
//     release store of tail0.
#include "batched.h"
#include "fput_crow.h"
#include "lane_kernel.h"

namespace chx {

namespace {

__device__ __forceinline__ unsigned long long ctr_acquire(unsigned long long *c) {
  return __hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ctr_relaxed(unsigned long long *c) {
  return __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ctr_release(unsigned long long *c, unsigned long long v) {
  __hip_atomic_store(c, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long tail0_of(const Pool &pl) {
  return ctr_acquire(&pl.ctr[2]);
}

// Wave-aggregated pop: lanes with need get an orbit index, or -1 when the
// launch's share of the queue is used up.
__device__ int64_t pop(const Pool &pl, unsigned long long t0, bool need) {
  const uint64_t m = __ballot(need);
  if (m == 0) return -1;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(&pl.ctr[0], (unsigned long long)__popcll(m));
  base = __shfl(base, leader);
  if (!need) return -1;
  const unsigned long long slot = base + __popcll(m & ((1ull << lane) - 1ull));
  if (slot >= t0) return -1;
  // acquire: pairs with the pushing launch's release of this slot
  return __hip_atomic_load(&pl.queue[slot % (unsigned long long)pl.qcap], __ATOMIC_ACQUIRE,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-aggregated push of unfinished orbits.
__device__ void push(const Pool &pl, bool want, int64_t idx) {
  const uint64_t m = __ballot(want);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(&pl.ctr[1], (unsigned long long)__popcll(m));
  base = __shfl(base, leader);
  if (want) {
    const unsigned long long slot = base + __popcll(m & ((1ull << lane) - 1ull));
    // release: the orbit's state and step count, stored before, are
    // visible to whoever acquires this slot
    __hip_atomic_store(&pl.queue[slot % (unsigned long long)pl.qcap], idx, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <class S>
__device__ int64_t run_lane_pool(const Pool &pl, int64_t left) {
  const StepArgs &a = pl.a;
  const unsigned long long t0 = tail0_of(pl);
  const StepCoef k(a.dt);
  const int K = a.K;
  LaneOrbit<S, 2, false, 2, true> o;
  int64_t idx = -1, s = 0;
  bool have = false;
  auto refill = [&]() {
    while (true) {
      const bool need = !have;
      if (!__any(need)) return;
      const int64_t got = pop(pl, t0, need);
      if (!__any(need && got >= 0)) return;
      if (need && got >= 0) {
        o.load(a, got);
        if (o.st == CHX_ORBIT_OK) {
          idx = got;
          s = gld<true>(&pl.sdone[got]);
          have = true;
        }
      }
    }
  };
  refill();
  while (left > 0 && __any(have)) {
    if (have) {
      o.block(a, k, K);
      s += K;
      const bool cont = o.checkpoint(a, (double)s * a.dt);
      if (!cont || s >= a.n_total) {
        o.store(a, idx);
        gst<true>(&pl.sdone[idx], s);
        have = false;
      }
    }
    left -= K;
    if (left > 0) refill();
  }
  if (have) {
    o.store(a, idx);
    gst<true>(&pl.sdone[idx], s);
  }
  push(pl, have, idx);
  return left;
}

template <int N>
__device__ int64_t run_crow_pool(const Pool &pl, int64_t left) {
  const StepArgs &a = pl.a;
  const unsigned long long t0 = tail0_of(pl);
  const StepCoef k(a.dt);
  const int K = a.K;
  CRowOrbit<N, 2, true> r;
  r.init_lane();
  const int lane = threadIdx.x & 63, head_lane = lane & ~15;
  int64_t idx = -1, s = 0;
  bool have = false;  // uniform over the row
  auto refill = [&]() {
    while (true) {
      const bool need = !have;
      if (!__any(need)) return;
      // one pop per row, by its first lane, then shared with the row; the
      // acquire is one wavefront instruction, so it orders the state loads
      // of every lane of the row after it
      int64_t got = pop(pl, t0, need && (lane & 15) == 0);
      got = __shfl(got, head_lane);
      if (!__any(need && got >= 0)) return;
      if (need && got >= 0) {
        r.load(a, got);
        if (r.st == CHX_ORBIT_OK) {
          idx = got;
          s = gld<true>(&pl.sdone[got]);
          have = true;
        }
      }
    }
  };
  refill();
  while (left > 0 && __any(have)) {
    if (have) {
      r.block(a, k, K);
      s += K;
      const bool cont = r.checkpoint(a, (double)s * a.dt);
      if (!cont || s >= a.n_total) {
        r.store(a, idx);
        if ((lane & 15) == 0) gst<true>(&pl.sdone[idx], s);
        have = false;
      }
    }
    left -= K;
    if (left > 0) refill();
  }
  if (have) {
    r.store(a, idx);
    if ((lane & 15) == 0) gst<true>(&pl.sdone[idx], s);
  }
  push(pl, have && (lane & 15) == 0, idx);
  return left;
}

// Three wavefronts per SIMD: the union of the four pool paths would take 180
// VGPRs (two wavefronts); held to 168 the compiler spills 6 dwords, all
// outside the step loops.  The ordering rules are in the header comment.
__global__ void __launch_bounds__(256, 3) batched_kernel(const BatchArgs b) {
  const int wave = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  int p = 0;
  while (p + 1 < b.npool && wave >= b.split[p + 1]) ++p;
  int64_t left = b.budget;
  for (int tried = 0; tried < b.npool && left > 0; ++tried, p = (p + 1) % b.npool) {
    const Pool &pl = b.pool[p];
    const unsigned long long head = ctr_relaxed(&pl.ctr[0]);
    if (head >= tail0_of(pl)) continue;
    switch (pl.kind) {
    case POOL_HH2: left = run_lane_pool<SysHH>(pl, left); break;
    case POOL_QUARTIC3_2: left = run_lane_pool<SysQuartic<3>>(pl, left); break;
    case POOL_FPUT16_2: left = run_crow_pool<16>(pl, left); break;
    case POOL_FPUT8_2: left = run_crow_pool<8>(pl, left); break;
    }
  }
}

// Between launches: claims past tail0 return to it, and what was pushed in
// the last launch becomes poppable.  Agent-scope atomics throughout (the
// counters were last moved by atomicAdd on any XCD): acquire on entry,
// release of the new tail0 last.
__global__ void flip_kernel(const BatchArgs b) {
  const int p = threadIdx.x;
  if (p >= b.npool) return;
  unsigned long long *c = b.pool[p].ctr;
  const unsigned long long t0 = ctr_acquire(&c[2]);
  const unsigned long long head = ctr_relaxed(&c[0]);
  const unsigned long long tail = ctr_relaxed(&c[1]);
  if (head > t0) __hip_atomic_store(&c[0], t0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  ctr_release(&c[2], tail);
}

// Queue of all orbits 0..n-1; head = tail0 = 0, tail = n.
__global__ void queue_init_kernel(int64_t *queue, int64_t n, unsigned long long *ctr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) queue[i] = i;
  if (i == 0) {
    ctr[0] = 0;
    ctr[1] = (unsigned long long)n;
    ctr[2] = 0;
    ctr[3] = 0;
  }
}

__global__ void fill_i64_kernel(int64_t *p, int64_t n, int64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

bool pool_kind_of(int sys, int ndof, int M, int *kind) {
  if (M != 2) return false;
  if (sys == SYS_HH && ndof == 2) *kind = POOL_HH2;
  else if (sys == SYS_QUARTIC && ndof == 3) *kind = POOL_QUARTIC3_2;
  else if (sys == SYS_FPUT && ndof == 16) *kind = POOL_FPUT16_2;
  else if (sys == SYS_FPUT && ndof == 8) *kind = POOL_FPUT8_2;
  else return false;
  return true;
}

int pool_slot_width(int kind) {
  return (kind == POOL_FPUT16_2 || kind == POOL_FPUT8_2) ? 16 : 1;
}

hipError_t launch_queue_init(int64_t *queue, int64_t n, unsigned long long *ctr,
                             int64_t *sdone, int64_t pitch, hipStream_t s) {
  const int64_t m = n > 1 ? n : 1;
  hipLaunchKernelGGL(queue_init_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, queue,
                     n, ctr);
  hipLaunchKernelGGL(fill_i64_kernel, dim3((unsigned)((pitch + 255) / 256)), dim3(256), 0, s,
                     sdone, pitch, (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_batched(const BatchArgs &b, int blocks, int threads, hipStream_t s) {
  hipLaunchKernelGGL(flip_kernel, dim3(1), dim3(64), 0, s, b);
  hipLaunchKernelGGL(batched_kernel, dim3(blocks), dim3(threads), 0, s, b);
  return hipGetLastError();
}

hipError_t batched_occupancy(int threads, int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batched_kernel, threads, 0);
}

}  // namespace chx
