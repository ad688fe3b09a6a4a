// batched.h -- pools and launch arguments of the persistent batched kernel.
#pragma once
#include "chx_internal.h"

namespace chx {

enum PoolKind { POOL_HH2 = 0, POOL_QUARTIC3_2 = 1, POOL_FPUT16_2 = 2, POOL_FPUT8_2 = 3 };

struct Pool {
  StepArgs a;                 // the pool's ensemble (s_begin/s_end unused)
  int64_t *sdone;             // [pitch] steps done per orbit
  int64_t *queue;             // [qcap] circular queue of orbit indices
  unsigned long long *ctr;    // head, tail, tail0, spare
  int64_t qcap;
  int kind;                   // PoolKind
};

constexpr int MAX_POOLS = 4;

struct BatchArgs {
  Pool pool[MAX_POOLS];
  int npool;
  int64_t budget;             // steps per wavefront per launch, multiple of every K
  int split[MAX_POOLS + 1];   // wavefronts [split[p], split[p+1]) start on pool p
};

bool pool_kind_of(int sys, int ndof, int M, int *kind);
int pool_slot_width(int kind);  // lanes per orbit
hipError_t launch_queue_init(int64_t *queue, int64_t n, unsigned long long *ctr,
                             int64_t *sdone, int64_t pitch, hipStream_t s);
// one flip kernel then one persistent launch
hipError_t launch_batched(const BatchArgs &b, int blocks, int threads, hipStream_t s);
hipError_t batched_occupancy(int threads, int *blocks_per_cu);

}  // namespace chx
