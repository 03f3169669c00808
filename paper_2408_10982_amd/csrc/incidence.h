// incidence.h -- the covering-subset build shared by the single-collection
// entry point and the batched path.
#pragma once

#include "common.h"

namespace im {

// A sample-major collection to transpose.  With ntasks == 0 it is one
// collection over vertices [0, nv).  With ntasks > 0, sample j belongs to the
// task t with sbase[t] <= j < sbase[t + 1]; its members are task-local ids,
// placed at vbase[t] + id, and its id inside S(v) is task-local (j - sbase[t]).
struct IncSrc {
  const int64_t* off;
  int64_t count;
  const int32_t* mem;
  int64_t total;
  const int64_t* sbase;
  const int64_t* vbase;
  int32_t ntasks;
  int64_t vspan;  // most vertices of one task (nv with ntasks == 0); 0: not known
};

// S(v) for v in [0, nv): inc_off nv + 1 entries, inc_mem total entries.
// Members outside [0, nv) are skipped.  Asynchronous on s.
int build_incidence(const IncSrc& src, int32_t nv, int64_t* inc_off, int32_t* inc_mem,
                    hipStream_t s);
// Workspace bytes of build_incidence: the least (a 2^24-pair round) or, with
// `full`, room to transpose every pair in one round.
size_t ws_incidence(int32_t nv, int64_t total, int32_t ntasks, bool full);

}  // namespace im
