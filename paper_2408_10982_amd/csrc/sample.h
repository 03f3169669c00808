// sample.h -- the sampling task table shared by the single-graph and batched
// entry points.
#pragma once

#include "common.h"

namespace im {

// One sampling task: sets [first, first+count) of (seed, stream) on a graph,
// written at positions [sample_base, sample_base+count) of the output.  A
// single-graph call is a one-task table; a batch lists many.
struct TaskDesc {
  const int32_t* in_off;
  const int32_t* in_src;
  const uint32_t* thr;
  const double* skip;      // IC run-length table or nullptr
  int32_t n;
  int32_t model;
  uint32_t seed_lo, seed_hi;
  uint32_t stream;
  uint32_t first;
  int64_t sample_base;
  int64_t count;
};

// Samples every task into one canonical CSR (off over all output positions,
// members task-local vertex ids, ascending per set).  max_n = largest n of
// the tasks.  Same contract as im_sample_rrr otherwise.
int sample_tasks(const TaskDesc* h_tasks, int ntasks, int64_t count_total, int32_t max_n,
                 int64_t* off, int32_t* mem, int64_t capacity, int64_t* total,
                 im_sample_stats* stats, bool sort_all, hipStream_t s);

int graph_ok(const im_graph* g);
TaskDesc task_of(const im_graph* g, uint64_t seed, uint32_t stream_tag, int64_t first,
                 int64_t count, int64_t sample_base);

}  // namespace im
