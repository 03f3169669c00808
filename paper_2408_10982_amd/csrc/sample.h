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
  const uint32_t* lt_index;  // LT search index or nullptr
  int64_t num_edges;
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

// Where phase 1 of a sampling call left its sets (the stream's staging arena
// and per-position metadata), and the call's exact counters.
struct ArenaRun {
  uint64_t cnt = 0;
  const int32_t* arena = nullptr;
  const int64_t* start = nullptr;
  const int32_t* lens = nullptr;
  bool sort = false;
  int32_t passes = 0;  // main launches run (more than 1: the arena was short)
  int64_t total = 0, examined = 0, live = 0;
  int64_t large_sets = 0, large_total = 0, large_examined = 0, large_live = 0;
  int64_t redo_examined = 0;
  double ms_main = 0.0, ms_large = 0.0;  // only when timed
};

// Phase 1: samples every task into the call's arena and writes the
// canonical offsets (off, count_total + 1 entries).  expect: a guess of the
// member total used to size the arena (0: none).  stop_above > 0: a total
// above it is only counted (the sets need not be kept: the caller reports
// IM_ERANGE), so a short arena is not refilled.  R->total holds the member
// total once a pass has counted it, also when the call then fails (a short
// workspace for the larger arena).  Synchronises s.
int sample_to_arena(const TaskDesc* h_tasks, int ntasks, int64_t count_total, int32_t max_n,
                    int64_t* off, int64_t expect, int64_t stop_above, bool sort_all, bool timed,
                    ArenaRun* R, hipStream_t s);
// Phase 2: copies the sets into mem (R.total entries at off).  The stream's
// arena must be untouched since phase 1.  ms (optional) gets the device time
// and then the call waits for the copy.
int gather_arena(const ArenaRun& R, const int64_t* off, int32_t* mem, double* ms, hipStream_t s);

int graph_ok(const im_graph* g);
// Returns the sampling slots (task table, metadata, arena, walk lists,
// large-set workers) to the workspace once the sets have been gathered.
void release_sampling();
// Workspace bytes of one sampling call (ws_sample): `full` with every
// large-set worker the launch can use, else the minimum (one worker).
size_t ws_sample(int num_cus, int64_t count, int64_t capacity, int32_t max_n, int32_t model,
                 bool full);
TaskDesc task_of(const im_graph* g, uint64_t seed, uint32_t stream_tag, int64_t first,
                 int64_t count, int64_t sample_base);

}  // namespace im
