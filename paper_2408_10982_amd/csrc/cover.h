// cover.h -- arguments of the greedy max-k-cover launches, shared by the
// standard greedy, the RandGreedi local step and the batched path.
#pragma once

#include "common.h"

namespace im {

constexpr int kMaxParts = 256;

// The greedy runs on m "partitions" at once; each has its own vertex range
// (positions [pbase[p], pbase[p+1]) of the count array), its own covered
// flags and its own picks.  Plain greedy: m = 1.  RandGreedi: m vertex
// partitions over one shared sample universe.  Batch: one partition per task,
// each with its own samples (sbase) and task-local ids (local_ids).
struct CoverArgs {
  int32_t n;                 // positions (vertices over all partitions)
  int32_t m;                 // partitions
  int64_t count;             // samples (all partitions together when sbase is set)
  int32_t k;                 // picks (the largest k when kpart is set)
  const int64_t* __restrict__ off;       // sample-major CSR over all samples
  const int32_t* __restrict__ mem;
  const int64_t* __restrict__ inc_off;   // by position
  const int32_t* __restrict__ inc_mem;   // sample ids (partition-local when sbase is set)
  const int32_t* __restrict__ order;     // n: vertex at each position (nullptr: identity)
  const int32_t* __restrict__ pos_of;    // n: position of each vertex (nullptr: identity)
  const uint8_t* __restrict__ part;      // n: partition of each vertex (RandGreedi), or nullptr
  const int32_t* __restrict__ mpos;      // off[count]: count position of each member
                                         // (RandGreedi: read in place of mem, part and
                                         // pos_of), or nullptr
  const int64_t* __restrict__ pbase;     // m+1: positions of partition p (nullptr: [0, n))
  const int32_t* __restrict__ kpart;     // m: picks per partition (nullptr: k)
  const int64_t* __restrict__ koff;      // m: first output slot (nullptr: p * k)
  const int64_t* __restrict__ sbase;     // m+1: samples of partition p (nullptr: shared)
  int32_t local_ids;                     // members and seeds are partition-local ids
  int32_t pos_keys;                      // argmax keys carry the position, not the vertex
                                         // (order ascending within each partition, so the
                                         // lowest position of a count is its lowest id)
  uint32_t* __restrict__ cnt;            // n, by position: uncovered samples of the vertex
  uint8_t* __restrict__ covered;         // sbase ? count : m * count
  unsigned long long* __restrict__ gmax; // k * m argmax keys, one row per pick
  int32_t* __restrict__ done;            // set once no partition can gain
  int32_t* __restrict__ seeds;           // output slots
  int64_t* __restrict__ gains;
  int32_t* __restrict__ nsel;            // m
  int64_t* __restrict__ cover;           // m
  // one-partition covers: a pick that covers at least this many samples
  // rebuilds all counts instead of decrementing per member (0: never);
  // set by launch_cover
  int64_t recount_min;
  // candidate lists of the partition argmax (nullptr: every pick scans all
  // counts): kListCap positions per partition, their number, and the count
  // that no position outside the list exceeds
  int32_t* __restrict__ cand;
  int32_t* __restrict__ cand_n;          // m
  uint32_t* __restrict__ tau;            // m
};

// Positions a partition's candidate list holds.
constexpr int kListCap = 1024;
// Candidate lists are used when partitions average at most this many
// positions (a rebuild scans one partition with one workgroup).
constexpr int64_t kListMaxPart = (int64_t)1 << 18;

// Destroys the calling thread's captured cover graphs (im_release).
void release_cover_graphs();

// Enqueues the whole greedy (2k + 2 launches, plus one per early pick of a
// one-partition cover).  gains must be zeroed first.
int launch_cover(CoverArgs& A, hipStream_t s);

// Workspace bytes of im_greedy_cover and im_randgreedi (each call's scratch
// and the scans it runs).
size_t ws_greedy(int32_t n, int64_t count, int32_t k);
size_t ws_randgreedi(int32_t n, int64_t count, int64_t total, int32_t k, int32_t m);
// Workspace bytes of im_stream_cover and im_greedi_offline.
size_t ws_stream(int32_t n, int64_t count, int32_t k, int32_t m, double delta);
size_t ws_offline(int32_t n, int64_t count, int32_t k, int32_t m);

}  // namespace im
