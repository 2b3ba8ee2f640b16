// gh_launch.h -- what the host side of the library and the per-k kernel
// objects share: launch arguments and the table of supported shapes.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/gheap.h"
#include "gh_device.h"

namespace gh {

// Parameters of a launch that are not pointers.  For the single-call entry
// points (ops == nullptr) `kind` and `n_total` describe the operations.
struct OpParams {
  u32 kind;
  u32 clock_mhz;   // device wall clock, ticks per microsecond
  u64 n_total;
  u32 nheaps;      // heaps in the set (operations naming another are rejected)
  u32 pad;
};

struct LaunchArgs {
  const HeapDesc* descs;
  const gh_op* ops;
  u32 nops;
  OpParams direct;
  const u64* in;
  u64* out;
  u32* counts;
  gh_logrec* log;
  Ctl* ctl;
  u32 workgroups;
  u32 threads;
  u32 form;         // 0: whole-root kernel; 1: general kernel (deleteMins of
                    // fewer than K entries, inserts of more than K entries);
                    // 2: bottom-up inserts; 3: whole-root operations run by
                    // one workgroup without locks (gh_private.hip)
  hipStream_t stream;
};

// A workgroup of T threads serves node capacity K when every thread handles
// 1..16 entries of a 2K-entry merge and T is a power of two in [64, 1024].
constexpr bool shape_ok(int K, int T) {
  return T >= 64 && T <= 1024 && (T & (T - 1)) == 0 && 2 * K >= T && 2 * K <= 16 * T;
}

// the persistent operation loop for entries of type Ent (u64 or e128):
// whole-root deleteMins only (gh_kernels.hip), or also deleteMins of fewer
// than K entries (gh_serve.hip)
template <int K, class Ent>
hipError_t launch_ops_k(const LaunchArgs& a);

// heap filter (gh_filter.hip): workspace size and the launch sequence
u64 filter_workspace_bytes(u64 max_nodes, u32 k, u32 ebytes);
hipError_t launch_filter(const HeapDesc* d, u64 max_nodes, u32 k, u32 ebytes, u64 bound,
                         void* work, u64* kept_out, hipStream_t st);
// the library's own filter workspace on device `dev` (heap_filter_noalloc):
// looked up once per device with that device current; nullptr on failure
hipError_t filter_scratch_init(int dev);
void* filter_scratch(int dev);
template <int K, class Ent>
hipError_t launch_ops_var_k(const LaunchArgs& a);
// the operation loop with bottom-up inserts (gh_bu.hip)
template <int K, class Ent>
hipError_t launch_ops_bu_k(const LaunchArgs& a);
// the one-workgroup operation loop (gh_private.hip)
template <int K, class Ent>
hipError_t launch_private_k(const LaunchArgs& a);
// tracing build only (GH_PHASE_TRACE): the whole-root kernels' phase trace
// (gh_kernels.hip): zero it (host == nullptr) or copy `words` words out
template <int K, class Ent>
hipError_t phase_trace_k(uint32_t* host, u64 words);

// ---------------------------------------------------------------------------
// Served form: device workspace layout
// ---------------------------------------------------------------------------
struct alignas(256) ServeHead {
  u32 claim;      // next queue slot a worker takes
  u32 pad0[31];
  u32 tail;       // queue slots the scheduler has published
  u32 done;       // the scheduler has admitted or rejected every request
  u32 pad1[30];
  u32 sched_cu;   // compute unit the scheduler runs on (valid once cu_ready)
  u32 cu_ready;
  u32 cu_left;    // slots that stepped aside from the scheduler's unit
  u32 pad2[29];
};
struct HeapSched {  // scheduler-private, one per heap
  u64 size;       // entries after every admitted request
  u32 seq;        // next operation rank on this heap
  u32 head;       // first deferred insert (request id), or NONE
  u32 last;       // last deferred insert
  u32 pad;
};
constexpr u32 SCHED_NONE = 0xFFFFFFFFu;

struct ServeWork {
  ServeHead* head;
  HeapSched* heaps;
  u32* next;      // per request: next deferred insert of the same heap
  u32* left;      // per request: operations not finished yet
  gh_op* queue;   // admitted operations, in admission order
  u32* qreq;      // request of each queued operation
  u64 max_ops;
  u32 ins_max;    // entries one insert operation takes (K, or the multi-batch limit)
  u32 pad;
};

struct ServeArgs {
  const HeapDesc* descs;
  u32 nheaps;
  const gh_op* reqs;
  u32 nreq;
  const u64* in;
  u64* out;
  gh_reqrec* recs;
  ServeWork w;
  Ctl* ctl;
  u32 clock_mhz;
  u32 workgroups;   // worker slots (the scheduler is one more workgroup)
  u32 threads;
  hipStream_t stream;
};

template <int K, class Ent>
hipError_t launch_serve_k(const ServeArgs& a);

// Knapsack branch and bound driver (one heap per instance).
struct KnapArgs {
  const HeapDesc* descs;
  u32 ninst;
  const u32* item_off;
  const u32* n;
  const u64* cap;
  const u32* w;
  const u32* v;
  u64* pool;
  u64 pool_per_inst;
  void* scratch;      // 3K entries per instance
  u32 gc_min;         // collect an instance's heap from this many entries (0: never)
  gh_knapres* res;
  Ctl* ctl;
  u32 workgroups;
  u32 threads;
  hipStream_t stream;
};

template <int K, class Ent>
hipError_t launch_knap_k(const KnapArgs& a);

// SSSP driver (one shared heap, dynamic tickets).
struct alignas(256) SsspState {
  u64 next_ticket;   // dynamic root tickets of heap 0
  u64 outstanding;   // entries pushed and not yet fully processed
  u64 trace_ops;     // trace cursors: records and entries claimed
  u64 trace_keys;
  u32 done;
  u32 pad[55];
};
struct SsspArgs {
  const HeapDesc* descs;
  u32 V;
  const u32* rowptr;
  const u32* col;
  const u32* w;
  u32 src;
  u32* dist;
  u64* push;
  u64 push_per_wg;
  gh_ssspstats* stats;
  SsspState* st;
  gh_sssptrace trace;   // d_ops == nullptr: no trace
  Ctl* ctl;
  u32 workgroups;
  u32 threads;
  hipStream_t stream;
};

template <int K>
hipError_t launch_sssp_k(const SsspArgs& a);

}  // namespace gh
