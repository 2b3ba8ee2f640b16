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
  hipStream_t stream;
};

// A workgroup of T threads serves node capacity K when every thread handles
// 1..16 entries of a 2K-entry merge and T is a power of two in [64, 1024].
constexpr bool shape_ok(int K, int T) {
  return T >= 64 && T <= 1024 && (T & (T - 1)) == 0 && 2 * K >= T && 2 * K <= 16 * T;
}

template <int K>
hipError_t launch_ops_k(const LaunchArgs& a);

}  // namespace gh
