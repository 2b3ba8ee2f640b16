// gh_kernels.hip -- kernels of the generalized heap for one node capacity.
// Compiled once per supported k with -DGH_K=<k>; each object exports
// gh::launch_ops_k<k>() and gh::launch_prep().
#include "gh_launch.h"
#include "gh_ops.h"

#ifndef GH_K
#error "compile with -DGH_K=<node capacity>"
#endif

namespace gh {

// Persistent operation loop: each workgroup claims the next operation in list
// order, waits for its arrival time, and runs it (many operations in flight,
// Sec. 3.3).  With ops == nullptr the operations are synthesized from
// `direct` (the single-call insert and deleteMin entry points).
template <int K, int T>
__global__ __launch_bounds__(T) void k_ops(const HeapDesc* __restrict__ descs,
                                           const gh_op* __restrict__ ops, u32 nops,
                                           OpParams direct, const u64* __restrict__ in,
                                           u64* __restrict__ out, u32* __restrict__ counts,
                                           gh_logrec* __restrict__ log, Ctl* __restrict__ ctl) {
  __shared__ __align__(16) u64 lds[5 * K];
  __shared__ OpShared sh;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      u32 i = atomicAdd(&ctl->next_op, 1u);
      if (ld_relaxed32(&ctl->abort)) i = nops;
      sh.op = i;
      sh.t_claim = now_ticks();
    }
    __syncthreads();
    const u32 i = sh.op;
    if (i >= nops) break;
    gh_op op;
    if (ops) {
      op = ops[i];
    } else {
      op.heap = 0;
      op.kind = direct.kind;
      op.seq = i;
      op.off = (u64)i * K;
      op.arrival_ns = 0;
      u64 rem = direct.n_total - (u64)i * K;
      op.n = direct.kind == GH_OP_INSERT ? (u32)(rem < (u64)K ? rem : (u64)K) : 0u;
    }
    if (op.heap >= direct.nheaps) {
      // no heap to pass: record the error and drop the record
      if (tid == 0) {
        note_error(ctl, ERR_INVAL);
        if (counts) counts[i] = 0;
        if (log) {
          gh_logrec rec{};
          rec.kind = (uint8_t)op.kind;
          rec.flags = (uint8_t)F_REJECT;
          log[i] = rec;
        }
      }
      __syncthreads();
      continue;
    }
    const HeapDesc H = descs[op.heap];
    const u64 ticket = H.meta->base + op.seq;
    if (op.arrival_ns != 0 && tid == 0) {
      // admission: the request may not start before its arrival time
      // (bounded to one minute after the submission started)
      u64 ns = op.arrival_ns < 60000000000ull ? op.arrival_ns : 60000000000ull;
      const u64 due = ctl->t0 + (ns * direct.clock_mhz) / 1000ull;
      while (now_ticks() < due) {
        if (ld_relaxed32(&ctl->abort)) break;
        __builtin_amdgcn_s_sleep(8);
      }
    }
    OpResult r;
    const bool malformed = op.kind > GH_OP_DELETE_MIN ||
                           (op.kind == GH_OP_INSERT && op.n > (u32)K);
    if (malformed || (op.kind == GH_OP_INSERT && op.n == 0)) {
      if (malformed && tid == 0) note_error(ctl, ERR_INVAL);
      r = op_pass_root(H, ticket, sh, ctl);
      if (malformed) r.flags |= F_REJECT;
    } else if (op.kind == GH_OP_INSERT) {
      r = op_insert<K, T>(H, ticket, in + op.off, op.n, lds, sh, ctl);
    } else {
      r = op_delete<K, T>(H, ticket, out + op.off, lds, sh, ctl);
    }
    if (tid == 0) {
      if (counts) counts[i] = op.kind == GH_OP_INSERT ? 0u : r.count;
      if (log) {
        const u64 t0 = ctl->t0;
        gh_logrec rec;
        rec.ticket = ticket;
        rec.count = r.count;
        rec.levels = (uint16_t)r.levels;
        rec.kind = (uint8_t)op.kind;
        rec.flags = (uint8_t)(r.flags | (r.ok ? 0u : F_ABORT));
        rec.pb = (uint16_t)sh.s;
        rec.reserved = 0;
        rec.t_claim = (u32)(sh.t_claim - t0);
        rec.t_root = (u32)(sh.t_root - t0);
        rec.t_done = (u32)(now_ticks() - t0);
        log[i] = rec;
      }
    }
    __syncthreads();
  }
}

template <int K, int T>
static hipError_t launch_t(const LaunchArgs& a) {
  hipLaunchKernelGGL((k_ops<K, T>), dim3(a.workgroups), dim3(T), 0, a.stream, a.descs, a.ops,
                     a.nops, a.direct, a.in, a.out, a.counts, a.log, a.ctl);
  return hipGetLastError();
}

template <>
hipError_t launch_ops_k<GH_K>(const LaunchArgs& a) {
  constexpr int K = GH_K;
  switch (a.threads) {
#define GH_CASE(TT)                                              \
  case TT:                                                       \
    if constexpr (shape_ok(K, TT)) return launch_t<K, TT>(a);    \
    break;
    GH_CASE(64)
    GH_CASE(128)
    GH_CASE(256)
    GH_CASE(512)
    GH_CASE(1024)
#undef GH_CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace gh
