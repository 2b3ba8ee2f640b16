// gh_kops.h -- the persistent operation loop (k_ops) and its launch, shared
// by three objects per node capacity, one per form:
//   FORM_WHOLE   (gh_kernels.hip) inserts of up to K entries, whole-root
//                deleteMins;
//   FORM_GENERAL (gh_serve.hip) also deleteMins of fewer than K entries and
//                inserts of more than K entries in one root hold;
//   FORM_BU      (gh_bu.hip) bottom-up inserts of up to K entries, and no
//                deleteMin (insert phases).
// They live in separate objects so that the whole-root kernel is compiled
// without the other code paths next to it.
#pragma once
#include "gh_launch.h"
#include "gh_ops.h"
#include "gh_ops_bu.h"
#include "gh_ops_multi.h"

namespace gh {

// Persistent operation loop: each workgroup claims the next operation in list
// order, waits for its arrival time, and runs it (many operations in flight,
// Sec. 3.3).  With ops == nullptr the operations are synthesized from
// `direct` (the single-call insert and deleteMin entry points).
// kind given to a record the kernel refuses (> GH_OP_DELETE_MIN)
constexpr u32 KIND_REFUSED = 0xFFu;

constexpr int FORM_WHOLE = 0, FORM_GENERAL = 1, FORM_BU = 2;

template <int K, int T, int Form, class Ent>
__global__ __launch_bounds__(T) void k_ops(const HeapDesc* __restrict__ descs,
                                           const gh_op* __restrict__ ops, u32 nops,
                                           OpParams direct, const Ent* __restrict__ in,
                                           Ent* __restrict__ out, u32* __restrict__ counts,
                                           gh_logrec* __restrict__ log, Ctl* __restrict__ ctl) {
  __shared__ __align__(16) Ent lds[5 * K];
  lds_t<Ent>* const L = (lds_t<Ent>*)lds;
  __shared__ OpShared sh;
  const int tid = threadIdx.x;
  constexpr bool VarDel = Form == FORM_GENERAL;
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
      // the whole-root kernel refuses deleteMins of other counts, the
      // bottom-up form every deleteMin: such a record reads as malformed
      // below (rejected, the root still passes)
      if (Form == FORM_WHOLE && op.kind == GH_OP_DELETE_MIN && op.n != 0 && op.n != (u32)K)
        op.kind = KIND_REFUSED;
      if (Form == FORM_BU && op.kind == GH_OP_DELETE_MIN) op.kind = KIND_REFUSED;
    } else {
      // an insert of n_total entries: operations of up to K entries, or in
      // the general kernel of up to multi_max_batches(K) * K
      constexpr u64 CH = VarDel ? (u64)multi_max_batches(K) * K : (u64)K;
      op.heap = 0;
      op.kind = direct.kind;
      op.seq = i;
      op.off = (u64)i * CH;
      op.arrival_ns = 0;
      u64 rem = direct.n_total - (u64)i * CH;
      op.n = direct.kind == GH_OP_INSERT ? (u32)(rem < CH ? rem : CH)
                                         : (VarDel ? (u32)direct.n_total : 0u);
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
    const u64 ticket = *gptr(&H.meta->base) + op.seq;
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
    // n: insert 1..K entries (up to multi_max_batches(K) * K in the general
    // instantiation); deleteMin 1..K entries, 0 meaning K (fewer than K only
    // in the general instantiation, more never)
    constexpr u32 INS_MAX = VarDel ? (u32)multi_max_batches(K) * K : (u32)K;
    const bool malformed = op.kind > GH_OP_DELETE_MIN ||
                           (op.kind == GH_OP_INSERT && op.n > INS_MAX) ||
                           (VarDel && op.kind == GH_OP_DELETE_MIN && op.n > (u32)K);
    if (malformed || (op.kind == GH_OP_INSERT && op.n == 0)) {
      if (malformed && tid == 0) note_error(ctl, ERR_INVAL);
      r = op_pass_root(H, ticket, sh, ctl);
      if (malformed) r.flags |= F_REJECT;
    } else if (op.kind == GH_OP_INSERT) {
      if constexpr (Form == FORM_BU) {
        r = op_insert_bu<K, T, Ent>(H, ticket, in + op.off, op.n, L, sh, ctl);
      } else if constexpr (VarDel) {
        if (op.n > (u32)K)
          r = op_insert_multi<K, T, Ent>(descs + op.heap, ticket, in + op.off, op.n, L, sh, ctl);
        else r = op_insert<K, T, Ent>(H, ticket, in + op.off, op.n, L, sh, ctl);
      } else {
        r = op_insert<K, T, Ent>(H, ticket, in + op.off, op.n, L, sh, ctl);
      }
    } else if constexpr (VarDel) {
      if (op.n == 0 || op.n == (u32)K)
        r = op_delete<K, T, Ent>(H, ticket, out + op.off, K, L, sh, ctl);
      else
        r = op_delete<K, T, Ent, true>(H, ticket, out + op.off, op.n, L, sh, ctl);
    } else {
      r = op_delete<K, T, Ent>(H, ticket, out + op.off, K, L, sh, ctl);
    }
    if (tid == 0) {
      if (counts) counts[i] = op.kind == GH_OP_INSERT ? 0u : r.count;
      if (log) {
        const u64 t0 = ctl->t0;
        gh_logrec rec;
        rec.ticket = ticket;
        rec.count = r.count;
        rec.levels = (uint16_t)r.levels;
        rec.kind = (uint8_t)(op.kind == KIND_REFUSED ? GH_OP_DELETE_MIN : op.kind);
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

template <int K, int T, int Form, class Ent>
static hipError_t launch_kops_t(const LaunchArgs& a) {
  hipLaunchKernelGGL((k_ops<K, T, Form, Ent>), dim3(a.workgroups), dim3(T), 0, a.stream,
                     a.descs, a.ops, a.nops, a.direct, reinterpret_cast<const Ent*>(a.in),
                     reinterpret_cast<Ent*>(a.out), a.counts, a.log, a.ctl);
  return hipGetLastError();
}

template <int K, int Form, class Ent>
static hipError_t launch_kops_shape(const LaunchArgs& a) {
  switch (a.threads) {
#define GH_CASE(TT)                                                             \
  case TT:                                                                      \
    if constexpr (shape_ok(K, TT)) return launch_kops_t<K, TT, Form, Ent>(a); \
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
