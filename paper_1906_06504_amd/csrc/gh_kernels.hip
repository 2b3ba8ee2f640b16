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

// ---------------------------------------------------------------------------
// Served form: one persistent launch.  Workgroup 0 is the scheduler: it
// walks the requests in arrival order, waits for each arrival time, admits
// the request if its heap's memory allows (deleteMins always; an insert when
// the heap's size after everything admitted plus n fits max_keys, otherwise
// it waits in the heap's FIFO of deferred inserts until admitted deleteMins
// make room), and appends the admitted request's operations to a queue with
// the heap's next tickets.  Every other workgroup is a slot that claims queue
// entries in order and runs them exactly like k_ops.  A heap's admission
// order depends only on its own requests, so its results are the same alone
// and in any mix.
// ---------------------------------------------------------------------------
// Scheduler's per-heap state, kept in LDS (dynamic shared memory sized by the
// number of heaps) so that admitting a request touches no global memory on
// its critical path.
struct SchedHot {
  u64 size;   // entries after every admitted request
  u64 cap;    // memory budget (the heap's max_keys)
  u64 base;   // ticket of the first operation of this launch
  u32 seq;    // next operation rank on this heap
  u32 head;   // first deferred insert (request id), or SCHED_NONE
};
static_assert(sizeof(SchedHot) == 32, "sched layout");
extern __shared__ __align__(16) unsigned char gh_dyn_lds[];

template <int K>
struct Scheduler {
  u32 nheaps;
  const gh_op* reqs;
  gh_reqrec* recs;
  ServeWork w;
  SchedHot* hot;
  u64 t0;
  u32 tail;       // queue slots written
  u32 published;  // queue slots published
  bool overflow;

  __device__ void put_op(u32 r, u32 heap, u32 kind, u32 n, u32 seq, u64 off) {
    u64* qw = reinterpret_cast<u64*>(w.queue + tail);
    st_relaxed(qw + 0, (u64)heap | ((u64)kind << 32));
    st_relaxed(qw + 1, (u64)n | ((u64)seq << 32));
    st_relaxed(qw + 2, off);
    __hip_atomic_store(w.qreq + tail, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ++tail;
  }

  __device__ void publish_queue() {
    if (published == tail) return;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // queue entries are complete
    __hip_atomic_store(&w.head->tail, tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    published = tail;
  }

  __device__ void write_rec(u32 r, const gh_reqrec& rec) {
    const u64* src = reinterpret_cast<const u64*>(&rec);
    u64* dst = reinterpret_cast<u64*>(recs + r);
#pragma unroll
    for (int i = 0; i < 4; ++i) st_relaxed(dst + i, src[i]);
  }

  __device__ void reject(u32 r, u32 kind) {
    gh_reqrec rec;
    rec.first_ticket = 0;
    rec.count = 0;
    rec.nops = 0;
    rec.kind = (uint8_t)kind;
    rec.flags = 0x40;
    rec.t_admit = (u32)(now_ticks() - t0);
    rec.t_done = rec.t_admit;
    rec.reserved = 0;
    write_rec(r, rec);
  }

  // Admit request r: its operations get the heap's next tickets.  A request
  // that no longer fits the operation queue is rejected instead (its heap's
  // tickets and size are left as they were).
  __device__ void admit(u32 r, const gh_op& q, SchedHot& hs, u32 flags) {
    const u32 nops = q.kind == GH_OP_DELETE_MIN ? 1u : (q.n + K - 1) / K;
    if ((u64)tail + nops > w.max_ops) {
      overflow = true;
      reject(r, q.kind);
      return;
    }
    gh_reqrec rec;
    rec.first_ticket = hs.base + hs.seq;
    rec.count = q.kind == GH_OP_DELETE_MIN ? 0u : q.n;
    rec.nops = (uint16_t)nops;
    rec.kind = (uint8_t)q.kind;
    rec.flags = (uint8_t)(flags | 1u);
    rec.t_admit = (u32)(now_ticks() - t0);
    rec.t_done = rec.t_admit;
    rec.reserved = 0;
    // slots write count and t_done of this record: every word goes out
    // coherently and is complete before the queue entries are published
    write_rec(r, rec);
    __hip_atomic_store(w.left + r, nops, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (q.kind == GH_OP_DELETE_MIN) {
      put_op(r, q.heap, GH_OP_DELETE_MIN, 0, hs.seq++, q.off);
      hs.size -= hs.size < (u64)K ? hs.size : (u64)K;
    } else {
      for (u32 c = 0; c < nops; ++c) {
        const u32 nc = (q.n - c * K) < (u32)K ? (q.n - c * K) : (u32)K;
        put_op(r, q.heap, GH_OP_INSERT, nc, hs.seq++, q.off + (u64)c * K);
      }
      hs.size += q.n;
    }
  }
};

template <int K, int T>
__global__ __launch_bounds__(T) void k_serve(const HeapDesc* __restrict__ descs, u32 nheaps,
                                             const gh_op* __restrict__ reqs, u32 nreq,
                                             const u64* __restrict__ in, u64* __restrict__ out,
                                             gh_reqrec* __restrict__ recs, ServeWork w,
                                             Ctl* __restrict__ ctl, u32 clock_mhz) {
  __shared__ __align__(16) u64 lds[5 * K];
  __shared__ OpShared sh;
  const int tid = threadIdx.x;

  if (blockIdx.x == 0) {
    // ---- scheduler ----
    SchedHot* hot = reinterpret_cast<SchedHot*>(gh_dyn_lds);
    for (u32 h = tid; h < nheaps; h += T) {
      const u64 rw = ld_relaxed(&descs[h].meta->root);
      SchedHot hs;
      hs.size = rw_m(rw) * (u64)K + rw_s(rw);
      hs.cap = descs[h].max_keys;
      hs.base = descs[h].meta->base;
      hs.seq = 0;
      hs.head = SCHED_NONE;
      hot[h] = hs;
      w.heaps[h].last = SCHED_NONE;
    }
    __syncthreads();
    constexpr u32 CH = (5 * K) / 4;   // request records staged in LDS per chunk
    gh_op* stage = reinterpret_cast<gh_op*>(lds);
    Scheduler<K> S;
    S.nheaps = nheaps;
    S.reqs = reqs;
    S.recs = recs;
    S.w = w;
    S.hot = hot;
    S.t0 = ctl->t0;
    S.tail = 0;
    S.published = 0;
    S.overflow = false;
    for (u32 c0 = 0; c0 < nreq; c0 += CH) {
      const u32 cn = nreq - c0 < CH ? nreq - c0 : CH;
      for (u32 j = tid; j < cn; j += T) stage[j] = reqs[c0 + j];
      __syncthreads();
      if (tid == 0) {
        for (u32 j = 0; j < cn; ++j) {
          const u32 r = c0 + j;
          const gh_op q = stage[j];
          // arrival (bounded to one minute after the start)
          const u64 ns = q.arrival_ns < 60000000000ull ? q.arrival_ns : 60000000000ull;
          const u64 due = S.t0 + (ns * clock_mhz) / 1000ull;
          if (now_ticks() < due) {
            S.publish_queue();   // nothing else to do until then
            while (now_ticks() < due) {
              if (ld_relaxed32(&ctl->abort)) break;
              __builtin_amdgcn_s_sleep(4);
            }
          }
          if (q.heap >= nheaps || q.kind > GH_OP_DELETE_MIN) {
            S.reject(r, q.kind);
            note_error(ctl, ERR_INVAL);
            continue;
          }
          SchedHot hs = hot[q.heap];
          if (q.kind == GH_OP_DELETE_MIN) {
            S.admit(r, q, hs, 0);
            // room freed: admit deferred inserts of this heap in order
            while (hs.head != SCHED_NONE) {
              const gh_op d = reqs[hs.head];
              if (hs.size + d.n > hs.cap) break;
              const u32 dr = hs.head;
              hs.head = w.next[dr];
              if (hs.head == SCHED_NONE) w.heaps[q.heap].last = SCHED_NONE;
              S.admit(dr, d, hs, 2u);
            }
          } else if ((u64)q.n > hs.cap || q.n > 65535u * (u32)K) {
            S.reject(r, q.kind);
          } else if (hs.head == SCHED_NONE && hs.size + q.n <= hs.cap) {
            S.admit(r, q, hs, 0);
          } else {
            // wait for memory behind earlier deferred inserts
            w.next[r] = SCHED_NONE;
            const u32 last = hs.head == SCHED_NONE ? SCHED_NONE : w.heaps[q.heap].last;
            if (last == SCHED_NONE) hs.head = r;
            else w.next[last] = r;
            w.heaps[q.heap].last = r;
          }
          hot[q.heap] = hs;
          if (S.tail - S.published >= 64) S.publish_queue();
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      // inserts still waiting for memory when the stream ends are rejected
      for (u32 h = 0; h < nheaps; ++h) {
        u32 r = hot[h].head;
        while (r != SCHED_NONE) {
          S.reject(r, GH_OP_INSERT);
          r = w.next[r];
        }
      }
      if (S.overflow) note_error(ctl, ERR_NOMEM);
      S.publish_queue();
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __hip_atomic_store(&w.head->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }

  // ---- slots ----
  for (;;) {
    if (tid == 0) {
      u32 i = atomicAdd(&w.head->claim, 1u);
      for (;;) {
        const u32 tl = ld_relaxed32(&w.head->tail);
        if (i < tl) break;
        if (ld_relaxed32(&w.head->done)) {
          if (i >= ld_relaxed32(&w.head->tail)) i = 0xFFFFFFFFu;
          break;
        }
        if (ld_relaxed32(&ctl->abort)) {
          i = 0xFFFFFFFFu;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      sh.op = i;
      sh.t_claim = now_ticks();
    }
    __syncthreads();
    const u32 i = sh.op;
    if (i == 0xFFFFFFFFu) break;
    const u64* qw = reinterpret_cast<const u64*>(w.queue + i);
    const u64 q0 = ld_relaxed(qw + 0), q1 = ld_relaxed(qw + 1), q2 = ld_relaxed(qw + 2);
    const u32 r = __hip_atomic_load(w.qreq + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    gh_op op;
    op.heap = (u32)q0;
    op.kind = (u32)(q0 >> 32);
    op.n = (u32)q1;
    op.seq = (u32)(q1 >> 32);
    op.off = q2;
    op.arrival_ns = 0;
    const HeapDesc H = descs[op.heap];
    const u64 ticket = H.meta->base + op.seq;
    OpResult res;
    if (op.kind == GH_OP_INSERT) {
      res = op_insert<K, T>(H, ticket, in + op.off, op.n, lds, sh, ctl);
    } else {
      res = op_delete<K, T>(H, ticket, out + op.off, lds, sh, ctl);
    }
    if (tid == 0) {
      if (op.kind == GH_OP_DELETE_MIN)
        __hip_atomic_store(&recs[r].count, res.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (atomicSub(&w.left[r], 1u) == 1u)
        __hip_atomic_store(&recs[r].t_done, (u32)(now_ticks() - ctl->t0), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

template <int K, int T>
static hipError_t launch_serve_t(const ServeArgs& a) {
  hipLaunchKernelGGL((k_serve<K, T>), dim3(a.workgroups + 1), dim3(T),
                     (size_t)a.nheaps * sizeof(SchedHot), a.stream, a.descs,
                     a.nheaps, a.reqs, a.nreq, a.in, a.out, a.recs, a.w, a.ctl, a.clock_mhz);
  return hipGetLastError();
}

template <>
hipError_t launch_serve_k<GH_K>(const ServeArgs& a) {
  constexpr int K = GH_K;
  switch (a.threads) {
#define GH_CASE(TT)                                                 \
  case TT:                                                          \
    if constexpr (shape_ok(K, TT)) return launch_serve_t<K, TT>(a); \
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
