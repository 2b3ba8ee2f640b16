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
  lu64* const L = (lu64*)lds;
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
    const bool malformed = op.kind > GH_OP_DELETE_MIN ||
                           (op.kind == GH_OP_INSERT && op.n > (u32)K);
    if (malformed || (op.kind == GH_OP_INSERT && op.n == 0)) {
      if (malformed && tid == 0) note_error(ctl, ERR_INVAL);
      r = op_pass_root(H, ticket, sh, ctl);
      if (malformed) r.flags |= F_REJECT;
    } else if (op.kind == GH_OP_INSERT) {
      r = op_insert<K, T>(H, ticket, in + op.off, op.n, L, sh, ctl);
    } else {
      r = op_delete<K, T>(H, ticket, out + op.off, L, sh, ctl);
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
// walks the requests in arrival order and admits every request once it is
// due: deleteMins always; an insert when the heap's size after everything
// admitted plus n fits max_keys, otherwise it waits in the heap's FIFO of
// deferred inserts until admitted deleteMins make room.  An admitted
// request's operations take the heap's next tickets and are appended to a
// queue.  Every other workgroup is a slot that claims queue entries in order
// and runs them exactly like k_ops.
//
// The scheduler works lane-parallel: heap h belongs to scheduler thread
// h mod T.  It takes the requests in windows (the due prefix of a staged
// chunk), sorts each window's requests stably by owner, and every thread
// admits its own requests in stream order; queue slots come from a shared
// counter, so one heap's operations stay in ticket order in the queue.  The
// queue tail is published at the end of each window.  A heap's admissions
// depend only on its own requests, so its results are the same alone and in
// any mix.
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
typedef __attribute__((address_space(3))) SchedHot lSchedHot;
__device__ __forceinline__ SchedHot hot_get(const lSchedHot* p) {
  SchedHot v;
  v.size = p->size;
  v.cap = p->cap;
  v.base = p->base;
  v.seq = p->seq;
  v.head = p->head;
  return v;
}
__device__ __forceinline__ void hot_put(lSchedHot* p, const SchedHot& v) {
  p->size = v.size;
  p->cap = v.cap;
  p->base = v.base;
  p->seq = v.seq;
  p->head = v.head;
}
extern __shared__ __align__(16) unsigned char gh_dyn_lds[];

// Scheduler values shared by its threads.
struct SchedShared {
  u64 now;        // clock of the current window
  u32 qtail;      // queue slots handed out
  u32 wend;       // end of the current window (index in the chunk)
  u32 overflow;   // the queue ran out of room
};
typedef __attribute__((address_space(3))) SchedShared lSchedShared;
typedef __attribute__((address_space(3))) gh_op lgh_op;
typedef __attribute__((address_space(3))) u32 lu32;
typedef __attribute__((address_space(3))) uint16_t lu16;
__device__ __forceinline__ gh_op stage_get(const lgh_op* p) {
  gh_op q;
  q.heap = p->heap;
  q.kind = p->kind;
  q.n = p->n;
  q.seq = p->seq;
  q.off = p->off;
  q.arrival_ns = p->arrival_ns;
  return q;
}
__device__ __forceinline__ void stage_put(lgh_op* p, const gh_op& q) {
  p->heap = q.heap;
  p->kind = q.kind;
  p->n = q.n;
  p->seq = q.seq;
  p->off = q.off;
  p->arrival_ns = q.arrival_ns;
}

// Queue entries of a request rejected after its slots were handed out.
constexpr u32 QUEUE_SKIP = 0xFFFFFFFFu;

template <int K>
struct Scheduler {
  u32 nheaps;
  const gh_op* reqs;
  gh_reqrec* recs;
  ServeWork w;
  lSchedHot* hot;
  lSchedShared* ss;
  u64 t0;

  __device__ void put_op(u32 slot, u32 r, u32 heap, u32 kind, u32 n, u32 seq, u64 off) const {
    u64* qw = reinterpret_cast<u64*>(w.queue + slot);
    st_relaxed(qw + 0, (u64)heap | ((u64)kind << 32));
    st_relaxed(qw + 1, (u64)n | ((u64)seq << 32));
    st_relaxed(qw + 2, off);
    __hip_atomic_store(w.qreq + slot, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  __device__ void write_rec(u32 r, const gh_reqrec& rec) const {
    const u64* src = reinterpret_cast<const u64*>(&rec);
    u64* dst = reinterpret_cast<u64*>(recs + r);
#pragma unroll
    for (int i = 0; i < 4; ++i) st_relaxed(dst + i, src[i]);
  }

  __device__ void reject(u32 r, u32 kind) const {
    gh_reqrec rec;
    rec.first_ticket = 0;
    rec.count = 0;
    rec.nops = 0;
    rec.kind = (uint8_t)kind;
    rec.flags = 0x40;
    rec.t_admit = (u32)(ss->now - t0);
    rec.t_done = rec.t_admit;
    rec.reserved = 0;
    write_rec(r, rec);
  }

  // Admit request r: its operations get the heap's next tickets and queue
  // slots.  A request that no longer fits the operation queue is rejected
  // instead (its heap's tickets and size are left as they were; slots it was
  // handed are marked to be skipped).
  __device__ void admit(u32 r, const gh_op& q, SchedHot& hs, u32 flags) const {
    const u32 nops = q.kind == GH_OP_DELETE_MIN ? 1u : (q.n + K - 1) / K;
    const u32 slot =
        __hip_atomic_fetch_add(&ss->qtail, nops, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if ((u64)slot + nops > w.max_ops) {
      for (u64 x = slot; x < w.max_ops && x < (u64)slot + nops; ++x)
        put_op((u32)x, QUEUE_SKIP, QUEUE_SKIP, 0, 0, 0, 0);
      ss->overflow = 1;
      reject(r, q.kind);
      return;
    }
    gh_reqrec rec;
    rec.first_ticket = hs.base + hs.seq;
    rec.count = q.kind == GH_OP_DELETE_MIN ? 0u : q.n;
    rec.nops = (uint16_t)nops;
    rec.kind = (uint8_t)q.kind;
    rec.flags = (uint8_t)(flags | 1u);
    rec.t_admit = (u32)(ss->now - t0);
    rec.t_done = rec.t_admit;
    rec.reserved = 0;
    // slots write count and t_done of this record: every word goes out
    // coherently and is complete before the queue entries are published
    write_rec(r, rec);
    __hip_atomic_store(w.left + r, nops, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (q.kind == GH_OP_DELETE_MIN) {
      put_op(slot, r, q.heap, GH_OP_DELETE_MIN, 0, hs.seq++, q.off);
      hs.size -= hs.size < (u64)K ? hs.size : (u64)K;
    } else {
      for (u32 c = 0; c < nops; ++c) {
        const u32 nc = (q.n - c * K) < (u32)K ? (q.n - c * K) : (u32)K;
        put_op(slot + c, r, q.heap, GH_OP_INSERT, nc, hs.seq++, q.off + (u64)c * K);
      }
      hs.size += q.n;
    }
  }

  // Request r (q) by its heap's owner thread, in stream order.
  __device__ void process(u32 r, const gh_op& q, Ctl* ctl) const {
    if (q.heap >= nheaps || q.kind > GH_OP_DELETE_MIN) {
      reject(r, q.kind);
      note_error(ctl, ERR_INVAL);
      return;
    }
    SchedHot hs = hot_get(hot + q.heap);
    if (q.kind == GH_OP_DELETE_MIN) {
      admit(r, q, hs, 0);
      // room freed: admit deferred inserts of this heap in order
      while (hs.head != SCHED_NONE) {
        const gh_op d = reqs[hs.head];
        if (hs.size + d.n > hs.cap) break;
        const u32 dr = hs.head;
        hs.head = w.next[dr];
        if (hs.head == SCHED_NONE) w.heaps[q.heap].last = SCHED_NONE;
        admit(dr, d, hs, 2u);
      }
    } else if ((u64)q.n > hs.cap || q.n > 65535u * (u32)K) {
      reject(r, q.kind);
    } else if (hs.head == SCHED_NONE && hs.size + q.n <= hs.cap) {
      admit(r, q, hs, 0);
    } else {
      // wait for memory behind earlier deferred inserts
      w.next[r] = SCHED_NONE;
      const u32 last = hs.head == SCHED_NONE ? SCHED_NONE : w.heaps[q.heap].last;
      if (last == SCHED_NONE) hs.head = r;
      else w.next[last] = r;
      w.heaps[q.heap].last = r;
    }
    hot_put(hot + q.heap, hs);
  }
};

// Which compute unit this wave runs on: the XCD number and the shader
// engine, array and unit fields of the hardware id register.
__device__ __forceinline__ u32 compute_unit_id() {
  const u32 hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);     // HW_ID
  const u32 xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20);   // XCC_ID
  return ((xcc & 0xF) << 8) | ((hw >> 8) & 0xFF);
}

// 16 consecutive u32 from LDS (16-byte aligned) with four 16-byte loads.
__device__ __forceinline__ void load_ids16(const lu32* p, u32 (&ids)[16]) {
  typedef const __attribute__((address_space(3))) u32x4 lu32x4;
  lu32x4* q = reinterpret_cast<lu32x4*>(p);
  const u32x4 a = q[0], b = q[1], c = q[2], d = q[3];
  ids[0] = a.x; ids[1] = a.y; ids[2] = a.z; ids[3] = a.w;
  ids[4] = b.x; ids[5] = b.y; ids[6] = b.z; ids[7] = b.w;
  ids[8] = c.x; ids[9] = c.y; ids[10] = c.z; ids[11] = c.w;
  ids[12] = d.x; ids[13] = d.y; ids[14] = d.z; ids[15] = d.w;
}

template <int K, int T>
__global__ __launch_bounds__(T) void k_serve(const HeapDesc* __restrict__ descs, u32 nheaps,
                                             const gh_op* __restrict__ reqs, u32 nreq,
                                             const u64* __restrict__ in, u64* __restrict__ out,
                                             gh_reqrec* __restrict__ recs, ServeWork w,
                                             Ctl* __restrict__ ctl, u32 clock_mhz) {
  __shared__ __align__(16) u64 lds[5 * K];
  lu64* const L = (lu64*)lds;
  __shared__ OpShared sh;
  const int tid = threadIdx.x;

  if (blockIdx.x == 0) {
    // ---- scheduler ----
    __shared__ SchedShared ss;
    lSchedHot* hot = (lSchedHot*)gh_dyn_lds;
    lu32* cnt = (lu32*)(gh_dyn_lds + (size_t)nheaps * sizeof(SchedHot));
    lu32* cur = cnt + T;
    for (u32 h = tid; h < nheaps; h += T) {
      const u64 rw = ld_relaxed(&descs[h].meta->root);
      SchedHot hs;
      hs.size = rw_m(rw) * (u64)K + rw_s(rw);
      hs.cap = descs[h].max_keys;
      hs.base = descs[h].meta->base;
      hs.seq = 0;
      hs.head = SCHED_NONE;
      hot_put(hot + h, hs);
      w.heaps[h].last = SCHED_NONE;
    }
    if (tid == 0) {
      ss.now = now_ticks();
      ss.qtail = 0;
      ss.overflow = 0;
      // let slots that landed on this compute unit step aside
      __hip_atomic_store(&w.head->sched_cu, compute_unit_id(), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __hip_atomic_store(&w.head->cu_ready, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // a chunk of K requests staged in LDS: records, heap ids, window order
    constexpr u32 CH = K;
    lgh_op* stage = (lgh_op*)lds;
    lu32* hid = (lu32*)(lds + 4 * K);
    lu16* list = (lu16*)(lds + 4 * K + K / 2);
    Scheduler<K> S;
    S.nheaps = nheaps;
    S.reqs = reqs;
    S.recs = recs;
    S.w = w;
    S.hot = hot;
    S.ss = (lSchedShared*)&ss;
    S.t0 = ctl->t0;
    auto due_of = [&](const gh_op& q) -> u64 {
      // arrival, bounded to one minute after the start
      const u64 ns = q.arrival_ns < 60000000000ull ? q.arrival_ns : 60000000000ull;
      return S.t0 + (ns * clock_mhz) / 1000ull;
    };
    __syncthreads();
    for (u32 c0 = 0; c0 < nreq; c0 += CH) {
      const u32 cn = nreq - c0 < CH ? nreq - c0 : CH;
      for (u32 j = tid; j < cn; j += T) {
        const gh_op q = reqs[c0 + j];
        stage_put(stage + j, q);
        hid[j] = q.heap;
      }
      __syncthreads();
      u32 w0 = 0;
      while (w0 < cn) {
        // the window: from w0 up to the first request not due yet (w0 itself
        // is waited for)
        if (tid == 0) {
          const u64 due0 = due_of(stage_get(stage + w0));
          u64 now = now_ticks();
          while (now < due0) {
            if (ld_relaxed32(&ctl->abort)) break;
            __builtin_amdgcn_s_sleep(4);
            now = now_ticks();
          }
          ss.now = now;
          ss.wend = cn;
        }
        __syncthreads();
        for (u32 j = w0 + 1 + tid; j < cn; j += T)
          if (due_of(stage_get(stage + j)) > ss.now) atomicMin(&ss.wend, j);
        __syncthreads();
        const u32 we = ss.wend;
        // stable order of the window's requests by owner thread: counts by
        // LDS atomics, an exclusive scan over the threads, then wave 0 places
        // the requests 64 at a time in stream order, ranking lanes of equal
        // owner with ballots
        cnt[tid] = 0;
        __syncthreads();
        for (u32 j = w0 + tid; j < we; j += T)
          __hip_atomic_fetch_add(cnt + (hid[j] & (T - 1)), 1u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();
        const u32 c = cnt[tid];
        u32 v = c;   // inclusive scan of the counts over the threads
        for (u32 off = 1; off < (u32)T; off <<= 1) {
          __syncthreads();
          cnt[tid] = v;
          __syncthreads();
          if ((u32)tid >= off) v += cnt[tid - off];
        }
        const u32 first = v - c;
        cur[tid] = first;
        __syncthreads();
        if (tid < 64) {
          const u64 below = (1ull << tid) - 1ull;
          for (u32 b0 = w0; b0 < we; b0 += 64) {
            const u32 j = b0 + tid;
            const bool valid = j < we;
            const u32 own = valid ? (hid[j] & (T - 1)) : 0u;
            u64 same = __ballot(valid);
#pragma unroll
            for (u32 bit = 1; bit < (u32)T; bit <<= 1) {
              const u64 m = __ballot((own & bit) != 0);
              same &= (own & bit) ? m : ~m;
            }
            if (valid) {
              const u32 pos = cur[own] + (u32)__popcll(same & below);
              list[pos] = (uint16_t)j;
              if ((same >> tid) >> 1 == 0) cur[own] = pos + 1;   // last of its owner
            }
          }
        }
        __syncthreads();
        // every thread admits its own requests in stream order
        for (u32 x = first; x < first + c; ++x) {
          const u32 j = list[x];
          const gh_op q = stage_get(stage + j);
          S.process(c0 + j, q, ctl);
        }
        // publish the window's queue entries
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) {
          const u32 qt = ss.qtail;
          const u32 tl = (u64)qt < w.max_ops ? qt : (u32)w.max_ops;
          __hip_atomic_store(&w.head->tail, tl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        w0 = we;
      }
      __syncthreads();
    }
    // inserts still waiting for memory when the stream ends are rejected
    for (u32 h = tid; h < nheaps; h += T) {
      u32 r = hot[h].head;
      while (r != SCHED_NONE) {
        S.reject(r, GH_OP_INSERT);
        r = w.next[r];
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (tid == 0) {
      if (ss.overflow) note_error(ctl, ERR_NOMEM);
      __hip_atomic_store(&w.head->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }

  // ---- slots ----
  // The scheduler admits every request; a slot sharing its compute unit
  // would slow it down for every other slot, so up to 8 such slots leave.
  if (tid == 0) {
    sh.ok = 1;
    // (bounded: after ~0.2 s without the scheduler's mark, just go on)
    for (u32 spins = 0; spins < (1u << 20) && !ld_relaxed32(&w.head->cu_ready); ++spins) {
      if (ld_relaxed32(&ctl->abort)) break;
      __builtin_amdgcn_s_sleep(8);
    }
    if (ld_relaxed32(&w.head->cu_ready) && compute_unit_id() == ld_relaxed32(&w.head->sched_cu) &&
        atomicAdd(&w.head->cu_left, 1u) < 8u)
      sh.ok = 0;
  }
  __syncthreads();
  if (!sh.ok) return;
  for (;;) {
    if (tid == 0) {
      u32 i = atomicAdd(&w.head->claim, 1u);
      // wait for queue entry i; an idle slot polls ever more gently (up to
      // ~1 us apart) so that a thousand of them do not crowd the line the
      // scheduler publishes to
      for (u32 spins = 0;; ++spins) {
        const u32 tl = ld_relaxed32(&w.head->tail);
        if (i < tl) break;
        if ((spins & 7) == 7) {
          if (ld_relaxed32(&w.head->done)) {
            if (i >= ld_relaxed32(&w.head->tail)) i = 0xFFFFFFFFu;
            break;
          }
          if (ld_relaxed32(&ctl->abort)) {
            i = 0xFFFFFFFFu;
            break;
          }
        }
        if (spins < 4) __builtin_amdgcn_s_sleep(2);
        else if (spins < 16) __builtin_amdgcn_s_sleep(8);
        else __builtin_amdgcn_s_sleep(32);
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
    if ((u32)q0 == QUEUE_SKIP) {
      __syncthreads();   // every thread has read the entry before sh is reused
      continue;
    }
    gh_op op;
    op.heap = (u32)q0;
    op.kind = (u32)(q0 >> 32);
    op.n = (u32)q1;
    op.seq = (u32)(q1 >> 32);
    op.off = q2;
    op.arrival_ns = 0;
    const HeapDesc H = descs[op.heap];
    const u64 ticket = *gptr(&H.meta->base) + op.seq;
    OpResult res;
    if (op.kind == GH_OP_INSERT) {
      res = op_insert<K, T>(H, ticket, in + op.off, op.n, L, sh, ctl);
    } else {
      res = op_delete<K, T>(H, ticket, out + op.off, L, sh, ctl);
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
                     (size_t)a.nheaps * sizeof(SchedHot) + 2 * T * sizeof(u32), a.stream, a.descs,
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

// ---------------------------------------------------------------------------
// 0/1 knapsack by best-first branch and bound on the heap (the application
// of Sec. 5.6.2).  One heap per instance; a workgroup claims an instance,
// pushes the root node, and repeats: deleteMin(K) the most promising nodes,
// expand those whose bound still exceeds the best value found, insert their
// promising children.  Items are sorted by value/weight descending.
//   bound(level, V, W): V plus the items from `level` on while they fit plus
//   the fitting fraction of the next one, in fixed point with scale 2^16
//   (floored, so never below the true bound);
//   entry = (2^35 - 1 - bound) << 29 | node id  (deleteMin = largest bound);
//   node  = level << 56 | V << 28 | W.
// ---------------------------------------------------------------------------
constexpr u64 KN_KEYMAX = (1ull << 35) - 1;
constexpr u32 KN_IDBITS = 29;
constexpr u64 KN_IDMASK = (1ull << KN_IDBITS) - 1;
constexpr u32 KN_MAXN = 255;

struct KnapShared {
  u32 w[KN_MAXN + 1];
  u32 v[KN_MAXN + 1];
  u64 pw[KN_MAXN + 2];   // prefix sums of the sorted weights and values
  u64 pv[KN_MAXN + 2];
  u64 best;
  u64 cap;
  u64 explored;
  u64 created;
  u64 pool_next;
  u32 n;
  u32 cnt;              // children produced in this round
  u32 popped;
  u32 inst;
  u32 overflow;
};

__device__ __forceinline__ u64 kn_bound(const KnapShared& ks, u32 level, u64 V, u64 W) {
  if (W > ks.cap) return 0;
  const u64 rem = ks.cap - W;
  u32 lo = level, hi = ks.n;   // largest j with pw[j] - pw[level] <= rem
  while (lo < hi) {
    const u32 mid = (lo + hi + 1) >> 1;
    if (ks.pw[mid] - ks.pw[level] <= rem) lo = mid;
    else hi = mid - 1;
  }
  u64 b = (V + ks.pv[lo] - ks.pv[level]) << 16;
  if (lo < ks.n) {
    const u64 r2 = rem - (ks.pw[lo] - ks.pw[level]);
    b += ((r2 * (u64)ks.v[lo]) << 16) / (u64)ks.w[lo];
  }
  return b;
}

template <int K, int T>
__global__ __launch_bounds__(T) void k_knap(const HeapDesc* __restrict__ descs, u32 ninst,
                                            const u32* __restrict__ item_off,
                                            const u32* __restrict__ nitems,
                                            const u64* __restrict__ caps,
                                            const u32* __restrict__ wts,
                                            const u32* __restrict__ vals, u64* __restrict__ pool,
                                            u64 pool_per_inst, u64* __restrict__ scratch,
                                            gh_knapres* __restrict__ res, Ctl* __restrict__ ctl) {
  __shared__ __align__(16) u64 lds[5 * K];
  lu64* const L = (lu64*)lds;
  __shared__ OpShared sh;
  __shared__ KnapShared ks;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      u32 i = atomicAdd(&ctl->next_op, 1u);
      if (ld_relaxed32(&ctl->abort)) i = ninst;
      ks.inst = i;
    }
    __syncthreads();
    const u32 inst = ks.inst;
    if (inst >= ninst) break;
    const HeapDesc H = descs[inst];
    u64 ticket = *gptr(&H.meta->base);
    u64* ipool = pool + (u64)inst * pool_per_inst;
    u64* out = scratch + (u64)inst * 3 * K;   // K popped entries, then 2K children
    u64* kids = out + K;
    // stage the instance
    const u32 n = nitems[inst] < KN_MAXN ? nitems[inst] : KN_MAXN;
    const u32 base = item_off[inst];
    for (u32 j = tid; j < n; j += T) {
      ks.w[j] = wts[base + j];
      ks.v[j] = vals[base + j];
    }
    if (tid == 0) {
      ks.n = n;
      ks.cap = caps[inst];
      ks.explored = 0;
      ks.created = 0;
      ks.overflow = 0;
    }
    __syncthreads();
    if (tid == 0) {
      ks.pw[0] = 0;
      ks.pv[0] = 0;
      for (u32 j = 0; j < n; ++j) {
        ks.pw[j + 1] = ks.pw[j] + ks.w[j];
        ks.pv[j + 1] = ks.pv[j] + ks.v[j];
      }
      // greedy incumbent: items in ratio order while they fit
      u64 W = 0, V = 0;
      for (u32 j = 0; j < n; ++j)
        if (W + ks.w[j] <= ks.cap) {
          W += ks.w[j];
          V += ks.v[j];
        }
      ks.best = V;
      // the root node
      const u64 b = kn_bound(ks, 0, 0, 0);
      ipool[0] = 0;
      kids[0] = ((KN_KEYMAX - b) << KN_IDBITS) | 0ull;
      ks.pool_next = 1;
      ks.cnt = (b > (V << 16)) ? 1u : 0u;
      ks.created = ks.cnt;
    }
    __syncthreads();
    u32 ops = 0;
    for (;;) {
      // push this round's children (at most 2K: two inserts)
      const u32 c = ks.cnt;
      for (u32 j = 0; j < c; j += K) {
        const u32 nn = c - j < (u32)K ? c - j : (u32)K;
        OpResult r = op_insert<K, T>(H, ticket++, kids + j, nn, L, sh, ctl);
        ++ops;
        if (!r.ok) break;
        __syncthreads();
      }
      // take the most promising nodes
      OpResult r = op_delete<K, T>(H, ticket++, out, L, sh, ctl);
      ++ops;
      __syncthreads();
      if (!r.ok || r.count == 0) break;
      if (tid == 0) {
        ks.cnt = 0;
        ks.popped = r.count;
      }
      __syncthreads();
      // expand
      const u32 popped = r.count;
      for (u32 e = tid; e < popped; e += T) {
        const u64 ent = out[e];
        const u64 id = ent & KN_IDMASK;
        const u64 b = KN_KEYMAX - (ent >> KN_IDBITS);
        if (b <= (__hip_atomic_load(&ks.best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) << 16))
          continue;   // cannot beat the incumbent any more
        const u64 node = ipool[id];
        const u32 level = (u32)(node >> 56);
        const u64 V = (node >> 28) & ((1ull << 28) - 1);
        const u64 W = node & ((1ull << 28) - 1);
        atomicAdd(reinterpret_cast<unsigned long long*>(&ks.explored), 1ull);
        if (level >= ks.n) {
          atomicMax(reinterpret_cast<unsigned long long*>(&ks.best), (unsigned long long)V);
          continue;
        }
        const u64 wl = ks.w[level], vl = ks.v[level];
        u64 cand[2];
        u64 cb[2];
        int nc = 0;
        if (W + wl <= ks.cap) {
          const u64 V1 = V + vl, W1 = W + wl;
          atomicMax(reinterpret_cast<unsigned long long*>(&ks.best), (unsigned long long)V1);
          cb[nc] = kn_bound(ks, level + 1, V1, W1);
          cand[nc++] = ((u64)(level + 1) << 56) | (V1 << 28) | W1;
        }
        cb[nc] = kn_bound(ks, level + 1, V, W);
        cand[nc++] = ((u64)(level + 1) << 56) | (V << 28) | W;
        const u64 bestnow =
            __hip_atomic_load(&ks.best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) << 16;
        for (int q = 0; q < nc; ++q) {
          if (cb[q] <= bestnow) continue;
          const u32 slot = atomicAdd(&ks.cnt, 1u);
          const u64 nid = ks.pool_next + slot;
          if (nid >= pool_per_inst || nid > KN_IDMASK) {
            atomicOr(&ks.overflow, 1u);
            continue;
          }
          ipool[nid] = cand[q];
          kids[slot] = ((KN_KEYMAX - cb[q]) << KN_IDBITS) | nid;
        }
      }
      __syncthreads();
      if (tid == 0) {
        u32 c2 = ks.cnt;
        if (ks.overflow) {
          // children beyond the pool were dropped; keep the ones written
          const u64 room = pool_per_inst > ks.pool_next ? pool_per_inst - ks.pool_next : 0;
          if ((u64)c2 > room) c2 = (u32)room;
          ks.cnt = c2;
        }
        ks.pool_next += c2;
        ks.created += c2;
      }
      // pool writes are read back by other threads after later barriers
      __syncthreads();
    }
    if (tid == 0) {
      gh_knapres o;
      o.best = ks.best;
      o.explored = ks.explored;
      o.created = ks.created;
      o.ops = ops;
      o.flags = 1u | (ks.overflow ? 0x40u : 0u);
      res[inst] = o;
    }
    __syncthreads();
  }
}

template <int K, int T>
static hipError_t launch_knap_t(const KnapArgs& a) {
  hipLaunchKernelGGL((k_knap<K, T>), dim3(a.workgroups), dim3(T), 0, a.stream, a.descs, a.ninst,
                     a.item_off, a.n, a.cap, a.w, a.v, a.pool, a.pool_per_inst, a.scratch, a.res,
                     a.ctl);
  return hipGetLastError();
}

template <>
hipError_t launch_knap_k<GH_K>(const KnapArgs& a) {
  constexpr int K = GH_K;
  switch (a.threads) {
#define GH_CASE(TT)                                                \
  case TT:                                                         \
    if constexpr (shape_ok(K, TT)) return launch_knap_t<K, TT>(a); \
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

// ---------------------------------------------------------------------------
// Single-source shortest paths with the heap as a shared priority queue (the
// application of Sec. 5.6.1), lazy deletion: entries are dist << 32 | vertex;
// every workgroup takes the K nearest, skips entries whose vertex was since
// reached by a shorter path, relaxes out-edges with an atomic minimum, and
// inserts one entry per strict improvement.  Tickets are taken dynamically.
// Termination: `outstanding` counts entries pushed and not yet processed.  A
// workgroup adds its pushes before it inserts them (an inserted entry can be
// popped and retired by another workgroup at once) and subtracts the entries
// it popped only after its inserts, so the count bounds the entries in the
// heap plus those held by workgroups; it reaches zero only when both are
// none, and stays zero from then on.
// ---------------------------------------------------------------------------
// Traced runs: record one heap operation.  Thread 0 claims a record and room
// for `count` entries; the workgroup copies the entries.
template <int T>
__device__ void sssp_trace(const gh_sssptrace& tr, SsspState* st, u64 ticket, u32 kind,
                           const u64* src, u32 count, const OpResult& r, const OpShared& sh,
                           u64& s_off) {
  if (threadIdx.x == 0) {
    const u64 i = atomicAdd(reinterpret_cast<unsigned long long*>(&st->trace_ops), 1ull);
    const u64 off = atomicAdd(reinterpret_cast<unsigned long long*>(&st->trace_keys),
                              (unsigned long long)count);
    const bool fits = i < tr.op_cap && off + count <= tr.key_cap;
    if (fits) {
      gh_ssspop rec{};
      rec.ticket = ticket;
      rec.off = off;
      rec.count = count;
      rec.kind = kind;
      // what the operation saw and did: m and s at the root, flags, levels
      rec.reserved = (sh.m & 0xFFFFFFFFull) << 32 | (sh.s & 0xFFFFull) << 16 |
                     (u64)(r.flags & 0xFF) << 8 | (u64)(r.levels & 0xFF);
      tr.d_ops[i] = rec;
    }
    s_off = fits ? off : ~0ull;
  }
  __syncthreads();
  const u64 off = s_off;
  if (off != ~0ull)
    for (u32 j = threadIdx.x; j < count; j += T) tr.d_keys[off + j] = src[j];
  __syncthreads();
}

template <int K, int T>
__global__ __launch_bounds__(T) void k_sssp(const HeapDesc* __restrict__ descs, u32 V,
                                            const u32* __restrict__ rowptr,
                                            const u32* __restrict__ col,
                                            const u32* __restrict__ wt, u32* __restrict__ dist,
                                            u64* __restrict__ push, u64 push_per_wg,
                                            gh_ssspstats* __restrict__ stats,
                                            SsspState* __restrict__ st, gh_sssptrace tr,
                                            Ctl* __restrict__ ctl) {
  __shared__ __align__(16) u64 lds[5 * K];
  lu64* const L = (lu64*)lds;
  __shared__ OpShared sh;
  __shared__ u64 s_ticket, s_toff;
  __shared__ u32 s_exit, s_idle, s_cnt, s_stale;
  const int tid = threadIdx.x;
  const HeapDesc H = descs[0];
  u64* out = push + (u64)blockIdx.x * (push_per_wg + K);   // K popped entries
  u64* mine = out + K;                                      // this workgroup's pushes
  u64 popped = 0, stale = 0, pushed = 0, ops = 0, heap_t = 0, relax_t = 0, rounds = 0;
  u32 idle = 0;
  u64 idle_since = 0;
  for (;;) {
    if (tid == 0) {
      s_exit = (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                ld_relaxed32(&ctl->abort)) ? 1u : 0u;
      // a heap that looks empty (no node, empty partial buffer, as of the
      // last root release) is not worth a ticket: idle without one
      s_idle = 0;
      if (!s_exit) {
        const u64 w = ld_relaxed(&H.meta->root);
        if (rw_m(w) == 0 && rw_s(w) == 0)
          s_idle = 1;
        else
          s_ticket = atomicAdd(reinterpret_cast<unsigned long long*>(&st->next_ticket), 1ull);
      }
    }
    __syncthreads();
    if (s_exit) break;
    OpResult r{0, 0, 0, true};
    if (!s_idle) {
      const u64 t0 = now_ticks();
      r = op_delete<K, T>(H, s_ticket, out, L, sh, ctl);
      ++ops;
      __syncthreads();
      heap_t += now_ticks() - t0;
      if (tr.d_ops && r.ok)
        sssp_trace<T>(tr, st, s_ticket, GH_OP_DELETE_MIN, out, r.count, r, sh, s_toff);
    }
    if (!r.ok) break;
    if (r.count == 0) {
      if (tid == 0) {
        const u64 now = now_ticks();
        if (ld_relaxed(&st->outstanding) == 0) {
          __hip_atomic_store(&st->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (idle != 0 && now - idle_since > ctl->timeout_ticks) {
          // entries outstanding yet the heap stayed empty for the whole
          // watchdog period: give up instead of spinning forever
          raise_error(ctl, ERR_TIMEOUT);
        } else {
          if (idle == 0) idle_since = now;
          // back off (growing to ~7 us) so idle workgroups leave the root to
          // those carrying entries (s_sleep 32 is 2048 clocks, ~0.9 us)
          const u32 n = idle < 3 ? (1u << idle) : 8u;
          for (u32 j = 0; j < n; ++j) __builtin_amdgcn_s_sleep(32);
        }
      }
      ++idle;
      __syncthreads();
      continue;
    }
    idle = 0;
    ++rounds;
    popped += r.count;
    // relax the out-edges of the popped vertices
    u64 t0 = now_ticks();
    if (tid == 0) {
      s_cnt = 0;
      s_stale = 0;
    }
    __syncthreads();
    for (u32 e = tid; e < r.count; e += T) {
      const u64 ent = out[e];
      const u32 d = (u32)(ent >> 32);
      const u32 u = (u32)ent;
      const u32 du = __hip_atomic_load(dist + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (d > du) {
        atomicAdd(&s_stale, 1u);
        continue;
      }
      const u32 j1 = rowptr[u + 1];
      for (u32 j = rowptr[u]; j < j1; ++j) {
        const u32 v = col[j];
        if (v >= V) {   // not a vertex: skip the edge, report the graph
          note_error(ctl, ERR_INVAL);
          continue;
        }
        const u64 nd64 = (u64)d + wt[j];
        if (nd64 >= 0xFFFFFFFFull) continue;
        const u32 nd = (u32)nd64;
        if (nd < __hip_atomic_load(dist + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          const u32 old = atomicMin(dist + v, nd);
          if (old > nd) {
            const u32 slot = atomicAdd(&s_cnt, 1u);
            if (slot < push_per_wg) mine[slot] = ((u64)nd << 32) | v;
          }
        }
      }
    }
    __syncthreads();
    relax_t += now_ticks() - t0;
    const u32 c = s_cnt < push_per_wg ? s_cnt : (u32)push_per_wg;
    if (tid == 0) {
      stale += s_stale;
      if (s_cnt > push_per_wg) raise_error(ctl, ERR_NOMEM);
      // count the pushes before any of them can be popped: once inserted,
      // another workgroup may pop and retire them at once
      if (c) {
        atomicAdd(reinterpret_cast<unsigned long long*>(&st->outstanding), (unsigned long long)c);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      }
    }
    // insert the improvements, K at a time
    t0 = now_ticks();
    bool ok = true;
    for (u32 j = 0; j < c && ok; j += K) {
      if (tid == 0)
        s_ticket = atomicAdd(reinterpret_cast<unsigned long long*>(&st->next_ticket), 1ull);
      __syncthreads();
      const u32 nn = c - j < (u32)K ? c - j : (u32)K;
      const OpResult ri = op_insert<K, T>(H, s_ticket, mine + j, nn, L, sh, ctl);
      ++ops;
      // (the batch in `mine` is unchanged by the insert)
      if (tr.d_ops && ri.ok)
        sssp_trace<T>(tr, st, s_ticket, GH_OP_INSERT, mine + j, nn, ri, sh, s_toff);
      ok = ri.ok && !(ri.flags & F_REJECT);
      if (ri.flags & F_REJECT) {
        // the heap is full: a dropped entry would lose a vertex, stop the run
        if (tid == 0) raise_error(ctl, ERR_NOMEM);
      }
      __syncthreads();
    }
    heap_t += now_ticks() - t0;
    pushed += c;
    if (tid == 0) {
      // the popped entries are retired after their pushes are in the heap
      atomicAdd(reinterpret_cast<unsigned long long*>(&st->outstanding),
                (unsigned long long)(0ull - (u64)r.count));
    }
    if (!ok) break;
  }
  if (tid == 0) {
    atomicAdd(reinterpret_cast<unsigned long long*>(&stats->popped), (unsigned long long)popped);
    atomicAdd(reinterpret_cast<unsigned long long*>(&stats->stale), (unsigned long long)stale);
    atomicAdd(reinterpret_cast<unsigned long long*>(&stats->pushed), (unsigned long long)pushed);
    atomicAdd(reinterpret_cast<unsigned long long*>(&stats->heap_ops), (unsigned long long)ops);
    atomicAdd(reinterpret_cast<unsigned long long*>(&stats->heap_ticks), (unsigned long long)heap_t);
    atomicAdd(reinterpret_cast<unsigned long long*>(&stats->relax_ticks),
              (unsigned long long)relax_t);
    atomicAdd(reinterpret_cast<unsigned long long*>(&stats->rounds), (unsigned long long)rounds);
  }
}

template <int K, int T>
static hipError_t launch_sssp_t(const SsspArgs& a) {
  hipLaunchKernelGGL((k_sssp<K, T>), dim3(a.workgroups), dim3(T), 0, a.stream, a.descs, a.V,
                     a.rowptr, a.col, a.w, a.dist, a.push, a.push_per_wg, a.stats, a.st, a.trace,
                     a.ctl);
  return hipGetLastError();
}

template <>
hipError_t launch_sssp_k<GH_K>(const SsspArgs& a) {
  constexpr int K = GH_K;
  switch (a.threads) {
#define GH_CASE(TT)                                                \
  case TT:                                                         \
    if constexpr (shape_ok(K, TT)) return launch_sssp_t<K, TT>(a); \
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
