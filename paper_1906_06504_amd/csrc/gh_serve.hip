// gh_serve.hip -- the served form (device-resident request loop) and the
// general persistent operation loop (deleteMins of fewer than k entries,
// inserts of more than k entries in one root hold), for one node capacity
// and entry width.  Compiled once per
// supported k and width with -DGH_K=<k> -DGH_ENT_BYTES=<8|16>; each object
// exports gh::launch_serve_k<k, Ent>() and gh::launch_ops_var_k<k, Ent>().
#include "gh_kops.h"

#ifndef GH_K
#error "compile with -DGH_K=<node capacity>"
#endif
#if GH_ENT_BYTES == 8
#define GH_ENT u64
#elif GH_ENT_BYTES == 16
#define GH_ENT e128
#else
#error "compile with -DGH_ENT_BYTES=8 or 16"
#endif

namespace gh {

// ---------------------------------------------------------------------------
// Served form: one persistent launch.  Workgroup 0 is the scheduler: it
// walks the requests in arrival order and admits every request once it is
// due: deleteMins always; an insert when the heap's size after everything
// admitted plus n fits max_keys, otherwise it waits in the heap's FIFO of
// deferred inserts until admitted deleteMins make room.  An admitted
// request's operations (a deleteMin, or an insert cut into operations of K
// entries, or of up to multi_max_batches(K) * K entries that each take the
// root once when the caller asks for that) take the heap's next tickets and
// are appended to a queue.  Every other workgroup is
// a slot that claims queue entries in order and runs them exactly like
// k_ops.
//
// The scheduler works lane-parallel: heap h belongs to scheduler thread
// h mod T.  It takes the requests in windows (the due prefix of a staged
// chunk), sorts each window's requests stably by owner, and every thread
// admits its own requests in stream order; queue slots come from a shared
// counter, so one heap's operations stay in ticket order in the queue.  The
// queue tail is published at the end of each window.  While the queue has
// room (max_ops at least the operations of every admitted request), a heap's
// admissions depend only on its own requests, so its results are the same
// alone and in any mix; once the shared queue overflows, which requests are
// rejected depends on every heap's traffic.
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
    rec.t_resp = rec.t_admit;
    rec.bytes = 0;
    write_rec(r, rec);
  }

  // Admit request r: its operations get the heap's next tickets and queue
  // slots.  A request that no longer fits the operation queue is rejected
  // instead (its heap's tickets and size are left as they were; slots it was
  // handed are marked to be skipped).
  __device__ __forceinline__ void admit(u32 r, const gh_op& q, SchedHot& hs, u32 flags) const {
    const u32 CH = w.ins_max;   // entries per insert operation
    const u32 nops = q.kind == GH_OP_DELETE_MIN ? 1u : (q.n + CH - 1) / CH;
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
    rec.t_resp = rec.t_admit;
    rec.bytes = 0;
    // slots write count, t_resp and t_done of this record: every word goes out
    // coherently and is complete before the queue entries are published
    write_rec(r, rec);
    __hip_atomic_store(w.left + r, nops, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (q.kind == GH_OP_DELETE_MIN) {
      const u32 want = q.n ? q.n : (u32)K;
      put_op(slot, r, q.heap, GH_OP_DELETE_MIN, want, hs.seq++, q.off);
      hs.size -= hs.size < (u64)want ? hs.size : (u64)want;
    } else {
      for (u32 c = 0; c < nops; ++c) {
        const u32 nc = (q.n - c * CH) < CH ? (q.n - c * CH) : CH;
        put_op(slot + c, r, q.heap, GH_OP_INSERT, nc, hs.seq++, q.off + (u64)c * CH);
      }
      hs.size += q.n;
    }
  }

  // Request r (q) by its heap's owner thread, in stream order.
  __device__ __forceinline__ void process(u32 r, const gh_op& q, Ctl* ctl) const {
    if (q.heap >= nheaps || q.kind > GH_OP_DELETE_MIN ||
        (q.kind == GH_OP_DELETE_MIN && q.n > (u32)K)) {
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
    } else if ((u64)q.n > hs.cap || (u64)q.n > 65535ull * w.ins_max) {
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

// Waves per SIMD the served kernel keeps with 256-thread slots and 8-byte
// entries at k <= 256: the register budget of six slots per compute unit
// that it had before the multi-batch insert path joined the slot loop (the
// compiler meets it there without spilling; other shapes are left free).
template <int K, int T, class Ent>
constexpr int serve_waves_per_eu() {
  return (T == 256 && K <= 256 && sizeof(Ent) == 8) ? 6 : 1;
}

template <int K, int T, class Ent>
__global__ __launch_bounds__(T)
__attribute__((amdgpu_waves_per_eu(serve_waves_per_eu<K, T, Ent>()))) void k_serve(const HeapDesc* __restrict__ descs, u32 nheaps,
                                             const gh_op* __restrict__ reqs, u32 nreq,
                                             const Ent* __restrict__ in, Ent* __restrict__ out,
                                             gh_reqrec* __restrict__ recs, ServeWork w,
                                             Ctl* __restrict__ ctl, u32 clock_mhz) {
  __shared__ __align__(16) Ent lds[5 * K];
  lds_t<Ent>* const L = (lds_t<Ent>*)lds;
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
    bool multi = false;
    if (op.kind == GH_OP_INSERT) {
      multi = op.n > (u32)K;
      if (multi)
        res = op_insert_multi<K, T, Ent, true>(descs + op.heap, ticket, in + op.off, op.n, L, sh,
                                               ctl);
      else res = op_insert<K, T, Ent, true>(H, ticket, in + op.off, op.n, L, sh, ctl);
    } else {
      if (__builtin_expect(op.n == (u32)K, 1))
        res = op_delete<K, T, Ent, false, true>(H, ticket, out + op.off, K, L, sh, ctl);
      else
        res = op_delete<K, T, Ent, true, true>(H, ticket, out + op.off, op.n, L, sh, ctl);
    }
    if (tid == 0) {
      if (op.kind == GH_OP_DELETE_MIN)
        __hip_atomic_store(&recs[r].count, res.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // the request is answered when its last operation releases the root
      // (operations of one request release it in ticket order)
      if (res.ok)
        __hip_atomic_fetch_max(&recs[r].t_resp, (u32)(sh.t_rel - ctl->t0), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      const u64 ob = multi ? ((res.flags & F_REJECT) ? 0ull : sh.mbytes)
                           : op_alg_bytes<K, Ent>(op.kind, res, sh.s);
      __hip_atomic_fetch_add(&recs[r].bytes, (u32)ob, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (atomicSub(&w.left[r], 1u) == 1u)
        __hip_atomic_store(&recs[r].t_done, (u32)(now_ticks() - ctl->t0), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

template <int K, int T, class Ent>
static hipError_t launch_serve_t(const ServeArgs& a) {
  hipLaunchKernelGGL((k_serve<K, T, Ent>), dim3(a.workgroups + 1), dim3(T),
                     (size_t)a.nheaps * sizeof(SchedHot) + 2 * T * sizeof(u32), a.stream, a.descs,
                     a.nheaps, a.reqs, a.nreq, reinterpret_cast<const Ent*>(a.in),
                     reinterpret_cast<Ent*>(a.out), a.recs, a.w, a.ctl, a.clock_mhz);
  return hipGetLastError();
}

template <>
hipError_t launch_serve_k<GH_K, GH_ENT>(const ServeArgs& a) {
  constexpr int K = GH_K;
  switch (a.threads) {
#define GH_CASE(TT)                                                         \
  case TT:                                                                  \
    if constexpr (shape_ok(K, TT)) return launch_serve_t<K, TT, GH_ENT>(a); \
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

template <>
hipError_t launch_ops_var_k<GH_K, GH_ENT>(const LaunchArgs& a) {
  return launch_kops_shape<GH_K, FORM_GENERAL, GH_ENT>(a);
}

}  // namespace gh
