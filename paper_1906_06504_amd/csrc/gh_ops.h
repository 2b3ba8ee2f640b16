// gh_ops.h -- one INS or DEL on a generalized heap, run by one workgroup
// (Sec. 4: one thread block per operation), with the TD-INS/TD-DEL locking
// protocol of Sec. 3.3.
//
// Locking summary (Sec. 3.3.1 lock order, Sec. 3.3.2 states):
//  * The root is taken with a ticket lock: an operation with ticket t waits
//    until the heap's root word shows t and releases it by storing t + 1
//    together with the new node count m and partial-buffer size s.  Root
//    order is the linearization order (Theorem 1).  The partial buffer and
//    (m, s) are guarded by the root.
//  * Every other node has a lock word.  Locks are taken parent before child
//    and a child is locked before its parent is released (hand-over-hand).
//  * An insert that needs a new node reserves it at the root as
//    TARGET(ticket).  A deleteMin that must take the last node while it is
//    still an in-flight insert's target marks it MARKED; the insert then
//    leaves its batch in the target slot, sets HANDED and stops, and the
//    deleteMin proceeds with those entries.
//  * A deleteMin that took the last node's batch sets its word to REMOVED.
//  * A deleteMin sifting down treats a child as absent when it does not
//    exist in the deleteMin's own view of the heap size, when it is REMOVED
//    (a later deleteMin moved its entries to the root), or when it is the
//    reserved target of a LATER insert (that insert will pass the parent
//    after this deleteMin).  A target of an EARLIER insert is waited for:
//    that insert is past the parent and only has to store its batch.
//
// The critical section at the root is a chain of dependent memory round
// trips.  Independent loads and lock atomics are issued together: node
// payloads go to registers first, the first attempt at each lock is a single
// compare-and-swap from AVAIL issued next to them, and only a failed attempt
// falls back to a waiting loop.  No lock is ever waited for while a lock
// taken later in the parent-to-child order is held.
#pragma once

#include "gh_device.h"

namespace gh {

// Phase timestamps for profiling the root critical section: compiled in only
// when GH_PHASE_TRACE is defined (the tracing build, never the library
// build).  Thread 0 writes the device clock of slot s of operation i to
// gh_phase_trace[i * GH_TRACE_SLOTS + s] (operations below 2^18); slot 15 is
// the root's release.  Each object has its own array (static); the
// whole-root kernels' copy is read back with heap_phase_trace.
#define GH_TRACE_SLOTS 16
#ifdef GH_PHASE_TRACE
static __device__ uint32_t gh_phase_trace[1 << 22];
#define GH_TRACE(slot)                                                                 \
  do {                                                                                 \
    if (threadIdx.x == 0 && sh.op < (1u << 18))                                        \
      gh_phase_trace[sh.op * GH_TRACE_SLOTS + (slot)] = (uint32_t)wall_clock64();      \
  } while (0)
#else
#define GH_TRACE(slot) \
  do {                 \
  } while (0)
#endif

struct OpShared {
  u64 m, s;            // root metadata read at root acquire
  u64 t_claim;         // clock when the operation was claimed
  u64 t_root;          // clock at root acquire
  u64 t_rel;           // clock at root release (stamped variants only)
  u64 mbytes;          // algorithmic bytes of a multi-batch insert
  u32 flag0, flag1;    // broadcast results from wave 0
  u32 ok;
  u32 op;
  u32 early;           // an insert's next path node was taken by an early try
  u32 marked;          // an insert's look at its target after a level's merge:
                       // MARKED (a field of its own: flag0, the look made with
                       // the node's load, may still be read by a late wave)
  u64 word;            // a root word read by thread 0 for everyone
};

struct OpResult {
  u32 count;
  u32 levels;
  u32 flags;
  bool ok;
};

constexpr u32 F_FULL = 1, F_HANDOFF = 2, F_TOOK = 4, F_ROOT = 8, F_REFILL = 16, F_STOPPED = 0x20,
              F_REJECT = 0x40, F_ABORT = 0x80;

// Algorithmic bytes of one operation: what the method has to move between
// HBM and the workgroup along the path the operation took (e = entry bytes,
// n = entries inserted or returned, s = partial-buffer size at the root,
// L = levels merged):
//   insert kept in the partial buffer:  e (2 (n + s)) + 2 e K if a root exists
//   insert of a full batch over L levels: e (n + s + (n + s - K)) + e (2 K L + K)
//   deleteMin with no node: 2 e s;  root only: 2 e K;
//   deleteMin refilled from the last node, L merged levels: e K (3 + 4 L) + 2 e s.
template <int K, class Ent>
__device__ __forceinline__ u64 op_alg_bytes(u32 kind, const OpResult& r, u64 s) {
  constexpr u64 e = sizeof(Ent);
  if (r.flags & F_REJECT) return 0;
  if (kind == 0) {   // insert
    const u64 n = r.count;
    if (r.flags & F_FULL) return e * (n + s + (n + s - K)) + e * (2ull * K * r.levels + K);
    return e * 2 * (n + s) + ((r.flags & F_ROOT) ? 2 * e * K : 0);
  }
  if (!(r.flags & F_ROOT)) return 2 * e * s;
  if (r.flags & F_REFILL) return e * K * (3 + 4ull * r.levels) + 2 * e * s;
  return 2 * e * K;
}

// --- lock primitives --------------------------------------------------------

// Thread 0: wait until the root word shows our ticket; returns the word.
__device__ __forceinline__ bool root_acquire(HeapMeta* meta, u64 ticket, Ctl* ctl, u64& word) {
  const u64 mine = ticket & RW_TICKET_MASK;
  Waiter w;
  for (;;) {
    const u64 v = ld_relaxed(&meta->root);
    if (rw_ticket(v) == mine) {
      word = v;
      break;
    }
    const u64 ahead = (mine - rw_ticket(v)) & RW_TICKET_MASK;  // operations in front of us
    if (!w.step(ctl, ahead > 8 ? 16 : (ahead > 2 ? 4 : 1))) return false;
  }
  fence_acquire();
  return true;
}

// Thread 0: hand the root to the next ticket, publishing the new (m, s).
// Node and partial-buffer stores were made visible by publish() before.
__device__ __forceinline__ void release_root(HeapMeta* meta, u64 ticket, u64 m, u64 s) {
  st_relaxed(&meta->root, rootword(ticket + 1, m, s));
}

// The same, and with Stamp the release clock goes to sh.t_rel: an insert is
// then linearized (its entries are seen by every later operation) and a
// deleteMin's entries are in its output buffer (stamped variants wait for
// their stores before every release).
template <bool Stamp>
__device__ __forceinline__ void release_root_at(HeapMeta* meta, u64 ticket, u64 m, u64 s,
                                                OpShared& sh) {
  GH_TRACE(15);
  release_root(meta, ticket, m, s);
  if constexpr (Stamp) sh.t_rel = now_ticks();
}

// How a lane wants to take a lock word.
enum LockMode : u32 {
  LM_PATH = 0,    // insert path node: AVAIL -> INUSE
  LM_CHILD = 2,   // deleteMin child: AVAIL -> INUSE, or absent (see above)
  LM_PEEK = 3,    // read only: reports MARKED as 1, anything else as 0
};

// Classify an observed lock word for a deleteMin child: 1 = free (try the
// swap), 0 = absent, -1 = wait.
__device__ __forceinline__ int child_view(u64 v, u64 ticket) {
  const u64 st = lw_state(v);
  if (st == ST_AVAIL) return 1;
  if (st == ST_REMOVED) return 0;
  if (st != ST_INUSE && lw_ticket(v) > ticket) return 0;  // a later insert's target
  return -1;
}

// One attempt: 1 = taken (or MARKED seen for LM_PEEK), 0 = absent / not
// marked, -1 = try again later.
__device__ __forceinline__ int try_lock(u64* lw, u32 mode, u64 ticket) {
  const u64 v = ld_relaxed(lw);
  const u64 st = lw_state(v);
  if (mode == LM_PEEK) return st == ST_MARKED ? 1 : 0;
  if (st == ST_AVAIL) return cas_relaxed(lw, v, lockword(ST_INUSE, ticket)) ? 1 : -1;
  if (mode == LM_CHILD) return child_view(v, ticket) == 0 ? 0 : -1;
  return -1;
}

// Executed by every lane of wave 0: each lane with `active` takes its own
// word; the wave leaves when every active lane has an answer.  Returns false
// (in every lane) when the wait is abandoned.  Ends with an acquire.
__device__ __forceinline__ bool lock_lanes(u64* lw, u32 mode, u64 ticket, bool active, int& result,
                                           Ctl* ctl) {
  int r = active ? -1 : 0;
  Waiter w;
  for (;;) {
    if (r < 0) r = try_lock(lw, mode, ticket);
    if (__all(r >= 0)) break;
    if (!w.step(ctl)) return false;
  }
  fence_acquire();
  result = r;
  return true;
}

// deleteMin taking the last node while holding the root (thread 0), after a
// failed first swap that saw `v`: 1 = plain lock, 2 = took an in-flight
// insert's batch (MARKED -> HANDED), -1 = abandoned.
__device__ __forceinline__ int take_last(u64* lw, u64 v, u64 ticket, Ctl* ctl) {
  Waiter w;
  for (;;) {
    const u64 st = lw_state(v);
    if (st == ST_AVAIL) {
      if (cas_relaxed(lw, v, lockword(ST_INUSE, ticket))) return 1;
    } else if (st == ST_TARGET) {
      const u64 owner = lw_ticket(v);
      if (cas_relaxed(lw, v, lockword(ST_MARKED, owner))) {
        Waiter w2;
        for (;;) {
          const u64 x = ld_relaxed(lw);
          if (x == lockword(ST_HANDED, owner)) break;
          if (!w2.step(ctl)) return -1;
        }
        return 2;
      }
    } else if (!w.step(ctl)) {
      return -1;
    }
    v = ld_relaxed(lw);
  }
}

// Thread 0, after publish() (or when the holder stored nothing).
__device__ __forceinline__ void unlock(u64* lw) { st_relaxed(lw, lockword(ST_AVAIL, 0)); }

// An operation that may not change the heap (an insert of 0 entries, or a
// malformed record) still passes the root in its turn, so the tickets after
// it keep flowing.
__device__ __forceinline__ OpResult op_pass_root(const HeapDesc& H, u64 ticket, OpShared& sh,
                                                 Ctl* ctl) {
  OpResult res{0, 0, 0, true};
  if (threadIdx.x == 0) {
    u64 w = 0;
    sh.ok = root_acquire(H.meta, ticket, ctl, w) ? 1u : 0u;
    sh.t_root = now_ticks();
    sh.s = rw_s(w);
    if (sh.ok) release_root(H.meta, ticket, rw_m(w), rw_s(w));
  }
  __syncthreads();
  res.ok = sh.ok != 0;
  return res;
}

// Take the root in turn and leave the heap empty (m = s = 0): every entry is
// discarded.  Only for a heap with no other operation in flight (all node
// locks AVAIL), such as a branch-and-bound instance's own heap once nothing
// left in it can matter.
__device__ __forceinline__ OpResult op_discard(const HeapDesc& H, u64 ticket, OpShared& sh,
                                               Ctl* ctl) {
  OpResult res{0, 0, 0, true};
  if (threadIdx.x == 0) {
    u64 w = 0;
    sh.ok = root_acquire(H.meta, ticket, ctl, w) ? 1u : 0u;
    if (sh.ok) release_root(H.meta, ticket, 0, 0);
  }
  __syncthreads();
  res.ok = sh.ok != 0;
  return res;
}

// Take the root in turn and lay n ascending entries from src (global
// memory) out as the heap: the first floor(n / K) * K become the nodes in
// addition order, the rest the partial buffer (the bulk build of Sec. 3.1),
// and the lock words of the node positions are cleared.  Only for an empty
// heap with no other operation in flight, such as a branch-and-bound
// instance's own heap after op_discard.
template <int K, int T, class Ent>
__device__ __forceinline__ OpResult op_build_from(const HeapDesc& H, u64 ticket,
                                                  const Ent* __restrict__ src, u64 n,
                                                  OpShared& sh, Ctl* ctl) {
  OpResult res{0, 0, 0, true};
  if (threadIdx.x == 0) {
    u64 w = 0;
    sh.ok = root_acquire(H.meta, ticket, ctl, w) ? 1u : 0u;
  }
  __syncthreads();
  if (!sh.ok) {
    res.ok = false;
    return res;
  }
  const u64 m = n / K, body = m * K;
  const glob_t<Ent>* gs = gptr(src);
  Ent* nodes = slot_ptr<K, Ent>(H, 1);
  const HeapRegion R(reinterpret_cast<const u64*>(nodes), (u32)(body * sizeof(Ent)));
  const HeapRegion P(reinterpret_cast<const u64*>(pb_ptr<Ent>(H)), K * sizeof(Ent));
  for (u64 i = threadIdx.x; i < n; i += T) {
    const Ent e = gs[i];
    if (i < body) R.store_ent((u32)(i * sizeof(Ent)), e);
    else P.store_ent((u32)((i - body) * sizeof(Ent)), e);
  }
  for (u64 p = threadIdx.x + 1; p <= m; p += T) st_relaxed(H.locks + p, lockword(ST_AVAIL, 0));
  publish();
  if (threadIdx.x == 0) release_root(H.meta, ticket, m, n - body);
  res.count = (u32)n;
  return res;
}

// Thread 0 takes the root; everyone learns (m, s) from the root word.
__device__ __forceinline__ bool acquire_root(const HeapDesc& H, u64 ticket, OpShared& sh,
                                             Ctl* ctl) {
  if (threadIdx.x == 0) {
    u64 w = 0;
    sh.ok = root_acquire(H.meta, ticket, ctl, w) ? 1u : 0u;
    sh.t_root = now_ticks();
    sh.m = rw_m(w);
    sh.s = rw_s(w);
  }
  __syncthreads();
  GH_TRACE(0);
  return sh.ok != 0;
}

// ---------------------------------------------------------------------------
// The part of a top-down insert below the root (Sec. 3.2.2, 3.3.2): the carry
// F goes from node `cur` on level 1 down the path to the target t (level L
// >= 2), merging with every path node (MergeAndSort with the shortcuts of
// Sec. 4.3), hand over hand.  On entry `cur` is locked by this operation and
// t is reserved as TARGET(ticket); with LoadF the carry is read from the
// target slot in the first round trip (where the root's owner left it),
// otherwise it is in F.  N and spare are free LDS buffers.
// ---------------------------------------------------------------------------
template <int K, int T, class Ent>
__device__ __forceinline__ OpResult ins_fill_target(const HeapDesc& H, u64 ticket, u32 t, int L,
                                                    lds_t<Ent>* F, OpShared& sh, OpResult res) {
  const int tid = threadIdx.x;
  u64* tlock = lock_ptr(H, t);
  store_node<K, T, Ent>(node_ptr<K, Ent>(H, t), F);
  publish();
  if (tid == 0) {
    if (!cas_relaxed(tlock, lockword(ST_TARGET, ticket), lockword(ST_AVAIL, 0))) {
      // MARKED by a deleteMin: the batch is already in the target slot
      st_relaxed(tlock, lockword(ST_HANDED, ticket));
      sh.flag1 = 1;
    } else {
      sh.flag1 = 0;
    }
  }
  __syncthreads();
  if (sh.flag1) res.flags |= F_HANDOFF;
  res.levels = L;
  return res;
}

template <int K, int T, class Ent, bool LoadF>
__device__ __forceinline__ OpResult ins_descend(const HeapDesc& H, u64 ticket, u32 t, int L,
                                                u32 cur, lds_t<Ent>* F, lds_t<Ent>* N,
                                                lds_t<Ent>* spare, OpShared& sh, Ctl* ctl,
                                                OpResult res) {
  constexpr int E = (2 * K) / T >= 1 ? (2 * K) / T : 1;
  const int tid = threadIdx.x;
  u64* tlock = lock_ptr(H, t);
  int level = 1;
  for (;;) {
    {
      // the path node, in the same round trip a look at the target (a
      // deleteMin that claimed it gets the carry now, before this level's
      // merge: the carry has not entered this subtree yet) and a first try
      // at the lock of the node after it (cur is held: parent before child)
      const u32 nxt = t >> (L - level - 1);
      NodeRegs<K, T, Ent> nr, fr;
      nr.load(node_ptr<K, Ent>(H, cur));
      if (LoadF && level == 1) fr.load(node_ptr<K, Ent>(H, t));
      u64 tw = 0, eo = 1;
      if (tid == 0) tw = ld_relaxed(tlock);
      if (tid == 1 && nxt != t) eo = cas_old(lock_ptr(H, nxt), 0, lockword(ST_INUSE, ticket));
      nr.store(N);
      if (LoadF && level == 1) fr.store(F);
      if (tid == 0) sh.flag0 = lw_state(tw) == ST_MARKED ? 1u : 0u;
      if (tid == 1) sh.early = eo == 0 ? 1u : 0u;
    }
    __syncthreads();
    if (sh.flag0) {
      store_node<K, T, Ent>(node_ptr<K, Ent>(H, t), F);
      publish();
      if (tid == 0) {
        if (sh.early) unlock(lock_ptr(H, t >> (L - level - 1)));
        unlock(lock_ptr(H, cur));
        st_relaxed(tlock, lockword(ST_HANDED, ticket));
      }
      res.levels = level;
      res.flags |= F_HANDOFF;
      return res;
    }
    // (node, F) = MergeAndSort(node, F) with the shortcuts of Sec. 4.3
    Ent* cur_ptr = node_ptr<K, Ent>(H, cur);
    if (ent_le(N[K - 1], F[0])) {
      // node already holds the smallest: nothing moves
    } else if (ent_le(F[K - 1], N[0])) {
      store_node<K, T, Ent>(cur_ptr, F);  // swap
      lds_t<Ent>* x = F; F = N; N = x;
    } else {
      merge_split<E, T>(N, K, F, K, K, HeapSink<Ent>(cur_ptr, K * sizeof(Ent)), sink(spare));
      lds_t<Ent>* x = F; F = spare; spare = x;
    }
    ++level;
    const u32 child = t >> (L - level);
    // lane 0 looks whether a deleteMin claimed our target, lane 1 locks the
    // next path node (child before parent release)
    if (tid < 64) {
      const bool next_is_path = child != t;
      u64* w = (tid == 0) ? tlock : lock_ptr(H, child);
      const u32 mode = (tid == 0) ? (u32)LM_PEEK : (u32)LM_PATH;
      // the next path node was tried when this node was loaded
      const bool active = tid == 0 || (tid == 1 && next_is_path && !sh.early);
      int r = 0;
      const bool ok = lock_lanes(w, mode, ticket, active, r, ctl);
      const bool allok = __all(ok);
      if (tid == 0) {
        sh.marked = r == 1 ? 1u : 0u;   // MARKED seen
        sh.ok = allok ? 1u : 0u;
      }
    }
    __syncthreads();
    if (!sh.ok) { res.ok = false; return res; }
    if (sh.marked) {
      // cooperation: leave the batch in the target slot for the deleteMin
      store_node<K, T, Ent>(node_ptr<K, Ent>(H, t), F);
      publish();
      if (tid == 0) {
        if (child != t) unlock(lock_ptr(H, child));
        unlock(lock_ptr(H, cur));
        st_relaxed(tlock, lockword(ST_HANDED, ticket));
      }
      res.levels = level;
      res.flags |= F_HANDOFF;
      return res;
    }
    publish();
    if (tid == 0) unlock(lock_ptr(H, cur));
    if (child == t) break;
    cur = child;
  }
  return ins_fill_target<K, T, Ent>(H, ticket, t, L, F, sh, res);
}

// ---------------------------------------------------------------------------
// INS (Sec. 3.2.2 top-down insert, Sec. 3.3.2 partial batches and
// cooperation).  `keys` holds n (1..K) entries in global memory.
// LDS: five buffers of K entries.
// ---------------------------------------------------------------------------
template <int K, int T, class Ent, bool Stamp = false>
__device__ __forceinline__ OpResult op_insert(const HeapDesc& H, u64 ticket,
                                              const Ent* __restrict__ keys, u32 n,
                                              lds_t<Ent>* lds, OpShared& sh, Ctl* ctl) {
  constexpr int E = (2 * K) / T >= 1 ? (2 * K) / T : 1;
  // entries a thread takes in the root phase's merge of input, root and pb
  // (up to 3K): one pass where that needs at most max(E, 8) a thread
  constexpr int E3a = pow2_at_least((3 * K + T - 1) / T);
  constexpr int E3 = E3a < (E > 8 ? E : 8) ? E3a : (E > 8 ? E : 8);
  const int tid = threadIdx.x;
  OpResult res{n, 0, 0, true};
  lds_t<Ent>* b0 = lds;
  lds_t<Ent>* b1 = lds + K;
  lds_t<Ent>* F = lds + 2 * K;   // the carry
  lds_t<Ent>* N = lds + 3 * K;   // node being merged (root first)
  lds_t<Ent>* P = lds + 4 * K;   // partial buffer, right after the root: by Property 3
                                 // root followed by pb is one sorted run
  HeapMeta* meta = H.meta;

  // sort the batch before touching the heap (holds no lock)
  load_n<T>(b0, keys, n);
  lds_t<Ent>* xs = block_sort<K, T, Ent>(b0, b1, (int)n);
  lds_t<Ent>* xfree = (xs == b0) ? b1 : b0;

  if (!acquire_root(H, ticket, sh, ctl)) { res.ok = false; return res; }
  const u64 m = sh.m;
  const u32 s = (u32)sh.s;
  if (m >= 1) res.flags |= F_ROOT;
  const bool full = n + s >= (u32)K;
  if (full && m + 1 > H.max_nodes) {
    // no room for another node: reject the insert, leave the heap unchanged
    if (tid == 0) {
      note_error(ctl, ERR_NOMEM);
      release_root_at<Stamp>(meta, ticket, m, s, sh);
    }
    res.count = 0;
    res.flags |= F_REJECT;
    return res;
  }
  const u64 m2 = m + 1;
  const u32 t = full ? bitrev_pos((u32)m2) : 0u;  // target node index
  const int L = full ? level_of(t) : 0;
  const u32 child1 = L >= 2 ? (t >> (L - 1)) : 0u;
  u64* tlock = H.locks + m2;

  // One round trip: partial buffer and root into registers, the target
  // reserved, and a first try at the root's child on the insert path.  The
  // target slot can only be AVAIL (never used) or REMOVED here: any in-flight
  // insert's target lies at or below position m, and only the root holder
  // reserves new ones.
  {
    NodeRegs<K, T, Ent> pr, rr;
    pr.load(pb_ptr<Ent>(H));
    if (m >= 1) rr.load(slot_ptr<K, Ent>(H, 1));
    u64 old = 0;
    if (tid == 0 && L >= 1) old = xchg_relaxed(tlock, lockword(ST_TARGET, ticket));
    if (tid == 1 && L >= 2) old = cas_old(lock_ptr(H, child1), 0, lockword(ST_INUSE, ticket));
    pr.store(P);
    if (m >= 1) rr.store(N);
    if (tid < 64) {
      const bool bad = tid == 0 && L >= 1 && lw_state(old) != ST_AVAIL &&
                       lw_state(old) != ST_REMOVED;
      // a busy first child is waited for after the root phase's merges,
      // before the root is released (its payload is loaded only then)
      const bool need = tid == 1 && L >= 2 && old != 0;
      if (tid == 1) sh.flag1 = need ? 1u : 0u;
      const bool anybad = __any(bad);
      if (tid == 0) {
        if (anybad) raise_error(ctl, ERR_STATE);
        sh.ok = anybad ? 0u : 1u;
      }
    }
  }
  __syncthreads();
  GH_TRACE(1);
  if (!sh.ok) { res.ok = false; return res; }

  // The root phase in one merge.  Property 3 makes root followed by pb one
  // sorted run, so S = merge(sorted input, root ++ pb) gives the top-down
  // insert's results directly: the new root is S[0, K); for a partial batch
  // the new pb is the rest; for a full batch the carry (the root-level
  // MergeAndSort's hi half) is S[K, 2K) and the new pb S[2K, ...), the n + s
  // - K largest of input and pb (an input entry below a root entry cannot be
  // among them, since n <= K).  When the input is no smaller than the root
  // the root stays as it is and only input and pb merge.
  const u32 tot = n + s;
  Ent* root = slot_ptr<K, Ent>(H, 1);  // position 1
  const HeapSink<Ent> pbsink(pb_ptr<Ent>(H), K * sizeof(Ent));
  const bool root_moves = m >= 1 && !ent_le((Ent)N[K - 1], (Ent)xs[0]);
  if (!full) {
    // the partial buffer keeps everything, Property 3 against the root
    if (root_moves)
      merge_split<E3, T>(xs, (int)n, N, K + (int)s, K, HeapSink<Ent>(root, K * sizeof(Ent)),
                         pbsink);
    else
      merge_split<E, T>(xs, (int)n, P, (int)s, (int)tot, pbsink, pbsink);
    GH_TRACE(2);
    publish();
    if (tid == 0) release_root_at<Stamp>(meta, ticket, m, tot, sh);
    return res;
  }

  // a full batch: the carry goes down from the root; the rest stays in the pb
  res.flags |= F_FULL;
  const u32 rest = tot - K;
  if (root_moves)
    merge_split3<E3, T>(xs, (int)n, N, K + (int)s, K, 2 * K,
                        HeapSink<Ent>(root, K * sizeof(Ent)), sink(F), pbsink);
  else
    merge_split<E, T>(xs, (int)n, P, (int)s, K, sink(F), pbsink);
  __syncthreads();
  GH_TRACE(2);
  if (L == 0) {
    store_node<K, T, Ent>(root, F);
    publish();
    if (tid == 0) release_root_at<Stamp>(meta, ticket, m2, rest, sh);
    return res;
  }

  // The root's MergeAndSort was part of the merge above.  Take the first
  // path node now if its first try failed (parent before child: the root is
  // still held), then release the root.
  if (L >= 2 && sh.flag1) {
    if (tid < 64) {
      int r = 0;
      const bool ok = lock_lanes(lock_ptr(H, child1), LM_PATH, ticket, tid == 1, r, ctl);
      const bool allok = __all(ok);
      if (tid == 0) sh.ok = allok ? 1u : 0u;
    }
    __syncthreads();
    if (!sh.ok) { res.ok = false; return res; }
  }
  GH_TRACE(3);
  publish();
  GH_TRACE(4);
  if (tid == 0) release_root_at<Stamp>(meta, ticket, m2, rest, sh);
  if (L == 1) return ins_fill_target<K, T, Ent>(H, ticket, t, L, F, sh, res);
  return ins_descend<K, T, Ent, false>(H, ticket, t, L, child1, F, N, xfree, sh, ctl, res);
}

// ---------------------------------------------------------------------------
// The sift-down of a deleteMin (Sec. 3.2.1, 3.3.2) from node c, which this
// operation holds with cur's batch in bufs[0] (c = 1: the root, released at
// the end of its level).  `loaded`: c's children are locked as hl / hr say
// and loaded into bufs[1] / bufs[2].  Otherwise, with `early`, lanes 0 and 1
// hold the result of a first try at c's children's locks in eoc.  While a
// level merges, lanes 0 and 1 make a first try at the locks of the next
// node's children (the next node is held), kept in eoc.
// ---------------------------------------------------------------------------
template <int K, int T, class Ent, bool Stamp = false>
__device__ __forceinline__ OpResult del_sift(const HeapDesc& H, u64 ticket, u32 c, bool loaded,
                                             bool hl, bool hr, bool early, u64 eoc,
                                             lds_t<Ent>* (&bufs)[4], u64 m2, u64 s2,
                                             OpShared& sh, Ctl* ctl, OpResult res) {
  constexpr int E = (2 * K) / T >= 1 ? (2 * K) / T : 1;
  const int tid = threadIdx.x;
  HeapMeta* meta = H.meta;
  lds_t<Ent>* C = bufs[0];
  for (;;) {
    const u64 l = 2ull * c, r = l + 1;
    lds_t<Ent>* Lb = bufs[1];
    lds_t<Ent>* Rb = bufs[2];
    if (!loaded) {
      const bool el = node_exists(l, m2), er = node_exists(r, m2);
      if (tid < 64) {
        const bool mine = (tid == 0 && el) || (tid == 1 && er);
        int got = 0;
        bool need = false;
        if (mine) {
          if (!early) need = true;
          else if (eoc == 0) got = 1;
          else if (child_view(eoc, ticket) == 0) got = 0;
          else need = true;
        }
        u64* w = need ? lock_ptr(H, (u32)(tid == 0 ? l : r)) : nullptr;
        bool ok = true;
        if (__any(need)) {
          int r2 = 0;
          ok = lock_lanes(w, LM_CHILD, ticket, need, r2, ctl);
          if (need) got = r2;
        }
        const bool allok = __all(ok);
        if (tid == 0) {
          sh.flag0 = got > 0 ? 1u : 0u;
          sh.ok = allok ? 1u : 0u;
        }
        if (tid == 1) sh.flag1 = got > 0 ? 1u : 0u;
      }
      __syncthreads();
      if (!sh.ok) { res.ok = false; return res; }
      hl = sh.flag0;
      hr = sh.flag1;
      {
        NodeRegs<K, T, Ent> lc, rc;
        if (hl) lc.load(node_ptr<K, Ent>(H, (u32)l));
        if (hr) rc.load(node_ptr<K, Ent>(H, (u32)r));
        if (hl) lc.store(Lb);
        if (hr) rc.store(Rb);
      }
      __syncthreads();
    }
    loaded = false;
    const Ent lmin = hl ? (Ent)Lb[0] : ent_max<Ent>();
    const Ent rmin = hr ? (Ent)Rb[0] : ent_max<Ent>();
    const Ent cmin = ent_lt(lmin, rmin) ? lmin : rmin;
    Ent* cptr = node_ptr<K, Ent>(H, c);

    if (ent_le(C[K - 1], cmin)) {
      // the property holds: place cur and stop (early stop, Sec. 4.3)
      store_node<K, T, Ent>(cptr, C);
      publish();
      if (tid == 0) {
        if (hl) unlock(lock_ptr(H, (u32)l));
        if (hr) unlock(lock_ptr(H, (u32)r));
        if (c == 1) release_root_at<Stamp>(meta, ticket, m2, s2, sh);
        else unlock(lock_ptr(H, c));
      }
      return res;
    }

    u32 next;
    lds_t<Ent>* newcur;
    if (hl && hr) {
      // (hi, lo) = MergeAndSort(l, r); lo stays in the child whose max was
      // larger (on a tie the right child counts as larger), hi merges with
      // cur; cur's k smallest stay here
      const bool big_is_l = ent_lt(Rb[K - 1], Lb[K - 1]);
      const u32 big = big_is_l ? (u32)l : (u32)r;
      const u32 small = big_is_l ? (u32)r : (u32)l;
      early = true;
      if (tid < 2) {
        const u64 g = 2ull * small + tid;
        eoc = node_exists(g, m2) ? cas_old(lock_ptr(H, (u32)g), 0, lockword(ST_INUSE, ticket))
                                 : ~0ull;
      }
      lds_t<Ent>* Bg = big_is_l ? Lb : Rb;
      lds_t<Ent>* Sm = big_is_l ? Rb : Lb;
      lds_t<Ent>* hi;
      lds_t<Ent>* freeb;
      if (ent_le(Sm[K - 1], Bg[0])) {
        hi = Sm;             // lo is the big child's batch, already in place
        freeb = bufs[3];
      } else {
        merge_split<E, T>(Lb, K, Rb, K, K, sink(bufs[3]), HeapSink<Ent>(node_ptr<K, Ent>(H, big), K * sizeof(Ent)));
        __syncthreads();
        hi = bufs[3];
        freeb = Lb;
      }
      if (ent_le(hi[K - 1], C[0])) {
        store_node<K, T, Ent>(cptr, hi);
        newcur = C;
      } else {
        merge_split<E, T>(C, K, hi, K, K, HeapSink<Ent>(cptr, K * sizeof(Ent)), sink(freeb));
        __syncthreads();
        newcur = freeb;
      }
      if (c == 1) GH_TRACE(6);
      publish();
      if (c == 1) GH_TRACE(7);
      if (tid == 0) {
        unlock(lock_ptr(H, big));
        if (c == 1) release_root_at<Stamp>(meta, ticket, m2, s2, sh);
        else unlock(lock_ptr(H, c));
      }
      next = small;
    } else {
      // one live child x
      const u32 x = hl ? (u32)l : (u32)r;
      lds_t<Ent>* X = hl ? Lb : Rb;
      early = true;
      if (tid < 2) {
        const u64 g = 2ull * x + tid;
        eoc = node_exists(g, m2) ? cas_old(lock_ptr(H, (u32)g), 0, lockword(ST_INUSE, ticket))
                                 : ~0ull;
      }
      lds_t<Ent>* freeb = bufs[3];
      if (ent_le(X[K - 1], C[0])) {
        store_node<K, T, Ent>(cptr, X);
        newcur = C;
      } else {
        merge_split<E, T>(C, K, X, K, K, HeapSink<Ent>(cptr, K * sizeof(Ent)), sink(freeb));
        __syncthreads();
        newcur = freeb;
      }
      publish();
      if (tid == 0) {
        if (c == 1) release_root_at<Stamp>(meta, ticket, m2, s2, sh);
        else unlock(lock_ptr(H, c));
      }
      next = x;
    }
    ++res.levels;
    // rotate buffers: newcur becomes C, the other three are free (in
    // their old order; newcur is one of the four)
    {
      lds_t<Ent>* const a0 = bufs[0];
      lds_t<Ent>* const a1 = bufs[1];
      lds_t<Ent>* const a2 = bufs[2];
      lds_t<Ent>* const a3 = bufs[3];
      const bool n0 = newcur == a0, n1 = newcur == a1, n2 = newcur == a2;
      bufs[0] = newcur;
      bufs[1] = n0 ? a1 : a0;
      bufs[2] = (n0 || n1) ? a2 : a1;
      bufs[3] = (n0 || n1 || n2) ? a3 : a2;
      C = bufs[0];
    }
    c = next;
  }
}

// ---------------------------------------------------------------------------
// DEL (Sec. 3.2.1 with the partial-buffer rules of Sec. 3.3.2/3.3.4) of
// `want` entries, 1 <= want <= K: writes min(want, size) entries to out.
// want < K (variable count): the root's other K - want entries and the
// partial buffer, merged, refill the top; only when they are fewer than K is
// the last node taken as well (its K entries and the merged rest give the new
// root and the partial buffer).  With a single node and fewer than K left,
// everything left becomes the partial buffer.  Var = false compiles the
// whole-root deleteMin only (want is K); callers pick Var = true for want < K.
// ---------------------------------------------------------------------------
template <int K, int T, class Ent, bool Var = false, bool Stamp = false>
__device__ __forceinline__ OpResult op_delete(const HeapDesc& H, u64 ticket,
                                              Ent* __restrict__ out, u32 want_n,
                                              lds_t<Ent>* lds, OpShared& sh, Ctl* ctl) {
  constexpr int E = (2 * K) / T >= 1 ? (2 * K) / T : 1;
  const u32 want = Var ? want_n : (u32)K;
  const int tid = threadIdx.x;
  OpResult res{0, 0, 0, true};
  HeapMeta* meta = H.meta;
  lds_t<Ent>* bufs[4] = {lds, lds + K, lds + 2 * K, lds + 3 * K};
  lds_t<Ent>* P = lds + 4 * K;

  if (!acquire_root(H, ticket, sh, ctl)) { res.ok = false; return res; }
  const u64 m = sh.m;
  const u32 s = (u32)sh.s;
  if (m >= 1) res.flags |= F_ROOT;

  if (m == 0) {
    // no node: the partial buffer is the whole heap
    const u32 cnt = Var && want < s ? want : s;   // the pb holds < K entries
    copy_heap_n<K, T, Ent>(out, pb_ptr<Ent>(H), cnt);
    if (cnt < s) {
      // what is left of the partial buffer moves to its front
      load_heap_n<K, T, Ent>(P, pb_ptr<Ent>(H), s - cnt, cnt);
      __syncthreads();   // every read of the pb is done before it is rewritten
      store_heap_n<K, T, Ent>(pb_ptr<Ent>(H), P, s - cnt);
      publish();
    } else if constexpr (Stamp) {
      publish();         // the output is in memory before the stamp
    } else {
      __syncthreads();   // every read of the pb is done before the root moves on
    }
    if (tid == 0) release_root_at<Stamp>(meta, ticket, 0, s - cnt, sh);
    res.count = cnt;
    return res;
  }
  res.count = want;
  const bool part = Var && want < (u32)K;
  const u32 nrest = K - want + s;   // what stays at the top (want = K: the pb)
  // the last node refills the root (a whole-root deleteMin: whenever there
  // are two or more nodes, and m == 1 returns before that matters)
  const bool refill = Var ? (m >= 2 && nrest < (u32)K) : true;
  // node count and pb size after the operation
  const u64 m2 = refill ? m - 1 : (nrest >= (u32)K ? m : 0);
  const u32 s2 = !part ? s : (nrest >= (u32)K ? nrest - K : nrest);
  const bool need_pb = s > 0 && (part || m >= 2);
  lds_t<Ent>* const PB0 = part ? bufs[3] : P;   // the pb's copy in LDS
  u64* llock = H.locks + m;
  Ent* lastp = slot_ptr<K, Ent>(H, m);

  // Round trip 1: root and partial buffer into registers, first try at the
  // last node's lock.
  u64 old_last = 0;
  {
    NodeRegs<K, T, Ent> rr, pr;
    rr.load(slot_ptr<K, Ent>(H, 1));
    if (need_pb) pr.load(pb_ptr<Ent>(H));
    if (tid == 0 && refill && m >= 2) old_last = cas_old(llock, 0, lockword(ST_INUSE, ticket));
    rr.store(bufs[1]);
    if (need_pb) pr.store(PB0);
  }
  __syncthreads();
  GH_TRACE(1);
  store_n<T>(out, bufs[1], want);   // the root's smallest are the answer
  if (m == 1 && !part) {
    if constexpr (Stamp) publish();   // the output is in memory before the stamp
    if (tid == 0) release_root_at<Stamp>(meta, ticket, 0, s, sh);
    return res;
  }
  if (part) {
    // the root's other entries merged with the pb
    if (nrest >= (u32)K) {
      // the K smallest are the new root, the rest the pb; no node goes away
      merge_split<E, T>(bufs[1] + want, K - want, PB0, (int)s, K, sink(bufs[0]),
                        HeapSink<Ent>(pb_ptr<Ent>(H), K * sizeof(Ent)));
      __syncthreads();
    } else if (!refill) {
      // a single node: everything left becomes the pb
      merge_split<E, T>(bufs[1] + want, K - want, PB0, (int)s, (int)nrest,
                        HeapSink<Ent>(pb_ptr<Ent>(H), K * sizeof(Ent)), sink(bufs[0]));
      publish();
      if (tid == 0) release_root_at<Stamp>(meta, ticket, 0, nrest, sh);
      return res;
    } else {
      // waits in P for the last node
      merge_split<E, T>(bufs[1] + want, K - want, PB0, (int)s, (int)nrest, sink(P),
                        sink(bufs[0]));
      __syncthreads();
    }
  }

  lds_t<Ent>* C = bufs[0];
  bool hl = false, hr = false;
  bool loaded = false;
  if (refill) {
    // refill the root from the last node (Sec. 3.2.1)
    res.flags |= F_REFILL;
    if (tid == 0) {
      int r = old_last == 0 ? 1 : take_last(llock, old_last, ticket, ctl);
      fence_acquire();
      sh.ok = r > 0 ? 1u : 0u;
      sh.flag0 = (r == 2) ? 1u : 0u;
    }
    __syncthreads();
    GH_TRACE(2);
    if (!sh.ok) { res.ok = false; return res; }
    if (sh.flag0) res.flags |= F_TOOK;

    // Round trip 2: the last node into registers, first tries at the root's
    // children (a failed try does not wait while the last node is held).
    const bool el1 = node_exists(2, m2), er1 = node_exists(3, m2);
    u64 oc = 0;
    {
      NodeRegs<K, T, Ent> lr;
      lr.load(lastp);
      // lanes 1 and 2 try children 2 and 3 with one vector atomic
      if ((tid == 1 && el1) || (tid == 2 && er1))
        oc = cas_old(lock_ptr(H, (u32)tid + 1), 0, lockword(ST_INUSE, ticket));
      lr.store(bufs[0]);
    }
    __syncthreads();
    GH_TRACE(3);
    // The batch is in LDS: mark the node REMOVED right away (nothing was
    // stored, so no fence).
    if (tid == 0)
      st_relaxed(llock, lockword(ST_REMOVED, ticket));
    // finish the children's locks if the first tries did not settle them
    if (tid < 64) {
      const bool mine = (tid == 1 && el1) || (tid == 2 && er1);
      int got = 0;
      bool need = false;
      if (mine) {
        if (oc == 0) got = 1;
        else if (child_view(oc, ticket) == 0) got = 0;
        else need = true;
      }
      bool ok = true;
      if (__any(need)) {
        int r2 = 0;
        u64* w = tid == 1 ? lock_ptr(H, 2) : lock_ptr(H, 3);
        ok = lock_lanes(w, LM_CHILD, ticket, need, r2, ctl);
        if (need) got = r2;
      } else if (__any(got == 1)) {
        fence_acquire();
      }
      const bool allok = __all(ok);
      if (tid == 0) sh.ok = allok ? 1u : 0u;
      if (tid == 1) sh.flag0 = got > 0 ? 1u : 0u;
      if (tid == 2) sh.flag1 = got > 0 ? 1u : 0u;
    }
    __syncthreads();
    GH_TRACE(4);
    if (!sh.ok) { res.ok = false; return res; }

    // Round trip 3: the children, loaded while cur merges with the partial
    // buffer (Property 3 again: the refilled root keeps the K smallest).
    // With want < K the merged rest takes the pb's place and always merges:
    // what does not stay in the root is the new pb.
    hl = sh.flag0;
    hr = sh.flag1;
    {
      NodeRegs<K, T, Ent> lc, rc;
      if (hl) lc.load(slot_ptr<K, Ent>(H, 2));   // node 2 is position 2
      if (hr) rc.load(node_ptr<K, Ent>(H, 3));
      const u32 np = part ? nrest : s;
      if (np > 0 && (part || !ent_le(C[K - 1], P[0]))) {
        merge_split<E, T>(C, K, P, (int)np, K, sink(bufs[3]), HeapSink<Ent>(pb_ptr<Ent>(H), K * sizeof(Ent)));
        __syncthreads();
        lds_t<Ent>* x = bufs[0]; bufs[0] = bufs[3]; bufs[3] = x;
        C = bufs[0];
      }
      if (hl) lc.store(bufs[1]);
      if (hr) rc.store(bufs[2]);
    }
    __syncthreads();
    GH_TRACE(5);
    loaded = true;
  }

  // sift down; after a refill the root level's children are already locked
  // and loaded
  return del_sift<K, T, Ent, Stamp>(H, ticket, 1, loaded, hl, hr, false, ~0ull, bufs, m2, s2, sh,
                                    ctl, res);
}

}  // namespace gh
