// gh_ops_bu.h -- the bottom-up insert (Sec. 3.2.2, "Bottom-up INS"
// paragraph; Sec. 3.3.4) for insert phases: submissions in which every
// operation is an insert.
//
// The root phase is the top-down insert's (Sec. 3.3.4 handles the partial
// buffer the same way in both heaps): with the root's ticket the insert
// merges its sorted batch with the partial buffer.  If everything fits the
// partial buffer it stays there and is merged with the root (Property 3).
// Otherwise the k smallest form a full batch F, the rest is the new partial
// buffer, the next node position is reserved as F's target, and the root
// goes to the next ticket without the root node being touched.  F is then
// placed at the target and climbs: the insert holds its current node,
// locks the parent, and merges the two (the parent keeps the k smallest)
// until the parent's largest entry is no larger than the node's smallest or
// the root has been merged.  Run one at a time this leaves exactly the
// top-down insert's layout: the batches on a root-to-target path are
// ordered, so both directions leave their sorted union in consecutive
// chunks.
//
// Locks.  A climbing insert holds a node and waits for its parent: every
// wait points one level up, so climbers cannot deadlock among themselves.
// The root node's content gets a lock word of its own (position 1's word,
// unused by the top-down form): a climber merging into the root and a
// root-phase insert that merges the partial buffer with the root take it;
// the latter already holds the root's ticket, and a climber never waits for
// a ticket, so no cycle forms.
//
// Why insert phases only.  With deleteMins in flight the root ticket is not
// a linearization point for a climbing insert (its batch reaches the root
// after later deleteMins), and the rule of Sec. 3.3.5 (linearize at the
// last locked node) does not hold either: a deleteMin sifting through a
// node that a climber has let go merges the climber's batch upward, and the
// next deleteMin can return entries of an insert that has not finished
// climbing.  The same holds for the partial-buffer part of a full batch,
// which can lie below the root's largest entry until the climb ends.  So
// bottom-up inserts run in submissions of inserts only; deleteMins run in
// the top-down form between such submissions, and every kernel boundary is
// a quiescent point at which Properties 1-3 hold.
#pragma once

#include "gh_ops.h"

namespace gh {

// Thread 0: take node c's lock word for a climber or for a root-phase merge
// with the root (AVAIL -> INUSE).  Position 1's word is the root node's own
// lock in this form.  A node that is still another insert's reserved target,
// or is held by another climber, is waited for.
__device__ __forceinline__ bool bu_lock(const HeapDesc& H, u32 c, u64 ticket, Ctl* ctl) {
  u64* lw = lock_ptr(H, c);
  Waiter w;
  for (;;) {
    const u64 v = ld_relaxed(lw);
    if (lw_state(v) == ST_AVAIL && cas_relaxed(lw, v, lockword(ST_INUSE, ticket))) break;
    if (!w.step(ctl)) return false;
  }
  fence_acquire();
  return true;
}

// Algorithmic bytes of a bottom-up insert: the input and partial buffer as
// for the top-down insert; for a full batch the target written (K), per
// merge the parent read and both nodes written (3K), and the parent read by
// the check that stopped the climb below the root (K).
template <int K, class Ent>
__device__ __forceinline__ u64 bu_alg_bytes(const OpResult& r, u64 s) {
  constexpr u64 e = sizeof(Ent);
  if (r.flags & F_REJECT) return 0;
  const u64 n = r.count;
  const bool stopped = (r.flags & F_STOPPED) != 0;
  if (r.flags & F_FULL)
    return e * (n + s + (n + s - K)) + e * ((u64)K + 3ull * K * r.levels + (stopped ? K : 0));
  return e * 2 * (n + s) + ((r.flags & F_ROOT) ? 2 * e * K : 0);
}

template <int K, int T, class Ent>
__device__ __forceinline__ OpResult op_insert_bu(const HeapDesc& H, u64 ticket,
                                                 const Ent* __restrict__ keys, u32 n,
                                                 lds_t<Ent>* lds, OpShared& sh, Ctl* ctl) {
  constexpr int E = (2 * K) / T >= 1 ? (2 * K) / T : 1;
  const int tid = threadIdx.x;
  OpResult res{n, 0, 0, true};
  lds_t<Ent>* b0 = lds;
  lds_t<Ent>* b1 = lds + K;
  lds_t<Ent>* P = lds + 2 * K;   // partial buffer
  lds_t<Ent>* F = lds + 3 * K;   // the batch (the climber's current node)
  lds_t<Ent>* N = lds + 4 * K;   // the parent / the root
  HeapMeta* meta = H.meta;

  // sort the batch before touching the heap
  load_n<T>(b0, keys, n);
  lds_t<Ent>* xs = block_sort<K, T, Ent>(b0, b1, (int)n);
  lds_t<Ent>* xfree = (xs == b0) ? b1 : b0;

  if (!acquire_root(H, ticket, sh, ctl)) { res.ok = false; return res; }
  const u64 m = sh.m;
  const u32 s = (u32)sh.s;
  if (m >= 1) res.flags |= F_ROOT;
  const bool full = n + s >= (u32)K;
  if (full && m + 1 > H.max_nodes) {
    if (tid == 0) {
      note_error(ctl, ERR_NOMEM);
      release_root(meta, ticket, m, s);
    }
    res.count = 0;
    res.flags |= F_REJECT;
    return res;
  }
  const u32 tot = n + s;

  if (!full) {
    // the partial buffer keeps everything and is merged with the root: the
    // root node's lock keeps climbers out meanwhile
    if (tid == 0) sh.ok = (m == 0 || bu_lock(H, 1, ticket, ctl)) ? 1u : 0u;
    __syncthreads();
    if (!sh.ok) { res.ok = false; return res; }
    {
      NodeRegs<K, T, Ent> pr, rr;
      pr.load(pb_ptr<Ent>(H));
      if (m >= 1) rr.load(slot_ptr<K, Ent>(H, 1));
      pr.store(P);
      if (m >= 1) rr.store(N);
    }
    __syncthreads();
    merge_split<E, T>(xs, (int)n, P, (int)s, K, sink(F), sink(xfree));
    __syncthreads();
    Ent* root = slot_ptr<K, Ent>(H, 1);
    if (m >= 1 && !ent_le((Ent)N[K - 1], (Ent)F[0])) {
      merge_split<E, T>(N, K, F, (int)tot, K, HeapSink<Ent>(root, K * sizeof(Ent)),
                        HeapSink<Ent>(pb_ptr<Ent>(H), K * sizeof(Ent)));
    } else {
      store_heap_n<K, T, Ent>(pb_ptr<Ent>(H), F, tot);
    }
    publish();
    if (tid == 0) {
      if (m >= 1) unlock(lock_ptr(H, 1));
      release_root(meta, ticket, m, tot);
    }
    return res;
  }

  // a full batch: the partial buffer only (the root node stays as it is)
  res.flags |= F_FULL;
  const u64 m2 = m + 1;
  const u32 t = bitrev_pos((u32)m2);
  {
    NodeRegs<K, T, Ent> pr;
    if (s > 0) pr.load(pb_ptr<Ent>(H));
    u64 old = 0;
    if (tid == 0 && t != 1) old = xchg_relaxed(H.locks + m2, lockword(ST_TARGET, ticket));
    if (s > 0) pr.store(P);
    if (tid == 0) {
      const bool bad = t != 1 && lw_state(old) != ST_AVAIL && lw_state(old) != ST_REMOVED;
      if (bad) raise_error(ctl, ERR_STATE);
      sh.ok = bad ? 0u : 1u;
    }
  }
  __syncthreads();
  if (!sh.ok) { res.ok = false; return res; }
  const u32 rest = tot - K;
  merge_split<E, T>(xs, (int)n, P, (int)s, K, sink(F), sink(xfree));
  __syncthreads();
  store_heap_n<K, T, Ent>(pb_ptr<Ent>(H), xfree, rest);
  if (t == 1) {
    // the heap had no node: the batch is the root
    store_node<K, T, Ent>(slot_ptr<K, Ent>(H, 1), F);
    publish();
    if (tid == 0) release_root(meta, ticket, m2, rest);
    return res;
  }
  publish();
  if (tid == 0) release_root(meta, ticket, m2, rest);

  // climb from the target
  lds_t<Ent>* spare = P;   // the partial buffer's copy is no longer needed
  u32 c = t;   // the climber's node; its lock word is TARGET(ticket) or INUSE
  for (;;) {
    const u32 p = c >> 1;
    if (tid == 0) sh.ok = bu_lock(H, p, ticket, ctl) ? 1u : 0u;
    __syncthreads();
    if (!sh.ok) { res.ok = false; return res; }
    Ent* pptr = node_ptr<K, Ent>(H, p);
    Ent* cptr = node_ptr<K, Ent>(H, c);
    {
      NodeRegs<K, T, Ent> nr;
      nr.load(pptr);
      nr.store(N);
    }
    __syncthreads();
    if (ent_le((Ent)N[K - 1], (Ent)F[0])) {
      // the property holds from here up: the batch stays at c
      store_node<K, T, Ent>(cptr, F);
      publish();
      if (tid == 0) {
        unlock(lock_ptr(H, c));   // our target (was TARGET) or a node we locked
        unlock(lock_ptr(H, p));
      }
      res.flags |= F_STOPPED;
      return res;
    }
    if (ent_le((Ent)F[K - 1], (Ent)N[0])) {
      // swap: the parent's batch goes down to c; the climber's batch (F)
      // is now p's
      store_node<K, T, Ent>(cptr, N);
    } else {
      // the parent keeps the K smallest (the climber's new batch), the rest
      // goes down to c
      merge_split<E, T>(N, K, F, K, K, sink(spare), HeapSink<Ent>(cptr, K * sizeof(Ent)));
      lds_t<Ent>* x = F; F = spare; spare = x;
    }
    ++res.levels;
    publish();
    if (tid == 0) unlock(lock_ptr(H, c));
    if (p == 1) {
      // merged into the root: the climb ends there
      store_node<K, T, Ent>(pptr, F);
      publish();
      if (tid == 0) unlock(lock_ptr(H, 1));
      return res;
    }
    c = p;
  }
}

}  // namespace gh
