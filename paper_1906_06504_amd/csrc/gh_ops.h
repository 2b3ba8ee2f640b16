// gh_ops.h -- one INS or DEL on a generalized heap, run by one workgroup
// (Sec. 4: one thread block per operation), with the TD-INS/TD-DEL locking
// protocol of Sec. 3.3.
//
// Locking summary (Sec. 3.3.1 lock order, Sec. 3.3.2 states):
//  * The root is taken with a ticket lock: an operation with ticket t waits
//    until meta.serving == t and releases it by storing t + 1.  Root order is
//    the linearization order (Theorem 1).  The partial buffer and the root
//    metadata (m, s) are guarded by the root.
//  * Every other node has a lock word.  Locks are taken parent before child
//    and a child is locked before its parent is released (hand-over-hand).
//  * An insert that needs a new node reserves it at the root as
//    TARGET(ticket).  A deleteMin that must take the last node while it is
//    still an in-flight insert's target marks it MARKED; the insert then
//    leaves its batch in the target slot, sets HANDED and stops, and the
//    deleteMin proceeds with those entries.
//  * A deleteMin sifting down treats a child as absent when it does not
//    exist in the deleteMin's own view of the heap size, when it is the
//    reserved target of a LATER insert (that insert will pass the parent
//    after this deleteMin), or when its first entry is ENT_MAX (a later
//    deleteMin already moved its entries to the root).  A target of an
//    EARLIER insert is waited for: that insert is past the parent and only
//    has to store its batch.
#pragma once

#include "gh_device.h"

namespace gh {

struct OpShared {
  u64 m, s;            // root metadata read at root acquire
  u64 t_claim;         // clock when the operation was claimed
  u64 t_root;          // clock at root acquire
  u32 flag0, flag1;    // broadcast results from thread 0
  u32 ok;
  u32 op;
};

struct OpResult {
  u32 count;
  u32 levels;
  u32 flags;
  bool ok;
};

constexpr u32 F_FULL = 1, F_HANDOFF = 2, F_TOOK = 4, F_ROOT = 8, F_REFILL = 16, F_REJECT = 0x40,
              F_ABORT = 0x80;

// --- thread-0 lock primitives (return false when the wait is abandoned) ---

__device__ __forceinline__ bool root_acquire(HeapMeta* meta, u64 ticket, Ctl* ctl) {
  Waiter w;
  for (;;) {
    u64 sv = ld_relaxed(&meta->serving);
    if (sv == ticket) break;
    u64 ahead = ticket - sv;  // operations still in front of us
    if (!w.step(ctl, ahead > 8 ? 16 : (ahead > 2 ? 4 : 1))) return false;
  }
  fence_acquire();
  return true;
}

// plain lock of a path node for an insert: AVAIL -> INUSE
__device__ __forceinline__ bool lock_path(u64* lw, u64 ticket, Ctl* ctl) {
  Waiter w;
  for (;;) {
    u64 v = ld_relaxed(lw);
    if (lw_state(v) == ST_AVAIL && cas_relaxed(lw, v, lockword(ST_INUSE, ticket))) break;
    if (!w.step(ctl)) return false;
  }
  fence_acquire();
  return true;
}

// reserve the new target: AVAIL -> TARGET(ticket)
__device__ __forceinline__ bool lock_target(u64* lw, u64 ticket, Ctl* ctl) {
  Waiter w;
  for (;;) {
    u64 v = ld_relaxed(lw);
    if (lw_state(v) == ST_AVAIL && cas_relaxed(lw, v, lockword(ST_TARGET, ticket))) return true;
    if (!w.step(ctl)) return false;
  }
}

// deleteMin locking a child: 1 = locked, 0 = absent, -1 = abandoned
__device__ __forceinline__ int lock_child(u64* lw, u64 ticket, Ctl* ctl) {
  Waiter w;
  for (;;) {
    u64 v = ld_relaxed(lw);
    u64 st = lw_state(v);
    if (st == ST_AVAIL) {
      if (cas_relaxed(lw, v, lockword(ST_INUSE, ticket))) {
        fence_acquire();
        return 1;
      }
      continue;
    }
    if (st != ST_INUSE && lw_ticket(v) > ticket) return 0;  // a later insert's target
    if (!w.step(ctl)) return -1;
  }
}

// deleteMin taking the last node while holding the root: 1 = plain lock,
// 2 = took an in-flight insert's batch (MARKED -> HANDED), -1 = abandoned
__device__ __forceinline__ int take_last(u64* lw, u64 ticket, Ctl* ctl) {
  Waiter w;
  for (;;) {
    u64 v = ld_relaxed(lw);
    u64 st = lw_state(v);
    if (st == ST_AVAIL) {
      if (cas_relaxed(lw, v, lockword(ST_INUSE, ticket))) {
        fence_acquire();
        return 1;
      }
      continue;
    }
    if (st == ST_TARGET) {
      u64 owner = lw_ticket(v);
      if (cas_relaxed(lw, v, lockword(ST_MARKED, owner))) {
        Waiter w2;
        for (;;) {
          u64 x = ld_relaxed(lw);
          if (x == lockword(ST_HANDED, owner)) break;
          if (lw_state(x) == ST_AVAIL) break;  // cannot happen: the insert saw MARKED
          if (!w2.step(ctl)) return -1;
        }
        st_release(lw, lockword(ST_INUSE, ticket));
        fence_acquire();
        return 2;
      }
      continue;
    }
    if (!w.step(ctl)) return -1;
  }
}

__device__ __forceinline__ void unlock(u64* lw) { st_release(lw, lockword(ST_AVAIL, 0)); }

// An operation that may not change the heap (an insert of 0 entries, or a
// malformed record) still passes the root in its turn, so the tickets after
// it keep flowing.
__device__ __forceinline__ OpResult op_pass_root(const HeapDesc& H, u64 ticket, OpShared& sh, Ctl* ctl) {
  OpResult res{0, 0, 0, true};
  if (threadIdx.x == 0) {
    sh.ok = root_acquire(H.meta, ticket, ctl) ? 1u : 0u;
    sh.t_root = now_ticks();
    sh.s = 0;
    if (sh.ok) st_release(&H.meta->serving, ticket + 1);
  }
  __syncthreads();
  res.ok = sh.ok != 0;
  return res;
}

// ---------------------------------------------------------------------------
// INS (Sec. 3.2.2 top-down insert, Sec. 3.3.2 partial batches and
// cooperation).  `keys` holds n (1..K) entries in global memory.
// LDS: buf[0..4] of K entries each.
// ---------------------------------------------------------------------------
template <int K, int T>
__device__ OpResult op_insert(const HeapDesc& H, u64 ticket, const u64* __restrict__ keys, u32 n,
                              u64* lds, OpShared& sh, Ctl* ctl) {
  constexpr int E = (2 * K) / T >= 1 ? (2 * K) / T : 1;
  const int tid = threadIdx.x;
  OpResult res{n, 0, 0, true};
  u64* b0 = lds;
  u64* b1 = lds + K;
  u64* b2 = lds + 2 * K;
  u64* b3 = lds + 3 * K;
  u64* b4 = lds + 4 * K;
  HeapMeta* meta = H.meta;

  // sort the batch before touching the heap (holds no lock)
  load_n<T>(b0, keys, n);
  u64* xs = block_sort<K, T>(b0, b1, (int)n);
  u64* xfree = (xs == b0) ? b1 : b0;

  if (tid == 0) {
    sh.ok = root_acquire(meta, ticket, ctl) ? 1u : 0u;
    sh.t_root = now_ticks();
    if (sh.ok) {
      sh.m = meta->m;
      sh.s = meta->s;
    }
  }
  __syncthreads();
  if (!sh.ok) { res.ok = false; return res; }
  const u64 m = sh.m;
  const u32 s = (u32)sh.s;
  if (m >= 1) res.flags |= F_ROOT;
  if (n + s >= (u32)K && m + 1 > H.max_nodes) {
    // no room for another node: reject the insert, leave the heap unchanged
    if (tid == 0) {
      note_error(ctl, ERR_NOMEM);
      st_release(&meta->serving, ticket + 1);
    }
    res.count = 0;
    res.flags |= F_REJECT;
    return res;
  }

  // merged = merge(sorted input, partial buffer): first K -> b3, rest -> xfree
  if (s > 0) load_n<T>(b2, H.pb, s);
  __syncthreads();
  const u32 tot = n + s;
  merge_split<E, T>(xs, (int)n, b2, (int)s, K, Sink{b3}, Sink{xfree});
  __syncthreads();

  u64* root = H.nodes;  // position 1
  if (tot <= (u32)(K - 1)) {
    // the partial buffer keeps everything; restore Property 3 against the root
    if (m >= 1) {
      load_node<K, T>(b4, root);
      __syncthreads();
      if (b4[K - 1] <= b3[0]) {
        store_n<T>(H.pb, b3, tot);
      } else {
        merge_split<E, T>(b4, K, b3, (int)tot, K, Sink{root}, Sink{H.pb});
      }
    } else {
      store_n<T>(H.pb, b3, tot);
    }
    if (tid == 0) meta->s = tot;
    publish();
    if (tid == 0) st_release(&meta->serving, ticket + 1);
    return res;
  }

  // a full batch F = b3 goes down from the root; the rest stays in the pb
  res.flags |= F_FULL;
  const u32 rest = tot - K;
  store_n<T>(H.pb, xfree, rest);
  const u64 m2 = m + 1;
  const u32 t = bitrev_pos((u32)m2);  // target node index
  const int L = level_of(t);
  if (tid == 0) {
    meta->m = m2;
    meta->s = rest;
  }
  if (L == 0) {
    store_node<K, T>(root, b3);
    publish();
    if (tid == 0) st_release(&meta->serving, ticket + 1);
    return res;
  }
  u64* tlock = H.locks + m2;
  if (tid == 0) sh.ok = lock_target(tlock, ticket, ctl) ? 1u : 0u;
  // root level: root keeps the K smallest of root + F
  load_node<K, T>(b4, root);
  __syncthreads();
  if (!sh.ok) { res.ok = false; return res; }

  u64* F = b3;        // carry
  u64* N = b4;        // node being merged
  u64* spare0 = b0;   // free buffers
  u32 cur = 1;
  int level = 0;
  for (;;) {
    // (node, F) = MergeAndSort(node, F) with the shortcuts of Sec. 4.3
    u64* cur_ptr = node_ptr<K>(H, cur);
    if (N[K - 1] <= F[0]) {
      // node already holds the smallest: nothing moves
    } else if (F[K - 1] <= N[0]) {
      store_node<K, T>(cur_ptr, F);  // swap
      u64* x = F; F = N; N = x;
    } else {
      merge_split<E, T>(N, K, F, K, K, Sink{cur_ptr}, Sink{spare0});
      __syncthreads();
      u64* x = F; F = spare0; spare0 = x;
    }
    ++level;
    const u32 child = t >> (L - level);
    if (child == t) break;
    // before moving on: was our target claimed by a deleteMin?  Otherwise
    // lock the next path node (child before parent release).
    if (tid == 0) {
      u64 w = ld_relaxed(tlock);
      if (lw_state(w) == ST_MARKED) {
        sh.flag0 = 1;
        sh.ok = 1;
      } else {
        sh.flag0 = 0;
        sh.ok = lock_path(lock_ptr(H, child), ticket, ctl) ? 1u : 0u;
      }
    }
    __syncthreads();
    if (!sh.ok) { res.ok = false; return res; }
    if (sh.flag0) {
      // cooperation: leave the batch in the target slot for the deleteMin
      store_node<K, T>(node_ptr<K>(H, t), F);
      publish();
      if (tid == 0) {
        if (cur == 1) st_release(&meta->serving, ticket + 1);
        else unlock(lock_ptr(H, cur));
        st_release(tlock, lockword(ST_HANDED, ticket));
      }
      res.levels = level;
      res.flags |= F_HANDOFF;
      return res;
    }
    publish();
    if (tid == 0) {
      if (cur == 1) st_release(&meta->serving, ticket + 1);
      else unlock(lock_ptr(H, cur));
    }
    cur = child;
    load_node<K, T>(N, node_ptr<K>(H, cur));
    __syncthreads();
  }
  // release the last path node, then fill the target
  store_node<K, T>(node_ptr<K>(H, t), F);
  publish();
  if (tid == 0) {
    if (cur == 1) st_release(&meta->serving, ticket + 1);
    else unlock(lock_ptr(H, cur));
    if (!cas_relaxed(tlock, lockword(ST_TARGET, ticket), lockword(ST_AVAIL, 0))) {
      // MARKED by a deleteMin: the batch is already in the target slot
      st_release(tlock, lockword(ST_HANDED, ticket));
      sh.flag1 = 1;
    } else {
      sh.flag1 = 0;
    }
  }
  __syncthreads();
  if (sh.flag1) res.flags |= F_HANDOFF;
  res.levels = L;
  (void)b2;
  return res;
}

// ---------------------------------------------------------------------------
// DEL (Sec. 3.2.1 with the partial-buffer rules of Sec. 3.3.2/3.3.4).
// Writes min(K, size) entries to out.
// ---------------------------------------------------------------------------
template <int K, int T>
__device__ OpResult op_delete(const HeapDesc& H, u64 ticket, u64* __restrict__ out, u64* lds,
                              OpShared& sh, Ctl* ctl) {
  constexpr int E = (2 * K) / T >= 1 ? (2 * K) / T : 1;
  const int tid = threadIdx.x;
  OpResult res{0, 0, 0, true};
  HeapMeta* meta = H.meta;
  u64* root = H.nodes;

  if (tid == 0) {
    sh.ok = root_acquire(meta, ticket, ctl) ? 1u : 0u;
    sh.t_root = now_ticks();
    if (sh.ok) {
      sh.m = meta->m;
      sh.s = meta->s;
    }
  }
  __syncthreads();
  if (!sh.ok) { res.ok = false; return res; }
  const u64 m = sh.m;
  const u32 s = (u32)sh.s;
  if (m >= 1) res.flags |= F_ROOT;

  if (m == 0) {
    // no node: the partial buffer is the whole heap
    copy_n<T>(out, H.pb, s);
    if (tid == 0) meta->s = 0;
    publish();
    if (tid == 0) st_release(&meta->serving, ticket + 1);
    res.count = s;
    return res;
  }
  res.count = K;
  for (int i = tid * 2; i < K; i += 2 * T) {
    ulonglong2 v = *reinterpret_cast<const ulonglong2*>(root + i);
    out[i] = v.x;
    out[i + 1] = v.y;
  }
  if (m == 1) {
    if (tid == 0) {
      meta->m = 0;
      root[0] = ENT_MAX;
    }
    publish();
    if (tid == 0) st_release(&meta->serving, ticket + 1);
    return res;
  }

  // refill the root from the last node (Sec. 3.2.1), MAX-marking that node
  res.flags |= F_REFILL;
  const u64 m2 = m - 1;
  u64* llock = H.locks + m;
  u64* lastp = H.nodes + (m - 1) * (u64)K;
  if (tid == 0) {
    int r = take_last(llock, ticket, ctl);
    sh.ok = r > 0 ? 1u : 0u;
    sh.flag0 = (r == 2) ? 1u : 0u;
  }
  __syncthreads();
  if (!sh.ok) { res.ok = false; return res; }
  if (sh.flag0) res.flags |= F_TOOK;

  u64* bufs[4] = {lds, lds + K, lds + 2 * K, lds + 3 * K};
  u64* P = lds + 4 * K;
  u64* C = bufs[0];
  load_node<K, T>(C, lastp);
  if (s > 0) load_n<T>(P, H.pb, s);
  __syncthreads();
  // Release the last node before locking any child of the root: an earlier
  // deleteMin may be waiting for it while holding a node on our way down.
  if (tid == 0) lastp[0] = ENT_MAX;
  publish();
  if (tid == 0) {
    unlock(llock);
    meta->m = m2;
  }
  if (s > 0) {
    // Property 3 again: the refilled root keeps the K smallest of root + pb
    if (!(C[K - 1] <= P[0])) {
      merge_split<E, T>(C, K, P, (int)s, K, Sink{bufs[1]}, Sink{H.pb});
      __syncthreads();
      u64* x = bufs[0]; bufs[0] = bufs[1]; bufs[1] = x;
      C = bufs[0];
    }
  }

  // sift down
  u32 c = 1;
  for (;;) {
    const u64 l = 2ull * c, r = l + 1;
    const bool el = node_exists(l, m2), er = node_exists(r, m2);
    if (tid == 0) {
      int pl = 0, pr = 0;
      bool ok = true;
      if (el) {
        pl = lock_child(lock_ptr(H, (u32)l), ticket, ctl);
        ok = pl >= 0;
      }
      if (ok && er) {
        pr = lock_child(lock_ptr(H, (u32)r), ticket, ctl);
        ok = pr >= 0;
      }
      sh.ok = ok ? 1u : 0u;
      sh.flag0 = pl > 0 ? 1u : 0u;
      sh.flag1 = pr > 0 ? 1u : 0u;
    }
    __syncthreads();
    if (!sh.ok) { res.ok = false; return res; }
    const bool pl = sh.flag0, pr = sh.flag1;
    u64* Lb = bufs[1];
    u64* Rb = bufs[2];
    if (pl) load_node<K, T>(Lb, node_ptr<K>(H, (u32)l));
    if (pr) load_node<K, T>(Rb, node_ptr<K>(H, (u32)r));
    __syncthreads();
    const bool hl = pl && Lb[0] != ENT_MAX;
    const bool hr = pr && Rb[0] != ENT_MAX;
    const u64 lmin = hl ? Lb[0] : ENT_MAX;
    const u64 rmin = hr ? Rb[0] : ENT_MAX;
    const u64 cmin = lmin < rmin ? lmin : rmin;
    u64* cptr = node_ptr<K>(H, c);

    if (C[K - 1] <= cmin) {
      // the property holds: place cur and stop (early stop, Sec. 4.3)
      store_node<K, T>(cptr, C);
      publish();
      if (tid == 0) {
        if (pl) unlock(lock_ptr(H, (u32)l));
        if (pr) unlock(lock_ptr(H, (u32)r));
        if (c == 1) st_release(&meta->serving, ticket + 1);
        else unlock(lock_ptr(H, c));
      }
      return res;
    }

    u32 next;
    u64* newcur;
    if (hl && hr) {
      // (hi, lo) = MergeAndSort(l, r); lo stays in the child whose max was
      // larger, hi merges with cur; cur's k smallest stay here
      // (on a tie of the maxima the right child counts as larger)
      const bool big_is_l = Lb[K - 1] > Rb[K - 1];
      const u32 big = big_is_l ? (u32)l : (u32)r;
      const u32 small = big_is_l ? (u32)r : (u32)l;
      u64* Bg = big_is_l ? Lb : Rb;
      u64* Sm = big_is_l ? Rb : Lb;
      u64* hi;
      u64* freeb;
      if (Sm[K - 1] <= Bg[0]) {
        hi = Sm;             // lo is the big child's batch, already in place
        freeb = bufs[3];
      } else {
        merge_split<E, T>(Lb, K, Rb, K, K, Sink{bufs[3]}, Sink{node_ptr<K>(H, big)});
        __syncthreads();
        hi = bufs[3];
        freeb = Lb;
      }
      if (hi[K - 1] <= C[0]) {
        store_node<K, T>(cptr, hi);
        newcur = C;
      } else {
        merge_split<E, T>(C, K, hi, K, K, Sink{cptr}, Sink{freeb});
        __syncthreads();
        newcur = freeb;
      }
      publish();
      if (tid == 0) {
        unlock(lock_ptr(H, big));
        if (c == 1) st_release(&meta->serving, ticket + 1);
        else unlock(lock_ptr(H, c));
      }
      next = small;
    } else {
      // one live child x
      const u32 x = hl ? (u32)l : (u32)r;
      u64* X = hl ? Lb : Rb;
      u64* freeb = bufs[3];
      if (X[K - 1] <= C[0]) {
        store_node<K, T>(cptr, X);
        newcur = C;
      } else {
        merge_split<E, T>(C, K, X, K, K, Sink{cptr}, Sink{freeb});
        __syncthreads();
        newcur = freeb;
      }
      publish();
      if (tid == 0) {
        // a child that was locked but found MAX-marked is released here
        if (pl && !hl) unlock(lock_ptr(H, (u32)l));
        if (pr && !hr) unlock(lock_ptr(H, (u32)r));
        if (c == 1) st_release(&meta->serving, ticket + 1);
        else unlock(lock_ptr(H, c));
      }
      next = x;
    }
    ++res.levels;
    // rotate buffers: newcur becomes C, the other three are free
    {
      u64* all[4] = {bufs[0], bufs[1], bufs[2], bufs[3]};
      int j = 1;
      bufs[0] = newcur;
      for (int q = 0; q < 4; ++q)
        if (all[q] != newcur) bufs[j++] = all[q];
      C = bufs[0];
    }
    c = next;
  }
}

}  // namespace gh
