// gh_ops_multi.h -- an insert of more than K entries that takes the root once
// (the footnote to the INS paragraph of Sec. 3.2.2 lets an insert of more
// than k keys run as several INS operations; here they share one root hold).
//
// Chunks.  The n entries are cut, in input order, into chunks of K and a
// last shorter chunk, exactly as consecutive single inserts would take them.
// While holding the root, the operation runs every chunk's root phase in
// chunk order with the root and the partial buffer kept in LDS: sort the
// chunk, merge it with the partial buffer, and either keep everything in the
// partial buffer (restoring Property 3 against the root) or cut a full batch,
// MergeAndSort it with the root and reserve the next node position as its
// target.  A full batch's carry (the K largest of root and batch) is staged
// in its target's own slot.  Root and partial buffer are written back once,
// the root's children on the carries' paths are locked, and the root goes to
// the next ticket.
//
// Descent.  The carries then travel down their root-to-target paths level
// by level: at each path node every carry passing through it merges with the
// node in chunk order (the node keeps the K smallest), the node's children on
// those paths are locked before the node is released (hand-over-hand, Sec.
// 3.3.1), and a carry whose target is a child of the node is final there.
// The same layout as chunk-by-chunk inserts follows: a chunk's descent
// touches only nodes below the root and a later chunk's root phase only the
// root and the partial buffer, so all root phases may run first; and every
// path node still sees the carries through it in chunk order.  A target
// reserved by an earlier chunk of the same operation can lie on a later
// carry's path (a heap smaller than the insert); its TARGET state, which
// carries this operation's ticket, then serves as the lock while later
// carries pass through it, and it is released like any target afterwards.
//
// Concurrency.  The root ticket is the whole operation's linearization
// point, as for a single insert (Theorem 1): after the root hold the root is
// the K smallest of everything and every carry holds entries no smaller than
// the root's.  Later operations cannot overtake the carries: they reach a
// path node only through its parent, which this operation holds until the
// node is locked.  A deleteMin that needs one of the reserved targets as the
// last node marks it; before each level the operation looks at the targets
// of the carries still travelling and hands a marked one over at once (the
// carry is at rest in the target's slot), and a carry that becomes final at
// a marked target is handed over there.
#pragma once

#include "gh_ops.h"

namespace gh {

constexpr u32 MH_OWN = 0x80000000u;   // a held node that is one of our own targets

struct MultiShared {
  u32 tgt[64];       // target node index of carry j (chunk order)
  u32 tpos[64];      // its position (bit-reversal order)
  u32 lvl[64];       // its level
  u32 alive[64];     // 1 while the carry travels
  u32 held[2][64];   // nodes held at the current and the next level (| MH_OWN)
  u32 nheld[2];
  u32 cl[64];        // carries through the node being processed, chunk order
  u32 ncl;
  u32 lockv[2];      // children to lock for them
  u32 nb;            // carries
  u32 flags;         // result flags gathered by thread 0
  u32 bad;           // a reserved target was in an unexpected state
};

// Thread 0: release one of our own targets whose final batch is published:
// TARGET -> AVAIL, or, if a deleteMin marked it, hand the batch over.
__device__ __forceinline__ bool mh_finalize(const HeapDesc& H, u64 pos, u64 ticket) {
  u64* lw = H.locks + pos;
  if (cas_relaxed(lw, lockword(ST_TARGET, ticket), lockword(ST_AVAIL, 0))) return false;
  st_relaxed(lw, lockword(ST_HANDED, ticket));
  return true;
}

// Wave 0: lane i < cnt takes node nodes[i] (unless it carries MH_OWN) on the
// insert path.  Returns false in every lane when the wait is abandoned.
__device__ __forceinline__ bool mh_lock_nodes(const HeapDesc& H, const u32* nodes, u32 cnt,
                                              u64 ticket, Ctl* ctl) {
  const int tid = threadIdx.x;
  const bool active = (u32)tid < cnt && !(nodes[tid] & MH_OWN);
  u64* w = active ? lock_ptr(H, nodes[tid]) : nullptr;
  int r = 0;
  if (!__any(active)) return true;
  const bool ok = lock_lanes(w, LM_PATH, ticket, active, r, ctl);
  return __all(ok);
}

// Kept out of line: the rarer, longer path should not raise the register
// budget of the kernels' common paths.  The heap descriptor is read from the
// set's descriptor array (hd), so nothing goes through private memory.
template <int K, int T, class Ent, bool Stamp = false>
__device__ __forceinline__ OpResult op_insert_multi(const HeapDesc* __restrict__ hd, u64 ticket,
                                                 const Ent* __restrict__ keys, u32 n,
                                                 lds_t<Ent>* lds, OpShared& sh, Ctl* ctl) {
  constexpr int E = (2 * K) / T >= 1 ? (2 * K) / T : 1;
  const HeapDesc H = *hd;
  __shared__ MultiShared ms;
  const int tid = threadIdx.x;
  OpResult res{n, 0, 0, true};
  HeapMeta* meta = H.meta;

  if (!acquire_root(H, ticket, sh, ctl)) { res.ok = false; return res; }
  const u64 m0 = sh.m;
  const u32 s0 = (u32)sh.s;
  if (m0 >= 1) res.flags |= F_ROOT;
  const u64 nfull = ((u64)n + s0) / (u64)K;
  if (m0 + nfull > H.max_nodes) {
    // not enough node slots for every batch: reject the whole insert
    if (tid == 0) {
      note_error(ctl, ERR_NOMEM);
      release_root_at<Stamp>(meta, ticket, m0, s0, sh);
    }
    res.count = 0;
    res.flags |= F_REJECT;
    return res;
  }

  // five LDS buffers of K entries: the root N, the partial buffer P, and
  // three free ones A, B, C (roles move by pointer)
  lds_t<Ent>* N = lds;
  lds_t<Ent>* P = lds + K;
  lds_t<Ent>* A = lds + 2 * K;
  lds_t<Ent>* B = lds + 3 * K;
  lds_t<Ent>* C = lds + 4 * K;
  {
    NodeRegs<K, T, Ent> pr, rr;
    pr.load(pb_ptr<Ent>(H));
    if (m0 >= 1) rr.load(slot_ptr<K, Ent>(H, 1));
    pr.store(P);
    if (m0 >= 1) rr.store(N);
  }
  if (tid == 0) {
    ms.nb = 0;
    ms.flags = 0;
    ms.bad = 0;
  }
  __syncthreads();

  // ---- root phases, chunk by chunk ----
  u64 m = m0;
  u32 s = s0;
  bool root_changed = false;
  u64 bytes = 0;   // algorithmic bytes, as the chunks' single inserts count them
  constexpr u64 e = sizeof(Ent);
  const u32 nch = (n + K - 1) / K;
  for (u32 c = 0; c < nch; ++c) {
    const u32 nc = (n - c * K) < (u32)K ? (n - c * K) : (u32)K;
    load_n<T>(A, keys + (u64)c * K, nc);
    lds_t<Ent>* const xs = block_sort<K, T, Ent>(A, B, (int)nc);
    lds_t<Ent>* const xo = xs == A ? B : A;
    const u32 tot = nc + s;
    // merged = merge(sorted chunk, partial buffer): first K -> C, rest -> xo
    merge_split<E, T>(xs, (int)nc, P, (int)s, K, sink(C), sink(xo));
    __syncthreads();
    lds_t<Ent>* const oN = N;
    lds_t<Ent>* const oP = P;
    lds_t<Ent>* const oC = C;
    if (tot < (u32)K) {
      // the partial buffer keeps everything; Property 3 against the root
      bytes += e * 2 * tot + (m >= 1 ? 2 * e * K : 0);
      if (m >= 1 && !ent_le((Ent)oN[K - 1], (Ent)oC[0])) {
        merge_split<E, T>(oN, K, oC, (int)tot, K, sink(xs), sink(xo));
        root_changed = true;
        N = xs; P = xo;
        A = oN; B = oP; C = oC;
      } else {
        P = oC;
        A = oP; B = xs; C = xo;
      }
      s = tot;
    } else {
      // a full batch in C; the rest (in xo) is the new partial buffer
      res.flags |= F_FULL;
      const u32 rest = tot - K;
      m += 1;
      const u32 t = bitrev_pos((u32)m);
      bytes += e * (tot + rest) + e * (2ull * K * level_of(t) + K);
      if (t == 1) {
        // the heap had no node: the batch is the root
        root_changed = true;
        N = oC; P = xo;
        A = oN; B = oP; C = xs;
      } else {
        Ent* slot = slot_ptr<K, Ent>(H, m);
        if (ent_le((Ent)oN[K - 1], (Ent)oC[0])) {
          store_node<K, T, Ent>(slot, oC);   // the root keeps its entries
          P = xo;
          A = oP; B = xs; C = oC;
        } else if (ent_le((Ent)oC[K - 1], (Ent)oN[0])) {
          store_node<K, T, Ent>(slot, oN);   // swap: the batch is the new root
          root_changed = true;
          N = oC; P = xo;
          A = oN; B = oP; C = xs;
        } else {
          merge_split<E, T>(oN, K, oC, K, K, sink(xs), HeapSink<Ent>(slot, K * sizeof(Ent)));
          root_changed = true;
          N = xs; P = xo;
          A = oN; B = oP; C = oC;
        }
        if (tid == 0) {
          const u64 old = xchg_relaxed(H.locks + m, lockword(ST_TARGET, ticket));
          if (lw_state(old) != ST_AVAIL && lw_state(old) != ST_REMOVED) ms.bad = 1;
          const u32 j = ms.nb++;
          ms.tgt[j] = t;
          ms.tpos[j] = (u32)m;
          ms.lvl[j] = (u32)level_of(t);
          ms.alive[j] = 1;
        }
      }
      s = rest;
    }
    __syncthreads();   // every read of the buffers freed above is done
  }

  // ---- write back, lock the root's children on the paths, release ----
  if (root_changed) store_node<K, T, Ent>(slot_ptr<K, Ent>(H, 1), N);
  store_heap_n<K, T, Ent>(pb_ptr<Ent>(H), P, s);
  const u32 nb = ms.nb;
  auto own = [&](u32 v) -> bool {
    const u64 p = bitrev_pos(v);
    return p > m0 && p <= m;
  };
  if (tid == 0) {
    u32 nh = 0;
    for (u32 j = 0; j < nb; ++j) {
      if (ms.lvl[j] < 2) continue;
      const u32 v = ms.tgt[j] >> (ms.lvl[j] - 1);
      bool seen = false;
      for (u32 q = 0; q < nh; ++q) seen |= (ms.held[0][q] & ~MH_OWN) == v;
      if (!seen) ms.held[0][nh++] = v | (own(v) ? MH_OWN : 0u);
    }
    ms.nheld[0] = nh;
  }
  __syncthreads();
  if (tid < 64) {
    const bool ok = mh_lock_nodes(H, ms.held[0], ms.nheld[0], ticket, ctl);
    if (tid == 0) {
      if (ms.bad) raise_error(ctl, ERR_STATE);
      sh.ok = (ok && !ms.bad) ? 1u : 0u;
    }
  }
  __syncthreads();
  if (!sh.ok) { res.ok = false; return res; }
  publish();
  if (tid == 0) {
    release_root_at<Stamp>(meta, ticket, m, s, sh);
    // targets on the first level are final, unless a later carry passes them
    for (u32 j = 0; j < nb; ++j) {
      if (ms.lvl[j] != 1) continue;
      bool path = false;
      for (u32 q = 0; q < ms.nheld[0]; ++q) path |= (ms.held[0][q] & ~MH_OWN) == ms.tgt[j];
      ms.alive[j] = 0;
      if (!path && mh_finalize(H, ms.tpos[j], ticket)) ms.flags |= F_HANDOFF;
    }
  }
  __syncthreads();

  // ---- descent, level by level ----
  int lv = 1, cur = 0;
  u32 maxlv = 0;
  for (u32 j = 0; j < nb; ++j) maxlv = ms.lvl[j] > maxlv ? ms.lvl[j] : maxlv;
  while (ms.nheld[cur] > 0) {
    const int nxt = cur ^ 1;
    // deleteMins that marked a travelling carry's target get it now
    if (tid < 64) {
      const bool look = (u32)tid < nb && ms.alive[tid] && ms.lvl[tid] > (u32)lv;
      bool marked = false;
      if (look) marked = lw_state(ld_relaxed(H.locks + ms.tpos[tid])) == ST_MARKED;
      if (marked) {
        st_relaxed(H.locks + ms.tpos[tid], lockword(ST_HANDED, ticket));
        ms.alive[tid] = 0;
      }
      if (__any(marked) && tid == 0) ms.flags |= F_HANDOFF;
    }
    if (tid == 0) ms.nheld[nxt] = 0;
    __syncthreads();
    const u32 nh = ms.nheld[cur];
    for (u32 h = 0; h < nh; ++h) {
      const u32 hv = ms.held[cur][h];
      const u32 v = hv & ~MH_OWN;
      if (tid == 0) {
        // carries through v, chunk order; children they need next
        u32 q = 0;
        ms.lockv[0] = ms.lockv[1] = 0;
        for (u32 j = 0; j < nb; ++j) {
          if (!ms.alive[j] || ms.lvl[j] <= (u32)lv) continue;
          if ((ms.tgt[j] >> (ms.lvl[j] - lv)) != v) continue;
          ms.cl[q++] = j;
          if (ms.lvl[j] > (u32)lv + 1) {
            const u32 u = ms.tgt[j] >> (ms.lvl[j] - lv - 1);
            const u32 uu = u | (own(u) ? MH_OWN : 0u);
            const int slot = (u & 1) ? 1 : 0;
            ms.lockv[slot] = uu;
          } else {
            // final at v's child: that child is our own target; it is also a
            // path node if a later carry passes it
            const u32 t = ms.tgt[j];
            for (u32 j2 = j + 1; j2 < nb; ++j2) {
              if (ms.alive[j2] && ms.lvl[j2] > (u32)lv + 1 &&
                  (ms.tgt[j2] >> (ms.lvl[j2] - lv - 1)) == t)
                ms.lockv[(t & 1) ? 1 : 0] = t | MH_OWN;
            }
          }
        }
        ms.ncl = q;
      }
      __syncthreads();
      const u32 ncl = ms.ncl;
      if (ncl == 0) {
        // every carry through v was handed over: release v unchanged
        if (tid == 0) {
          if (hv & MH_OWN) {
            if (mh_finalize(H, bitrev_pos(v), ticket)) ms.flags |= F_HANDOFF;
          } else {
            unlock(lock_ptr(H, v));
          }
        }
        __syncthreads();
        continue;
      }
      // node v and the first carry in one round trip
      lds_t<Ent>* Nn = lds;
      lds_t<Ent>* Fc = lds + K;
      lds_t<Ent>* Sp = lds + 2 * K;
      Ent* vptr = node_ptr<K, Ent>(H, v);
      {
        NodeRegs<K, T, Ent> nr, cr;
        nr.load(vptr);
        cr.load(slot_ptr<K, Ent>(H, ms.tpos[ms.cl[0]]));
        nr.store(Nn);
        cr.store(Fc);
      }
      __syncthreads();
      bool changed = false;
      for (u32 q = 0; q < ncl; ++q) {
        const u32 j = ms.cl[q];
        Ent* cslot = slot_ptr<K, Ent>(H, ms.tpos[j]);
        if (q > 0) {
          NodeRegs<K, T, Ent> cr;
          cr.load(cslot);
          cr.store(Fc);
          __syncthreads();
        }
        if (ent_le((Ent)Nn[K - 1], (Ent)Fc[0])) {
          // the node keeps its entries; the carry goes on unchanged
        } else if (ent_le((Ent)Fc[K - 1], (Ent)Nn[0])) {
          store_node<K, T, Ent>(cslot, Nn);   // swap
          lds_t<Ent>* x = Nn; Nn = Fc; Fc = x;
          changed = true;
        } else {
          merge_split<E, T>(Nn, K, Fc, K, K, sink(Sp), HeapSink<Ent>(cslot, K * sizeof(Ent)));
          lds_t<Ent>* x = Nn; Nn = Sp; Sp = x;
          changed = true;
        }
        __syncthreads();
      }
      // the children the carries need next, before v is released
      if (tid < 64) {
        const u32 w0 = ms.lockv[0], w1 = ms.lockv[1];
        const u32 mine = tid == 0 ? w0 : w1;
        const bool act = tid < 2 && mine != 0 && !(mine & MH_OWN);
        u64* w = act ? lock_ptr(H, mine & ~MH_OWN) : nullptr;
        int r = 0;
        bool ok = true;
        if (__any(act)) ok = lock_lanes(w, LM_PATH, ticket, act, r, ctl);
        const bool allok = __all(ok);
        if (tid == 0) {
          sh.ok = allok ? 1u : 0u;
          if (allok) {
            u32 hn = ms.nheld[nxt];
            if (w0) ms.held[nxt][hn++] = w0;
            if (w1) ms.held[nxt][hn++] = w1;
            ms.nheld[nxt] = hn;
          }
        }
      }
      __syncthreads();
      if (!sh.ok) { res.ok = false; return res; }
      if (changed) store_node<K, T, Ent>(vptr, Nn);
      publish();
      if (tid == 0) {
        if (hv & MH_OWN) {
          if (mh_finalize(H, bitrev_pos(v), ticket)) ms.flags |= F_HANDOFF;
        } else {
          unlock(lock_ptr(H, v));
        }
        // carries final at v's children: release their targets (those that
        // later carries pass stay held as path nodes of the next level)
        for (u32 q = 0; q < ncl; ++q) {
          const u32 j = ms.cl[q];
          if (ms.lvl[j] != (u32)lv + 1) continue;
          ms.alive[j] = 0;
          const u32 t = ms.tgt[j];
          const bool path = ms.lockv[(t & 1) ? 1 : 0] == (t | MH_OWN);
          if (!path && mh_finalize(H, ms.tpos[j], ticket)) ms.flags |= F_HANDOFF;
        }
      }
      __syncthreads();
    }
    cur = nxt;
    ++lv;
  }
  res.flags |= ms.flags;
  res.levels = maxlv;
  sh.mbytes = bytes;
  return res;
}

}  // namespace gh
