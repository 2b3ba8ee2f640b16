// gh_private.h -- the generalized heap when one workgroup owns it.
//
// A heap that only one workgroup touches has one operation in flight, so the
// concurrency control of Sec. 3.3 (root ticket, node locks, the TARGET /
// MARKED hand-over, device-scope transfers) has nothing to order.  Here the
// owning workgroup keeps the root node and the partial buffer in its LDS,
// takes no lock, and reaches the other nodes with cached loads and stores
// that are coherent within the workgroup (one L1 serves all its waves).
// The operations are the paper's sequential ones: the top-down insert with
// its partial-buffer rules (Sec. 3.2.2, 3.3.2) and the deleteMin with the
// refill from the last node and the sift-down (Sec. 3.2.1), each
// MergeAndSort with the shortcuts of Sec. 4.3; nodes are placed in the
// bit-reversal order (Sec. 4.3).  One operation at a time this is the same
// layout the shared-root loop leaves with one workgroup, and the oracle's.
//
// Ordering rules: node stores of one operation are never loaded again by the
// same operation (each node is visited once), so an operation's first node
// load waits for the workgroup's earlier stores (publish) and the others do
// not; a deleteMin ends with a publish so that its output is readable by
// every thread.  The state (m, s, which LDS pair holds root and partial
// buffer) is held in registers, identical in every thread; priv_begin reads
// it from the heap's memory and priv_end writes it back with the root word
// (the ticket after the last operation run), so that the shared-root loop
// can continue the heap in a later launch.
//
// LDS: pair 0 = root [0, K) and partial buffer [K, 2K), pair 1 = [2K, 4K)
// (root followed by partial buffer is one sorted run, Property 3, which the
// insert's one-pass merge reads), four work buffers [4K, 8K), and, where it
// fits, a path buffer of priv_path_nodes() nodes from 8K on.
//
// The insert's descent in one merge: by Property 1 the nodes on the path
// from level 1 down to the target, read top-down, are one sorted run, and
// keeping at each level the K smallest of node and carry (Sec. 3.2.2) leaves
// exactly the consecutive K-entry chunks of merge(path, carry) on the path
// and the last chunk at the target.  So a group of path nodes is loaded in
// one round trip and merged with the carry in one pass; the group's last K
// outputs are the carry for the next group.  The nodes before the carry's
// smallest entry keep their batches and are not rewritten (the shortcut of
// Sec. 4.3); the layout is the level-by-level one.
#pragma once
#include "gh_launch.h"
#include "gh_ops.h"

namespace gh {

struct PrivState {
  u64 m;      // nodes
  u32 s;      // partial-buffer entries
  bool pq;    // the root and partial buffer are in pair 1
  u64 served; // tickets the root word shows served since the submission's base
};

template <int K, class Ent>
__device__ __forceinline__ lds_t<Ent>* priv_pair(lds_t<Ent>* lds, bool p) {
  return p ? lds + 2 * K : lds;
}

// Path nodes an insert loads in one round trip: at most priv_path_pieces()
// 16-byte pieces a thread (registers held until the pieces are in LDS), and
// at most 72 KB of LDS in all (eight K-entry buffers and the path buffer, so
// that two 512-thread workgroups share a compute unit).  Below two the
// descent goes level by level.
template <class Ent>
__host__ __device__ constexpr int priv_path_pieces() {
  return 2;
}
template <int K, int T, class Ent>
__host__ __device__ constexpr int priv_path_nodes() {
  constexpr int node_bytes = K * (int)sizeof(Ent);
  constexpr int by_regs = priv_path_pieces<Ent>() * T * 16 / node_bytes;
  constexpr int left = 72 * 1024 - 8 * node_bytes;
  constexpr int by_lds = left > 0 ? left / node_bytes : 0;
  constexpr int p = by_regs < by_lds ? by_regs : by_lds;
  return p > 16 ? 16 : p;
}
template <int K, int T, class Ent>
__host__ __device__ constexpr int priv_lds_entries() {
  return 8 * K + (priv_path_nodes<K, T, Ent>() >= 2 ? priv_path_nodes<K, T, Ent>() * K : 0);
}

// Merge output on the insert path: output chunk q of K entries is the path
// node at level level0 + q (plain stores: the heap is this workgroup's).
template <int K, class Ent>
struct PathSink {
  Ent* nodes;   // the heap's node array
  u32 t;        // the target node
  int L;        // the target's level
  int level0;   // level of output chunk 0
  __device__ __forceinline__ glob_t<Ent>* at(int off) const {
    const u32 c = t >> (L - level0 - off / K);
    return gptr(nodes + (u64)(bitrev_pos(c) - 1) * K) + off % K;
  }
  __device__ __forceinline__ void put1(int off, Ent x) const { *at(off) = x; }
  template <int E>
  __device__ __forceinline__ void put_range(int off, const Ent (&v)[E]) const {
    glob_t<Ent>* g = at(off);   // E divides K: the range stays in one node
#pragma unroll
    for (int e = 0; e < E; ++e) g[e] = v[e];
  }
};

// K entries from one LDS buffer to another, 16 bytes a lane.
template <int K, int T, class Ent>
__device__ __forceinline__ void lds_copy(lds_t<Ent>* __restrict__ dst,
                                         const lds_t<Ent>* __restrict__ src) {
  constexpr int CH = K * (int)sizeof(Ent) / 16;
  lu64x2* d = reinterpret_cast<lu64x2*>(dst);
  const lu64x2* q = reinterpret_cast<const lu64x2*>(src);
  for (int c = threadIdx.x; c < CH; c += T) d[c] = q[c];
}

// Read the heap's state: (m, s) and the tickets served since the
// submission's base from the root word, root and partial buffer into pair 0
// (device scope: earlier launches may have written them).
template <int K, int T, class Ent>
__device__ __forceinline__ void priv_begin(const HeapDesc& H, lds_t<Ent>* lds, PrivState& st,
                                           OpShared& sh) {
  if (threadIdx.x == 0) sh.word = ld_relaxed(&H.meta->root);
  __syncthreads();
  const u64 w = sh.word;
  const u64 base = *gptr(&H.meta->base);
  st.m = rw_m(w);
  st.s = (u32)rw_s(w);
  st.pq = false;
  st.served = (rw_ticket(w) - base) & RW_TICKET_MASK;
  {
    NodeRegs<K, T, Ent> rr, pr;
    if (st.m >= 1) rr.load(slot_ptr<K, Ent>(H, 1));
    pr.load(pb_ptr<Ent>(H));
    if (st.m >= 1) rr.store(lds);
    pr.store(lds + K);
  }
  __syncthreads();
}

// Write the state back: root node, partial buffer and the root word (next
// ticket `ticket`, m, s).
template <int K, int T, class Ent>
__device__ __forceinline__ void priv_end(const HeapDesc& H, lds_t<Ent>* lds, const PrivState& st,
                                         u64 ticket) {
  lds_t<Ent>* R = priv_pair<K, Ent>(lds, st.pq);
  if (st.m >= 1) store_node<K, T, Ent>(slot_ptr<K, Ent>(H, 1), R);
  store_heap_n<K, T, Ent>(pb_ptr<Ent>(H), R + K, st.s);
  publish();
  if (threadIdx.x == 0) st_relaxed(&H.meta->root, rootword(ticket, st.m, st.s));
}

// Insert n (1..K) sorted entries xs (an LDS buffer at lds + 4K or lds + 5K).
template <int K, int T, class Ent>
__device__ __forceinline__ OpResult priv_insert(const HeapDesc& H, lds_t<Ent>* lds, PrivState& st,
                                                const lds_t<Ent>* xs, u32 n, OpShared& sh,
                                                Ctl* ctl) {
  constexpr int E = (2 * K) / T >= 1 ? (2 * K) / T : 1;
  constexpr int E3a = pow2_at_least((3 * K + T - 1) / T);
  constexpr int E3 = E3a < (E > 8 ? E : 8) ? E3a : (E > 8 ? E : 8);
  const int tid = threadIdx.x;
  lds_t<Ent>* const Rc = priv_pair<K, Ent>(lds, st.pq);
  lds_t<Ent>* const Ro = priv_pair<K, Ent>(lds, !st.pq);
  lds_t<Ent>* const Pc = Rc + K;
  lds_t<Ent>* const Po = Ro + K;
  lds_t<Ent>* F = lds + 6 * K;   // the carry
  lds_t<Ent>* N = lds + 7 * K;   // the path node
  lds_t<Ent>* spare = xs == lds + 4 * K ? lds + 5 * K : lds + 4 * K;
  const u64 m = st.m;
  const u32 s = st.s;
  OpResult res{n, 0, m >= 1 ? F_ROOT : 0u, true};
  if (tid == 0) sh.s = s;
  const bool full = n + s >= (u32)K;
  if (full && m + 1 > H.max_nodes) {
    // no room for another node: reject the insert, the heap is unchanged
    if (tid == 0) note_error(ctl, ERR_NOMEM);
    res.count = 0;
    res.flags |= F_REJECT;
    __syncthreads();
    return res;
  }
  // the root phase in one merge of the batch with root ++ pb (see op_insert):
  // new root, carry and new partial buffer
  if (m >= 1) {
    if (!full)
      merge_split<E3, T>(xs, (int)n, Rc, K + (int)s, K, sink(Ro), sink(Po));
    else
      merge_split3<E3, T>(xs, (int)n, Rc, K + (int)s, K, 2 * K, sink(Ro), sink(F), sink(Po));
  } else {
    // no root: a partial batch joins the pb, a full one becomes the root
    merge_split<E, T>(xs, (int)n, Pc, (int)s, full ? K : (int)(n + s), sink(full ? Ro : Po),
                      sink(Po));
  }
  __syncthreads();
  st.pq = !st.pq;
  if (!full) {
    st.s = n + s;
    return res;
  }
  res.flags |= F_FULL;
  st.s = n + s - K;
  st.m = m + 1;
  if (m == 0) return res;   // the batch is the root
  const u32 t = bitrev_pos((u32)(m + 1));
  const int L = level_of(t);
  // the carry goes down the path to the target, MergeAndSort at every node
  // (the node keeps the K smallest); the earlier operations' stores are
  // complete before the first node is loaded
  publish();
  constexpr int PC = priv_path_nodes<K, T, Ent>();
  if constexpr (PC >= 2) {
    // groups of up to PC path nodes, each loaded in one round trip and
    // merged with the carry in one pass (see the top of this file)
    constexpr int CH = K * (int)sizeof(Ent) / 16;
    constexpr int PP = priv_path_pieces<Ent>();
    constexpr int EP = sizeof(Ent) == 16 ? 2 : 4;   // outputs a thread per merge pass
    lds_t<Ent>* const PB = lds + 8 * K;
    Ent* const nodes = reinterpret_cast<Ent*>(H.nodes);
    for (int level = 1; level < L;) {
      const int n = L - level < PC ? L - level : PC;
      {
        u64x2 v[PP];
#pragma unroll
        for (int j = 0; j < PP; ++j) {
          const int i = tid + j * T;
          if (i < n * CH) {
            const int q = i / CH;
            const u32 c = t >> (L - level - q);
            const glob_t<u64x2>* src =
                gptr(reinterpret_cast<const u64x2*>(nodes + (u64)(bitrev_pos(c) - 1) * K));
            v[j] = src[i - q * CH];
          }
        }
#pragma unroll
        for (int j = 0; j < PP; ++j) {
          const int i = tid + j * T;
          if (i < n * CH) reinterpret_cast<lu64x2*>(PB)[i] = v[j];
        }
      }
      __syncthreads();
      int keep = 0;   // leading nodes wholly below the carry keep their batches
      while (keep < n && ent_le((Ent)PB[(keep + 1) * K - 1], (Ent)F[0])) ++keep;
      if (keep < n) {
        const int na = (n - keep) * K;
        merge_split<EP, T>(PB + keep * K, na, F, K, na,
                           PathSink<K, Ent>{nodes, t, L, level + keep}, sink(spare));
        __syncthreads();
        lds_t<Ent>* x = F;
        F = spare;
        spare = x;
      }
      level += n;
    }
  } else {
  for (int level = 1; level < L; ++level) {
    Ent* cp = node_ptr<K, Ent>(H, t >> (L - level));
    {
      NodeRegs<K, T, Ent, CP_LOCAL> nr;
      nr.load(cp);
      nr.store(N);
    }
    __syncthreads();
    if (ent_le((Ent)N[K - 1], (Ent)F[0])) {
      // the node already holds the smallest: nothing moves
    } else if (ent_le((Ent)F[K - 1], (Ent)N[0])) {
      store_node<K, T, Ent, CP_LOCAL>(cp, F);   // swap
      lds_t<Ent>* x = F;
      F = N;
      N = x;
    } else {
      merge_split<E, T>(N, K, F, K, K, HeapSink<Ent, CP_LOCAL>(cp, K * sizeof(Ent)), sink(spare));
      lds_t<Ent>* x = F;
      F = spare;
      spare = x;
    }
    __syncthreads();
  }
  }
  store_node<K, T, Ent, CP_LOCAL>(node_ptr<K, Ent>(H, t), F);
  if (tid == 0) st_relaxed(lock_ptr(H, t), lockword(ST_AVAIL, 0));   // an existing node's word
  res.levels = L;
  return res;
}

// The sift-down below the root from node c (level >= 1), whose batch is in
// the work buffer `cur`; returns the levels merged.
template <int K, int T, class Ent>
__device__ __forceinline__ u32 priv_sift(const HeapDesc& H, lds_t<Ent>* work, lds_t<Ent>* cur,
                                         u32 c, u64 m2) {
  constexpr int E = (2 * K) / T >= 1 ? (2 * K) / T : 1;
  lds_t<Ent>* bufs[4];
  {
    int j = 1;
    bufs[0] = cur;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      lds_t<Ent>* b = work + q * K;
      if (b != cur) {
        if (j == 1) bufs[1] = b;
        else if (j == 2) bufs[2] = b;
        else bufs[3] = b;
        ++j;
      }
    }
  }
  u32 levels = 0;
  for (;;) {
    const u64 l = 2ull * c, r = l + 1;
    const bool hl = node_exists(l, m2), hr = node_exists(r, m2);
    lds_t<Ent>* C = bufs[0];
    lds_t<Ent>* Lb = bufs[1];
    lds_t<Ent>* Rb = bufs[2];
    {
      NodeRegs<K, T, Ent, CP_LOCAL> lc, rc;
      if (hl) lc.load(node_ptr<K, Ent>(H, (u32)l));
      if (hr) rc.load(node_ptr<K, Ent>(H, (u32)r));
      if (hl) lc.store(Lb);
      if (hr) rc.store(Rb);
    }
    __syncthreads();
    Ent* cptr = node_ptr<K, Ent>(H, c);
    const Ent lmin = hl ? (Ent)Lb[0] : ent_max<Ent>();
    const Ent rmin = hr ? (Ent)Rb[0] : ent_max<Ent>();
    const Ent cmin = ent_lt(lmin, rmin) ? lmin : rmin;
    if (ent_le((Ent)C[K - 1], cmin)) {
      // the property holds: place the batch and stop (Sec. 4.3)
      store_node<K, T, Ent, CP_LOCAL>(cptr, C);
      return levels;
    }
    lds_t<Ent>* newcur;
    u32 next;
    if (hl && hr) {
      // MergeAndSort(l, r): the K largest stay in the child whose max was
      // larger (on a tie the right child), the K smallest merge with cur
      const bool big_is_l = ent_lt((Ent)Rb[K - 1], (Ent)Lb[K - 1]);
      const u32 big = big_is_l ? (u32)l : (u32)r;
      next = big_is_l ? (u32)r : (u32)l;
      lds_t<Ent>* Bg = big_is_l ? Lb : Rb;
      lds_t<Ent>* Sm = big_is_l ? Rb : Lb;
      lds_t<Ent>* up;
      lds_t<Ent>* freeb;
      if (ent_le((Ent)Sm[K - 1], (Ent)Bg[0])) {
        up = Sm;   // the big child keeps its batch
        freeb = bufs[3];
      } else {
        merge_split<E, T>(Lb, K, Rb, K, K, sink(bufs[3]),
                          HeapSink<Ent, CP_LOCAL>(node_ptr<K, Ent>(H, big), K * sizeof(Ent)));
        __syncthreads();
        up = bufs[3];
        freeb = Lb;
      }
      if (ent_le((Ent)up[K - 1], (Ent)C[0])) {
        store_node<K, T, Ent, CP_LOCAL>(cptr, up);
        newcur = C;
      } else {
        merge_split<E, T>(C, K, up, K, K, HeapSink<Ent, CP_LOCAL>(cptr, K * sizeof(Ent)),
                          sink(freeb));
        newcur = freeb;
      }
    } else {
      // one live child x
      next = hl ? (u32)l : (u32)r;
      lds_t<Ent>* X = hl ? Lb : Rb;
      if (ent_le((Ent)X[K - 1], (Ent)C[0])) {
        store_node<K, T, Ent, CP_LOCAL>(cptr, X);
        newcur = C;
      } else {
        merge_split<E, T>(C, K, X, K, K, HeapSink<Ent, CP_LOCAL>(cptr, K * sizeof(Ent)),
                          sink(bufs[3]));
        newcur = bufs[3];
      }
    }
    __syncthreads();
    ++levels;
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
    }
    c = next;
  }
}

// deleteMin of K entries (Sec. 3.2.1): the root's entries to `out` (the
// partial buffer's when there is no node), the last node refills the root,
// the refilled root merges with the partial buffer (Property 3), and the
// sift-down restores Property 1.  Ends with the output and the node stores
// complete (publish).
template <int K, int T, class Ent>
__device__ __forceinline__ OpResult priv_delete(const HeapDesc& H, lds_t<Ent>* lds, PrivState& st,
                                                Ent* __restrict__ out, OpShared& sh) {
  constexpr int E = (2 * K) / T >= 1 ? (2 * K) / T : 1;
  const int tid = threadIdx.x;
  lds_t<Ent>* const Rc = priv_pair<K, Ent>(lds, st.pq);
  lds_t<Ent>* const Ro = priv_pair<K, Ent>(lds, !st.pq);
  lds_t<Ent>* const Pc = Rc + K;
  lds_t<Ent>* const Po = Ro + K;
  lds_t<Ent>* const Cb = lds + 4 * K;
  lds_t<Ent>* const X = lds + 5 * K;
  lds_t<Ent>* const Lb = lds + 6 * K;
  lds_t<Ent>* const Rb = lds + 7 * K;
  const u64 m = st.m;
  const u32 s = st.s;
  OpResult res{0, 0, 0, true};
  if (tid == 0) sh.s = s;
  if (m == 0) {
    // no node: the partial buffer is the whole heap
    store_n<T>(out, Pc, s);
    res.count = s;
    st.s = 0;
    publish();
    return res;
  }
  res.flags = F_ROOT;
  res.count = K;
  store_n<T>(out, Rc, K);   // the root's K entries are the answer
  if (m == 1) {
    st.m = 0;
    publish();
    return res;
  }
  res.flags |= F_REFILL;
  const u64 m2 = m - 1;
  const bool hl = node_exists(2, m2), hr = node_exists(3, m2);
  // the last node and the root's children in one round trip, after the
  // earlier operations' stores are complete
  publish();
  {
    NodeRegs<K, T, Ent, CP_LOCAL> lr, lc, rc;
    lr.load(slot_ptr<K, Ent>(H, m));
    if (hl) lc.load(slot_ptr<K, Ent>(H, 2));   // node 2 is position 2
    if (hr) rc.load(node_ptr<K, Ent>(H, 3));
    lr.store(Cb);
    if (hl) lc.store(Lb);
    if (hr) rc.store(Rb);
  }
  __syncthreads();
  // the refilled root and the partial buffer: the K smallest stay at the top
  lds_t<Ent>* Cp = Cb;
  bool tp = st.pq;
  if (s > 0 && !ent_le((Ent)Cb[K - 1], (Ent)Pc[0])) {
    merge_split<E, T>(Cb, K, Pc, (int)s, K, sink(X), sink(Po));
    __syncthreads();
    Cp = X;
    tp = !st.pq;
  }
  lds_t<Ent>* const Rt = priv_pair<K, Ent>(lds, tp);   // the new root's buffer
  lds_t<Ent>* const freeb = Cp == X ? Cb : X;
  const Ent lmin = hl ? (Ent)Lb[0] : ent_max<Ent>();
  const Ent rmin = hr ? (Ent)Rb[0] : ent_max<Ent>();
  const Ent cmin = ent_lt(lmin, rmin) ? lmin : rmin;
  u32 next = 0;
  lds_t<Ent>* cur = Cp;
  if (ent_le((Ent)Cp[K - 1], cmin)) {
    // the property holds at the root: early stop (Sec. 4.3)
    lds_copy<K, T, Ent>(Rt, Cp);
  } else if (hl && hr) {
    const bool big_is_l = ent_lt((Ent)Rb[K - 1], (Ent)Lb[K - 1]);
    const u32 big = big_is_l ? 2u : 3u;
    next = big_is_l ? 3u : 2u;
    lds_t<Ent>* Bg = big_is_l ? Lb : Rb;
    lds_t<Ent>* Sm = big_is_l ? Rb : Lb;
    lds_t<Ent>* up;
    lds_t<Ent>* nc;
    if (ent_le((Ent)Sm[K - 1], (Ent)Bg[0])) {
      up = Sm;
      nc = freeb;
    } else {
      merge_split<E, T>(Lb, K, Rb, K, K, sink(freeb),
                        HeapSink<Ent, CP_LOCAL>(node_ptr<K, Ent>(H, big), K * sizeof(Ent)));
      __syncthreads();
      up = freeb;
      nc = Lb;
    }
    if (ent_le((Ent)up[K - 1], (Ent)Cp[0])) {
      lds_copy<K, T, Ent>(Rt, up);
      cur = Cp;
    } else {
      merge_split<E, T>(Cp, K, up, K, K, sink(Rt), sink(nc));
      cur = nc;
    }
  } else {
    // one live child x: the root keeps the K smallest of the two
    next = hl ? 2u : 3u;
    lds_t<Ent>* Xc = hl ? Lb : Rb;
    if (ent_le((Ent)Xc[K - 1], (Ent)Cp[0])) {
      lds_copy<K, T, Ent>(Rt, Xc);
      cur = Cp;
    } else {
      merge_split<E, T>(Cp, K, Xc, K, K, sink(Rt), sink(freeb));
      cur = freeb;
    }
  }
  __syncthreads();
  st.pq = tp;
  st.m = m2;
  if (next != 0) res.levels = 1 + priv_sift<K, T, Ent>(H, lds + 4 * K, cur, next, m2);
  publish();
  return res;
}

// Drop every entry (op_discard).
__device__ __forceinline__ void priv_discard(PrivState& st) {
  st.m = 0;
  st.s = 0;
}

// Lay n ascending entries from src (written by this workgroup) out as the
// heap: the first floor(n / K) * K become the nodes in addition order (the
// first one the root, in LDS), the rest the partial buffer (the bulk build of
// Sec. 3.1).  For an empty heap; the nodes' lock words are cleared.
template <int K, int T, class Ent>
__device__ __forceinline__ void priv_build_from(const HeapDesc& H, lds_t<Ent>* lds, PrivState& st,
                                                const Ent* __restrict__ src, u64 n) {
  publish();   // src is complete
  const u64 m = n / K, body = m * K;
  lds_t<Ent>* R = lds;   // pair 0
  const glob_t<Ent>* gs = gptr(src);
  for (u64 i = threadIdx.x; i < n; i += T) {
    const Ent e = gs[i];
    if (i < body) {
      if (i < (u64)K) R[i] = e;
      else gptr(slot_ptr<K, Ent>(H, 1))[i] = e;
    } else {
      R[K + (i - body)] = e;
    }
  }
  for (u64 p = threadIdx.x + 1; p <= m; p += T) st_relaxed(H.locks + p, lockword(ST_AVAIL, 0));
  st.m = m;
  st.s = (u32)(n - body);
  st.pq = false;
  __syncthreads();
}

}  // namespace gh
