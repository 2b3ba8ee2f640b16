// gh_kernels.hip -- kernels of the generalized heap for one node capacity
// and entry width: the persistent operation loop with whole-root deleteMins,
// the knapsack driver, and (8-byte entries) the SSSP driver.  Compiled once
// per supported k and width with -DGH_K=<k> -DGH_ENT_BYTES=<8|16>; each
// object exports gh::launch_ops_k<k, Ent>() and gh::launch_knap_k<k, Ent>(),
// the 8-byte objects also gh::launch_sssp_k<k>().
#include "gh_kops.h"
#include "gh_private.h"

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
// 0/1 knapsack by best-first branch and bound on the heap (the application
// of Sec. 5.7.2).  One heap per instance; a workgroup claims an instance,
// pushes the root node, and repeats: deleteMin(K) the most promising nodes,
// expand those whose bound still exceeds the best value found, insert their
// promising children.  Items are sorted by value/weight descending.
//   bound(level, V, W): V plus the items from `level` on while they fit plus
//   the fitting fraction of the next one, in fixed point with scale 2^16
//   (floored, so never below the true bound);
//   node  = level << 56 | V << 28 | W  (the node pool, 8 bytes a node);
//   entry: the smallest entry is the node with the largest bound (KnapKey).
// ---------------------------------------------------------------------------
constexpr u32 KN_MAXN = 255;
constexpr u64 KN_VW_LIMIT = 1ull << 28;   // V and W fields of a pool node

// Heap entry of a search node with fixed-point bound b and pool index id.
template <class Ent>
struct KnapKey;
// 8 bytes: (2^35 - 1 - b) << 29 | id; b needs the instance's values to sum
// below 2^18 (b < 2^34), ids stay below 2^29.
template <>
struct KnapKey<u64> {
  static constexpr u64 KEYMAX = (1ull << 35) - 1;
  static constexpr u32 IDBITS = 29;
  static constexpr u64 VSUM_LIMIT = 1ull << 18;
  static constexpr u64 ID_LIMIT = 1ull << IDBITS;
  __device__ static u64 make(u64 b, u64 id) { return ((KEYMAX - b) << IDBITS) | id; }
  __device__ static u64 bound(u64 e) { return KEYMAX - (e >> IDBITS); }
  __device__ static u64 id(u64 e) { return e & (ID_LIMIT - 1); }
  // the smallest entry whose bound is <= best_fp
  __device__ static u64 cut(u64 best_fp) { return (KEYMAX - best_fp) << IDBITS; }
};
// 16 bytes: the key word is -b as a signed 64-bit fixed-point number, biased
// by 2^63 so that it orders as unsigned; the id word holds the pool index.
// Values are limited only by the pool node's 28-bit fields.
template <>
struct KnapKey<e128> {
  static constexpr u64 SIGN = 1ull << 63;
  static constexpr u64 VSUM_LIMIT = KN_VW_LIMIT;
  static constexpr u64 ID_LIMIT = 1ull << 32;
  __device__ static e128 make(u64 b, u64 id) {
    e128 e;
    e.x = (0ull - b) ^ SIGN;
    e.y = id;
    return e;
  }
  __device__ static u64 bound(e128 e) { return 0ull - (e.x ^ SIGN); }
  __device__ static u64 id(e128 e) { return e.y & 0xFFFFFFFFull; }
  __device__ static e128 cut(u64 best_fp) {
    e128 e;
    e.x = (0ull - best_fp) ^ SIGN;
    e.y = 0;
    return e;
  }
};

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
  u64 popped_total;     // entries taken from the heap by the search
  u64 hsize;            // entries in the heap
  u64 gc_best;          // incumbent at the last garbage collection
  u64 gc_dropped;       // entries the collections removed
  u64 alg_bytes;        // algorithmic bytes of the instance's heap operations
  u32 gdead;            // nodes found dead by a collection
  u32 gkept;            // entries of a drained batch below the cut
  u32 gc_runs;
  u32 n;
  u32 cnt;              // children produced in this round
  u32 popped;
  u32 inst;
  u32 overflow;
  u32 refused;
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

// Garbage collection of the instance's own heap (Sec. 5.7.2: nodes whose
// bound cannot beat the incumbent leave the heap while the search runs).
// The heap belongs to this workgroup alone.  Every entry below the cut is
// kept: the collection takes the heap's batches in order with deleteMin
// (ascending, so the kept entries come first) into the free node slots
// after the heap until a batch reaches the cut, empties the heap, and lays
// the kept entries out again as a bulk build (Sec. 3.1), which is the
// layout a filter of the same heap at the same cut gives.  It runs only when
// nodes whose first entry is already dead (their subtrees are all dead)
// hold at least a quarter of the heap, and when the staged batches fit the
// heap's free slots.  Returns false after a failed heap operation.
template <int K, int T, class Ent>
__device__ __forceinline__ bool knap_collect(const HeapDesc& H, PrivState& st, u64& ticket, u32& ops,
                                             lds_t<Ent>* L, OpShared& sh, KnapShared& ks) {
  typedef KnapKey<Ent> KK;
  const int tid = threadIdx.x;
  const Ent cut = KK::cut(ks.best << 16);
  if (tid == 0) ks.gdead = 0;
  const u64 m = st.m;
  // the earlier operations' node stores are complete, and every wave has
  // evaluated the caller's condition, which reads gc_best: it may change
  // only after this barrier, or a late wave would skip the collection that
  // the others run and the waves would meet at each other's barriers
  publish();
  if (tid == 0) ks.gc_best = ks.best;
  const lds_t<Ent>* root = priv_pair<K, Ent>(L, st.pq);
  for (u64 p = tid + 1; p <= m; p += T) {
    const Ent e = p == 1 ? (Ent)root[0] : gptr(slot_ptr<K, Ent>(H, p))[0];
    if (!ent_lt(e, cut)) atomicAdd(&ks.gdead, 1u);
  }
  __syncthreads();
  const u64 total = m * K + st.s;
  const u64 dead_nodes = ks.gdead;
  // the drain writes at most ceil(kept / K) + 1 batches, kept <= total - dead_nodes * K
  if (dead_nodes == 0 || 4 * dead_nodes * K < total || m + (m - dead_nodes) + 2 > H.max_nodes)
    return true;
  Ent* stage = slot_ptr<K, Ent>(H, m + 1);
  u64 staged = 0;
  for (;;) {
    const OpResult r = priv_delete<K, T, Ent>(H, L, st, stage + staged, sh);
    ++ticket;
    ++ops;
    if (tid == 0) {
      ks.gkept = 0;
      ks.alg_bytes += op_alg_bytes<K, Ent>(1, r, sh.s);
    }
    __syncthreads();
    if (r.count == 0) break;
    u32 mine = 0;
    for (u32 e = tid; e < r.count; e += T)
      if (ent_lt(gptr(stage + staged)[e], cut)) ++mine;
    if (mine) atomicAdd(&ks.gkept, mine);
    __syncthreads();
    const u32 kept = ks.gkept;
    staged += kept;
    if (kept < r.count) break;
  }
  priv_discard(st);
  ++ticket;
  ++ops;
  priv_build_from<K, T, Ent>(H, L, st, stage, staged);
  ++ticket;
  ++ops;
  if (tid == 0) {
    ks.gc_dropped += ks.hsize - staged;
    ks.hsize = staged;
    ++ks.gc_runs;
    ks.alg_bytes += 2 * staged * sizeof(Ent);   // the kept entries read and laid out
  }
  __syncthreads();
  return true;
}

template <int K, int T, class Ent>
__global__ __launch_bounds__(T) void k_knap(const HeapDesc* __restrict__ descs, u32 ninst,
                                            const u32* __restrict__ item_off,
                                            const u32* __restrict__ nitems,
                                            const u64* __restrict__ caps,
                                            const u32* __restrict__ wts,
                                            const u32* __restrict__ vals, u64* __restrict__ pool,
                                            u64 pool_per_inst, Ent* __restrict__ scratch,
                                            gh_knapres* __restrict__ res, u32 gc_min,
                                            Ctl* __restrict__ ctl) {
  typedef KnapKey<Ent> KK;
  __shared__ __align__(16) Ent lds[priv_lds_entries<K, T, Ent>()];
  lds_t<Ent>* const L = (lds_t<Ent>*)lds;
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
    Ent* out = scratch + (u64)inst * 3 * K;   // K popped entries, then 2K children
    Ent* kids = out + K;
    const u64 id_limit = pool_per_inst < KK::ID_LIMIT ? pool_per_inst : KK::ID_LIMIT;
    // stage the instance; one the entry cannot encode is refused
    const u32 n = nitems[inst];
    const u32 base = item_off[inst];
    if (tid == 0) {
      ks.refused = n > KN_MAXN || caps[inst] >= KN_VW_LIMIT ? 1u : 0u;
      ks.n = n;
    }
    __syncthreads();
    if (!ks.refused)
      for (u32 j = tid; j < n; j += T) {
        ks.w[j] = wts[base + j];
        ks.v[j] = vals[base + j];
      }
    if (tid == 0) {
      ks.cap = caps[inst];
      ks.explored = 0;
      ks.created = 0;
      ks.popped_total = 0;
      ks.overflow = 0;
      ks.hsize = 0;
      ks.gc_dropped = 0;
      ks.gc_runs = 0;
      ks.alg_bytes = 0;
    }
    __syncthreads();
    if (tid == 0 && !ks.refused) {
      ks.pw[0] = 0;
      ks.pv[0] = 0;
      for (u32 j = 0; j < n; ++j) {
        ks.pw[j + 1] = ks.pw[j] + ks.w[j];
        ks.pv[j + 1] = ks.pv[j] + ks.v[j];
      }
      if (ks.pv[n] >= KK::VSUM_LIMIT) ks.refused = 1;
    }
    __syncthreads();
    if (ks.refused) {
      if (tid == 0) {
        note_error(ctl, ERR_INVAL);
        gh_knapres o{};
        o.flags = 0x20u;
        res[inst] = o;
      }
      __syncthreads();
      continue;
    }
    if (tid == 0) {
      // greedy incumbent: items in ratio order while they fit
      u64 W = 0, V = 0;
      for (u32 j = 0; j < n; ++j)
        if (W + ks.w[j] <= ks.cap) {
          W += ks.w[j];
          V += ks.v[j];
        }
      ks.best = V;
      ks.gc_best = V;
      // the root node
      const u64 b = kn_bound(ks, 0, 0, 0);
      ipool[0] = 0;
      kids[0] = KK::make(b, 0);
      ks.pool_next = 1;
      ks.cnt = (b > (V << 16)) ? 1u : 0u;
      ks.created = ks.cnt;
    }
    __syncthreads();
    u32 ops = 0;
    bool ok = true;
    // the instance's heap is this workgroup's alone: it runs without locks,
    // root and partial buffer in LDS (gh_private.h)
    PrivState st;
    priv_begin<K, T, Ent>(H, L, st, sh);
    for (;;) {
      // push this round's children (at most 2K: two inserts of K sorted
      // entries)
      const u32 c = ks.cnt;
      for (u32 j = 0; j < c; j += K) {
        const u32 nn = c - j < (u32)K ? c - j : (u32)K;
        load_n<T>(L + 4 * K, kids + j, nn);
        const lds_t<Ent>* xs = block_sort<K, T, Ent>(L + 4 * K, L + 5 * K, (int)nn);
        OpResult r = priv_insert<K, T, Ent>(H, L, st, xs, nn, sh, ctl);
        ++ticket;
        ++ops;
        if (tid == 0) {
          if (!(r.flags & F_REJECT)) ks.hsize += nn;
          ks.alg_bytes += op_alg_bytes<K, Ent>(0, r, sh.s);
        }
        __syncthreads();
      }
      if (gc_min != 0 && ks.hsize >= gc_min && ks.gc_best != ks.best)
        knap_collect<K, T, Ent>(H, st, ticket, ops, L, sh, ks);
      // take the most promising nodes
      OpResult r = priv_delete<K, T, Ent>(H, L, st, out, sh);
      ++ticket;
      ++ops;
      if (tid == 0) {
        ks.popped_total += r.count;
        ks.hsize -= r.count;
        ks.alg_bytes += op_alg_bytes<K, Ent>(1, r, sh.s);
      }
      __syncthreads();
      if (!r.ok || r.count == 0) break;
      // best-first stopping rule: the batch's first entry has the largest
      // bound left in the heap; if it cannot beat the incumbent, nothing
      // left can, and the rest of the heap is dropped unread
      if (KK::bound(out[0]) <= (ks.best << 16)) {
        priv_discard(st);
        ++ticket;
        ++ops;
        break;
      }
      if (tid == 0) {
        ks.cnt = 0;
        ks.popped = r.count;
      }
      __syncthreads();
      // expand
      const u32 popped = r.count;
      for (u32 e = tid; e < popped; e += T) {
        const Ent ent = out[e];
        const u64 id = KK::id(ent);
        const u64 b = KK::bound(ent);
        if (b <= (__hip_atomic_load(&ks.best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) << 16))
          continue;   // cannot beat the incumbent any more
        const u64 node = ipool[id];
        const u32 level = (u32)(node >> 56);
        const u64 V = (node >> 28) & (KN_VW_LIMIT - 1);
        const u64 W = node & (KN_VW_LIMIT - 1);
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
          // the child that takes the item has the parent's bound: the item
          // fits, so the greedy fill from the next level with the smaller
          // capacity stops at the same critical item with the same
          // remainder, and the entry holds the bound exactly
          cb[nc] = b;
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
          if (nid >= id_limit) {
            atomicOr(&ks.overflow, 1u);
            continue;
          }
          ipool[nid] = cand[q];
          kids[slot] = KK::make(cb[q], nid);
        }
      }
      __syncthreads();
      if (tid == 0) {
        u32 c2 = ks.cnt;
        if (ks.overflow) {
          // children beyond the pool were dropped; keep the ones written
          const u64 room = id_limit > ks.pool_next ? id_limit - ks.pool_next : 0;
          if ((u64)c2 > room) c2 = (u32)room;
          ks.cnt = c2;
        }
        ks.pool_next += c2;
        ks.created += c2;
      }
      // pool writes are read back by other threads after later barriers
      __syncthreads();
    }
    // the heap's state back to its memory (empty after the last operation)
    priv_end<K, T, Ent>(H, L, st, ticket);
    if (tid == 0) {
      gh_knapres o;
      o.best = ks.best;
      o.explored = ks.explored;
      o.created = ks.created;
      o.popped = ks.popped_total;
      o.gc_dropped = ks.gc_dropped;
      o.alg_bytes = ks.alg_bytes;
      o.ops = ops;
      o.flags = (ok ? 1u : 0u) | (ks.overflow ? 0x40u : 0u);
      o.gc_runs = ks.gc_runs;
      o.reserved = 0;
      res[inst] = o;
    }
    __syncthreads();
  }
}

template <int K, int T, class Ent>
static hipError_t launch_knap_t(const KnapArgs& a) {
  hipLaunchKernelGGL((k_knap<K, T, Ent>), dim3(a.workgroups), dim3(T), 0, a.stream, a.descs,
                     a.ninst, a.item_off, a.n, a.cap, a.w, a.v, a.pool, a.pool_per_inst,
                     reinterpret_cast<Ent*>(a.scratch), a.res, a.gc_min, a.ctl);
  return hipGetLastError();
}

template <>
hipError_t launch_knap_k<GH_K, GH_ENT>(const KnapArgs& a) {
  constexpr int K = GH_K;
  switch (a.threads) {
#define GH_CASE(TT)                                                        \
  case TT:                                                                 \
    if constexpr (shape_ok(K, TT)) return launch_knap_t<K, TT, GH_ENT>(a); \
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

#if GH_ENT_BYTES == 8
// ---------------------------------------------------------------------------
// Single-source shortest paths with the heap as a shared priority queue (the
// application of Sec. 5.7.1), lazy deletion: entries are dist << 32 | vertex;
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
  u64 popped = 0, stale = 0, pushed = 0, ops = 0, heap_t = 0, relax_t = 0, rounds = 0, alg = 0;
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
      r = op_delete<K, T, u64>(H, s_ticket, out, (u32)K, L, sh, ctl);
      ++ops;
      alg += op_alg_bytes<K, u64>(1, r, sh.s);
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
      const OpResult ri = op_insert<K, T, u64>(H, s_ticket, mine + j, nn, L, sh, ctl);
      ++ops;
      alg += op_alg_bytes<K, u64>(0, ri, sh.s);
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
    atomicAdd(reinterpret_cast<unsigned long long*>(&stats->alg_bytes), (unsigned long long)alg);
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

#endif  // GH_ENT_BYTES == 8

#ifdef GH_PHASE_TRACE
template <>
hipError_t phase_trace_k<GH_K, GH_ENT>(uint32_t* host, u64 words) {
  if (!host) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(gh_phase_trace));
    if (e != hipSuccess) return e;
    return hipMemset(p, 0, sizeof(gh_phase_trace));
  }
  return hipMemcpyFromSymbol(host, HIP_SYMBOL(gh_phase_trace), words * sizeof(uint32_t), 0,
                             hipMemcpyDeviceToHost);
}
#endif

template <>
hipError_t launch_ops_k<GH_K, GH_ENT>(const LaunchArgs& a) {
  return launch_kops_shape<GH_K, FORM_WHOLE, GH_ENT>(a);
}

}  // namespace gh
