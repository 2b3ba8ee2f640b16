// gh_kernels.hip -- kernels of the generalized heap for one node capacity:
// the persistent operation loop with whole-root deleteMins, and the
// knapsack and SSSP drivers.  Compiled once per supported k with
// -DGH_K=<k>; each object exports gh::launch_ops_k<k>(),
// gh::launch_knap_k<k>() and gh::launch_sssp_k<k>().
#include "gh_kops.h"

#ifndef GH_K
#error "compile with -DGH_K=<node capacity>"
#endif

namespace gh {

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
  u64 popped_total;     // entries taken from the heap
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
      ks.popped_total = 0;
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
      OpResult r = op_delete<K, T>(H, ticket++, out, (u32)K, L, sh, ctl);
      ++ops;
      if (tid == 0) ks.popped_total += r.count;
      __syncthreads();
      if (!r.ok || r.count == 0) break;
      // best-first stopping rule: the batch's first entry has the largest
      // bound left in the heap; if it cannot beat the incumbent, nothing
      // left can, and the rest of the heap is dropped unread
      if (KN_KEYMAX - (out[0] >> KN_IDBITS) <= (ks.best << 16)) {
        op_discard(H, ticket++, sh, ctl);
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
      o.popped = ks.popped_total;
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
      r = op_delete<K, T>(H, s_ticket, out, (u32)K, L, sh, ctl);
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

template <>
hipError_t launch_ops_k<GH_K>(const LaunchArgs& a) {
  return launch_kops_shape<GH_K, false>(a);
}

}  // namespace gh
