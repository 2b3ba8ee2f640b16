// gh_device.h -- device-side building blocks of the generalized heap:
// heap-state layout, node lock words, memory-ordering helpers, bit-reversal
// node order, and LDS-staged merge-path merge and sort for one workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gh {

typedef uint64_t u64;
typedef uint32_t u32;
typedef u64 u64x2 __attribute__((ext_vector_type(2)));

// LDS (workgroup-local) data.  Buffers in LDS are always reached through
// pointers of these types, so that every access is an LDS instruction: a
// generic pointer would make the compiler emit flat accesses, each of which
// also waits for every outstanding global memory operation.
template <class X>
using lds_t = __attribute__((address_space(3))) X;
typedef lds_t<u64> lu64;
typedef lds_t<u64x2> lu64x2;

// ---------------------------------------------------------------------------
// Entries.  Two widths, fixed per heap set and compiled separately:
//  * u64: 8 bytes, ordered as an unsigned integer (a 32-bit key above a
//    32-bit id);
//  * e128: 16 bytes, two 64-bit words ordered lexicographically, the word at
//    the lower address first (a biased signed 64-bit key, then a 32-bit id
//    and 32 zero bits).
// The all-ones value of either width is the reserved filler (never live).
// ---------------------------------------------------------------------------
typedef u64x2 e128;

constexpr u64 ENT_MAX = ~0ull;  // the 8-byte filler

__device__ __forceinline__ bool ent_lt(u64 a, u64 b) { return a < b; }
__device__ __forceinline__ bool ent_le(u64 a, u64 b) { return a <= b; }
__device__ __forceinline__ bool ent_lt(e128 a, e128 b) {
  return a.x < b.x || (a.x == b.x && a.y < b.y);
}
__device__ __forceinline__ bool ent_le(e128 a, e128 b) {
  return a.x < b.x || (a.x == b.x && a.y <= b.y);
}
template <class Ent>
__device__ __forceinline__ Ent ent_max();
template <>
__device__ __forceinline__ u64 ent_max<u64>() {
  return ~0ull;
}
template <>
__device__ __forceinline__ e128 ent_max<e128>() {
  e128 v;
  v.x = ~0ull;
  v.y = ~0ull;
  return v;
}
__device__ __forceinline__ bool ent_is_max(u64 a) { return a == ~0ull; }
__device__ __forceinline__ bool ent_is_max(e128 a) { return (a.x & a.y) == ~0ull; }

// Full batches one insert operation of the general kernels may form: such an
// operation takes up to multi_max_batches(K) * K entries (4096, or 2048 for
// K = 32) in one root hold.
__host__ __device__ constexpr int multi_max_batches(int K) {
  return (4096 / K) < 64 ? (4096 / K) : 64;
}

// ---------------------------------------------------------------------------
// Heap state in device memory
// ---------------------------------------------------------------------------

// Root metadata of one heap.  The word every waiting operation polls also
// carries the root-guarded counters, so the operation that gets the root
// learns m and s without another round trip:
//   root = (ticket allowed at the root, low 24 bits) << 40 | m << 10 | s
// (m < 2^30 nodes, s < 1024 partial-buffer entries).  `base` is the full
// ticket of seq 0 in the current submission.
struct alignas(256) HeapMeta {
  u64 root;
  u64 pad0[15];
  u64 base;
  u64 pad1[15];
};
constexpr u64 RW_TICKET_MASK = 0xFFFFFFull;
constexpr u64 RW_M_MASK = (1ull << 30) - 1;
__host__ __device__ __forceinline__ u64 rootword(u64 ticket, u64 m, u64 s) {
  return ((ticket & RW_TICKET_MASK) << 40) | ((m & RW_M_MASK) << 10) | (s & 1023);
}
__host__ __device__ __forceinline__ u64 rw_ticket(u64 w) { return w >> 40; }
__host__ __device__ __forceinline__ u64 rw_m(u64 w) { return (w >> 10) & RW_M_MASK; }
__host__ __device__ __forceinline__ u64 rw_s(u64 w) { return w & 1023; }
static_assert(sizeof(HeapMeta) == 256, "meta layout");

// Where one heap lives.  Node storage is indexed by the order in which nodes
// are added (position p >= 1 at nodes + (p-1)*k), so a heap of m nodes
// occupies the first m slots; tree navigation uses node indices (root 1,
// children 2c and 2c+1) and converts with the bit-reversal map.
struct alignas(64) HeapDesc {
  u64* nodes;         // max_nodes * k entries
  u64* locks;         // lock word per position, [0] unused, [1..max_nodes]
  u64* pb;            // partial buffer, k entries
  HeapMeta* meta;
  u32 max_nodes;
  u32 k;
  u64 max_keys;       // capacity in entries (the served form admits by it)
  u32 ewords;         // 8-byte words per entry: 1 (u64) or 2 (e128)
  u32 pad;
};
static_assert(sizeof(HeapDesc) == 64, "desc layout");

// Per-set control block.
struct alignas(256) Ctl {
  u32 next_op;        // claim counter of the running submission
  u32 pad0[31];
  u64 t0;             // device clock when the submission started
  u64 timeout_ticks;  // watchdog limit for one lock wait
  u32 status;         // sticky error code (0 = ok), first error wins
  u32 abort;          // nonzero: every workgroup leaves as soon as it can
  u32 build_ok;       // a bulk build found its heap empty
  u32 pad1[25];
};
static_assert(sizeof(Ctl) == 256, "ctl layout");

// Error codes stored in Ctl::status (negated GH_E* codes).
constexpr u32 ERR_INVAL = 1;
constexpr u32 ERR_NOMEM = 2;
constexpr u32 ERR_TIMEOUT = 3;
constexpr u32 ERR_STATE = 5;

// ---------------------------------------------------------------------------
// Node lock words: the multi-state lock of the TD-INS/TD-DEL heap (Sec. 3.3.2)
// Low 3 bits hold the state, the rest the ticket of the operation that set it.
// ---------------------------------------------------------------------------
constexpr u64 ST_AVAIL = 0;   // free
constexpr u64 ST_INUSE = 1;   // held by one operation (Lemma 1)
constexpr u64 ST_TARGET = 2;  // reserved target of an in-flight insert
constexpr u64 ST_MARKED = 3;  // a deleteMin asked that insert for its batch
constexpr u64 ST_HANDED = 4;  // the insert left its batch in the target slot
constexpr u64 ST_REMOVED = 5; // a deleteMin took this node's batch as the last node

__device__ __forceinline__ u64 lockword(u64 st, u64 ticket) { return (ticket << 3) | st; }
__device__ __forceinline__ u64 lw_state(u64 w) { return w & 7; }
__device__ __forceinline__ u64 lw_ticket(u64 w) { return w >> 3; }

// ---------------------------------------------------------------------------
// Memory ordering across the XCDs (each has its own L2).
//
// Lock words and the root word are agent-scope atomics.  Heap payload (nodes
// and the partial buffer) also moves with device-scope accesses: buffer
// loads and stores carrying the device-scope cache bit, which read from and
// write through to the point of coherence of all XCDs.  So no whole-cache
// write-back or invalidate is needed: a holder publishes with publish()
// (every wave waits until its stores are complete, then the workgroup meets
// at a barrier) and thread 0 then releases with a relaxed store; an acquirer
// waits for the lock atomic to return before any payload load is issued.
// ---------------------------------------------------------------------------
// Global memory through global-address-space pointers: global instructions
// count only against the vector memory counter, while flat ones (generic
// pointers) also hold up every later LDS wait.
template <class X>
using glob_t = __attribute__((address_space(1))) X;
typedef glob_t<u64> gu64;
typedef glob_t<u32> gu32;
template <class X>
__device__ __forceinline__ glob_t<X>* gptr(X* p) {
  return (glob_t<X>*)p;
}
template <class X>
__device__ __forceinline__ const glob_t<X>* gptr(const X* p) {
  return (const glob_t<X>*)p;
}

__device__ __forceinline__ u64 ld_relaxed(const u64* p) {
  return __hip_atomic_load(gptr(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u32 ld_relaxed32(const u32* p) {
  return __hip_atomic_load(gptr(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(u64* p, u64 v) {
  __hip_atomic_store(gptr(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas_relaxed(u64* p, u64 expect, u64 desired) {
  return __hip_atomic_compare_exchange_strong(gptr(p), &expect, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// compare-and-swap returning the previous value (== expect on success)
__device__ __forceinline__ u64 cas_old(u64* p, u64 expect, u64 desired) {
  __hip_atomic_compare_exchange_strong(gptr(p), &expect, desired, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return expect;
}
__device__ __forceinline__ u64 xchg_relaxed(u64* p, u64 v) {
  return __hip_atomic_exchange(gptr(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Acquire side: the lock atomic has returned before any later load issues.
__device__ __forceinline__ void fence_acquire() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// All threads: this workgroup's heap stores are complete at the point of
// coherence.  Afterwards thread 0 may release locks with relaxed stores.
__device__ __forceinline__ void publish() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
}

// Device-scope transfers of heap memory.  A buffer resource describes one
// region (a node or the partial buffer) whose base is the same in every
// lane; offsets are per lane, in bytes.
constexpr int CP_DEVICE = 16;   // cache-policy operand: device scope (sc1)
constexpr int CP_LOCAL = 0;     // cached; coherent within one workgroup (a
                                // heap that only that workgroup touches)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <int CP = CP_DEVICE>
struct HeapRegionT {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ HeapRegionT(const u64* base, u32 bytes) {
    const u64 a = reinterpret_cast<u64>(base);
    const u32 lo = __builtin_amdgcn_readfirstlane((u32)a);
    const u32 hi = __builtin_amdgcn_readfirstlane((u32)(a >> 32));
    r = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((u64)hi << 32) | lo), 0,
                                          bytes, 0x00020000);
  }
  __device__ __forceinline__ ulonglong2 load16(u32 off) const {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, CP);
    ulonglong2 o;
    o.x = (u64)v.x | ((u64)v.y << 32);
    o.y = (u64)v.z | ((u64)v.w << 32);
    return o;
  }
  __device__ __forceinline__ u64 load8(u32 off) const {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, CP);
    return (u64)v.x | ((u64)v.y << 32);
  }
  __device__ __forceinline__ void store16(u32 off, u64 a, u64 b) const {
    u32x4 v;
    v.x = (u32)a;
    v.y = (u32)(a >> 32);
    v.z = (u32)b;
    v.w = (u32)(b >> 32);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, CP);
  }
  __device__ __forceinline__ void store8(u32 off, u64 a) const {
    u32x2 v;
    v.x = (u32)a;
    v.y = (u32)(a >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, CP);
  }
  // one entry at byte offset off
  __device__ __forceinline__ void load_ent(u32 off, u64& e) const { e = load8(off); }
  __device__ __forceinline__ void load_ent(u32 off, e128& e) const {
    const ulonglong2 v = load16(off);
    e.x = v.x;
    e.y = v.y;
  }
  __device__ __forceinline__ void store_ent(u32 off, u64 e) const { store8(off, e); }
  __device__ __forceinline__ void store_ent(u32 off, e128 e) const { store16(off, e.x, e.y); }
};
typedef HeapRegionT<CP_DEVICE> HeapRegion;

__device__ __forceinline__ u64 now_ticks() { return wall_clock64(); }

// Sticky error: the first code wins; every waiting workgroup then leaves.
__device__ __forceinline__ void raise_error(Ctl* ctl, u32 code) {
  u32 zero = 0;
  __hip_atomic_compare_exchange_strong(&ctl->status, &zero, code, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sticky error that leaves the heap consistent: record it, keep running.
__device__ __forceinline__ void note_error(Ctl* ctl, u32 code) {
  u32 zero = 0;
  __hip_atomic_compare_exchange_strong(&ctl->status, &zero, code, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait step for thread 0: sleeps a little, checks the abort flag and
// the watchdog.  Returns false when the wait must be abandoned.
struct Waiter {
  u64 start;
  u32 iters;
  __device__ __forceinline__ Waiter() : start(0), iters(0) {}
  __device__ __forceinline__ bool step(Ctl* ctl, u32 sleep = 1) {
    ++iters;
    if ((iters & 31) == 1) {
      u64 t = now_ticks();
      if (iters == 1) start = t;
      else if (t - start > ctl->timeout_ticks) {
        raise_error(ctl, ERR_TIMEOUT);
        return false;
      }
      if (ld_relaxed32(&ctl->abort)) return false;
    }
    if (sleep <= 1) __builtin_amdgcn_s_sleep(1);
    else if (sleep <= 4) __builtin_amdgcn_s_sleep(4);
    else __builtin_amdgcn_s_sleep(16);
    return true;
  }
};

// ---------------------------------------------------------------------------
// Bit-reversal node order (Sec. 4.3).  The p-th node added (p >= 1) is on
// level l = floor(log2 p) at offset reverse_l(p - 2^l); the map is an
// involution, so the same function turns a node index into its position.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int level_of(u32 c) { return 31 - __builtin_clz(c); }
__device__ __forceinline__ u32 bitrev_pos(u32 c) {
  int l = level_of(c);
  if (l == 0) return 1;
  u32 off = c - (1u << l);
  return (1u << l) | (__builtin_bitreverse32(off) >> (32 - l));
}

// Does node index c exist in a heap of m nodes?  (c may be up to 2^32 - 1.)
__device__ __forceinline__ bool node_exists(u64 c, u64 m) {
  if (c == 0 || c > 0xFFFFFFFFull) return false;
  return (u64)bitrev_pos((u32)c) <= m;
}

// Node c's slot and the partial buffer, as arrays of entries.
template <int K, class Ent = u64>
__device__ __forceinline__ Ent* node_ptr(const HeapDesc& H, u32 c) {
  return reinterpret_cast<Ent*>(H.nodes) + (u64)(bitrev_pos(c) - 1) * K;
}
template <int K, class Ent>
__device__ __forceinline__ Ent* slot_ptr(const HeapDesc& H, u64 pos) {
  return reinterpret_cast<Ent*>(H.nodes) + (pos - 1) * (u64)K;
}
template <class Ent>
__device__ __forceinline__ Ent* pb_ptr(const HeapDesc& H) {
  return reinterpret_cast<Ent*>(H.pb);
}
__device__ __forceinline__ u64* lock_ptr(const HeapDesc& H, u32 c) {
  return H.locks + bitrev_pos(c);
}

// ---------------------------------------------------------------------------
// Coalesced node transfers between heap memory and LDS (16 bytes a lane:
// two 8-byte entries or one 16-byte entry).
// ---------------------------------------------------------------------------
template <int K, int T, class Ent = u64, int CP = CP_DEVICE>
__device__ __forceinline__ void store_node(Ent* g, const lds_t<Ent>* __restrict__ lds) {
  constexpr int CH = K * (int)sizeof(Ent) / 16;   // 16-byte chunks per node
  const HeapRegionT<CP> R(reinterpret_cast<const u64*>(g), K * sizeof(Ent));
  const lu64x2* l = reinterpret_cast<const lu64x2*>(lds);
  for (int c = threadIdx.x; c < CH; c += T) {
    const u64x2 v = l[c];
    R.store16(c * 16, v.x, v.y);
  }
}
// A node's share per thread held in registers, so that several node loads
// (and lock atomics) can be in flight before anything is written to LDS.
template <int K, int T, class Ent = u64, int CP = CP_DEVICE>
struct NodeRegs {
  static constexpr int CH = K * (int)sizeof(Ent) / 16;   // 16-byte chunks per node
  static constexpr int C = (CH + T - 1) / T;             // chunks per thread
  ulonglong2 v[C];
  __device__ __forceinline__ void load(const Ent* g) {
    const HeapRegionT<CP> R(reinterpret_cast<const u64*>(g), K * sizeof(Ent));
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int i = threadIdx.x + c * T;
      if (i < CH) v[c] = R.load16(i * 16);
    }
  }
  __device__ __forceinline__ void store(lds_t<Ent>* __restrict__ lds) const {
    lu64x2* l = reinterpret_cast<lu64x2*>(lds);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int i = threadIdx.x + c * T;
      if (i < CH) {
        u64x2 t;
        t.x = v[c].x;
        t.y = v[c].y;
        l[i] = t;
      }
    }
  }
};

// n entries, any n, one entry a lane: caller memory to LDS and back
template <int T, class Ent>
__device__ __forceinline__ void load_n(lds_t<Ent>* __restrict__ lds, const Ent* __restrict__ g,
                                       u32 n) {
  const glob_t<Ent>* gg = gptr(g);
  for (u32 i = threadIdx.x; i < n; i += T) lds[i] = gg[i];
}
template <int T, class Ent>
__device__ __forceinline__ void store_n(Ent* __restrict__ g, const lds_t<Ent>* __restrict__ lds,
                                        u32 n) {
  glob_t<Ent>* gg = gptr(g);
  for (u32 i = threadIdx.x; i < n; i += T) gg[i] = lds[i];
}
// n entries from LDS to heap memory (the partial buffer)
template <int K, int T, class Ent>
__device__ __forceinline__ void store_heap_n(Ent* g, const lds_t<Ent>* __restrict__ lds, u32 n) {
  const HeapRegion R(reinterpret_cast<const u64*>(g), K * sizeof(Ent));
  for (u32 i = threadIdx.x; i < n; i += T) R.store_ent(i * sizeof(Ent), (Ent)lds[i]);
}
// n entries from heap memory (the partial buffer) to caller memory
template <int K, int T, class Ent>
__device__ __forceinline__ void copy_heap_n(Ent* __restrict__ dst, const Ent* src, u32 n) {
  const HeapRegion R(reinterpret_cast<const u64*>(src), K * sizeof(Ent));
  glob_t<Ent>* gd = gptr(dst);
  for (u32 i = threadIdx.x; i < n; i += T) {
    Ent e;
    R.load_ent(i * sizeof(Ent), e);
    gd[i] = e;
  }
}
// n entries from heap memory (the partial buffer) to LDS
template <int K, int T, class Ent>
__device__ __forceinline__ void load_heap_n(lds_t<Ent>* __restrict__ lds, const Ent* src, u32 n,
                                            u32 first = 0) {
  const HeapRegion R(reinterpret_cast<const u64*>(src), K * sizeof(Ent));
  for (u32 i = threadIdx.x; i < n; i += T) {
    Ent e;
    R.load_ent((first + i) * sizeof(Ent), e);
    lds[i] = e;
  }
}

// ---------------------------------------------------------------------------
// Merge path (Green, McColl and Bader, "GPU merge path", cited in Sec. 4.2):
// output positions [d, d+E) of the stable merge of sorted A[0,na) and
// B[0,nb) (A first on ties), found by a binary search along the diagonal and
// a short sequential merge.  Positions past na+nb yield ENT_MAX.  (A 4-ary
// search with a register-window merge measured slower on gfx950: the merge
// is bound by dependent LDS latency, and the extra probes cost more than the
// rounds they save.)
// ---------------------------------------------------------------------------
template <int E, class Ent>
__device__ __forceinline__ void merge_path(const lds_t<Ent>* A, int na, const lds_t<Ent>* B, int nb,
                                           int d, Ent (&v)[E]) {
  const int total = na + nb;
  if (d >= total) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = ent_max<Ent>();
    return;
  }
  int lo = d > nb ? d - nb : 0;
  int hi = d < na ? d : na;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ent_le((Ent)A[mid], (Ent)B[d - 1 - mid])) lo = mid + 1;
    else hi = mid;
  }
  int i = lo, j = d - lo;
  Ent a = i < na ? (Ent)A[i] : ent_max<Ent>();
  Ent b = j < nb ? (Ent)B[j] : ent_max<Ent>();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (ent_le(a, b)) {
      v[e] = a;
      ++i;
      a = i < na ? (Ent)A[i] : ent_max<Ent>();
    } else {
      v[e] = b;
      ++j;
      b = j < nb ? (Ent)B[j] : ent_max<Ent>();
    }
  }
}

// Destinations for merge output, written E entries a thread: LDS or caller
// memory (Sink), or a region of heap memory (HeapSink, device scope).
template <class Ent = u64>
struct Sink {
  lds_t<Ent>* p;
  __device__ __forceinline__ void put1(int off, Ent x) const { p[off] = x; }
  template <int E>
  __device__ __forceinline__ void put_range(int off, const Ent (&v)[E]) const {
    lds_t<Ent>* q = p + off;
    if constexpr (sizeof(Ent) == 8 && E % 2 == 0) {
      if ((off & 1) == 0) {   // LDS buffers are 16-byte aligned
#pragma unroll
        for (int e = 0; e < E; e += 2) {
          u64x2 w;
          w.x = v[e];
          w.y = v[e + 1];
          *reinterpret_cast<lu64x2*>(q + e) = w;
        }
        return;
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) q[e] = v[e];
  }
};
template <class Ent>
__device__ __forceinline__ Sink<Ent> sink(lds_t<Ent>* p) {
  return Sink<Ent>{p};
}
template <class Ent = u64, int CP = CP_DEVICE>
struct HeapSink {
  HeapRegionT<CP> R;
  __device__ __forceinline__ HeapSink(Ent* p, u32 bytes)
      : R(reinterpret_cast<const u64*>(p), bytes) {}
  __device__ __forceinline__ void put1(int off, Ent x) const { R.store_ent(off * sizeof(Ent), x); }
  template <int E>
  __device__ __forceinline__ void put_range(int off, const Ent (&v)[E]) const {
    if constexpr (sizeof(Ent) == 8 && E % 2 == 0) {
      if ((off & 1) == 0) {
#pragma unroll
        for (int e = 0; e < E; e += 2) R.store16((off + e) * 8, v[e], v[e + 1]);
        return;
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) R.store_ent((off + e) * sizeof(Ent), v[e]);
  }
};

// Workgroup-wide MergeAndSort (Sec. 3.2.1 display equation, generalized to
// unequal sizes): the stable merge of A[0,na) and B[0,nb) is split at
// `split`; positions < split go to lo[p], the rest to hi[p - split].  Inputs
// must be in LDS and must not overlap the outputs.  No barrier inside: the
// caller synchronizes before reusing inputs or reading outputs.
template <int E, int T, class Ent, class SinkLo, class SinkHi>
__device__ __forceinline__ void merge_split(const lds_t<Ent>* A, int na, const lds_t<Ent>* B,
                                            int nb, int split, const SinkLo& lo,
                                            const SinkHi& hi) {
  const int total = na + nb;
  for (int d = threadIdx.x * E; d < total; d += T * E) {
    Ent v[E];
    merge_path<E>(A, na, B, nb, d, v);
    if (d + E <= total && d + E <= split) {
      lo.template put_range<E>(d, v);
    } else if (d + E <= total && d >= split) {
      hi.template put_range<E>(d - split, v);
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int p = d + e;
        if (p < total) {
          if (p < split) lo.put1(p, v[e]);
          else hi.put1(p - split, v[e]);
        }
      }
    }
  }
}

// The same with two split points: positions < s1 go to a[p], [s1, s2) to
// b[p - s1], the rest to c[p - s2].
template <int E, int T, class Ent, class SinkA, class SinkB, class SinkC>
__device__ __forceinline__ void merge_split3(const lds_t<Ent>* A, int na, const lds_t<Ent>* B,
                                             int nb, int s1, int s2, const SinkA& a,
                                             const SinkB& b, const SinkC& c) {
  const int total = na + nb;
  for (int d = threadIdx.x * E; d < total; d += T * E) {
    Ent v[E];
    merge_path<E>(A, na, B, nb, d, v);
    if (d + E <= total && d + E <= s1) {
      a.template put_range<E>(d, v);
    } else if (d + E <= total && d >= s1 && d + E <= s2) {
      b.template put_range<E>(d - s1, v);
    } else if (d + E <= total && d >= s2) {
      c.template put_range<E>(d - s2, v);
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int p = d + e;
        if (p < total) {
          if (p < s1) a.put1(p, v[e]);
          else if (p < s2) b.put1(p - s1, v[e]);
          else c.put1(p - s2, v[e]);
        }
      }
    }
  }
}

// Entries a thread takes in a merge of up to 3K entries in one pass: a
// power of two (even counts store 16 bytes at a time).
constexpr int pow2_at_least(int x) { return x <= 1 ? 1 : 2 * pow2_at_least((x + 1) / 2); }

// A 32-bit word from the lane whose index differs from this lane's in bit
// pattern J (a cross-lane move within the wave, in registers): distances 1
// and 2 are quad permutations, 4 a quad permutation and a half-row mirror, 8
// a rotation by 8 within each row of 16 lanes (DPP moves of the vector
// unit), 16 and 32 the row and half-wave swaps of gfx950 (permlane16_swap,
// permlane32_swap).  Every lane of the wave must take part.
template <int J>
__device__ __forceinline__ u32 lane_xor32(u32 v) {
  if constexpr (J == 1) {
    return (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // [1,0,3,2]
  } else if constexpr (J == 2) {
    return (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // [2,3,0,1]
  } else if constexpr (J == 4) {
    // [3,2,1,0] (distance 3), then the mirror within each half row (7)
    const int a = __builtin_amdgcn_update_dpp(0, (int)v, 0x1B, 0xF, 0xF, false);
    return (u32)__builtin_amdgcn_update_dpp(0, a, 0x141, 0xF, 0xF, false);
  } else if constexpr (J == 8) {
    return (u32)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (J == 16) {
    // rows of 16 swapped pairwise: the odd rows of the first result hold the
    // even rows' values, the even rows of the second the odd rows'
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (threadIdx.x & 16) ? r[0] : r[1];
  } else {
    static_assert(J == 32, "lane distances 1, 2, 4, 8, 16, 32");
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
  }
}
template <int J>
__device__ __forceinline__ u64 ent_shfl_xor(u64 x) {
  return (u64)lane_xor32<J>((u32)x) | ((u64)lane_xor32<J>((u32)(x >> 32)) << 32);
}
template <int J>
__device__ __forceinline__ e128 ent_shfl_xor(e128 x) {
  e128 r;
  r.x = ent_shfl_xor<J>((u64)x.x);
  r.y = ent_shfl_xor<J>((u64)x.y);
  return r;
}

// One compare-exchange stage of the network below: lane pairs J apart, in
// blocks of KB lanes that ascend or descend alternately.
template <int KB, int J, class Ent>
__device__ __forceinline__ Ent bitonic_stage(Ent x, int lane) {
  const Ent y = ent_shfl_xor<J>(x);
  const bool up = (lane & KB) == 0;    // this block ascends
  const bool low = (lane & J) == 0;    // this lane is the lower of the pair
  const bool take_min = low == up;
  const bool lt = ent_lt(y, x);
  return (take_min == lt) ? y : x;
}

// Bitonic sorting network over the 64 lanes of a wave, one entry a lane:
// returns this lane's entry of the ascending order (Batcher's network,
// 21 compare-exchange stages, each a cross-lane move).
template <class Ent>
__device__ __forceinline__ Ent wave_sort64(Ent x) {
  const int lane = threadIdx.x & 63;
  x = bitonic_stage<2, 1>(x, lane);
  x = bitonic_stage<4, 2>(x, lane);
  x = bitonic_stage<4, 1>(x, lane);
  x = bitonic_stage<8, 4>(x, lane);
  x = bitonic_stage<8, 2>(x, lane);
  x = bitonic_stage<8, 1>(x, lane);
  x = bitonic_stage<16, 8>(x, lane);
  x = bitonic_stage<16, 4>(x, lane);
  x = bitonic_stage<16, 2>(x, lane);
  x = bitonic_stage<16, 1>(x, lane);
  x = bitonic_stage<32, 16>(x, lane);
  x = bitonic_stage<32, 8>(x, lane);
  x = bitonic_stage<32, 4>(x, lane);
  x = bitonic_stage<32, 2>(x, lane);
  x = bitonic_stage<32, 1>(x, lane);
  x = bitonic_stage<64, 32>(x, lane);
  x = bitonic_stage<64, 16>(x, lane);
  x = bitonic_stage<64, 8>(x, lane);
  x = bitonic_stage<64, 4>(x, lane);
  x = bitonic_stage<64, 2>(x, lane);
  x = bitonic_stage<64, 1>(x, lane);
  return x;
}

// ---------------------------------------------------------------------------
// Workgroup merge sort of up to K entries in LDS (sorts the insert batch,
// Sec. 4.1): with K > T every thread sorts EPT = K / T entries in registers;
// with one entry a thread each wave sorts 64 of them with wave_sort64.  Then
// rounds of merge path double the sorted run length.  A holds the n inputs
// (padded with the filler to a power of two); returns the buffer (A or B)
// that holds the sorted result.
// ---------------------------------------------------------------------------
template <int K, int T, class Ent>
__device__ lds_t<Ent>* block_sort(lds_t<Ent>* A, lds_t<Ent>* B, int n) {
  constexpr int EPT = (K >= T) ? (K / T) : 1;
  if constexpr (EPT == 1) {
    // one entry a thread: runs of 64 sorted within each wave by a bitonic
    // network in registers (lanes past n hold the filler), then rounds of
    // merge path from runs of 64 on
    int np = 1;
    while (np < n) np <<= 1;
    const int tid = threadIdx.x;
    const int lanes = np < 64 ? 64 : np;   // whole waves
    if (tid < lanes) {
      Ent x = tid < n ? (Ent)A[tid] : ent_max<Ent>();
      x = wave_sort64(x);
      if (tid < np) A[tid] = x;
    }
    __syncthreads();
    lds_t<Ent>* src = A;
    lds_t<Ent>* dst = B;
    for (int w = 64; w < np; w <<= 1) {
      if (tid < np) {
        const int base = tid & ~(2 * w - 1);
        Ent v[1];
        merge_path<1>(src + base, w, src + base + w, w, tid - base, v);
        dst[tid] = v[0];
      }
      __syncthreads();
      lds_t<Ent>* t = src;
      src = dst;
      dst = t;
    }
    return src;
  }
  int np = EPT;
  while (np < n) np <<= 1;
  for (int i = n + threadIdx.x; i < np; i += T) A[i] = ent_max<Ent>();
  __syncthreads();
  const int active = np / EPT;
  const int tid = threadIdx.x;
  if (tid < active) {
    Ent v[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) v[e] = A[tid * EPT + e];
    // odd-even transposition sort of EPT registers
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
#pragma unroll
      for (int e = (r & 1); e + 1 < EPT; e += 2) {
        Ent x = v[e], y = v[e + 1];
        const bool o = ent_lt(x, y);
        v[e] = o ? x : y;
        v[e + 1] = o ? y : x;
      }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) A[tid * EPT + e] = v[e];
  }
  __syncthreads();
  lds_t<Ent>* src = A;
  lds_t<Ent>* dst = B;
  for (int w = EPT; w < np; w <<= 1) {
    if (tid < active) {
      int d0 = tid * EPT;
      int base = d0 & ~(2 * w - 1);
      Ent v[EPT];
      merge_path<EPT>(src + base, w, src + base + w, w, d0 - base, v);
#pragma unroll
      for (int e = 0; e < EPT; ++e) dst[d0 + e] = v[e];
    }
    __syncthreads();
    lds_t<Ent>* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

}  // namespace gh
