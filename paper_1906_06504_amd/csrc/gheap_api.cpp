// gheap_api.cpp -- host side of libgheap.so: arena layout, handle
// management, launches, graphs and error reporting for the C ABI declared in
// include/gheap.h.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "gh_launch.h"
#ifdef GH_PHASE_TRACE
#include "../../include/gheap_trace.h"
#endif

using namespace gh;

namespace gh {
hipError_t launch_init(HeapDesc* descs_dev, const HeapDesc* descs_host, u32 nheaps, Ctl* ctl,
                       u64 timeout_ticks, hipStream_t st);
hipError_t launch_prep(const HeapDesc* descs, u32 nheaps, Ctl* ctl, hipStream_t st);
hipError_t launch_serve_reset(ServeHead* head, hipStream_t st);
hipError_t launch_build(const HeapDesc* d, const void* keys, u64 n, u32 ewords, Ctl* ctl,
                        hipStream_t st);
hipError_t launch_sssp_init(const HeapDesc* descs, SsspState* st, u32* dist, u32 V, u32 src,
                            u64* push, gh_ssspstats* stats, hipStream_t stream);
hipError_t launch_sssp_fini(const HeapDesc* descs, const SsspState* st, gh_ssspstats* stats,
                            hipStream_t stream);
}  // namespace gh

struct gh_heap {
  u32 k;
  u32 ebytes;                      // entry bytes: 8 (GH_U32_ID) or 16 (GH_I64_ID)
  u32 nheaps;
  hipStream_t stream;
  unsigned char* arena;
  u64 arena_bytes;
  Ctl* ctl;                        // device
  SsspState* sssp;                 // device
  HeapDesc* descs;                 // device
  std::vector<HeapDesc> host_descs;
  std::vector<u64> max_keys;
  u64 size0;                       // host-tracked entry count of heap 0
  bool size0_known;
  int sticky;                      // last device error seen by the host
  u32 clock_mhz;
  int device;                      // HIP device current at creation
};

namespace {

constexpr u64 ALIGN = 256;
inline u64 align_up(u64 x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

bool k_supported(u32 k) {
  return k == 32 || k == 64 || k == 128 || k == 256 || k == 512 || k == 1024;
}

// Workgroup size per node capacity when the caller gives none: measured on
// insert-all-then-drain workloads (2^22-2^24 keys, 64 operations in flight)
// and, for k = 1024, on the mixed insert/deleteMin workload (1024 threads 8 %
// faster than 512 there, 1 % on insert-then-drain).
u32 default_threads(u32 k) {
  switch (k) {
    case 32: return 64;
    case 64: return 128;
    case 128: return 128;
    case 256: return 512;
    case 512: return 512;
    default: return 1024;
  }
}

// The served form's slots: at k = 256 (256 heaps, 2048 slots) 256 threads
// give 3 % less saturated throughput than 128 but 14-22 % lower p50/p99
// request latency under Poisson load, and 512 lose 39 % of the throughput;
// smaller workgroups keep more slots resident.
u32 serve_default_threads(u32 k) { return k <= 128 ? default_threads(k) : 256; }

u64 max_nodes_for(u64 max_keys, u32 k) { return max_keys / k + 1; }

// Entry bytes of a key type, 0 if unknown.
u32 entry_bytes(int keytype) {
  return keytype == GH_U32_ID ? 8u : (keytype == GH_I64_ID ? 16u : 0u);
}

struct Layout {
  u64 ctl_off, sssp_off, desc_off, total;
  std::vector<u64> meta_off, pb_off, lock_off, node_off, max_nodes;
};

// Heaps per set.  With at most 2^30 nodes of at most 1024 entries a heap,
// every arena offset fits in 64 bits.
constexpr u32 MAX_HEAPS = 1u << 20;

bool make_layout(u32 k, u32 eb, u32 nheaps, const u64* max_keys, u64 each, Layout& L) {
  if (nheaps == 0 || nheaps > MAX_HEAPS || (eb != 8 && eb != 16)) return false;
  L.ctl_off = 0;
  L.sssp_off = align_up(sizeof(Ctl));
  L.desc_off = align_up(L.sssp_off + sizeof(SsspState));
  u64 off = align_up(L.desc_off + (u64)nheaps * sizeof(HeapDesc));
  L.meta_off.resize(nheaps);
  L.pb_off.resize(nheaps);
  L.lock_off.resize(nheaps);
  L.node_off.resize(nheaps);
  L.max_nodes.resize(nheaps);
  for (u32 i = 0; i < nheaps; ++i) {
    u64 mk = max_keys ? max_keys[i] : each;
    u64 mn = max_nodes_for(mk, k);
    if (mn >= RW_M_MASK) return false;
    L.max_nodes[i] = mn;
    L.meta_off[i] = off;
    off = align_up(off + sizeof(HeapMeta));
    L.pb_off[i] = off;
    off = align_up(off + (u64)k * eb);
    L.lock_off[i] = off;
    off = align_up(off + (mn + 1) * 8);
    L.node_off[i] = off;
    off = align_up(off + mn * (u64)k * eb);
  }
  L.total = off;
  return true;
}

int from_status(u32 st) {
  switch (st) {
    case 0: return GH_OK;
    case ERR_INVAL: return GH_EINVAL;
    case ERR_NOMEM: return GH_ENOMEM;
    case ERR_TIMEOUT: return GH_ETIMEDOUT;
    default: return GH_ESTATE;
  }
}

// Per (k, entry width) kernels: F<K, Ent>::run(args) for the set's shape.
template <template <int, class> class F, class A>
hipError_t by_shape(const gh_heap* h, const A& a) {
  if (h->ebytes == 16) {
    switch (h->k) {
      case 32: return F<32, e128>::run(a);
      case 64: return F<64, e128>::run(a);
      case 128: return F<128, e128>::run(a);
      case 256: return F<256, e128>::run(a);
      case 512: return F<512, e128>::run(a);
      case 1024: return F<1024, e128>::run(a);
      default: return hipErrorInvalidValue;
    }
  }
  switch (h->k) {
    case 32: return F<32, u64>::run(a);
    case 64: return F<64, u64>::run(a);
    case 128: return F<128, u64>::run(a);
    case 256: return F<256, u64>::run(a);
    case 512: return F<512, u64>::run(a);
    case 1024: return F<1024, u64>::run(a);
    default: return hipErrorInvalidValue;
  }
}
template <int K, class Ent>
struct ServeF {
  static hipError_t run(const ServeArgs& a) { return launch_serve_k<K, Ent>(a); }
};
template <int K, class Ent>
struct KnapF {
  static hipError_t run(const KnapArgs& a) { return launch_knap_k<K, Ent>(a); }
};
template <int K, class Ent>
struct OpsF {
  static hipError_t run(const LaunchArgs& a) {
    switch (a.form) {
      case 1: return launch_ops_var_k<K, Ent>(a);
      case 2: return launch_ops_bu_k<K, Ent>(a);
      case 3: return launch_private_k<K, Ent>(a);
      default: return launch_ops_k<K, Ent>(a);
    }
  }
};

hipError_t launch_serve(const gh_heap* h, const ServeArgs& a) { return by_shape<ServeF>(h, a); }

hipError_t launch_sssp(const gh_heap* h, const SsspArgs& a) {
  switch (h->k) {
    case 32: return launch_sssp_k<32>(a);
    case 64: return launch_sssp_k<64>(a);
    case 128: return launch_sssp_k<128>(a);
    case 256: return launch_sssp_k<256>(a);
    case 512: return launch_sssp_k<512>(a);
    case 1024: return launch_sssp_k<1024>(a);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_knap(const gh_heap* h, const KnapArgs& a) { return by_shape<KnapF>(h, a); }

struct ServeLayout {
  u64 head, heaps, next, left, queue, qreq, total;
};

ServeLayout serve_layout(u32 nheaps, u32 nreq, u64 max_ops) {
  ServeLayout L;
  u64 off = 0;
  L.head = off;
  off = align_up(off + sizeof(ServeHead));
  L.heaps = off;
  off = align_up(off + (u64)nheaps * sizeof(HeapSched));
  L.next = off;
  off = align_up(off + (u64)nreq * 4);
  L.left = off;
  off = align_up(off + (u64)nreq * 4);
  L.queue = off;
  off = align_up(off + max_ops * sizeof(gh_op));
  L.qreq = off;
  off = align_up(off + max_ops * 4);
  L.total = off;
  return L;
}

hipError_t launch_ops(const gh_heap* h, const LaunchArgs& a) { return by_shape<OpsF>(h, a); }

u32 clock_mhz_of_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 100;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return 100;
  return (u32)(khz / 1000);
}

u64 watchdog_ticks(u32 clock_mhz) {
  u64 ms = 5000;
  if (const char* e = std::getenv("GHEAP_WATCHDOG_MS")) {
    long long v = std::atoll(e);
    if (v > 0) ms = (u64)v;
  }
  return ms * 1000ull * clock_mhz;
}

// Launch the prep kernel (ticket bases, claim counter, start clock) and the
// operation loop on the set's stream.
int run_ops(gh_heap* h, const gh_op* d_ops, u32 nops, const OpParams& p, const void* d_in,
            void* d_out, u32* d_counts, gh_logrec* d_log, const gh_tuning* t) {
  if (nops == 0) return GH_OK;
  if (nops > RW_TICKET_MASK) return GH_EINVAL;   // tickets of one submission fit 24 bits
  u32 threads = (t && t->threads) ? t->threads : default_threads(h->k);
  if (!heap_supported_shape(h->k, threads)) return GH_EINVAL;
  u32 wg = (t && t->workgroups) ? t->workgroups : 256;
  if (wg > nops) wg = nops;
  if (wg == 0) wg = 1;
  const u32 fl = t ? t->flags : 0u;
  if ((fl & GH_TUNE_BOTTOM_UP) && (fl & (GH_TUNE_VARIABLE_DELETE | GH_TUNE_MULTI_INSERT)))
    return GH_EINVAL;   // bottom-up inserts run in submissions of inserts of up to k entries
  if (launch_prep(h->descs, h->nheaps, h->ctl, h->stream) != hipSuccess) return GH_EDEVICE;
  LaunchArgs a{};
  a.descs = h->descs;
  a.ops = d_ops;
  a.nops = nops;
  a.direct = p;
  a.direct.clock_mhz = h->clock_mhz;
  a.direct.nheaps = h->nheaps;
  a.in = static_cast<const u64*>(d_in);
  a.out = static_cast<u64*>(d_out);
  a.counts = d_counts;
  a.log = d_log;
  a.ctl = h->ctl;
  a.workgroups = wg;
  a.threads = threads;
  a.form = (fl & GH_TUNE_BOTTOM_UP) ? 2u
                                    : ((fl & (GH_TUNE_VARIABLE_DELETE | GH_TUNE_MULTI_INSERT)) ? 1u
                                                                                              : 0u);
  // one workgroup, whole-root operations: one operation in flight, so the
  // heaps are private to it and run without locks
  if (a.form == 0 && wg == 1 && !(fl & GH_TUNE_SHARED_ROOT)) a.form = 3;
  a.stream = h->stream;
  if (launch_ops(h, a) != hipSuccess) return GH_EDEVICE;
  return GH_OK;
}

int refresh_status(gh_heap* h) {
  if (hipStreamSynchronize(h->stream) != hipSuccess) return GH_EDEVICE;
  u32 st = 0;
  if (hipMemcpy(&st, &h->ctl->status, sizeof(u32), hipMemcpyDeviceToHost) != hipSuccess)
    return GH_EDEVICE;
  int rc = from_status(st);
  if (rc != GH_OK) h->sticky = rc;
  return h->sticky;
}

}  // namespace

extern "C" {

uint64_t heap_arena_bytes(uint32_t k, int keytype, uint32_t nheaps, const uint64_t* max_keys,
                          uint64_t max_keys_each) {
  if (!k_supported(k) || nheaps == 0 || entry_bytes(keytype) == 0) return 0;
  Layout L;
  if (!make_layout(k, entry_bytes(keytype), nheaps, max_keys, max_keys_each, L)) return 0;
  return L.total;
}

uint32_t heap_insert_max(uint32_t k) {
  return k_supported(k) ? (uint32_t)multi_max_batches((int)k) * k : 0u;
}

int heap_supported_shape(uint32_t k, uint32_t threads) {
  return k_supported(k) && shape_ok((int)k, (int)threads) ? 1 : 0;
}

int heap_create_many(gh_heap_t* out, uint32_t k, int keytype, uint32_t nheaps,
                     const uint64_t* max_keys, void* d_arena, uint64_t arena_bytes,
                     void* stream) {
  const u32 eb = entry_bytes(keytype);
  if (!out || !d_arena || !max_keys || nheaps == 0 || !k_supported(k) || eb == 0)
    return GH_EINVAL;
  if ((reinterpret_cast<uintptr_t>(d_arena) & (ALIGN - 1)) != 0) return GH_EINVAL;
  Layout L;
  if (!make_layout(k, eb, nheaps, max_keys, 0, L)) return GH_EINVAL;
  if (arena_bytes < L.total) return GH_ENOMEM;
  gh_heap* h = new (std::nothrow) gh_heap();
  if (!h) return GH_ENOMEM;
  h->k = k;
  h->ebytes = eb;
  h->nheaps = nheaps;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  h->arena = reinterpret_cast<unsigned char*>(d_arena);
  h->arena_bytes = arena_bytes;
  h->ctl = reinterpret_cast<Ctl*>(h->arena + L.ctl_off);
  h->sssp = reinterpret_cast<SsspState*>(h->arena + L.sssp_off);
  h->descs = reinterpret_cast<HeapDesc*>(h->arena + L.desc_off);
  h->max_keys.assign(max_keys, max_keys + nheaps);
  h->size0 = 0;
  h->size0_known = true;
  h->sticky = GH_OK;
  h->clock_mhz = clock_mhz_of_device();
  h->device = 0;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return GH_EDEVICE;
  }
  // the no-allocation filter's workspace on this device (a failed lookup
  // is reported by heap_filter_noalloc, which tries again)
  (void)filter_scratch_init(h->device);
  h->host_descs.resize(nheaps);
  for (u32 i = 0; i < nheaps; ++i) {
    HeapDesc& d = h->host_descs[i];
    std::memset(&d, 0, sizeof(d));
    d.meta = reinterpret_cast<HeapMeta*>(h->arena + L.meta_off[i]);
    d.pb = reinterpret_cast<u64*>(h->arena + L.pb_off[i]);
    d.locks = reinterpret_cast<u64*>(h->arena + L.lock_off[i]);
    d.nodes = reinterpret_cast<u64*>(h->arena + L.node_off[i]);
    d.max_nodes = (u32)L.max_nodes[i];
    d.k = k;
    d.max_keys = max_keys[i];
    d.ewords = eb / 8;
  }
  if (launch_init(h->descs, h->host_descs.data(), nheaps, h->ctl, watchdog_ticks(h->clock_mhz),
                  h->stream) != hipSuccess) {
    delete h;
    return GH_EDEVICE;
  }
  *out = h;
  return GH_OK;
}

int heap_create(gh_heap_t* out, uint32_t k, uint64_t max_keys, int keytype, void* d_arena,
                uint64_t arena_bytes, void* stream) {
  return heap_create_many(out, k, keytype, 1, &max_keys, d_arena, arena_bytes, stream);
}

int heap_insert(gh_heap_t h, const void* d_keys, uint64_t n) {
  if (!h) return GH_EINVAL;
  if (h->sticky != GH_OK) return h->sticky;
  if (n == 0) return GH_OK;
  if (!d_keys) return GH_EINVAL;
  if (!h->size0_known) {
    uint64_t sz = 0;
    int rc = heap_size(h, 0, &sz);
    if (rc != GH_OK) return rc;
  }
  if (h->size0 > h->max_keys[0] || n > h->max_keys[0] - h->size0) return GH_ENOMEM;
  // operations of k entries in the whole-root kernel (their descents run on
  // several workgroups at once, which beats one root hold per 4096 entries)
  const u64 nops = n / h->k + (n % h->k != 0 ? 1 : 0);
  if (nops > 0xFFFFFFFFull) return GH_EINVAL;
  OpParams p{GH_OP_INSERT, 0, n, 0, 0};
  gh_tuning t{(u32)(nops < 64 ? nops : 64), 0, 0};
  int rc = run_ops(h, nullptr, (u32)nops, p, d_keys, nullptr, nullptr, nullptr, &t);
  if (rc == GH_OK) h->size0 += n;
  return rc;
}

int heap_build(gh_heap_t h, uint32_t i, const void* d_sorted, uint64_t n) {
  if (!h) return GH_EINVAL;
  if (h->sticky != GH_OK) return h->sticky;
  if (i >= h->nheaps) return GH_EINVAL;
  if (n == 0) return GH_OK;
  if (!d_sorted) return GH_EINVAL;
  if (n > h->max_keys[i]) return GH_ENOMEM;
  if (i == 0) h->size0_known = false;
  if (launch_build(h->descs + i, d_sorted, n, h->ebytes / 8, h->ctl, h->stream) != hipSuccess)
    return GH_EDEVICE;
  return GH_OK;
}

uint64_t heap_filter_workspace_bytes(gh_heap_t h, uint32_t i) {
  if (!h || i >= h->nheaps) return 0;
  return filter_workspace_bytes(h->host_descs[i].max_nodes, h->k, h->ebytes);
}

int heap_filter(gh_heap_t h, uint32_t i, uint64_t bound, void* d_work, uint64_t work_bytes,
                uint64_t* d_kept) {
  if (!h || i >= h->nheaps || !d_work) return GH_EINVAL;
  if (h->sticky != GH_OK) return h->sticky;
  if ((reinterpret_cast<uintptr_t>(d_work) & (ALIGN - 1)) != 0) return GH_EINVAL;
  if (work_bytes < filter_workspace_bytes(h->host_descs[i].max_nodes, h->k, h->ebytes))
    return GH_EINVAL;
  if (i == 0) h->size0_known = false;
  if (launch_filter(h->descs + i, h->host_descs[i].max_nodes, h->k, h->ebytes, bound, d_work,
                    d_kept, h->stream) != hipSuccess)
    return GH_EDEVICE;
  return GH_OK;
}

int heap_filter_noalloc(gh_heap_t h, uint32_t i, uint64_t bound, uint64_t* d_kept) {
  if (!h || i >= h->nheaps) return GH_EINVAL;
  if (h->sticky != GH_OK) return h->sticky;
  if (filter_workspace_bytes(h->host_descs[i].max_nodes, h->k, h->ebytes) >
      GH_FILTER_NOALLOC_MAX_BYTES)
    return GH_ENOMEM;
  void* work = filter_scratch(h->device);
  if (!work) {
    if (filter_scratch_init(h->device) != hipSuccess) return GH_EDEVICE;
    work = filter_scratch(h->device);
    if (!work) return GH_EDEVICE;
  }
  if (i == 0) h->size0_known = false;
  if (launch_filter(h->descs + i, h->host_descs[i].max_nodes, h->k, h->ebytes, bound, work,
                    d_kept, h->stream) != hipSuccess)
    return GH_EDEVICE;
  return GH_OK;
}

int heap_delete_min(gh_heap_t h, void* d_out, uint32_t c, uint32_t* d_count) {
  if (!h || !d_out || !d_count || c == 0 || c > h->k) return GH_EINVAL;
  if (h->sticky != GH_OK) return h->sticky;
  OpParams p{GH_OP_DELETE_MIN, 0, c, 0, 0};
  gh_tuning t{1, 0, c < h->k ? GH_TUNE_VARIABLE_DELETE : 0u};
  int rc = run_ops(h, nullptr, 1, p, nullptr, d_out, d_count, nullptr, &t);
  if (rc == GH_OK && h->size0_known) h->size0 -= (h->size0 < c ? h->size0 : c);
  return rc;
}

int heap_submit(gh_heap_t h, const gh_op* d_ops, uint32_t nops, const void* d_in, void* d_out,
                uint32_t* d_counts, gh_logrec* d_log, const gh_tuning* tuning) {
  if (!h) return GH_EINVAL;
  if (h->sticky != GH_OK) return h->sticky;
  if (nops == 0) return GH_OK;
  if (!d_ops) return GH_EINVAL;
  h->size0_known = false;
  OpParams p{GH_OP_INSERT, 0, 0, 0, 0};
  return run_ops(h, d_ops, nops, p, d_in, d_out, d_counts, d_log, tuning);
}

int heap_submit_graph(gh_heap_t h, const gh_op* d_ops, uint32_t nops, const void* d_in,
                      void* d_out, uint32_t* d_counts, gh_logrec* d_log,
                      const gh_tuning* tuning, void** graph_out) {
  if (!h || !graph_out || !d_ops || nops == 0) return GH_EINVAL;
  if (h->sticky != GH_OK) return h->sticky;
  if (h->stream == nullptr) return GH_EINVAL;  // the legacy stream cannot be captured
  h->size0_known = false;
  if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return GH_EDEVICE;
  OpParams p{GH_OP_INSERT, 0, 0, 0, 0};
  int rc = run_ops(h, d_ops, nops, p, d_in, d_out, d_counts, d_log, tuning);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->stream, &g);
  if (rc != GH_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess || !g) return GH_EDEVICE;
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return GH_EDEVICE;
  *graph_out = reinterpret_cast<void*>(ex);
  return GH_OK;
}

int heap_graph_launch(gh_heap_t h, void* graph) {
  if (!h || !graph) return GH_EINVAL;
  if (h->sticky != GH_OK) return h->sticky;
  h->size0_known = false;
  if (hipGraphLaunch(reinterpret_cast<hipGraphExec_t>(graph), h->stream) != hipSuccess)
    return GH_EDEVICE;
  return GH_OK;
}

int heap_graph_destroy(void* graph) {
  if (!graph) return GH_EINVAL;
  return hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(graph)) == hipSuccess ? GH_OK
                                                                                     : GH_EDEVICE;
}

uint64_t heap_serve_workspace_bytes(uint32_t nheaps, uint32_t nreq, uint64_t max_ops) {
  if (nheaps == 0 || nheaps > MAX_HEAPS || max_ops == 0 || max_ops > RW_TICKET_MASK) return 0;
  return serve_layout(nheaps, nreq, max_ops).total;
}

int heap_serve(gh_heap_t h, const gh_op* d_reqs, uint32_t nreq, const void* d_in, void* d_out,
               gh_reqrec* d_recs, void* d_work, uint64_t work_bytes, uint64_t max_ops,
               const gh_tuning* t) {
  if (!h) return GH_EINVAL;
  if (h->sticky != GH_OK) return h->sticky;
  if (nreq == 0) return GH_OK;
  if (!d_reqs || !d_recs || !d_work || max_ops == 0 || max_ops > RW_TICKET_MASK) return GH_EINVAL;
  if ((reinterpret_cast<uintptr_t>(d_work) & (ALIGN - 1)) != 0) return GH_EINVAL;
  const ServeLayout L = serve_layout(h->nheaps, nreq, max_ops);
  if (work_bytes < L.total) return GH_ENOMEM;
  u32 threads = (t && t->threads) ? t->threads : serve_default_threads(h->k);
  if (!heap_supported_shape(h->k, threads)) return GH_EINVAL;
  u32 wg = (t && t->workgroups) ? t->workgroups : 512;
  // the scheduler keeps 32 bytes per heap and 8 per thread in LDS next to
  // the k-entry buffers
  if ((u64)h->nheaps * 32 + (u64)threads * 8 + (u64)h->k * 5 * h->ebytes + 1024 > 65536)
    return GH_EINVAL;
  h->size0_known = false;
  unsigned char* base = reinterpret_cast<unsigned char*>(d_work);
  ServeArgs a{};
  a.descs = h->descs;
  a.nheaps = h->nheaps;
  a.reqs = d_reqs;
  a.nreq = nreq;
  a.in = static_cast<const u64*>(d_in);
  a.out = static_cast<u64*>(d_out);
  a.recs = d_recs;
  a.w.head = reinterpret_cast<ServeHead*>(base + L.head);
  a.w.heaps = reinterpret_cast<HeapSched*>(base + L.heaps);
  a.w.next = reinterpret_cast<u32*>(base + L.next);
  a.w.left = reinterpret_cast<u32*>(base + L.left);
  a.w.queue = reinterpret_cast<gh_op*>(base + L.queue);
  a.w.qreq = reinterpret_cast<u32*>(base + L.qreq);
  a.w.max_ops = max_ops;
  a.w.ins_max = (t && (t->flags & GH_TUNE_MULTI_INSERT)) ? heap_insert_max(h->k) : h->k;
  a.ctl = h->ctl;
  a.clock_mhz = h->clock_mhz;
  a.workgroups = wg;
  a.threads = threads;
  a.stream = h->stream;
  if (launch_prep(h->descs, h->nheaps, h->ctl, h->stream) != hipSuccess) return GH_EDEVICE;
  if (launch_serve_reset(a.w.head, h->stream) != hipSuccess) return GH_EDEVICE;
  if (launch_serve(h, a) != hipSuccess) return GH_EDEVICE;
  return GH_OK;
}

int heap_knapsack(gh_heap_t h, uint32_t ninst, const uint32_t* d_item_off, const uint32_t* d_n,
                  const uint64_t* d_cap, const uint32_t* d_w, const uint32_t* d_v,
                  uint64_t* d_pool, uint64_t pool_per_inst, void* d_scratch, gh_knapres* d_res,
                  uint32_t gc_min, const gh_tuning* t) {
  if (!h) return GH_EINVAL;
  if (h->sticky != GH_OK) return h->sticky;
  if (ninst == 0) return GH_OK;
  if (ninst > h->nheaps || !d_item_off || !d_n || !d_cap || !d_w || !d_v || !d_pool ||
      !d_scratch || !d_res || pool_per_inst == 0 ||
      pool_per_inst >= (h->ebytes == 8 ? (1ull << 29) : (1ull << 32)))
    return GH_EINVAL;
  for (u32 i = 0; i < ninst; ++i)
    if (h->max_keys[i] < pool_per_inst) return GH_ENOMEM;
  u32 threads = (t && t->threads) ? t->threads : default_threads(h->k);
  if (!heap_supported_shape(h->k, threads)) return GH_EINVAL;
  u32 wg = (t && t->workgroups) ? t->workgroups : (ninst < 1024 ? ninst : 1024);
  h->size0_known = false;
  KnapArgs a{};
  a.descs = h->descs;
  a.ninst = ninst;
  a.item_off = d_item_off;
  a.n = d_n;
  a.cap = d_cap;
  a.w = d_w;
  a.v = d_v;
  a.pool = d_pool;
  a.pool_per_inst = pool_per_inst;
  a.scratch = d_scratch;
  a.gc_min = gc_min;
  a.res = d_res;
  a.ctl = h->ctl;
  a.workgroups = wg;
  a.threads = threads;
  a.stream = h->stream;
  if (launch_prep(h->descs, h->nheaps, h->ctl, h->stream) != hipSuccess) return GH_EDEVICE;
  if (launch_knap(h, a) != hipSuccess) return GH_EDEVICE;
  return GH_OK;
}

int heap_sssp(gh_heap_t h, uint32_t V, const uint32_t* d_rowptr, const uint32_t* d_col,
              const uint32_t* d_w, uint32_t src, uint32_t* d_dist, uint64_t* d_push,
              uint64_t push_per_wg, gh_ssspstats* d_stats, const gh_tuning* t,
              const gh_sssptrace* trace) {
  if (!h) return GH_EINVAL;
  if (h->sticky != GH_OK) return h->sticky;
  if (V == 0 || src >= V || !d_rowptr || !d_col || !d_w || !d_dist || !d_push || !d_stats ||
      push_per_wg == 0 || h->ebytes != 8)
    return GH_EINVAL;
  if (trace && (!trace->d_ops || !trace->d_keys)) return GH_EINVAL;
  u32 threads = (t && t->threads) ? t->threads : default_threads(h->k);
  if (!heap_supported_shape(h->k, threads)) return GH_EINVAL;
  u32 wg = (t && t->workgroups) ? t->workgroups : 256;
  h->size0_known = false;
  // prep (ticket base), init, the source's insert (ticket base), the run
  if (launch_prep(h->descs, h->nheaps, h->ctl, h->stream) != hipSuccess) return GH_EDEVICE;
  if (launch_sssp_init(h->descs, h->sssp, d_dist, V, src, d_push, d_stats, h->stream) !=
      hipSuccess)
    return GH_EDEVICE;
  LaunchArgs la{};
  la.descs = h->descs;
  la.ops = nullptr;
  la.nops = 1;
  la.direct = OpParams{GH_OP_INSERT, h->clock_mhz, 1, h->nheaps, 0};
  la.in = d_push;
  la.out = nullptr;
  la.counts = nullptr;
  la.log = nullptr;
  la.ctl = h->ctl;
  la.workgroups = 1;
  la.threads = threads;
  la.form = 0;
  la.stream = h->stream;
  if (launch_ops(h, la) != hipSuccess) return GH_EDEVICE;
  SsspArgs a{};
  a.descs = h->descs;
  a.V = V;
  a.rowptr = d_rowptr;
  a.col = d_col;
  a.w = d_w;
  a.src = src;
  a.dist = d_dist;
  a.push = d_push;
  a.push_per_wg = push_per_wg;
  a.stats = d_stats;
  a.st = h->sssp;
  a.trace = trace ? *trace : gh_sssptrace{nullptr, 0, nullptr, 0};
  a.ctl = h->ctl;
  a.workgroups = wg;
  a.threads = threads;
  a.stream = h->stream;
  if (launch_sssp(h, a) != hipSuccess) return GH_EDEVICE;
  if (launch_sssp_fini(h->descs, h->sssp, d_stats, h->stream) != hipSuccess) return GH_EDEVICE;
  return GH_OK;
}

int heap_sync(gh_heap_t h) {
  if (!h) return GH_EINVAL;
  return refresh_status(h);
}

int heap_size(gh_heap_t h, uint32_t i, uint64_t* out_host) {
  if (!h || !out_host || i >= h->nheaps) return GH_EINVAL;
  int rc = refresh_status(h);
  if (rc == GH_EDEVICE) return rc;
  u64 w = 0;
  const HeapDesc& d = h->host_descs[i];
  if (hipMemcpy(&w, &d.meta->root, sizeof(w), hipMemcpyDeviceToHost) != hipSuccess)
    return GH_EDEVICE;
  *out_host = rw_m(w) * h->k + rw_s(w);
  if (i == 0 && rc == GH_OK) {
    h->size0 = *out_host;
    h->size0_known = true;
  }
  return rc;
}

int heap_read_state(gh_heap_t h, uint32_t i, uint64_t* meta_host, void* nodes_host,
                    void* pb_host) {
  if (!h || !meta_host || i >= h->nheaps) return GH_EINVAL;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return GH_EDEVICE;
  const HeapDesc& d = h->host_descs[i];
  HeapMeta m;
  if (hipMemcpy(&m, d.meta, sizeof(m), hipMemcpyDeviceToHost) != hipSuccess) return GH_EDEVICE;
  const u64 mm = rw_m(m.root), ss = rw_s(m.root);
  meta_host[0] = mm;
  meta_host[1] = ss;
  meta_host[2] = m.base + ((rw_ticket(m.root) - m.base) & RW_TICKET_MASK);
  meta_host[3] = d.max_nodes;
  if (nodes_host &&
      hipMemcpy(nodes_host, d.nodes, (u64)d.max_nodes * h->k * h->ebytes, hipMemcpyDeviceToHost) !=
          hipSuccess)
    return GH_EDEVICE;
  if (pb_host && ss > 0 &&
      hipMemcpy(pb_host, d.pb, ss * h->ebytes, hipMemcpyDeviceToHost) != hipSuccess)
    return GH_EDEVICE;
  return GH_OK;
}

int heap_destroy(gh_heap_t h) {
  if (!h) return GH_EINVAL;
  int rc = refresh_status(h);
  delete h;
  return rc;
}

const char* heap_strerror(int code) {
  switch (code) {
    case GH_OK: return "success";
    case GH_EINVAL: return "invalid argument";
    case GH_ENOMEM: return "out of heap capacity or arena space";
    case GH_ETIMEDOUT: return "a device lock wait exceeded the watchdog limit";
    case GH_EDEVICE: return "HIP runtime error";
    case GH_ESTATE: return "heap left inconsistent by an earlier error";
    default: return "unknown error";
  }
}

uint64_t heap_clock_hz(void) { return (uint64_t)clock_mhz_of_device() * 1000000ull; }

#ifdef GH_PHASE_TRACE
int gheap_phase_trace(gh_heap_t h, uint32_t* host_out, uint64_t words) {
  if (!h || words > (1ull << 22)) return GH_EINVAL;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return GH_EDEVICE;
  hipError_t e = hipErrorInvalidValue;
#define GH_TRACE_CASE(KK)                                                          \
  case KK:                                                                          \
    e = h->ebytes == 16 ? phase_trace_k<KK, e128>(host_out, words)                  \
                        : phase_trace_k<KK, u64>(host_out, words);                  \
    break;
  switch (h->k) {
    GH_TRACE_CASE(32)
    GH_TRACE_CASE(64)
    GH_TRACE_CASE(128)
    GH_TRACE_CASE(256)
    GH_TRACE_CASE(512)
    GH_TRACE_CASE(1024)
    default:
      return GH_EINVAL;
  }
#undef GH_TRACE_CASE
  return e == hipSuccess ? GH_OK : GH_EDEVICE;
}
#endif

}  // extern "C"
