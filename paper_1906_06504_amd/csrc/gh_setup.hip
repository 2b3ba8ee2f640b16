// gh_setup.hip -- arena initialization and per-submission preparation
// kernels (no heap arithmetic).
#include "gh_launch.h"

namespace gh {

// Fill every node and partial-buffer slot with the filler, every lock with
// AVAIL, and zero the metadata, for one heap per y-block row.
__global__ void k_init_heap(const HeapDesc* __restrict__ descs, u32 nheaps) {
  const u32 h = blockIdx.y;
  if (h >= nheaps) return;
  const HeapDesc d = descs[h];
  // the filler is all ones in either entry width
  const u64 n_words = (u64)d.max_nodes * d.k * d.ewords;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  const u64 start = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  for (u64 i = start; i < n_words; i += stride) d.nodes[i] = ENT_MAX;
  for (u64 i = start; i <= d.max_nodes; i += stride) d.locks[i] = 0;
  for (u64 i = start; i < (u64)d.k * d.ewords; i += stride) d.pb[i] = ENT_MAX;
  if (start < sizeof(HeapMeta) / 8) reinterpret_cast<u64*>(d.meta)[start] = 0;
}

__global__ void k_init_ctl(Ctl* ctl, u64 timeout_ticks) {
  u32* w = reinterpret_cast<u32*>(ctl);
  for (u32 i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) w[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) ctl->timeout_ticks = timeout_ticks;
}

// Before a submission: every heap's ticket base becomes its current serving
// count, the claim counter restarts, and the start clock is taken.
__global__ void k_prep(const HeapDesc* __restrict__ descs, u32 nheaps, Ctl* ctl) {
  for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nheaps; i += gridDim.x * blockDim.x) {
    // the root word keeps the low 24 bits of the next ticket; a submission
    // runs fewer than 2^24 operations, so the full ticket is recovered from
    // the previous base
    HeapMeta* m = descs[i].meta;
    const u64 b = m->base;
    m->base = b + ((rw_ticket(m->root) - b) & RW_TICKET_MASK);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->next_op = 0;
    ctl->t0 = wall_clock64();
  }
}

// Before a serving launch: empty queue, no claims, scheduler not done.
__global__ void k_serve_reset(ServeHead* head) {
  u32* w = reinterpret_cast<u32*>(head);
  for (u32 i = threadIdx.x; i < sizeof(ServeHead) / 4; i += blockDim.x) w[i] = 0;
}

hipError_t launch_serve_reset(ServeHead* head, hipStream_t st) {
  hipLaunchKernelGGL(k_serve_reset, dim3(1), dim3(64), 0, st, head);
  return hipGetLastError();
}

// Before an SSSP run: distances unreached, the source at 0, its entry ready
// in the first push slot, counters cleared, dynamic tickets after the one
// the source's insert takes.
__global__ void k_sssp_init(const HeapDesc* __restrict__ descs, SsspState* st, u32* dist, u32 V,
                            u32 src, u64* push, gh_ssspstats* stats) {
  const u64 i0 = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  for (u64 i = i0; i < V; i += (u64)gridDim.x * blockDim.x) dist[i] = i == src ? 0u : 0xFFFFFFFFu;
  if (i0 == 0) {
    st->next_ticket = descs[0].meta->base + 1;
    st->outstanding = 1;   // the source's entry
    st->trace_ops = 0;
    st->trace_keys = 0;
    st->done = 0;
    push[0] = (u64)src;   // entry (0 << 32 | src)
    u64* sw = reinterpret_cast<u64*>(stats);
    for (int j = 0; j < (int)(sizeof(gh_ssspstats) / 8); ++j) sw[j] = 0;
  }
}

hipError_t launch_sssp_init(const HeapDesc* descs, SsspState* st, u32* dist, u32 V, u32 src,
                            u64* push, gh_ssspstats* stats, hipStream_t stream) {
  u32 blocks = (V + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_sssp_init, dim3(blocks), dim3(256), 0, stream, descs, st, dist, V, src, push,
                     stats);
  return hipGetLastError();
}

// After an SSSP run: the ticket base becomes the next dynamic ticket, so the
// next submission's base is exact however many tickets the run took.
__global__ void k_sssp_fini(const HeapDesc* __restrict__ descs, const SsspState* st,
                            gh_ssspstats* stats) {
  if (threadIdx.x == 0) {
    descs[0].meta->base = st->next_ticket;
    stats->traced = st->trace_ops;
  }
}

hipError_t launch_sssp_fini(const HeapDesc* descs, const SsspState* st, gh_ssspstats* stats,
                            hipStream_t stream) {
  hipLaunchKernelGGL(k_sssp_fini, dim3(1), dim3(64), 0, stream, descs, st, stats);
  return hipGetLastError();
}

// Bulk build of one empty heap from an ascending array: entries go to the
// node slots in storage order (slot p - 1 is the p-th node added; its parent
// was added earlier) and the remainder to the partial buffer.  Three
// launches: the emptiness check, the copy, and the new root word.
__global__ void k_build_check(const HeapDesc* __restrict__ d, Ctl* ctl) {
  if (threadIdx.x == 0) {
    const u64 w = ld_relaxed(&d->meta->root);
    const bool empty = rw_m(w) == 0 && rw_s(w) == 0;
    ctl->build_ok = empty ? 1u : 0u;
    if (!empty) note_error(ctl, ERR_STATE);
  }
}

template <class Ent>
__global__ void k_build_copy(const HeapDesc* __restrict__ d, const Ent* __restrict__ keys, u64 n,
                             Ctl* ctl) {
  if (!ctl->build_ok) return;
  const HeapDesc H = *d;
  const u64 m = n / H.k, body = m * H.k;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  const u64 i0 = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  Ent* nodes = reinterpret_cast<Ent*>(H.nodes);
  Ent* pb = reinterpret_cast<Ent*>(H.pb);
  bool sorted = true;
  for (u64 i = i0; i < n; i += stride) {
    const Ent x = keys[i];
    if (i + 1 < n && ent_lt(keys[i + 1], x)) sorted = false;
    if (i < body) nodes[i] = x;
    else pb[i - body] = x;
  }
  if (!sorted) note_error(ctl, ERR_INVAL);
  for (u64 p = i0 + 1; p <= m; p += stride) H.locks[p] = 0;
}

__global__ void k_build_root(const HeapDesc* __restrict__ d, u64 n, Ctl* ctl) {
  if (threadIdx.x == 0 && ctl->build_ok) {
    const HeapDesc H = *d;
    const u64 m = n / H.k;
    const u64 w = ld_relaxed(&H.meta->root);
    st_relaxed(&H.meta->root, rootword(rw_ticket(w), m, n - m * H.k));
  }
}

hipError_t launch_build(const HeapDesc* d, const void* keys, u64 n, u32 ewords, Ctl* ctl,
                        hipStream_t st) {
  u64 blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_build_check, dim3(1), dim3(64), 0, st, d, ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ewords == 2)
    hipLaunchKernelGGL(k_build_copy<e128>, dim3((u32)blocks), dim3(256), 0, st, d,
                       static_cast<const e128*>(keys), n, ctl);
  else
    hipLaunchKernelGGL(k_build_copy<u64>, dim3((u32)blocks), dim3(256), 0, st, d,
                       static_cast<const u64*>(keys), n, ctl);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_build_root, dim3(1), dim3(64), 0, st, d, n, ctl);
  return hipGetLastError();
}

hipError_t launch_init(HeapDesc* descs_dev, const HeapDesc* descs_host, u32 nheaps, Ctl* ctl,
                       u64 timeout_ticks, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(descs_dev, descs_host, sizeof(HeapDesc) * nheaps,
                                hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  u64 biggest = 0;
  for (u32 i = 0; i < nheaps; ++i) {
    u64 n = (u64)descs_host[i].max_nodes * descs_host[i].k * descs_host[i].ewords;
    if (n > biggest) biggest = n;
  }
  u32 gx = (u32)((biggest + 255) / 256);
  if (gx > 1024) gx = 1024;
  if (gx == 0) gx = 1;
  for (u32 y0 = 0; y0 < nheaps; y0 += 65535) {
    u32 ny = nheaps - y0 < 65535 ? nheaps - y0 : 65535;
    hipLaunchKernelGGL(k_init_heap, dim3(gx, ny), dim3(256), 0, st, descs_dev + y0, ny);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(64), 0, st, ctl, timeout_ticks);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the host copy of the descriptors must outlive the upload
  return hipStreamSynchronize(st);
}

hipError_t launch_prep(const HeapDesc* descs, u32 nheaps, Ctl* ctl, hipStream_t st) {
  u32 blocks = (nheaps + 255) / 256;
  if (blocks > 64) blocks = 64;
  hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(256), 0, st, descs, nheaps, ctl);
  return hipGetLastError();
}

}  // namespace gh
