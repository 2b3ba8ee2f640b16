// gh_setup.hip -- arena initialization and per-submission preparation
// kernels (no heap arithmetic).
#include "gh_launch.h"

namespace gh {

// Fill every node and partial-buffer slot with ENT_MAX, every lock with
// AVAIL, and zero the metadata, for one heap per y-block row.
__global__ void k_init_heap(const HeapDesc* __restrict__ descs, u32 nheaps) {
  const u32 h = blockIdx.y;
  if (h >= nheaps) return;
  const HeapDesc d = descs[h];
  const u64 n_nodes = (u64)d.max_nodes * d.k;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  const u64 start = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  for (u64 i = start; i < n_nodes; i += stride) d.nodes[i] = ENT_MAX;
  for (u64 i = start; i <= d.max_nodes; i += stride) d.locks[i] = 0;
  for (u64 i = start; i < d.k; i += stride) d.pb[i] = ENT_MAX;
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
    for (int j = 0; j < 8; ++j) sw[j] = 0;
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

hipError_t launch_init(HeapDesc* descs_dev, const HeapDesc* descs_host, u32 nheaps, Ctl* ctl,
                       u64 timeout_ticks, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(descs_dev, descs_host, sizeof(HeapDesc) * nheaps,
                                hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  u64 biggest = 0;
  for (u32 i = 0; i < nheaps; ++i) {
    u64 n = (u64)descs_host[i].max_nodes * descs_host[i].k;
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
