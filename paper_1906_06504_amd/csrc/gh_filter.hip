// gh_filter.hip -- filter of one quiescent heap: every entry >= a bound is
// removed (the garbage collection of a branch-and-bound search, Sec. 5.7.2:
// nodes whose bound can no longer beat the incumbent are dropped while the
// search runs).  The entries kept are the heap's smallest; in a generalized
// heap they are the whole of a top subtree of nodes plus a prefix of each
// node below it and of the partial buffer, which do not occupy the first
// positions of the addition order.  So they are gathered, sorted (tiles in
// LDS, then merge-path passes in global memory) and laid out again as a bulk
// build (Sec. 3.1: a sorted array is a generalized heap).  Node capacity
// comes from the heap descriptor, so this object is compiled once.
#include <mutex>

#include "gh_launch.h"

namespace gh {

constexpr int FT = 512;      // threads of the filter kernels
constexpr int TILE = 2048;   // entries sorted in LDS, and merged, per workgroup

// The workspace starts with this header; then the per-node counts (one u64
// per node position and one for the pb), then two sort buffers.
struct alignas(256) FilterHead {
  u64 m;      // node count when the filter started
  u64 s;      // partial-buffer size then
  u64 kept;   // entries below the bound
  u64 pad[29];
};
static_assert(sizeof(FilterHead) == 256, "filter head layout");

// Entries below the bound in every node (a binary search: nodes are sorted)
// and in the partial buffer; slot m of cnt is the pb.
template <class Ent>
__global__ void k_filter_count(const HeapDesc* __restrict__ d, Ent bound, FilterHead* fh,
                               u64* __restrict__ cnt) {
  const HeapDesc H = *d;
  const u64 w = ld_relaxed(&H.meta->root);
  const u64 m = rw_m(w), s = rw_s(w);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    fh->m = m;
    fh->s = s;
  }
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 p = (u64)blockIdx.x * blockDim.x + threadIdx.x; p <= m; p += stride) {
    const Ent* e = p < m ? reinterpret_cast<const Ent*>(H.nodes) + p * H.k
                         : reinterpret_cast<const Ent*>(H.pb);
    u32 lo = 0, hi = p < m ? H.k : (u32)s;
    while (lo < hi) {
      const u32 mid = (lo + hi) >> 1;
      if (ent_lt(e[mid], bound)) lo = mid + 1;
      else hi = mid;
    }
    cnt[p] = lo;
  }
}

// Exclusive scan of cnt[0..m] in place (one workgroup); the total is the
// number of entries kept.  Each thread takes SI consecutive counts, all
// loaded before any is used, so a heap of up to FT * SI nodes costs one
// memory round trip.
constexpr int SI = 16;
__global__ __launch_bounds__(FT) void k_filter_scan(FilterHead* fh, u64* __restrict__ cnt) {
  __shared__ u64 part[FT];
  const u64 n = fh->m + 1;
  const int tid = threadIdx.x;
  u64 carry = 0;
  for (u64 base = 0; base < n; base += (u64)FT * SI) {
    const u64 b = base + (u64)tid * SI;
    u64 v[SI];
    u64 sum = 0;
#pragma unroll
    for (int j = 0; j < SI; ++j) {
      v[j] = b + j < n ? cnt[b + j] : 0;
      sum += v[j];
    }
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < FT; off <<= 1) {
      const u64 t = tid >= off ? part[tid - off] : 0;
      __syncthreads();
      part[tid] += t;
      __syncthreads();
    }
    u64 run = carry + part[tid] - sum;
#pragma unroll
    for (int j = 0; j < SI; ++j) {
      if (b + j < n) cnt[b + j] = run;
      run += v[j];
    }
    carry += part[FT - 1];
    __syncthreads();
  }
  if (tid == 0) fh->kept = carry;
}

// Each node's (and the pb's) kept prefix to its offset in out.
template <class Ent>
__global__ __launch_bounds__(FT) void k_filter_gather(const HeapDesc* __restrict__ d,
                                                      const FilterHead* fh,
                                                      const u64* __restrict__ off,
                                                      Ent* __restrict__ out) {
  const HeapDesc H = *d;
  const u64 m = fh->m;
  for (u64 p = blockIdx.x; p <= m; p += gridDim.x) {
    const Ent* e = p < m ? reinterpret_cast<const Ent*>(H.nodes) + p * H.k
                         : reinterpret_cast<const Ent*>(H.pb);
    const u64 o = off[p];
    const u64 n = (p < m ? off[p + 1] : fh->kept) - o;
    for (u64 i = threadIdx.x; i < n; i += FT) out[o + i] = e[i];
  }
}

// Sort every TILE-entry tile of buf in place.
template <class Ent>
__global__ __launch_bounds__(FT) void k_filter_tiles(const FilterHead* fh, Ent* __restrict__ buf) {
  __shared__ __align__(16) Ent lds[2 * TILE];
  lds_t<Ent>* const A = (lds_t<Ent>*)lds;
  lds_t<Ent>* const B = A + TILE;
  const u64 n = fh->kept;
  for (u64 t0 = (u64)blockIdx.x * TILE; t0 < n; t0 += (u64)gridDim.x * TILE) {
    const int c = n - t0 < (u64)TILE ? (int)(n - t0) : TILE;
    load_n<FT>(A, buf + t0, (u32)c);
    __syncthreads();
    const lds_t<Ent>* r = block_sort<TILE, FT, Ent>(A, B, c);
    store_n<FT>(buf + t0, r, (u32)c);
    __syncthreads();
  }
}

// Merge passes that a sort of n entries takes after the tile sort: one per
// run width w = TILE, 2 TILE, ... below n.  The sorted result is in the first
// sort buffer after an even count, in the second after an odd one.
__device__ __forceinline__ u32 merge_passes(u64 n) {
  u32 p = 0;
  for (u64 w = TILE; w < n; w *= 2) ++p;
  return p;
}

// One merge pass: adjacent sorted runs of w entries (w a multiple of TILE)
// are merged pairwise from src to dst.  Each workgroup writes TILE outputs
// between two merge-path diagonals; the input ranges between the two splits
// are staged in LDS and merged there.  The host sizes the passes for the
// heap's capacity; a pass whose runs already span the kept entries does
// nothing.
//
// A split is the number of entries of A among the first dd outputs (A first
// on ties): the boundary of the predicate A[i] <= B[dd - 1 - i], which holds
// for every i below it and for none from it on.  Half of the workgroup (SG
// lanes) finds each of the two splits.  With NP = 1 one lane bisects (log2(r)
// dependent loads for a range of r entries); with NP > 1 every round probes
// NP evenly spaced points of the remaining range at once and keeps the gap
// between the last probe that holds and the first that does not: about
// log(r) / log(NP + 1) rounds of one memory round trip, but NP scattered
// cache lines fetched from each run per round.
constexpr int SG = FT / 2;
constexpr int NP = 16;
static_assert(SG % 64 == 0 && NP >= 1 && NP <= SG, "split search lanes");

template <class Ent>
__global__ __launch_bounds__(FT) void k_filter_merge(const FilterHead* fh,
                                                     const Ent* __restrict__ src,
                                                     Ent* __restrict__ dst, u64 w) {
  __shared__ __align__(16) Ent lds[2 * TILE];
  __shared__ u64 rng[2][2];        // [search][lo, hi]
  __shared__ u32 hits[FT / 64];    // probes that hold, per wavefront
  const u64 n = fh->kept;
  if (w >= n) return;
  const int half = threadIdx.x / SG;
  const int g = threadIdx.x % SG;
  for (u64 o = (u64)blockIdx.x * TILE; o < n; o += (u64)gridDim.x * TILE) {
    const u64 ps = o / (2 * w) * (2 * w);
    const u64 na = n - ps < w ? n - ps : w;
    const u64 nb = n - ps > w ? (n - ps - w < w ? n - ps - w : w) : 0;
    const Ent* A = src + ps;
    const Ent* B = src + ps + na;
    const u64 d0 = o - ps;
    const u64 d1 = d0 + TILE < na + nb ? d0 + TILE : na + nb;
    const u64 dd = half ? d1 : d0;
    if (g == 0) {
      rng[half][0] = dd > nb ? dd - nb : 0;
      rng[half][1] = dd < na ? dd : na;
    }
    if constexpr (NP == 1) {
      if (g == 0) {
        u64 lo = rng[half][0], hi = rng[half][1];
        while (lo < hi) {
          const u64 mid = (lo + hi) >> 1;
          if (ent_le(A[mid], B[dd - 1 - mid])) lo = mid + 1;
          else hi = mid;
        }
        rng[half][0] = lo;
      }
    } else {
      __syncthreads();
      for (;;) {
        if (rng[0][0] == rng[0][1] && rng[1][0] == rng[1][1]) break;
        const u64 lo = rng[half][0], hi = rng[half][1];
        const u64 span = hi - lo;
        bool t = false;
        if (g < NP) {
          if (span > (u64)NP) {
            const u64 i = lo + ((u64)(g + 1) * span) / (NP + 1);
            t = ent_le(A[i], B[dd - 1 - i]);
          } else if ((u64)g < span) {
            const u64 i = lo + g;
            t = ent_le(A[i], B[dd - 1 - i]);
          }
        }
        const u64 m = __ballot(t);
        if ((threadIdx.x & 63) == 0) hits[threadIdx.x >> 6] = (u32)__popcll(m);
        __syncthreads();
        if (g == 0 && span > 0) {
          u32 c = 0;
          for (int v = 0; v < SG / 64; ++v) c += hits[half * (SG / 64) + v];
          u64 nlo, nhi;
          if (span <= (u64)NP) {
            nlo = nhi = lo + c;
          } else {
            nlo = c == 0 ? lo : lo + ((u64)c * span) / (NP + 1) + 1;
            nhi = c == (u32)NP ? hi : lo + ((u64)(c + 1) * span) / (NP + 1);
          }
          rng[half][0] = nlo;
          rng[half][1] = nhi;
        }
        __syncthreads();
      }
    }
    __syncthreads();
    const u64 a0 = rng[0][0], b0 = d0 - a0, a1 = rng[1][0], b1 = d1 - a1;
    const int la = (int)(a1 - a0), lb = (int)(b1 - b0);
    lds_t<Ent>* const LA = (lds_t<Ent>*)lds;
    lds_t<Ent>* const LB = LA + la;
    lds_t<Ent>* const LO = (lds_t<Ent>*)lds + TILE;
    load_n<FT>(LA, A + a0, (u32)la);
    load_n<FT>(LB, B + b0, (u32)lb);
    __syncthreads();
    merge_split<TILE / FT, FT>(LA, la, LB, lb, la + lb, sink(LO), sink(LO));
    __syncthreads();
    store_n<FT>(dst + o, LO, (u32)(la + lb));
    __syncthreads();
  }
}

// The kept entries, ascending, become the heap again: nodes in addition
// order, the rest the partial buffer; the lock words of every position that
// held a node are cleared.
template <class Ent>
__global__ void k_filter_build(const HeapDesc* __restrict__ d, const FilterHead* fh,
                               const Ent* __restrict__ bufA, const Ent* __restrict__ bufB) {
  const HeapDesc H = *d;
  const u64 n = fh->kept;
  const Ent* __restrict__ sorted = (merge_passes(n) & 1u) ? bufB : bufA;
  Ent* nodes = reinterpret_cast<Ent*>(H.nodes);
  Ent* pb = reinterpret_cast<Ent*>(H.pb);
  const u64 body = n / H.k * H.k;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  const u64 i0 = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  for (u64 i = i0; i < n; i += stride) {
    if (i < body) nodes[i] = sorted[i];
    else pb[i - body] = sorted[i];
  }
  for (u64 p = i0 + 1; p <= fh->m; p += stride) H.locks[p] = 0;
}

__global__ void k_filter_root(const HeapDesc* __restrict__ d, const FilterHead* fh) {
  if (threadIdx.x == 0) {
    const HeapDesc H = *d;
    const u64 n = fh->kept;
    const u64 m = n / H.k;
    const u64 w = ld_relaxed(&H.meta->root);
    st_relaxed(&H.meta->root, rootword(rw_ticket(w), m, n - m * H.k));
  }
}

u64 filter_workspace_bytes(u64 max_nodes, u32 k, u32 ebytes) {
  const u64 cnt = (max_nodes + 1) * 8;
  const u64 cap = (max_nodes * k + k + TILE - 1) / TILE * TILE;
  return sizeof(FilterHead) + (cnt + 255) / 256 * 256 + 2 * cap * ebytes;
}

template <class Ent>
static hipError_t launch_filter_t(const HeapDesc* d, u64 max_nodes, u32 k, Ent bound, void* work,
                                  u64* kept_out, hipStream_t st) {
  unsigned char* base = static_cast<unsigned char*>(work);
  FilterHead* fh = reinterpret_cast<FilterHead*>(base);
  u64* cnt = reinterpret_cast<u64*>(base + sizeof(FilterHead));
  const u64 cap = (max_nodes * k + k + TILE - 1) / TILE * TILE;
  Ent* bufA = reinterpret_cast<Ent*>(base + sizeof(FilterHead) +
                                     ((max_nodes + 1) * 8 + 255) / 256 * 256);
  Ent* bufB = bufA + cap;
  auto grid = [](u64 items, u64 per, u64 most) {
    u64 g = (items + per - 1) / per;
    if (g > most) g = most;
    return (u32)(g == 0 ? 1 : g);
  };
  hipLaunchKernelGGL(k_filter_count<Ent>, dim3(grid(max_nodes + 1, FT, 1024)), dim3(FT), 0, st, d,
                     bound, fh, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_filter_scan, dim3(1), dim3(FT), 0, st, fh, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_filter_gather<Ent>, dim3(grid(max_nodes + 1, 1, 4096)), dim3(FT), 0, st, d,
                     fh, cnt, bufA);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_filter_tiles<Ent>, dim3(grid(cap, TILE, 4096)), dim3(FT), 0, st, fh, bufA);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  Ent* src = bufA;
  Ent* dst = bufB;
  for (u64 w = TILE; w < cap; w *= 2) {
    hipLaunchKernelGGL(k_filter_merge<Ent>, dim3(grid(cap, TILE, 4096)), dim3(FT), 0, st, fh, src,
                       dst, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    Ent* t = src;
    src = dst;
    dst = t;
  }
  hipLaunchKernelGGL(k_filter_build<Ent>, dim3(grid(cap, FT, 2048)), dim3(FT), 0, st, d, fh, bufA,
                     bufB);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_filter_root, dim3(1), dim3(64), 0, st, d, fh);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (kept_out) {
    e = hipMemcpyAsync(kept_out, &fh->kept, sizeof(u64), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// 16-byte entries: an entry is removed when its key word is >= bound (the
// entry is >= the entry (bound, 0)).
hipError_t launch_filter(const HeapDesc* d, u64 max_nodes, u32 k, u32 ebytes, u64 bound,
                         void* work, u64* kept_out, hipStream_t st) {
  if (ebytes == 16) {
    e128 b;
    b.x = bound;
    b.y = 0;
    return launch_filter_t<e128>(d, max_nodes, k, b, work, kept_out, st);
  }
  return launch_filter_t<u64>(d, max_nodes, k, bound, work, kept_out, st);
}

// ---------------------------------------------------------------------------
// Workspace of heap_filter_noalloc, for callers that cannot allocate device
// memory: a fixed array, one copy on every GPU the library runs on, held
// until the process ends.  In host code `scratch` names the array only for
// hipGetSymbolAddress; its device address is looked up once per device,
// with that device current, and every launch gets that address.  Nothing in
// it has to start at zero: the count and scan kernels write the header and
// every count the later kernels read, and the sort buffers are read only
// below the kept count that the same call wrote.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[GH_FILTER_NOALLOC_MAX_BYTES];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_addr[SCRATCH_DEVICES];
}  // namespace

hipError_t filter_scratch_init(int dev) {
  if (dev < 0 || dev >= SCRATCH_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(scratch_mu);
  if (scratch_addr[dev]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  scratch_addr[dev] = p;
  return hipSuccess;
}

void* filter_scratch(int dev) {
  if (dev < 0 || dev >= SCRATCH_DEVICES) return nullptr;
  std::lock_guard<std::mutex> g(scratch_mu);
  return scratch_addr[dev];
}

}  // namespace gh
