// gh_private.hip -- the operation loop of a submission launched with one
// workgroup: with one operation in flight every heap of the set is private
// to that workgroup, so the operations run without root ticket and node
// locks (gh_private.h), in list order, with each heap's root and partial
// buffer resident in LDS while its operations run.  Compiled once per
// supported k and width with -DGH_K=<k> -DGH_ENT_BYTES=<8|16>; each object
// exports gh::launch_private_k<k, Ent>().
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

// The whole-root loop's records (inserts of 1..K entries, deleteMins of K)
// in list order.  Each operation's ticket is its heap's base plus its seq,
// and seq must count the heap's operations in list order (what one workgroup
// taking the root in seq order needs); a record out of that order is
// refused (GH_EINVAL) and takes no ticket.
template <int K, int T, class Ent>
__global__ __launch_bounds__(T) void k_private(const HeapDesc* __restrict__ descs,
                                               const gh_op* __restrict__ ops, u32 nops,
                                               OpParams direct, const Ent* __restrict__ in,
                                               Ent* __restrict__ out, u32* __restrict__ counts,
                                               gh_logrec* __restrict__ log, Ctl* __restrict__ ctl) {
  __shared__ __align__(16) Ent lds[priv_lds_entries<K, T, Ent>()];
  lds_t<Ent>* const L = (lds_t<Ent>*)lds;
  __shared__ OpShared sh;
  const int tid = threadIdx.x;
  PrivState st{0, 0, false, 0};
  u32 cur = 0xFFFFFFFFu;   // the heap whose state is in LDS
  u64 base = 0, served = 0;
  for (u32 i = 0; i < nops; ++i) {
    if (tid == 0) {
      sh.ok = ld_relaxed32(&ctl->abort) ? 0u : 1u;
      sh.t_claim = now_ticks();
    }
    __syncthreads();
    if (!sh.ok) break;
    gh_op op;
    if (ops) {
      op = ops[i];
    } else {
      // an insert of n_total entries as operations of up to K entries
      op.heap = 0;
      op.kind = direct.kind;
      op.seq = i;
      op.off = (u64)i * K;
      op.arrival_ns = 0;
      const u64 rem = direct.n_total - (u64)i * K;
      op.n = direct.kind == GH_OP_INSERT ? (u32)(rem < (u64)K ? rem : (u64)K) : 0u;
    }
    if (op.heap >= direct.nheaps) {
      if (tid == 0) {
        note_error(ctl, ERR_INVAL);
        if (counts) counts[i] = 0;
        if (log) {
          gh_logrec rec{};
          rec.kind = (uint8_t)op.kind;
          rec.flags = (uint8_t)F_REJECT;
          log[i] = rec;
        }
      }
      __syncthreads();
      continue;
    }
    if (op.heap != cur) {
      if (cur != 0xFFFFFFFFu) priv_end<K, T, Ent>(descs[cur], L, st, base + served);
      cur = op.heap;
      base = *gptr(&descs[cur].meta->base);
      priv_begin<K, T, Ent>(descs[cur], L, st, sh);
      served = st.served;   // the heap may have run earlier operations of this launch
    }
    const HeapDesc H = descs[cur];
    const u64 ticket = base + op.seq;
    if (op.arrival_ns != 0 && tid == 0) {
      u64 ns = op.arrival_ns < 60000000000ull ? op.arrival_ns : 60000000000ull;
      const u64 due = ctl->t0 + (ns * direct.clock_mhz) / 1000ull;
      while (now_ticks() < due) {
        if (ld_relaxed32(&ctl->abort)) break;
        __builtin_amdgcn_s_sleep(8);
      }
    }
    OpResult r{0, 0, 0, true};
    const bool out_of_order = op.seq != served;
    const bool malformed = out_of_order || op.kind > GH_OP_DELETE_MIN ||
                           (op.kind == GH_OP_INSERT && op.n > (u32)K) ||
                           (op.kind == GH_OP_DELETE_MIN && op.n != 0 && op.n != (u32)K);
    if (tid == 0) {
      sh.s = st.s;
      sh.t_root = now_ticks();
    }
    if (malformed) {
      if (tid == 0) note_error(ctl, ERR_INVAL);
      r.flags = F_REJECT;
    } else if (op.kind == GH_OP_INSERT) {
      if (op.n != 0) {
        load_n<T>(L + 4 * K, in + op.off, op.n);
        const lds_t<Ent>* xs = block_sort<K, T, Ent>(L + 4 * K, L + 5 * K, (int)op.n);
        r = priv_insert<K, T, Ent>(H, L, st, xs, op.n, sh, ctl);
      }
    } else {
      r = priv_delete<K, T, Ent>(H, L, st, out + op.off, sh);
    }
    if (!out_of_order) ++served;
    if (tid == 0) {
      if (counts) counts[i] = op.kind == GH_OP_INSERT ? 0u : r.count;
      if (log) {
        const u64 t0 = ctl->t0;
        gh_logrec rec;
        rec.ticket = ticket;
        rec.count = r.count;
        rec.levels = (uint16_t)r.levels;
        rec.kind = (uint8_t)op.kind;
        rec.flags = (uint8_t)r.flags;
        rec.pb = (uint16_t)sh.s;
        rec.reserved = 0;
        rec.t_claim = (u32)(sh.t_claim - t0);
        rec.t_root = (u32)(sh.t_root - t0);
        rec.t_done = (u32)(now_ticks() - t0);
        log[i] = rec;
      }
    }
    __syncthreads();
  }
  if (cur != 0xFFFFFFFFu) priv_end<K, T, Ent>(descs[cur], L, st, base + served);
}

template <int K, int T, class Ent>
static hipError_t launch_private_t(const LaunchArgs& a) {
  hipLaunchKernelGGL((k_private<K, T, Ent>), dim3(1), dim3(T), 0, a.stream, a.descs, a.ops,
                     a.nops, a.direct, reinterpret_cast<const Ent*>(a.in),
                     reinterpret_cast<Ent*>(a.out), a.counts, a.log, a.ctl);
  return hipGetLastError();
}

template <>
hipError_t launch_private_k<GH_K, GH_ENT>(const LaunchArgs& a) {
  switch (a.threads) {
#define GH_CASE(TT)                                                                \
  case TT:                                                                         \
    if constexpr (shape_ok(GH_K, TT)) return launch_private_t<GH_K, TT, GH_ENT>(a); \
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

}  // namespace gh
