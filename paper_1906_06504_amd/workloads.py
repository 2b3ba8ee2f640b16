"""Seeded synthetic inputs for the heap workloads.

This module only draws random numbers and lays out operation lists; it holds
none of the heap's arithmetic (no ordering, merging or tree logic), so the
oracle-side tests and the GPU side can both use it.

Randomness comes from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written here from its published
definition and used in counter mode: draw i of stream `seed` is
mix(seed + (i + 1) * golden_gamma).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

OP_INSERT = 0
OP_DELETE_MIN = 1
ENTRY_MAX = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64_block(z: np.ndarray, base: np.uint64, first: int):
    """z[i] = draw (first + i) of the stream with seed `base`, in place."""
    z[:] = np.arange(first + 1, first + 1 + z.size, dtype=np.uint64)
    z *= GOLDEN_GAMMA
    z += base
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)


_BLOCK = 1 << 16   # cache-sized pieces


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Draws start .. start+count-1 of the SplitMix64 stream `seed`."""
    out = np.empty(count, dtype=np.uint64)
    base = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    for a in range(0, count, _BLOCK):
        _splitmix64_block(out[a:a + _BLOCK], base, start + a)
    return out


class Stream:
    """Sequential reader over one SplitMix64 stream."""

    def __init__(self, seed: int):
        self.seed = int(seed)
        self.pos = 0

    def u64(self, count: int) -> np.ndarray:
        out = splitmix64(self.seed, self.pos, count)
        self.pos += count
        return out

    def u32(self, count: int) -> np.ndarray:
        return (self.u64(count) >> np.uint64(32)).astype(np.uint32)

    def uniform_int(self, lo: int, hi: int, count: int) -> np.ndarray:
        """Integers uniform on [lo, hi] (multiply-shift of the top 32 bits)."""
        span = np.uint64(hi - lo + 1)
        r = self.u64(count) >> np.uint64(32)
        return (np.uint64(lo) + ((r * span) >> np.uint64(32))).astype(np.int64)

    def unit(self, count: int) -> np.ndarray:
        """Doubles uniform on [0, 1) from the top 53 bits."""
        return (self.u64(count) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def pack(keys: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """(u32 key, u32 id) -> u64 entry key<<32 | id (id 0xFFFFFFFF is reserved)."""
    return (keys.astype(np.uint64) << np.uint64(32)) | ids.astype(np.uint64)


@dataclass
class OpList:
    """A list of heap operations in submission order.

    kind[i]  0 = insert, 1 = deleteMin
    n[i]     insert: number of entries; deleteMin: entries requested, 0 = k
    off[i]   insert: offset into `keys`; deleteMin: offset of its k-entry slot
             in the output buffer
    heap[i]  heap index (0 for single-heap lists)
    arrival  optional earliest start time per op, in nanoseconds from launch
    """

    kind: np.ndarray
    n: np.ndarray
    off: np.ndarray
    keys: np.ndarray
    out_entries: int
    heap: np.ndarray | None = None
    arrival: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    def __len__(self):
        return int(self.kind.size)

    def heap_ids(self) -> np.ndarray:
        return self.heap if self.heap is not None else np.zeros(self.kind.size, dtype=np.uint32)

    def seq(self) -> np.ndarray:
        """Rank of each op among the list's ops on the same heap."""
        h = self.heap_ids().astype(np.int64)
        order = np.argsort(h, kind="stable")
        hs = h[order]
        starts = np.r_[0, np.flatnonzero(np.diff(hs)) + 1]
        run_start = np.repeat(starts, np.diff(np.r_[starts, hs.size]))
        rank = np.empty(h.size, dtype=np.int64)
        rank[order] = np.arange(h.size) - run_start
        return rank.astype(np.uint32)


def build_oplist(kinds, sizes, key_source, k: int, heap=None, arrival=None) -> OpList:
    """Lay out an op list; inserts take their keys from `key_source(count)` in
    op order, deleteMin ops each get a k-entry output slot.  `sizes` holds an
    insert's entry count and a deleteMin's requested count (0 = k)."""
    kinds = np.asarray(kinds, dtype=np.uint8)
    sizes = np.asarray(sizes, dtype=np.int64)
    n = sizes.astype(np.uint32)
    n_in = np.where(kinds == OP_INSERT, n, 0).astype(np.uint64)
    ins_off = np.cumsum(n_in) - n_in
    del_rank = np.cumsum(kinds == OP_DELETE_MIN) - (kinds == OP_DELETE_MIN)
    off = np.where(kinds == OP_INSERT, ins_off, del_rank.astype(np.uint64) * np.uint64(k)).astype(np.uint64)
    total_in = int(n_in.sum())
    keys = key_source(total_in)
    out_entries = int((kinds == OP_DELETE_MIN).sum()) * k
    return OpList(kinds, n, off, keys, out_entries,
                  None if heap is None else np.asarray(heap, dtype=np.uint32),
                  None if arrival is None else np.asarray(arrival, dtype=np.uint64))


def _keys_with_ids(stream: Stream, first_id: int):
    state = {"next": first_id}

    def src(count: int) -> np.ndarray:
        if count and state["next"] + count - 1 >= 0xFFFFFFFF:
            raise ValueError("id space exhausted")
        # key = top 32 bits of the draw (as Stream.u32), already in place;
        # built block by block so that every pass stays in cache
        out = np.empty(count, dtype=np.uint64)
        base = np.uint64(stream.seed & 0xFFFFFFFFFFFFFFFF)
        hi = np.uint64(0xFFFFFFFF00000000)
        for a in range(0, count, _BLOCK):
            z = out[a:a + _BLOCK]
            _splitmix64_block(z, base, stream.pos + a)
            z &= hi
            z |= np.arange(state["next"] + a, state["next"] + a + z.size, dtype=np.uint64)
        stream.pos += count
        state["next"] += count
        return out

    return src


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------

def insert_then_drain(total: int, k: int, batch: int, seed: int) -> OpList:
    """Insert `total` uniform u32 keys (ids 0..total-1) in batches of `batch`,
    then deleteMin until the heap is empty (one extra deleteMin returns 0)."""
    st = Stream(seed)
    n_ins = -(-total // batch)
    sizes = [batch] * (total // batch) + ([total % batch] if total % batch else [])
    n_del = -(-total // k) + 1
    kinds = [OP_INSERT] * n_ins + [OP_DELETE_MIN] * n_del
    sizes = sizes + [0] * n_del
    return build_oplist(kinds, sizes, _keys_with_ids(st, 0), k)


def ordered_insert_then_drain(total: int, k: int, order: str, seed: int) -> OpList:
    """The workload of the paper's comparison with CPU heaps (Table vscpu):
    insert `total` keys in batches of k, then deleteMin until empty (one
    extra deleteMin returns 0).  Keys are uniform u32 ("random"), or
    0, 1, 2, ... ("ascending") or total-1, ..., 0 ("descending"), each
    with its insertion rank as id."""
    if total > (1 << 32) - 1:
        raise ValueError("at most 2^32 - 1 keys")
    n_ins = -(-total // k)
    sizes = [k] * (total // k) + ([total % k] if total % k else [])
    n_del = -(-total // k) + 1
    kinds = [OP_INSERT] * n_ins + [OP_DELETE_MIN] * n_del
    sizes = sizes + [0] * n_del
    if order == "random":
        src = _keys_with_ids(Stream(seed), 0)
    elif order in ("ascending", "descending"):
        def src(count: int) -> np.ndarray:
            ids = np.arange(count, dtype=np.uint64)
            keys = ids if order == "ascending" else np.uint64(count - 1) - ids
            return (keys << np.uint64(32)) | ids
    else:
        raise ValueError("order must be random, ascending or descending")
    return build_oplist(kinds, sizes, src, k)


def prefill_ops(nkeys: int, k: int, seed: int, first_id: int = 0) -> OpList:
    """`nkeys` uniform u32 keys inserted as full batches of k."""
    st = Stream(seed)
    sizes = [k] * (nkeys // k) + ([nkeys % k] if nkeys % k else [])
    kinds = [OP_INSERT] * len(sizes)
    return build_oplist(kinds, sizes, _keys_with_ids(st, first_id), k)


def mixed_ops(total_requested: int, k: int, seed: int, first_id: int,
              max_insert: int | None = None, p_insert: float = 0.5,
              var_delete: bool = False) -> OpList:
    """Random interleave: each op is an insert of U[1, max_insert] fresh keys
    (probability p_insert) or a deleteMin(k) -- with var_delete a
    deleteMin(c), c uniform on [1, k] -- drawn until the requested keys
    (insert sizes plus each deleteMin's count) reach `total_requested`."""
    max_insert = k if max_insert is None else max_insert
    st = Stream(seed)
    cst = Stream(seed ^ 0x0C0C0C0C0C0C0C0C)
    kinds, sizes = [], []
    acc = 0
    chunk = 4096
    while acc < total_requested:
        coin = st.unit(chunk)
        sz = st.uniform_int(1, max_insert, chunk)
        dc = cst.uniform_int(1, k, chunk) if var_delete else None
        for j, (c, s) in enumerate(zip(coin, sz)):
            if acc >= total_requested:
                break
            if c < p_insert:
                kinds.append(OP_INSERT)
                sizes.append(int(s))
                acc += int(s)
            else:
                kinds.append(OP_DELETE_MIN)
                want = int(dc[j]) if var_delete else 0
                sizes.append(want)
                acc += want or k
    key_stream = Stream(seed ^ 0x5A5A5A5A5A5A5A5A)
    return build_oplist(kinds, sizes, _keys_with_ids(key_stream, first_id), k)


def wide_entries(keys: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """16-byte entries [n, 2] uint64 in the device layout: word 0 = the signed
    64-bit key XOR 2^63 (so that it orders as unsigned), word 1 = the 32-bit
    id (32 zero bits above it)."""
    k = np.asarray(keys, dtype=np.int64).view(np.uint64) ^ np.uint64(1 << 63)
    i = np.asarray(ids, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    return np.ascontiguousarray(np.stack([k, i], axis=1))


def to_wide(ops: OpList, seed: int, key_bits: int = 64) -> OpList:
    """The same operation list with 16-byte entries: each entry keeps its id
    (the low 32 bits of its 8-byte form) and gets a fresh signed key drawn
    uniformly from [-2^(key_bits-1), 2^(key_bits-1)) (key_bits < 64 makes
    equal keys with distinct ids common)."""
    ids = ops.keys & np.uint64(0xFFFFFFFF)
    raw = Stream(seed).u64(ids.size)
    if key_bits < 64:
        raw = (raw >> np.uint64(64 - key_bits)).astype(np.int64) - np.int64(1 << (key_bits - 1))
    keys = raw.view(np.int64) if raw.dtype == np.uint64 else raw
    out = OpList(ops.kind, ops.n, ops.off, wide_entries(keys, ids), ops.out_entries,
                 ops.heap, ops.arrival, dict(ops.meta))
    return out


def concat(a: OpList, b: OpList, k: int) -> OpList:
    """Ops of a followed by ops of b (b's offsets shifted past a's buffers)."""
    kind = np.concatenate([a.kind, b.kind])
    n = np.concatenate([a.n, b.n])
    boff = b.off.copy()
    boff[b.kind == OP_INSERT] += np.uint64(a.keys.size)
    boff[b.kind == OP_DELETE_MIN] += np.uint64(a.out_entries)
    off = np.concatenate([a.off, boff])
    keys = np.concatenate([a.keys, b.keys])
    return OpList(kind, n, off, keys, a.out_entries + b.out_entries)


CONFIG_SEED = {1: 0x5EED0001, 2: 0x5EED0002, 3: 0x5EED0003, 4: 0x5EED0004, 5: 0x5EED0005}


def config1(scale: int = 1 << 16) -> tuple[OpList, int]:
    """Plain heap, k = 64: insert 2^16 keys in batches of 64, then drain."""
    k = 64
    return insert_then_drain(scale, k, 64, CONFIG_SEED[1]), k


def config2(prefill: int = 1 << 22, requested: int = 1 << 24, k: int = 1024):
    """Plain heap, k = 1024: prefill `prefill` keys as full batches, then a
    50/50 interleave of inserts of U[1, 1024] keys and deleteMin(1024) until
    `requested` keys have been requested.  Returns (prefill ops, mixed ops, k)."""
    pre = prefill_ops(prefill, k, CONFIG_SEED[2])
    mix = mixed_ops(requested, k, CONFIG_SEED[2] + 1, first_id=prefill)
    return pre, mix, k


def _interleave(lists, st: Stream):
    """Random interleave of per-heap op lists (each keeps its order)."""
    counts = np.array([len(l) for l in lists], dtype=np.int64)
    owner = np.repeat(np.arange(len(lists)), counts)
    perm = np.argsort(st.u64(owner.size), kind="stable")
    owner = owner[perm]
    # stable per owner: j-th occurrence of heap h takes op j of list h
    order = np.argsort(owner, kind="stable")
    rank = np.empty(owner.size, dtype=np.int64)
    starts = np.r_[0, np.cumsum(counts)[:-1]]
    rank[order] = np.arange(owner.size) - np.repeat(starts, counts)
    return owner, rank


def multi_heap(lists, k: int, st: Stream) -> OpList:
    """One op list over several heaps: a random interleave of `lists` (each an
    OpList for one heap, offsets into its own buffers)."""
    owner, rank = _interleave(lists, st)
    key_base = np.r_[0, np.cumsum([l.keys.size for l in lists])[:-1]].astype(np.uint64)
    out_base = np.r_[0, np.cumsum([l.out_entries for l in lists])[:-1]].astype(np.uint64)
    kind = np.empty(owner.size, dtype=np.uint8)
    n = np.empty(owner.size, dtype=np.uint32)
    off = np.empty(owner.size, dtype=np.uint64)
    for h, l in enumerate(lists):
        sel = owner == h
        r = rank[sel]
        kind[sel] = l.kind[r]
        n[sel] = l.n[r]
        off[sel] = np.where(l.kind[r] == OP_INSERT, l.off[r] + key_base[h], l.off[r] + out_base[h])
    keys = np.concatenate([l.keys for l in lists]) if lists else np.zeros(0, np.uint64)
    out = OpList(kind, n, off, keys, int(sum(l.out_entries for l in lists)),
                 heap=owner.astype(np.uint32))
    out.meta["k"] = k
    return out


def uneven_sizes(nheaps: int, total: int, spread_log2: int, seed: int) -> list[int]:
    """Heap sizes log-uniform over a 2^spread_log2 range, scaled so that they
    sum to `total` (the last heap takes the rounding remainder)."""
    u = Stream(seed).unit(nheaps)
    w = 2.0 ** (spread_log2 * u)
    sizes = np.floor(w / w.sum() * total).astype(np.int64)
    sizes[-1] += total - int(sizes.sum())
    return [int(x) for x in sizes]


def batched_mixed(nheaps: int, k: int, prefill_each, requested_each: int, seed: int):
    """nheaps independent heaps, each prefilled (`prefill_each` keys, or
    prefill_each[h] for heap h: heaps of uneven sizes) and then given a 50/50
    insert U[1,k] / deleteMin(k) mix requesting `requested_each` keys;
    returns (prefill list, mixed list, per-heap prefill lists, per-heap mixed
    lists), the first two over all heaps (ids unique across heaps)."""
    st = Stream(seed)
    pres, mixes = [], []
    next_id = 0
    sizes = (list(prefill_each) if np.ndim(prefill_each) else [int(prefill_each)] * nheaps)
    for h in range(nheaps):
        p = prefill_ops(sizes[h], k, seed + 101 * (h + 1), first_id=next_id)
        next_id += sizes[h]
        m = mixed_ops(requested_each, k, seed + 101 * (h + 1) + 7, first_id=next_id)
        next_id += int(m.n.sum())
        pres.append(p)
        mixes.append(m)
    return multi_heap(pres, k, st), multi_heap(mixes, k, st), pres, mixes


def served_stream(nheaps: int, k: int, nreq: int, seed: int, rate_per_s: float | None = None,
                  min_log2: int = 10, max_log2: int = 22, ins_frac: float = 0.6,
                  max_ins_log2: int = 12):
    """Request stream for the served form.

    Heap h is prefilled with floor(2^(min_log2 + (max_log2-min_log2) u)) keys
    (log-uniform).  Each request picks a heap uniformly; it is an insert of
    floor(2^(max_ins_log2 u)) fresh keys (log-uniform on [1, 2^max_ins_log2])
    with probability ins_frac, else a deleteMin(k).  Arrivals are a Poisson
    process of rate `rate_per_s` (exponential gaps; None = all at time 0).
    Returns (prefill list over all heaps, request list, prefill sizes)."""
    st = Stream(seed)
    u = st.unit(nheaps)
    sizes = np.floor(2.0 ** (min_log2 + (max_log2 - min_log2) * u)).astype(np.int64)
    pre_lists = []
    next_id = 0
    for h in range(nheaps):
        pre_lists.append(prefill_ops(int(sizes[h]), k, seed + 7 * (h + 1), first_id=next_id))
        next_id += int(sizes[h])
    pre = multi_heap(pre_lists, k, st)
    heap = np.minimum((st.unit(nreq) * nheaps).astype(np.int64), nheaps - 1)
    is_ins = st.unit(nreq) < ins_frac
    n_ins = np.floor(2.0 ** (max_ins_log2 * st.unit(nreq))).astype(np.int64)
    kinds = np.where(is_ins, OP_INSERT, OP_DELETE_MIN).astype(np.uint8)
    sizes_req = np.where(is_ins, n_ins, 0)
    if rate_per_s is None:
        arrival = np.zeros(nreq, dtype=np.uint64)
    else:
        gaps = -np.log1p(-st.unit(nreq)) / rate_per_s * 1e9
        arrival = np.floor(np.cumsum(gaps)).astype(np.uint64)
    key_stream = Stream(seed ^ 0x77777777)
    reqs = build_oplist(kinds, sizes_req, _keys_with_ids(key_stream, next_id), k,
                        heap=heap.astype(np.uint32), arrival=arrival)
    reqs.meta["k"] = k
    pre.meta["k"] = k
    return pre, reqs, sizes


def poisson_arrivals(n: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (ns) of a Poisson process of the given rate."""
    st = Stream(seed)
    gaps = -np.log1p(-st.unit(n)) / rate_per_s * 1e9
    return np.floor(np.cumsum(gaps)).astype(np.uint64)


def served_capacity(prefill_sizes: np.ndarray, extra: int | None = None) -> np.ndarray:
    """Memory budget (entries) per heap for the served form: the prefill plus
    `extra` entries, or (extra None) the prefill plus a quarter of it plus
    4096, a tight budget under which inserts regularly wait for memory."""
    if extra is not None:
        return (prefill_sizes + int(extra)).astype(np.int64)
    return (np.ceil(1.25 * prefill_sizes) + 4096).astype(np.int64)


def knapsack_instances(ninst: int, seed: int, n_lo: int = 40, n_hi: int = 200,
                       w_hi: int = 1000, extra_hi: int = 100):
    """0/1 knapsack instances: n ~ U[n_lo, n_hi] items, weights U[1, w_hi],
    value = weight + U[0, extra_hi], capacity = floor(sum of weights / 2).
    Returns a list of (weights, values, capacity)."""
    st = Stream(seed)
    ns = st.uniform_int(n_lo, n_hi, ninst)
    out = []
    for i in range(ninst):
        n = int(ns[i])
        w = st.uniform_int(1, w_hi, n).astype(np.uint32)
        v = (w.astype(np.int64) + st.uniform_int(0, extra_hi, n)).astype(np.uint32)
        out.append((w, v, int(w.astype(np.int64).sum() // 2)))
    return out


def poisson_cdf(lam: float, dmax: int) -> np.ndarray:
    """P(X <= d) for d = 0..dmax of a Poisson(lam) variable."""
    pmf = np.empty(dmax + 1)
    pmf[0] = np.exp(-lam)
    for d in range(1, dmax + 1):
        pmf[d] = pmf[d - 1] * lam / d
    return np.cumsum(pmf)


def sssp_graph(V: int, seed: int, mean_degree: float = 8.0, w_lo: int = 1, w_hi: int = 1000):
    """Random directed graph in CSR: out-degrees Poisson(mean_degree) by
    inverse CDF, targets uniform on [0, V) with self-loops redrawn (multi-edges
    kept), weights uniform on [w_lo, w_hi].  Returns (rowptr[V+1], col[E],
    w[E]) as uint32 arrays."""
    st = Stream(seed)
    cdf = poisson_cdf(mean_degree, 200)
    deg = np.searchsorted(cdf, st.unit(V), side="right").astype(np.int64)
    deg = np.minimum(deg, 200)
    rowptr = np.zeros(V + 1, dtype=np.int64)
    np.cumsum(deg, out=rowptr[1:])
    E = int(rowptr[-1])
    if V > 1:
        src = np.repeat(np.arange(V, dtype=np.int64), deg)
        col = st.uniform_int(0, V - 1, E)
        bad = np.flatnonzero(col == src)
        while bad.size:
            col[bad] = st.uniform_int(0, V - 1, bad.size)
            bad = bad[col[bad] == src[bad]]
    else:
        # a single vertex can only have self-loops: it gets no edges
        rowptr[:] = 0
        E = 0
        col = np.zeros(0, dtype=np.int64)
    w = st.uniform_int(w_lo, w_hi, E)
    return rowptr.astype(np.uint32), col.astype(np.uint32), w.astype(np.uint32)


def config3(V: int = 1 << 20):
    """SSSP workload: V vertices, out-degree Poisson(8), weights U[1, 1000],
    source vertex 0, k = 512."""
    rowptr, col, w = sssp_graph(V, CONFIG_SEED[3])
    return rowptr, col, w, 0, 512
