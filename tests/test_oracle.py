"""Pins for the CPU oracle, against facts fixed outside the oracle itself.

* brute force: a deleteMin returns exactly the min(k, size) smallest live
  entries in ascending order (the root holds the k smallest by Properties 1
  and 3, Sec. 3.1; the partial buffer is read only when no node exists,
  Sec. 3.3.2), checked against a sorted Python list on small random traces;
  likewise deleteMin(c) returns the min(c, size) smallest, and a filter
  keeps exactly the entries below its bound;
* bulk build (Sec. 3.1): a built heap satisfies the properties and drains
  to its input;
* Properties 1-3 and the closed form m = size // k, s = size % k after every
  operation (the partial buffer never reaches k entries, Sec. 3.1);
* k = 1 reduces to the conventional heap (Sec. 3.1, note after Property 3):
  pop order equals Python's heapq;
* insert-all-then-drain returns the fully sorted sequence;
* the bit-reversal target order (Sec. 4.3) against an independent string
  reversal, and the stated property that consecutive insert paths share
  only the root;
* MergeAndSort (Sec. 3.2.1 display equation) against sorted();
* planted mistakes: variants of the oracle with one plausible error each must
  fail these pins.
"""
import heapq
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

MAXE = np.uint64(0xFFFFFFFFFFFFFFFF)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def random_trace(rng, k, nops, key_range, max_ins=None, var_del=False, filt=False, bu=False):
    """Random op sequence: ('ins', array), ('del',), with var_del also
    ('del', c) with c uniform on [1, k], with filt also ('filter', bound),
    with bu also ('insbu', array) (the bottom-up insert)."""
    max_ins = max_ins or 3 * k
    ops = []
    for _ in range(nops):
        if filt and rng.random() < 0.12:
            ops.append(("filter", int(rng.integers(0, key_range + 1))))
        elif rng.random() < 0.55:
            n = int(rng.integers(0, max_ins + 1))
            kind = "insbu" if bu and rng.random() < 0.6 else "ins"
            ops.append((kind, rng.integers(0, key_range, n).astype(np.uint64)))
        elif var_del and rng.random() < 0.7:
            ops.append(("del", int(rng.integers(1, k + 1))))
        else:
            ops.append(("del",))
    return ops


def run_against_brute_force(k, ops, lib=None):
    """Returns None if the oracle matches brute force on every op, else a
    string describing the first mismatch."""
    h = oracle.OracleHeap(k, lib=lib)
    live = []
    for i, op in enumerate(ops):
        if op[0] in ("ins", "insbu"):
            h.insert(op[1], bottom_up=op[0] == "insbu")
            live = sorted(live + [int(v) for v in op[1]])
        elif op[0] == "filter":
            live = [v for v in live if v < op[1]]
            if h.filter(op[1]) != len(live):
                return "op %d: filter kept the wrong number" % i
        else:
            want_n = op[1] if len(op) > 1 else k
            got = h.delete_min(op[1] if len(op) > 1 else None)
            c = min(want_n, len(live))
            want = live[:c]
            live = live[c:]
            if [int(v) for v in got] != want:
                return "op %d: deleteMin mismatch" % i
        rc = h.check()
        if rc:
            return "op %d: invariant code %d" % (i, rc)
        if h.size != len(live) or h.m != len(live) // k or h.s != len(live) % k:
            return "op %d: size bookkeeping" % i
    return None


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 16])
def test_brute_force_random_traces(k):
    rng = np.random.default_rng(1000 + k)
    for trial in range(60):
        key_range = 50 if trial % 3 == 0 else 1 << 40   # duplicates and distinct
        ops = random_trace(rng, k, int(rng.integers(5, 80)), key_range)
        msg = run_against_brute_force(k, ops)
        assert msg is None, "k=%d trial=%d %s" % (k, trial, msg)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 16])
def test_brute_force_variable_count_deletes(k):
    """deleteMin(c), 1 <= c <= k: the min(c, size) smallest live entries,
    ascending, with Properties 1-3 and m = size // k, s = size % k after
    every operation."""
    rng = np.random.default_rng(3000 + k)
    for trial in range(60):
        key_range = 50 if trial % 3 == 0 else 1 << 40
        ops = random_trace(rng, k, int(rng.integers(5, 120)), key_range, var_del=True)
        msg = run_against_brute_force(k, ops)
        assert msg is None, "k=%d trial=%d %s" % (k, trial, msg)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 16])
def test_brute_force_with_filters(k):
    """Filter(bound) removes exactly the entries >= bound; afterwards the
    heap satisfies Properties 1-3 and the m/s closed form, and every later
    deleteMin returns the smallest survivors."""
    rng = np.random.default_rng(4000 + k)
    for trial in range(60):
        key_range = 50 if trial % 2 == 0 else 1 << 40
        ops = random_trace(rng, k, int(rng.integers(5, 120)), key_range, var_del=True, filt=True)
        msg = run_against_brute_force(k, ops)
        assert msg is None, "k=%d trial=%d %s" % (k, trial, msg)


def test_build_then_drain_is_sorted():
    """Bulk build (Sec. 3.1): Properties 1-3 hold right after the build and
    draining returns the input; a non-empty heap or unsorted input is
    refused."""
    rng = np.random.default_rng(9)
    for k in (1, 3, 8, 64):
        for n in (0, 1, k - 1, k, k + 1, 7 * k + 3, 100 * k):
            keys = np.sort(rng.integers(0, 1 << 40, n).astype(np.uint64))
            h = oracle.OracleHeap(k)
            h.build(keys)
            assert h.check() == 0 and h.size == n
            got = []
            while True:
                b = h.delete_min()
                if b.size == 0:
                    break
                got.extend(int(x) for x in b)
            assert got == [int(x) for x in keys]
    h = oracle.OracleHeap(4)
    h.insert([5])
    with pytest.raises(RuntimeError):
        h.build(np.array([1, 2], dtype=np.uint64))
    with pytest.raises(ValueError):
        oracle.OracleHeap(4).build(np.array([3, 2], dtype=np.uint64))


def test_variable_count_delete_bounds_and_full_count():
    """c = k is the ordinary deleteMin (same output and same internal
    state); c = 0 and c > k are refused."""
    rng = np.random.default_rng(5)
    k = 8
    a, b = oracle.OracleHeap(k), oracle.OracleHeap(k)
    for _ in range(200):
        if rng.random() < 0.6:
            x = rng.integers(0, 1 << 40, int(rng.integers(1, 3 * k))).astype(np.uint64)
            a.insert(x)
            b.insert(x)
        else:
            assert np.array_equal(a.delete_min(), b.delete_min(k))
        na, pa = a.export()
        nb, pb = b.export()
        assert np.array_equal(na, nb) and np.array_equal(pa, pb)
    for bad in (0, k + 1):
        with pytest.raises(ValueError):
            a.delete_min(bad)


def test_replay_variable_count_deletes():
    """Replay reads a deleteMin's count from n (0 = k) and refuses n > k."""
    k = 4
    keys = np.arange(100, 130, dtype=np.uint64)
    types = np.array([0, 0, 1, 1, 1, 1], dtype=np.uint8)
    n = np.array([4, 4, 3, 0, 1, 0], dtype=np.uint32)
    off = np.array([0, 4, 0, 3, 7, 8], dtype=np.uint64)
    out, counts = oracle.OracleHeap(k).replay(types, n, off, keys, 16, check=True)
    assert list(counts) == [0, 0, 3, 4, 1, 0]
    assert list(out[:8]) == list(range(100, 108))
    with pytest.raises(RuntimeError):
        oracle.OracleHeap(k).replay(np.array([1], np.uint8), np.array([5], np.uint32),
                                    np.array([0], np.uint64), keys, 16)


def test_k1_matches_heapq_order():
    rng = np.random.default_rng(7)
    h = oracle.OracleHeap(1)
    ref = []
    for step in range(3000):
        if rng.random() < 0.6:
            v = int(rng.integers(0, 1000))
            h.insert([v])
            heapq.heappush(ref, v)
        else:
            got = h.delete_min()
            if ref:
                assert list(got) == [heapq.heappop(ref)]
            else:
                assert got.size == 0
        assert h.check() == 0


@pytest.mark.parametrize("k,batch,total", [(64, 64, 1 << 16), (32, 17, 5000), (7, 100, 3001)])
def test_insert_all_then_drain_is_sorted(k, batch, total):
    rng = np.random.default_rng(k)
    keys = rng.integers(0, 1 << 32, total).astype(np.uint64) << np.uint64(32) | np.arange(total, dtype=np.uint64)
    h = oracle.OracleHeap(k)
    for i in range(0, total, batch):
        h.insert(keys[i:i + batch])
    assert h.check() == 0
    outs = []
    while True:
        o = h.delete_min()
        if o.size == 0:
            break
        assert o.size == k or h.size == 0
        outs.append(o)
    assert np.array_equal(np.concatenate(outs), np.sort(keys))


def _rev_by_string(p):
    l = p.bit_length() - 1
    if l == 0:
        return 1
    off = p - (1 << l)
    return (1 << l) + int(format(off, "0%db" % l)[::-1], 2)


def test_bit_reversal_golden_table():
    """The hand-typed table of the first 32 positions (Sec. 4.3)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "bitrev_order_1_32.txt")
    rows = [tuple(int(x) for x in line.split()) for line in open(path)
            if line.strip() and not line.startswith("#")]
    assert [p for p, _ in rows] == list(range(1, 33))
    for p, c in rows:
        assert oracle.idx(p) == c, "position %d" % p


def test_bit_reversal_order():
    for p in range(1, 5000):
        assert oracle.idx(p) == _rev_by_string(p)
        assert oracle.idx(oracle.idx(p)) == p
    for l in range(0, 13):
        level = list(range(1 << l, 1 << (l + 1)))
        assert sorted(oracle.idx(p) for p in level) == level


def _path(t):
    out = []
    while t >= 1:
        out.append(t)
        t //= 2
    return set(out)


def test_consecutive_insert_paths_share_only_root():
    for p in range(2, 5000):
        shared = _path(oracle.idx(p)) & _path(oracle.idx(p + 1))
        assert shared == {1}, p


def test_merge_and_sort_matches_sorted():
    rng = np.random.default_rng(3)
    for _ in range(200):
        na, nb = int(rng.integers(0, 40)), int(rng.integers(0, 40))
        a = np.sort(rng.integers(0, 30, na).astype(np.uint64))
        b = np.sort(rng.integers(0, 30, nb).astype(np.uint64))
        hi, lo = oracle.merge_and_sort(a, b)
        allv = sorted([int(x) for x in a] + [int(x) for x in b])
        assert [int(x) for x in hi] == allv[:na]
        assert [int(x) for x in lo] == allv[na:]


def test_delete_on_empty_and_pb_only():
    h = oracle.OracleHeap(8)
    assert h.delete_min().size == 0
    h.insert([5, 3, 9])
    assert h.m == 0 and h.s == 3
    assert list(h.delete_min()) == [3, 5, 9]
    assert h.size == 0


def test_replay_matches_step_by_step():
    from paper_1906_06504_amd import workloads as W
    ops = W.mixed_ops(20000, 16, seed=11, first_id=0)
    h1 = oracle.OracleHeap(16)
    out, counts = h1.replay(ops.kind, ops.n, ops.off, ops.keys, ops.out_entries, check=True)
    h2 = oracle.OracleHeap(16)
    for i in range(len(ops)):
        if ops.kind[i] == 0:
            h2.insert(ops.keys[int(ops.off[i]):int(ops.off[i]) + int(ops.n[i])])
        else:
            got = h2.delete_min()
            o = int(ops.off[i])
            assert counts[i] == got.size
            assert np.array_equal(out[o:o + got.size], got)


# ---------------------------------------------------------------------------
# planted mistakes: each must be caught by the pins above
# ---------------------------------------------------------------------------

SRC = os.path.join(os.path.dirname(oracle.__file__), "gheap_oracle.c")

MUTANTS = {
    "no_pb_merge_on_delete": (
        "    if (h->s > 0)\n        merge_and_sort(h, node_at(h, 1), k, h->pb, h->s, node_at(h, 1), h->pb);\n    sift_down(h);\n    return k;",
        "    sift_down(h);\n    return k;"),
    "filter_keeps_the_bound": (
        "            if (N[i] < bound) buf[kept++] = N[i];",
        "            if (N[i] <= bound) buf[kept++] = N[i];"),
    "filter_drops_pb": (
        "        if (h->pb[i] < bound) buf[kept++] = h->pb[i];",
        "        if (0) buf[kept++] = h->pb[i];"),
    "build_at_tree_index_p": (
        "        uint64_t c = gho_idx(p);\n        if (ensure_cap(h, c)) return -1;",
        "        uint64_t c = p;\n        if (ensure_cap(h, c)) return -1;"),
    "partial_delete_no_sift": (
        "    sift_down(h);\n    return c;",
        "    return c;"),
    "partial_delete_always_takes_last": (
        "    if (nrest >= k) {",
        "    if (0) {"),
    "partial_delete_pb_not_shifted": (
        "        memmove(h->pb, h->pb + cnt, (h->s - cnt) * sizeof(gho_ent));\n",
        ""),
    "partial_delete_drops_root_rest": (
        "    merge_into(root + c, k - c, h->pb, h->s, rest);",
        "    merge_into(root + k, 0, h->pb, h->s, rest);"),
    "lo_to_smaller_max_child": (
        "uint64_t big = (L[k - 1] > R[k - 1]) ? l : r;",
        "uint64_t big = (L[k - 1] > R[k - 1]) ? r : l;"),
    "early_stop_on_min": (
        "if (cur[k - 1] <= cmin) break;",
        "if (cur[0] <= cmin) break;"),
    "partial_insert_skips_root_merge": (
        "    h->s += n;\n    if (h->m >= 1)\n        merge_and_sort(h, node_at(h, 1), k, h->pb, h->s, node_at(h, 1), h->pb);\n}",
        "    h->s += n;\n}"),
    "pb_capacity_k": (
        "return n + h->s <= h->k - 1; }",
        "return n + h->s <= h->k; }"),
    "no_max_fill": (
        "    for (uint64_t i = 0; i < k; i++) node_at(h, last)[i] = GHO_MAX;\n    h->m -= 1;",
        "    h->m -= 1;"),
    "insert_path_skips_root": (
        "for (int j = 0; j < L; j++) {",
        "for (int j = 1; j < L; j++) {"),
    "one_child_no_merge": (
        "            if (cur[k - 1] <= X[0]) break;",
        "            break;"),
    "bu_no_climb": (
        "        if (P[k - 1] <= C[0]) break;             /* the property holds from here up */",
        "        break;"),
    "bu_stop_on_parent_min": (
        "        if (P[k - 1] <= C[0]) break;             /* the property holds from here up */",
        "        if (P[0] <= C[0]) break;"),
    "bu_parent_keeps_largest": (
        "        merge_and_sort(h, P, k, C, k, P, C);     /* parent keeps the k smallest */",
        "        merge_and_sort(h, P, k, C, k, C, P);"),
    "bu_climb_stops_below_root": (
        "    while (c > 1) {\n        gho_ent *C = node_at(h, c), *P = node_at(h, c / 2);",
        "    while (c > 3) {\n        gho_ent *C = node_at(h, c), *P = node_at(h, c / 2);"),
    "bu_target_at_tree_index": (
        "    uint64_t t = gho_idx(h->m + 1);\n    if (ensure_cap(h, t)) { free(merged); return -1; }",
        "    uint64_t t = h->m + 1;\n    if (ensure_cap(h, t)) { free(merged); return -1; }"),
    "full_batch_takes_largest": (
        "    memcpy(F, merged, k * sizeof(gho_ent));\n    memcpy(h->pb, merged + k, rest * sizeof(gho_ent));",
        "    memcpy(F, merged + rest, k * sizeof(gho_ent));\n    memcpy(h->pb, merged, rest * sizeof(gho_ent));"),
}


def _build_mutant(name, tmpdir):
    before, after = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(before) == 1, "mutation anchor for %s not found exactly once" % name
    path = os.path.join(tmpdir, name + ".c")
    with open(path, "w") as f:
        f.write(src.replace(before, after))
    so = os.path.join(tmpdir, name + ".so")
    apps = os.path.join(os.path.dirname(SRC), "apps_oracle.c")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-w", "-o", so, path, apps])
    return oracle.load(so)


def _mutant_caught(lib):
    rng = np.random.default_rng(99)
    for k in (1, 2, 3, 4, 8):
        for trial in range(40):
            ops = random_trace(rng, k, 60, 1 << 40 if trial % 2 else 40, var_del=trial % 4 >= 2,
                               filt=trial % 8 >= 4, bu=trial % 3 == 0)
            try:
                if run_against_brute_force(k, ops, lib=lib) is not None:
                    return True
            except Exception:
                return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    with tempfile.TemporaryDirectory() as d:
        lib = _build_mutant(name, d)
        assert _mutant_caught(lib), "planted mistake %s was not detected" % name


def test_sorted_array_in_addition_order_is_a_heap():
    """Sec. 3.1: a sorted array satisfies the properties.  Laid out in the
    order nodes are added (the p-th chunk of k at position p, node index
    idx(p)), every parent's chunk precedes its children's, so Properties 1-3
    hold for any n and k (checked directly, for k = 1..9 and many n)."""
    import random
    rnd = random.Random(3)
    for k in range(1, 10):
        for n in [0, 1, k - 1, k, k + 1, 5 * k + 3, 37 * k, rnd.randint(1, 400)]:
            keys = sorted(rnd.randint(0, 50) for _ in range(n))
            m, s = n // k, n % k
            node = {}
            for p in range(1, m + 1):
                node[oracle.idx(p)] = keys[(p - 1) * k:p * k]
            pb = keys[m * k:]
            assert sorted(node) == sorted(oracle.idx(p) for p in range(1, m + 1))
            for c, batch in node.items():
                assert batch == sorted(batch)                       # Property 1
                if c > 1:
                    assert c // 2 in node                            # complete shape
                    assert node[c // 2][-1] <= batch[0]              # Property 2
            if m and pb:
                assert node[1][-1] <= pb[0]                          # Property 3
            assert len(pb) < k


# ---------------------------------------------------------------------------
# 16-byte entries (signed 64-bit key, 32-bit id), ordered by key, then id
# ---------------------------------------------------------------------------

SIGN = 1 << 63


def _wide(pairs):
    """[(signed key, id)] -> [n, 2] uint64 in the device layout (key XOR 2^63,
    then the id), written out here independently of the library."""
    a = np.zeros((len(pairs), 2), dtype=np.uint64)
    for i, (key, ident) in enumerate(pairs):
        a[i, 0] = (key + (1 << 64) if key < 0 else key) ^ SIGN
        a[i, 1] = ident
    return a


def _pairs(a):
    out = []
    for w0, w1 in np.asarray(a, dtype=np.uint64).reshape(-1, 2):
        u = int(w0) ^ SIGN
        out.append((u - (1 << 64) if u >= SIGN else u, int(w1)))
    return out


def run_wide_against_brute_force(k, ops, lib=None):
    """As run_against_brute_force with 16-byte entries: the live multiset is
    a sorted list of (key, id) tuples (Python's tuple order is the
    lexicographic order the entry defines)."""
    h = oracle.OracleHeap(k, lib=lib, wide=True)
    live = []
    for i, op in enumerate(ops):
        if op[0] == "ins":
            h.insert(_wide(op[1]))
            live = sorted(live + list(op[1]))
        elif op[0] == "filter":
            key = op[1]
            live = [p for p in live if p[0] < key]
            word = (key + (1 << 64) if key < 0 else key) ^ SIGN
            if h.filter(word) != len(live):
                return "op %d: filter kept the wrong number" % i
        else:
            want_n = op[1] if len(op) > 1 else k
            got = _pairs(h.delete_min(op[1] if len(op) > 1 else None))
            c = min(want_n, len(live))
            if got != live[:c]:
                return "op %d: deleteMin mismatch" % i
            live = live[c:]
        rc = h.check()
        if rc:
            return "op %d: invariant code %d" % (i, rc)
        if h.size != len(live) or h.m != len(live) // k or h.s != len(live) % k:
            return "op %d: size bookkeeping" % i
    return None


def wide_trace(rng, k, nops, key_span, next_id):
    """Random ops on (key, id) pairs: keys signed, uniform on
    [-key_span, key_span) (a small span gives many equal keys), ids unique."""
    ops = []
    for _ in range(nops):
        r = rng.random()
        if r < 0.08:
            ops.append(("filter", int(rng.integers(-key_span, key_span + 1))))
        elif r < 0.6:
            n = int(rng.integers(0, 3 * k + 1))
            keys = rng.integers(-key_span, key_span, n)
            ops.append(("ins", [(int(x), next_id + j) for j, x in enumerate(keys)]))
            next_id += n
        elif r < 0.8:
            ops.append(("del", int(rng.integers(1, k + 1))))
        else:
            ops.append(("del",))
    return ops


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 16])
def test_wide_brute_force_random_traces(k):
    """16-byte entries: every deleteMin returns the min(c, size) smallest
    (key, id) pairs, with negative keys, keys near the ends of the 64-bit
    range and many equal keys told apart by the id only."""
    rng = np.random.default_rng(7000 + k)
    for trial in range(50):
        span = [3, 1000, 1 << 62][trial % 3]
        ops = wide_trace(rng, k, int(rng.integers(5, 70)), span, next_id=trial * 100000)
        msg = run_wide_against_brute_force(k, ops)
        assert msg is None, "k=%d trial=%d %s" % (k, trial, msg)


def test_wide_extreme_keys_and_drain():
    """The most negative and most positive keys, and equal keys with ids in
    descending insertion order, drain in (key, id) order."""
    k = 4
    pairs = [(-(1 << 63), 9), ((1 << 63) - 1, 1), (0, 5), (0, 2), (-1, 7), (1, 0),
             ((1 << 63) - 1, 0), (-(1 << 63), 3), (0, 4)]
    h = oracle.OracleHeap(k, wide=True)
    h.insert(_wide(pairs))
    got = []
    while True:
        out = _pairs(h.delete_min())
        if not out:
            break
        got += out
    assert got == sorted(pairs)


def test_wide_layout_conversion_is_pinned(monkeypatch):
    """Planted mistake in the wrapper's layout conversion (the key and id
    words not swapped into the oracle's 128-bit order, so that entries order
    by id first): the brute-force pin must catch it."""
    monkeypatch.setattr(oracle, "wide_to_c", lambda a: np.ascontiguousarray(
        np.asarray(a, dtype=np.uint64).reshape(-1, 2)))
    monkeypatch.setattr(oracle, "wide_from_c", lambda a: np.ascontiguousarray(
        np.asarray(a, dtype=np.uint64).reshape(-1, 2)))
    rng = np.random.default_rng(5)
    caught = False
    for trial in range(20):
        ops = wide_trace(rng, 4, 40, 1000, next_id=0)
        if run_wide_against_brute_force(4, ops) is not None:
            caught = True
            break
    assert caught


# ---------------------------------------------------------------------------
# traffic counters (the measurement's algorithmic bytes come from them)
# ---------------------------------------------------------------------------

def test_traffic_counter_hand_computed_trace():
    """k = 2, worked by hand: insert [5] stays in the partial buffer (2
    entries moved: 2 (n + s)); insert [3] makes a full batch that becomes
    the root (n + s + (n + s - k) = 2, plus 2kL + k = 2); insert [9, 1] makes
    a full batch to node 2 one level down (2 + 2*2*1 + 2 = 8); a deleteMin
    refills the root from node 2 with nothing to sift (3k = 6); a deleteMin
    of the only node (2k = 4); a deleteMin of the empty heap (0)."""
    h = oracle.OracleHeap(2)
    h.insert([5 << 32])
    assert h.counters()["traffic_entries"] == 2
    h.insert([3 << 32 | 1])
    assert h.counters()["traffic_entries"] == 6
    h.insert([9 << 32 | 2, 1 << 32 | 3])
    assert h.counters()["traffic_entries"] == 14
    h.delete_min()
    c = h.counters()
    assert c["traffic_entries"] == 20 and c["del_refill"] == 1 and c["del_levels"] == 0
    h.delete_min()
    assert h.counters()["traffic_entries"] == 24
    assert len(h.delete_min()) == 0
    assert h.counters()["traffic_entries"] == 24


@pytest.mark.parametrize("k", [4, 64])
def test_traffic_counter_full_batches_closed_form(k):
    """m full batches into an empty heap: batch p goes to level
    floor(log2 p), so the traffic is sum over p of 2k + 2k floor(log2 p),
    and the path nodes are sum of floor(log2 p)."""
    m = 300
    h = oracle.OracleHeap(k)
    keys = (np.arange(m * k, dtype=np.uint64) * np.uint64(2654435761)) % np.uint64(1 << 40)
    for p in range(m):
        h.insert(keys[p * k:(p + 1) * k])
    levels = sum(int(np.floor(np.log2(p))) for p in range(1, m + 1))
    c = h.counters()
    assert c["ins_path_nodes"] == levels and c["ins_full"] == m
    assert c["traffic_entries"] == 2 * k * m + 2 * k * levels


# ---------------------------------------------------------------------------
# bottom-up INS (Sec. 3.2.2, "Bottom-up INS" paragraph)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 3, 4, 8, 16])
def test_bottom_up_brute_force_random_traces(k):
    """Traces mixing bottom-up inserts, top-down inserts and deleteMins:
    every deleteMin returns the min(k, size) smallest live entries, and
    Properties 1-3 with the m/s closed form hold after every operation."""
    rng = np.random.default_rng(3000 + k)
    for trial in range(50):
        key_range = 50 if trial % 3 == 0 else 1 << 40
        ops = random_trace(rng, k, int(rng.integers(5, 80)), key_range, bu=True)
        msg = run_against_brute_force(k, ops)
        assert msg is None, "k=%d trial=%d %s" % (k, trial, msg)


def _path_down(t):
    """Node indices from the root down to node t."""
    out = []
    while t >= 1:
        out.append(t)
        t //= 2
    return out[::-1]


@pytest.mark.parametrize("k", [2, 3, 8])
def test_bottom_up_path_is_the_sorted_union_in_chunks(k):
    """Closed form of one full-batch bottom-up insert: with F the k smallest
    of (input + partial buffer), the nodes on the root-to-target path hold,
    from the root down, consecutive k-chunks of the sorted union of F and
    their entries before the insert (the heap property orders the path's
    batches, so climbing merges sort their union; where the climb stops the
    upper chunks are already in place).  Nodes off the path do not change."""
    rng = np.random.default_rng(77 + k)
    for trial in range(40):
        h = oracle.OracleHeap(k)
        for _ in range(int(rng.integers(0, 30))):
            h.insert(rng.integers(0, 1 << 30, int(rng.integers(1, k + 1))).astype(np.uint64))
        m0, s0 = h.m, h.s
        nodes0, pb0 = h.export()
        n = k - s0 + int(rng.integers(0, s0 + 1))          # makes a full batch
        x = rng.integers(0, 1 << 30, n).astype(np.uint64)
        merged = np.sort(np.concatenate([x, pb0]))
        F, rest = merged[:k], merged[k:]
        h.insert(x, bottom_up=True)
        nodes1, pb1 = h.export()
        t = oracle.idx(m0 + 1)
        path = _path_down(t)
        union = np.sort(np.concatenate([F] + [nodes0[c - 1] for c in path[:-1]]))
        for j, c in enumerate(path):
            assert np.array_equal(nodes1[c - 1], union[j * k:(j + 1) * k]), "trial %d node %d" % (trial, c)
        assert np.array_equal(pb1, rest)
        for c in range(1, m0 + 1):
            if c not in path:
                assert np.array_equal(nodes1[c - 1], nodes0[c - 1])


def test_bottom_up_hand_worked_trace():
    """k = 2, bottom-up inserts worked by hand (positions 1, 2, 3, 4 are
    node indices 1, 2, 3, 4):
      [5,9] -> root [5,9];
      [1,7] at node 2, merged with the root: root [1,5], node 2 [7,9];
      [3,4] at node 3, merged with the root: root [1,3], node 3 [4,5];
      [8,6] at node 4 (child of 2): node 2 [6,7], node 4 [8,9], and the
            root's largest 3 <= 6 stops the climb;
      [0,2] at node 5 (idx(5) = 6, child of 3): node 3 [0,2], node 6 [4,5];
            root [1,3] vs [0,2]: root [0,1], node 3 [2,3]."""
    h = oracle.OracleHeap(2)
    steps = [([5, 9], {1: [5, 9]}),
             ([1, 7], {1: [1, 5], 2: [7, 9]}),
             ([3, 4], {1: [1, 3], 2: [7, 9], 3: [4, 5]}),
             ([8, 6], {1: [1, 3], 2: [6, 7], 3: [4, 5], 4: [8, 9]}),
             ([0, 2], {1: [0, 1], 2: [6, 7], 3: [2, 3], 4: [8, 9], 6: [4, 5]})]
    for keys, want in steps:
        h.insert(np.array(keys, dtype=np.uint64), bottom_up=True)
        nodes, pb = h.export()
        assert h.m == len(want) and h.s == 0
        for c, row in want.items():
            assert [int(v) for v in nodes[c - 1]] == row, (keys, c)
    c = h.counters()
    assert c["ins_path_nodes"] == 5   # merges: root; root; node 2; node 3 and the root


def test_bottom_up_ascending_batches_never_climb():
    """Ascending full batches: each new batch is no smaller than its parent,
    so no merge happens and the layout is the bulk build of the input."""
    k = 4
    keys = np.arange(40 * k, dtype=np.uint64)
    h = oracle.OracleHeap(k)
    for i in range(40):
        h.insert(keys[i * k:(i + 1) * k], bottom_up=True)
    assert h.counters()["ins_path_nodes"] == 0
    b = oracle.OracleHeap(k)
    b.build(keys)
    n1, p1 = h.export()
    n2, p2 = b.export()
    assert np.array_equal(n1[:40], n2[:40]) and np.array_equal(p1, p2)
