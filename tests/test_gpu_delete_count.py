"""GPU parity tests for the variable-count deleteMin: deleteMin(c) with
1 <= c <= k returns the min(c, size) smallest live entries.  The HIP heap
(through the C ABI) is compared with the CPU oracle bit for bit: outputs by
ticket-log replay (the root is the linearization point, Sec. 3.3.3 Theorem 1),
with one operation in flight also the node array and partial buffer, and
quiescent states against Properties 1-3 (Sec. 3.1).
"""
import numpy as np
import pytest

import oracle
from paper_1906_06504_amd import workloads as W

from heap_harness import check_gpu_state, gpu_state_by_index, replay_and_compare, run_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

F_REJECT = 0x40


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_06504_amd import gheap
    gheap.load_library()
    oracle.build(force=False)
    return gheap


def _print(*a):
    print(*a, flush=True)


def _live(oh):
    onodes, opb = oh.export()
    if oh.m == 0:
        return np.sort(opb)
    return np.sort(np.concatenate([onodes[oracle.idx(p) - 1] for p in range(1, oh.m + 1)] + [opb]))


@pytest.mark.parametrize("k", [32, 64, 128, 256, 512, 1024])
def test_serialized_state_equals_oracle(G, k):
    """One operation in flight, deleteMin counts uniform on [1, k]: outputs
    and the whole node array and partial buffer equal the oracle's."""
    ops = W.mixed_ops(60 * k, k, seed=200 + k, first_id=0, var_delete=True)
    assert np.any((ops.kind == W.OP_DELETE_MIN) & (ops.n > 0) & (ops.n < k))
    _print("serialized variable count k=%d ops=%d" % (k, len(ops)))
    hs, out, counts, log = run_gpu(ops, k, max_keys=60 * k, workgroups=1)
    oh = replay_and_compare(ops, k, out, counts, log)
    m, s, byidx, pb = gpu_state_by_index(hs, 0, k)
    assert (m, s) == (oh.m, oh.s)
    onodes, opb = oh.export()
    assert np.array_equal(pb, opb)
    for c, row in byidx.items():
        assert np.array_equal(row, onodes[c - 1]), "node %d differs" % c
    hs.close()


@pytest.mark.parametrize("k,threads,wg", [(32, 64, 64), (64, 128, 128), (256, 128, 64),
                                           (512, 512, 64), (1024, 512, 32), (1024, 1024, 16)])
def test_concurrent_replay(G, k, threads, wg):
    """Many operations in flight after a prefill: deleteMin(c) and inserts
    of U[1, k] entries; ticket-log replay is exact and the final state holds
    the oracle's live multiset."""
    pre = W.prefill_ops(40 * k, k, seed=17 + k)
    mix = W.mixed_ops(200 * k, k, seed=18 + k, first_id=40 * k, var_delete=True)
    allops = W.concat(pre, mix, k)
    _print("concurrent variable count k=%d threads=%d wg=%d ops=%d"
           % (k, threads, wg, len(allops)))
    hs, out, counts, log = run_gpu(allops, k, max_keys=400 * k, workgroups=wg, threads=threads)
    oh = replay_and_compare(allops, k, out, counts, log)
    assert np.array_equal(check_gpu_state(hs, 0, k), _live(oh))
    hs.close()


@pytest.mark.parametrize("k,wg", [(32, 128), (256, 96), (1024, 64)])
def test_concurrent_near_empty(G, k, wg):
    """From an empty heap: most operations find no node or a single one, so
    the partial-buffer-only and single-node paths of deleteMin(c) run
    concurrently with inserts."""
    ops = W.mixed_ops(400 * k, k, seed=300 + k, first_id=0, var_delete=True)
    _print("near empty variable count k=%d wg=%d ops=%d" % (k, wg, len(ops)))
    hs, out, counts, log = run_gpu(ops, k, max_keys=400 * k, workgroups=wg)
    oh = replay_and_compare(ops, k, out, counts, log)
    assert np.array_equal(check_gpu_state(hs, 0, k), _live(oh))
    hs.close()


def test_single_calls(G):
    """heap_delete_min(c) one call at a time against the oracle, with counts
    from 1 to k, including ones that take the last node, ones that do not,
    and ones on a heap with a single node or none."""
    k, total = 64, 3000
    st = W.Stream(2)
    keys = W.pack(st.u32(total), np.arange(total, dtype=np.uint64))
    h = G.Heap(k, total)
    h.insert(G.to_device_u64(keys))
    oh = oracle.OracleHeap(k)
    oh.insert(keys)
    out = torch.empty(k, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    cycle = [1, 63, k, 5, 32, 64, 17, 2, 60]
    step = 0
    while oh.size > 0:
        c = cycle[step % len(cycle)]
        step += 1
        h.delete_min(out, cnt, c=c)
        want = oh.delete_min(c)
        got = int(cnt.item())
        assert got == want.size, "step %d c=%d" % (step, c)
        assert np.array_equal(G.to_host_u64(out)[:got], want), "step %d c=%d" % (step, c)
        if step % 7 == 0:
            extra = W.pack(st.u32(50), np.arange(total + step * 50, total + step * 50 + 50,
                                                  dtype=np.uint64))
            if oh.size + 50 <= total:
                h.insert(G.to_device_u64(extra))
                oh.insert(extra)
    h.delete_min(out, cnt, c=3)
    assert int(cnt.item()) == 0
    check_gpu_state(h, 0, k)
    lib = G.load_library()
    for bad in (0, k + 1):
        assert lib.heap_delete_min(h.h, out.data_ptr(), bad, cnt.data_ptr()) == G.GH_EINVAL
    assert h.close() == G.GH_OK


def test_count_above_k_rejected_in_submission(G):
    """A deleteMin record asking for more than k entries is rejected on the
    device (sticky GH_EINVAL, flag in its log record, count 0); it still
    passes the root in its turn and every other operation replays."""
    k = 64
    pre = W.prefill_ops(30 * k, k, seed=61)
    mix = W.mixed_ops(100 * k, k, seed=62, first_id=30 * k, var_delete=True)
    allops = W.concat(pre, mix, k)
    dels = np.flatnonzero(allops.kind == W.OP_DELETE_MIN)
    bad = dels[::9]
    gpu_ops = W.OpList(allops.kind.copy(), allops.n.copy(), allops.off, allops.keys,
                       allops.out_entries)
    gpu_ops.n[bad] = k + 1 + (np.arange(bad.size) % 5)
    hs = G.HeapSet(k, [200 * k])
    d_ops, n, keys, out, counts = G.ops_to_device(gpu_ops)
    log = G.new_log(n)
    hs.submit(d_ops, n, keys, out, counts, log, workgroups=32, var_delete=True)
    assert hs.sync() == G.GH_EINVAL
    torch.cuda.synchronize()
    out = G.to_host_u64(out)
    counts = counts.cpu().numpy()[:n].astype(np.uint32)
    log = G.log_to_host(log, n)
    assert np.all((log["flags"][bad] & F_REJECT) != 0)
    assert np.all(counts[bad] == 0)
    # for the oracle a rejected record is an empty insert (no effect)
    ref_ops = W.OpList(allops.kind.copy(), allops.n.copy(), allops.off, allops.keys,
                       allops.out_entries)
    ref_ops.kind[bad] = W.OP_INSERT
    ref_ops.n[bad] = 0
    oh = replay_and_compare(ref_ops, k, out, counts, log)
    assert np.array_equal(check_gpu_state(hs, 0, k), _live(oh))
    hs.close()


def test_variable_count_needs_the_flag(G):
    """Without GH_TUNE_VARIABLE_DELETE a submission runs the whole-root
    kernel, which rejects deleteMin records of 1..k-1 entries (sticky
    GH_EINVAL, flag in the log, count 0); records of 0 or k entries run and
    replay exactly."""
    k = 128
    pre = W.prefill_ops(30 * k, k, seed=71)
    mix = W.mixed_ops(100 * k, k, seed=72, first_id=30 * k, var_delete=True)
    allops = W.concat(pre, mix, k)
    dels = np.flatnonzero(allops.kind == W.OP_DELETE_MIN)
    full = dels[::3]
    ops = W.OpList(allops.kind.copy(), allops.n.copy(), allops.off, allops.keys,
                   allops.out_entries)
    ops.n[full] = np.where(np.arange(full.size) % 2 == 0, 0, k).astype(np.uint32)
    bad = dels[(ops.n[dels] != 0) & (ops.n[dels] != k)]
    full = np.setdiff1d(dels, bad)
    assert bad.size > 0
    hs = G.HeapSet(k, [200 * k])
    d_ops, n, keys, out, counts = G.ops_to_device(ops)
    log = G.new_log(n)
    hs.submit(d_ops, n, keys, out, counts, log, workgroups=32)
    assert hs.sync() == G.GH_EINVAL
    torch.cuda.synchronize()
    out = G.to_host_u64(out)
    counts = counts.cpu().numpy()[:n].astype(np.uint32)
    log = G.log_to_host(log, n)
    assert np.all((log["flags"][bad] & F_REJECT) != 0)
    assert np.all(counts[bad] == 0)
    assert not np.any(log["flags"][full] & F_REJECT)
    ref = W.OpList(ops.kind.copy(), ops.n.copy(), ops.off, ops.keys, ops.out_entries)
    ref.kind[bad] = W.OP_INSERT
    ref.n[bad] = 0
    oh = replay_and_compare(ref, k, out, counts, log)
    assert np.array_equal(check_gpu_state(hs, 0, k), _live(oh))
    hs.close()


def test_variable_count_graph_replays(G):
    """A submission with deleteMin(c) records captured once as a HIP graph
    (GH_TUNE_VARIABLE_DELETE) and replayed three times, the arena restored
    and eager work done in between: every replay equals the eager run."""
    k = 64
    pre = W.prefill_ops(20 * k, k, seed=81)
    mix = W.mixed_ops(80 * k, k, seed=82, first_id=20 * k, var_delete=True)
    hs = G.HeapSet(k, [200 * k], stream=torch.cuda.Stream())
    with torch.cuda.stream(hs.stream):
        d = G.ops_to_device(pre)
        hs.submit(*d[:5], workgroups=32)
        assert hs.sync() == 0
        snap = hs.arena.clone()
        ops, n, keys, out, counts = G.ops_to_device(mix)
        hs.submit(ops, n, keys, out, counts, workgroups=32, var_delete=True)
        assert hs.sync() == 0
        ref_out, ref_counts = out.clone(), counts.clone()
        g = hs.submit_graph(ops, n, keys, out, counts, workgroups=32, var_delete=True)
        for rep in range(3):
            hs.arena.copy_(snap)
            out.fill_(-1)
            counts.zero_()
            torch.cuda.synchronize()
            hs.graph_launch(g)
            assert hs.sync() == 0
            torch.cuda.synchronize()
            assert torch.equal(counts, ref_counts), "replay %d counts" % rep
            assert torch.equal(out, ref_out), "replay %d outputs" % rep
            _ = (keys.sum() + 1).item()   # unrelated eager work between replays
    hs.close()
