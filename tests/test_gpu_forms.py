"""GPU parity tests of the batched and served forms.

Batched: many heaps in one persistent launch (and as a captured HIP graph);
each heap's deleteMin results must equal the oracle replaying that heap's
ticket log, and equal the same heap run alone in its own launch.

Served: the device-resident request loop admits requests by heap memory;
every heap's admitted requests, replayed on the oracle in ticket order, give
the same deleteMin results bit for bit, no heap ever exceeds its budget, and
a heap's results are the same alone and in the mix.
"""
import numpy as np
import pytest

import oracle
from paper_1906_06504_amd import workloads as W

from heap_harness import replay_and_compare, run_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_06504_amd import gheap
    gheap.load_library()
    oracle.build(force=False)
    return gheap


def _p(*a):
    print(*a, flush=True)


def test_batched_many_heaps_replay_and_alone(G):
    k, nh = 64, 16
    sizes = W.uneven_sizes(nh, nh * 10 * k, 5, seed=20)   # heaps of uneven sizes
    pre, mix, pres, mixes = W.batched_mixed(nh, k, sizes, 60 * k, seed=21)
    _p("batched heaps=%d sizes %d..%d prefill ops=%d mixed ops=%d"
       % (nh, min(sizes), max(sizes), len(pre), len(mix)))
    cap = max(sizes) + 60 * k
    hs, _, _, prelog = run_gpu(pre, k, max_keys=cap, workgroups=128, nheaps=nh)
    hs, out, counts, log = run_gpu(mix, k, max_keys=cap, workgroups=256, heapset=hs)
    for h in range(nh):
        # prefill tickets come first on every heap
        oh = oracle.OracleHeap(k)
        pl = pres[h]
        oh.replay(pl.kind, pl.n, pl.off, pl.keys, 1)
        replay_and_compare(mix, k, out, counts, log, heap=h, base_ticket=len(pl), oracle_heap=oh)
    # heap 3 alone, in its own launch: same results
    h = 3
    hs1, _, _, _ = run_gpu(pres[h], k, max_keys=cap, workgroups=32)
    hs1, out1, counts1, log1 = run_gpu(mixes[h], k, max_keys=cap, workgroups=32, heapset=hs1)
    sel = np.flatnonzero(mix.heap == h)
    dsel = sel[mix.kind[sel] == W.OP_DELETE_MIN]
    dalone = np.flatnonzero(mixes[h].kind == W.OP_DELETE_MIN)
    assert dsel.size == dalone.size
    base = sum(p.out_entries for p in mixes[:h])
    for i_mix, i_alone in zip(dsel, dalone):
        c = int(counts[i_mix])
        assert c == int(counts1[i_alone])
        o = int(mix.off[i_mix])
        o1 = int(mixes[h].off[i_alone])
        assert o == o1 + base
        assert np.array_equal(out[o:o + c], out1[o1:o1 + c])
    hs.close()
    hs1.close()


def test_batched_full_size(G):
    """The benchmark's batched workload and launch shape: 64 heaps, k = 1024,
    prefill sizes log-uniform over a 64x range summing to 2^22, 2^18 keys
    requested each, 256 workgroups of 512 threads; every heap's log replayed
    on its own oracle."""
    k, nh = 1024, 64
    sizes = W.uneven_sizes(nh, 1 << 22, 6, seed=0x5EED0012)
    pre, mix, pres, mixes = W.batched_mixed(nh, k, sizes, 1 << 18, seed=0x5EED0002)
    _p("batched-full heaps=%d prefill ops=%d mixed ops=%d" % (nh, len(pre), len(mix)))
    cap = max(sizes) + (1 << 18) + k
    hs, _, _, _ = run_gpu(pre, k, max_keys=cap, workgroups=256, threads=512, nheaps=nh)
    hs, out, counts, log = run_gpu(mix, k, max_keys=cap, workgroups=256, threads=512, heapset=hs)
    for h in range(nh):
        oh = oracle.OracleHeap(k)
        pl = pres[h]
        oh.replay(pl.kind, pl.n, pl.off, pl.keys, 1)
        replay_and_compare(mix, k, out, counts, log, heap=h, base_ticket=len(pl), oracle_heap=oh)
    hs.close()


def test_batched_graph_replays(G):
    """The batched launch captured once as a HIP graph and replayed three
    times (arena restored between replays, eager work in between): every
    replay gives the eager results."""
    k, nh = 64, 8
    sizes = W.uneven_sizes(nh, nh * 8 * k, 4, seed=32)
    pre, mix, pres, mixes = W.batched_mixed(nh, k, sizes, 40 * k, seed=33)
    cap = max(sizes) + 40 * k
    hs = G.HeapSet(k, [cap] * nh, stream=torch.cuda.Stream())
    with torch.cuda.stream(hs.stream):
        d = G.ops_to_device(pre)
        hs.submit(*d[:5], workgroups=64)
        assert hs.sync() == 0
        snap = hs.arena.clone()
        ops, n, keys, out, counts = G.ops_to_device(mix)
        hs.submit(ops, n, keys, out, counts, workgroups=64)
        assert hs.sync() == 0
        ref_out = out.clone()
        ref_counts = counts.clone()
        g = hs.submit_graph(ops, n, keys, out, counts, workgroups=64)
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


def _serve(G, pre, reqs, k, caps, workgroups, threads=0, multi_insert=False):
    hs = G.HeapSet(k, caps)
    d = G.ops_to_device(pre)
    hs.submit(*d[:5], workgroups=64)
    assert hs.sync() == 0
    r, nreq, keys, out, recs, max_ops = G.requests_to_device(reqs)
    hs.serve(r, nreq, keys, out, recs, max_ops, workgroups=workgroups, threads=threads,
             multi_insert=multi_insert)
    rc = hs.sync()
    assert rc == G.GH_OK, G.strerror(rc)
    torch.cuda.synchronize()
    return hs, G.to_host_u64(out), G.recs_to_host(recs, nreq)


def _replay_served(G, pre, reqs, recs, out, k, heap, caps):
    oh = oracle.OracleHeap(k)
    psel = np.flatnonzero(pre.heap == heap)
    for i in psel:
        oh.insert(pre.keys[int(pre.off[i]):int(pre.off[i]) + int(pre.n[i])])
    sel = np.flatnonzero((reqs.heap == heap) & ((recs["flags"] & G.REQ_ADMITTED) != 0))
    sel = sel[np.argsort(recs["first_ticket"][sel], kind="stable")]
    for i in sel:
        o = int(reqs.off[i])
        if reqs.kind[i] == W.OP_INSERT:
            oh.insert(reqs.keys[o:o + int(reqs.n[i])])
            assert int(recs["count"][i]) == int(reqs.n[i])
            assert oh.size <= caps[heap], "heap %d over its budget" % heap
        else:
            want = oh.delete_min(int(reqs.n[i]) or None)   # n = 0 means k
            c = int(recs["count"][i])
            assert c == want.size, "heap %d request %d count" % (heap, i)
            assert np.array_equal(out[o:o + c], want), "heap %d request %d output" % (heap, i)
    return oh


@pytest.mark.parametrize("rate", [None, 2e6])
def test_served_replay(G, rate):
    k, nh, nreq = 64, 8, 3000
    pre, reqs, sizes = W.served_stream(nh, k, nreq, seed=41, rate_per_s=rate, min_log2=6,
                                       max_log2=12, max_ins_log2=9)
    caps = W.served_capacity(sizes)
    _p("served heaps=%d requests=%d rate=%s" % (nh, nreq, rate))
    hs, out, recs = _serve(G, pre, reqs, k, caps, workgroups=64)
    assert np.all((recs["flags"] & (G.REQ_ADMITTED | G.REQ_REJECTED)) != 0)
    assert np.any((recs["flags"] & G.REQ_DEFERRED) != 0), "no insert ever waited for memory"
    for h in range(nh):
        _replay_served(G, pre, reqs, recs, out, k, h, caps)
    done = recs["flags"] & G.REQ_ADMITTED != 0
    assert np.all(recs["t_done"][done] >= recs["t_admit"][done])
    # answered (last root release) after admission and no later than done
    assert np.all(recs["t_resp"][done] > recs["t_admit"][done])
    assert np.all(recs["t_resp"][done] <= recs["t_done"][done])
    hs.close()


def test_served_alone_equals_mix(G):
    k, nh, nreq = 64, 6, 2000
    pre, reqs, sizes = W.served_stream(nh, k, nreq, seed=43, rate_per_s=None, min_log2=6,
                                       max_log2=11, max_ins_log2=9)
    caps = W.served_capacity(sizes)
    hs, out, recs = _serve(G, pre, reqs, k, caps, workgroups=48)
    h = 2
    # the same heap's prefill and requests alone (one heap in its own set)
    psel = np.flatnonzero(pre.heap == h)
    pl = W.OpList(pre.kind[psel], pre.n[psel], pre.off[psel], pre.keys, 0,
                  heap=np.zeros(psel.size, np.uint32))
    rsel = np.flatnonzero(reqs.heap == h)
    rl = W.OpList(reqs.kind[rsel], reqs.n[rsel], reqs.off[rsel], reqs.keys, reqs.out_entries,
                  heap=np.zeros(rsel.size, np.uint32), arrival=reqs.arrival[rsel])
    rl.meta["k"] = k
    hs1, out1, recs1 = _serve(G, pl, rl, k, [caps[h]], workgroups=16)
    assert np.array_equal(recs1["flags"] & (G.REQ_ADMITTED | G.REQ_REJECTED),
                          recs["flags"][rsel] & (G.REQ_ADMITTED | G.REQ_REJECTED))
    assert np.array_equal(recs1["count"], recs["count"][rsel])
    for j, i in enumerate(rsel):
        if reqs.kind[i] != W.OP_DELETE_MIN:
            continue
        o = int(reqs.off[i])
        c = int(recs["count"][i])
        assert np.array_equal(out[o:o + c], out1[o:o + c]), "request %d differs alone" % i
    hs.close()
    hs1.close()


def test_served_full_size_sampled(G):
    """The benchmark's served workload and launch shape (256 heaps, k = 256,
    prefill log-uniform up to 2^22, 2^20 requests, 1024 slots, budget prefill
    + 2^20): every request is admitted or rejected, and a sample of heaps
    (the largest, the smallest and six more) replays bit for bit."""
    k, nh, nreq = 256, 256, 1 << 20
    pre, reqs, sizes = W.served_stream(nh, k, nreq, seed=0x5EED0005, rate_per_s=None,
                                       max_log2=22)
    caps = W.served_capacity(sizes, extra=1 << 20)
    _p("served-full heaps=%d requests=%d prefill=%d" % (nh, nreq, int(sizes.sum())))
    hs = G.HeapSet(k, caps)
    d = G.ops_to_device(pre)
    hs.submit(*d[:5], workgroups=1024)
    assert hs.sync() == 0
    del d
    r, n, keys, out, recs, max_ops = G.requests_to_device(reqs)
    hs.serve(r, n, keys, out, recs, max_ops, workgroups=1024)
    rc = hs.sync()
    assert rc == G.GH_OK, G.strerror(rc)
    torch.cuda.synchronize()
    out = G.to_host_u64(out)
    recs = G.recs_to_host(recs, n)
    assert np.all((recs["flags"] & (G.REQ_ADMITTED | G.REQ_REJECTED)) != 0)
    sample = [int(np.argmax(sizes)), int(np.argmin(sizes))] + list(range(3, nh, nh // 6))[:6]
    for h in sample:
        _replay_served(G, pre, reqs, recs, out, k, h, caps)
    hs.close()


def test_served_queue_overflow_rejects_and_replays(G):
    """An operation queue too small for the stream: requests that no longer
    fit are rejected (their queue slots skipped by the slots), the launch
    ends with GH_ENOMEM, and every admitted request still replays."""
    k, nh, nreq = 64, 8, 2000
    pre, reqs, sizes = W.served_stream(nh, k, nreq, seed=47, rate_per_s=None, min_log2=6,
                                       max_log2=11, max_ins_log2=9)
    caps = W.served_capacity(sizes, extra=1 << 14)
    hs = G.HeapSet(k, caps)
    d = G.ops_to_device(pre)
    hs.submit(*d[:5], workgroups=64)
    assert hs.sync() == 0
    r, n, keys, out, recs, max_ops = G.requests_to_device(reqs)
    _p("served overflow: queue %d of %d operations" % (max_ops // 2, max_ops))
    hs.serve(r, n, keys, out, recs, max_ops // 2, workgroups=48)
    assert hs.sync() == G.GH_ENOMEM
    torch.cuda.synchronize()
    out = G.to_host_u64(out)
    recs = G.recs_to_host(recs, n)
    flags = recs["flags"]
    assert np.all((flags & (G.REQ_ADMITTED | G.REQ_REJECTED)) != 0)
    assert np.any((flags & G.REQ_REJECTED) != 0) and np.any((flags & G.REQ_ADMITTED) != 0)
    assert int(recs["nops"][(flags & G.REQ_ADMITTED) != 0].astype(np.int64).sum()) <= max_ops // 2
    for h in range(nh):
        _replay_served(G, pre, reqs, recs, out, k, h, caps)
    hs.close()


def test_served_invalid_heap_rejected(G):
    """Requests naming a heap outside the set are rejected (GH_EINVAL at the
    end); the other heaps' requests replay."""
    k, nh, nreq = 64, 6, 1200
    pre, reqs, sizes = W.served_stream(nh, k, nreq, seed=53, rate_per_s=None, min_log2=6,
                                       max_log2=10, max_ins_log2=8)
    bad = np.arange(7, nreq, 97)
    reqs.heap = reqs.heap.copy()
    reqs.heap[bad] = nh + 5
    caps = W.served_capacity(sizes, extra=1 << 14)
    hs = G.HeapSet(k, caps)
    d = G.ops_to_device(pre)
    hs.submit(*d[:5], workgroups=64)
    assert hs.sync() == 0
    r, n, keys, out, recs, max_ops = G.requests_to_device(reqs)
    hs.serve(r, n, keys, out, recs, max_ops, workgroups=32)
    assert hs.sync() == G.GH_EINVAL
    torch.cuda.synchronize()
    out = G.to_host_u64(out)
    recs = G.recs_to_host(recs, n)
    assert np.all((recs["flags"][bad] & G.REQ_REJECTED) != 0)
    for h in range(nh):
        _replay_served(G, pre, reqs, recs, out, k, h, caps)
    hs.close()


def test_served_variable_count_deletes(G):
    """deleteMin requests of c = U[1, k] entries (and a few asking for more
    than k, which are rejected with GH_EINVAL) through the serving loop;
    every heap replays on the oracle."""
    k, nh, nreq = 64, 6, 2500
    pre, reqs, sizes = W.served_stream(nh, k, nreq, seed=57, rate_per_s=None, min_log2=6,
                                       max_log2=11, max_ins_log2=8)
    dels = np.flatnonzero(reqs.kind == W.OP_DELETE_MIN)
    rng = np.random.default_rng(5)
    reqs.n = reqs.n.copy()
    reqs.n[dels] = rng.integers(1, k + 1, dels.size)
    bad = dels[::50]
    reqs.n[bad] = k + 3
    caps = W.served_capacity(sizes)
    _p("served variable count heaps=%d requests=%d" % (nh, nreq))
    hs = G.HeapSet(k, caps)
    d = G.ops_to_device(pre)
    hs.submit(*d[:5], workgroups=64)
    assert hs.sync() == 0
    r, n, keys, out, recs, max_ops = G.requests_to_device(reqs)
    hs.serve(r, n, keys, out, recs, max_ops, workgroups=32)
    assert hs.sync() == G.GH_EINVAL
    torch.cuda.synchronize()
    out = G.to_host_u64(out)
    recs = G.recs_to_host(recs, n)
    assert np.all((recs["flags"][bad] & G.REQ_REJECTED) != 0)
    good = np.setdiff1d(dels, bad)
    assert np.all((recs["flags"][good] & G.REQ_ADMITTED) != 0)
    for h in range(nh):
        _replay_served(G, pre, reqs, recs, out, k, h, caps)
    hs.close()
