"""GPU parity tests of 16-byte entries (GH_I64_ID: a signed 64-bit key and a
32-bit id, ordered by key, then id) through the C ABI against the oracle
built for the same entries, bit for bit: serialized state equality,
concurrent ticket replay, single calls, variable-count deleteMins, bulk
build and filter, a captured graph and the served form.  Keys are drawn so
that negative keys and equal keys with distinct ids are common."""
import numpy as np
import pytest

import oracle
from paper_1906_06504_amd import workloads as W

from heap_harness import (assert_same_state, check_gpu_state, oracle_live, replay_and_compare,
                          run_gpu, sort_entries)

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


def _mixed_wide(n_pre, n_mix, k, seed, key_bits=20, var_delete=False):
    pre = W.prefill_ops(n_pre, k, seed=seed)
    mix = W.mixed_ops(n_mix, k, seed=seed + 1, first_id=n_pre, var_delete=var_delete)
    return W.to_wide(W.concat(pre, mix, k), seed + 2, key_bits)


@pytest.mark.parametrize("k", [32, 256, 1024])
def test_wide_serialized_state_equals_oracle(G, k):
    ops = W.to_wide(W.mixed_ops(60 * k, k, seed=300 + k, first_id=0), 301 + k, 16)
    _p("wide serialized k=%d ops=%d" % (k, len(ops)))
    hs, out, counts, log = run_gpu(ops, k, max_keys=60 * k, workgroups=1)
    oh = replay_and_compare(ops, k, out, counts, log)
    assert_same_state(hs, 0, oh, k)
    assert hs.close() == G.GH_OK


@pytest.mark.parametrize("k,wg,threads", [(32, 64, 0), (256, 32, 0), (256, 64, 256),
                                          (1024, 16, 0), (1024, 32, 512)])
def test_wide_concurrent_replay(G, k, wg, threads):
    ops = _mixed_wide(40 * k, 200 * k, k, seed=310 + k + wg)
    _p("wide concurrent k=%d wg=%d threads=%d ops=%d" % (k, wg, threads, len(ops)))
    hs, out, counts, log = run_gpu(ops, k, max_keys=400 * k, workgroups=wg, threads=threads)
    oh = replay_and_compare(ops, k, out, counts, log)
    assert np.array_equal(check_gpu_state(hs, 0, k), oracle_live(oh))
    assert hs.close() == G.GH_OK


@pytest.mark.parametrize("k", [64, 1024])
def test_wide_variable_count_deletes_replay(G, k):
    ops = _mixed_wide(30 * k, 150 * k, k, seed=330 + k, var_delete=True)
    _p("wide deleteMin(c) k=%d ops=%d" % (k, len(ops)))
    hs, out, counts, log = run_gpu(ops, k, max_keys=300 * k, workgroups=48)
    oh = replay_and_compare(ops, k, out, counts, log)
    assert np.array_equal(check_gpu_state(hs, 0, k), oracle_live(oh))
    assert hs.close() == G.GH_OK


def test_wide_single_calls_and_extremes(G):
    """heap_insert / heap_delete_min one call at a time on a GH_I64_ID heap:
    the drain is the (key, id) order of the input, including the most
    negative and most positive keys and runs of equal keys."""
    k = 64
    n = 3000
    st = W.Stream(41)
    keys = (st.u64(n) >> np.uint64(54)).astype(np.int64) - 512     # many equal keys
    keys[:4] = [-(1 << 63), (1 << 63) - 1, -(1 << 63), (1 << 63) - 1]
    ids = np.arange(n, dtype=np.uint64)[::-1].copy()
    ent = G.pack_i64(keys, ids)
    h = G.Heap(k, n, keytype=G.GH_I64_ID)
    d = G.to_device_u64(ent)
    h.insert(d[: 2 * 1000])
    h.insert(d[2 * 1000: 2 * 1001])
    h.insert(d[2 * 1001:])
    assert h.size() == n
    got = []
    out = torch.empty(2 * k, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    c_seq = [k, 1, 17, k - 1]
    i = 0
    while True:
        c = c_seq[i % len(c_seq)]
        i += 1
        h.delete_min(out, cnt, c=c)
        m = int(cnt.item())
        if m == 0:
            break
        got.append(G.to_host_u64(out, 2)[:m].copy())
    got = np.concatenate(got)
    assert np.array_equal(got, sort_entries(ent))
    kk, ii = G.unpack_i64(got)
    assert kk[0] == -(1 << 63) and kk[-1] == (1 << 63) - 1
    assert h.close() == G.GH_OK


@pytest.mark.parametrize("k", [32, 1024])
def test_wide_build_filter_and_mix(G, k):
    """Bulk build from sorted 16-byte entries, a concurrent mix, then a
    filter by key: the state equals the oracle's after each step."""
    n = 50 * k + 5
    st = W.Stream(50 + k)
    keys = (st.u64(n) >> np.uint64(40)).astype(np.int64) - (1 << 23)
    ent = sort_entries(G.pack_i64(keys, np.arange(n)))
    hs = G.HeapSet(k, [200 * k], keytype=G.GH_I64_ID)
    hs.build(0, G.to_device_u64(ent))
    assert hs.sync() == G.GH_OK
    oh = oracle.OracleHeap(k, wide=True)
    oh.build(ent)
    assert_same_state(hs, 0, oh, k)
    mix = W.to_wide(W.mixed_ops(100 * k, k, seed=60 + k, first_id=n), 61 + k, 24)
    hs, out, counts, log = run_gpu(mix, k, max_keys=200 * k, workgroups=32, heapset=hs)
    # the build took no ticket: the mix's tickets start at 0
    oh2 = replay_and_compare(mix, k, out, counts, log, oracle_heap=oh)
    live = check_gpu_state(hs, 0, k)
    assert np.array_equal(live, oracle_live(oh2))
    bound_key = int(G.unpack_i64(live[live.shape[0] // 3:live.shape[0] // 3 + 1])[0][0])
    word = (bound_key + (1 << 64) if bound_key < 0 else bound_key) ^ (1 << 63)
    kept, _ = hs.filter(0, word)
    assert hs.sync() == G.GH_OK
    assert int(kept.item()) == oh2.filter(word)
    assert_same_state(hs, 0, oh2, k)
    assert hs.close() == G.GH_OK


def test_wide_graph_replays_equal_eager(G):
    """A GH_I64_ID submission captured as a HIP graph and replayed three
    times (arena restored between replays): every replay equals the eager
    run."""
    k = 256
    ops = _mixed_wide(20 * k, 80 * k, k, seed=77)
    hs = G.HeapSet(k, [200 * k], keytype=G.GH_I64_ID, stream=torch.cuda.Stream())
    with torch.cuda.stream(hs.stream):
        snap = hs.arena.clone()
        d_ops, n, keys, out, counts = G.ops_to_device(ops)
        hs.submit(d_ops, n, keys, out, counts, workgroups=64)
        assert hs.sync() == G.GH_OK
        eager = out.clone()
        eager_counts = counts.clone()
        g = hs.submit_graph(d_ops, n, keys, out, counts, workgroups=64)
        for rep in range(3):
            hs.arena.copy_(snap)
            out.fill_(-1)
            counts.zero_()
            torch.cuda.synchronize()
            hs.graph_launch(g)
            assert hs.sync() == G.GH_OK
            torch.cuda.synchronize()
            assert torch.equal(out, eager), "replay %d" % rep
            assert torch.equal(counts, eager_counts), "replay %d" % rep
    assert hs.close() == G.GH_OK


def test_wide_served_replays_per_heap(G):
    """The served form on a GH_I64_ID set (saturated, with inserts that wait
    for memory): every heap's admitted requests, replayed in ticket order on
    its own oracle, give the same deleteMins."""
    k, nh, nreq = 64, 8, 2000
    pre, reqs, sizes = W.served_stream(nh, k, nreq, seed=51, rate_per_s=None, min_log2=6,
                                       max_log2=11, max_ins_log2=9)
    pre = W.to_wide(pre, 52, 20)
    reqs = W.to_wide(reqs, 53, 20)
    caps = W.served_capacity(sizes)
    hs = G.HeapSet(k, caps, keytype=G.GH_I64_ID)
    d = G.ops_to_device(pre)
    hs.submit(*d[:5], workgroups=64)
    assert hs.sync() == G.GH_OK
    r, n, keys, out, recs, max_ops = G.requests_to_device(reqs)
    _p("wide served heaps=%d requests=%d" % (nh, nreq))
    hs.serve(r, n, keys, out, recs, max_ops, workgroups=48)
    assert hs.sync() == G.GH_OK
    out = G.to_host_u64(out, 2)
    recs = G.recs_to_host(recs, n)
    assert np.all((recs["flags"] & (G.REQ_ADMITTED | G.REQ_REJECTED)) != 0)
    for h in range(nh):
        oh = oracle.OracleHeap(k, wide=True)
        for i in np.flatnonzero(pre.heap == h):
            oh.insert(pre.keys[int(pre.off[i]):int(pre.off[i]) + int(pre.n[i])])
        sel = np.flatnonzero((reqs.heap == h) & ((recs["flags"] & G.REQ_ADMITTED) != 0))
        sel = sel[np.argsort(recs["first_ticket"][sel], kind="stable")]
        for i in sel:
            o = int(reqs.off[i])
            if reqs.kind[i] == W.OP_INSERT:
                oh.insert(reqs.keys[o:o + int(reqs.n[i])])
            else:
                want = oh.delete_min(int(reqs.n[i]) or None)
                c = int(recs["count"][i])
                assert c == want.shape[0], "heap %d request %d count" % (h, i)
                assert np.array_equal(out[o:o + c], want), "heap %d request %d output" % (h, i)
    assert hs.close() == G.GH_OK


def test_wide_sssp_refused(G):
    """heap_sssp needs 8-byte entries (dist << 32 | vertex)."""
    lib = G.load_library()
    hs = G.HeapSet(64, [1024], keytype=G.GH_I64_ID)
    buf = torch.zeros(1024, dtype=torch.int64, device="cuda")
    p = buf.data_ptr()
    rc = lib.heap_sssp(hs.h, 4, p, p, p, 0, p, p, 64, p, None, None)
    assert rc == G.GH_EINVAL
    assert hs.close() == G.GH_OK
