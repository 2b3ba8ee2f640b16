"""GPU test of heap_filter_noalloc, the filter entry point that allocates
nothing (its workspace is the library's own device array): called through
the C ABI, its result equals heap_filter's (which takes a caller workspace)
bit for bit, on two calls in a row, the second on a smaller heap, and both
equal the oracle's filter.  A heap whose workspace would exceed the array is
refused before any launch."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1906_06504_amd import workloads as W

from heap_harness import replay_and_compare

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


def _twin_heaps(G, k, n_pre, n_mix, seed):
    """A set of two heaps that went through the same operations (the same
    records for each heap, so the same ticket order and the same live
    entries), and the oracle replaying heap 0's log."""
    pre = W.prefill_ops(n_pre, k, seed=seed)
    mix = W.mixed_ops(n_mix, k, seed=seed + 1, first_id=n_pre)
    ops = W.concat(pre, mix, k)
    both = W.multi_heap([ops, ops], k, W.Stream(seed + 2))
    hs = G.HeapSet(k, [n_pre + n_mix + 4 * k] * 2)
    d_ops, n, keys, out, counts = G.ops_to_device(both)
    log = G.new_log(n)
    hs.submit(d_ops, n, keys, out, counts, log, workgroups=64)
    assert hs.sync() == G.GH_OK
    lg = G.log_to_host(log, n)
    oh = replay_and_compare(both, k, G.to_host_u64(out), counts.cpu().numpy()[:n], lg, heap=0)
    return hs, oh


def _state(hs, i):
    m, s, _, _, nodes, pb = hs.read_state(i)
    return m, s, nodes[:m].copy(), pb.copy()


@pytest.mark.parametrize("k,sizes", [(256, ((900, 1500), (60, 90))),
                                     (1024, ((700, 900), (20, 30)))])
def test_noalloc_filter_equals_workspace_filter(G, k, sizes):
    lib = G.load_library()
    for call, (pre_b, mix_b) in enumerate(sizes):
        hs, oh = _twin_heaps(G, k, pre_b * k + 17, mix_b * k, seed=900 + 10 * call + k)
        m0, _, _, _, nodes0, pb0 = hs.read_state(0)
        live = np.sort(np.concatenate([nodes0[:m0].reshape(-1), pb0]))
        bound = int(live[(live.size * 3) // 5])
        _p("k=%d call %d: %d live entries, bound at the 60th percentile" % (k, call, live.size))
        kept0 = torch.zeros(1, dtype=torch.int64, device="cuda")
        rc = lib.heap_filter_noalloc(hs.h, 0, bound, ctypes.c_void_p(kept0.data_ptr()))
        assert rc == G.GH_OK, G.strerror(rc)
        kept1, _ = hs.filter(1, bound)
        assert hs.sync() == G.GH_OK
        want = oh.filter(bound)
        assert int(kept0.item()) == int(kept1.item()) == want
        a, b = _state(hs, 0), _state(hs, 1)
        assert (a[0], a[1]) == (b[0], b[1]) == (oh.m, oh.s)
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
        onodes, opb = oh.export()
        assert np.array_equal(a[3], opb)
        assert np.array_equal(a[2].reshape(-1), np.sort(live[live < np.uint64(bound)])[:a[0] * k])
        assert hs.close() == G.GH_OK


def test_noalloc_filter_refuses_a_heap_beyond_its_array(G):
    lib = G.load_library()
    k = 1024
    cap = 5 << 20   # needs about 80 MiB of workspace
    hs = G.HeapSet(k, [cap])
    need = int(lib.heap_filter_workspace_bytes(hs.h, 0))
    assert need > (64 << 20)
    assert lib.heap_filter_noalloc(hs.h, 0, 0, None) == G.GH_ENOMEM
    assert lib.heap_filter_noalloc(hs.h, 1, 0, None) == G.GH_EINVAL
    assert lib.heap_filter_noalloc(None, 0, 0, None) == G.GH_EINVAL
    assert hs.close() == G.GH_OK
