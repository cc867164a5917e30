"""Error paths through the C ABI: device allocations that fail (through a
caller allocator that refuses the k-th request), sizes beyond the packed
adjacency, and the handle staying usable after an error."""
import ctypes

import numpy as np
import pytest

from oracle import core
from paper_2504_02271_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def htri():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2504_02271_amd import htri as h
    h.load_library()
    return h


class FailingMemory:
    """Device memory from torch's caching allocator that refuses request
    number `fail_at` (1-based; 0 = never) and counts what is outstanding."""

    def __init__(self, htri, fail_at: int):
        import torch
        self.torch = torch
        self.fail_at = fail_at
        self.calls = 0
        self.live = {}

        def _alloc(nbytes, stream, ctx):
            self.calls += 1
            if self.fail_at and self.calls == self.fail_at:
                return None
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream)
            except Exception:
                return None
            self.live[p] = int(nbytes)
            return p

        def _free(ptr, stream, ctx):
            if ptr:
                self.live.pop(ptr, None)
                torch.cuda.caching_allocator_delete(ptr)

        self._alloc_cb = htri.ALLOC_FN(_alloc)
        self._free_cb = htri.FREE_FN(_free)
        self.struct = htri.Allocator(self._alloc_cb, self._free_cb, None)

    def stream_handle(self) -> int:
        return int(self.torch.cuda.current_stream(0).cuda_stream)


def _run_all(htri, g, mem):
    G = htri.graph_load(g.offsets, g.members, g.num_vertices, mem=mem)
    try:
        G.build_wedges()
        counts, pe, _ = G.count_patterns(per_edge=True)
        return counts, pe
    finally:
        G.close()


def test_every_failing_allocation_returns_oom_and_frees(htri):
    """The allocator refuses its k-th request, for every k the pipeline
    (load, hyperwedges, count with per-hyperedge counts) makes: each run
    ends with HTRI_E_OOM naming the allocator -- or, where the count has a
    fallback for a middle-side list that does not fit (probing around the
    owner instead), with the oracle's counts -- and nothing stays allocated
    once the handle is freed."""
    g = synth.random_small(8, 160, 20, 1, 7)
    want = core.OracleGraph(g.offsets, g.members, g.num_vertices).count()
    probe = FailingMemory(htri, 0)
    counts, pe = _run_all(htri, g, probe)
    assert np.array_equal(counts, want.H) and np.array_equal(pe, want.t)
    total = probe.calls
    assert total > 5 and not probe.live
    refused = 0
    for k in range(1, total + 1):
        mem = FailingMemory(htri, k)
        try:
            counts, pe = _run_all(htri, g, mem)
        except htri.HtriError as e:
            assert e.code == -5, (k, e)
            assert "allocator" in str(e), (k, e)
            refused += 1
        else:
            assert np.array_equal(counts, want.H) and np.array_equal(pe, want.t), k
        assert not mem.live, (k, mem.live)
    assert refused >= total // 2, (refused, total)
    counts, pe = _run_all(htri, g, FailingMemory(htri, 0))
    assert np.array_equal(counts, want.H) and np.array_equal(pe, want.t)


def test_handle_usable_after_a_failed_count(htri):
    """A count that fails part-way (the allocator refuses once) leaves the
    handle usable: the same handle then counts correctly."""
    g = synth.random_small(9, 140, 18, 1, 7)
    want = core.OracleGraph(g.offsets, g.members, g.num_vertices).count()
    mem = FailingMemory(htri, 0)
    G = htri.graph_load(g.offsets, g.members, g.num_vertices, mem=mem)
    G.build_wedges()
    failed = False
    for off in range(1, 64):
        mem.fail_at = mem.calls + off
        try:
            counts, pe, _ = G.count_patterns(per_edge=True)
        except htri.HtriError as e:
            assert e.code == -5
            failed = True
            break
        assert np.array_equal(counts, want.H) and np.array_equal(pe, want.t)
    assert failed
    mem.fail_at = 0
    counts, pe, _ = G.count_patterns(per_edge=True)
    assert np.array_equal(counts, want.H) and np.array_equal(pe, want.t)
    G.close()
    assert not mem.live


def test_packed_adjacency_limit_is_unsupported(htri):
    """Ranks and omegas share one 32-bit word per hyperwedge: 2^20
    hyperedges (21 bits of rank) with one of 4,097 vertices (13 bits of
    omega) do not fit, and step 1 says so instead of counting wrong."""
    n1 = 1 << 20
    edges_off = np.zeros(n1 + 2, np.int64)
    edges_off[1:n1 + 1] = np.arange(1, n1 + 1)
    edges_off[n1 + 1] = n1 + 4097
    members = np.concatenate([np.arange(n1, dtype=np.int32), np.arange(4097, dtype=np.int32)])
    G = htri.graph_load(edges_off, members, n1)
    with pytest.raises(htri.HtriError) as e:
        G.build_wedges()
    assert e.value.code == -9 and "32-bit" in str(e.value)
    G.close()


def test_invalid_arguments(htri):
    lib = htri.load_library()
    assert lib.htri_count_patterns(None, 0, None, None, None, 0) == -1
    out = ctypes.c_double(0.0)
    assert lib.htri_clustering_coefficient(None, 1, None, ctypes.byref(out)) == -1
    g = synth.from_lists([[0, 1], [1, 2], [0, 2]], 3)
    G = htri.graph_load(g.offsets, g.members, 3)
    G.build_wedges()
    with pytest.raises(htri.HtriError) as e:
        G.close_wedges(np.array([5]))
    assert e.value.code == -1
    with pytest.raises(htri.HtriError) as e:
        G.enumerate(21)
    assert e.value.code == -1
    with pytest.raises(htri.HtriError) as e:
        G.estimate(num_samples=10, proposal=3)
    assert e.value.code == -1
    with pytest.raises(htri.HtriError) as e:
        G.estimate(num_samples=10, proposal=2, exact_inclusion=True)
    assert e.value.code == -1
    with pytest.raises(htri.HtriError) as e:
        G.local_clustering(np.full(21, -0.5))
    assert e.value.code == -1
    # the handle still works after the refusals
    counts, _, _ = G.count_patterns()
    assert counts[0] == 1
