"""The no-allocation entry point (htri_estimate_uniform_noalloc) against the
allocating one (htri_estimate, uniform proposal) and the oracle's replay of
the same Philox draws: two calls in a row, the second with fewer samples."""
import numpy as np
import pytest

from oracle import core, sampling
from paper_2504_02271_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def htri():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2504_02271_amd import htri as h
    h.load_library()
    return h


def test_noalloc_uniform_estimate_matches_htri_estimate(htri):
    import torch
    g = synth.generate(synth.config("coauth", 0.1))
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    off, mem, _ = o.csr()
    rank = core.prec_rank(off, mem, g.num_vertices)
    wi, wj, _ = o.wedges()
    lo, hi = sampling.prec_wedge_order(rank, wi, wj)
    nw = lo.shape[0]
    est_t = torch.full((21,), -1.0, dtype=torch.float64, device="cuda")
    se_t = torch.full((21,), -1.0, dtype=torch.float64, device="cuda")
    for seed, n in ((3, 30000), (4, 700)):         # the second call is smaller
        G.estimate_uniform_noalloc(n, seed, est_t, se_t)
        torch.cuda.synchronize()
        got, got_se = est_t.cpu().numpy(), se_t.cpu().numpy()
        want, want_se, _ = G.estimate(num_samples=n, seed=seed, proposal=0)
        assert np.array_equal(got, want), (seed, n, got, want)
        assert np.allclose(got_se, want_se, rtol=1e-12, atol=1e-9)
        idx = sampling.uniform_indices(seed, 0, n, nw)
        ref, ref_se = sampling.uniform_estimate(o.wedge_closure_ranked(rank, lo[idx], hi[idx]), nw)
        assert np.array_equal(got, ref)
        assert np.allclose(got_se, ref_se, rtol=1e-9, atol=1e-9)
    G.close()


def test_noalloc_refusals_and_empty_graph(htri):
    import torch
    g = synth.from_lists([[0, 1], [2, 3]], 4)
    G = htri.graph_load(g.offsets, g.members, 4)
    with pytest.raises(htri.HtriError) as e:
        G.estimate_uniform_noalloc(10)
    assert e.value.code == -8                        # no hyperwedges built yet
    G.build_wedges()
    with pytest.raises(htri.HtriError) as e:
        G.estimate_uniform_noalloc(0)
    assert e.value.code == -1
    est, se = G.estimate_uniform_noalloc(10)        # no hyperwedge at all: zeros
    torch.cuda.synchronize()
    assert (est.cpu().numpy() == 0).all() and (se.cpu().numpy() == 0).all()
