"""Appro-adv (Algorithm 7, proposal 2 of htri_estimate) against the
oracle's replay of the same Philox draws: the draw split, the per-class
forward closures and the mixed-class counts around inclusion hyperwedges,
bit for bit."""
import numpy as np
import pytest

from oracle import brute, core, sampling
from paper_2504_02271_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def htri():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2504_02271_amd import htri as h
    h.load_library()
    return h


def _replay_setup(g):
    edges = [g.edge(x).tolist() for x in range(g.num_edges)]
    E = brute.normalise(edges)
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    off, mem, _ = o.csr()
    rank = core.prec_rank(off, mem, g.num_vertices)
    wi, wj, wo = o.wedges()
    lo, hi = sampling.prec_wedge_order(rank, wi, wj)
    sizes = np.diff(off)
    k_or = np.minimum(wi, wj).astype(np.int64) * (1 << 32) + np.maximum(wi, wj)
    order = np.argsort(k_or, kind="stable")
    k_lib = np.minimum(lo, hi).astype(np.int64) * (1 << 32) + np.maximum(lo, hi)
    om = wo[order][np.searchsorted(k_or[order], k_lib)]
    incl = om == np.minimum(sizes[lo], sizes[hi])
    t_pos, c_pos = np.flatnonzero(~incl), np.flatnonzero(incl)
    cpart = {}
    for a, b in zip(lo[incl].tolist(), hi[incl].tolist()):
        cpart.setdefault(a, set()).add(b)
        cpart.setdefault(b, set()).add(a)

    def close_fwd(pos):
        return o.wedge_closure_ranked(rank, lo[pos], hi[pos])

    def cross(cls, pos):
        return np.array([sampling.adv_cross_count(E, rank, int(lo[q]), int(hi[q]), cpart, cls) for q in pos]
                        ).reshape(-1, 21)
    return o, t_pos, c_pos, close_fwd, cross


@pytest.mark.parametrize("name", ["small3", "small9", "coauth"])
def test_appro_adv_matches_oracle_replay(htri, name):
    if name == "coauth":
        g = synth.generate(synth.config("coauth", 0.1))
        runs = ((0, 20000), (5, 3000))
    else:
        g = synth.random_small(int(name[5:]), 120, 12, 1, 6)
        runs = ((0, 400), (17, 2500), (3, 60))
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    s = G.build_wedges()
    o, t_pos, c_pos, close_fwd, cross = _replay_setup(g)
    assert (t_pos.shape[0], c_pos.shape[0]) == (int(s[1]), int(s[2]))
    for seed, alpha in runs:
        est, se, ms = G.estimate(num_samples=alpha, seed=seed, proposal=2)
        want, alphas = sampling.appro_adv(seed, alpha, t_pos, c_pos, close_fwd, cross)
        assert list(htri.adv_split(int(s[1]), int(s[2]), alpha)) == alphas
        assert np.array_equal(est, want), (name, seed, est, want)
        assert np.isfinite(se).all() and (se >= 0).all()
        print(f"\n[adv] {name} seed {seed} alpha {alpha} split {alphas}: total {est[0]:.1f}", flush=True)
    G.close()


def test_appro_adv_refuses_the_exact_inclusion_flag(htri):
    g = synth.random_small(3, 60, 10, 1, 5)
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    with pytest.raises(htri.HtriError) as e:
        G.estimate(num_samples=100, proposal=2, exact_inclusion=True)
    assert e.value.code == -1
