"""Pins for the oracle's Appro-adv (Algorithm 7): the draw split of line 4,
the per-class attribution (each hyper-triangle of a class is attributed to
exactly one hyperwedge of the type its class is drawn from), and
unbiasedness over many seeds -- against the brute-force triple scan."""
import numpy as np
import pytest

from oracle import brute, core, sampling
from paper_2504_02271_amd import synth


def _setup(seed, m=70, nv=9):
    g = synth.random_small(seed, m, nv, 1, 5)
    edges = [g.edge(x).tolist() for x in range(g.num_edges)]
    E = brute.normalise(edges)
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    off, mem, _ = o.csr()
    rank = core.prec_rank(off, mem, g.num_vertices)
    wi, wj, wo = o.wedges()
    lo, hi = sampling.prec_wedge_order(rank, wi, wj)
    sizes = np.diff(off)
    key = {(min(a, b), max(a, b)): w for a, b, w in zip(wi.tolist(), wj.tolist(), wo.tolist())}
    om = np.array([key[(min(a, b), max(a, b))] for a, b in zip(lo.tolist(), hi.tolist())])
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
    H, _ = brute.count(edges)
    return dict(E=E, o=o, rank=rank, lo=lo, hi=hi, t_pos=t_pos, c_pos=c_pos, cpart=cpart, close_fwd=close_fwd,
                cross=cross, H=H)


def test_split_of_the_budget():
    assert sampling.adv_split(3, 1, 16) == [9, 1, 3, 3]
    assert sampling.adv_split(100, 0, 50) == [50, 0, 0, 0]
    assert sampling.adv_split(1000, 1, 100) == [100, 1, 1, 1]      # tiny shares round up to one draw
    assert sampling.adv_split(0, 5, 10) == [0, 10, 0, 0]
    a = sampling.adv_split(4000, 1000, 100000)
    assert a == [64000, 4000, 16000, 16000]


@pytest.mark.parametrize("seed", [0, 3, 7, 12])
def test_every_triangle_of_a_class_is_attributed_once(seed):
    """Summed over every hyperwedge of the type drawn for each class, the
    attributed counts are exactly the class's pattern counts."""
    d = _setup(seed)
    H = d["H"]
    assert d["c_pos"].shape[0] > 5 and d["t_pos"].shape[0] > 5
    fT = d["close_fwd"](d["t_pos"]).sum(axis=0)
    fC = d["close_fwd"](d["c_pos"]).sum(axis=0)
    xT = d["cross"]("TTC", d["t_pos"]).sum(axis=0)
    xC = d["cross"]("TCC", d["c_pos"]).sum(axis=0)
    for p in range(9, 21):
        assert fT[p] == H[p], p          # TTT: the earliest hyperwedge is intersection-type
    assert fC[1] == H[1]                 # CCC: the earliest is inclusion-type
    for p in (6, 7, 8):
        assert xT[p] == H[p], p
    for p in (2, 3, 4, 5):
        assert xC[p] == H[p], p
    assert xT[0] == H[6:9].sum() and xC[0] == H[2:6].sum()
    assert (H[1:9] > 0).sum() >= 4, H     # the family exercises the mixed classes


def test_appro_adv_is_unbiased():
    d = _setup(5, m=90, nv=10)
    H = d["H"].astype(np.float64)
    R = 300
    ests = np.array([sampling.appro_adv(1000 + s, 60, d["t_pos"], d["c_pos"], d["close_fwd"], d["cross"])[0]
                     for s in range(R)])
    m = ests.mean(axis=0)
    sem = ests.std(axis=0, ddof=1) / np.sqrt(R)
    for p in range(21):
        if H[p] > 0 and sem[p] > 0:
            assert abs(m[p] - H[p]) < 4.5 * sem[p], (p, m[p], H[p], sem[p])
        if H[p] == 0:
            assert m[p] == 0
