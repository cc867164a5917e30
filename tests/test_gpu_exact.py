"""GPU parity of the exact path (CSR build, hyperwedges, closure + classify +
reduce) against the CPU oracle, element by element, through the C ABI."""
import math

import numpy as np
import pytest

from conftest import load_golden
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


def _orient(rank, a, b):
    lo = np.where(rank[a] < rank[b], a, b)
    hi = np.where(rank[a] < rank[b], b, a)
    return lo, hi


def check_exact(htri, g, flags=None, wedge_sample=None, nthreads=0, seed=0, windows=("off", "always", "auto")):
    """Full parity on one hypergraph, with the dense window forced off, forced
    on and chosen automatically; returns (GPU graph, oracle graph, counts)."""
    if flags is None:
        flags = htri.HTRI_DEDUPE_EDGES
    print(f"\n[check_exact] {g.name} m={g.num_edges} nnz={g.nnz} flags={flags}", flush=True)
    G = htri.graph_load(g.offsets, g.members, g.num_vertices, flags=flags)
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    # a0: normalised CSR, byte for byte, and the id map
    off, mem = G.csr()
    ooff, omem, orig = o.csr()
    assert G.num_edges == o.m and G.removed == o.removed
    assert np.array_equal(off, ooff) and np.array_equal(mem, omem)
    assert np.array_equal(G.edge_map(), orig)
    # a1: hyperwedges with omega; summary
    s = G.build_wedges()
    assert np.array_equal(s, o.summary()), (s, o.summary())
    src, dst, om = G.get_wedges()
    if src.shape[0]:
        pick = np.random.default_rng(seed).choice(src.shape[0], size=min(50, src.shape[0]), replace=False)
        ls, ld, lw = G.get_wedge_list(pick)
        assert np.array_equal(ls, src[pick]) and np.array_equal(ld, dst[pick]) and np.array_equal(lw, om[pick])
    wi, wj, wo = o.wedges()
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    got = np.lexsort((hi, lo))
    assert np.array_equal(lo[got], wi) and np.array_equal(hi[got], wj) and np.array_equal(om[got], wo)
    # a2 + a3: per-pattern and per-hyperedge counts, per-wedge closure
    r = o.count(nthreads=nthreads)
    if flags & htri.HTRI_ORDER_INPUT:
        rank = np.arange(o.m, dtype=np.int64)
    else:
        rank = core.prec_rank(ooff, omem, g.num_vertices)
    assert (rank[src] < rank[dst]).all()
    idx = np.arange(src.shape[0])
    if wedge_sample is not None and wedge_sample < idx.shape[0]:
        rng = np.random.default_rng(seed)
        idx = np.sort(rng.choice(idx.shape[0], size=wedge_sample, replace=False))
    want = o.wedge_closure_ranked(rank, src[idx], dst[idx])[:, 0]
    for win in windows:
        for probe in ("middle", "owner"):
            counts, pe, pw = G.count_patterns(per_edge=True, per_wedge=True, window=win, probe=probe)
            st = G.closure_stats()
            print(f"[check_exact]   window={win} probe={probe}: rows {st[5]}, wedges inside {st[6]}, "
                  f"enumerated {st[11]}, middle-centric {st[12]}, in-list {st[13]}", flush=True)
            if win == "always" and G.num_wedges > 0 and 3 <= G.num_edges <= 16384:
                assert st[5] == G.num_edges
            if win == "off":
                assert st[5] == 0
            if probe == "owner" or st[5] == G.num_edges:
                assert st[12] == 0 and st[13] == 0
            else:
                # every hyperwedge outside the window is in the in-list
                assert st[12] == 1 and st[13] == st[8], (st[12], st[13], st[8])
            assert np.array_equal(counts, r.H), (win, probe, counts, r.H)
            assert np.array_equal(pe, r.t), (win, probe)
            assert int(pw.astype(np.int64).sum()) == int(counts[0])
            assert np.array_equal(pw[idx].astype(np.int64), want), (win, probe)
    # classes with an inclusion hyperwedge only (patterns 1-8), searched around those hyperwedges
    incl_mask = 0x1FE
    ci, pei, _ = G.count_patterns(mask=incl_mask, per_edge=True, window="inclusion_classes")
    ri = o.count(nthreads=nthreads, edge_mask=incl_mask)
    assert np.array_equal(ci[1:9], r.H[1:9]) and (ci[9:] == 0).all() and ci[0] == r.H[1:9].sum(), (ci, r.H)
    assert np.array_equal(pei, ri.t)
    return G, o, counts


def test_tiny_workload(htri):
    check_exact(htri, synth.generate(synth.config("tiny")))


def test_tiny_input_order(htri):
    check_exact(htri, synth.generate(synth.config("tiny")),
                flags=htri.HTRI_DEDUPE_EDGES | htri.HTRI_ORDER_INPUT)


@pytest.mark.parametrize("seed", range(12))
def test_small_universes_every_pattern(htri, seed):
    g = synth.random_small(seed, 50 + 5 * seed, 5 + 3 * seed, 1, 6)
    check_exact(htri, g)


def test_all_patterns_covered_together(htri):
    tot = np.zeros(21, np.int64)
    for seed in range(12):
        g = synth.random_small(seed, 50 + 5 * seed, 5 + 3 * seed, 1, 6)
        G = htri.graph_load(g.offsets, g.members, g.num_vertices)
        G.build_wedges()
        tot += G.count_patterns()[0]
    assert (tot[1:] > 0).all(), tot


def test_printed_examples(htri):
    for name, want in (("fig6_coauthorship.txt", {10: 5, 12: 2}), ("fig7_email.txt", {5: 3})):
        edges, _, _ = load_golden(name)
        g = synth.from_lists(edges)
        G, _, counts = check_exact(htri, g)
        for p, c in want.items():
            assert counts[p] == c


def test_unsorted_members_with_repeats(htri):
    g = synth.generate(synth.config("tiny"))
    rng = np.random.default_rng(1)
    edges = []
    for x in range(g.num_edges):
        e = list(g.edge(x))
        if x % 3 == 0:
            e = e + [e[0]]           # a repeated id counts once
        rng.shuffle(e)
        edges.append(e)
    edges += [list(reversed(edges[5])), edges[7]]   # duplicate hyperedges
    h = synth.from_lists(edges, g.num_vertices, "tiny-shuffled")
    G, o, _ = check_exact(htri, h)
    assert G.removed == 2


def test_heavy_clique_multichunk_and_wide_edges(htri):
    """Owners whose forward list spans several LDS chunks, partner pieces that
    need the chunk's rank range, and hyperedges too wide for stored masks."""
    rng = np.random.default_rng(7)
    edges = []
    for x in range(1500):                        # all share vertex 0
        extra = rng.choice(np.arange(1, 300), size=int(rng.integers(1, 4)), replace=False)
        edges.append([0] + sorted(extra.tolist()))
    for x in range(400):                         # background over the same pool
        edges.append(sorted(rng.choice(np.arange(1, 300), size=3, replace=False).tolist()))
    edges.append(list(range(100, 400)))          # 300 vertices: no stored mask
    edges.append(list(range(150, 290)))          # 140 vertices, inside the previous one
    edges.append([0] + list(range(1, 200)))      # wide hyperedge with the hub
    g = synth.from_lists(edges, 400, "clique")
    G, o, counts = check_exact(htri, g, wedge_sample=20000)
    hub = len({tuple(e) for e in edges if e[0] == 0})   # distinct hyperedges with vertex 0
    assert hub > 1000 and counts[0] >= math.comb(hub, 3)


def test_partial_window_with_middle_probing(htri):
    """A dense hub (1,100 hyperedges through vertex 0) over a sparse
    background: the top 2,048 ranks form the dense window and the other
    owners are probed around the middle, with middles inside the window (the
    window's per-hyperedge counters receive the probing's k-role counts)."""
    rng = np.random.default_rng(21)
    edges = []
    for x in range(1100):
        extra = rng.choice(np.arange(1, 400), size=int(rng.integers(1, 4)), replace=False)
        edges.append([0] + sorted(extra.tolist()))
    for x in range(3900):
        edges.append(sorted(rng.choice(np.arange(400, 20000), size=3, replace=False).tolist()))
    for x in range(200):   # links between the hub's vertices and the background
        edges.append(sorted([int(rng.integers(1, 400))] + rng.choice(np.arange(400, 20000), size=2,
                                                                       replace=False).tolist()))
    g = synth.from_lists(edges, 20000, "partial-window")
    G, o, counts = check_exact(htri, g, wedge_sample=20000, windows=("auto",))
    G.count_patterns(per_edge=True, window="auto")
    st = G.closure_stats()
    assert st[5] == 2048 and 0 < st[8] < G.num_wedges and st[12] == 1, st


def test_empty_and_wedgeless(htri):
    g = synth.from_lists([], 5, "empty")
    G = htri.graph_load(g.offsets, g.members, 5)
    assert G.num_edges == 0
    assert G.build_wedges().tolist() == [0, 0, 0, 0, 0, 0]
    counts, pe, pw = G.count_patterns(per_edge=True, per_wedge=True)
    assert (counts == 0).all() and pe.shape == (0,) and pw.shape == (0,)
    g = synth.from_lists([[0, 1], [2, 3], [4]], 5, "disjoint")
    G = htri.graph_load(g.offsets, g.members, 5)
    assert G.build_wedges()[0] == 0
    counts, pe, _ = G.count_patterns(per_edge=True)
    assert (counts == 0).all() and (pe == 0).all()
    g = synth.from_lists([[0, 1], [1, 2]], 3, "one-wedge")
    check_exact(htri, g)


def test_errors(htri):
    g = synth.from_lists([[0, 1], [1, 0], [2]], 3)
    with pytest.raises(htri.HtriError) as e:
        htri.graph_load(g.offsets, g.members, 3, flags=0)
    assert e.value.code == -4
    g = synth.from_lists([[0, 1], [], [2]], 3)
    with pytest.raises(htri.HtriError) as e:
        htri.graph_load(g.offsets, g.members, 3)
    assert e.value.code == -3
    g = synth.from_lists([[0, 1], [5]], 3)
    with pytest.raises(htri.HtriError) as e:
        htri.graph_load(g.offsets, g.members, 3)
    assert e.value.code == -2
    bad = np.array([0, 2, 1], np.int64)
    with pytest.raises(htri.HtriError) as e:
        htri.graph_load(bad, np.zeros(2, np.int32), 3)
    assert e.value.code == -1
    g = synth.from_lists([[0, 1], [1, 2]], 3)
    G = htri.graph_load(g.offsets, g.members, 3)
    with pytest.raises(htri.HtriError) as e:
        G.count_patterns()
    assert e.value.code == -8
    G.build_wedges()
    with pytest.raises(htri.HtriError) as e:
        G.count_patterns(per_wedge=True, window="inclusion_classes")
    assert e.value.code == -1


def test_pattern_mask_for_per_edge_counts(htri):
    g = synth.random_small(3, 120, 12, 1, 6)
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    for mask in ((1 << 9), (1 << 1) | (1 << 5) | (1 << 17), 0x1FFFFE & ~(1 << 9)):
        r = o.count(edge_mask=mask)
        for win in ("off", "always"):
            counts, pe, _ = G.count_patterns(mask=mask, per_edge=True, window=win)
            assert np.array_equal(counts, r.H), (mask, win)
            assert np.array_equal(pe, r.t), (mask, win)
        ci, pei, _ = G.count_patterns(mask=mask, per_edge=True, window="inclusion_classes")
        assert np.array_equal(ci[1:9], r.H[1:9])
        assert np.array_equal(pei, o.count(edge_mask=mask & 0x1FE).t), mask


def test_device_input_and_output(htri):
    import torch
    g = synth.generate(synth.config("tiny"))
    off = torch.from_numpy(g.offsets).cuda()
    mem = torch.from_numpy(g.members).cuda()
    G = htri.graph_load(off, mem, g.num_vertices, flags=htri.HTRI_DEDUPE_EDGES | htri.HTRI_INPUT_ON_DEVICE)
    G.build_wedges()
    counts, pe, pw = G.count_patterns(per_edge=True, per_wedge=True, device_out=True)
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    r = o.count()
    assert np.array_equal(counts, r.H)
    assert np.array_equal(pe.cpu().numpy(), r.t)
    assert int(pw.sum().item()) == int(r.H[0])


def test_coauthorship_workload(htri):
    """|V|=1e5, |E|=5e5, sizes TPL[2,25], Zipf(1.1) head: every count exact,
    per-wedge closures on a sample, and bit-identical repeat runs."""
    g = synth.generate(synth.config("coauth"))
    G, o, counts = check_exact(htri, g, wedge_sample=5000)
    c2, pe2, pw2 = G.count_patterns(per_edge=True, per_wedge=True)
    c3, pe3, pw3 = G.count_patterns(per_edge=True, per_wedge=True)
    assert np.array_equal(c2, c3) and np.array_equal(pe2, pe3) and np.array_equal(pw2, pw3)


def test_wide_tile_keys(htri):
    """The 64-bit tile keys (the form graphs of 2^24 or more hyperedges take)
    against the oracle, and the same hyperwedges as the 32-bit keys on the
    co-authorship workload."""
    wide = htri.HTRI_DEDUPE_EDGES | htri.HTRI_WIDE_TILE_KEYS
    check_exact(htri, synth.generate(synth.config("tiny")), flags=wide)
    check_exact(htri, synth.generate(synth.config("tiny")), flags=wide | htri.HTRI_ORDER_INPUT)
    g = synth.generate(synth.config("coauth"))
    res = []
    for flags in (htri.HTRI_DEDUPE_EDGES, wide):
        G = htri.graph_load(g.offsets, g.members, g.num_vertices, flags=flags)
        s = G.build_wedges()
        src, dst, om = G.get_wedges()
        res.append((s, src, dst, om, G.count_patterns(per_edge=True)[:2]))
        G.close()
    (s0, a0, b0, w0, (c0, t0)), (s1, a1, b1, w1, (c1, t1)) = res
    assert np.array_equal(s0, s1)
    assert np.array_equal(a0, a1) and np.array_equal(b0, b1) and np.array_equal(w0, w1)
    assert np.array_equal(c0, c1) and np.array_equal(t0, t1)


def test_owner_with_many_incidences(htri):
    """An owner meeting more incidences than an LDS tile holds (4,600) is
    sorted by a block of its own: hyperedge 0 (3,000 vertices, no stored mask)
    owns its hyperwedges in input order; a 1,501-vertex partner gives a large
    omega and a 101-vertex one uses all four mask words."""
    edges = [list(range(3000)), list(range(0, 3000, 2)) + [3000], list(range(100)) + [5000]]
    edges += [[i, 3001 + (i % 50)] for i in range(3000)]
    g = synth.from_lists(edges, 5001, "many-incidences")
    for flags in (htri.HTRI_DEDUPE_EDGES | htri.HTRI_ORDER_INPUT, htri.HTRI_DEDUPE_EDGES):
        check_exact(htri, g, flags=flags)


def test_owners_on_both_sides_of_the_block_limit(htri):
    """Large owners in one graph on both sides of the 16,384 incidences one
    block sorts in LDS, in input order: hyperedge 0 (22,120 incidences) goes
    through the global sort, hyperedge 1 (10,311, no stored mask) and
    hyperedge 3 (3,120, 120 vertices: four mask words) through the block
    sort, hyperedge 2 (600) through a tile; then the same graph ordered by
    delta, and with the 64-bit keys that send every large owner to the
    global sort."""
    edges = [list(range(3000)), list(range(0, 3000, 2)) + [5000], list(range(100)) + [5000], list(range(100, 220))]
    edges += [[i, 3000 + (7 * i + 13 * c) % 2000] for i in range(3000) for c in range(6)]
    edges += [[i, 3000 + (7 * i + 13 * c) % 2000] for i in range(100, 220) for c in range(6, 26)]
    g = synth.from_lists(edges, 5001, "block-limit")
    d = htri.HTRI_DEDUPE_EDGES
    for flags in (d | htri.HTRI_ORDER_INPUT, d, d | htri.HTRI_ORDER_INPUT | htri.HTRI_WIDE_TILE_KEYS):
        check_exact(htri, g, flags=flags, windows=("off", "auto"))


@pytest.mark.parametrize("name", ["small0", "small5", "small9", "small11", "tiny", "clique", "coauth"])
def test_class_targeted_ttt_counts(htri, name):
    """Count-DenseTTT (patterns 9-16 by vertex groups and thick pairs; 9 alone
    by its closed form), and Count-SparseTTT (patterns 17-20, the closure with
    every hit holding a common vertex dropped), against the oracle's full
    count, with the per-hyperedge counts of the sparse patterns."""
    if name.startswith("small"):
        q = int(name[5:])
        g = synth.random_small(q, 50 + 5 * q, 5 + 3 * q, 1, 6)
    elif name == "clique":
        rng = np.random.default_rng(9)
        edges = [[0] + sorted(rng.choice(np.arange(1, 200), size=2, replace=False).tolist()) for _ in range(900)]
        edges += [[0, 1, 2] + sorted(rng.choice(np.arange(3, 90), size=3, replace=False).tolist()) for _ in range(300)]
        edges.append(list(range(50, 250)))
        g = synth.from_lists(edges, 260, "clique")
    elif name == "coauth":
        g = synth.generate(synth.config("coauth"))
    else:
        g = synth.generate(synth.config("tiny"))
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    r = o.count(edge_mask=0x1E0000)
    H = r.H
    cd, _, _ = G.count_patterns(window="dense_ttt")
    assert np.array_equal(cd[9:17], H[9:17]), (cd, H)
    assert (cd[1:9] == 0).all() and (cd[17:] == 0).all() and cd[0] == cd[1:].sum()
    dense_ms = G.last_timings()[2]
    cv, _, _ = G.count_patterns(window="common_vertex")
    assert cv[9] == H[9] and cv[0] == H[9]
    cs, pes, _ = G.count_patterns(window="sparse_ttt", per_edge=True, mask=0x1E0000)
    assert np.array_equal(cs[17:21], H[17:21]) and (cs[1:17] == 0).all(), (cs, H)
    assert np.array_equal(pes, r.t)
    sparse_ms = G.last_timings()[2]
    G.count_patterns()
    full_ms = G.last_timings()[2]
    print(f"\n[ttt] {name}: dense {dense_ms:.2f} ms, sparse {sparse_ms:.2f} ms, full closure {full_ms:.2f} ms; "
          f"H9 {H[9]}", flush=True)
    with pytest.raises(htri.HtriError):
        G.count_patterns(window="dense_ttt", per_edge=True)
