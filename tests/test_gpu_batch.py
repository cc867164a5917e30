"""Batched counting: one persistent launch over many hypergraphs, replayed
from a captured HIP graph, against per-graph counts and the oracle."""
import numpy as np
import pytest

from conftest import expected_counts
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


@pytest.fixture(scope="module")
def small_batch():
    specs = synth.batch_specs(num_graphs=24, e_lo=300, e_hi=6000)
    graphs = [synth.generate(s) for s in specs]
    graphs.append(synth.random_small(3, 70, 10, 1, 6))      # every pattern
    graphs.append(synth.from_lists([[0, 1]], 2, "single"))   # no hyperwedge
    return graphs


def test_batch_matches_oracle_and_per_graph(htri, small_batch):
    B = htri.Batch(small_batch)
    want = np.array([core.OracleGraph(g.offsets, g.members, g.num_vertices).count(per_edge=False).H
                     for g in small_batch])
    for sched in ((512, 256, 0), (256, 128, 1), (512, 128, 1), (256, 256, 0)):
        got, ms = B.count_patterns(sched, use_graph=False)
        assert np.array_equal(got, want), sched
        per, ms2 = B.count_per_graph(sched)
        assert np.array_equal(per, want), sched
    nw = B.wedges()
    for g, x in zip(small_batch, nw):
        G = htri.graph_load(g.offsets, g.members, g.num_vertices)
        assert G.build_wedges()[0] == x


def test_graph_replays_agree_with_eager(htri, small_batch):
    """Replay the captured launch several times, with eager work and
    synchronisations in between; every replay gives the eager counts."""
    import torch
    B = htri.Batch(small_batch)
    eager, _ = B.count_patterns((512, 256, 1), use_graph=False)
    x = torch.arange(1 << 16, device="cuda", dtype=torch.float32)
    for r in range(5):
        got, ms = B.count_patterns((512, 256, 1), use_graph=True)
        assert np.array_equal(got, eager), r
        y = (x * r).sum().item()                       # eager work between replays
        torch.cuda.synchronize()
        assert y >= 0


def test_full_pipeline_replay_matches_oracle(htri, small_batch):
    """Step 1, work items and closure of every graph captured in one HIP
    graph: every replay (with eager work and synchronisations in between)
    gives the oracle's counts, as does the graph-by-graph baseline, and the
    batch's other plans still count correctly afterwards."""
    import torch
    B = htri.Batch(small_batch)
    want = np.array([core.OracleGraph(g.offsets, g.members, g.num_vertices).count(per_edge=False).H
                     for g in small_batch])
    x = torch.arange(1 << 16, device="cuda", dtype=torch.float32)
    for sched in ((512, 256, 1), (256, 128, 0)):
        for r in range(4):
            got, ms = B.count_full(sched)
            assert np.array_equal(got, want), (sched, r)
            assert ms > 0
            y = (x * r).sum().item()
            torch.cuda.synchronize()
            assert y >= 0
        per, wall = B.count_full_per_graph(sched)
        assert np.array_equal(per, want), sched
        got, _ = B.count_full(sched)                  # replay after the graphs were rebuilt eagerly
        assert np.array_equal(got, want), sched
    got, _ = B.count_patterns((512, 256, 0), use_graph=True)
    assert np.array_equal(got, want)
    assert np.array_equal(B.wedges(), [G.build_wedges()[0] for G in
                                       (htri.graph_load(g.offsets, g.members, g.num_vertices) for g in small_batch)])


def test_size_class_schedules_and_their_cache(htri, small_batch, tmp_path):
    """Per-size-class autotuning: the classes follow the hyperwedge counts,
    the tuned schedules go to a JSON cache that a second call reads back
    without timing, and counting with one schedule per class (eager or
    graph-replayed) gives the oracle's counts."""
    import json
    B = htri.Batch(small_batch)
    nw = B.wedges()
    cls = B.size_classes()
    assert np.array_equal(cls, np.where(nw < 2 ** 18, 0, np.where(nw < 2 ** 21, 1, 2)))
    path = str(tmp_path / "schedules.json")
    sc, ms, hit = B.autotune_classes(repeats=1, cache_path=path)
    assert not hit
    doc = json.load(open(path))
    assert doc["format"] == "htri-batch-schedules" and len(doc["classes"]) == 3
    for c in range(3):
        assert (doc["classes"][c]["chunk"], doc["classes"][c]["partners"], doc["classes"][c]["order"]) == sc[c]
        if (cls == c).any():
            assert ms[c] > 0
    sc2, _, hit2 = B.autotune_classes(repeats=1, cache_path=path)
    assert hit2 and sc2 == sc
    want = np.array([core.OracleGraph(g.offsets, g.members, g.num_vertices).count(per_edge=False).H
                     for g in small_batch])
    for use_graph in (False, True, True):
        got, _ = B.count_classes(sc, use_graph=use_graph)
        assert np.array_equal(got, want), use_graph


def test_autotune_picks_a_valid_schedule(htri, small_batch):
    B = htri.Batch(small_batch[:8])
    sched, ms = B.autotune(repeats=1)
    assert sched[0] in (256, 512) and sched[1] in (128, 256) and sched[2] in (0, 1)
    assert ms > 0
    got, _ = B.count_patterns(sched)
    want = np.array([core.OracleGraph(g.offsets, g.members, g.num_vertices).count(per_edge=False).H
                     for g in small_batch[:8]])
    assert np.array_equal(got, want)


def test_batch_load_errors(htri):
    bad = synth.from_lists([[0, 1], [1, 0]], 2)
    with pytest.raises(htri.HtriError) as e:
        htri.Batch([synth.from_lists([[0, 1], [1, 2]], 3), bad], flags=0)
    assert e.value.code == -4 and "graph 1" in str(e.value)


def test_full_batch_of_512_graphs(htri):
    """The 512-graph batch at full size: the batched replay equals the
    per-graph launches and the oracle's full count on every graph."""
    specs = synth.batch_specs()
    graphs = [synth.generate(s) for s in specs]
    print(f"\n[batch512] {len(graphs)} graphs, {sum(g.num_edges for g in graphs)} hyperedges", flush=True)
    B = htri.Batch(graphs)
    sched, _ = B.autotune(repeats=1)
    got, _ = B.count_patterns(sched, use_graph=True)
    per, _ = B.count_per_graph((512, 256, 0))
    assert np.array_equal(got, per)
    # every graph against the oracle's full count, stored by input SHA-256
    nw = B.wedges()
    for q, g in enumerate(graphs):
        rec = expected_counts(g.sha256())
        assert rec is not None, f"no stored oracle count for graph {q}"
        assert got[q].tolist() == rec["H"], q
        assert nw[q] == rec["summary"][0], q
    # step 1 + items + closure of all 512 graphs in one captured replay
    full, ms = B.count_full(sched)
    assert np.array_equal(full, got)
    full2, ms2 = B.count_full(sched)
    assert np.array_equal(full2, got)
    print(f"[batch512] full pipeline replay {ms:.1f} / {ms2:.1f} ms", flush=True)
    # one schedule per size class, tuned and replayed
    print(f"[batch512] size classes {np.bincount(B.size_classes(), minlength=3).tolist()}", flush=True)
    sc, cms, _ = B.autotune_classes(repeats=1)
    bycls, cls_ms = B.count_classes(sc)
    assert np.array_equal(bycls, got)
    print(f"[batch512] class schedules {sc} ({cms}), replay {cls_ms:.1f} ms", flush=True)
