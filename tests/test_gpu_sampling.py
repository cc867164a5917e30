"""GPU parity of the sampling path (closure of drawn hyperwedges, uniform and
learned estimators) and of the proposal network kernels."""
import numpy as np
import pytest

from oracle import core, features_ref, mlp_ref, sampling
from paper_2504_02271_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def htri():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2504_02271_amd import htri as h
    h.load_library()
    return h


def _setup(htri, g):
    G = htri.graph_load(g.offsets, g.members, g.num_vertices)
    G.build_wedges()
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    off, mem, _ = o.csr()
    rank = core.prec_rank(off, mem, g.num_vertices)
    return G, o, rank


def test_wedge_order_is_prec_order(htri):
    g = synth.generate(synth.config("tiny"))
    G, o, rank = _setup(htri, g)
    src, dst, _ = G.get_wedges()
    wi, wj, _ = o.wedges()
    lo, hi = sampling.prec_wedge_order(rank, wi, wj)
    assert np.array_equal(src, lo) and np.array_equal(dst, hi)


@pytest.mark.parametrize("name", ["tiny", "small", "clique", "coauth"])
def test_close_listed_wedges(htri, name):
    if name == "tiny":
        g = synth.generate(synth.config("tiny"))
    elif name == "small":
        g = synth.random_small(4, 90, 14, 1, 6)
    elif name == "clique":
        rng = np.random.default_rng(9)
        edges = [[0] + sorted(rng.choice(np.arange(1, 200), size=2, replace=False).tolist()) for _ in range(900)]
        edges.append(list(range(50, 250)))
        g = synth.from_lists(edges, 260, "clique")
    else:
        g = synth.generate(synth.config("coauth"))
    print(f"\n[close_listed_wedges] {name}", flush=True)
    G, o, rank = _setup(htri, g)
    src, dst, _ = G.get_wedges()
    rng = np.random.default_rng(1)
    n = min(3000, src.shape[0])
    idx = rng.choice(src.shape[0], size=n, replace=False)
    got = G.close_wedges(idx)
    want = o.wedge_closure_ranked(rank, src[idx], dst[idx])
    assert np.array_equal(got, want)


def test_uniform_estimate_matches_oracle_draws(htri):
    """Same Philox draws on both sides: the estimate is bit-identical."""
    g = synth.generate(synth.config("coauth", 0.1))
    G, o, rank = _setup(htri, g)
    wi, wj, _ = o.wedges()
    lo, hi = sampling.prec_wedge_order(rank, wi, wj)
    nw = lo.shape[0]
    for seed, n in ((0, 500), (7, 4321), (123456789, 20000)):
        est, se, ms = G.estimate(num_samples=n, seed=seed, proposal=0)
        idx = sampling.uniform_indices(seed, 0, n, nw)
        cl = o.wedge_closure_ranked(rank, lo[idx], hi[idx])
        want, wse = sampling.uniform_estimate(cl, nw)
        assert np.array_equal(est, want), (seed, est, want)
        assert np.allclose(se, wse, rtol=1e-9, atol=1e-9)
        assert ms > 0


def test_uniform_estimate_unbiased(htri):
    g = synth.generate(synth.config("coauth", 0.1))
    G, o, rank = _setup(htri, g)
    H = o.count().H
    R = 48
    ests = np.array([G.estimate(budget=0.01, seed=s, proposal=0)[0] for s in range(R)])
    mean = ests.mean(axis=0)
    se = ests.std(axis=0, ddof=1) / np.sqrt(R)
    for p in range(21):
        if H[p] > 0 and se[p] > 0:
            assert abs(mean[p] - H[p]) < 4.5 * se[p], (p, mean[p], H[p], se[p])


def test_whole_graph_sample_is_exact_in_expectation_limit(htri):
    """Sampling with q = 1/|wedges| and every wedge closed gives H exactly
    when the draws cover all wedges once (explicit list)."""
    g = synth.generate(synth.config("tiny"))
    G, o, rank = _setup(htri, g)
    nw = G.num_wedges
    cl = G.close_wedges(np.arange(nw))
    est, _ = sampling.uniform_estimate(cl, nw)
    assert np.allclose(est, o.count().H, rtol=0, atol=1e-6)


# ---------------------------------------------------------------- features and network

def test_features_match_reference(htri):
    import torch
    g = synth.random_small(6, 150, 30, 2, 7)
    G, o, rank = _setup(htri, g)
    X = G.wedge_features().cpu().numpy()
    src, dst, _ = G.get_wedges()
    off, mem, _ = o.csr()
    wi, wj, wo = o.wedges()
    ref = features_ref.features(off, mem, g.num_vertices, rank, wi, wj, wo, src, dst)
    assert X.shape == ref.shape
    assert np.allclose(X, ref, rtol=1e-5, atol=1e-5)


def _rand_rows(n, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 16)).astype(np.float32)
    X[:, 15] = 1.0
    y = (np.abs(X[:, :4]).sum(axis=1) + rng.normal(scale=0.1, size=n)).astype(np.float32)
    return X, y


def test_network_forward_matches_float64(htri):
    import torch
    m = htri.Model(seed=3)
    theta = m.get_params().astype(np.float64)
    X, _ = _rand_rows(5000)
    out = m.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = mlp_ref.forward(theta, X)
    assert np.allclose(out, ref, rtol=1e-4, atol=1e-4)


def test_network_gradient_matches_float64(htri):
    """Loss and every parameter gradient of the GPU backward kernels against
    the float64 reference (relative error of the gradient vector <= 1e-4)."""
    import torch
    m = htri.Model(seed=5)
    theta = m.get_params().astype(np.float64)
    X, y = _rand_rows(3000, 1)
    L, g = m.loss_grad(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda())
    Lr, gr = mlp_ref.loss_grad(theta, X, y)
    assert abs(L - Lr) <= 1e-5 * max(1.0, abs(Lr))
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
    assert np.allclose(g, gr, rtol=1e-3, atol=1e-6)


def test_training_reduces_loss(htri):
    import torch
    m = htri.Model(seed=1)
    X, y = _rand_rows(20000, 2)
    Xt, yt = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    L0, _ = m.loss_grad(Xt, yt)
    m.train(Xt, yt, steps=300, batch=1024, lr=3e-3, seed=4)
    L1, _ = m.loss_grad(Xt, yt)
    assert L1 < 0.2 * L0, (L0, L1)


def test_learned_estimate_unbiased(htri):
    """Importance sampling with an untrained (arbitrary) proposal, with and
    without a candidate pool: the mean of many estimates is within 4.5
    standard errors of the exact counts."""
    g = synth.generate(synth.config("coauth", 0.1))
    G, o, rank = _setup(htri, g)
    H = o.count().H
    m = htri.Model(seed=2)
    for pool_factor in (0.0, 8.0):
        R = 48
        ests = np.array([G.estimate(budget=0.01, seed=100 + s, proposal=1, model=m, defensive_mix=0.2,
                                    pool_factor=pool_factor)[0] for s in range(R)])
        mean = ests.mean(axis=0)
        se = ests.std(axis=0, ddof=1) / np.sqrt(R)
        for p in range(21):
            if H[p] > 0 and se[p] > 0:
                assert abs(mean[p] - H[p]) < 4.5 * se[p], (pool_factor, p, mean[p], H[p], se[p])


def test_exact_inclusion_stratum_matches_oracle(htri):
    """Inclusion stratum closed exactly, the same Philox draws over the
    intersection-type hyperwedges: the estimate equals the oracle's sum
    of the exact stratum and the sampled part, bit for bit."""
    g = synth.generate(synth.config("coauth", 0.1))
    G, o, rank = _setup(htri, g)
    wi, wj, wo = o.wedges()
    lo, hi = sampling.prec_wedge_order(rank, wi, wj)
    nw = lo.shape[0]
    off, mem, _ = o.csr()
    size = np.diff(off)
    # omega of each hyperwedge in the library's order, from the oracle's list
    order = np.lexsort((np.maximum(wi, wj), np.minimum(wi, wj)))
    key = lambda a, b: np.minimum(a, b).astype(np.int64) * (1 << 32) + np.maximum(a, b)
    k_or = key(wi, wj)
    k_lib = key(lo, hi)
    pos = np.searchsorted(k_or[order], k_lib)
    omega = wo[order][pos]
    incl = omega == np.minimum(size[lo], size[hi])
    assert incl.sum() == G.build_wedges()[2]
    exact = o.wedge_closure_ranked(rank, lo[incl], hi[incl]).sum(axis=0).astype(np.float64)
    for seed, n in ((0, 700), (9, 5000)):
        est, _, _ = G.estimate(num_samples=n, seed=seed, proposal=0, exact_inclusion=True)
        idx = sampling.uniform_indices(seed, 0, n, nw)
        cl = o.wedge_closure_ranked(rank, lo[idx], hi[idx])
        cl[incl[idx]] = 0
        want, _ = sampling.uniform_estimate(cl, nw)
        assert np.array_equal(est, want + exact), (seed, est, want + exact)


def test_exact_inclusion_stratum_unbiased(htri):
    g = synth.generate(synth.config("coauth", 0.1))
    G, o, rank = _setup(htri, g)
    H = o.count().H
    m = htri.Model(seed=2)
    R = 48
    for proposal, model in ((0, None), (1, m)):
        ests = np.array([G.estimate(budget=0.01, seed=300 + s, proposal=proposal, model=model, defensive_mix=0.2,
                                    pool_factor=8.0, exact_inclusion=True)[0] for s in range(R)])
        mean = ests.mean(axis=0)
        se = ests.std(axis=0, ddof=1) / np.sqrt(R)
        for p in range(21):
            # a pattern with a handful of triangles is zero in most runs; its
            # sample standard error is then no guide, so it is not tested
            if H[p] > 0 and se[p] > 0 and (ests[:, p] != 0).mean() >= 0.5:
                assert abs(mean[p] - H[p]) < 4.5 * se[p], (proposal, p, mean[p], H[p], se[p])


# ---------------------------------------------------------------- learned proposal, exact replay

def _inclusion_mask(o, lo, hi):
    """Inclusion type (omega = smaller size) of each listed hyperwedge, from
    the oracle's own hyperwedge list."""
    wi, wj, wo = o.wedges()
    off, _, _ = o.csr()
    size = np.diff(off)
    key = lambda a, b: np.minimum(a, b).astype(np.int64) * (1 << 32) + np.maximum(a, b)
    k_or = key(wi, wj)
    order = np.argsort(k_or, kind="stable")
    pos = np.searchsorted(k_or[order], key(lo, hi))
    omega = wo[order][pos]
    return omega == np.minimum(size[lo], size[hi])


@pytest.mark.parametrize("pool_factor,lam,exact_incl", [(0.0, 0.1, False), (8.0, 0.1, False),
                                                        (8.0, 0.5, True), (0.0, 0.3, True)])
def test_learned_estimate_matches_oracle_replay(htri, pool_factor, lam, exact_incl):
    """The learned estimate replayed on the CPU from the same Philox pool and
    draws and the library's proposal scores: float64 CDF, inverse-CDF draws,
    realised probabilities and the Hansen-Hurwitz sum of the oracle's
    closures agree with htri_estimate.

    Tolerance: q_u = (C_u - C_{u-1}) / C_P is a difference of two prefix
    sums of the order of C_P, each carrying a rounding error of about
    2^-53 C_P that depends on the summation order (the library scans in
    parallel, the replay sequentially), so q_u -- about C_P / P -- agrees to
    a few P * 2^-53 relative; the estimate, a weighted mean of closures over
    q, inherits that bound.  8 P 2^-53 is used (1.5e-9 at P = 1.7e6)."""
    g = synth.generate(synth.config("coauth", 0.1))
    G, o, rank = _setup(htri, g)
    m = htri.Model(seed=2)
    wi, wj, _ = o.wedges()
    lo, hi = sampling.prec_wedge_order(rank, wi, wj)
    nw = lo.shape[0]
    incl = _inclusion_mask(o, lo, hi)
    exact = o.wedge_closure_ranked(rank, lo[incl], hi[incl]).sum(axis=0).astype(np.float64)

    def close(idx):
        cl = o.wedge_closure_ranked(rank, lo[idx], hi[idx])
        if exact_incl:
            cl[incl[idx]] = 0
        return cl

    for seed, n in ((0, 1500), (11, 12000)):
        est, se, _ = G.estimate(num_samples=n, seed=seed, proposal=1, model=m, defensive_mix=lam,
                                pool_factor=pool_factor, exact_inclusion=exact_incl)
        if pool_factor > 0:
            P = int(np.floor(pool_factor * n + 0.5))
            pool = sampling.uniform_indices(seed, 1, P, nw)
        else:
            pool = np.arange(nw, dtype=np.int64)
        scores = G.proposal_scores(m, pool)
        assert (scores >= 0).all()
        want, wse, q, u = sampling.learned_estimate(scores, pool, nw, lam, seed, n, close)
        assert abs(q.sum() - 1.0) < 1e-12 and (q[u] > 0).all() and (q > 0).all()
        if exact_incl:
            want = want + exact
        rtol = 8.0 * pool.shape[0] * 2.0 ** -53
        rel = np.abs(est - want) / np.maximum(np.abs(want), 1e-300)
        print(f"\n[learned replay] P={pool.shape[0]} n={n} max rel diff {rel[want != 0].max():.3e} "
              f"(tolerance {rtol:.1e})", flush=True)
        assert np.allclose(est, want, rtol=rtol, atol=1e-9), (seed, est, want)
        assert np.allclose(se, wse, rtol=1e-9, atol=1e-6)
    # the scores themselves against the float64 network on float64 features
    off, mem, _ = o.csr()
    wo = o.wedges()[2]
    pick = np.random.default_rng(5).choice(nw, size=1500, replace=False)
    X = features_ref.features(off, mem, g.num_vertices, rank, wi, wj, wo, lo[pick], hi[pick])
    f = mlp_ref.forward(m.get_params().astype(np.float64), X)
    ref = np.expm1(np.clip(f, 0.0, 30.0))
    assert np.allclose(G.proposal_scores(m, pick), ref, rtol=1e-3, atol=1e-4)


def test_learned_estimate_refuses_zero_floor(htri):
    """Without the uniform floor (lambda = 0) a hyperwedge the network scores
    at or below zero could never be drawn: the library refuses it."""
    g = synth.generate(synth.config("tiny"))
    G, _, _ = _setup(htri, g)
    m = htri.Model(seed=1)
    with pytest.raises(htri.HtriError) as e:
        G.estimate(num_samples=100, seed=0, proposal=1, model=m, defensive_mix=0.0)
    assert e.value.code == -1 and "defensive_mix" in str(e.value)
    est, _, _ = G.estimate(num_samples=100, seed=0, proposal=1, model=m, defensive_mix=1e-6)
    assert np.isfinite(est).all()


def test_model_save_load_round_trip(htri, tmp_path):
    """Raw float32 parameters plus JSON metadata: a saved model loads back
    bit for bit; a truncated file or foreign metadata is refused."""
    import json
    m = htri.Model(seed=11)
    path = str(tmp_path / "proposal.f32")
    m.save(path)
    meta = json.load(open(path + ".json"))
    assert meta["num_params"] == htri.HTRI_MODEL_NUM_PARAMS and meta["layers"] == [16, 64, 64, 1]
    raw = np.fromfile(path, dtype="<f4")
    assert np.array_equal(raw, m.get_params())
    m2 = htri.Model(seed=99)
    m2.load(path)
    assert np.array_equal(m2.get_params(), m.get_params())
    with open(path, "r+b") as fh:
        fh.truncate(4 * 100)
    with pytest.raises(htri.HtriError) as e:
        m2.load(path)
    assert e.value.code == -1
    bad = str(tmp_path / "other.f32")
    raw.tofile(bad)
    with open(bad + ".json", "w") as fh:
        fh.write('{"format": "something-else"}')
    with pytest.raises(htri.HtriError):
        m2.load(bad)
    assert np.array_equal(m2.get_params(), m.get_params())


@pytest.mark.parametrize("with_total", [False, True])
def test_training_target_matches_oracle_closures(htri, with_total):
    """htri_wedge_importance: log1p(sqrt(sum_p (c_p(w) |W| / H_p)^2) / n) of
    every hyperwedge (with the total as a further term when asked), against
    the same quantity from the oracle's per-wedge closures, in float64."""
    g = synth.random_small(6, 400, 40, 1, 7)
    G, o, rank = _setup(htri, g)
    wi, wj, _ = o.wedges()
    lo, hi = sampling.prec_wedge_order(rank, wi, wj)
    C = o.wedge_closure_ranked(rank, lo, hi).astype(np.float64)
    H = o.count(per_edge=False).H
    nw = lo.shape[0]
    live = np.concatenate([[with_total and H[0] > 0], H[1:] > 0])
    scale = np.where(live, nw / np.where(H > 0, H, 1), 0.0)
    want = np.log1p(np.sqrt(((C * scale) ** 2).sum(axis=1)) / max(live.sum(), 1))
    got = G.wedge_importance(H, with_total=with_total).cpu().numpy()
    assert got.shape == want.shape
    assert np.allclose(got, want, rtol=2e-6, atol=1e-6)


def test_trained_proposal_beats_uniform_at_equal_time(htri):
    """What the trained network gains: the proposal trained as the benchmark
    trains it (20 co-authorship-shaped graphs), on the samplers' evaluation
    graph (tags-shaped, seed 5; exact counts from the oracle's stored full
    count, never from the library), with the inclusion stratum closed
    exactly and 0.1% of the hyperwedges drawn through a uniform candidate
    pool: at the same device time the learned sampler's mean per-pattern
    relative error over 16 seeds is below the uniform sampler's.  (On small
    graphs, or with every hyperwedge scored, the fixed scoring cost buys
    uniform sampling many more draws; the gain is a large-graph,
    small-budget one.)"""
    from conftest import expected_counts
    from paper_2504_02271_amd import learn
    ev = synth.generate(synth.config("tags_eval"))
    rec = expected_counts(ev.sha256())
    assert rec is not None, "no stored oracle count for the evaluation graph"
    exact = np.array(rec["H"], dtype=np.int64)
    train = [synth.generate(sp) for sp in synth.training_specs(20)]
    X, y = learn.training_rows(train, rows_per_graph=200_000, top_rows=50_000, seed=0, target="importance")
    del train
    model = learn.train_proposal(X, y, steps=3000, batch=4096, lr=2e-3, seed=0)
    del X, y
    G = htri.graph_load(ev.offsets, ev.members, ev.num_vertices)
    G.build_wedges()
    rows = learn.equal_time_study(G, exact, model, budgets=(0.001,), seeds=16, log=lambda s: print(s, flush=True),
                                  exact_inclusion=True, with_adv=False)
    r = rows[0]
    print(f"\n[learned-vs-uniform] learned {r['learned_rel_err']:.4f} ({r['learned_samples']} draws, "
          f"{r['learned_ms']:.2f} ms) vs uniform {r['uniform_rel_err']:.4f} ({r['uniform_samples']} draws, "
          f"{r['uniform_ms']:.2f} ms); total {r['learned_total_rel_err']:.2e} vs {r['uniform_total_rel_err']:.2e}",
          flush=True)
    assert r["pool_factor"] > 0
    assert r["uniform_ms"] <= 1.1 * r["learned_ms"]
    assert r["learned_rel_err"] < r["uniform_rel_err"], r
    G.close()
