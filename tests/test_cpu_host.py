"""CPU-side checks: the HIP library loads and exports every declared entry
point, the host-side references (Philox, estimators, network gradient) are
pinned, and the input generators are deterministic."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from oracle import mlp_ref, sampling
from paper_2504_02271_amd import synth

HEADER = os.path.join(ROOT, "include", "htri.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(htri_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_2504_02271_amd import htri
    if not os.path.exists(htri.LIB_PATH):
        pytest.skip("libhtri.so not built here (run __graft_entry__.build())")
    lib = ctypes.CDLL(htri.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_constants_match_the_header():
    """Every HTRI_* constant the binding defines has the header's value, and
    the header's flag bits of one function do not collide."""
    from paper_2504_02271_amd import htri
    text = open(HEADER).read()
    defs = {k: int(v) for k, v in re.findall(r"#define\s+(HTRI_[A-Z0-9_]+)\s+(\d+)u?\b", text)}
    consts = {k: v for k, v in vars(htri).items() if re.fullmatch(r"HTRI_[A-Z0-9_]+", k) and isinstance(v, int)}
    assert len(consts) >= 10
    for k, v in consts.items():
        if k in defs:
            assert defs[k] == v, (k, defs[k], v)
        else:
            assert k == "HTRI_OK", k               # an enum value, not a #define
    load = [defs[k] for k in ("HTRI_DEDUPE_EDGES", "HTRI_INPUT_ON_DEVICE", "HTRI_OUTPUT_ON_DEVICE",
                              "HTRI_ORDER_INPUT", "HTRI_WIDE_TILE_KEYS")]
    count = [defs[k] for k in ("HTRI_OUTPUT_ON_DEVICE", "HTRI_COUNT_NO_WINDOW", "HTRI_COUNT_WINDOW_ALWAYS",
                               "HTRI_COUNT_INCLUSION_CLASSES", "HTRI_COUNT_OWNER_PROBE")]
    for bits in (load, count):
        assert all(b & (b - 1) == 0 for b in bits) and len(set(bits)) == len(bits)   # distinct single bits


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2504_02271_amd import htri
    monkeypatch.setattr(htri, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(htri, "_lib", None)
    with pytest.raises(ImportError):
        htri.load_library()


def test_status_strings_without_gpu():
    from paper_2504_02271_amd import htri
    if not os.path.exists(htri.LIB_PATH):
        pytest.skip("libhtri.so not built here")
    lib = htri.load_library()
    assert lib.htri_status_string(0) == b"ok"
    assert lib.htri_status_string(-4) == b"duplicate hyperedge"
    # argument checks run on the host and never touch the device
    h = ctypes.c_void_p()
    assert lib.htri_graph_load(None, 0, None, 0, 0, None, None, ctypes.byref(h)) == -1


# ---------------------------------------------------------------- Philox

def test_philox_known_answers():
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")):
        line = line.split("#", 1)[0].strip()
        if line:
            c, k, o = (part.split() for part in line.split("|"))
            rows.append(([int(x, 16) for x in c], [int(x, 16) for x in k], [int(x, 16) for x in o]))
    assert len(rows) == 3
    for c, k, o in rows:
        got = [int(v) for v in sampling.philox4x32_10(c, k)]
        assert got == o


def test_uniform_indices_are_exact_mulhi():
    u = sampling.draws_u64(42, 3, 2000)
    for N in (1, 7, 10**6, 2**40 + 3):
        idx = sampling.uniform_indices(42, 3, 2000, N)
        assert all(int(a) * N >> 64 == int(b) for a, b in zip(u, idx))
        assert idx.min() >= 0 and idx.max() < N


def test_uniform_estimator_without_replacement_limit_is_exact():
    """Closing every hyperwedge once and scaling by |wedges|/n recovers H."""
    from oracle import core
    g = synth.generate(synth.config("tiny"))
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    wi, wj, _ = o.wedges()
    cl = o.wedge_closure(wi, wj)
    est, _ = sampling.uniform_estimate(cl, wi.shape[0])
    assert np.allclose(est, o.count().H, rtol=0, atol=1e-6)


def test_uniform_estimator_is_unbiased_statistically():
    """Lemma 4.1: mean of independent estimates within 4 standard errors."""
    from oracle import core
    g = synth.generate(synth.config("tiny"))
    o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
    H = o.count().H
    wi, wj, _ = o.wedges()
    cl = o.wedge_closure(wi, wj)
    R, n = 64, 2000
    ests = []
    for seed in range(R):
        idx = sampling.uniform_indices(seed, 0, n, wi.shape[0])
        ests.append(sampling.uniform_estimate(cl[idx], wi.shape[0])[0])
    ests = np.array(ests)
    mean = ests.mean(axis=0)
    se = ests.std(axis=0, ddof=1) / np.sqrt(R)
    for p in range(21):
        if H[p] > 0 and se[p] > 0:
            assert abs(mean[p] - H[p]) < 4 * se[p] + 1e-9, (p, mean[p], H[p], se[p])


def test_relative_error_metric():
    exact = np.zeros(21)
    exact[[1, 9, 10]] = [4, 100, 10]
    est = exact.copy()
    est[9] = 110
    m, rel = sampling.relative_error(est, exact)
    assert abs(m - (0.1 / 3)) < 1e-12 and np.isnan(rel[1])


# ---------------------------------------------------------------- network

def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = rng.normal(scale=0.3, size=mlp_ref.NUM_PARAMS)
    X = rng.normal(size=(40, 16))
    y = rng.normal(size=40)
    L, g = mlp_ref.loss_grad(theta, X, y)
    assert abs(L - mlp_ref.loss(theta, X, y)) < 1e-12
    idx = rng.choice(mlp_ref.NUM_PARAMS, size=80, replace=False).tolist() + [mlp_ref.NUM_PARAMS - 1]
    fd = mlp_ref.finite_difference(theta, X, y, idx)
    assert np.allclose(g[idx], fd, rtol=1e-5, atol=1e-7)
    assert mlp_ref.NUM_PARAMS == 5313


def test_network_layout_matches_the_header():
    text = open(HEADER).read()
    assert f"#define HTRI_MODEL_NUM_PARAMS {mlp_ref.NUM_PARAMS}" in text


# ---------------------------------------------------------------- generators

def test_generators_deterministic_and_shaped():
    a = synth.generate(synth.config("coauth", 0.02))
    b = synth.generate(synth.config("coauth", 0.02))
    assert a.sha256() == b.sha256()
    sizes = np.diff(a.offsets)
    assert sizes.min() >= 2 and sizes.max() <= 25
    for x in range(0, a.num_edges, 97):
        e = a.edge(x)
        assert (np.diff(e) > 0).all()
    t = synth.generate(synth.config("tiny"))
    assert t.num_edges == 2000 and np.diff(t.offsets).min() >= 2 and np.diff(t.offsets).max() <= 5
    specs = synth.batch_specs(512)
    es = np.array([s.num_edges for s in specs])
    assert len(specs) == 512 and es.min() >= 1000 and es.max() <= 200000


class _OracleWedges:
    """Stand-in for a loaded graph: per-pattern forward closures of every
    hyperwedge from the oracle, in the order of the oracle's wedge list."""

    def __init__(self, g):
        from oracle import core
        o = core.OracleGraph(g.offsets, g.members, g.num_vertices)
        off, mem, _ = o.csr()
        rank = core.prec_rank(off, mem, g.num_vertices)
        wi, wj, _ = o.wedges()
        lo, hi = sampling.prec_wedge_order(rank, wi, wj)
        self.C = o.wedge_closure_ranked(rank, lo, hi)
        self.H = o.count().H
        self.num_wedges = lo.shape[0]

    def close_wedges(self, idx):
        return self.C[idx]


def _pattern_variance(C, H, q):
    """sum_p Var(c_p(w)/q(w)) / H_p^2 for one draw w ~ q (exact, by summation)."""
    live = H[1:] > 0
    c = C[:, 1:][:, live].astype(np.float64)
    h = H[1:][live].astype(np.float64)
    return float(((((c ** 2) / q[:, None]).sum(axis=0) - h ** 2) / h ** 2).sum())


def _importance_reference(C, H, nw):
    """u(w) = sqrt(sum_p (c_p(w) |W| / H_p)^2) / n over the patterns with H_p > 0
    (the quantity htri_wedge_importance returns as log1p)."""
    live = H[1:] > 0
    scale = np.where(live, nw / np.where(live, H[1:], 1), 0.0)
    return np.sqrt(((C[:, 1:] * scale) ** 2).sum(axis=1)) / max(live.sum(), 1)


def test_wedge_importance_minimises_the_pattern_variance():
    """The training target of the learned proposal: q proportional to
    wedge_importance gives a smaller summed relative variance than uniform,
    than q proportional to the total closure, and than perturbed versions
    of itself (it is the minimiser, by Cauchy-Schwarz)."""
    g = synth.random_small(5, 160, 30, 1, 6)
    G = _OracleWedges(g)
    u = _importance_reference(G.C.astype(np.float64), G.H.astype(np.float64), G.num_wedges)
    assert u.shape == (G.num_wedges,) and (u >= 0).all()
    live = G.H[1:] > 0
    assert np.array_equal(u > 0, (G.C[:, 1:][:, live] > 0).any(axis=1))
    # one wedge's value from the definition
    w = int(np.argmax(u))
    want = np.sqrt(((G.C[w, 1:][live] * G.num_wedges / G.H[1:][live]) ** 2).sum()) / live.sum()
    assert np.isclose(u[w], want, rtol=1e-12)
    sup = u > 0
    C, H = G.C[sup], G.H
    q_opt = u[sup] / u[sup].sum()
    v_opt = _pattern_variance(C, H, q_opt)
    q_uni = np.full(sup.sum(), 1.0 / sup.sum())
    tot = C[:, 0].astype(np.float64)
    q_tot = (tot + 1e-12) / (tot + 1e-12).sum()
    assert v_opt <= _pattern_variance(C, H, q_uni) + 1e-9
    assert v_opt <= _pattern_variance(C, H, q_tot) + 1e-9
    rng = np.random.default_rng(0)
    for _ in range(5):
        q = q_opt * np.exp(rng.normal(scale=0.3, size=q_opt.shape[0]))
        q /= q.sum()
        assert v_opt <= _pattern_variance(C, H, q) + 1e-9


def test_pool_policy():
    from paper_2504_02271_amd import learn
    assert learn.pool_factor_for(1000, 10_000_000) == learn.POOL_FACTOR
    assert learn.pool_factor_for(100_000, 10_000_000) == 0.0


def test_clustering_coefficient_closed_forms():
    """Def. 5.1 through the library (host arithmetic, no GPU): a 2-uniform
    hypergraph is a simple graph, where the classical coefficient is
    3 * triangles / connected triples; a triangle of pairs gives 1; weights
    select patterns; invalid weights are rejected."""
    from oracle import brute
    from paper_2504_02271_amd import htri
    tri = [[0, 1], [1, 2], [0, 2]]
    H, _ = brute.count(tri)
    W = sum(math.comb(2, 2) for _ in range(3))           # each hyperedge meets the other two
    assert htri.clustering_coefficient(H, W) == pytest.approx(1.0)
    rng = np.random.default_rng(3)
    pairs = {tuple(sorted(rng.choice(12, size=2, replace=False).tolist())) for _ in range(30)}
    edges = [list(p) for p in sorted(pairs)]
    H, _ = brute.count(edges)
    deg = [sum(1 for f in edges if f != e and set(e) & set(f)) for e in edges]
    W = sum(d * (d - 1) // 2 for d in deg)
    assert htri.clustering_coefficient(H, W) == pytest.approx(3 * H[0] / W)
    eps = np.zeros(21)
    eps[17] = 0.5
    assert htri.clustering_coefficient(H, W, eps) == pytest.approx(1.5 * H[17] / W)
    assert htri.clustering_coefficient(H, 0) == 0.0
    bad = np.zeros(21)
    bad[3] = 1.5
    with pytest.raises(htri.HtriError):
        htri.clustering_coefficient(H, W, bad)


# ---------------------------------------------------------------- learned proposal replay

def _tiny_closures():
    """Forward closures of every hyperwedge of a small hypergraph in id order,
    by the brute-force triple scan (patterns by canonical region masks)."""
    from oracle import brute
    g = synth.random_small(2, 40, 12, 1, 5)
    E = brute.normalise([g.edge(x).tolist() for x in range(g.num_edges)])
    wedges = [(i, j) for i in range(len(E)) for j in range(i + 1, len(E)) if E[i] & E[j]]
    cl = np.zeros((len(wedges), 21), np.int64)
    for w, (i, j) in enumerate(wedges):
        for k in range(j + 1, len(E)):
            if E[i] & E[k] and E[j] & E[k]:
                p = brute.pattern_of(E[i], E[j], E[k])
                cl[w, p] += 1
                cl[w, 0] += 1
    H = cl.sum(axis=0)
    return cl, H


def test_learned_estimator_arithmetic():
    """The learned-proposal replay: probabilities sum to 1 and are positive
    with a uniform floor; with lam = 1 it is the uniform estimate over the
    pool; the draws follow q; and its mean over many seeds is unbiased for
    the brute-force counts (Lemma 4.1 with importance weights)."""
    cl, H = _tiny_closures()
    nw = cl.shape[0]
    rng = np.random.default_rng(0)
    scores = np.where(rng.random(nw) < 0.3, 0.0, rng.exponential(3.0, nw))
    pool = np.arange(nw, dtype=np.int64)
    close = lambda idx: cl[idx]
    est, se, q, u = sampling.learned_estimate(scores, pool, nw, 0.1, 7, 5000, close)
    assert abs(q.sum() - 1.0) < 1e-12 and (q > 0).all()
    assert (q[scores == 0] > 0).all()
    # lam = 1: the uniform estimate of the drawn pool members
    est1, _, q1, u1 = sampling.learned_estimate(scores, pool, nw, 1.0, 3, 4000, close)
    assert np.allclose(q1, 1.0 / nw, rtol=1e-12)
    assert np.allclose(est1, cl[u1].sum(axis=0) * nw / 4000.0, rtol=1e-12)
    # draws follow q: chi-square over the pool
    counts = np.bincount(u, minlength=nw)
    exp = 5000 * q
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < nw + 6 * np.sqrt(2 * nw), chi2
    # a uniform pool of half the wedges: unbiased for H over pool draws
    R = 400
    ests = []
    for s in range(R):
        pl = sampling.uniform_indices(1000 + s, 1, nw // 2, nw)
        ests.append(sampling.learned_estimate(scores[pl], pl, nw, 0.2, 2000 + s, 300, close)[0])
    ests = np.array(ests)
    m = ests.mean(axis=0)
    sem = ests.std(axis=0, ddof=1) / np.sqrt(R)
    for p in range(21):
        if H[p] > 0:
            assert abs(m[p] - H[p]) < 4.5 * sem[p] + 1e-9, (p, m[p], H[p], sem[p])
