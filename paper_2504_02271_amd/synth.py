"""Seeded synthetic hypergraph generators.

This module only draws inputs.  It holds none of the counting method's
arithmetic, so both the HIP path and the CPU oracle may read its output.

Every generator returns a hyperedge->vertex CSR as numpy arrays:

    offsets : int64[m+1]   hyperedge x owns members[offsets[x]:offsets[x+1]]
    members : int32[nnz]   vertex ids in [0, num_vertices)

Hyperedges are emitted as drawn (members of one hyperedge are distinct and
sorted, but two hyperedges may hold the same vertex set); removing duplicate
hyperedges is the loader's job, the same way the paper deduplicated its
datasets before counting (Section 6.1, "Datasets").

The shapes stand in for the paper's Table 4 datasets, which are not
available: co-authorship-like (sizes up to 25) and tags/threads-like (heavy
tail, sizes up to 100) hypergraphs.  Vertex popularity is a Zipf head plus a
uniform background:

    w_r = d_max * r**(-s) + beta,   r = 1..|V|

where beta spreads the incidences the head does not absorb evenly over all
vertices, so that the most popular vertex has expected degree ~d_max.
Popularity ranks are assigned to vertex ids by a random permutation so that
ids carry no degree information.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "HyperGraph", "GenSpec", "truncated_power_law_sizes", "generate",
    "config", "CONFIGS", "batch_specs", "training_specs", "sha256_of",
]


@dataclasses.dataclass
class HyperGraph:
    offsets: np.ndarray        # int64[m+1]
    members: np.ndarray        # int32[nnz]
    num_vertices: int
    name: str = ""

    @property
    def num_edges(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.members.shape[0])

    def edge(self, x: int) -> np.ndarray:
        return self.members[self.offsets[x]:self.offsets[x + 1]]

    def sha256(self) -> str:
        return sha256_of(self.offsets, self.members, self.num_vertices)


@dataclasses.dataclass(frozen=True)
class GenSpec:
    num_vertices: int
    num_edges: int
    size_lo: int
    size_hi: int
    gamma: Optional[float]      # None -> sizes uniform on [lo, hi]
    zipf_s: Optional[float]     # None -> uniform vertex popularity
    d_max: Optional[float]      # expected degree of the most popular vertex
    seed: int
    name: str = ""


def sha256_of(offsets: np.ndarray, members: np.ndarray, num_vertices: int) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(offsets, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(members, dtype=np.int32).tobytes())
    h.update(int(num_vertices).to_bytes(8, "little"))
    return h.hexdigest()


def truncated_power_law_sizes(rng: np.random.Generator, n: int, lo: int, hi: int,
                              gamma: Optional[float]) -> np.ndarray:
    """i.i.d. sizes with P(k) proportional to k**-gamma on [lo, hi] (uniform if gamma is None)."""
    if gamma is None:
        return rng.integers(lo, hi + 1, size=n, dtype=np.int64)
    ks = np.arange(lo, hi + 1, dtype=np.float64)
    p = ks ** (-gamma)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    u = rng.random(n)
    return (lo + np.searchsorted(cdf, u, side="right")).astype(np.int64)


def _expected_size(lo: int, hi: int, gamma: Optional[float]) -> float:
    ks = np.arange(lo, hi + 1, dtype=np.float64)
    if gamma is None:
        return float(ks.mean())
    p = ks ** (-gamma)
    return float((ks * p).sum() / p.sum())


def _popularity_weights(spec: GenSpec) -> np.ndarray:
    nv = spec.num_vertices
    if spec.zipf_s is None:
        return np.ones(nv, dtype=np.float64)
    r = np.arange(1, nv + 1, dtype=np.float64)
    head = float(spec.d_max) * r ** (-float(spec.zipf_s))
    nnz_est = spec.num_edges * _expected_size(spec.size_lo, spec.size_hi, spec.gamma)
    beta = max(nnz_est - head.sum(), 0.0) / nv
    return head + beta


def generate(spec: GenSpec) -> HyperGraph:
    """Draw one hypergraph.  Deterministic in ``spec`` (numpy PCG64)."""
    rng = np.random.default_rng(spec.seed)
    m = spec.num_edges
    nv = spec.num_vertices
    sizes = truncated_power_law_sizes(rng, m, spec.size_lo, spec.size_hi, spec.gamma)
    sizes = np.minimum(sizes, nv)
    offsets = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    nnz = int(offsets[-1])

    # popularity rank -> vertex id (random permutation)
    perm = rng.permutation(nv).astype(np.int64)
    w = _popularity_weights(spec)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    row = np.repeat(np.arange(m, dtype=np.int64), sizes)
    ranks = np.searchsorted(cdf, rng.random(nnz), side="right")
    np.minimum(ranks, nv - 1, out=ranks)
    key = row * nv + perm[ranks]

    # Without replacement inside a hyperedge: redraw repeated vertices until
    # every hyperedge holds distinct vertices.  Keys (hyperedge, vertex) are
    # kept sorted, so members come out sorted within each hyperedge.
    key.sort(kind="stable")
    for _ in range(10000):
        dup = np.flatnonzero(key[1:] == key[:-1]) + 1
        if dup.size == 0:
            break
        rr = np.searchsorted(cdf, rng.random(dup.size), side="right")
        np.minimum(rr, nv - 1, out=rr)
        key[dup] = (key[dup] // nv) * nv + perm[rr]
        key.sort(kind="stable")
    else:  # pragma: no cover - only with absurd parameters
        raise RuntimeError("could not draw distinct members")
    mem = key % nv

    return HyperGraph(offsets=offsets, members=mem.astype(np.int32), num_vertices=nv,
                      name=spec.name)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

CONFIGS = {
    # exact count, tiny: uniform sizes in [2,5], uniform membership, seed 0
    "tiny": GenSpec(1000, 2000, 2, 5, None, None, None, 0, "tiny"),
    # exact count, co-authorship-shaped
    "coauth": GenSpec(100_000, 500_000, 2, 25, 2.5, 1.1, 2000.0, 2, "coauth"),
    # exact count, tags/threads-shaped heavy tail (parity + roofline workload)
    "tags": GenSpec(1_000_000, 5_000_000, 2, 100, 2.2, 1.3, 10_000.0, 3, "tags"),
    # the same shape with the annotated 1e5 head (stress; oracle only spot-checks)
    "tags_stress": GenSpec(1_000_000, 5_000_000, 2, 100, 2.2, 1.3, 100_000.0, 3, "tags_stress"),
    # evaluation graph for the samplers: tags shape, new seed
    "tags_eval": GenSpec(1_000_000, 5_000_000, 2, 100, 2.2, 1.3, 10_000.0, 5, "tags_eval"),
}


def config(name: str, scale: float = 1.0) -> GenSpec:
    """A named workload, optionally shrunk by ``scale`` (|V|, |E| and d_max scale together)."""
    s = CONFIGS[name]
    if scale == 1.0:
        return s
    nv = max(16, int(round(s.num_vertices * scale)))
    ne = max(16, int(round(s.num_edges * scale)))
    dm = None if s.d_max is None else max(4.0, s.d_max * scale)
    return dataclasses.replace(s, num_vertices=nv, num_edges=ne, d_max=dm,
                               name=f"{s.name}@{scale:g}")


def batch_specs(num_graphs: int = 512, seed: int = 4, e_lo: float = 1e3,
                e_hi: float = 2e5) -> List[GenSpec]:
    """Many independent hypergraphs of uneven size: |E| log-uniform in [e_lo, e_hi],
    |V| = |E|/4, sizes power law on [2,20] (exponent 2.5), Zipf(1.1) head with
    d_max = |E|/250; graph g is drawn with seed 4000+g."""
    rng = np.random.default_rng(seed)
    es = np.rint(np.exp(rng.uniform(math.log(e_lo), math.log(e_hi), size=num_graphs))).astype(np.int64)
    out = []
    for g, ne in enumerate(es.tolist()):
        nv = max(8, ne // 4)
        out.append(GenSpec(nv, int(ne), 2, 20, 2.5, 1.1, max(4.0, ne / 250.0), 4000 + g,
                           f"batch{g}"))
    return out


def training_specs(count: int = 20, scale: float = 1.0) -> List[GenSpec]:
    """Co-authorship-shaped graphs (seeds 100..) that train the sampling proposal."""
    base = config("coauth", scale)
    return [dataclasses.replace(base, seed=100 + t, name=f"train{t}") for t in range(count)]


def from_lists(edges: List[List[int]], num_vertices: Optional[int] = None, name: str = "") -> HyperGraph:
    """Build a CSR from explicit vertex lists (used for printed examples and tests)."""
    sizes = [len(e) for e in edges]
    offsets = np.zeros(len(edges) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    members = np.array([v for e in edges for v in e], dtype=np.int32)
    if num_vertices is None:
        num_vertices = int(members.max()) + 1 if members.size else 0
    return HyperGraph(offsets, members, int(num_vertices), name)


def random_small(seed: int, num_edges: int, num_vertices: int, size_lo: int = 1,
                 size_hi: int = 6) -> HyperGraph:
    """Tiny hypergraphs over a small vertex universe, so that inclusion
    hyperwedges and every pattern occur.  May contain duplicate hyperedges."""
    rng = np.random.default_rng(seed)
    edges = []
    for _ in range(num_edges):
        k = int(rng.integers(size_lo, min(size_hi, num_vertices) + 1))
        edges.append(sorted(rng.choice(num_vertices, size=k, replace=False).tolist()))
    return from_lists(edges, num_vertices, f"small{seed}")
