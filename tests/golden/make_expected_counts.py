"""Write the oracle's exact counts for the large parity workloads.

Run once on the CPU; the GPU parity tests read the result.  Only the CPU
oracle (``oracle/``) and the seeded input generators (``synth``) are used: no
value here comes from the HIP library.

For each workload the hypergraph is drawn, its input SHA-256 taken, the
oracle's plain two-step count run over owner ranges that tile [0, m) (the
hyper-triangles whose smallest id lies in the range; the ranges sum to the
full count), and the sum stored under the input SHA-256 in
``expected_counts.json``:

    H           int64[21] per-pattern counts, [0] = total
    summary     [|wedges|, |intersection|, |inclusion|, W, max omega, m]
    t_sha256    SHA-256 of the per-hyperedge counts t (int64 little endian,
                normalised ids, every pattern): the whole array, compared
                element by element through its digest
    t_sum       sum of t (= 3 * H[0])
    t_sample    [[x, t_x], ...] for a few hundred hyperedges (seeded draw plus
                the largest t)

Each range's partial H and t is saved under --partial-dir before the next
one starts, so an interrupted run resumes where it stopped.

    python tests/golden/make_expected_counts.py --workload tags --threads 6
    python tests/golden/make_expected_counts.py --workload tags_eval
    python tests/golden/make_expected_counts.py --workload batch
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(os.path.dirname(_HERE))
sys.path.insert(0, _ROOT)

from oracle import core as oc  # noqa: E402
from paper_2504_02271_amd import synth  # noqa: E402

OUT = os.path.join(_HERE, "expected_counts.json")


def t_digest(t: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(t, dtype="<i8").tobytes()).hexdigest()


def t_sample(t: np.ndarray, n: int = 256, top: int = 32) -> list:
    rng = np.random.default_rng(12345)
    idx = set(rng.choice(t.shape[0], size=min(n, t.shape[0]), replace=False).tolist())
    idx.update(np.argsort(t, kind="stable")[-top:].tolist())
    return [[int(x), int(t[x])] for x in sorted(idx)]


def load_table() -> dict:
    if os.path.exists(OUT):
        with open(OUT) as f:
            return json.load(f)
    return {}


def save_table(tab: dict) -> None:
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, OUT)


def count_one(hg: synth.HyperGraph, workload: str, threads: int, chunks: int,
              partial_dir: str, log, sample: bool = True) -> dict:
    sha = hg.sha256()
    t0 = time.time()
    og = oc.OracleGraph(hg.offsets, hg.members, hg.num_vertices, dedupe=True)
    og.build_wedges(nthreads=threads)
    summ = og.summary()
    log(f"{workload}: m={og.m} wedges={summ[0]} W={summ[3]} step1 {time.time() - t0:.1f}s")
    m = og.m
    bounds = np.linspace(0, m, chunks + 1).round().astype(np.int64)
    pdir = os.path.join(partial_dir, sha[:16])
    os.makedirs(pdir, exist_ok=True)
    H = np.zeros(21, np.int64)
    t = np.zeros(m, np.int64)
    for c in range(chunks):
        i0, i1 = int(bounds[c]), int(bounds[c + 1])
        path = os.path.join(pdir, f"range_{i0}_{i1}.npz")
        if os.path.exists(path):
            z = np.load(path)
            Hc, tc = z["H"], z["t"]
        else:
            t1 = time.time()
            r = og.count_range(i0, i1, nthreads=threads)
            Hc, tc = r.H, r.t
            np.savez_compressed(path + ".tmp.npz", H=Hc, t=tc)
            os.replace(path + ".tmp.npz", path)
            log(f"{workload}: owners [{i0}, {i1}) {Hc[0]} triangles in {time.time() - t1:.1f}s")
        H += Hc
        t += tc
    assert int(t.sum()) == 3 * int(H[0]), "sum of t must be 3T"
    return {
        "workload": workload,
        "sha256": sha,
        "num_vertices": int(hg.num_vertices),
        "m": int(m),
        "removed": int(og.removed),
        "summary": [int(x) for x in summ],
        "H": [int(x) for x in H],
        "t_sha256": t_digest(t),
        "t_sum": int(t.sum()),
        "t_sample": t_sample(t) if sample else [],
        "oracle_seconds": round(time.time() - t0, 1),
    }


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True, help="tags | tags_eval | coauth | tiny | batch")
    ap.add_argument("--threads", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    ap.add_argument("--chunks", type=int, default=0, help="owner ranges (default by size)")
    ap.add_argument("--partial-dir", default=os.path.join(tempfile.gettempdir(), "htri_expected_partial"))
    ap.add_argument("--batch-range", default="0:512", help="graphs a:b of the 512-graph batch")
    args = ap.parse_args()

    def log(msg: str) -> None:
        print(time.strftime("%H:%M:%S"), msg, flush=True)

    tab = load_table()
    if args.workload == "batch":
        a, b = (int(x) for x in args.batch_range.split(":"))
        specs = synth.batch_specs()[a:b]
        for g, spec in enumerate(specs, start=a):
            hg = synth.generate(spec)
            if hg.sha256() in tab:
                continue
            rec = count_one(hg, f"batch{g}", args.threads, args.chunks or 1, args.partial_dir, log,
                            sample=False)
            tab[rec["sha256"]] = rec
            if g % 16 == 15:
                save_table(tab)
        save_table(tab)
        return
    hg = synth.generate(synth.config(args.workload))
    chunks = args.chunks or (64 if hg.num_edges >= 1_000_000 else 1)
    rec = count_one(hg, args.workload, args.threads, chunks, args.partial_dir, log)
    tab = load_table()
    tab[rec["sha256"]] = rec
    save_table(tab)
    log(f"{args.workload}: H = {rec['H']}")


if __name__ == "__main__":
    main()
