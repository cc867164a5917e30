"""Training and evaluating the learned sampling proposal.

The network is trained on exact per-hyperwedge closure counts produced by the
exact path (target log(1 + c)), on graphs other than the one it is used on,
so the proposal is independent of the sample and the importance-sampling
estimator stays unbiased.  Every computation runs in the HIP library; torch
holds the device arrays.
"""
from __future__ import annotations

import math
import time
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np

from . import htri


def training_rows(graphs: Iterable, rows_per_graph: int = 200_000, top_rows: int = 50_000, seed: int = 0,
                  target: str = "importance"):
    """(X float32 [N,16], y float32 [N]) on the GPU for the proposal network.

    target "importance": y = log1p(u(w)) of htri_wedge_importance (u(w) =
    sqrt(sum_p (c_p(w) |W| / H_p)^2) / n_p, which minimises the summed
    squared relative errors of the per-pattern estimates), rows = a uniform
    sample of each graph's hyperwedges plus its top_rows most important ones
    (the wedges that carry the rare patterns are too few for a uniform sample
    to show them).  "importance_total": the same with the total count as one
    more term.  "closure": y = log1p of the exact forward closure count,
    uniform rows only."""
    import torch
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for g in graphs:
        G = htri.graph_load(g.offsets, g.members, g.num_vertices)
        G.build_wedges()
        n = G.num_wedges
        if n == 0:
            G.close()
            continue
        if target == "closure":
            _, _, pw = G.count_patterns(per_wedge=True, device_out=True)
            idx = np.sort(rng.choice(n, size=min(n, rows_per_graph), replace=False))
            idt = torch.from_numpy(idx).cuda()
            y = torch.log1p(pw[idt].to(torch.float32))
        elif target in ("importance", "importance_total"):
            # log1p(u(w)) of every hyperwedge, computed by the library
            H, _, _ = G.count_patterns()
            y_all = G.wedge_importance(H, with_total=target == "importance_total")
            uni = torch.from_numpy(rng.choice(n, size=min(n, rows_per_graph), replace=False)).cuda()
            top = torch.topk(y_all, k=min(n, top_rows)).indices
            idt = torch.unique(torch.cat([uni, top]))
            y = y_all[idt].contiguous()
        else:
            raise ValueError(f"unknown target {target!r}")
        X = G.wedge_features()
        xs.append(X[idt].contiguous())
        ys.append(y)
        del X
        G.close()
    return torch.cat(xs).contiguous(), torch.cat(ys).contiguous()


def train_proposal(X, y, steps: int = 3000, batch: int = 4096, lr: float = 2e-3, seed: int = 0,
                   lr_decay_every: int = 1000) -> "htri.Model":
    """Adam on the hand-written forward/backward kernels; the learning rate is
    halved every `lr_decay_every` steps."""
    m = htri.Model(seed=seed)
    done = 0
    cur = lr
    while done < steps:
        k = min(lr_decay_every, steps - done)
        m.train(X, y, steps=k, batch=batch, lr=cur, seed=seed * 7919 + done)
        done += k
        cur *= 0.5
    return m


def relative_error(est: np.ndarray, exact: np.ndarray) -> float:
    """Mean over the patterns with H > 0 of |H - est| / H."""
    H = exact[1:].astype(np.float64)
    nz = H > 0
    if not nz.any():
        return 0.0
    return float(np.mean(np.abs(H[nz] - est[1:][nz]) / H[nz]))


def _run(G, proposal, n, seed, model, mix, pool_factor, exact_inclusion=False):
    return G.estimate(num_samples=n, seed=seed, proposal=proposal, model=model, defensive_mix=mix,
                      pool_factor=pool_factor, exact_inclusion=exact_inclusion)


POOL_FACTOR = 32.0   # chosen on a validation graph (tags-shaped, seed 7), not the evaluation graph
FULL_SCORING_FRACTION = 0.1


def pool_factor_for(n: int, nw: int, pool_factor: float = POOL_FACTOR,
                    full_fraction: float = FULL_SCORING_FRACTION) -> float:
    """Candidate source of the learned sampler for n draws out of nw
    hyperwedges: a uniform pool of pool_factor * n candidates while that pool
    covers less than full_fraction of the wedges, else every wedge scored
    (pool factor 0).  Scoring all wedges has a fixed cost that only pays off
    once the pool would be a sizeable part of the graph anyway."""
    return pool_factor if pool_factor * n < full_fraction * nw else 0.0


def equal_time_study(G, exact: np.ndarray, model, budgets: Sequence[float] = (0.001, 0.01, 0.05),
                     seeds: int = 32, mix: float = 0.1, pool_factor="auto",
                     log=print, exact_inclusion: bool = False, with_adv: bool = True) -> List[Dict]:
    """Learned vs uniform hyperwedge sampling at equal GPU time.  For each
    budget b: the learned sampler draws b*|wedges| samples (from a uniform pool
    of pool_factor times as many candidates, or from all wedges with pool
    factor 0; "auto" picks with pool_factor_for); its device time sets the
    time budget; the uniform sampler gets as many samples as fit in that time
    (calibrated to within 5%).  Errors over `seeds` independent runs.
    exact_inclusion: both samplers close the inclusion stratum exactly and
    sample the intersection-type hyperwedges.  with_adv: also Appro-adv
    (Algorithm 7) at the same time (plain study only)."""
    xi = exact_inclusion
    nw = G.num_wedges
    out = []
    for b in budgets:
        nL = max(1, int(round(b * nw)))
        pf = pool_factor_for(nL, nw) if pool_factor == "auto" else float(pool_factor)
        _run(G, 1, nL, 10_000, model, mix, pf, xi)                 # warm-up
        rl, tl, el = [], [], []
        for s in range(seeds):
            est, se, ms = _run(G, 1, nL, s, model, mix, pf, xi)
            rl.append(relative_error(est, exact))
            tl.append(ms)
            el.append(est)
        t_target = float(np.median(tl))
        nU = nL
        for _ in range(6):                                              # calibrate the uniform count
            ts = [_run(G, 0, nU, 20_000 + r, None, 0, 0, xi)[2] for r in range(3)]
            t = float(np.median(ts))
            if abs(t - t_target) <= 0.05 * t_target:
                break
            nU = max(1, int(nU * t_target / max(t, 1e-6)))
        ru, tu, eu = [], [], []
        for s in range(seeds):
            est, se, ms = _run(G, 0, nU, s, None, 0, 0, xi)
            ru.append(relative_error(est, exact))
            tu.append(ms)
            eu.append(est)
        row = {"budget": b, "exact_inclusion": bool(xi), "learned_samples": nL, "uniform_samples": nU,
               "pool_factor": pf, "learned_ms": t_target, "uniform_ms": float(np.median(tu)),
               "learned_rel_err": float(np.mean(rl)), "uniform_rel_err": float(np.mean(ru))}
        row.update(_error_summary("learned", np.array(el), exact))
        row.update(_error_summary("uniform", np.array(eu), exact))
        if with_adv and not xi:
            # Appro-adv (Algorithm 7) at the same time: its draw count calibrated like uniform's
            nA = nL
            for _ in range(6):
                ts = [_run(G, 2, nA, 30_000 + r, None, 0, 0)[2] for r in range(3)]
                t = float(np.median(ts))
                if abs(t - t_target) <= 0.05 * t_target:
                    break
                nA = max(1, int(nA * t_target / max(t, 1e-6)))
            ra, ta, ea = [], [], []
            for s in range(seeds):
                est, se, ms = _run(G, 2, nA, s, None, 0, 0)
                ra.append(relative_error(est, exact))
                ta.append(ms)
                ea.append(est)
            row.update({"adv_samples": nA, "adv_ms": float(np.median(ta)), "adv_rel_err": float(np.mean(ra))})
            row.update(_error_summary("adv", np.array(ea), exact))
        lp, up = row["learned_per_pattern"], row["uniform_per_pattern"]
        row["learned_wins_patterns"] = int(sum(1 for a, c in zip(lp, up) if a is not None and a < c))
        row["uniform_wins_patterns"] = int(sum(1 for a, c in zip(lp, up) if a is not None and c < a))
        log(f"[equal-time] budget {b:g}: learned n={nL} {t_target:.2f} ms err {row['learned_rel_err']:.4f} "
            f"(total {row['learned_total_rel_err']:.2e}) | uniform n={nU} {row['uniform_ms']:.2f} ms err "
            f"{row['uniform_rel_err']:.4f} (total {row['uniform_total_rel_err']:.2e})"
            + (f" | adv n={row['adv_samples']} {row['adv_ms']:.2f} ms err {row['adv_rel_err']:.4f}"
               if "adv_samples" in row else ""))
        out.append(row)
    return out


def _error_summary(name: str, ests: np.ndarray, exact: np.ndarray) -> Dict:
    """Per-pattern mean relative error and relative RMSE over the runs, and
    the same for the total (patterns with H_p = 0 are None)."""
    H = exact.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        mae = np.where(H > 0, np.abs(ests - H).mean(axis=0) / H, np.nan)
        rmse = np.where(H > 0, np.sqrt(((ests - H) ** 2).mean(axis=0)) / H, np.nan)
    clean = lambda a: [None if math.isnan(x) else float(x) for x in a]
    return {f"{name}_per_pattern": clean(mae[1:]), f"{name}_per_pattern_rmse": clean(rmse[1:]),
            f"{name}_total_rel_err": float(mae[0]), f"{name}_total_rel_rmse": float(rmse[0])}


def sigma_study(G, exact: np.ndarray, sigmas: Sequence[float] = (1.0, 0.5, 0.25), seeds: int = 8,
                budget: float = 0.01, log=print) -> List[Dict]:
    """Appro-bs with sigma < 1 (Algorithm 6): a uniform subset of
    floor(sigma*m + 1/2) hyperedges, the induced sub-hypergraph's hyperwedges,
    `budget` of them sampled uniformly, the estimate multiplied by the
    subgraph's triangle scale.  Also the subgraph's exact count, scaled the
    same way (the error sigma alone causes).  Time: selection + load +
    hyperwedges + estimate, wall clock with the device synchronised."""
    import torch
    rows = []
    for sigma in sigmas:
        err_s, err_x, tot_s, ms, nws = [], [], [], [], []
        for seed in range(seeds):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Gs, kept, scale = G.subgraph(sigma, 7000 + seed, fixed_size=True)
            Gs.build_wedges()
            est, _, _ = Gs.estimate(budget=budget, seed=seed, proposal=0)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
            est = est * scale
            err_s.append(relative_error(est, exact))
            tot_s.append(abs(est[0] - exact[0]) / exact[0])
            c, _, _ = Gs.count_patterns()
            err_x.append(relative_error(c.astype(np.float64) * scale, exact))
            nws.append(Gs.num_wedges)
            Gs.close()
        row = {"sigma": sigma, "hyperedges_kept": int(math.floor(sigma * G.num_edges + 0.5)),
               "subgraph_hyperwedges": float(np.mean(nws)), "samples": int(round(budget * np.mean(nws))),
               "ms": float(np.mean(ms)), "rel_err": float(np.mean(err_s)),
               "total_rel_err": float(np.mean(tot_s)), "subgraph_exact_rel_err": float(np.mean(err_x))}
        rows.append(row)
        log(f"[sigma] {sigma:g}: {row['subgraph_hyperwedges']:.3g} hyperwedges, {row['ms']:.1f} ms, "
            f"err {row['rel_err']:.4f} (total {row['total_rel_err']:.4f}), exact-on-subgraph err "
            f"{row['subgraph_exact_rel_err']:.4f}")
    return rows
