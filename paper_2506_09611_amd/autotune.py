"""Autotuner for the delay rank k of the delayed update.

The delayed update takes the same decisions for every k (Sec. III A: the
group's ratios are the local update's, evaluated in k x k space), so k is a
pure speed parameter.  The best k depends on N_sigma, on the acceptance
and on the batch (Sec. IV A puts the optimum near 0.5-1.0 L on a CPU; here
the tile kernel's MFMA shape and the decision kernel's per-site chain
shift it).  The tuner times the update phase of a short forward window for
each candidate k on walkers of the job's own problem, picks the fastest
and caches the choice per problem shape and coupling.

The block size b of the block force-bias update is not tuned: it changes
the proposal, hence the Markov chain and its acceptance, and so it is a
modelling choice rather than a speed parameter.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Dict, Optional, Sequence

DEFAULT_CANDIDATES = (8, 16, 32, 64, 128)


@dataclasses.dataclass
class TuneResult:
    k: int
    update_s_per_slice: Dict[int, float]   # candidate -> update-phase seconds per slice visit
    key: str
    cached: bool = False


def shape_key(n_sites: int, n_up: int, n_dn: int, U: float, walkers: int, fp32: bool) -> str:
    """Cache key: the sizes, U (through the acceptance, hence the flush
    rank), the batch and the precision form."""
    return f"N{n_sites}_up{n_up}_dn{n_dn}_U{float(U):g}_w{walkers}_{'f32' if fp32 else 'f64'}"


def choose(times: Dict[int, float]) -> int:
    """Fastest candidate; ties go to the smaller k (smaller workspace)."""
    if not times:
        raise ValueError("no candidate was timed")
    return min(times, key=lambda k: (times[k], k))


def _load(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def _store(path: Optional[str], data: dict) -> None:
    if not path:
        return
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_delay(hopping, trial_up, trial_dn, U, dtau, stab_every, *,
               candidates: Sequence[int] = DEFAULT_CANDIDATES, walkers: int = 1,
               window: Optional[int] = None, fp32: bool = False, seed: int = 0,
               cache: Optional[str] = None, repeats: int = 2) -> TuneResult:
    """Time the update phase of a `window`-slice forward window (default
    k_tau) for each candidate k on `walkers` batched walkers of this problem
    and return the fastest.  Walkers are built with M = 2 k_tau slices: the
    cost of one slice visit does not depend on M.  Each candidate gets fresh
    contexts sized for it, since the workspace bound also selects the kernel
    path (fused tile kernel for groups of at most 64 sites).  `repeats`
    windows per candidate (each from the same rebuilt state); the minimum
    counts, so that the first launches of a kernel do not."""
    from .binding import Chain, Scheme, batch_forward_window, MAX_BATCH
    import numpy as np
    n_sites = int(np.asarray(hopping).shape[0])
    n_up, n_dn = int(np.asarray(trial_up).shape[1]), int(np.asarray(trial_dn).shape[1])
    if not 1 <= walkers <= MAX_BATCH:
        raise ValueError(f"walkers must be 1..{MAX_BATCH}")
    cands = sorted({min(int(k), n_sites) for k in candidates if k >= 1})
    if fp32:
        cands = [k for k in cands if k <= 64]
    key = shape_key(n_sites, n_up, n_dn, U, walkers, fp32)
    data = _load(cache)
    hit = data.get(key)
    if hit and set(int(k) for k in hit["times"]) == set(cands):
        times = {int(k): float(v) for k, v in hit["times"].items()}
        return TuneResult(int(hit["k"]), times, key, cached=True)
    win = int(window or stab_every)
    M = 2 * int(stab_every)
    if win > M:
        raise ValueError("window must be at most 2 k_tau")
    times: Dict[int, float] = {}
    for k in cands:
        chains = [Chain(hopping, trial_up, trial_dn, U, dtau, M, stab_every, seed, w,
                        scheme=Scheme.DELAYED, k=k, timing=True, fp32=fp32,
                        tile_chunks=64 if walkers == 1 else 0)
                  for w in range(walkers)]
        try:
            start = [c.fields() for c in chains]
            best = None
            for r in range(max(1, repeats)):
                if r:
                    for c, f in zip(chains, start):
                        c.set_fields(f)
                st = batch_forward_window(chains, win)[0]
                t = st["t_update_s"] / win
                best = t if best is None else min(best, t)
            times[k] = best
        finally:
            for c in chains:
                c.close()
    k_best = choose(times)
    data[key] = {"k": k_best, "times": {str(k): v for k, v in times.items()}}
    _store(cache, data)
    return TuneResult(k_best, times, key)
