"""Autotuner for the delay rank k of the delayed update and the tile shape of
its flush kernel.

The delayed update takes the same decisions for every k (Sec. III A: the
group's ratios are the local update's, evaluated in k x k space), so k is a
pure speed parameter.  The best k depends on N_sigma, on the acceptance
and on the batch (Sec. IV A puts the optimum near 0.5-1.0 L on a CPU; here
the tile kernel's MFMA shape and the decision kernel's per-site chain
shift it).  The tuner times the update phase of a short forward window for
each candidate k on walkers of the job's own problem, picks the fastest,
then times the flush kernel's column chunks per row strip (`tile_chunks`)
at that k, and caches both choices per problem shape and coupling.  The
chunking changes only the order in which the panel partials are added, so
the decisions stay those of the local update (up to rounding at margins
below the low-margin threshold).

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
DEFAULT_CHUNKS = (1, 2, 4, 64)   # tile_chunks: one per strip (the pipelined strip kernel
                                 # for groups of 17-32 sites), two, four, one tile per workgroup


@dataclasses.dataclass
class TuneResult:
    k: int
    update_s_per_slice: Dict[int, float]   # candidate k -> update-phase seconds per slice visit
    key: str
    cached: bool = False
    tile_chunks: int = 0                   # chosen column chunks (0: not tuned, library default)
    chunk_s_per_slice: Dict[int, float] = dataclasses.field(default_factory=dict)   # at k


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


def default_chunks(walkers: int) -> int:
    """The chunking the k sweep runs with: one tile per workgroup for a walker
    alone (it must fill the GPU by itself), two per strip for a batch."""
    return 64 if walkers == 1 else 2


def tune_delay(hopping, trial_up, trial_dn, U, dtau, stab_every, *,
               candidates: Sequence[int] = DEFAULT_CANDIDATES, walkers: int = 1,
               window: Optional[int] = None, fp32: bool = False, seed: int = 0,
               cache: Optional[str] = None, repeats: int = 2,
               chunk_candidates: Sequence[int] = DEFAULT_CHUNKS) -> TuneResult:
    """Time the update phase of a `window`-slice forward window (default
    k_tau) for each candidate k on `walkers` batched walkers of this problem
    and return the fastest.  Walkers are built with M = 2 k_tau slices: the
    cost of one slice visit does not depend on M.  Each candidate gets fresh
    contexts sized for it, since the workspace bound also selects the kernel
    path (fused tile kernel for groups of at most 64 sites).  `repeats`
    windows per candidate (each from the same rebuilt state); the minimum
    counts, so that the first launches of a kernel do not.  Then each of
    `chunk_candidates` (column chunks per row strip of the flush kernel; the
    fused path only, groups of at most 64 sites) is timed at the chosen k,
    the k sweep's own chunking counting as already timed; an empty sequence
    skips this stage."""
    from .binding import Chain, Scheme, batch_forward_window, MAX_BATCH
    import numpy as np
    n_sites = int(np.asarray(hopping).shape[0])
    n_up, n_dn = int(np.asarray(trial_up).shape[1]), int(np.asarray(trial_dn).shape[1])
    if not 1 <= walkers <= MAX_BATCH:
        raise ValueError(f"walkers must be 1..{MAX_BATCH}")
    cands = sorted({min(int(k), n_sites) for k in candidates if k >= 1})
    if fp32:
        cands = [k for k in cands if k <= 64]
    chunks = sorted({int(c) for c in chunk_candidates if int(c) >= 1})
    key = shape_key(n_sites, n_up, n_dn, U, walkers, fp32)
    data = _load(cache)
    hit = data.get(key)
    if (hit and set(int(k) for k in hit["times"]) == set(cands)
            and set(int(c) for c in hit.get("chunk_candidates", [])) == set(chunks)):
        times = {int(k): float(v) for k, v in hit["times"].items()}
        ctimes = {int(c): float(v) for c, v in hit.get("chunk_times", {}).items()}
        return TuneResult(int(hit["k"]), times, key, cached=True,
                          tile_chunks=int(hit.get("tile_chunks", 0)), chunk_s_per_slice=ctimes)
    win = int(window or stab_every)
    M = 2 * int(stab_every)
    if win > M:
        raise ValueError("window must be at most 2 k_tau")

    def time_window(k: int, tile_chunks: int) -> float:
        chains = [Chain(hopping, trial_up, trial_dn, U, dtau, M, stab_every, seed, w,
                        scheme=Scheme.DELAYED, k=k, timing=True, fp32=fp32,
                        tile_chunks=tile_chunks)
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
            return best
        finally:
            for c in chains:
                c.close()

    c0 = default_chunks(walkers)
    times: Dict[int, float] = {k: time_window(k, c0) for k in cands}
    k_best = choose(times)
    ctimes: Dict[int, float] = {}
    c_best = 0
    if chunks and k_best <= 64:
        ctimes[c0] = times[k_best]
        for c in chunks:
            if c not in ctimes:
                ctimes[c] = time_window(k_best, c)
        c_best = choose(ctimes)
    data[key] = {"k": k_best, "times": {str(k): v for k, v in times.items()},
                 "tile_chunks": c_best, "chunk_candidates": chunks,
                 "chunk_times": {str(c): v for c, v in ctimes.items()}}
    _store(cache, data)
    return TuneResult(k_best, times, key, tile_chunks=c_best, chunk_s_per_slice=ctimes)
