"""Continuous-batching job server for PQMC sweeps on one GPU.

A job is one lattice problem (hopping matrix, trial orbitals, U, dtau,
M, k_tau) with `n_walkers` independent walkers -- Philox keys
(seed, walker_id) for walker_id = 0 .. n_walkers-1 -- each of which runs
`n_sweeps` sweeps.  Jobs arrive over time (for instance as a Poisson
stream).  The server

* admits jobs first come, first served, a whole job at a time, while the
  device footprint of all admitted walkers fits the memory budget.  The
  footprint of a walker is its pqmc_workspace_bytes, which is everything
  the library uses on the device; a job larger than the whole budget is
  rejected;
* runs one sweep per step for a batch of up to MAX_BATCH compatible walkers
  (pqmc_batch_sweep, or pqmc_soc_batch_sweep for spin-orbit coupled ones).  The walker first in line picks the batch and the
  compatible walkers behind it fill it, in line order.  The line is
  ordered by job arrival, then by sweeps done ("fcfs"), or by sweeps done,
  then arrival ("rr", round robin).  The delayed and block schemes batch
  lattices of different sizes together;
* re-forms the batches at every sweep boundary, so the walkers of a newly
  admitted job join at the next step (continuous batching);
* with several lanes (one HIP stream each), places every admitted walker on
  the lane with the fewest active walkers, forms one batch per lane at each
  step and runs the lanes' batches concurrently (pqmc_multi_sweep), so that
  one batch's serial phases overlap another's matrix work;
* frees a walker's workspace as soon as it finishes and retires the job with
  its last walker, then admits from the queue.

A walker's fields and G depend only on its own key and on the sweeps it has
run, never on its batch partners or the interleaving: its result is the same,
bit for bit, alone or in any mix.

Execution sits behind a small backend interface (walker_bytes, open,
sweep, collect, close); GpuBackend drives the HIP library.  The clock is also
pluggable, so that the scheduling logic runs on the CPU against a
simulated backend and clock.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Dict, List, Optional, Sequence

import numpy as np

from .binding import MAX_BATCH, Scheme


@dataclasses.dataclass
class Job:
    """One request: a problem, its walkers and their sweep count.  `arrival`
    is in seconds from the start of the run."""
    job_id: int
    arrival: float
    hopping: np.ndarray
    trial_up: np.ndarray
    trial_dn: np.ndarray
    U: float
    dtau: float
    n_slices: int
    stab_every: int
    seed: int
    n_walkers: int = 1
    n_sweeps: int = 1
    scheme: Scheme = Scheme.DELAYED
    k: int = 32
    b: int = 16
    fp32: bool = False
    keep_green: bool = True
    soc: bool = False      # spin-orbit coupled model: hopping 2N x 2N complex, trial_up
                           # the 2N x N_e trial, trial_dn unused; local or delayed scheme

    @property
    def n_sites(self) -> int:
        return int(self.hopping.shape[0]) // (2 if self.soc else 1)

    @property
    def n_up(self) -> int:
        return int(self.trial_up.shape[1])

    @property
    def n_dn(self) -> int:
        return 0 if self.soc else int(self.trial_dn.shape[1])


def batch_key(job: Job) -> tuple:
    """Walkers batch together iff their keys are equal: the library's rule
    for pqmc_batch_sweep (same M, k_tau, scheme, k, b, precision form and
    group-size class; the local scheme also needs one lattice shape), and for
    pqmc_soc_batch_sweep (SOC walkers of one lattice, N_e, M, k_tau, scheme
    and group size)."""
    if job.soc:
        gk = job.b if job.scheme == Scheme.BLOCK_FB else (job.k if job.scheme == Scheme.DELAYED
                                                          else 1)
        return ("soc", job.n_sites, job.n_up, job.n_slices, job.stab_every, int(job.scheme),
                min(gk, job.n_sites))
    N = job.n_sites
    gmax = max(min(job.k, N), min(job.b, N))
    key = (job.n_slices, job.stab_every, int(job.scheme), job.k, job.b, bool(job.fp32),
           gmax <= 64)
    if job.scheme == Scheme.LOCAL:
        key += (N, job.n_up, job.n_dn)
    return key


@dataclasses.dataclass
class WalkerResult:
    walker_id: int
    fields: Any
    green: Any                    # (G_up, G_dn) at the end ((G,) for SOC), or None
    stats: Dict[str, float]       # sums over the walker's sweeps


@dataclasses.dataclass
class JobResult:
    job_id: int
    arrival: float
    admitted: Optional[float] = None
    finished: Optional[float] = None
    rejected: bool = False
    walkers: List[WalkerResult] = dataclasses.field(default_factory=list)

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


@dataclasses.dataclass
class ServeReport:
    results: List[JobResult]
    makespan_s: float             # first arrival to last completion
    jobs_per_s: float
    latency_p50_s: float
    latency_p99_s: float
    steps: int                    # scheduling steps (one sweep of each lane's batch)
    mean_batch: float             # walkers per batch
    peak_bytes: int               # largest admitted footprint
    budget_bytes: int
    batch_log: List[List[tuple]]  # per step: (job_id, walker_id) of the batch

    def summary(self) -> dict:
        done = [r for r in self.results if r.finished is not None]
        return {"jobs": len(self.results), "completed": len(done),
                "rejected": sum(r.rejected for r in self.results),
                "makespan_s": self.makespan_s, "jobs_per_s": self.jobs_per_s,
                "latency_p50_s": self.latency_p50_s, "latency_p99_s": self.latency_p99_s,
                "steps": self.steps, "mean_batch": self.mean_batch,
                "peak_gb": self.peak_bytes / 1e9, "budget_gb": self.budget_bytes / 1e9}


def percentile(values: Sequence[float], q: float) -> float:
    """q-th percentile with linear interpolation between order statistics
    (numpy's default), nan for no values."""
    if len(values) == 0:
        return float("nan")
    return float(np.percentile(np.asarray(values, dtype=np.float64), q))


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of n jobs of a Poisson stream of `rate` jobs/s starting
    at 0: cumulative sums of exponential gaps (the first job at t = 0)."""
    gen = np.random.Generator(np.random.Philox(key=[seed & (2**64 - 1), 0x53455256]))
    gaps = gen.exponential(1.0 / rate, size=n)
    gaps[0] = 0.0
    return np.cumsum(gaps)


class RealClock:
    def now(self) -> float:
        return time.perf_counter()

    def sleep_until(self, t: float) -> None:
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)


class GpuBackend:
    """Walkers as library contexts on torch's current device, lane j on its
    own HIP stream (lane 0: torch's current stream).  One step: the lanes'
    spin-decoupled batches in one pqmc_multi_sweep, each SOC batch's
    pqmc_soc_batch_sweep on a host thread of its own, all concurrently."""

    def __init__(self, lanes: int = 1):
        import torch
        from . import binding
        if not 1 <= lanes <= 8:
            raise ValueError("lanes must be 1..8")
        self._b = binding
        self.lanes = lanes
        self.streams = [torch.cuda.current_stream()] + [torch.cuda.Stream()
                                                        for _ in range(lanes - 1)]

    @staticmethod
    def default_budget(fraction: float = 0.9) -> int:
        import torch
        free, _ = torch.cuda.mem_get_info()
        return int(free * fraction)

    def _soc_k(self, job: Job) -> int:
        """The SOC context's group size: the block size for block force bias."""
        return job.b if int(job.scheme) == int(self._b.Scheme.BLOCK_FB) else job.k

    def walker_bytes(self, job: Job) -> int:
        if job.soc:
            return self._b.soc_workspace_bytes(job.n_sites, job.n_up, job.n_slices,
                                               job.stab_every, job.scheme, self._soc_k(job))
        return self._b.workspace_bytes(job.n_sites, job.n_up, job.n_dn, job.n_slices,
                                       job.stab_every, job.scheme, job.k, job.b, job.fp32)

    def open(self, job: Job, walker_id: int, lane: int = 0):
        if job.soc:
            return self._b.SocChain(job.hopping, job.trial_up, job.U, job.dtau, job.n_slices,
                                    job.stab_every, job.seed, walker_id, scheme=job.scheme,
                                    k=self._soc_k(job), stream=self.streams[lane])
        return self._b.Chain(job.hopping, job.trial_up, job.trial_dn, job.U, job.dtau,
                             job.n_slices, job.stab_every, job.seed, walker_id,
                             scheme=job.scheme, k=job.k, b=job.b, fp32=job.fp32,
                             stream=self.streams[lane])

    def sweep(self, batches: List[list]) -> List[List[dict]]:
        out: List[Optional[List[dict]]] = [None] * len(batches)
        plain = [i for i, b in enumerate(batches) if not isinstance(b[0], self._b.SocChain)]
        socs = [i for i in range(len(batches)) if i not in plain]

        def run_plain():
            flat = [h for i in plain for h in batches[i]]
            st = self._b.multi_sweep(flat, 1)
            k = 0
            for i in plain:
                out[i] = st[k:k + len(batches[i])]
                k += len(batches[i])

        def run_soc(i):
            out[i] = self._b.soc_batch_sweep(batches[i], 1)

        tasks = ([run_plain] if plain else []) + [(lambda i=i: run_soc(i)) for i in socs]
        if len(tasks) == 1:
            tasks[0]()
        else:
            import concurrent.futures
            with concurrent.futures.ThreadPoolExecutor(max_workers=len(tasks)) as ex:
                for f in [ex.submit(t) for t in tasks]:
                    f.result()
        return out

    def collect(self, job: Job, handle):
        if job.soc:
            return handle.fields(), ((handle.green(),) if job.keep_green else None)
        green = (handle.green(0), handle.green(1)) if job.keep_green else None
        return handle.fields(), green

    def close(self, handle) -> None:
        handle.close()


_STAT_KEYS = ("proposed", "accepted", "flips", "low_margin", "negative", "field_updates")


class _Walker:
    __slots__ = ("job", "wid", "handle", "done", "stats", "key", "order", "lane")

    def __init__(self, job, wid, handle, key, order, lane):
        self.job, self.wid, self.handle, self.key, self.order = job, wid, handle, key, order
        self.lane = lane
        self.done = 0
        self.stats = {k: 0 for k in _STAT_KEYS}


class Server:
    """Admission, batching and retirement of jobs (see the module text).

    budget_bytes: device memory the walkers may hold together.
    policy: "fcfs" (line ordered by job arrival) or "rr" (by sweeps done).
    lanes: concurrent batches per step (the backend's lanes, e.g. streams).
    """

    def __init__(self, backend, budget_bytes: int, policy: str = "fcfs", clock=None,
                 max_batch: int = MAX_BATCH, lanes: Optional[int] = None,
                 on_step: Optional[Callable[[int, list], None]] = None):
        if policy not in ("fcfs", "rr"):
            raise ValueError("policy must be 'fcfs' or 'rr'")
        if not 1 <= max_batch <= MAX_BATCH:
            raise ValueError(f"max_batch must be 1..{MAX_BATCH}")
        self.backend = backend
        self.budget = int(budget_bytes)
        self.policy = policy
        self.clock = clock or RealClock()
        self.max_batch = max_batch
        self.lanes = int(lanes if lanes is not None else getattr(backend, "lanes", 1))
        if self.lanes < 1:
            raise ValueError("lanes must be >= 1")
        self.on_step = on_step

    def _line_key(self, w: _Walker):
        if self.policy == "fcfs":
            return (w.order, w.done, w.wid)
        return (w.done, w.order, w.wid)

    def _pick(self, active: List[_Walker]) -> List[_Walker]:
        line = sorted(active, key=self._line_key)
        head = line[0]
        return [w for w in line if w.key == head.key][:self.max_batch]

    def _pick_lanes(self, active: List[_Walker]) -> List[List[_Walker]]:
        out = []
        for lane in range(self.lanes):
            mine = [w for w in active if w.lane == lane]
            if mine:
                out.append(self._pick(mine))
        return out

    def run(self, jobs: Sequence[Job]) -> ServeReport:
        for j in jobs:
            if j.n_walkers < 1 or j.n_sweeps < 1:
                raise ValueError(f"job {j.job_id}: n_walkers and n_sweeps must be >= 1")
        order = sorted(range(len(jobs)), key=lambda i: (jobs[i].arrival, i))
        pending = collections.deque(jobs[i] for i in order)
        results = {j.job_id: JobResult(j.job_id, float(j.arrival)) for j in jobs}
        if len(results) != len(jobs):
            raise ValueError("job ids must be unique")
        wbytes = {}
        queue: collections.deque = collections.deque()
        active: List[_Walker] = []
        left: Dict[int, int] = {}
        used = peak = steps = walked = 0
        batch_log: List[List[tuple]] = []
        seq = 0
        t0 = self.clock.now()

        while pending or queue or active:
            now = self.clock.now() - t0
            while pending and pending[0].arrival <= now:
                j = pending.popleft()
                wbytes[j.job_id] = self.backend.walker_bytes(j)
                if wbytes[j.job_id] * j.n_walkers > self.budget:
                    results[j.job_id].rejected = True
                else:
                    queue.append(j)
            # first come, first served: the head job is admitted whole or waits
            while queue and used + wbytes[queue[0].job_id] * queue[0].n_walkers <= self.budget:
                j = queue.popleft()
                key = batch_key(j)
                for w in range(j.n_walkers):
                    load = [0] * self.lanes
                    for x in active:
                        load[x.lane] += 1
                    lane = min(range(self.lanes), key=lambda q: (load[q], q))
                    h = self.backend.open(j, w, lane) if self.lanes > 1 else \
                        self.backend.open(j, w)
                    active.append(_Walker(j, w, h, key, seq, lane))
                seq += 1
                used += wbytes[j.job_id] * j.n_walkers
                peak = max(peak, used)
                left[j.job_id] = j.n_walkers
                results[j.job_id].admitted = self.clock.now() - t0
            if not active:
                if pending:
                    self.clock.sleep_until(t0 + pending[0].arrival)
                continue
            batches = self._pick_lanes(active)
            stats = self.backend.sweep([[w.handle for w in b] for b in batches])
            steps += 1
            for b in batches:
                walked += len(b)
                batch_log.append([(w.job.job_id, w.wid) for w in b])
            if self.on_step:
                self.on_step(steps, batches)
            for w, st in ((w, st) for b, sb in zip(batches, stats) for w, st in zip(b, sb)):
                w.done += 1
                for k in _STAT_KEYS:
                    w.stats[k] += st.get(k, 0)
                if w.done < w.job.n_sweeps:
                    continue
                fields, green = self.backend.collect(w.job, w.handle)
                self.backend.close(w.handle)
                active.remove(w)
                used -= wbytes[w.job.job_id]
                r = results[w.job.job_id]
                r.walkers.append(WalkerResult(w.wid, fields, green, dict(w.stats)))
                left[w.job.job_id] -= 1
                if left[w.job.job_id] == 0:
                    r.walkers.sort(key=lambda x: x.walker_id)
                    r.finished = self.clock.now() - t0

        out = [results[j.job_id] for j in jobs]
        lat = [r.latency for r in out if r.finished is not None]
        fin = [r.finished for r in out if r.finished is not None]
        first = min((r.arrival for r in out), default=0.0)
        makespan = (max(fin) - first) if fin else 0.0
        return ServeReport(
            results=out, makespan_s=makespan,
            jobs_per_s=(len(fin) / makespan) if makespan > 0 else float("nan"),
            latency_p50_s=percentile(lat, 50), latency_p99_s=percentile(lat, 99),
            steps=steps, mean_batch=(walked / len(batch_log)) if batch_log else 0.0,
            peak_bytes=peak,
            budget_bytes=self.budget, batch_log=batch_log)
