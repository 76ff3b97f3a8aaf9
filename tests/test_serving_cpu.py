"""Scheduling logic of the job server on the CPU: a simulated backend (each
walker a counter, each step a fixed cost growing with the largest lattice of
the batch) and a simulated clock stand in for the GPU."""
import numpy as np
import pytest

from paper_2506_09611_amd.binding import Scheme
from paper_2506_09611_amd.serving import (Job, Server, batch_key, percentile, poisson_arrivals)


class SimClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


class SimBackend:
    """Walker state = sweeps run; footprint 1 unit per site; a step costs
    1 ms + 1 us per site of the largest walker of the batch."""

    def __init__(self, clock):
        self.clock = clock
        self.open_handles = set()
        self.held = 0
        self.peak_held = 0

    def walker_bytes(self, job):
        return job.n_sites

    def open(self, job, w, lane=0):
        h = {"job": job, "w": w, "sweeps": 0, "id": (job.job_id, w), "lane": lane}
        self.open_handles.add(h["id"])
        self.held += job.n_sites
        self.peak_held = max(self.peak_held, self.held)
        return h

    def sweep(self, batches):
        """Lanes' batches run concurrently: the step costs the slowest one."""
        cost = 0.0
        lanes = [b[0]["lane"] for b in batches]
        assert len(set(lanes)) == len(lanes), "two batches on one lane"
        for handles in batches:
            assert 1 <= len(handles) <= 8
            keys = {batch_key(h["job"]) for h in handles}
            assert len(keys) == 1, "incompatible walkers batched"
            assert len({h["lane"] for h in handles}) == 1, "a batch spans lanes"
            for h in handles:
                assert h["id"] in self.open_handles
                h["sweeps"] += 1
            cost = max(cost, 1e-3 + 1e-6 * max(h["job"].n_sites for h in handles))
        self.clock.t += cost
        return [[{"proposed": h["job"].n_sites, "accepted": 1} for h in handles]
                for handles in batches]

    def collect(self, job, h):
        return ("fields", job.job_id, h["w"], h["sweeps"]), None

    def close(self, h):
        self.open_handles.remove(h["id"])
        self.held -= h["job"].n_sites


def _job(i, arrival, L, n_walkers=3, n_sweeps=2, scheme=Scheme.DELAYED, k=32, b=16,
         n_slices=40):
    N = L * L
    return Job(job_id=i, arrival=float(arrival), hopping=np.zeros((N, N)),
               trial_up=np.zeros((N, N // 2)), trial_dn=np.zeros((N, N // 2)), U=4.0,
               dtau=0.05, n_slices=n_slices, stab_every=10, seed=i, n_walkers=n_walkers,
               n_sweeps=n_sweeps, scheme=scheme, k=k, b=b)


def _mix(n=40, rate=200.0, seed=7):
    t = poisson_arrivals(n, rate, seed)
    Ls = [8, 12, 16, 24, 32]
    gen = np.random.default_rng(seed)
    return [_job(i, t[i], Ls[gen.integers(len(Ls))], n_walkers=int(gen.integers(1, 12)),
                 n_sweeps=int(gen.integers(1, 4))) for i in range(n)]


@pytest.mark.parametrize("policy,lanes", [("fcfs", 1), ("rr", 1), ("fcfs", 3)])
def test_every_job_completes_within_budget(policy, lanes):
    clock = SimClock()
    be = SimBackend(clock)
    jobs = _mix()
    budget = max(j.n_sites * j.n_walkers for j in jobs)   # the largest job fits alone
    rep = Server(be, budget, policy=policy, clock=clock, lanes=lanes).run(jobs)
    assert be.peak_held <= budget and rep.peak_bytes <= budget
    assert not be.open_handles, "every workspace released"
    for j, r in zip(jobs, rep.results):
        assert r.finished is not None and not r.rejected
        assert r.arrival <= r.admitted <= r.finished
        assert [w.walker_id for w in r.walkers] == list(range(j.n_walkers))
        for w in r.walkers:
            # each walker ran exactly its own sweeps, whatever its partners
            assert w.fields == ("fields", j.job_id, w.walker_id, j.n_sweeps)
            assert w.stats["proposed"] == j.n_sites * j.n_sweeps
    steps = sum(len(b) for b in rep.batch_log)
    assert steps == sum(j.n_walkers * j.n_sweeps for j in jobs)
    assert rep.mean_batch > 1.0


def test_admission_is_first_come_first_served():
    clock = SimClock()
    jobs = _mix()
    rep = Server(SimBackend(clock), max(j.n_sites * j.n_walkers for j in jobs),
                 clock=clock).run(jobs)
    adm = [r.admitted for r in sorted(rep.results, key=lambda r: (r.arrival, r.job_id))]
    assert all(a <= b for a, b in zip(adm, adm[1:]))


def test_continuous_batching_admits_during_a_long_job():
    """A short job arriving while a long one runs is admitted and finished
    before the long one ends, and shares its batches."""
    clock = SimClock()
    long = _job(0, 0.0, 16, n_walkers=2, n_sweeps=50)
    short = _job(1, 0.01, 8, n_walkers=2, n_sweeps=2)
    rep = Server(SimBackend(clock), 10**6, clock=clock).run([long, short])
    rl, rs = rep.results
    assert rs.admitted < rl.finished and rs.finished < rl.finished
    mixed = [b for b in rep.batch_log if {j for j, _ in b} == {0, 1}]
    assert mixed, "the short job never shared a batch with the long one"


def test_incompatible_walkers_never_share_a_batch():
    clock = SimClock()
    jobs = [_job(0, 0.0, 8, k=32), _job(1, 0.0, 8, k=16), _job(2, 0.0, 8, scheme=Scheme.LOCAL),
            _job(3, 0.0, 12, scheme=Scheme.LOCAL), _job(4, 0.0, 12, k=16)]
    rep = Server(SimBackend(clock), 10**6, clock=clock).run(jobs)
    for b in rep.batch_log:
        assert len({batch_key(jobs[j]) for j, _ in b}) == 1
    # the delayed k = 16 jobs of both sizes share batches; the local ones do not
    assert any({j for j, _ in b} == {1, 4} for b in rep.batch_log)
    assert not any({2, 3} <= {j for j, _ in b} for b in rep.batch_log)


def test_oversized_job_rejected_rest_served():
    clock = SimClock()
    jobs = [_job(0, 0.0, 32, n_walkers=4), _job(1, 0.0, 8)]
    rep = Server(SimBackend(clock), 2000, clock=clock).run(jobs)
    assert rep.results[0].rejected and rep.results[0].finished is None
    assert rep.results[1].finished is not None


def test_idle_server_waits_for_arrivals():
    clock = SimClock()
    jobs = [_job(0, 0.0, 8, n_sweeps=1), _job(1, 5.0, 8, n_sweeps=1)]
    rep = Server(SimBackend(clock), 10**6, clock=clock).run(jobs)
    assert rep.results[1].admitted == pytest.approx(5.0)
    assert rep.results[1].latency < 0.1


def test_batch_key_follows_library_rules():
    a = _job(0, 0, 8, k=32)
    assert batch_key(a) == batch_key(_job(1, 0, 24, k=32))           # sizes mix
    assert batch_key(a) != batch_key(_job(1, 0, 8, k=16))            # k differs
    assert batch_key(a) != batch_key(_job(1, 0, 8, k=32, n_slices=80))
    assert batch_key(_job(0, 0, 8, scheme=Scheme.LOCAL)) != batch_key(
        _job(1, 0, 12, scheme=Scheme.LOCAL))                          # local: one shape
    # group-size class: min(k, N) on either side of 64
    assert batch_key(_job(0, 0, 8, k=128)) != batch_key(_job(1, 0, 16, k=128))


def test_percentile_and_arrivals():
    assert percentile([1.0, 2.0, 3.0, 4.0], 50) == 2.5
    assert percentile(list(range(101)), 99) == 99.0
    assert np.isnan(percentile([], 50))
    t = poisson_arrivals(20000, 50.0, 3)
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 50.0) < 0.03 / 50.0 * 5       # mean 1/rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05             # exponential: cv = 1
    assert np.array_equal(t, poisson_arrivals(20000, 50.0, 3))


def test_lanes_run_batches_concurrently():
    """Two lanes: walkers spread evenly over them, two batches per step while
    both lanes hold walkers, and the same jobs finish sooner than on one."""
    jobs = [_job(i, 0.0, 8, n_walkers=8, n_sweeps=3) for i in range(4)]
    ends = {}
    for lanes in (1, 2):
        clock = SimClock()
        rep = Server(SimBackend(clock), 10**6, clock=clock, lanes=lanes).run(jobs)
        ends[lanes] = max(r.finished for r in rep.results)
        assert rep.mean_batch == 8.0
    assert ends[2] < 0.6 * ends[1]


def _soc_job(i, arrival, L, n_walkers=2, n_sweeps=2):
    N = L * L
    return Job(job_id=i, arrival=float(arrival), hopping=np.zeros((2 * N, 2 * N), complex),
               trial_up=np.zeros((2 * N, N), complex), trial_dn=None, U=-4.0, dtau=0.05,
               n_slices=40, stab_every=10, seed=i, n_walkers=n_walkers, n_sweeps=n_sweeps,
               scheme=Scheme.DELAYED, k=16, soc=True)


def test_soc_walkers_batch_by_shape_beside_batches():
    """SOC walkers batch only with SOC walkers of the same shape (lattice,
    N_e, M, k_tau, scheme, group size), never with spin-decoupled ones, and
    run on the lanes beside the spin-decoupled batches."""
    clock = SimClock()
    jobs = [_job(0, 0.0, 8, n_walkers=6), _soc_job(1, 0.0, 8), _job(2, 0.0, 12, n_walkers=4),
            _soc_job(3, 0.001, 4, n_walkers=3), _soc_job(4, 0.002, 8, n_walkers=3)]
    assert jobs[1].n_sites == 64 and jobs[1].n_up == 64
    rep = Server(SimBackend(clock), 10**6, clock=clock, lanes=2).run(jobs)
    shared = False
    for b in rep.batch_log:
        socs = [j for j, _ in b if jobs[j].soc]
        assert not socs or len(socs) == len(b), b                       # never mixed
        assert len({batch_key(jobs[j]) for j, _ in b}) == 1, b          # one shape
        shared |= len({j for j, _ in b if jobs[j].soc}) > 1
    assert shared   # the two 8x8 SOC jobs (same shape) share batches
    assert all(r.finished is not None for r in rep.results)
    assert batch_key(jobs[1]) != batch_key(jobs[3])
    assert batch_key(jobs[1]) == batch_key(jobs[4])
