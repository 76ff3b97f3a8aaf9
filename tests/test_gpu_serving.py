"""The job server on the GPU: jobs of mixed lattice sizes arriving as a
Poisson stream under a memory budget that forces queueing; every walker's
fields and G must equal, bit for bit, those of the same walker run alone."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_09611_amd import load_library
    load_library()


def _jobs(scheme, **kw):
    from paper_2506_09611_amd.serving import Job, poisson_arrivals
    t = poisson_arrivals(6, 40.0, synth.SEED_BASE + 60)
    sizes = [(6, 18, 17), (4, 8, 7), (8, 32, 30), (6, 18, 18), (4, 5, 3), (8, 31, 32)]
    jobs = []
    for i, (L, nu, nd) in enumerate(sizes):
        p = synth.make_problem(L, nu, nd, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                               seed=synth.SEED_BASE + 61 + i)
        jobs.append(Job(job_id=i, arrival=float(t[i]), hopping=p.hopping, trial_up=p.trial_up,
                        trial_dn=p.trial_dn, U=p.U, dtau=p.dtau, n_slices=p.n_slices,
                        stab_every=p.stab_every, seed=p.seed, n_walkers=3, n_sweeps=2,
                        scheme=scheme, **kw))
    return jobs


@pytest.mark.parametrize("scheme_name,kw,lanes", [("delayed", {"k": 16}, 1),
                                                  ("block", {"b": 8}, 1),
                                                  ("delayed", {"k": 16}, 2)])
def test_served_results_equal_alone(scheme_name, kw, lanes):
    from paper_2506_09611_amd import Chain, Scheme
    from paper_2506_09611_amd.serving import GpuBackend, Server
    scheme = {"delayed": Scheme.DELAYED, "block": Scheme.BLOCK_FB}[scheme_name]
    jobs = _jobs(scheme, **kw)
    be = GpuBackend(lanes=lanes)
    per_job = sorted(be.walker_bytes(j) * j.n_walkers for j in jobs)
    budget = per_job[-1] + per_job[-2]          # at most about two jobs at once
    rep = Server(be, budget).run(jobs)
    s = rep.summary()
    print(f"served {scheme_name}: {s}", flush=True)
    assert s["completed"] == len(jobs) and rep.peak_bytes <= budget
    mixed = [b for b in rep.batch_log if len({j for j, _ in b}) > 1]
    assert mixed, "no batch mixed two jobs"
    assert any(len({jobs[j].n_sites for j, _ in b}) > 1 for b in mixed), "no mixed sizes"
    for j, r in zip(jobs, rep.results):
        for w in r.walkers:
            alone = Chain(j.hopping, j.trial_up, j.trial_dn, j.U, j.dtau, j.n_slices,
                          j.stab_every, j.seed, w.walker_id, scheme=scheme, **kw)
            alone.sweep(j.n_sweeps)
            assert np.array_equal(w.fields, alone.fields()), (j.job_id, w.walker_id)
            for sp in range(2):
                assert np.array_equal(w.green[sp], alone.green(sp)), (j.job_id, w.walker_id, sp)
            alone.close()


def test_served_mix_with_soc_jobs_equal_alone():
    """Half spin-decoupled, half spin-orbit coupled jobs on two lanes: each
    walker's fields and G equal those of its run alone."""
    from paper_2506_09611_amd import Chain, SocChain, Scheme
    from paper_2506_09611_amd.serving import GpuBackend, Job, Server, poisson_arrivals
    t = poisson_arrivals(4, 40.0, synth.SEED_BASE + 66)
    jobs = []
    for i in range(4):
        if i % 2 == 0:
            p = synth.make_problem(6, 18, 17, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                                   seed=synth.SEED_BASE + 67 + i)
            jobs.append(Job(job_id=i, arrival=float(t[i]), hopping=p.hopping,
                            trial_up=p.trial_up, trial_dn=p.trial_dn, U=p.U, dtau=p.dtau,
                            n_slices=p.n_slices, stab_every=p.stab_every, seed=p.seed,
                            n_walkers=3, n_sweeps=2, scheme=Scheme.DELAYED, k=16))
        else:
            q = synth.make_soc_problem(4, 14, -4.0, lam=0.5, n_slices=20, stab_every=5,
                                       perturb=1e-3, seed=synth.SEED_BASE + 67 + i)
            jobs.append(Job(job_id=i, arrival=float(t[i]), hopping=q.hopping, trial_up=q.trial,
                            trial_dn=None, U=q.U, dtau=q.dtau, n_slices=q.n_slices,
                            stab_every=q.stab_every, seed=q.seed, n_walkers=2, n_sweeps=2,
                            scheme=Scheme.DELAYED, k=8, soc=True))
    probs = {}
    for i in range(4):
        probs[i] = (synth.make_problem(6, 18, 17, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                                       seed=synth.SEED_BASE + 67 + i) if i % 2 == 0 else
                    synth.make_soc_problem(4, 14, -4.0, lam=0.5, n_slices=20, stab_every=5,
                                           perturb=1e-3, seed=synth.SEED_BASE + 67 + i))
    be = GpuBackend(lanes=2)
    rep = Server(be, be.default_budget()).run(jobs)
    print("served mix:", rep.summary(), flush=True)
    assert rep.summary()["completed"] == 4
    # one served walker of each model against the oracle (decisions and G)
    import dataclasses
    from oracle.pqmc import Walker
    from oracle.soc import SocWalker
    for ji in (0, 1):
        j, r = jobs[ji], rep.results[ji]
        w = r.walkers[-1]
        q = dataclasses.replace(probs[ji], walker_id=w.walker_id)
        ref = SocWalker(q, "delayed", k=j.k) if j.soc else Walker(q, "delayed", k=j.k)
        for _ in range(j.n_sweeps):
            ref.sweep()
        assert np.array_equal(w.fields, ref.fields), ("oracle fields", ji)
        Gs = [w.green[0]] if j.soc else [w.green[0], w.green[1]]
        Gr = [ref.green()] if j.soc else [ref.green(0), ref.green(1)]
        for G, R in zip(Gs, Gr):
            err = np.max(np.abs(G - R)) / max(1.0, np.max(np.abs(R)))
            print(f"served job {ji} ({'soc' if j.soc else 'hubbard'}) walker {w.walker_id} "
                  f"vs oracle: G err {err:.2e}", flush=True)
            assert err < 1e-10
    for j, r in zip(jobs, rep.results):
        for w in r.walkers:
            if j.soc:
                alone = SocChain(j.hopping, j.trial_up, j.U, j.dtau, j.n_slices, j.stab_every,
                                 j.seed, w.walker_id, scheme=j.scheme, k=j.k)
                alone.sweep(j.n_sweeps)
                assert np.array_equal(w.fields, alone.fields())
                assert np.array_equal(w.green[0], alone.green())
            else:
                alone = Chain(j.hopping, j.trial_up, j.trial_dn, j.U, j.dtau, j.n_slices,
                              j.stab_every, j.seed, w.walker_id, scheme=j.scheme, k=j.k)
                alone.sweep(j.n_sweeps)
                assert np.array_equal(w.fields, alone.fields())
                for sp in range(2):
                    assert np.array_equal(w.green[sp], alone.green(sp))
            alone.close()
