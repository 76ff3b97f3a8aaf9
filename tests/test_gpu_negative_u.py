"""The paper's own convention, U < 0 (Sec. II B, Eqs. (13)-(14)), on the GPU
through the spin-decoupled calls, against the oracle's complex128 walker.

alpha = i gamma makes B_dn the complex conjugate of B_up: the library keeps
the one spin-up sector and takes R = r_up r_dn = |r_up|^2; the oracle
propagates both sectors explicitly.  Same bar as the U > 0 parity tests:
every decision exact, margins to 1e-9, fields equal, G to 1e-10 relative,
and G_dn = conj(G_up).
"""
import numpy as np
import pytest

import synth
from oracle.pqmc import Walker
from gpu_util import make_chain, compare_decisions, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_09611_amd import load_library
    load_library()


def _check(ch, w, sweep, M, label):
    meta, margin = ch.decisions()
    n, _ = compare_decisions(meta, margin, w.log, sweep, M)
    print(f"{label}: {n} decisions equal", flush=True)
    assert np.array_equal(ch.fields(), w.fields), label
    G0, G1 = ch.green(0), ch.green(1)
    assert G0.dtype == np.complex128
    assert np.array_equal(G1, np.conj(G0))
    err = max(rel_err(G0, w.green(0)), rel_err(G1, w.green(1)))
    print(f"{label}: G rel err {err:.2e}", flush=True)
    assert err < 1e-10, label
    # the oracle's two sectors are conjugate, as the library assumes
    assert rel_err(w.green(1), np.conj(w.green(0))) < 1e-12


@pytest.mark.parametrize("scheme,kw", [("local", {}), ("delayed", {"k": 4}), ("delayed", {"k": 7}),
                                       ("block", {"b": 4}), ("block", {"b": 3})])
def test_negative_u_4x4_two_sweeps(scheme, kw):
    p = synth.make_problem(4, 5, 5, -4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 71)
    w = Walker(p, scheme, **kw)
    ch = make_chain(p, scheme, **kw)
    assert rel_err(ch.green(0), w.green(0)) < 1e-12          # initial state
    assert np.array_equal(ch.fields(), w.fields)
    for sw in range(2):
        w.sweep()
        ch.sweep(1)
        _check(ch, w, sw, p.n_slices, f"U=-4 4x4 {scheme} {kw} sweep {sw}")
    ch.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("scheme,kw", [("delayed", {"k": 16}), ("block", {"b": 8}), ("local", {})])
def test_negative_u_c2_one_sweep(scheme, kw):
    """16x16, N_sigma = 121, U/t = -4, dtau = 0.05, M = 400, k_tau = 10, bond
    perturbation: one whole sweep (the paper-convention run of the 16 x 16
    workload)."""
    p = synth.workload("c2", U=-4.0)
    w = Walker(p, scheme, **kw)
    ch = make_chain(p, scheme, **kw)
    w.sweep()
    ch.sweep(1)
    _check(ch, w, 0, p.n_slices, f"U=-4 c2 {scheme} {kw}")
    ch.close()


def test_negative_u_replay_cross_scheme():
    """The oracle chain's accepted flips replayed through the one-sector
    local, delayed and block updates: identical fields and G."""
    p = synth.make_problem(6, 13, 13, -4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 72)
    src = Walker(p, "local")
    src.sweep()
    flips = np.zeros((2 * p.n_slices, p.n_sites), np.int8)
    for (sw, d, li, site, acc, margin, sgn) in src.log:
        if acc:
            flips[d * p.n_slices + li, site] = 1
    for scheme, kw in [("local", {}), ("delayed", {"k": 8}), ("block", {"b": 6})]:
        ch = make_chain(p, scheme, **kw)
        ch.replay(flips)
        assert np.array_equal(ch.fields(), src.fields), scheme
        assert rel_err(ch.green(0), src.green(0)) < 1e-10, scheme
        ch.close()


def test_negative_u_rejects_unequal_sectors():
    from paper_2506_09611_amd import Chain, PQMCError, Scheme
    p = synth.make_problem(4, 5, 3, -4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 73)
    with pytest.raises(PQMCError):
        Chain(p.hopping, p.trial_up, p.trial_dn, p.U, p.dtau, p.n_slices, p.stab_every, p.seed,
              scheme=Scheme.DELAYED, k=4)
    q = synth.make_problem(4, 5, 5, -4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 73)
    with pytest.raises(PQMCError):
        Chain(q.hopping, q.trial_up, q.trial_dn, q.U, q.dtau, q.n_slices, q.stab_every, q.seed,
              scheme=Scheme.DELAYED, k=4, fp32=True)
