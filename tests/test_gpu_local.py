"""The persistent local updates on the GPU against the oracle (through the C ABI).

PQMC_LOCAL for one walker runs the paper's T-form local update (Sec. II D,
Eqs. (20)-(21)) as one cooperative launch per slice with T in registers;
PQMC_LOCAL_G runs the same chain on G itself (O(N^2) per site).  Both must
take the oracle's local decisions exactly and reach its G to 1e-10; the
per-site-launch form (the one batches use) must agree with both.
"""
import numpy as np
import pytest

import synth
from oracle.pqmc import Walker
from gpu_util import make_chain, compare_decisions, green_rel_err, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_09611_amd import load_library
    load_library()


def _parity(p, scheme, sweeps=1, window=None, **extra):
    w = Walker(p, "local")
    ch = make_chain(p, scheme, **extra)
    for sw in range(sweeps if window is None else 1):
        if window is None:
            w.sweep()
            st = ch.sweep(1)
        else:
            w.forward_window(window)
            st = ch.forward_window(window)
        meta, margin = ch.decisions()
        n, _ = compare_decisions(meta, margin, w.log, sw, p.n_slices)
        err = green_rel_err(ch, w)
        print(f"{scheme} L={p.L}: {n} decisions equal, G err {err:.2e}, "
              f"drift {st['max_stab_drift']:.1e}", flush=True)
        assert np.array_equal(ch.fields(), w.fields)
        assert err < 1e-10
    return ch, w


@pytest.mark.parametrize("scheme", ["local", "local_g"])
def test_persistent_local_4x4_two_sweeps(scheme):
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 81)
    ch, _ = _parity(p, scheme, sweeps=2)
    ch.close()


@pytest.mark.parametrize("scheme", ["local", "local_g"])
def test_persistent_local_uneven_sectors(scheme):
    """10 x 10 with 70 + 66 fermions: two row blocks per spin of unequal size
    (T-form), 13 rows per workgroup group of the G-form."""
    p = synth.make_problem(10, 70, 66, 4.0, n_slices=10, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 82)
    ch, _ = _parity(p, scheme, sweeps=1)
    ch.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("scheme", ["local_g"])
def test_persistent_local_c2_one_sweep(scheme):
    """16x16, N_sigma = 121, M = 400: one whole sweep of the G-form (the T-form
    runs the same workload in test_gpu_parity)."""
    p = synth.workload("c2")
    ch, _ = _parity(p, scheme, sweeps=1)
    ch.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("scheme", ["local", "local_g"])
def test_persistent_local_c3_window(scheme):
    """40x40, N_sigma = 800: the benchmark's local baselines over a two-slice
    window (T-form: 13 x 7 blocks per spin; G-form: 229 workgroups of 7 rows)."""
    p = synth.workload("c3", n_slices=20, stab_every=10)
    ch, _ = _parity(p, scheme, window=2)
    ch.close()


def test_site_launches_equal_persistent():
    """The per-site-launch local update and the persistent one take the same
    decisions and reach the same G (to rounding: their sums are ordered
    differently)."""
    from paper_2506_09611_amd import Scheme
    p = synth.make_problem(8, 30, 30, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 83)
    a = make_chain(p, "local")
    b = make_chain(p, "local")
    b.set_opts(Scheme.LOCAL, site_launches=True)
    a.sweep(1)
    b.sweep(1)
    assert np.array_equal(a.decisions()[0], b.decisions()[0])
    assert np.array_equal(a.fields(), b.fields())
    for s in range(2):
        assert rel_err(a.green(s), b.green(s)) < 1e-12
    a.close()
    b.close()


def test_local_g_replay_and_switch():
    """G-form replay of the oracle chain's flips gives its fields and G; the
    G-form context also runs the other schemes after a sweep."""
    from paper_2506_09611_amd import Scheme
    p = synth.make_problem(6, 17, 17, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 84)
    src = Walker(p, "local")
    src.sweep()
    flips = np.zeros((2 * p.n_slices, p.n_sites), np.int8)
    for (sw, d, li, site, acc, margin, sgn) in src.log:
        if acc:
            flips[d * p.n_slices + li, site] = 1
    ch = make_chain(p, "local_g", k_max=8)
    ch.replay(flips)
    assert np.array_equal(ch.fields(), src.fields)
    for s in range(2):
        assert rel_err(ch.green(s), src.green(s)) < 1e-10
    # on to the delayed update from the same state, against the oracle
    src.scheme, src.k = "delayed", 8
    ch.set_opts(Scheme.DELAYED, k=8)
    src.sweep()
    ch.sweep(1)
    meta, margin = ch.decisions()
    compare_decisions(meta, margin, src.log, 1, p.n_slices)
    assert green_rel_err(ch, src) < 1e-10
    ch.close()
