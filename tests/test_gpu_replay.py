"""Replay (forced outcomes) and the stabilisation drift statistic on the GPU,
through the C ABI, against the oracle's replay mode.

The cross-scheme invariant: local, delayed and block force-bias updates that
apply the same accepted flips (Eq. (19)) leave the same fields and G.
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


def _flips_of(w):
    M, N = w.M, w.N
    flips = np.zeros((2 * M, N), np.int8)
    last = max(e[0] for e in w.log)
    for (sw, d, li, site, acc, margin, sgn) in w.log:
        if sw == last and acc:
            flips[d * M + li, site] = 1
    return flips


@pytest.mark.parametrize("scheme,kw", [("local", {}), ("delayed", {"k": 4}), ("delayed", {"k": 7}),
                                       ("block", {"b": 4}), ("block", {"b": 3})])
def test_replay_matches_oracle_4x4(scheme, kw):
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 61)
    src = Walker(p, "local")
    src.sweep()
    flips = _flips_of(src)
    w = Walker(p, scheme, **kw)
    w.replay_sweep(flips)
    ch = make_chain(p, scheme, **kw)
    ch.replay(flips)
    meta, margin = ch.decisions()
    n, _ = compare_decisions(meta, margin, w.log, 0, p.n_slices)
    print(f"replay {scheme} {kw}: {n} decisions equal", flush=True)
    assert np.array_equal(ch.fields(), src.fields)
    assert green_rel_err(ch, w) < 1e-10
    ch.close()


@pytest.mark.timeout(300)
def test_replay_cross_scheme_identical_green_16x16():
    """16x16, N_sigma = 121 (projection shortened to M = 20): the oracle's
    local chain's accepted flips replayed through the GPU's local, delayed
    (k = 16) and block force-bias (b = 8) updates give the same fields and G
    to 1e-10, and the G of the oracle chain itself."""
    p = synth.workload("c2", n_slices=20, stab_every=10)
    src = Walker(p, "local")
    src.sweep()
    flips = _flips_of(src)
    Gs = []
    for scheme, kw in [("local", {}), ("delayed", {"k": 16}), ("block", {"b": 8})]:
        ch = make_chain(p, scheme, **kw)
        st = ch.replay(flips)
        assert np.array_equal(ch.fields(), src.fields), scheme
        Gs.append([ch.green(s) for s in range(2)])
        print(f"{scheme}: drift {st['max_stab_drift']:.2e}", flush=True)
        ch.close()
    for g in Gs:
        for s in range(2):
            assert rel_err(g[s], src.green(s)) < 1e-10
            assert rel_err(g[s], Gs[0][s]) < 1e-10


def test_replay_refused_mid_sweep():
    from paper_2506_09611_amd import PQMCError
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=20, stab_every=5, seed=synth.SEED_BASE + 62)
    ch = make_chain(p, "delayed", k=4)
    ch.forward_window(3)
    with pytest.raises(PQMCError):
        ch.replay(np.zeros((40, 16), np.int8))
    ch.close()


@pytest.mark.parametrize("fp32", [False, True])
def test_stabilisation_drift_statistic(fp32):
    """The largest entry of G that a stabilisation corrects: at rounding level
    for the float64 chain, at the float32 level for the precision form, and
    never zero (it is measured, not assumed)."""
    p = synth.workload("c2", n_slices=40, stab_every=10)
    ch = make_chain(p, "delayed", k=16, fp32=fp32)
    st = ch.sweep(1)
    d = st["max_stab_drift"]
    print(f"fp32={fp32}: drift {d:.3e}", flush=True)
    assert np.isfinite(d) and d > 0.0
    if fp32:
        assert 1e-9 < d < 1e-3
    else:
        assert d < 1e-9
    ch.close()
