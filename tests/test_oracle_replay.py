"""Pins of the oracle's replay mode and the cross-scheme invariant (CPU).

The local (Sec. II D), delayed (Sec. III A) and block force-bias (Sec. III B)
updates all apply Eq. (19) to the flips they accept.  Forced to accept the
same flips, they must leave the same fields and the same G, and that G must
equal the one rebuilt from the final fields alone (Eq. (12)).
"""
import numpy as np
import pytest

import synth
from oracle import brute
from oracle.pqmc import Walker


def _flip_list_from(w):
    """The accepted flips of the walker's last sweep as a 2M x N list."""
    M, N = w.M, w.N
    flips = np.zeros((2 * M, N), np.int8)
    last = max(e[0] for e in w.log)
    for (sw, d, li, site, acc, margin, sgn) in w.log:
        if sw == last and acc:
            flips[d * M + li, site] = 1
    return flips


@pytest.mark.parametrize("U", [4.0, -4.0])
def test_replay_is_identical_across_schemes(U):
    p = synth.make_problem(4, 5, 5, U, n_slices=20, stab_every=5, perturb=1e-3, seed=61)
    src = Walker(p, "local")
    X0 = src.fields.copy()
    src.sweep()
    flips = _flip_list_from(src)
    assert 0 < flips.sum() < flips.size
    ends = {}
    for scheme, kw in [("local", {}), ("delayed", {"k": 3}), ("delayed", {"k": 7}),
                       ("block", {"b": 4}), ("block", {"b": 5})]:
        w = Walker(p, scheme, fields=X0, **kw)
        w.replay_sweep(flips)
        ends[(scheme, tuple(kw.items()))] = w
        assert np.array_equal(w.fields, src.fields), scheme
    ref = ends[("local", ())]
    # replaying a chain's own decisions reproduces the chain
    for s in range(2):
        assert np.max(np.abs(ref.green(s) - src.green(s))) < 1e-12
    for key, w in ends.items():
        for s in range(2):
            G = brute.green_at(w.P[s], w.K, w.alpha, s, w.fields, 0)
            assert np.max(np.abs(w.green(s) - G)) < 1e-10, key
            assert np.max(np.abs(w.green(s) - ref.green(s))) < 1e-10, key


def test_replay_random_flip_list_and_forced_log():
    """A random list (30% of the visits flip) through every scheme; the log
    records the forced outcomes with margins |A| (taken) and -inf."""
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=10, stab_every=5, perturb=1e-3, seed=62)
    rng = np.random.default_rng(3)
    flips = (rng.random((2 * p.n_slices, p.n_sites)) < 0.3).astype(np.int8)
    Gs = []
    for scheme, kw in [("local", {}), ("delayed", {"k": 6}), ("block", {"b": 3})]:
        w = Walker(p, scheme, **kw)
        X0 = w.fields.copy()
        w.replay_sweep(flips)
        # each slice's parity of flips decides its final field
        changed = (w.fields != X0)
        want = (flips[:p.n_slices] + flips[p.n_slices:][::1]) % 2
        assert np.array_equal(changed, want.astype(bool)), scheme
        Gs.append([w.green(s) for s in range(2)])
        if scheme != "block":
            for (sw, d, li, site, acc, margin, sgn) in w.log:
                assert acc == bool(flips[d * p.n_slices + li, site])
                assert (margin > 0.0) if acc else (margin == -np.inf)
        G0 = brute.green_at(w.P[0], w.K, w.alpha, 0, w.fields, 0)
        assert np.max(np.abs(w.green(0) - G0)) < 1e-10, scheme
    for g in Gs[1:]:
        for s in range(2):
            assert np.max(np.abs(g[s] - Gs[0][s])) < 1e-10
