"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test would fail for a plausible slip in the oracle: a wrong coupling or
spin sign (HS identity, brute-force ratios), a wrong Sherman-Morrison term or
a transposed operand (ratios and G from scratch after many updates), a wrong
propagation order or stack slot (U = 0 projector, G from scratch at every
stabilisation point), a wrong delayed recursion (local == delayed decisions),
a wrong force bias or prior ratio (exact detailed balance by enumeration).
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import philox, brute
from oracle.pqmc import Walker, coupling, kinetic_propagators, SPIN_SIGN


# ----------------------------------------------------------------- Philox
def test_philox_matches_numpy_library():
    """Philox4x64-10 bit stream equals numpy.random.Philox (a library routine).
    numpy increments the counter before each block, so start it one below."""
    for key, ctr in [((0, 0), (1, 0, 0, 0)), ((2506096111, 0), (3, 817, 5, 2)),
                     ((2**64 - 1, 12345), (2**64 - 1, 7, 2**63, 3))]:
        c = list(ctr)
        # borrow across words for the pre-decrement
        for w in range(4):
            if c[w] > 0:
                c[w] -= 1
                break
            c[w] = 2**64 - 1
        g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                              counter=np.array(c, dtype=np.uint64))
        ref = tuple(int(v) for v in g.random_raw(4))
        assert philox.philox4x64_10(ctr, key) == ref


def test_uniform_range_and_mean():
    us = [philox.uniform((7, 1), 0, 3, i, philox.PURPOSE_MH) for i in range(4000)]
    assert min(us) >= 0.0 and max(us) < 1.0
    assert abs(np.mean(us) - 0.5) < 0.02


# ------------------------------------------------------------ model pieces
@pytest.mark.parametrize("U", [4.0, 8.0, -4.0, -1.0])
def test_hs_identity(U):
    """Eq. (13): e^{-dtau U (n_up n_dn - (n_up+n_dn)/2)} = 1/2 sum_x e^{alpha x (n_up - n_dn)}
    on all four occupations, for both signs of U (U > 0: real continuation)."""
    dtau = 0.05
    a = coupling(U, dtau)
    for nu, nd in itertools.product((0, 1), (0, 1)):
        lhs = math.exp(-dtau * U * (nu * nd - (nu + nd) / 2.0))
        rhs = 0.5 * sum(np.exp(a * x * (nu - nd)) for x in (+1, -1))
        assert abs(rhs - lhs) < 1e-14


def test_kinetic_propagator_matches_expm():
    p = synth.make_problem(4, 5, 5, 4.0, perturb=1e-3, seed=11)
    K, Kinv = kinetic_propagators(p.hopping, 0.05)
    assert np.max(np.abs(K - scipy.linalg.expm(-0.05 * p.hopping))) < 1e-14
    assert np.max(np.abs(K @ Kinv - np.eye(16))) < 1e-13


def test_lattice_dispersion_and_closed_shells():
    """Unperturbed spectrum equals eps_k = -2t(cos kx + cos ky) (Sec. II A);
    4x4 with N_sigma = 5 is a closed shell with gap 2t."""
    L = 6
    H = synth.square_lattice_hopping(L)
    k = 2 * np.pi * np.arange(L) / L
    ek = np.sort((-2 * (np.cos(k)[:, None] + np.cos(k)[None, :])).ravel())
    assert np.max(np.abs(np.linalg.eigvalsh(H) - ek)) < 1e-12
    p = synth.workload("c1")
    assert abs(p.gap_up - 2.0) < 1e-12


def test_perturbation_keeps_particle_hole_symmetry():
    p = synth.make_problem(6, 17, 17, 4.0, perturb=1e-3, seed=3)
    e = np.linalg.eigvalsh(p.hopping)
    assert np.max(np.abs(e + e[::-1])) < 1e-13


# ------------------------------------------------------------------ U = 0
def test_u0_green_is_projector_everywhere():
    """U = 0: alpha = 0, every ratio is 1, every proposal accepted, and G equals
    the free projector 1 - P P^T at every point of every sweep."""
    p = synth.make_problem(4, 5, 5, 0.0, n_slices=20, stab_every=5, perturb=1e-3, seed=5)
    w = Walker(p, "local")
    G0 = np.eye(16) - p.trial_up @ p.trial_up.T
    orig = w.refresh_T
    errs = []

    def hooked():
        orig()
        errs.append(np.max(np.abs(w.green(0) - G0)))
    w.refresh_T = hooked
    w.sweep(); w.sweep()
    assert len(errs) == 2 * 2 * (20 // 5)
    assert max(errs) < 1e-12
    assert all(e[4] for e in w.log)
    assert max(abs(e[5] + philox.uniform(w.key, e[0], e[1] * 20 + e[2], e[3], 2) - 1.0)
               for e in w.log) < 1e-12


# ----------------------------------------------------- ratios from scratch
def _tiny(L=2, n=1, U=4.0, M=8, kt=4, perturb=1e-3, seed=9, Lx=None):
    return synth.make_problem(L, n, n, U, n_slices=M, stab_every=kt, perturb=perturb, seed=seed)


def _check_trace_against_brute(w, max_checks=400, tol=1e-10):
    P2 = w.P
    n = 0
    for (d, li, site, R, prior, X) in w.trace[:max_checks]:
        Xp = X.copy()
        Xp[li, site] = -Xp[li, site]
        ref = brute.weight_ratio(P2, w.K, w.alpha, X, Xp)
        assert abs(R - ref) <= tol * max(1.0, abs(ref)), (d, li, site, R, ref)
        n += 1
    return n


@pytest.mark.parametrize("scheme,k", [("local", 1), ("delayed", 3)])
def test_ratios_equal_weight_ratios(scheme, k):
    """Eqs. (20)/(28): every proposal's r_up r_dn equals W(X')/W(X) (Eq. (8))
    recomputed from the fields alone, across a full forward+backward sweep."""
    p = synth.make_problem(2, 1, 1, 4.0, n_slices=8, stab_every=4, perturb=1e-3, seed=9)
    w = Walker(p, scheme, k=k)
    w.trace = []
    w.sweep()
    assert _check_trace_against_brute(w) == 2 * 8 * 4


def test_ratios_equal_weight_ratios_4x4():
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=12, stab_every=4, perturb=1e-3, seed=21)
    w = Walker(p, "delayed", k=5)
    w.trace = []
    w.sweep()
    assert _check_trace_against_brute(w, max_checks=120) == 120


def test_negative_u_conjugate_spins():
    """U < 0 (the paper's case): B_dn = conj(B_up) (Sec. II B) so r_dn = conj(r_up)
    and R = |r_up|^2 >= 0 for every proposal."""
    p = synth.make_problem(4, 5, 5, -4.0, n_slices=8, stab_every=4, perturb=1e-3, seed=4)
    w = Walker(p, "local")
    rs = []
    orig = w.metropolis

    def hooked(d, li, site, R, extra=1.0):
        rs.append(R)
        return orig(d, li, site, R, extra)
    w.metropolis = hooked
    # record r_up, r_dn separately through the trace of local ratios
    w.trace = []
    w.sweep()
    Rs = np.array([t[3] for t in w.trace])
    assert np.max(np.abs(Rs.imag)) < 1e-12 * np.max(np.abs(Rs))
    assert np.min(Rs.real) > -1e-12
    X0 = w.trace[0][5]
    Xp = X0.copy(); Xp[0, 0] *= -1
    ru = brute.spin_ratio(w.P[0], w.K, w.alpha, 0, X0, Xp)
    rd = brute.spin_ratio(w.P[1], w.K, w.alpha, 1, X0, Xp)
    assert abs(rd - np.conj(ru)) < 1e-12


def test_green_from_scratch_after_updates():
    """After whole sweeps (thousands of rank-1 updates), G = 1 - U_R T U_L equals
    G recomputed from the fields alone (Eq. (12)), for every scheme."""
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=20, stab_every=5, perturb=1e-3, seed=8)
    for scheme, kw in [("local", {}), ("delayed", {"k": 6}), ("block", {"b": 4})]:
        w = Walker(p, scheme, **kw)
        w.sweep(); w.sweep()
        for s in range(2):
            G = brute.green_at(w.P[s], w.K, w.alpha, s, w.fields, 0)
            assert np.max(np.abs(w.green(s) - G)) < 1e-10, scheme


def test_green_from_scratch_mid_sweep():
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=20, stab_every=5, perturb=1e-3, seed=8)
    w = Walker(p, "local")
    w.forward_window(13)          # position 13, between stabilisations
    for s in range(2):
        G = brute.green_at(w.P[s], w.K, w.alpha, s, w.fields, 13)
        assert np.max(np.abs(w.green(s) - G)) < 1e-10


# ------------------------------------------------- local == delayed chains
@pytest.mark.parametrize("k", [1, 2, 3, 7, 16, 40])
def test_local_and_delayed_make_identical_decisions(k):
    """Sec. III A: the delayed update computes the local update's ratios exactly
    (k = 1 is the local update), so on the same uniforms the chains coincide."""
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=20, stab_every=5, perturb=1e-3, seed=12)
    a = Walker(p, "local")
    b = Walker(p, "delayed", k=k)
    a.sweep(); b.sweep()
    assert [e[4] for e in a.log] == [e[4] for e in b.log]
    assert np.array_equal(a.fields, b.fields)
    for s in range(2):
        assert np.max(np.abs(a.green(s) - b.green(s))) < 1e-10
    assert a.n_accepted / a.n_proposed > 0.5


# ------------------------------------------ block force bias: exact balance
def _walker_at(p, X, l):
    w = Walker(p, "block", b=p.n_slices and 1, fields=X)
    for ll in range(1, l + 1):
        w.prop_forward(ll)
        if ll % w.kt == 0:
            for s in range(2):
                w.UR[s] = np.linalg.qr(w.UR[s])[0]
                w.UL[s] = w.Lstack[s][ll // w.kt].copy()
            w.refresh_T()
    return w


@pytest.mark.parametrize("U,n", [(4.0, 1), (8.0, 2), (-4.0, 1)])
def test_block_force_bias_detailed_balance_by_enumeration(U, n):
    """Sec. III B: one block update with the heat-bath prior and the Metropolis
    test of Eq. (16) satisfies pi(X) K(X->X') = pi(X') K(X'->X), pi ~ |W|,
    for every pair of configurations of a 2x2 lattice with M = 2 (2^8 states)."""
    p = synth.make_problem(2, n, n, U, n_slices=2, stab_every=1, perturb=1e-3, seed=31)
    K, _ = kinetic_propagators(p.hopping, p.dtau)
    alpha = coupling(U, p.dtau)
    Ps = [np.asarray(p.trial_up), np.asarray(p.trial_dn)]
    l, sites = 1, [1, 2, 3]          # slice 1 (position 1), block of three sites
    confs = [np.array(c, np.int8).reshape(2, 4) for c in itertools.product((1, -1), repeat=8)]
    logw = {}
    for X in confs:
        ph, la = brute.log_weight(Ps, K, alpha, X)
        logw[X.tobytes()] = la
    lmax = max(logw.values())

    def pi(X):
        return math.exp(logw[X.tobytes()] - lmax)

    def kernel(X, Xp):
        w = _walker_at(p, X, l)
        s = w.block_force_bias(l - 1, sites)
        pu = w.heat_bath_prob(s)
        xnew = Xp[l - 1, sites].astype(np.int64)
        q = np.prod([pu[j] if xnew[j] > 0 else 1 - pu[j] for j in range(len(sites))])
        F, idx, per_spin, prior = w.block_ratio(l - 1, sites, xnew, s)
        A = abs(per_spin[0][0] * per_spin[1][0] * prior)
        # the ratio must also equal the brute-force weight ratio
        ref = brute.weight_ratio(Ps, K, alpha, X, Xp)
        assert abs(per_spin[0][0] * per_spin[1][0] - ref) < 1e-10 * max(1, abs(ref))
        return q * min(1.0, A)

    rng = np.random.default_rng(0)
    checked = 0
    for X in confs[::7]:
        for _ in range(4):
            Xp = X.copy()
            Xp[l - 1, sites] = rng.choice([1, -1], size=len(sites))
            if np.array_equal(Xp, X):
                continue
            lhs = pi(X) * kernel(X, Xp)
            rhs = pi(Xp) * kernel(Xp, X)
            assert abs(lhs - rhs) < 1e-12 * max(lhs, rhs, 1e-300) + 1e-15
            checked += 1
    assert checked > 60


def test_local_detailed_balance_by_enumeration():
    """Local proposal is symmetric, so pi(X) min(1, W'/W) is symmetric (Eq. (16))."""
    p = synth.make_problem(2, 1, 1, 4.0, n_slices=2, stab_every=1, perturb=1e-3, seed=31)
    w0 = Walker(p, "local")
    X = w0.fields.copy()
    w0.trace = []
    w0.sweep()
    for (d, li, site, R, prior, Xb) in w0.trace[:8]:
        Xp = Xb.copy(); Xp[li, site] *= -1
        ref = brute.weight_ratio(w0.P, w0.K, w0.alpha, Xb, Xp)
        back = brute.weight_ratio(w0.P, w0.K, w0.alpha, Xp, Xb)
        assert abs(ref * back - 1) < 1e-12
        assert abs(R - ref) < 1e-10 * max(1, abs(ref))
