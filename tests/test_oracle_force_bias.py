"""Pins of the oracle's block force bias (Sec. III B) against quantities built
without the walker's running state (CPU).

The force bias of a block is s_i = alpha (nbar_up_i - nbar_dn_i), with
nbar_si the mixed estimate <n_is> = <psi_L| n_is |psi_R> / <psi_L|psi_R> at
the slice being updated, taken with the block's own fields on that slice
removed (their e^{H_I} factors replaced by 1).  Two independent evaluations:

  * from the fields alone: nbar = 1 - diag(G) with G rebuilt from scratch by
    products of propagators in which the block's entries of the slice are 0
    (Eq. (12); the density is <c+_i c_i> = 1 - G_ii for G_ij = <c_i c+_j>);
  * in Fock space: the mixed expectation value of n_is between the two
    Slater determinants R = B_l ... B_1 P and L = P^+ B_M ... B_{l+1}
    (2 x 2 lattice, 2^8 states).

A sign flip of s, G_ii used in place of <n_i>, or a block whose fields are
not removed fails both.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import brute
from oracle.pqmc import Walker, coupling, kinetic_propagators


def _removed(X, li, sites):
    Xr = np.asarray(X, np.float64).copy()
    Xr[li, sites] = 0.0
    return Xr


def _recorded_force_biases(p, b, sweeps=1):
    """Run block-FB sweeps and record every call of the force bias with the
    fields at that moment: (li, sites, s, X)."""
    w = Walker(p, "block", b=b)
    rec = []
    orig = w.block_force_bias

    def hooked(li, sites):
        s = orig(li, sites)
        rec.append((li, list(sites), s.copy(), w.fields.copy()))
        return s
    w.block_force_bias = hooked
    for _ in range(sweeps):
        w.sweep()
    return w, rec


@pytest.mark.parametrize("U,L,n,b", [(4.0, 2, 1, 3), (8.0, 2, 2, 4), (4.0, 4, 5, 3),
                                     (-4.0, 2, 1, 2), (-4.0, 4, 5, 5)])
def test_force_bias_equals_density_from_scratch(U, L, n, b):
    """Every force bias of a forward + backward sweep (slice l is updated at
    position l in both passes) equals alpha (nbar_up - nbar_dn) with nbar =
    1 - G_ii of the configuration whose block fields on slice l are removed."""
    p = synth.make_problem(L, n, n, U, n_slices=8, stab_every=4, perturb=1e-3, seed=41)
    w, rec = _recorded_force_biases(p, b)
    K, _ = kinetic_propagators(p.hopping, p.dtau)
    alpha = coupling(U, p.dtau)
    assert len(rec) == 2 * p.n_slices * ((p.n_sites + b - 1) // b)
    worst = 0.0
    for li, sites, s, X in rec:
        Xr = _removed(X, li, sites)
        nbar = []
        for sp in range(2):
            G = brute.green_at(w.P[sp], K, alpha, sp, Xr, li + 1)
            nbar.append(1.0 - np.diag(G)[sites])
        want = alpha * (nbar[0] - nbar[1])
        if np.iscomplexobj(want):
            assert np.max(np.abs(want.imag)) < 1e-10
            want = want.real
        err = np.max(np.abs(s - want)) / max(1.0, np.max(np.abs(want)))
        worst = max(worst, err)
    assert worst < 1e-9, worst
    # the pin is not vacuous: the force biases are not all near zero
    assert max(np.max(np.abs(r[2])) for r in rec) > 1e-3


def _fock_cdag(nmodes):
    """Creation operators on the 2^nmodes Fock space (Jordan-Wigner order)."""
    dim = 1 << nmodes
    ops = []
    for m in range(nmodes):
        C = np.zeros((dim, dim))
        for st in range(dim):
            if not (st >> m) & 1:
                sign = -1.0 if bin(st & ((1 << m) - 1)).count("1") % 2 else 1.0
                C[st | (1 << m), st] = sign
        ops.append(C)
    return ops


def _slater(cdag, orb, N):
    """prod_s prod_n (sum_i orb[s][i, n] c+_{s N + i}) |0> (complex allowed)."""
    dim = cdag[0].shape[0]
    v = np.zeros(dim, np.complex128)
    v[0] = 1.0
    for s, Pm in enumerate(orb):
        for n in range(Pm.shape[1]):
            v = sum(Pm[i, n] * cdag[s * N + i] for i in range(N)) @ v
    return v


@pytest.mark.parametrize("U,n", [(4.0, 1), (8.0, 2), (-4.0, 2)])
def test_force_bias_equals_fock_space_mixed_density(U, n):
    """2 x 2 lattice, M = 2: s_i / alpha equals <psi_L|n_iup - n_idn|psi_R> /
    <psi_L|psi_R> with the block's fields on the slice removed, the two
    determinants built as states of the 2^8-dimensional Fock space."""
    p = synth.make_problem(2, n, n, U, n_slices=2, stab_every=1, perturb=1e-3, seed=31)
    K, _ = kinetic_propagators(p.hopping, p.dtau)
    alpha = coupling(U, p.dtau)
    N, M = p.n_sites, p.n_slices
    Ps = [np.asarray(p.trial_up), np.asarray(p.trial_dn)]
    cdag = _fock_cdag(2 * N)
    nops = [cdag[m] @ cdag[m].T for m in range(2 * N)]
    sign = (1.0, -1.0)
    rng = np.random.default_rng(5)
    checked = 0
    for trial in range(6):
        X = rng.choice([1, -1], size=(M, N)).astype(np.int8)
        l = 1 + trial % M
        sites = [1, 2, 3] if trial % 2 == 0 else [0, 1]
        w = Walker(p, "block", b=len(sites), fields=X)
        for ll in range(1, l + 1):
            w.prop_forward(ll)
            if ll % w.kt == 0:
                for s in range(2):
                    w.UR[s] = np.linalg.qr(w.UR[s])[0]
                    w.UL[s] = w.Lstack[s][ll // w.kt].copy()
                w.refresh_T()
        s_oracle = w.block_force_bias(l - 1, sites)
        # Slater determinants of the removed configuration, no QR needed at M = 2
        Xr = _removed(X, l - 1, sites)
        Rs, Ls = [], []
        for sp in range(2):
            R = Ps[sp].astype(np.complex128)
            for li in range(l):
                R = np.exp(alpha * sign[sp] * Xr[li])[:, None] * (K @ R)
            Lm = Ps[sp].conj().T.astype(np.complex128)
            for li in range(M - 1, l - 1, -1):
                Lm = (Lm * np.exp(alpha * sign[sp] * Xr[li])[None, :]) @ K
            Rs.append(R)
            Ls.append(Lm.conj().T)        # ket orbitals of |psi_L>
        vR = _slater(cdag, Rs, N)
        vL = _slater(cdag, Ls, N).conj()  # bra <psi_L|
        ov = vL @ vR
        for j, i in enumerate(sites):
            dn = (vL @ (nops[i] - nops[N + i]) @ vR) / ov
            want = alpha * dn
            assert abs(want.imag) < 1e-10 * max(1.0, abs(want))
            assert abs(s_oracle[j] - want.real) < 1e-10 * max(1.0, abs(want)), (trial, j)
            checked += 1
    assert checked >= 12
