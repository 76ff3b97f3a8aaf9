"""Pins of the SOC-Hubbard oracle (oracle/soc.py) against the paper's
definitions, many-body evaluations in Fock space and brute force (CPU).

  * the Rashba hopping matrix against its k-space definition, Eq. (2);
  * the spin-s^y decoupling, Eq. (A4), as an operator identity on one site;
  * B_l (the 2x2 rotations of Eq. (A6) on rows (i, N+i) after e^{-dtau H0}) as
    the one-body form of the Fock-space propagator (Thouless), and the sum
    over all fields of a 2x2 lattice against the Trotter product;
  * the rank-two ratios, Eqs. (A7)-(A8), against brute-force weight ratios;
  * G against its definition; delayed = local; real non-negative ratios.
"""
import itertools

import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import soc
from oracle.soc import SocWalker


def _fock_ops(nmodes):
    dim = 1 << nmodes
    ops = []
    for m in range(nmodes):
        C = np.zeros((dim, dim))
        for s in range(dim):
            if not (s >> m) & 1:
                sign = -1.0 if bin(s & ((1 << m) - 1)).count("1") % 2 else 1.0
                C[s | (1 << m), s] = sign
        ops.append(C)
    return ops


def _one_body(cdag, h):
    """c+ h c on Fock space."""
    c = [C.T for C in cdag]
    out = np.zeros(cdag[0].shape, dtype=np.complex128)
    for p, q in itertools.product(range(h.shape[0]), repeat=2):
        if h[p, q] != 0:
            out += h[p, q] * (cdag[p] @ c[q])
    return out


def _slater(cdag, P):
    v = np.zeros(cdag[0].shape[0], dtype=np.complex128)
    v[0] = 1.0
    for n in range(P.shape[1]):
        v = sum(P[p, n] * cdag[p] for p in range(P.shape[0])) @ v
    return v


def test_rashba_hopping_matches_k_space_definition():
    """H[s i, s' j] = (1/N) sum_k h_{s s'}(k) e^{i k (r_i - r_j)} with
    h(k) = [[eps_k, conj(L_k)], [L_k, eps_k]] in (up, dn), eps_k =
    -2t(cos kx + cos ky), L_k = 2 lambda (sin ky - i sin kx)."""
    L, t, lam = 4, 1.0, 0.37
    N = L * L
    H = synth.rashba_hopping(L, t, lam, 0.0)
    ks = [(2 * np.pi * a / L, 2 * np.pi * b / L) for b in range(L) for a in range(L)]
    r = np.array([(i % L, i // L) for i in range(N)], dtype=float)
    ref = np.zeros((2 * N, 2 * N), dtype=np.complex128)
    for kx, ky in ks:
        eps = -2 * t * (np.cos(kx) + np.cos(ky))
        Lk = 2 * lam * (np.sin(ky) - 1j * np.sin(kx))
        h = np.array([[eps, np.conj(Lk)], [Lk, eps]])
        ph = np.exp(1j * (r @ np.array([kx, ky])))          # e^{i k r_i}
        F = np.outer(ph, ph.conj()) / N                     # e^{i k (r_i - r_j)} / N
        for s, sp in itertools.product(range(2), repeat=2):
            ref[s * N:(s + 1) * N, sp * N:(sp + 1) * N] += h[s, sp] * F
    assert np.abs(H - ref).max() < 1e-12
    e = np.linalg.eigvalsh(H)
    spec = sorted(-2 * t * (np.cos(kx) + np.cos(ky)) + sgn * 2 * lam *
                  np.hypot(np.sin(ky), np.sin(kx)) for kx, ky in ks for sgn in (-1, 1))
    assert np.allclose(e, spec, atol=1e-12)


@pytest.mark.parametrize("U,dtau", [(-4.0, 0.05), (-1.0, 0.1), (-8.0, 0.02)])
def test_spin_sy_decoupling_is_an_operator_identity(U, dtau):
    """Eq. (A4) on the 4-dimensional Fock space of one site."""
    cdag = _fock_ops(2)                       # mode 0: up, mode 1: dn
    c = [C.T for C in cdag]
    nu, nd = cdag[0] @ c[0], cdag[1] @ c[1]
    lhs = expm(-dtau * U * (nu @ nd - 0.5 * (nu + nd)))
    g = soc.soc_coupling(U, dtau)
    O = cdag[0] @ c[1] - cdag[1] @ c[0]
    rhs = 0.5 * sum(expm(g * x * O) for x in (1, -1))
    assert np.abs(lhs - rhs).max() < 1e-13
    # its one-body matrix is A(x) of Eq. (A6): e^{c+ h c} c+_a|0> = sum_b (e^h)_{ba} c+_b|0>
    for x in (1, -1):
        E = expm(g * x * O)
        A = np.array([[E[1 << b, 1 << a] for a in range(2)] for b in range(2)])
        assert np.allclose(A, soc.rotation(g, x), atol=1e-14)


def _small_problem(U=-4.0, n_slices=2):
    return synth.make_soc_problem(2, 4, U, lam=0.5, dtau=0.1, n_slices=n_slices, stab_every=1,
                                  perturb=5e-2, seed=synth.SEED_BASE + 81)


def test_weight_is_the_fock_space_amplitude():
    """det(P^+ B_M..B_1 P) = <Psi_T| prod_l B_I(x_l) e^{-dtau H0} |Psi_T> (Thouless)
    on a 2x2 lattice (8 modes), for random fields."""
    p = _small_problem()
    N = 4
    cdag = _fock_ops(2 * N)
    c = [C.T for C in cdag]
    g = soc.soc_coupling(p.U, p.dtau)
    Kf = expm(-p.dtau * _one_body(cdag, p.hopping))
    Oi = [cdag[i] @ c[N + i] - cdag[N + i] @ c[i] for i in range(N)]
    psi = _slater(cdag, p.trial)
    K, _ = soc.kinetic_propagators(p.hopping, p.dtau)
    rng = np.random.default_rng(3)
    for _ in range(3):
        X = rng.choice([-1, 1], size=(p.n_slices, N)).astype(np.int8)
        v = psi.copy()
        for li in range(p.n_slices):
            BI = expm(g * sum(float(X[li, i]) * Oi[i] for i in range(N)))
            v = BI @ (Kf @ v)
        amp = psi.conj() @ v
        w = soc.weight(p.trial, K, g, X)
        assert abs(w - amp) < 1e-12 * max(1.0, abs(amp))


def test_field_sum_reproduces_the_trotter_product():
    """sum_X W(X) / 2^{N M} = <Psi_T| (e^{-dtau H_I} e^{-dtau H0})^M |Psi_T> with
    H_I = U sum_i (n_up n_dn - (n_up + n_dn)/2): Eq. (A4) applied to every
    site and slice of a 2x2 lattice, M = 2 (256 configurations)."""
    p = _small_problem()
    N, M = 4, p.n_slices
    cdag = _fock_ops(2 * N)
    c = [C.T for C in cdag]
    Hk = _one_body(cdag, p.hopping)
    HI = sum(p.U * (cdag[i] @ c[i] @ cdag[N + i] @ c[N + i]
                    - 0.5 * (cdag[i] @ c[i] + cdag[N + i] @ c[N + i])) for i in range(N))
    step = expm(-p.dtau * HI) @ expm(-p.dtau * Hk)
    psi = _slater(cdag, p.trial)
    ref = psi.conj() @ np.linalg.matrix_power(step, M) @ psi
    g = soc.soc_coupling(p.U, p.dtau)
    K, _ = soc.kinetic_propagators(p.hopping, p.dtau)
    tot = 0.0
    for bits in range(1 << (N * M)):
        X = np.array([1 if (bits >> b) & 1 else -1 for b in range(N * M)], np.int8).reshape(M, N)
        tot += soc.weight(p.trial, K, g, X)
    assert abs(tot / 2 ** (N * M) - ref) < 1e-12 * abs(ref)


def _traced(walker_cls):
    """A walker whose Metropolis calls record (R, fields before the decision)."""
    class Traced(walker_cls):
        def metropolis(self, d, li, site, R):
            self.trace.append((d, li, site, R, self.fields.copy()))
            return super().metropolis(d, li, site, R)
    return Traced


@pytest.mark.parametrize("scheme,k", [("local", 1), ("delayed", 3)])
def test_ratios_equal_brute_force_weight_ratios(scheme, k):
    """Every proposal's R = W(X') / W(X) (Eq. (A7)) on a 2x2 lattice, through a
    whole sweep that crosses stabilisations; R real and non-negative."""
    p = synth.make_soc_problem(2, 4, -4.0, lam=0.5, dtau=0.1, n_slices=4, stab_every=2,
                               perturb=5e-2, seed=synth.SEED_BASE + 82)
    w = _traced(SocWalker)(p, scheme, k=k)
    w.trace = []
    w.sweep()
    g = soc.soc_coupling(p.U, p.dtau)
    K, _ = soc.kinetic_propagators(p.hopping, p.dtau)
    assert len(w.trace) == 2 * p.n_slices * 4
    for d, li, site, R, X in w.trace:
        Xp = X.copy()
        Xp[li, site] = -Xp[li, site]
        ref = soc.weight(p.trial, K, g, Xp) / soc.weight(p.trial, K, g, X)
        assert abs(R - ref) < 1e-9 * max(1.0, abs(ref)), (d, li, site, R, ref)
        assert abs(np.imag(R)) < 1e-9 * max(1.0, abs(R)) and np.real(R) > -1e-12


def test_green_matches_definition_after_a_sweep():
    p = synth.make_soc_problem(4, 14, -4.0, lam=0.5, dtau=0.05, n_slices=8, stab_every=4,
                               perturb=1e-3, seed=synth.SEED_BASE + 83)
    w = SocWalker(p, "local")
    w.sweep()
    g = soc.soc_coupling(p.U, p.dtau)
    K, _ = soc.kinetic_propagators(p.hopping, p.dtau)
    ref = soc.green_at(p.trial, K, g, w.fields, 0)
    assert np.abs(w.green() - ref).max() < 1e-9
    w.forward_window(5)
    ref5 = soc.green_at(p.trial, K, g, w.fields, 5)
    assert np.abs(w.green() - ref5).max() < 1e-9


@pytest.mark.parametrize("k", [2, 5, 16])
def test_delayed_takes_the_local_decisions(k):
    """The delayed update is the local update reorganised (Sec. III A): same
    decisions, same G, for any group size."""
    p = synth.make_soc_problem(4, 16, -4.0, lam=0.5, dtau=0.05, n_slices=10, stab_every=5,
                               perturb=1e-3, seed=synth.SEED_BASE + 84)
    a, b = SocWalker(p, "local"), SocWalker(p, "delayed", k=k)
    a.sweep()
    b.sweep()
    assert [e[4] for e in a.log] == [e[4] for e in b.log]
    assert np.array_equal(a.fields, b.fields)
    assert np.abs(a.green() - b.green()).max() < 1e-10
    assert 0.3 < a.n_accepted / a.n_proposed < 1.0


def test_zero_coupling_accepts_everything():
    """U = 0: gamma = 0, A = 1, every ratio is 1 (all proposals accepted)."""
    p = synth.make_soc_problem(2, 4, 0.0, lam=0.5, dtau=0.1, n_slices=2, stab_every=1,
                               perturb=5e-2, seed=synth.SEED_BASE + 85)
    w = SocWalker(p, "local")
    w.sweep()
    assert all(e[4] for e in w.log) and w.n_flips == w.n_proposed


# ------------------------------------------------------------ block force bias
def test_mixed_one_body_density_index_order():
    """<L| c+_p c_q |R> / <L|R> = [R (L R)^{-1} L]_{qp} for Slater determinants
    (8 modes, random complex orbitals): the order the force bias uses."""
    rng = np.random.default_rng(11)
    n, ne = 8, 3
    R = rng.normal(size=(n, ne)) + 1j * rng.normal(size=(n, ne))
    Lh = rng.normal(size=(n, ne)) + 1j * rng.normal(size=(n, ne))   # |L> has orbitals Lh
    cdag = _fock_ops(n)
    c = [C.T for C in cdag]
    vr, vl = _slater(cdag, R), _slater(cdag, Lh)
    L = Lh.conj().T
    M = R @ np.linalg.inv(L @ R) @ L
    ov = vl.conj() @ vr
    for p_, q_ in [(0, 1), (3, 5), (6, 2), (4, 4)]:
        amp = vl.conj() @ (cdag[p_] @ c[q_]) @ vr / ov
        assert abs(amp - M[q_, p_]) < 1e-12


def _walker_at_slice(p, X, scheme="block", b=4):
    w = SocWalker(p, scheme, b=b, fields=X)
    w.prop_forward(1)
    return w


def test_force_bias_is_the_fock_space_mixed_estimate():
    """s_i / gamma = <psi_l| O_i |psi_r> / <psi_l|psi_r> with O_i the operator of
    Eq. (A4), <psi_l| = U_L and |psi_r> = U_R with the block's fields removed,
    evaluated in the 2^8-dimensional Fock space of a 2x2 lattice."""
    p = synth.make_soc_problem(2, 4, -4.0, lam=0.5, dtau=0.1, n_slices=2, stab_every=1,
                               perturb=5e-2, seed=synth.SEED_BASE + 86)
    rng = np.random.default_rng(5)
    X = rng.choice([-1, 1], size=(p.n_slices, 4)).astype(np.int8)
    w = _walker_at_slice(p, X)
    N, sites = 4, [0, 1, 2, 3]
    svec = w.block_force_bias(0, sites)
    URb = w.UR.copy()
    for i in sites:
        URb[[i, N + i], :] = soc.rotation(w.gamma, -float(X[0, i])) @ w.UR[[i, N + i], :]
    cdag = _fock_ops(2 * N)
    c = [C.T for C in cdag]
    vr, vl = _slater(cdag, URb), _slater(cdag, w.UL.conj().T)
    ov = vl.conj() @ vr
    for i in sites:
        O = cdag[i] @ c[N + i] - cdag[N + i] @ c[i]
        o = vl.conj() @ O @ vr / ov
        assert abs(w.gamma * o - svec[i]) < 1e-10 * max(1.0, abs(svec[i])), (i, o, svec[i])
    assert np.max(np.abs(svec)) > 1e-3


def test_block_ratios_equal_brute_force():
    """R of a block proposal equals W(X') / W(X) from scratch, and whole
    sweeps of the block update keep G equal to its definition."""
    p = synth.make_soc_problem(2, 4, -4.0, lam=0.5, dtau=0.1, n_slices=4, stab_every=2,
                               perturb=5e-2, seed=synth.SEED_BASE + 87)

    g = soc.soc_coupling(p.U, p.dtau)
    K, _ = soc.kinetic_propagators(p.hopping, p.dtau)
    # one proposal (3 of 4 fields flipped) against W(X') / W(X)
    w2 = SocWalker(p, "block", b=4)
    w2.prop_forward(1)
    sites = [0, 1, 2, 3]
    svec = w2.block_force_bias(0, sites)
    xnew = -w2.fields[0, sites].astype(np.int64)
    xnew[1] = w2.fields[0, 1]
    F, idx, R, *_ = w2.block_ratio(0, sites, xnew, svec)
    Xp = w2.fields.copy()
    Xp[0, sites] = xnew
    ref = soc.weight(p.trial, K, g, Xp) / soc.weight(p.trial, K, g, w2.fields)
    assert len(F) == 3 and abs(R - ref) < 1e-9 * abs(ref)
    # every proposal of two sweeps (T upgraded between them by Eq. (36))
    class Traced(SocWalker):
        def block_ratio(self, li, sites, xnew, svec):
            out = super().block_ratio(li, sites, xnew, svec)
            self.trace.append((li, list(sites), np.array(xnew), self.fields.copy(), out[2]))
            return out

    w3 = Traced(p, "block", b=3)
    w3.trace = []
    w3.sweep()
    w3.sweep()
    n = 0
    for li, sites, xnew, X, R in w3.trace:
        Xp = X.copy()
        Xp[li, sites] = xnew
        if np.array_equal(Xp, X):
            continue
        ref = soc.weight(p.trial, K, g, Xp) / soc.weight(p.trial, K, g, X)
        assert abs(R - ref) < 1e-9 * max(1.0, abs(ref)), (li, sites, R, ref)
        n += 1
    assert n > 10 and w3.n_flips > 0


def test_block_update_detailed_balance_by_enumeration():
    """2x2 lattice, M = 2 with slice 2 fixed, one block of the 4 sites of
    slice 1: the Markov kernel
    K(X -> X') = q(X') min(1, pi(X') q(X) / (pi(X) q(X'))) built from the
    walker's force bias and ratios satisfies pi(X) K(X -> X') = pi(X') K(X' -> X)
    with pi = |W| (16 configurations)."""
    p = synth.make_soc_problem(2, 4, -4.0, lam=0.5, dtau=0.1, n_slices=2, stab_every=1,
                               perturb=5e-2, seed=synth.SEED_BASE + 88)
    g = soc.soc_coupling(p.U, p.dtau)
    K, _ = soc.kinetic_propagators(p.hopping, p.dtau)
    x2 = np.array([1, -1, -1, 1], np.int8)          # slice 2 fixed: the force bias is not 0
    confs = [np.array([1 if (c >> i) & 1 else -1 for i in range(4)], np.int8) for c in range(16)]
    pi = [abs(soc.weight(p.trial, K, g, np.stack([x, x2]))) for x in confs]
    sites = [0, 1, 2, 3]
    Km = np.zeros((16, 16))
    for a, xa in enumerate(confs):
        w = _walker_at_slice(p, np.stack([xa, x2]))
        if a == 0:
            assert np.max(np.abs(w.block_force_bias(0, sites))) > 1e-2
        svec = w.block_force_bias(0, sites)
        pu = w.heat_bath_prob(svec)
        for bidx, xb in enumerate(confs):
            q = np.prod([pu[j] if xb[j] > 0 else 1.0 - pu[j] for j in range(4)])
            if bidx == a:
                continue
            F, idx, R, Vp, Up, Wp, dF, prior = w.block_ratio(0, sites, xb.astype(np.int64), svec)
            Km[a, bidx] = q * min(1.0, abs(R * prior))
    for a in range(16):
        for bidx in range(16):
            assert abs(pi[a] * Km[a, bidx] - pi[bidx] * Km[bidx, a]) < 1e-12 * max(pi)
    assert Km.sum() > 0
