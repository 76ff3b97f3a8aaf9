"""Pins of oracle/observables.py against a many-body evaluation in Fock space
and the U = 0 closed form (CPU)."""
import itertools

import numpy as np

import synth
from oracle.observables import energy, double_occupancy


def _fock_ops(nmodes):
    """Dense creation operators c+_m on the 2^nmodes Fock space (Jordan-Wigner:
    sign (-1)^(number of occupied modes below m))."""
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


def _slater(cdag, P_up, P_dn, N):
    """|Phi> = prod_s prod_n (sum_i P_in c+_{i,s}) |0>; mode index s*N + i."""
    dim = cdag[0].shape[0]
    v = np.zeros(dim)
    v[0] = 1.0
    for s, P in enumerate((P_up, P_dn)):
        for n in range(P.shape[1]):
            b = sum(P[i, n] * cdag[s * N + i] for i in range(N))
            v = b @ v
    return v


def _hamiltonian(cdag, H0, U, N):
    c = [C.T for C in cdag]
    H = np.zeros_like(cdag[0])
    for s in range(2):
        for i, j in itertools.product(range(N), range(N)):
            if H0[i, j] != 0.0:
                H += H0[i, j] * cdag[s * N + i] @ c[s * N + j]
    for i in range(N):
        nu = cdag[i] @ c[i]
        nd = cdag[N + i] @ c[N + i]
        H += U * (nu @ nd - 0.5 * (nu + nd))
    return H


def test_mixed_energy_matches_fock_space():
    """Different left and right determinants (the PQMC mixed estimate): the
    formula in G = 1 - R (L R)^{-1} L against <L|H|R> / <L|R> built in the
    2^8-dimensional Fock space of a 2x2 lattice with 2 + 1 fermions."""
    rng = np.random.default_rng(7)
    p = synth.make_problem(2, 2, 1, 3.0, perturb=1e-2, seed=11)
    H0, N = p.hopping, p.n_sites
    cdag = _fock_ops(2 * N)
    H = _hamiltonian(cdag, H0, 3.0, N)
    def orth(n):
        q, _ = np.linalg.qr(rng.standard_normal((N, n)))
        return q
    R_up, R_dn, L_up, L_dn = orth(2), orth(1), orth(2), orth(1)
    vR = _slater(cdag, R_up, R_dn, N)
    vL = _slater(cdag, L_up, L_dn, N)
    want = vL @ H @ vR / (vL @ vR)
    G = [np.eye(N) - R @ np.linalg.inv(L.T @ R) @ L.T for L, R in ((L_up, R_up), (L_dn, R_dn))]
    got = energy(H0, G[0], G[1], 3.0)
    assert abs(got - want) < 1e-12 * max(1.0, abs(want)), (got, want)
    # double occupancy against the Fock-space operator as well
    c = [C.T for C in cdag]
    D = sum(cdag[i] @ c[i] @ cdag[N + i] @ c[N + i] for i in range(N)) / N
    assert abs(double_occupancy(G[0], G[1]) - vL @ D @ vR / (vL @ vR)) < 1e-12


def test_u0_energy_is_sum_of_occupied_levels():
    """U = 0 with the trial state itself: G = 1 - P P^T and E = sum_s sum_{n<N_s} eps_n."""
    p = synth.make_problem(6, 13, 13, 0.0, perturb=1e-3, seed=5)
    eps = np.linalg.eigvalsh(p.hopping)
    G = np.eye(p.n_sites) - p.trial_up @ p.trial_up.T
    assert abs(energy(p.hopping, G, G, 0.0) - 2 * eps[:13].sum()) < 1e-11
