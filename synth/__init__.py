"""Seeded synthetic inputs for the PQMC field-update sweep.

This module builds the *inputs* of a projector-QMC run on the periodic square
lattice: the hopping matrix H0 (optionally with a seeded random bond
perturbation) and the trial Slater determinant P (the lowest N_sigma orbitals
of H0).  It holds none of the sweep's arithmetic: no propagator, no Green's
function, no ratio, no update.  Both the CPU oracle and the GPU library
consume exactly these arrays, so they start from identical bits.

Model (paper, Sec. II A, Eq. (1)): nearest-neighbour hopping -t on a periodic
L x L lattice, site index i = x + L*y.  The trial state is the ground state of
the non-interacting part (Sec. II B, Eq. (5) and the text after it).

The bond perturbation t_ij = t (1 + eps_ij), eps_ij ~ U(-p, p), lifts the
degeneracy of open-shell fillings; it keeps the lattice bipartite.  Its random
numbers come from numpy's Philox bit generator, keyed by the workload seed.
"""
from __future__ import annotations

import dataclasses
import numpy as np

#: Base of the per-workload seeds: seed_c = SEED_BASE + c.
SEED_BASE = 2506096110


@dataclasses.dataclass
class Problem:
    """One PQMC workload: model inputs plus sweep parameters."""
    L: int
    n_up: int
    n_dn: int
    U: float
    dtau: float
    n_slices: int          # M = 2*Theta/dtau
    stab_every: int        # k_tau
    seed: int
    walker_id: int
    hopping: np.ndarray    # N x N float64, symmetric
    trial_up: np.ndarray   # N x n_up float64, orthonormal columns
    trial_dn: np.ndarray   # N x n_dn float64
    t: float = 1.0
    perturb: float = 0.0
    gap_up: float = 0.0
    gap_dn: float = 0.0

    @property
    def n_sites(self) -> int:
        return self.L * self.L


def square_lattice_hopping(L: int, t: float = 1.0, perturb: float = 0.0,
                           seed: int = 0) -> np.ndarray:
    """H0 for the periodic L x L square lattice, bonds (i, i+x) and (i, i+y).

    With perturb > 0 each of the 2N bonds gets amplitude t(1+eps), eps drawn
    uniformly in [-perturb, perturb) from Philox keyed by (seed, 0x50455254).
    """
    N = L * L
    H = np.zeros((N, N), dtype=np.float64)
    eps = np.zeros(2 * N)
    if perturb > 0.0:
        gen = np.random.Generator(np.random.Philox(key=[seed & (2**64 - 1), 0x50455254]))
        eps = gen.uniform(-perturb, perturb, size=2 * N)
    b = 0
    for y in range(L):
        for x in range(L):
            i = x + L * y
            for dx, dy in ((1, 0), (0, 1)):
                j = ((x + dx) % L) + L * ((y + dy) % L)
                amp = -t * (1.0 + eps[b])
                b += 1
                H[i, j] += amp
                H[j, i] += amp
    return H


def trial_orbitals(H: np.ndarray, n: int):
    """Lowest n eigenvectors of H (ascending) and the gap above them."""
    e, V = np.linalg.eigh(H)
    gap = float(e[n] - e[n - 1]) if n < len(e) else float("inf")
    return np.ascontiguousarray(V[:, :n]), gap


def make_problem(L: int, n_up: int, n_dn: int, U: float, dtau: float = 0.05,
                 n_slices: int = 400, stab_every: int = 10, seed: int = SEED_BASE,
                 walker_id: int = 0, t: float = 1.0, perturb: float = 0.0,
                 min_gap: float = 1e-8) -> Problem:
    H = square_lattice_hopping(L, t, perturb, seed)
    Pu, gu = trial_orbitals(H, n_up)
    Pd, gd = trial_orbitals(H, n_dn)
    if min(gu, gd) <= min_gap:
        raise ValueError(f"open shell: gap {min(gu, gd):.3e} <= {min_gap:g}; add a perturbation")
    return Problem(L=L, n_up=n_up, n_dn=n_dn, U=U, dtau=dtau, n_slices=n_slices,
                   stab_every=stab_every, seed=seed, walker_id=walker_id,
                   hopping=H, trial_up=Pu, trial_dn=Pd, t=t, perturb=perturb,
                   gap_up=gu, gap_dn=gd)


# ---------------------------------------------------------------------------
# Named workloads.  c1: 4x4, N_sigma = 5 (closed shell), U/t = 4.  c2: 16x16,
# N_sigma = 121, U/t = 4, bond perturbation 1e-3.  c3: 40x40, N_sigma = 800
# (half filling), U/t = 4 or 8, bond perturbation 1e-3.  All: dtau = 0.05,
# 2 Theta = 20 (M = 400), stabilisation every 10 slices.
# ---------------------------------------------------------------------------

def workload(name: str, **over) -> Problem:
    specs = {
        "c1": dict(L=4, n_up=5, n_dn=5, U=4.0, perturb=0.0, seed=SEED_BASE + 1),
        "c2": dict(L=16, n_up=121, n_dn=121, U=4.0, perturb=1e-3, seed=SEED_BASE + 2),
        "c3": dict(L=40, n_up=800, n_dn=800, U=4.0, perturb=1e-3, seed=SEED_BASE + 3),
        "c3u8": dict(L=40, n_up=800, n_dn=800, U=8.0, perturb=1e-3, seed=SEED_BASE + 3),
    }
    if name not in specs:
        raise KeyError(name)
    kw = dict(dtau=0.05, n_slices=400, stab_every=10)
    kw.update(specs[name])
    kw.update(over)
    return make_problem(**kw)


# ---------------------------------------------------------------------------
# Spin-orbit coupled (Rashba) Hubbard model, paper Eq. (2) and Appendix A:
# one 2N x 2N complex Hermitian hopping matrix in the basis
# (c_1up .. c_Nup, c_1dn .. c_Ndn) and a trial determinant of N_e orbitals.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SocProblem:
    """One SOC-Hubbard workload: model inputs plus sweep parameters."""
    L: int
    n_e: int
    U: float               # < 0 (the spin-s^y decoupling needs e^{dtau U/2} <= 1)
    lam: float             # Rashba strength lambda
    dtau: float
    n_slices: int
    stab_every: int
    seed: int
    walker_id: int
    hopping: np.ndarray    # 2N x 2N complex128, Hermitian
    trial: np.ndarray      # 2N x n_e complex128, orthonormal columns
    t: float = 1.0
    perturb: float = 0.0
    gap: float = 0.0

    @property
    def n_sites(self) -> int:
        return self.L * self.L


def rashba_hopping(L: int, t: float = 1.0, lam: float = 0.5, perturb: float = 0.0,
                   seed: int = SEED_BASE) -> np.ndarray:
    """2N x 2N hopping of the Rashba model in real space, index s*N + i.

    Spin-diagonal blocks: the square-lattice hopping (with the same seeded
    bond perturbation as square_lattice_hopping).  Spin-flip block: the
    Fourier transform of L_k = 2 lambda (sin k_y - i sin k_x) for
    c+_{k dn} c_{k up}, i.e. for the bond j -> j + d:
        H[dn (j+x), up j] = +lambda,   H[dn (j-x), up j] = -lambda,
        H[dn (j+y), up j] = +i lambda, H[dn (j-y), up j] = -i lambda,
    and the Hermitian conjugate in the up-dn block.
    """
    N = L * L
    H = np.zeros((2 * N, 2 * N), dtype=np.complex128)
    K = square_lattice_hopping(L, t, perturb, seed)
    H[:N, :N] = K
    H[N:, N:] = K
    for y in range(L):
        for x in range(L):
            j = x + L * y
            for (dx, dy), amp in (((1, 0), lam), ((-1, 0), -lam),
                                  ((0, 1), 1j * lam), ((0, -1), -1j * lam)):
                i = ((x + dx) % L) + L * ((y + dy) % L)
                H[N + i, j] += amp
                H[j, N + i] += np.conj(amp)
    return H


def make_soc_problem(L: int, n_e: int, U: float, lam: float = 0.5, dtau: float = 0.05,
                     n_slices: int = 400, stab_every: int = 10, seed: int = SEED_BASE,
                     walker_id: int = 0, t: float = 1.0, perturb: float = 0.0,
                     min_gap: float = 1e-8) -> SocProblem:
    H = rashba_hopping(L, t, lam, perturb, seed)
    e, V = np.linalg.eigh(H)
    gap = float(e[n_e] - e[n_e - 1]) if n_e < len(e) else float("inf")
    if gap <= min_gap:
        raise ValueError(f"open shell: gap {gap:.3e} <= {min_gap:g}; change n_e or perturb")
    return SocProblem(L=L, n_e=n_e, U=U, lam=lam, dtau=dtau, n_slices=n_slices,
                      stab_every=stab_every, seed=seed, walker_id=walker_id, hopping=H,
                      trial=np.ascontiguousarray(V[:, :n_e]), t=t, perturb=perturb, gap=gap)
