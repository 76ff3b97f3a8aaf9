"""Energy and double occupancy from equal-time Green's functions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Written from the paper's
standard Hubbard Hamiltonian (Sec. II A, Eq. (1)),

    H = sum_{ij,s} H0_ij c+_is c_js + U sum_i [n_iup n_idn - (n_iup + n_idn) / 2],

evaluated as the PQMC mixed estimate <psi_L| O |psi_R> / <psi_L|psi_R> for
one field configuration.  With G_ij = <c_i c+_j> (Sec. II B, the Green's
function of Eq. (15)), <c+_i c_j> = delta_ij - G_ji; the two spin sectors
are independent Slater determinants, so <n_iup n_idn> is the product of the
two densities (Wick's theorem within each sector).
"""
from __future__ import annotations

import numpy as np


def densities(G):
    """<n_i> = 1 - G_ii for one spin sector."""
    return 1.0 - np.real_if_close(np.diag(G))


def kinetic_energy(H0, G):
    """sum_ij H0_ij <c+_i c_j> = sum_ij H0_ij (delta_ij - G_ji) for one sector."""
    return np.trace(H0) - np.sum(H0 * G.T)


def energy(H0, G_up, G_dn, U):
    n_up, n_dn = densities(G_up), densities(G_dn)
    pot = U * np.sum(n_up * n_dn - 0.5 * (n_up + n_dn))
    return kinetic_energy(H0, G_up) + kinetic_energy(H0, G_dn) + pot


def double_occupancy(G_up, G_dn):
    """N^{-1} sum_i <n_iup n_idn>."""
    return float(np.mean(densities(G_up) * densities(G_dn)))
