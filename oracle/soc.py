"""Oracle walker for the spin-orbit coupled Hubbard model (PQMC, complex128).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain NumPy, written from
Du & He, arXiv:2506.09611, Appendix A (PQMC for spin-coupled systems) and
Sec. IV C (the SOC-Hubbard tests):

  * one sector in the generalised Hartree-Fock basis (c_1up..c_Nup,
    c_1dn..c_Ndn): P is 2N x N_e, U_R 2N x N_e, U_L N_e x 2N, T N_e x N_e
    and G = 1 - U_R T U_L is 2N x 2N (Appendix A);
  * HS transformation in the spin-s^y channel, Eq. (A4): coupling
    gamma = arccos(e^{dtau U/2}) for U < 0, and e^{H_I(x)} the product over
    sites of the 2x2 rotation A(x_i) = e^{gamma x_i i sigma_y}, Eq. (A6), acting
    on the pair of rows (i, N + i);
  * B_l = e^{H_I(x_l)} e^{-dtau H0} (Appendix A), the same sweep and QR
    stabilisation as the spin-decoupled walker (Sec. II B);
  * local update of rank two, Eqs. (A7)-(A9): delta_i = A(x') A(x)^{-1} - 1,
    V = (v_i | v_{N+i}) delta_i, Y = (u_i | u_{N+i})^T T, R = det(1_2 + Y V);
  * delayed update with the x_m, y_m of Eqs. (28)-(30) grown into N_e x 2 and
    2 x N_e blocks (end of Appendix A);
  * block force-bias update (Sec. III B, Eqs. (31)-(36), with the force bias
    of the spin-s^y decoupling as Appendix A describes it).

Readings (each listed in the design notes):
  * The T upgrade of Eq. (A9) is written with X = T V / R; for the rank-two
    update X = T V (1_2 + Y V)^{-1} (the Woodbury identity that Eq. (A8)
    reduces to), which is what is used here.
  * Accept iff u < |R| (R is real and non-negative up to rounding: the
    decoupling keeps time-reversal symmetry, so the weight has no sign
    problem, Sec. II A); the sign of Re R is logged.
  * Block force bias: the block's fields are removed by rotating its row
    pairs of U_R by A(-x_i); the exponent is s_i = gamma <O_i> with
    O_i = c+_{i up} c_{i dn} - c+_{i dn} c_{i up} (the operator of Eq. (A4)),
    whose mixed estimate is real here; <c+_p c_q> = [R (L R)^{-1} L]_{q p}
    (the paper prints the index pair as (i, N+i); the Fock-space pin fixes
    the order).  Heat bath P(x' = +1) = 1 / (1 + e^{-2 s}); an empty flip set
    is an accepted no-op; accept iff u < |R prior| with
    prior = prod_F e^{s_i (x_i - x'_i)}, as in the spin-decoupled walker.
"""
from __future__ import annotations

import math
import numpy as np

from . import philox

SOC_SCHEMES = ("local", "delayed", "block")


def soc_coupling(U: float, dtau: float) -> float:
    """gamma = arccos(e^{dtau U/2}) of Eq. (A4); needs U <= 0."""
    if U > 0:
        raise ValueError("the spin-s^y decoupling needs U <= 0")
    return math.acos(math.exp(dtau * U / 2.0))


def rotation(gamma: float, x: float) -> np.ndarray:
    """A(x) = e^{gamma x i sigma_y}, Eq. (A6)."""
    c, s = math.cos(gamma * x), math.sin(gamma * x)
    return np.array([[c, s], [-s, c]])


def kinetic_propagators(H0: np.ndarray, dtau: float):
    """K = e^{-dtau H0}, K^{-1} = e^{dtau H0} for Hermitian H0 (eigendecomposition)."""
    e, V = np.linalg.eigh(H0)
    K = (V * np.exp(-dtau * e)) @ V.conj().T
    Kinv = (V * np.exp(dtau * e)) @ V.conj().T
    return K, Kinv


def apply_rows(gamma, xrow, A, sign=1.0):
    """e^{sign H_I(x)} A: rows (i, N+i) of A mixed by A(sign x_i)."""
    N = len(xrow)
    out = A.copy()
    for i in range(N):
        R = rotation(gamma, sign * float(xrow[i]))
        out[[i, N + i], :] = R @ A[[i, N + i], :]
    return out


def apply_cols(gamma, xrow, A, sign=1.0):
    """A e^{sign H_I(x)}: columns (i, N+i) of A mixed by A(sign x_i)."""
    N = len(xrow)
    out = A.copy()
    for i in range(N):
        R = rotation(gamma, sign * float(xrow[i]))
        out[:, [i, N + i]] = A[:, [i, N + i]] @ R
    return out


def b_matrix(gamma, K, xrow):
    """B_l = e^{H_I(x_l)} e^{-dtau H0} (Appendix A), dense 2N x 2N."""
    return apply_rows(gamma, xrow, K)


def orthonormalize_columns(A):
    return np.linalg.qr(A)[0]


def orthonormalize_rows(A):
    return np.linalg.qr(A.conj().T)[0].conj().T


class SocWalker:
    """One Markov chain of the SOC-Hubbard PQMC field configuration.

    fields[l-1, i] = x_{l,i} = +-1; UR (2N x N_e), UL (N_e x 2N), T (N_e x N_e).
    """

    def __init__(self, prob, scheme="local", k=1, b=1, fields=None):
        if scheme not in SOC_SCHEMES:
            raise ValueError(scheme)
        self.b = max(1, int(b))
        self.p = prob
        self.N = prob.hopping.shape[0] // 2
        self.M = prob.n_slices
        self.kt = prob.stab_every
        if self.M % self.kt:
            raise ValueError("stab_every must divide n_slices")
        self.scheme, self.k = scheme, max(1, int(k))
        self.gamma = soc_coupling(prob.U, prob.dtau)
        self.K, self.Kinv = kinetic_propagators(prob.hopping, prob.dtau)
        self.P = np.asarray(prob.trial, np.complex128)
        self.key = (prob.seed, prob.walker_id)
        self.sweep_index = 0
        if fields is None:
            fields = self.initial_fields()
        self.fields = np.array(fields, dtype=np.int8).reshape(self.M, self.N)
        self.log = []          # (sweep, dir, slice, site, accept, margin, sign)
        self.hb_log = []       # block force bias: (sweep, dir, slice, site, x_new, margin)
        self.n_proposed = self.n_accepted = self.n_flips = 0
        self.build_initial_state()

    # ------------------------------------------------------------------ setup
    def initial_fields(self):
        """x_{l,i} = +1 iff u(INIT; 0, l-1, i) < 1/2 (as in the spin-decoupled walker)."""
        X = np.empty((self.M, self.N), np.int8)
        for li in range(self.M):
            for i in range(self.N):
                u = philox.uniform(self.key, 0, li, i, philox.PURPOSE_INIT)
                X[li, i] = 1 if u < 0.5 else -1
        return X

    def build_initial_state(self):
        M, kt = self.M, self.kt
        ns = M // kt
        self.Lstack = [None] * (ns + 1)
        self.Rstack = [None] * (ns + 1)
        UL = self.P.conj().T.copy()
        self.Lstack[ns] = UL.copy()
        for l in range(M, 0, -1):
            UL = apply_cols(self.gamma, self.fields[l - 1], UL) @ self.K     # U_L B_l
            if (l - 1) % kt == 0:
                UL = orthonormalize_rows(UL)
                self.Lstack[(l - 1) // kt] = UL.copy()
        self.Rstack[0] = self.P.copy()
        self.UR = self.P.copy()
        self.UL = self.Lstack[0].copy()
        self.T = np.linalg.inv(self.UL @ self.UR)

    # ------------------------------------------------------------ propagation
    def prop_forward(self, l):
        """U_R <- B_l U_R, U_L <- U_L B_l^{-1} = U_L K^{-1} e^{-H_I(x_l)}."""
        x = self.fields[l - 1]
        self.UR = apply_rows(self.gamma, x, self.K @ self.UR)
        self.UL = apply_cols(self.gamma, x, self.UL @ self.Kinv, -1.0)

    def prop_backward(self, l):
        """U_L <- U_L B_l, U_R <- B_l^{-1} U_R = K^{-1} e^{-H_I(x_l)} U_R."""
        x = self.fields[l - 1]
        self.UL = apply_cols(self.gamma, x, self.UL) @ self.K
        self.UR = self.Kinv @ apply_rows(self.gamma, x, self.UR, -1.0)

    def refresh_T(self):
        self.T = np.linalg.inv(self.UL @ self.UR)

    def _stab_forward(self, l):
        j = l // self.kt
        self.UR = orthonormalize_columns(self.UR)
        self.Rstack[j] = self.UR.copy()
        self.UL = self.Lstack[j].copy()
        self.refresh_T()

    def _stab_backward(self, l):
        j = (l - 1) // self.kt
        self.UL = orthonormalize_rows(self.UL)
        self.Lstack[j] = self.UL.copy()
        self.UR = self.Rstack[j].copy()
        self.refresh_T()

    def sweep(self):
        M, kt = self.M, self.kt
        for l in range(1, M + 1):
            self.prop_forward(l)
            self.update_slice(l, 0)
            if l % kt == 0:
                self._stab_forward(l)
        for l in range(M, 0, -1):
            self.update_slice(l, 1)
            self.prop_backward(l)
            if (l - 1) % kt == 0:
                self._stab_backward(l)
        self.sweep_index += 1

    def forward_window(self, n_slices):
        for l in range(1, n_slices + 1):
            self.prop_forward(l)
            self.update_slice(l, 0)
            if l % self.kt == 0:
                self._stab_forward(l)

    def update_slice(self, l, d):
        if self.scheme == "local":
            self.local_slice(l, d)
        elif self.scheme == "delayed":
            self.delayed_slice(l, d)
        else:
            self.block_slice(l, d)

    # ---------------------------------------------------------- decisions
    def flip_block(self, li, i):
        """delta_i = A(x') A(x)^{-1} - 1 with x' = -x (Appendix A)."""
        x = float(self.fields[li, i])
        return rotation(self.gamma, -x) @ rotation(self.gamma, -x) - np.eye(2)

    def metropolis(self, d, li, site, R, extra=1.0):
        with np.errstate(over="ignore", invalid="ignore"):
            R = R * extra
            absR = abs(R)
        if np.isnan(absR):
            raise FloatingPointError("acceptance ratio is NaN")
        u = philox.uniform(self.key, self.sweep_index, d * self.M + li, site, philox.PURPOSE_MH)
        acc = u < absR
        sgn = 1.0 if np.real(R) >= 0 else -1.0
        self.log.append((self.sweep_index, d, li, site, bool(acc), absR - u, sgn))
        self.n_proposed += 1
        self.n_accepted += int(acc)
        return acc

    def _accept_rows(self, li, i, delta):
        rows = [i, self.N + i]
        self.UR[rows, :] = (np.eye(2) + delta) @ self.UR[rows, :]
        self.fields[li, i] = -self.fields[li, i]
        self.n_flips += 1

    # ----------------------------------------------------------- local update
    def local_slice(self, l, d):
        """Rank-two local update of slice l, Eqs. (A7)-(A9), sites in order."""
        li = l - 1
        N = self.N
        for i in range(N):
            delta = self.flip_block(li, i)
            V = self.UL[:, [i, N + i]] @ delta              # N_e x 2
            Y = self.UR[[i, N + i], :] @ self.T             # 2 x N_e
            S = np.eye(2) + Y @ V
            if self.metropolis(d, li, i, np.linalg.det(S)):
                X = self.T @ V @ np.linalg.inv(S)
                self.T = self.T - X @ Y
                self._accept_rows(li, i, delta)

    # --------------------------------------------------------- delayed update
    def delayed_slice(self, l, d):
        """Delayed update with N_e x 2 blocks X_m and 2 x N_e blocks Y_m: the
        spin-decoupled Eqs. (28)-(30) with every vector grown to two columns."""
        li = l - 1
        N, k = self.N, min(self.k, self.N)
        ne = self.T.shape[0]
        for g0 in range(0, N, k):
            sites = list(range(g0, min(g0 + k, N)))
            T0 = self.T
            Xs = np.zeros((ne, 0), np.complex128)
            Ys = np.zeros((0, ne), np.complex128)
            for i in sites:
                delta = self.flip_block(li, i)
                W = self.UR[[i, N + i], :]                  # rows of site i (not yet changed)
                V = self.UL[:, [i, N + i]] @ delta
                c = W @ Xs                                  # 2 x 2|A|
                dd = Ys @ V                                 # 2|A| x 2
                Y = W @ T0 - c @ Ys                         # W T_current
                TV = T0 @ V - Xs @ dd                       # T_current V
                S = np.eye(2) + W @ T0 @ V - c @ dd         # 1 + W T_current V
                if self.metropolis(d, li, i, np.linalg.det(S)):
                    X = TV @ np.linalg.inv(S)
                    Xs = np.concatenate([Xs, X], axis=1)
                    Ys = np.concatenate([Ys, Y], axis=0)
                    self._accept_rows(li, i, delta)
            self.T = T0 - Xs @ Ys

    # ---------------------------------------------------- block force bias
    def _pairs(self, sites):
        return list(sites) + [self.N + i for i in sites]

    def block_force_bias(self, li, sites):
        """s_i = gamma <O_i>, O_i = c+_{i up} c_{i dn} - c+_{i dn} c_{i up}, with
        the block's own fields removed: UU_R = e^{-H_I^(b)(x)} U_R (row pairs of
        the block rotated by A(-x_i)) and (U_L UU_R)^{-1} from T by the matrix
        Sherman-Morrison form (Eq. (35)); <c+_p c_q> = [UU_R (U_L UU_R)^{-1} U_L]_{qp}."""
        N, nb = self.N, len(sites)
        rows = self._pairs(sites)
        Db = np.zeros((2 * nb, 2 * nb))
        for j in range(nb):
            x = float(self.fields[li, sites[j]])
            Db[np.ix_([j, nb + j], [j, nb + j])] = rotation(self.gamma, -x) - np.eye(2)
        V = self.UL[:, rows] @ Db
        Um = self.UR[rows, :]
        T = self.T
        TV, UT = T @ V, Um @ T
        Tb = T - TV @ np.linalg.inv(np.eye(2 * nb) + UT @ V) @ UT
        URb = (np.eye(2 * nb) + Db) @ Um
        svec = np.empty(nb)
        for j, i in enumerate(sites):
            c_up_dn = URb[nb + j] @ Tb @ self.UL[:, i]          # <c+_{i up} c_{i dn}>
            c_dn_up = URb[j] @ Tb @ self.UL[:, N + i]           # <c+_{i dn} c_{i up}>
            o = self.gamma * (c_up_dn - c_dn_up)
            if abs(np.imag(o)) > 1e-10 * (1.0 + abs(o)):
                raise FloatingPointError("force bias exponent is not real")
            svec[j] = float(np.real(o))
        return svec

    @staticmethod
    def heat_bath_prob(svec):
        with np.errstate(over="ignore"):
            return np.array([1.0 / (1.0 + np.exp(-2.0 * float(s))) for s in svec])

    def block_ratio(self, li, sites, xnew, svec):
        """R = det[1 + (U' T) V'] over the row pairs of the flip set F (the
        rank-2|F| form of Eq. (A7)) and the prior ratio prod_F e^{s_i (x_i - x'_i)}."""
        xold = self.fields[li, sites].astype(np.int64)
        F = [j for j in range(len(sites)) if xnew[j] != xold[j]]
        idx = [sites[j] for j in F]
        nf = len(F)
        dF = np.zeros((2 * nf, 2 * nf))
        for q, j in enumerate(F):
            dF[np.ix_([q, nf + q], [q, nf + q])] = self.flip_block(li, sites[j])
        rows = self._pairs(idx)
        Vp = self.UL[:, rows] @ dF
        Up = self.UR[rows, :]
        Wp = np.eye(2 * nf) + (Up @ self.T) @ Vp
        with np.errstate(over="ignore"):
            prior = float(np.exp(float(np.sum(svec[F] * (xold[F] - xnew[F])))))
        return F, idx, np.linalg.det(Wp), Vp, Up, Wp, dF, prior

    def block_slice(self, l, d):
        """Block force-bias update of slice l (Sec. III B) for the spin-coupled
        model: blocks of b consecutive sites, each with its own force bias."""
        li = l - 1
        N, b = self.N, min(self.b, self.N)
        for b0 in range(0, N, b):
            sites = list(range(b0, min(b0 + b, N)))
            svec = self.block_force_bias(li, sites)
            p_up = self.heat_bath_prob(svec)
            xnew = np.empty(len(sites), np.int64)
            for j, i in enumerate(sites):
                u = philox.uniform(self.key, self.sweep_index, d * self.M + li, i,
                                   philox.PURPOSE_HB)
                xnew[j] = 1 if u < p_up[j] else -1
                self.hb_log.append((self.sweep_index, d, li, i, int(xnew[j]), p_up[j] - u))
            F, idx, R, Vp, Up, Wp, dF, prior = self.block_ratio(li, sites, xnew, svec)
            if not F:
                self.metropolis(d, li, b0, 1.0)          # empty flip set: accepted no-op
                continue
            if self.metropolis(d, li, b0, R, prior):
                T = self.T
                self.T = T - (T @ Vp) @ np.linalg.inv(Wp) @ (Up @ T)   # Eq. (36)
                rows = self._pairs(idx)
                self.UR[rows, :] = (np.eye(2 * len(F)) + dF) @ self.UR[rows, :]
                for j in F:
                    self.fields[li, sites[j]] = xnew[j]
                self.n_flips += len(F)

    # ------------------------------------------------------------ observables
    def green(self):
        """G = 1 - U_R T U_L (2N x 2N), Appendix A."""
        return np.eye(2 * self.N) - self.UR @ self.T @ self.UL


# ---------------------------------------------------------------- brute force
def weight(P, K, gamma, X):
    """W(X) = det(P^+ B_M ... B_1 P) from the definition (Appendix A)."""
    R = P.copy()
    for li in range(X.shape[0]):
        R = b_matrix(gamma, K, X[li]) @ R
    return np.linalg.det(P.conj().T @ R)


def green_at(P, K, gamma, X, l):
    """G at position l from its definition: R = B_l..B_1 P, L = P^+ B_M..B_{l+1},
    G = 1 - R (L R)^{-1} L (Appendix A)."""
    R = P.copy()
    for li in range(l):
        R = b_matrix(gamma, K, X[li]) @ R
    Lm = P.conj().T.copy()
    for li in range(X.shape[0] - 1, l - 1, -1):
        Lm = Lm @ b_matrix(gamma, K, X[li])
    return np.eye(P.shape[0]) - R @ np.linalg.inv(Lm @ R) @ Lm
