"""Oracle walker for the ground-state AFQMC (PQMC) field-update sweep.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain NumPy, float64
(complex128 when U < 0), written step by step from Du & He, arXiv:2506.09611:

  * configuration weight W(X) and propagators B_l = e^{H_I(x_l)} e^{-dtau H0}
    -- Sec. II B, Eqs. (8)-(9); discrete spin-channel HS field, Eqs. (13)-(14);
  * the tracked state (U_L, U_R, T = (U_L U_R)^{-1}), G = 1 - U_R T U_L and
    the QR stabilisation every k_tau slices -- Sec. II B, Eq. (15);
  * the general ratio and T upgrade -- Sec. II C, Eqs. (16)-(19);
  * local update -- Sec. II D, Eqs. (20)-(21);
  * delayed update (first strategy: n_d proposals per flush) -- Sec. III A,
    Eqs. (27)-(30);
  * block force-bias update -- Sec. III B, Eqs. (31)-(36).

Readings where the paper is silent (each listed in the design notes):
  * U > 0 uses the real continuation of the coupling, alpha = arccosh(e^{dtau U/2}),
    two real spin sectors; U < 0 uses the paper's alpha = i*arccos(e^{dtau U/2}).
  * A sweep is a forward pass l = 1..M followed by a backward pass l = M..1.
  * Accept iff u < |A| with u uniform in [0,1) from Philox (oracle.philox).
  * Block force bias: an empty flip set is an accepted no-op; the heat-bath
    proposal is p(x'=+1) = 1 / (1 + exp(-2 s)), s = alpha (nbar_up - nbar_dn).
"""
from __future__ import annotations

import math
import numpy as np

from . import philox

SPIN_SIGN = (+1.0, -1.0)       # f_up = +1, f_dn = -1  (Sec. II B, after Eq. (14))
SCHEMES = ("local", "delayed", "block")


def coupling(U: float, dtau: float):
    """HS coupling alpha with H_I^sigma(x) = alpha f_sigma diag(x).

    U < 0: alpha = i*gamma, gamma = arccos(e^{dtau U/2})  (Eq. (13)).
    U > 0: alpha = arccosh(e^{dtau U/2}), the real continuation (Hirsch).
    """
    if U > 0:
        return math.acosh(math.exp(dtau * U / 2.0))
    if U < 0:
        return 1j * math.acos(math.exp(dtau * U / 2.0))
    return 0.0


def kinetic_propagators(H0: np.ndarray, dtau: float):
    """K = e^{-dtau H0} and K^{-1} = e^{+dtau H0} from the eigendecomposition."""
    e, V = np.linalg.eigh(H0)
    K = (V * np.exp(-dtau * e)) @ V.T
    Kinv = (V * np.exp(dtau * e)) @ V.T
    return K, Kinv


def orthonormalize_columns(A):
    return np.linalg.qr(A)[0]


def orthonormalize_rows(A):
    return np.linalg.qr(A.conj().T)[0].conj().T


class Walker:
    """One Markov chain of the PQMC field configuration.

    fields[l-1, i] holds x_{l,i} = +-1 for slice l = 1..M and site i.
    For each spin s: UR[s] (N x N_s), UL[s] (N_s x N), T[s] (N_s x N_s).
    """

    def __init__(self, prob, scheme="local", k=1, b=1, fields=None):
        if scheme not in SCHEMES:
            raise ValueError(scheme)
        self.p = prob
        self.N = prob.hopping.shape[0]
        self.M = prob.n_slices
        self.kt = prob.stab_every
        if self.M % self.kt:
            raise ValueError("stab_every must divide n_slices")
        self.scheme, self.k, self.b = scheme, max(1, int(k)), max(1, int(b))
        self.alpha = coupling(prob.U, prob.dtau)
        self.dtype = np.complex128 if isinstance(self.alpha, complex) else np.float64
        self.K, self.Kinv = kinetic_propagators(prob.hopping, prob.dtau)
        self.P = [np.asarray(prob.trial_up, self.dtype), np.asarray(prob.trial_dn, self.dtype)]
        self.key = (prob.seed, prob.walker_id)
        self.sweep_index = 0
        if fields is None:
            fields = self.initial_fields()
        self.fields = np.array(fields, dtype=np.int8).reshape(self.M, self.N)
        self.log = []          # decisions: (sweep, dir, slice, site, accept, margin, sign)
        self.hb_log = []       # block force bias: (sweep, dir, slice, site, x_new, margin)
        self.n_proposed = 0
        self.n_accepted = 0
        self.n_flips = 0
        self.trace = None      # when a list: (dir, slice, site, R, prior, fields before)
        self.replay = None     # when set: 2M x N forced outcomes (see replay_sweep)
        self.build_initial_state()

    # ------------------------------------------------------------------ setup
    def initial_fields(self):
        """x_{l,i} = +1 iff u(INIT; 0, l-1, i) < 1/2."""
        X = np.empty((self.M, self.N), np.int8)
        for li in range(self.M):
            for i in range(self.N):
                u = philox.uniform(self.key, 0, li, i, philox.PURPOSE_INIT)
                X[li, i] = 1 if u < 0.5 else -1
        return X

    def expv(self, li, s, sign=+1.0):
        """Diagonal of e^{sign * H_I^s(x_l)} = exp(sign * alpha f_s x_l)."""
        return np.exp(sign * self.alpha * SPIN_SIGN[s] * self.fields[li].astype(np.float64))

    def build_initial_state(self):
        """L-stack at every k_tau, then position 0: U_R = P, U_L = L_0 (Sec. II B)."""
        M, kt = self.M, self.kt
        ns = M // kt
        self.Lstack = [[None] * (ns + 1) for _ in range(2)]
        self.Rstack = [[None] * (ns + 1) for _ in range(2)]
        for s in range(2):
            UL = self.P[s].conj().T.copy()
            self.Lstack[s][ns] = UL.copy()
            for l in range(M, 0, -1):
                UL = (UL * self.expv(l - 1, s)[None, :]) @ self.K        # U_L B_l
                if (l - 1) % kt == 0:
                    UL = orthonormalize_rows(UL)
                    self.Lstack[s][(l - 1) // kt] = UL.copy()
            self.Rstack[s][0] = self.P[s].copy()
        self.UR = [self.P[s].copy() for s in range(2)]
        self.UL = [self.Lstack[s][0].copy() for s in range(2)]
        self.T = [np.linalg.inv(self.UL[s] @ self.UR[s]) for s in range(2)]

    # ------------------------------------------------------------ propagation
    def prop_forward(self, l):
        """Position l-1 -> l: U_R <- B_l U_R, U_L <- U_L B_l^{-1}; T unchanged."""
        li = l - 1
        for s in range(2):
            self.UR[s] = self.expv(li, s)[:, None] * (self.K @ self.UR[s])
            self.UL[s] = (self.UL[s] @ self.Kinv) * self.expv(li, s, -1.0)[None, :]

    def prop_backward(self, l):
        """Position l -> l-1: U_L <- U_L B_l, U_R <- B_l^{-1} U_R; T unchanged."""
        li = l - 1
        for s in range(2):
            self.UL[s] = (self.UL[s] * self.expv(li, s)[None, :]) @ self.K
            self.UR[s] = self.Kinv @ (self.expv(li, s, -1.0)[:, None] * self.UR[s])

    def refresh_T(self):
        for s in range(2):
            self.T[s] = np.linalg.inv(self.UL[s] @ self.UR[s])

    # ----------------------------------------------------------------- sweeps
    def sweep(self):
        """Forward l = 1..M then backward l = M..1, stabilising every k_tau."""
        M, kt = self.M, self.kt
        for l in range(1, M + 1):
            self.prop_forward(l)
            self.update_slice(l, 0)
            if l % kt == 0:
                for s in range(2):
                    self.UR[s] = orthonormalize_columns(self.UR[s])
                    self.Rstack[s][l // kt] = self.UR[s].copy()
                    self.UL[s] = self.Lstack[s][l // kt].copy()
                self.refresh_T()
        for l in range(M, 0, -1):
            self.update_slice(l, 1)
            self.prop_backward(l)
            if (l - 1) % kt == 0:
                for s in range(2):
                    self.UL[s] = orthonormalize_rows(self.UL[s])
                    self.Lstack[s][(l - 1) // kt] = self.UL[s].copy()
                    self.UR[s] = self.Rstack[s][(l - 1) // kt].copy()
                self.refresh_T()
        self.sweep_index += 1

    def forward_window(self, n_slices):
        """Forward pass over slices 1..n_slices only (for windowed comparisons)."""
        for l in range(1, n_slices + 1):
            self.prop_forward(l)
            self.update_slice(l, 0)
            if l % self.kt == 0:
                for s in range(2):
                    self.UR[s] = orthonormalize_columns(self.UR[s])
                    self.Rstack[s][l // self.kt] = self.UR[s].copy()
                    self.UL[s] = self.Lstack[s][l // self.kt].copy()
                self.refresh_T()

    def update_slice(self, l, d):
        if self.scheme == "local":
            self.local_slice(l, d)
        elif self.scheme == "delayed":
            self.delayed_slice(l, d)
        else:
            self.block_slice(l, d)

    def replay_sweep(self, flips):
        """One sweep with every outcome forced instead of drawn (the invariant
        that all three schemes apply Eq. (19) to the same accepted flips).
        flips[d*M + l-1, i] != 0: site i flips on that visit of slice l.
        Local / delayed: the site's Metropolis test is accepted iff listed.
        Block: the heat-bath proposal is the listed flip set and the block's
        Metropolis test is accepted.  A forced outcome is the uniform -0
        (taken for any nonzero finite |A|, and the logged margin is |A|) or
        +inf (not taken) in place of the draw."""
        self.replay = np.asarray(flips, dtype=np.int8).reshape(2 * self.M, self.N)
        try:
            self.sweep()
        finally:
            self.replay = None

    # ---------------------------------------------------------- decisions
    def mh_uniform(self, d, li, site):
        if self.replay is not None:
            take = self.scheme == "block" or self.replay[d * self.M + li, site] != 0
            return -0.0 if take else math.inf
        return philox.uniform(self.key, self.sweep_index, d * self.M + li, site, philox.PURPOSE_MH)

    def hb_uniform(self, d, li, site):
        if self.replay is not None:
            x = int(self.fields[li, site])
            target = -x if self.replay[d * self.M + li, site] != 0 else x
            return -0.0 if target > 0 else math.inf
        return philox.uniform(self.key, self.sweep_index, d * self.M + li, site, philox.PURPOSE_HB)

    def flip_delta(self, li, i, s):
        """Delta^s_ii = e^{alpha f_s (x' - x)} - 1 with x' = -x  (Sec. II D)."""
        x = float(self.fields[li, i])
        return np.exp(-2.0 * self.alpha * SPIN_SIGN[s] * x) - 1.0

    def metropolis(self, d, li, site, R, extra=1.0):
        """Eq. (16) with a symmetric proposal: accept iff u < |R * extra|."""
        with np.errstate(over="ignore", invalid="ignore"):
            A = R * extra
            absA = abs(A)
        if np.isnan(absA):
            raise FloatingPointError("acceptance ratio is NaN")
        if self.trace is not None:
            self.trace.append((d, li, site, R, extra, self.fields.copy()))
        u = self.mh_uniform(d, li, site)
        acc = u < absA
        sgn = 1.0 if np.real(A) >= 0 else -1.0
        self.log.append((self.sweep_index, d, li, site, bool(acc), absA - u, sgn))
        self.n_proposed += 1
        self.n_accepted += int(acc)
        return acc

    # ----------------------------------------------------------- local update
    def local_slice(self, l, d):
        """Local update of slice l: Eqs. (20)-(21), sites i = 1..N in order."""
        li = l - 1
        for i in range(self.N):
            ys, vs, rs, Ds = [], [], [], []
            for s in range(2):
                D = self.flip_delta(li, i, s)
                u = self.UR[s][i, :]
                v = D * self.UL[s][:, i]
                y = u @ self.T[s]                      # y^T = u_i^T T
                r = 1.0 + y @ v                        # Eq. (20)
                ys.append(y); vs.append(v); rs.append(r); Ds.append(D)
            if self.metropolis(d, li, i, rs[0] * rs[1]):
                for s in range(2):
                    x = (self.T[s] @ vs[s]) / rs[s]
                    self.T[s] = self.T[s] - np.outer(x, ys[s])   # Eq. (21)
                    self.UR[s][i, :] *= (1.0 + Ds[s])           # Eq. (19), row i
                self.fields[li, i] = -self.fields[li, i]
                self.n_flips += 1

    # --------------------------------------------------------- delayed update
    def delayed_slice(self, l, d):
        """Delayed update, first strategy (n_d = proposals): Eqs. (27)-(30)."""
        li = l - 1
        N, k = self.N, min(self.k, self.N)
        for g0 in range(0, N, k):
            sites = list(range(g0, min(g0 + k, N)))
            T0, TV, UT, Vm, Xs, Ys = [], [], [], [], [], []
            for s in range(2):
                D = np.array([self.flip_delta(li, i, s) for i in sites])
                V = self.UL[s][:, sites] * D[None, :]       # columns v_i
                Um = self.UR[s][sites, :]                   # rows u_i^T
                T0.append(self.T[s])
                TV.append(T0[s] @ V)                        # T_[0] V
                UT.append(Um @ T0[s])                       # U T_[0]
                Vm.append(V)
                Xs.append(np.zeros((self.T[s].shape[0], 0), self.dtype))
                Ys.append(np.zeros((0, self.T[s].shape[0]), self.dtype))
            for j, i in enumerate(sites):
                rs, cs, ds = [], [], []
                for s in range(2):
                    u = self.UR[s][i, :]
                    v = Vm[s][:, j]
                    c = u @ Xs[s]                           # c_m = u^T x_m
                    dd = Ys[s] @ v                          # d_m = y_m^T v
                    r = 1.0 + UT[s][j] @ v - c @ dd         # Eq. (28)
                    rs.append(r); cs.append(c); ds.append(dd)
                if self.metropolis(d, li, i, rs[0] * rs[1]):
                    for s in range(2):
                        xk = (TV[s][:, j] - Xs[s] @ ds[s]) / rs[s]      # Eq. (29)
                        yk = UT[s][j] - cs[s] @ Ys[s]
                        Xs[s] = np.concatenate([Xs[s], xk[:, None]], axis=1)
                        Ys[s] = np.concatenate([Ys[s], yk[None, :]], axis=0)
                        self.UR[s][i, :] *= (1.0 + self.flip_delta(li, i, s))
                    self.fields[li, i] = -self.fields[li, i]
                    self.n_flips += 1
            for s in range(2):
                self.T[s] = T0[s] - Xs[s] @ Ys[s]                # Eq. (30)

    # ---------------------------------------------------- block force bias
    def block_force_bias(self, li, sites):
        """Force bias of one block with the block's own fields removed.

        nbar^s_i = [UU_R (U_L UU_R)^{-1} U_L]_ii with UU_R = (1 + Delta_b) U_R,
        (Delta_b)_ii = e^{-alpha f_s x_i} - 1 on the block (Sec. III B), and
        (U_L UU_R)^{-1} from T by the matrix Sherman-Morrison form, Eq. (35).
        Returns s_i = alpha (nbar_up_i - nbar_dn_i), real by construction.
        """
        a, nb = self.alpha, len(sites)
        nbar = np.zeros((2, nb), self.dtype)
        x = self.fields[li, sites].astype(np.float64)
        for s in range(2):
            Db = np.exp(-a * SPIN_SIGN[s] * x) - 1.0
            V = self.UL[s][:, sites] * Db[None, :]
            Um = self.UR[s][sites, :]
            T = self.T[s]
            TV, UT = T @ V, Um @ T
            Tb = T - TV @ np.linalg.inv(np.eye(nb) + UT @ V) @ UT      # Eq. (35)
            URb = Um * (1.0 + Db)[:, None]
            for j, i in enumerate(sites):
                nbar[s, j] = URb[j] @ Tb @ self.UL[s][:, i]             # Eq. (25)
        svec = a * (nbar[0] - nbar[1])
        if np.iscomplexobj(svec):
            if np.max(np.abs(svec.imag)) > 1e-10 * (1.0 + np.max(np.abs(svec))):
                raise FloatingPointError("force bias exponent is not real")
            svec = svec.real
        return np.asarray(svec, np.float64)

    @staticmethod
    def heat_bath_prob(svec):
        """P(x' = +1) = e^{s} / (e^{s} + e^{-s}) per site (Sec. II D, second step).

        For U > 0 the mixed-estimate force bias is unbounded when the overlap
        with the block's fields removed nearly vanishes, so e^{-2s} may
        overflow: it is evaluated in IEEE arithmetic (inf gives P = 0)."""
        with np.errstate(over="ignore"):
            return np.array([1.0 / (1.0 + np.exp(-2.0 * float(s))) for s in svec])

    def block_ratio(self, li, sites, xnew, svec):
        """det ratios r_s = det[1 + (U' T) V'] over the flip set (Sec. III B) and
        the prior ratio P(X'->X)/P(X->X') = prod_F e^{s_i (x_i - x'_i)}."""
        a = self.alpha
        xold = self.fields[li, sites].astype(np.int64)
        F = [j for j in range(len(sites)) if xnew[j] != xold[j]]
        idx = [sites[j] for j in F]
        out = []
        for s in range(2):
            Dp = np.exp(a * SPIN_SIGN[s] * (xnew[F] - xold[F]).astype(np.float64)) - 1.0
            Vp = self.UL[s][:, idx] * Dp[None, :]
            Up = self.UR[s][idx, :]
            Wp = np.eye(len(F)) + (Up @ self.T[s]) @ Vp
            out.append((np.linalg.det(Wp), Vp, Up, Wp, Dp))
        with np.errstate(over="ignore"):
            prior = float(np.exp(float(np.sum(svec[F] * (xold[F] - xnew[F])))))
        return F, idx, out, prior

    def block_slice(self, l, d):
        """Block force-bias update of slice l: Sec. III B, Eqs. (31)-(36)."""
        li = l - 1
        N, b = self.N, min(self.b, self.N)
        for b0 in range(0, N, b):
            sites = list(range(b0, min(b0 + b, N)))
            svec = self.block_force_bias(li, sites)
            p_up = self.heat_bath_prob(svec)
            xnew = np.empty(len(sites), np.int64)
            for j, i in enumerate(sites):
                u = self.hb_uniform(d, li, i)
                xnew[j] = 1 if u < p_up[j] else -1
                self.hb_log.append((self.sweep_index, d, li, i, int(xnew[j]), p_up[j] - u))
            F, idx, per_spin, prior = self.block_ratio(li, sites, xnew, svec)
            if not F:
                self.metropolis(d, li, b0, 1.0)          # empty flip set: accepted no-op
                continue
            R = per_spin[0][0] * per_spin[1][0]
            if self.metropolis(d, li, b0, R, prior):
                for s in range(2):
                    _, Vp, Up, Wp, Dp = per_spin[s]
                    T = self.T[s]
                    self.T[s] = T - (T @ Vp) @ np.linalg.inv(Wp) @ (Up @ T)   # Eq. (36)
                    self.UR[s][idx, :] *= (1.0 + Dp)[:, None]
                for j in F:
                    self.fields[li, sites[j]] = xnew[j]
                self.n_flips += len(F)

    # ------------------------------------------------------------ observables
    def green(self, s):
        """G^s = 1 - U_R T U_L at the current position (Eq. (15))."""
        return np.eye(self.N) - self.UR[s] @ self.T[s] @ self.UL[s]

    def low_margin(self, tol=1e-12):
        return sum(1 for e in self.log if abs(e[5]) < tol) + \
            sum(1 for e in self.hb_log if abs(e[5]) < tol)
