"""Time integration loops (oracle; FP64, assembled sparse matrices).

Section "Time Integration": Newmark's formulas (Eqs. Newmark1, Newmark2),
the central difference method as the two-step sum (Eq. CDMstep) with the
acceleration from Eq. CDMacc, the trapezoidal Newmark predictor / solve /
corrector with beta = 1/4, gamma = 1/2 (trapezoidal flowchart figure), and
the Newmark IMEX scheme (Newmark IMEX flowchart figure): per step a diagonal
CDM step on the d dofs, then the trapezoidal predictor on the c dofs with
u^d_pred = u^d_{n+1}, the solve with S = M^cc + beta dt^2 K^cc (factorised
once, here with SciPy's sparse LU as in the paper's own runs), and the
corrector.

With beta = 0 on the c block the same loop is the explicit central
difference method on all dofs, with the block mass (lumped on d, consistent
on c): the CDM comparator of Section "Time Integration", stable only below
the global critical step 2 / sqrt(lambda_max(K, M)).

Readings (the flowchart leaves them open):
  * the right-hand side of the initial solve and of the per-step solve is
    the c part f_x^c, and the predictor uses u^c_n;
  * the CDM start value is u^d_{-1} = u^d_0 - dt v^d_0 + dt^2/2 a^d_0, which
    makes the two-step CDM identical to Newmark with beta = 0, gamma = 1/2;
  * a fixed number of steps is taken (instead of testing t_{n+1} <= T); the
    explicit step uses f_t(t_n) and the implicit one f_t(t_{n+1}).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

BETA, GAMMA = 0.25, 0.5


@dataclass
class ImexState:
    u: np.ndarray          # u_n on the full vector (inactive entries 0)
    ud_prev: np.ndarray    # u^d_{n-1} on the d dofs
    vc: np.ndarray         # velocity of the c dofs
    ac: np.ndarray         # acceleration of the c dofs
    n: int = 0


class NewmarkImex:
    """Newmark IMEX on M u'' + K u = f_t(t) f_x with d dofs Id, c dofs Ic."""

    def __init__(self, M, K, fx, Id, Ic, dt, beta=None):
        self.beta = BETA if beta is None else float(beta)  # beta of the c block
        self.M = sp.csr_matrix(M)
        self.K = sp.csr_matrix(K)
        self.fx = np.asarray(fx, dtype=np.float64)
        self.Id = np.asarray(Id, dtype=np.int64)
        self.Ic = np.asarray(Ic, dtype=np.int64)
        self.dt = float(dt)
        self.Mdd = self.M[self.Id][:, self.Id].diagonal().copy()
        self.Kd = self.K[self.Id].tocsr()
        self.Kc = self.K[self.Ic].tocsr()
        self.Mcc = self.M[self.Ic][:, self.Ic].tocsc()
        self.Kcc = self.K[self.Ic][:, self.Ic].tocsc()
        self.S = (self.Mcc + self.beta * self.dt ** 2 * self.Kcc).tocsc()
        self._lu_S = spla.splu(self.S) if len(self.Ic) else None
        self._lu_M = spla.splu(self.Mcc) if len(self.Ic) else None

    def solve_S(self, r):
        return self._lu_S.solve(r) if len(self.Ic) else np.zeros(0)

    def initial_state(self, u0, v0, ft0) -> ImexState:
        """Initial c acceleration from M^cc a = f_t(0) f_x^c - K^c u_0 and the
        CDM start value for the d dofs."""
        u0 = np.asarray(u0, dtype=np.float64).copy()
        v0 = np.asarray(v0, dtype=np.float64)
        Id, Ic, dt = self.Id, self.Ic, self.dt
        ac = self._lu_M.solve(ft0 * self.fx[Ic] - self.Kc @ u0) if len(Ic) else np.zeros(0)
        ad = (ft0 * self.fx[Id] - self.Kd @ u0) / self.Mdd
        ud_prev = u0[Id] - dt * v0[Id] + 0.5 * dt * dt * ad
        return ImexState(u=u0, ud_prev=ud_prev, vc=v0[Ic].copy(), ac=ac, n=0)

    def step(self, st: ImexState, ft_n, ft_np1) -> ImexState:
        Id, Ic, dt = self.Id, self.Ic, self.dt
        u = st.u
        # diagonal CDM step (Eq. CDMacc restricted to d, Eq. CDMstep)
        ad = (ft_n * self.fx[Id] - self.Kd @ u) / self.Mdd
        ud_new = 2.0 * u[Id] - st.ud_prev + dt * dt * ad
        # trapezoidal prediction of the c dofs
        uc_pred = u[Ic] + dt * st.vc + (0.5 - self.beta) * dt * dt * st.ac
        vc_pred = st.vc + (1.0 - GAMMA) * dt * st.ac
        u_pred = u.copy()
        u_pred[Id] = ud_new
        u_pred[Ic] = uc_pred
        # acceleration of the c dofs
        ac = self.solve_S(ft_np1 * self.fx[Ic] - self.Kc @ u_pred)
        # correction
        uc = uc_pred + self.beta * dt * dt * ac
        vc = vc_pred + GAMMA * dt * ac
        u_new = u_pred
        u_new[Ic] = uc
        return ImexState(u=u_new, ud_prev=u[Id].copy(), vc=vc, ac=ac, n=st.n + 1)

    def run(self, st: ImexState, ft, n_steps, every: Optional[int] = None,
            callback=None) -> ImexState:
        """Advance n_steps; ft[k] = f_t(t_{st.n + k}) (n_steps + 1 values)."""
        for k in range(n_steps):
            st = self.step(st, ft[k], ft[k + 1])
            if callback is not None and every and (k + 1) % every == 0:
                callback(st)
        return st

    # ---- discrete energy ---------------------------------------------------
    def energy(self, st_prev: ImexState, st: ImexState, st_next: ImexState):
        """Conserved discrete energy of the unforced IMEX scheme at step n.

        E_n = 1/2 v^T M v + 1/2 u^T K u - dt^2/8 (a^d)^T M^dd a^d, with the
        central-difference velocity v^d_n = (u^d_{n+1} - u^d_{n-1}) / (2 dt),
        the Newmark velocity v^c_n, and a^d_n = -(K^d u_n) / M^dd.  It follows
        from Newmark's formulas with gamma = 1/2 and a per-dof beta (0 on d,
        1/4 on c), which is valid because M is block diagonal over d and c.
        """
        Id, Ic, dt = self.Id, self.Ic, self.dt
        u = st.u
        vd = (st_next.u[Id] - st_prev.u[Id]) / (2.0 * dt)
        ad = -(self.Kd @ u) / self.Mdd
        e = 0.5 * float(vd @ (self.Mdd * vd))
        e += 0.5 * float(st.vc @ (self.Mcc @ st.vc))
        e += 0.5 * float(u @ (self.K @ u))
        e -= dt * dt / 8.0 * float(ad @ (self.Mdd * ad))
        return e


def imex_mass(M, Id, Ic):
    """The block mass of the IMEX splitting on the given dofs: the lumped
    diagonal on d, the consistent block on c, no d-c coupling."""
    M = sp.csr_matrix(M)
    n = M.shape[0]
    D = sp.csr_matrix((M.diagonal()[Id], (Id, Id)), shape=(n, n))
    C = sp.csr_matrix(M[Ic][:, Ic])
    P = sp.csr_matrix((np.ones(len(Ic)), (Ic, np.arange(len(Ic)))), shape=(n, len(Ic)))
    return (D + P @ C @ P.T).tocsr()


def global_critical_step(M, K, active):
    """2 / sqrt(lambda_max) of K x = lambda M x on the active dofs (Lanczos,
    SciPy's eigsh), the stability limit of the central difference method."""
    act = np.asarray(active)
    Ma = sp.csc_matrix(sp.csr_matrix(M)[act][:, act])
    Ka = sp.csc_matrix(sp.csr_matrix(K)[act][:, act])
    lam = spla.eigsh(Ka, k=1, M=Ma, which="LA", return_eigenvectors=False, tol=1e-10)[0]
    return 2.0 / np.sqrt(lam)


def cdm_run(M, K, fx, ft, u0, v0, dt, n_steps):
    """Explicit CDM on all dofs (consistent M factorised once)."""
    lu = spla.splu(sp.csc_matrix(M))
    a0 = lu.solve(ft[0] * fx - K @ u0)
    u_prev = u0 - dt * v0 + 0.5 * dt * dt * a0
    u = u0.copy()
    for n in range(n_steps):
        a = lu.solve(ft[n] * fx - K @ u)
        u, u_prev = 2.0 * u - u_prev + dt * dt * a, u
    return u


def trapezoidal_run(M, K, fx, ft, u0, v0, dt, n_steps):
    """Implicit trapezoidal Newmark on all dofs (trapezoidal flowchart)."""
    M = sp.csc_matrix(M)
    K = sp.csc_matrix(K)
    a = spla.splu(M).solve(ft[0] * fx - K @ u0)
    S = spla.splu((M + BETA * dt * dt * K).tocsc())
    u, v = u0.copy(), v0.copy()
    for n in range(n_steps):
        up = u + dt * v + (0.5 - BETA) * dt * dt * a
        vp = v + (1.0 - GAMMA) * dt * a
        a = S.solve(ft[n + 1] * fx - K @ up)
        u = up + BETA * dt * dt * a
        v = vp + GAMMA * dt * a
    return u
