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

    def __init__(self, M, K, fx, Id, Ic, dt, beta=None, solver="splu", sum_perm=None, k_apply=None):
        """solver: how S (and M^cc) are factorised: "splu" (SciPy's sparse LU,
        as in the paper's own runs) or "dense_cholesky" (dense Cholesky of
        each connected component).  sum_perm: an optional permutation of the
        dofs; the products with K then sum each row in that permuted column
        order.  k_apply: a function u -> K u used for the products with K in
        the steps instead of the assembled matrix (e.g. fcm.sumfact_stiffness,
        the cell-by-cell form).  These choices change rounding only; the
        spread they produce along a trajectory is what two correct FP64
        implementations of the same scheme can differ by."""
        self.k_apply = k_apply
        self.beta = BETA if beta is None else float(beta)  # beta of the c block
        self.M = sp.csr_matrix(M)
        self.K = sp.csr_matrix(K)
        if sum_perm is not None:
            self.K = _column_order(self.K, np.asarray(sum_perm))
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
        if solver == "splu":
            self._lu_S = spla.splu(self.S) if len(self.Ic) else None
            self._lu_M = spla.splu(self.Mcc) if len(self.Ic) else None
        elif solver == "dense_cholesky":
            self._lu_S = _BlockCholesky(self.S) if len(self.Ic) else None
            self._lu_M = _BlockCholesky(self.Mcc) if len(self.Ic) else None
        else:
            raise ValueError(solver)

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
        ku = self.Kd @ u if self.k_apply is None else self.k_apply(u)[Id]
        ad = (ft_n * self.fx[Id] - ku) / self.Mdd
        ud_new = 2.0 * u[Id] - st.ud_prev + dt * dt * ad
        # trapezoidal prediction of the c dofs
        uc_pred = u[Ic] + dt * st.vc + (0.5 - self.beta) * dt * dt * st.ac
        vc_pred = st.vc + (1.0 - GAMMA) * dt * st.ac
        u_pred = u.copy()
        u_pred[Id] = ud_new
        u_pred[Ic] = uc_pred
        # acceleration of the c dofs
        kp = self.Kc @ u_pred if self.k_apply is None else self.k_apply(u_pred)[Ic]
        ac = self.solve_S(ft_np1 * self.fx[Ic] - kp)
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


def _column_order(A, perm):
    """A copy of the CSR matrix A whose rows store their entries in the
    column order of perm (entry j before entry k when perm places j first),
    so that A @ x sums every row in that order."""
    A = sp.csr_matrix(A)
    rank = np.empty(len(perm), dtype=np.int64)
    rank[perm] = np.arange(len(perm))
    B = sp.csr_matrix(A, copy=True)
    for i in range(B.shape[0]):
        lo, hi = B.indptr[i], B.indptr[i + 1]
        o = np.argsort(rank[B.indices[lo:hi]], kind="stable")
        B.indices[lo:hi] = B.indices[lo:hi][o]
        B.data[lo:hi] = B.data[lo:hi][o]
    B.has_sorted_indices = False
    return B


class _BlockCholesky:
    """Dense Cholesky factors of the diagonal blocks of a symmetric positive
    definite matrix that is block diagonal over its connected components."""

    def __init__(self, A):
        import scipy.linalg as sla
        from scipy.sparse.csgraph import connected_components
        A = sp.csr_matrix(A)
        ncomp, lab = connected_components(A, directed=False)
        self.blocks = []
        for k in range(ncomp):
            idx = np.flatnonzero(lab == k)
            self.blocks.append((idx, sla.cho_factor(A[idx][:, idx].toarray(), lower=True)))
        self.n = A.shape[0]

    def solve(self, r):
        import scipy.linalg as sla
        x = np.zeros(self.n)
        for idx, f in self.blocks:
            x[idx] = sla.cho_solve(f, r[idx])
        return x


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


def lts_leapfrog_run(M, K, fx, ft, fine, u0, v0, dt, m, n_steps, callback=None):
    """Leap-frog with local time stepping on the fine dofs (oracle).

    The paper names substepping of the cut cells with dt_fine = dt_coarse / m
    (Section "Time Integration", the leap-frog paragraph) and defers the
    formulation to references that are not available here.  This is the
    energy-conserving local time-stepping leap-frog of Diaz and Grote
    (SIAM J. Sci. Comput. 31, 2009), written for M u'' + K u = f_t f_x with
    the block mass M (lumped on d, consistent or HRZ-lumped on c) and the
    fine dofs `fine` (the c dofs: nodes of cut cells).  With A = M^-1 K and
    P the projection onto the fine dofs, one coarse step from (u_{n-1}, u_n):

        w   = A (I - P) u_n - M^-1 f_t(t_n) f_x        (frozen over the step)
        q_0 = u_n,  q_1 = q_0 - (tau^2 / 2) (w + A P q_0),  tau = dt / m
        q_{k+1} = 2 q_k - q_{k-1} - tau^2 (w + A P q_k),  k = 1 .. m-1
        u_{n+1} = 2 q_m - u_{n-1}

    With m = 1 this is the central difference method on all dofs with the
    block mass (Newmark beta = 0, gamma = 1/2).  The start value is the
    central-difference one, u_{-1} = u_0 - dt v_0 + dt^2/2 M^-1 (f_0 - K u_0).
    Returns u after n_steps; callback(n, u_prev, u) after every step."""
    M = sp.csc_matrix(M)
    K = sp.csr_matrix(K)
    lu = spla.splu(M)
    fine = np.asarray(fine, dtype=np.int64)
    Pm = np.zeros(M.shape[0], dtype=bool)
    Pm[fine] = True
    tau = dt / m
    u = np.array(u0, dtype=np.float64)
    u_prev = u - dt * np.asarray(v0) + 0.5 * dt * dt * lu.solve(ft[0] * fx - K @ u)

    def AP(q):
        y = np.zeros_like(q)
        y[Pm] = q[Pm]
        return lu.solve(K @ y)

    for n in range(n_steps):
        uc = u.copy()
        uc[Pm] = 0.0
        w = lu.solve(K @ uc - ft[n] * fx)
        q_old = u
        q = u - 0.5 * tau * tau * (w + AP(u))
        for _ in range(1, m):
            q, q_old = 2.0 * q - q_old - tau * tau * (w + AP(q)), q
        u, u_prev = 2.0 * q - u_prev, u
        if callback is not None:
            callback(n + 1, u_prev, u)
    return u


def lts_operator(M, K, fine, dt, m):
    """B with u_{n+1} = 2 u_n - u_{n-1} - dt^2 B u_n for the unforced local
    time-stepping leap-frog (dense; tiny meshes): the coarse step of
    lts_leapfrog_run applied to every unit vector.  The scheme is stable iff
    every eigenvalue of dt^2 B lies in [0, 4)."""
    Md = np.asarray(sp.csr_matrix(M).toarray())
    Kd = np.asarray(sp.csr_matrix(K).toarray())
    n = Md.shape[0]
    Pm = np.zeros(n, dtype=bool)
    Pm[np.asarray(fine, dtype=np.int64)] = True
    A = np.linalg.solve(Md, Kd)
    AP = A * Pm[None, :]                      # A P
    tau = dt / m
    U = np.eye(n)
    W = A @ (U * (~Pm)[:, None])             # w for every unit vector (columns)
    Q_old = U
    Q = U - 0.5 * tau * tau * (W + AP @ U)
    for _ in range(1, m):
        Q, Q_old = 2.0 * Q - Q_old - tau * tau * (W + AP @ Q), Q
    # u_{n+1} = 2 q_m - u_{n-1} with u_{n-1} = 0: 2 e - dt^2 B e = 2 Q e
    return (2.0 * U - 2.0 * Q) / (dt * dt)
