"""Learned per-cut-cell preconditioner for the implicit block and the
flexible conjugate gradient it drives (oracle; FP64 with optional BF16
rounding at the points where the device computes in BF16).

Test infrastructure only (see the package docstring).  The paper solves the
implicit system S a = r of Section "Time Integration" by a sparse direct
solver; the iterative solvers are an addition of this project, defined here
and mirrored by the device kernels.

Element-block (additive Schwarz) preconditioner: for every cut cell e with
local c dofs idx_e (all (p+1)^d nodes of a cut cell are c dofs) and Binv_e
the inverse of S[idx_e, idx_e],

    B r = sum_e P_e^T Binv_e r_e     (symmetric positive definite).

Learned preconditioner: a learned correction on top of B.  With r_e =
r[idx_e], s_e = ||r_e||_2, d_e = diag(S)[idx_e] and w the partition of unity
1 / (number of cut cells sharing a dof),

    x_e = [ r_e / s_e ,  d_e .* (B r)_e / s_e ,  d_e / max d_e ]     (3 n_e features)
    h1  = relu(W1 x_e + b1),  h2 = relu(W2 h1 + b2),  y_e = W3 h2 + b3
    c   = w .* sum_e P_e^T (s_e y_e / d_e)                            (learned correction)
    z   = beta1 B r + beta2 c

where (beta1, beta2) minimise the S-norm of the error ||S^-1 r - z||_S over
span{B r, c}: with a11 = (Br)^T S Br, a12 = (Br)^T S c, a22 = c^T S c,
b1 = (Br)^T r, b2 = c^T r, beta = [a11 a12; a12 a22]^-1 [b1; b2], or, when
c = 0 or the pair is degenerate (a11 a22 - a12^2 <= 1e-12 a11 a22),
beta = (b1 / a11, 0).  The element-block step scaled by b1 / a11 is thus
always in reach (CG does not see a scalar factor), and

trained on pairs (r, x) from the method's own implicit solves (x = S^-1 r:
each step's right-hand side with the new acceleration, and the warm-start
residual rhs - S a^c_n with the change of the acceleration) so that y_e
reproduces

    t_e = d_e .* (x - B r)_e / s_e,

the part of the exact solution that B misses, seen from cell e.  With
y_e = t_e for every cell the correction is c = x - B r (w sums to one over
the cells of every c dof), the span holds x and z = x exactly, so a perfect
network makes the flexible CG converge in one iteration; a zero network
leaves the (scaled) element-block step.  The loss is the
mean over (pair, cell) of ||y_e - t_e||^2 over the first n_e outputs; a
cell enters a pair's loss only when s_e > 0 and s_e >= TRAIN_REL times the
pair's largest s_e (on cells with negligible residual t_e answers residuals
elsewhere, which the cell's features do not see).

BF16 emulation (bf16=True): the GEMM operands (features, weights, hidden
activations, output gradients) are rounded to BF16 (round to nearest even)
exactly where the device does; sums are FP64 here and FP32 on the device.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import scipy.sparse as sp

from .fcm import CUT, cell_nodes

HIDDEN = 128
TRAIN_REL = 1e-3   # a cell enters a pair's loss when its residual norm is at least this times the pair's largest


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64).reshape(a.shape)


def pad16(n):
    return (n + 15) // 16 * 16


@dataclass
class ElementData:
    idx: np.ndarray        # (E, n_e) c indices of every cut cell's nodes
    diag: np.ndarray       # (n_c,) diagonal of S
    gfeat: np.ndarray      # (E, n_e) diag(S)[idx_e] / max diag(S)[idx_e]
    inv_mult: np.ndarray   # (n_c,) 1 / number of cut cells sharing the dof
    binv: np.ndarray       # (E, n_e, n_e) inverses of the cells' diagonal blocks of S
    S: sp.csr_matrix = None  # the system matrix (for the combination step)

    @property
    def n_e(self):
        return self.idx.shape[1]


def element_data(disc, S, c_of_grid=None) -> ElementData:
    """Cut cells in ascending cell id; S in the c order whose grid ids are
    disc.Ic (ascending) unless c_of_grid maps grid ids to another c order."""
    cells = np.nonzero(disc.flags == CUT)[0]
    dim = len(disc.n_cells)
    if c_of_grid is None:
        c_of_grid = np.full(disc.n_grid, -1, dtype=np.int64)
        c_of_grid[disc.Ic] = np.arange(len(disc.Ic))
    rows = []
    for cid in cells:
        ci = np.unravel_index(cid, disc.n_cells[::-1])[::-1]
        g = cell_nodes(disc.grid, disc.p, ci)
        rows.append(c_of_grid[g])
    idx = np.array(rows, dtype=np.int64).reshape(len(cells), (disc.p + 1) ** dim)
    assert np.all(idx >= 0)
    diag = np.asarray(S.diagonal(), dtype=np.float64)
    de = diag[idx]
    gfeat = de / de.max(axis=1, keepdims=True)
    mult = np.bincount(idx.ravel(), minlength=len(diag)).astype(np.float64)
    Sc = sp.csr_matrix(S)
    binv = np.array([np.linalg.inv(Sc[ix][:, ix].toarray()) for ix in idx]).reshape(len(idx), idx.shape[1],
                                                                                    idx.shape[1])
    return ElementData(idx=idx, diag=diag, gfeat=gfeat, inv_mult=1.0 / np.maximum(mult, 1.0), binv=binv, S=Sc)


def scatter(ze, ed: ElementData):
    """sum_e P_e^T ze_e for per-cell vectors ze (E, n_e)."""
    z = np.zeros(len(ed.diag))
    np.add.at(z, ed.idx.ravel(), ze.ravel())
    return z


def block_precond(r, ed: ElementData):
    """Element-block (additive Schwarz) preconditioner."""
    return scatter(np.einsum("eij,ej->ei", ed.binv, r[ed.idx]), ed)


@dataclass
class Params:
    W1: np.ndarray   # (H, F_pad)
    b1: np.ndarray
    W2: np.ndarray   # (H, H)
    b2: np.ndarray
    W3: np.ndarray   # (O_pad, H)
    b3: np.ndarray

    def names(self):
        return ["W1", "b1", "W2", "b2", "W3", "b3"]

    def copy(self):
        return Params(*[getattr(self, k).copy() for k in self.names()])


def features(r, ed: ElementData, f_pad, br=None):
    """(E, f_pad) features and the local norms s_e (br: B r when known)."""
    if br is None:
        br = block_precond(r, ed)
    re = r[ed.idx]
    s = np.sqrt(np.sum(re * re, axis=1))
    safe = np.where(s > 0, s, 1.0)
    X = np.zeros((len(re), f_pad))
    n = ed.n_e
    de = ed.diag[ed.idx]
    X[:, :n] = re / safe[:, None]
    X[:, n:2 * n] = de * br[ed.idx] / safe[:, None]
    X[:, 2 * n:3 * n] = ed.gfeat
    return X, s


def forward(P: Params, X, bf=True):
    q = bf16 if bf else (lambda a: a)
    Xq, W1, W2, W3 = q(X), q(P.W1), q(P.W2), q(P.W3)
    a1 = Xq @ W1.T + P.b1
    h1 = np.maximum(a1, 0.0)
    h1q = q(h1)
    a2 = h1q @ W2.T + P.b2
    h2 = np.maximum(a2, 0.0)
    h2q = q(h2)
    y = h2q @ W3.T + P.b3
    return y, {"Xq": Xq, "W1": W1, "W2": W2, "W3": W3, "a1": a1, "h1q": h1q, "a2": a2, "h2q": h2q}


def combine(r, br, c, S):
    """beta1 br + beta2 c minimising the S-norm of S^-1 r - z over span{br, c}
    (module docstring; a degenerate pair keeps the scaled br)."""
    q1, q2 = S @ br, S @ c
    a11, a22, a12 = br @ q1, c @ q2, br @ q2
    b1, b2 = br @ r, c @ r
    det = a11 * a22 - a12 * a12
    be1, be2 = (b1 / a11 if a11 > 0 else 0.0), 0.0
    if a22 > 0 and det > 1e-12 * a11 * a22:
        be1 = (b1 * a22 - b2 * a12) / det
        be2 = (a11 * b2 - a12 * b1) / det
    return be1 * br + be2 * c


def apply_outputs(y, r, ed: ElementData, br=None):
    """The assembly step of the learned preconditioner for given outputs y:
    the correction c = w .* sum_e P_e^T (s_e y_e / d_e), then the
    energy-optimal combination of B r and c."""
    if br is None:
        br = block_precond(r, ed)
    re = r[ed.idx]
    s = np.sqrt(np.sum(re * re, axis=1))
    c = ed.inv_mult * scatter(s[:, None] * y[:, :ed.n_e] / ed.diag[ed.idx], ed)
    return combine(r, br, c, ed.S)


def apply(P: Params, r, ed: ElementData, bf=True):
    """z = learned preconditioner(r) (see the module docstring)."""
    br = block_precond(r, ed)
    X, _ = features(r, ed, P.W1.shape[1], br)
    y, _ = forward(P, X, bf)
    return apply_outputs(y, r, ed, br)


def targets(r, x, ed: ElementData, o_pad, br=None):
    """Per-cell targets t_e of y_e for a pair (r, x = S^-1 r), and the mask
    of the cells that enter the loss (local residual norm positive and at
    least TRAIN_REL times the pair's largest)."""
    if br is None:
        br = block_precond(r, ed)
    re = r[ed.idx]
    s = np.sqrt(np.sum(re * re, axis=1))
    # cells whose residual is negligible against the pair's largest local
    # residual carry targets set by residuals elsewhere: left out
    ok = (s > 0) & (s >= TRAIN_REL * s.max()) if len(s) else s > 0
    safe = np.where(s > 0, s, 1.0)
    T = np.zeros((len(re), o_pad))
    T[:, :ed.n_e] = ed.diag[ed.idx] * (x - br)[ed.idx] / safe[:, None]
    T[~ok] = 0.0
    return T, ok


def loss_and_grads(P: Params, pairs, ed: ElementData, bf=True):
    """Mean over (pair, cell) of ||y_e - t_e||^2 on the first n_e outputs,
    for pairs (r, x), and its gradients by back-propagation (BF16 rounding of
    the GEMM operands as on the device when bf)."""
    q = bf16 if bf else (lambda a: a)
    n = ed.n_e
    o_pad = P.W3.shape[0]
    Xs, Ts = [], []
    for r, x in pairs:
        br = block_precond(r, ed)
        X, _ = features(r, ed, P.W1.shape[1], br)
        T, ok = targets(r, x, ed, o_pad, br)
        Xs.append(X[ok])
        Ts.append(T[ok])
    X = np.concatenate(Xs)
    T = np.concatenate(Ts)
    B = len(X)
    y, c = forward(P, X, bf)
    diff = np.zeros_like(y)
    diff[:, :n] = y[:, :n] - T[:, :n]
    loss = np.sum(diff * diff) / B
    dy = 2.0 * diff / B
    dyq = q(dy)
    g = {}
    g["W3"] = dyq.T @ c["h2q"]
    g["b3"] = dy.sum(axis=0)
    dh2 = dyq @ c["W3"]
    da2 = dh2 * (c["a2"] > 0)
    da2q = q(da2)
    g["W2"] = da2q.T @ c["h1q"]
    g["b2"] = da2.sum(axis=0)
    dh1 = da2q @ c["W2"]
    da1 = dh1 * (c["a1"] > 0)
    da1q = q(da1)
    g["W1"] = da1q.T @ c["Xq"]
    g["b1"] = da1.sum(axis=0)
    return loss, g, B


def adam_step(P: Params, g, state: Dict, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) of every parameter in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in P.names():
        m = state.setdefault("m_" + k, np.zeros_like(getattr(P, k)))
        v = state.setdefault("v_" + k, np.zeros_like(getattr(P, k)))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        getattr(P, k)[...] -= lr * mh / (np.sqrt(vh) + eps)


def flexible_cg(S, b, x0, precond, tol=1e-10, maxit=1000, fallback=None):
    """Flexible preconditioned CG (Polak-Ribiere form, which tolerates a
    preconditioner that changes from one application to the next).  Where
    the preconditioned residual is not a descent direction (r.z <= 0) the
    fallback preconditioner is used for that application.  Stops when
    ||r|| <= tol ||b||; returns (x, iterations, converged)."""
    def prec(r):
        z = precond(r)
        if fallback is not None and not (r @ z > 0):
            z = fallback(r)
        return z

    x = np.array(x0, dtype=np.float64)
    r = b - S @ x
    nb = np.linalg.norm(b)
    if nb == 0:
        return np.zeros_like(b), 0, True
    if np.linalg.norm(r) <= tol * nb:
        return x, 0, True
    z = prec(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = S @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r_new = r - alpha * q
        if np.linalg.norm(r_new) <= tol * nb:
            return x, it, True
        z_new = prec(r_new)
        beta = (z_new @ (r_new - r)) / rz
        rz = r_new @ z_new
        p = z_new + beta * p
        r = r_new
    return x, maxit, False
