"""Ten spring-coupled masses (Section "Spring-coupled masses"; oracle).

Chain wall - k - m1 - k - ... - m1 (eight masses of 1 kg) - k - m2 - k - m2
(two masses of 1e-3 kg), k = 1 N/m, free end.  The harmonic load
sin(2 pi 0.1 t) acts on the third-last mass.  The eight heavy masses are the
"uncut" (explicit) dofs, the two light ones the "badly cut" (implicit) dofs.
The reference solution is the steady harmonic response u(t) = a sin(w t)
with (K - w^2 M) a = e (the Helmholtz solution named in that section).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

N_MASSES = 10
FS = 0.1


def matrices():
    m = np.array([1.0] * 8 + [1e-3] * 2)
    M = np.diag(m)
    K = 2.0 * np.eye(N_MASSES) - np.eye(N_MASSES, k=1) - np.eye(N_MASSES, k=-1)
    K[-1, -1] = 1.0                      # free end: one spring on the last mass
    fx = np.zeros(N_MASSES)
    fx[N_MASSES - 3] = 1.0               # third-last mass
    Id = np.arange(8)
    Ic = np.arange(8, 10)
    return M, K, fx, Id, Ic


def ft(t):
    return np.sin(2.0 * np.pi * FS * np.asarray(t, dtype=np.float64))


def reference(t):
    """Exact harmonic response, its displacement at times t (len(t), 10)."""
    M, K, fx, _, _ = matrices()
    w = 2.0 * np.pi * FS
    a = np.linalg.solve(K - w * w * M, fx)
    return np.outer(np.sin(w * np.asarray(t)), a), w * a


def dt_crit(K, M):
    lam = scipy.linalg.eigh(K, M, eigvals_only=True)[-1]
    return 2.0 / np.sqrt(lam)
