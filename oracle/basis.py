"""GLL / Gauss-Legendre points and the Lagrange basis (oracle; FP64).

Follows Section "Spatial Discretization": Lagrange polynomials of degree p on
the p+1 Gauss-Lobatto-Legendre points, i.e. -1, +1 and the roots of the
Lobatto polynomial of order p-1 (which is proportional to P_p', the
derivative of the Legendre polynomial P_p).
"""
from __future__ import annotations

import numpy as np


def legendre(p: int, x):
    """P_p(x) and P_{p-1}(x) by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if p == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(1, p):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    return p1, p0


def gll(p: int):
    """Gauss-Lobatto-Legendre nodes (ascending) and weights for order p >= 1.

    Interior nodes are the roots of P_p', found by Newton's method with
    P_p'' taken from Legendre's differential equation.  Weights are
    w_j = 2 / (p (p+1) P_p(x_j)^2).
    """
    if p < 1:
        raise ValueError("p >= 1")
    x = -np.cos(np.pi * np.arange(p + 1) / p)          # Chebyshev-Lobatto start
    inner = x[1:-1].copy()
    for _ in range(100):
        P, Pm1 = legendre(p, inner)
        dP = p * (Pm1 - inner * P) / (1.0 - inner ** 2)
        d2P = (2.0 * inner * dP - p * (p + 1) * P) / (1.0 - inner ** 2)
        step = dP / d2P
        inner = inner - step
        if np.max(np.abs(step), initial=0.0) < 1e-16:
            break
    x[1:-1] = inner
    x[0], x[-1] = -1.0, 1.0
    P, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * P ** 2)
    return x, w


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule on [-1, 1] (library routine)."""
    return np.polynomial.legendre.leggauss(n)


def lagrange(nodes, xi):
    """Values N_i(xi) of the Lagrange polynomials on ``nodes``.

    Returns an array of shape (len(xi), len(nodes)):
    N_i(xi) = prod_{j != i} (xi - x_j) / (x_i - x_j).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    n = len(nodes)
    out = np.ones((len(xi), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                out[:, i] *= (xi - nodes[j]) / (nodes[i] - nodes[j])
    return out


def lagrange_deriv(nodes, xi):
    """Derivatives N_i'(xi), shape (len(xi), len(nodes)), by the product rule."""
    nodes = np.asarray(nodes, dtype=np.float64)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    n = len(nodes)
    out = np.zeros((len(xi), n))
    for i in range(n):
        for k in range(n):
            if k == i:
                continue
            term = np.full(len(xi), 1.0 / (nodes[i] - nodes[k]))
            for j in range(n):
                if j != i and j != k:
                    term *= (xi - nodes[j]) / (nodes[i] - nodes[j])
            out[:, i] += term
    return out
