"""Brute-force dense solves of the interior-point Newton system (Sec. 2.3).

Test infrastructure only (see package docstring).  Only for tiny instances:
the 3x3 Newton matrix has 2 n_tot + m_tot rows and is built and solved densely.
"""
from __future__ import annotations

import numpy as np

from . import lp


def newton_matrix(inst, x, z):
    """The unreduced Newton matrix [[0, A', I], [A, 0, 0], [Z, 0, X]] of Sec. 2.3."""
    A = lp.full_matrix(inst).toarray()
    m, n = A.shape
    K = np.zeros((2 * n + m, 2 * n + m))
    K[:n, n:n + m] = A.T
    K[:n, n + m:] = np.eye(n)
    K[n:n + m, :n] = A
    K[n + m:, :n] = np.diag(z)
    K[n + m:, n + m:] = np.diag(x)
    return K


def solve_newton(inst, x, z, rx, ry, rz):
    """(dx, dy, dz) solving the unreduced Newton system by dense LU."""
    K = newton_matrix(inst, x, z)
    d = np.linalg.solve(K, np.concatenate([rx, ry, rz]))
    n, m = x.size, ry.size
    return d[:n], d[n:n + m], d[n + m:]


def augmented_matrix(inst, x, z, rho, delta):
    """Regularized augmented matrix [[-(X^-1 Z + rho I), A'], [A, delta I]]:
    the system left after eliminating dz (Sec. 2.3), with a primal
    regularization rho and a dual regularization delta added."""
    A = lp.full_matrix(inst).toarray()
    m, n = A.shape
    K = np.zeros((n + m, n + m))
    K[:n, :n] = -np.diag(z / x + rho)
    K[:n, n:] = A.T
    K[n:, :n] = A
    K[n:, n:] = delta * np.eye(m)
    return K


def solve_regularized(inst, x, z, rx, ry, rz, rho, delta):
    """Dense solve of the regularized augmented system, then dz by the
    elimination formula dz = X^-1 (rz - Z dx)."""
    K = augmented_matrix(inst, x, z, rho, delta)
    n = x.size
    d = np.linalg.solve(K, np.concatenate([rx - rz / x, ry]))
    dx, dy = d[:n], d[n:]
    return dx, dy, (rz - z * dx) / x


def schur_indices(inst):
    """Indices of (y_L, y_G, x_0) inside the augmented vector [x; y]: the
    unknowns that the block elimination keeps in its Schur complement."""
    n_tot = int(inst.n.sum()) + inst.n0
    m_blocks = int(inst.m.sum())
    ylg = n_tot + m_blocks + np.arange(int(inst.l.sum()) + lp.ng(inst))
    x0 = int(inst.n.sum()) + np.arange(inst.n0)
    return np.concatenate([ylg, x0])
