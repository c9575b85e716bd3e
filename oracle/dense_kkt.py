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


def solve_newton_bounded(inst, x, z, s, w, U, rd, rp, ru, rxz, rsw):
    """Dense LU of the whole Newton system with upper bounds (unknowns dx, dy,
    dz and ds, dw of the bounded variables U):
        A'dy + dz - E dw = r_d,  A dx = r_p,  E'dx + ds = r_u,
        Z dx + X dz = r_xz,  W ds + S dw = r_sw,
    E the columns of the identity on U.  Returns (dx, dy, dz, ds, dw) with ds,
    dw zero off U."""
    A = lp.full_matrix(inst).toarray()
    m, n = A.shape
    idx = np.flatnonzero(U)
    k = idx.size
    E = np.zeros((n, k))
    E[idx, np.arange(k)] = 1.0
    ox, oy, oz, os_, ow = 0, n, n + m, 2 * n + m, 2 * n + m + k
    N = 2 * n + m + 2 * k
    K = np.zeros((N, N))
    # rows in the order of the equations above, columns in that of the unknowns
    K[ox:ox + n, oy:oy + m] = A.T
    K[ox:ox + n, oz:oz + n] = np.eye(n)
    K[ox:ox + n, ow:ow + k] = -E
    K[oy:oy + m, ox:ox + n] = A
    K[oz:oz + n, ox:ox + n] = np.diag(z)
    K[oz:oz + n, oz:oz + n] = np.diag(x)
    K[os_:os_ + k, ox:ox + n] = E.T
    K[os_:os_ + k, os_:os_ + k] = np.eye(k)
    K[ow:ow + k, os_:os_ + k] = np.diag(w[idx])
    K[ow:ow + k, ow:ow + k] = np.diag(s[idx])
    rhs = np.concatenate([rd, rp, rxz, ru[idx], rsw[idx]])
    d = np.linalg.solve(K, rhs)
    ds = np.zeros(n)
    dw = np.zeros(n)
    ds[idx] = d[os_:os_ + k]
    dw[idx] = d[ow:ow + k]
    return d[ox:ox + n], d[oy:oy + m], d[oz:oz + n], ds, dw
