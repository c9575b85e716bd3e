"""Constraint operator of the arrowhead LP (Sec. 2.2 standard form, Sec. 3.2
block structure restricted to equalities; local links and global linking rows,
Sec. 3.3).  Rows: the blocks, then the link pairs, then the global rows.

Test infrastructure only (see package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def offsets(inst):
    xo = np.concatenate([[0], np.cumsum(inst.n)]).astype(np.int64)
    yo = np.concatenate([[0], np.cumsum(inst.m)]).astype(np.int64)
    lo = np.concatenate([[0], np.cumsum(inst.l)]).astype(np.int64)
    return xo, yo, lo


def ng(inst):
    """Number of global linking rows."""
    return 0 if getattr(inst, "Wg", None) is None else int(inst.Wg[0].shape[0])


def matvec(inst, x):
    """A x for the full constraint matrix (block rows, link rows, global rows)."""
    xo, yo, lo = offsets(inst)
    x0 = x[xo[-1]:]
    out = np.empty(int(yo[-1] + lo[-1]) + ng(inst))
    for i in range(inst.N):
        out[yo[i]:yo[i + 1]] = inst.A[i] @ x[xo[i]:xo[i + 1]] + inst.C[i] @ x0
    base = yo[-1]
    for j in range(inst.N - 1):
        r = inst.FR[j] @ x[xo[j]:xo[j + 1]] + inst.FL[j] @ x[xo[j + 1]:xo[j + 2]]
        if inst.F0 is not None:
            r = r + inst.F0[lo[j]:lo[j + 1]] @ x0
        out[base + lo[j]: base + lo[j + 1]] = r
    gb = int(base + lo[-1])
    for k in range(ng(inst)):
        r = 0.0
        for i in range(inst.N):
            r += inst.Wg[i][k] @ x[xo[i]:xo[i + 1]]
        out[gb + k] = r + inst.Wg0[k] @ x0
    return out


def rmatvec(inst, y):
    """A' y for the full constraint matrix."""
    xo, yo, lo = offsets(inst)
    out = np.zeros(int(xo[-1]) + inst.n0)
    base = yo[-1]
    for i in range(inst.N):
        yi = y[yo[i]:yo[i + 1]]
        out[xo[i]:xo[i + 1]] += inst.A[i].T @ yi
        out[xo[-1]:] += inst.C[i].T @ yi
    for j in range(inst.N - 1):
        yl = y[base + lo[j]: base + lo[j + 1]]
        out[xo[j]:xo[j + 1]] += inst.FR[j].T @ yl
        out[xo[j + 1]:xo[j + 2]] += inst.FL[j].T @ yl
        if inst.F0 is not None:
            out[xo[-1]:] += inst.F0[lo[j]:lo[j + 1]].T @ yl
    if ng(inst):
        yg = y[int(base + lo[-1]):]
        for i in range(inst.N):
            out[xo[i]:xo[i + 1]] += inst.Wg[i].T @ yg
        out[xo[-1]:] += inst.Wg0.T @ yg
    return out


def full_matrix(inst):
    """The whole constraint matrix as a scipy CSR matrix (rows y, columns x)."""
    xo, yo, lo = offsets(inst)
    N = inst.N
    n_tot = int(xo[-1]) + inst.n0
    m_tot = int(yo[-1] + lo[-1]) + ng(inst)
    rows = []
    for i in range(N):
        row = [None] * (N + 1)
        row[i] = sp.csr_matrix(inst.A[i])
        row[N] = sp.csr_matrix(inst.C[i])
        rows.append(row)
    blocks = sp.bmat(rows, format="csr") if N else sp.csr_matrix((0, n_tot))
    link = sp.lil_matrix((int(lo[-1]), n_tot))
    for j in range(N - 1):
        r = slice(lo[j], lo[j + 1])
        link[r, xo[j]:xo[j + 1]] = inst.FR[j]
        link[r, xo[j + 1]:xo[j + 2]] = inst.FL[j]
        if inst.F0 is not None:
            link[r, xo[-1]:] = inst.F0[lo[j]:lo[j + 1]]
    glob = sp.lil_matrix((ng(inst), n_tot))
    if ng(inst):
        for i in range(N):
            glob[:, xo[i]:xo[i + 1]] = inst.Wg[i]
        glob[:, xo[-1]:] = inst.Wg0
    full = sp.vstack([blocks, link.tocsr(), glob.tocsr()], format="csr")
    assert full.shape == (m_tot, n_tot)
    return full


def abs_row_col_sums(inst):
    """Row sums and column sums of |A| (used for the infinity norm of the KKT
    matrix in the refinement stopping test)."""
    Af = abs(full_matrix(inst))
    return np.asarray(Af.sum(axis=1)).ravel(), np.asarray(Af.sum(axis=0)).ravel()


def kkt_inf_norm(rowabs, colabs, x, z):
    """Infinity norm of the 3x3 Newton matrix [[0, A', I], [A, 0, 0], [Z, 0, X]]
    (Sec. 2.3): the largest absolute row sum over its three row blocks."""
    return max(float(np.max(colabs + 1.0)) if colabs.size else 1.0,
               float(np.max(rowabs)) if rowabs.size else 0.0,
               float(np.max(x + z)))
