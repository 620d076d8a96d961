"""Per-axis finite-element operators (oracle; test infrastructure).

The paper treats the data as the piecewise linear function that takes the
data values at the nodes (Section IV-A) and corrects each level with the L2
projection of the multilevel coefficients.  On a tensor grid with piecewise
linear hat functions every operator is a Kronecker product of 1D operators:

* P (prolongation, n_fine x n_coarse): the coarse hat functions written in the
  fine basis.  A coarse node keeps its value; a new node j between coarse
  neighbours a < j < b gets (x_b - x_j)/(x_b - x_a) of G_a and
  (x_j - x_a)/(x_b - x_a) of G_b.
* M (mass matrix of the hats on one level): with spacings h_i = x_{i+1} - x_i,
  M_ii = (h_{i-1} + h_i)/3 and M_{i,i+1} = M_{i+1,i} = h_i/6 (h outside the
  grid is 0).

Multi-dimensional operators are applied one active axis at a time, axis 0
first.
"""
from __future__ import annotations

import bisect

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from .hierarchy import coarse_positions, new_positions


def prolongation(x: np.ndarray) -> sp.csr_matrix:
    """P for one axis whose level nodes have coordinates ``x``."""
    n = len(x)
    cpos = coarse_positions(n)
    col_of = {int(p): k for k, p in enumerate(cpos)}
    rows, cols, vals = [], [], []
    for p, k in col_of.items():
        rows.append(p)
        cols.append(k)
        vals.append(1.0)
    cl = [int(p) for p in cpos]  # ascending
    for j in new_positions(n):
        j = int(j)
        t = bisect.bisect_left(cl, j)
        a, b = cl[t - 1], cl[t]  # nearest coarse nodes left and right of j
        rows += [j, j]
        cols += [col_of[a], col_of[b]]
        vals += [(x[b] - x[j]) / (x[b] - x[a]), (x[j] - x[a]) / (x[b] - x[a])]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, len(cpos)))


def mass(x: np.ndarray) -> sp.csr_matrix:
    """Mass matrix of the piecewise linear hats on nodes ``x``."""
    n = len(x)
    h = np.diff(x)
    hl = np.concatenate([[0.0], h])  # spacing to the left of node i
    hr = np.concatenate([h, [0.0]])  # spacing to the right of node i
    diag = (hl + hr) / 3.0
    off = h / 6.0
    return sp.diags([off, diag, off], [-1, 0, 1], shape=(n, n), format="csr")


def mass_banded(x: np.ndarray) -> np.ndarray:
    """The same mass matrix in LAPACK banded storage (for solve_banded)."""
    n = len(x)
    h = np.diff(x)
    ab = np.zeros((3, n))
    ab[0, 1:] = h / 6.0
    ab[1, :] = (np.concatenate([[0.0], h]) + np.concatenate([h, [0.0]])) / 3.0
    ab[2, :-1] = h / 6.0
    return ab


def apply_along(A, X: np.ndarray, axis: int) -> np.ndarray:
    """Y = A applied to every line of X along ``axis`` (A may be sparse)."""
    Xm = np.moveaxis(X, axis, 0)
    sh = Xm.shape
    Y = A @ Xm.reshape(sh[0], -1)
    Y = np.asarray(Y).reshape((A.shape[0],) + sh[1:])
    return np.moveaxis(Y, 0, axis)


def solve_along(x: np.ndarray, F: np.ndarray, axis: int) -> np.ndarray:
    """Solve M z = f along ``axis`` for every line (M = mass matrix on x)."""
    Fm = np.moveaxis(F, axis, 0)
    sh = Fm.shape
    if sh[0] == 1:
        Z = Fm / mass(x).toarray()[0, 0]
    else:
        Z = scipy.linalg.solve_banded((1, 1), mass_banded(x), Fm.reshape(sh[0], -1))
    return np.moveaxis(np.asarray(Z).reshape(sh), 0, axis)


KAPPA_GRID = 2.0 ** 20


def transfer_norm(x: np.ndarray) -> float:
    """kappa = ||M_c^{-1} P^T M||_inf for the axis whose level nodes are ``x``.

    M_c^{-1} P^T M maps a function's nodal values on this level to the nodal
    values of its L2 projection onto the next coarser level (the correction
    step of the decomposition).  Its infinity norm (largest absolute row sum
    of the dense nc x n matrix, formed by a banded solve per column) bounds
    how much one projection can amplify a maximum.  It is rounded up to a
    multiple of 2^-20 so that every implementation computing it in FP64
    arrives at the same value.
    """
    xc = x[coarse_positions(len(x))]
    B = (prolongation(x).T @ mass(x)).toarray()
    if len(xc) == 1:
        X = B / mass(xc).toarray()[0, 0]
    else:
        X = scipy.linalg.solve_banded((1, 1), mass_banded(xc), B)
    kappa = float(np.max(np.sum(np.abs(X), axis=1)))
    return float(np.ceil(kappa * KAPPA_GRID) / KAPPA_GRID)
