"""Multilevel decomposition, recomposition and its adjoint (oracle).

TEST INFRASTRUCTURE ONLY.

Decomposition follows Algorithm 1 and Section IV-A of the paper, one level at
a time from the input grid (level L) down to level 1:

1. ``lerp``: the multilevel coefficients are the level-l values minus their
   multilinear interpolant from the coarse nodes, c = G_l - P G_l[coarse]
   (zero at the coarse nodes);
2. ``mass_trans``: f = (P^T M_l) c, the load vector of the coefficient
   function tested against the coarse hats;
3. ``tridiag``: z = M_{l-1}^{-1} f, one tridiagonal solve per line along each
   axis (the L2 projection of the coefficient function onto level l-1);
4. ``add``: G_{l-1} = G_l[coarse] + z.

The paper prints the correction as "Q_{l-1}u = Q_l u + Omega_l mc_l" and the
coefficients with an unbalanced parenthesis; the reading used is
mc_l = (I - Pi_{l-1}) Q_l u and Q_{l-1} u = Pi_{l-1} Q_l u + Q_{l-1} mc_l,
i.e. steps 1-4 above.

Recomposition inverts each level exactly: G_l[coarse] = G_{l-1} - z(c_l),
then G_l = P G_l[coarse] + c_l.

Stream order (the paper does not fix one): the level-0 nodal values in
row-major order, then for l = 1..L the 2^D - 1 subbands m = 1, 2, ...; in
subband m active axis d (0 = slowest) runs over the level's new nodes when bit
d of m is set and over its coarse nodes otherwise; each subband is row-major
(last axis fastest).
"""
from __future__ import annotations

import numpy as np

from .hierarchy import Hierarchy, coarse_positions, new_positions
from .operators import apply_along, mass, prolongation, solve_along


def _subband_index_sets(sizes, m: int):
    sets = []
    for d, n in enumerate(sizes):
        sets.append(new_positions(n) if (m >> d) & 1 else coarse_positions(n))
    return sets


def level_slices(h: Hierarchy):
    """[(start, stop)] of each level's entries in the stream, l = 0..L."""
    out, pos = [], 0
    for l in range(h.L + 1):
        cnt = h.level_count(l)
        out.append((pos, pos + cnt))
        pos += cnt
    return out


def pack_level(c: np.ndarray, sizes) -> np.ndarray:
    """Coefficients at the new nodes of one level, in subband order."""
    D = len(sizes)
    parts = []
    for m in range(1, 1 << D):
        idx = _subband_index_sets(sizes, m)
        parts.append(c[np.ix_(*idx)].ravel())
    return np.concatenate(parts) if parts else np.zeros(0)


def unpack_level(vals: np.ndarray, sizes) -> np.ndarray:
    """Inverse of pack_level: a level grid with zeros at the coarse nodes."""
    D = len(sizes)
    c = np.zeros(sizes, dtype=np.float64)
    pos = 0
    for m in range(1, 1 << D):
        idx = _subband_index_sets(sizes, m)
        shp = tuple(len(i) for i in idx)
        cnt = int(np.prod(shp, dtype=np.int64))
        c[np.ix_(*idx)] = vals[pos:pos + cnt].reshape(shp)
        pos += cnt
    assert pos == len(vals)
    return c


def _level_ops(h: Hierarchy, l: int):
    """Per active axis: (P, M_l, coords of level l-1) for level l >= 1."""
    ops = []
    for d in range(h.D):
        x = h.coords[l][d]
        ops.append((prolongation(x), mass(x), h.coords[l - 1][d]))
    return ops


def _prolong(G_c: np.ndarray, ops) -> np.ndarray:
    Y = G_c
    for d, (P, _, _) in enumerate(ops):
        Y = apply_along(P, Y, d)
    return Y


def _correction(c: np.ndarray, ops) -> np.ndarray:
    """z = (M_{l-1}^{-1} P^T M_l)^{kron} c: mass_trans then tridiag."""
    f = c
    for d, (P, M, _) in enumerate(ops):
        f = apply_along(M, f, d)
        f = apply_along(P.T.tocsr(), f, d)
    z = f
    for d, (_, _, xc) in enumerate(ops):
        z = solve_along(xc, z, d)
    return z


def decompose_level(G: np.ndarray, h: Hierarchy, l: int):
    """One level of Algorithm 1: returns (G_{l-1}, coefficients in stream order)."""
    sizes = h.sizes[l]
    ops = _level_ops(h, l)
    cidx = [coarse_positions(n) for n in sizes]
    G_c = G[np.ix_(*cidx)]
    c = G - _prolong(G_c, ops)                 # lerp
    z = _correction(c, ops)                     # mass_trans + tridiag
    G_prev = G_c + z                            # add
    return G_prev, pack_level(c, sizes)


def recompose_level(G_prev: np.ndarray, coeffs: np.ndarray, h: Hierarchy, l: int):
    """Inverse of decompose_level."""
    sizes = h.sizes[l]
    ops = _level_ops(h, l)
    c = unpack_level(coeffs, sizes)
    G_c = G_prev - _correction(c, ops)
    return _prolong(G_c, ops) + c


def _active_view(u: np.ndarray, h: Hierarchy) -> np.ndarray:
    return np.asarray(u, dtype=np.float64).reshape(h.sizes[h.L] if h.D else ())


def decompose(u: np.ndarray, h: Hierarchy | None = None, keep_levels: bool = False):
    """Full decomposition of ``u`` into the stream-ordered coefficient vector.

    Returns the FP64 vector of length N (and, with ``keep_levels``, the list
    of nodal grids G_0 .. G_L).
    """
    h = h or Hierarchy(u.shape)
    if h.N == 0:
        return (np.zeros(0), []) if keep_levels else np.zeros(0)
    G = _active_view(u, h)
    per_level = [None] * (h.L + 1)
    grids = [None] * (h.L + 1)
    grids[h.L] = G
    for l in range(h.L, 0, -1):
        G, per_level[l] = decompose_level(G, h, l)
        grids[l - 1] = G
    per_level[0] = np.asarray(G, dtype=np.float64).ravel()
    out = np.concatenate(per_level) if h.N else np.zeros(0)
    return (out, grids) if keep_levels else out


def recompose(stream: np.ndarray, h: Hierarchy, keep_levels: bool = False):
    """Inverse of decompose: the nodal values on the input grid (FP64)."""
    stream = np.asarray(stream, dtype=np.float64)
    if h.N == 0:
        out = np.zeros(h.shape)
        return (out, []) if keep_levels else out
    sl = level_slices(h)
    G = stream[sl[0][0]:sl[0][1]].reshape(h.sizes[0] if h.D else ())
    grids = [G]
    for l in range(1, h.L + 1):
        G = recompose_level(G, stream[sl[l][0]:sl[l][1]], h, l)
        grids.append(G)
    out = np.asarray(G).reshape(h.shape)
    return (out, grids) if keep_levels else out


def recompose_adjoint(grad_u: np.ndarray, h: Hierarchy) -> np.ndarray:
    """Transpose of recompose, applied to a gradient on the input grid.

    Recompose is linear in the coefficient vector: per level
    G_l = P (G_{l-1} - Z c_l) + E c_l with Z = M_{l-1}^{-1} P^T M_l E and E
    the embedding of the new-node values into the level grid.  Its transpose,
    taken level by level from the finest, is
    Gbar_{l-1} = P^T g,  cbar_l = E^T (g - M_l P M_{l-1}^{-1} Gbar_{l-1}).
    """
    if h.N == 0:
        return np.zeros(0)
    g = _active_view(grad_u, h)
    per_level = [None] * (h.L + 1)
    for l in range(h.L, 0, -1):
        sizes = h.sizes[l]
        ops = _level_ops(h, l)
        gc = g
        for d, (P, _, _) in enumerate(ops):
            gc = apply_along(P.T.tocsr(), gc, d)          # P^T g
        v = gc
        for d, (_, _, xc) in enumerate(ops):
            v = solve_along(xc, v, d)                      # M_{l-1}^{-1}
        w = v
        for d, (P, M, _) in enumerate(ops):
            w = apply_along(P, w, d)                       # P
            w = apply_along(M, w, d)                       # M_l
        per_level[l] = pack_level(g - w, sizes)            # E^T (g - ...)
        g = gc
    per_level[0] = np.asarray(g, dtype=np.float64).ravel()
    return np.concatenate(per_level) if h.N else np.zeros(0)


def finest_coefficients_at(u: np.ndarray, h: Hierarchy, flat_idx):
    """Finest-level coefficients at the given flat input indices, one by one.

    For each index that is a new node of the input grid: the value minus the
    multilinear interpolant from its nearest coarse neighbours on each axis
    where it is new (the lerp step), and its stream position.  Indices of
    coarse nodes are skipped.  Returns (stream positions, coefficients).
    With no decomposition level (L = 0) the stream is the nodal block itself,
    so every index is returned with its own value at its row-major position.
    """
    sizes = h.sizes[h.L]
    ua = np.asarray(u).reshape(sizes)
    l = h.L
    if l == 0:
        fi = np.asarray(flat_idx, dtype=np.int64)
        return fi.copy(), np.asarray(ua, dtype=np.float64).ravel()[fi]
    sl = level_slices(h)
    sub_sets = {}
    sub_off = {}
    acc = sl[l][0]
    for m in range(1, 1 << h.D):
        sets = _subband_index_sets(sizes, m)
        sub_sets[m] = sets
        sub_off[m] = acc
        acc += int(np.prod([len(x) for x in sets], dtype=np.int64))
    cpos = [coarse_positions(n) for n in sizes]
    pos_out, c_out = [], []
    for fi in flat_idx:
        idx = np.unravel_index(int(fi), sizes)
        m = 0
        taps = []
        for d, i in enumerate(idx):
            x = h.coords[l][d]
            if i in set(cpos[d].tolist()):
                taps.append([(i, 1.0)])
            else:
                m |= 1 << d
                k = int(np.searchsorted(cpos[d], i))
                a, b = int(cpos[d][k - 1]), int(cpos[d][k])
                taps.append([(a, (x[b] - x[i]) / (x[b] - x[a])), (b, (x[i] - x[a]) / (x[b] - x[a]))])
        if m == 0:
            continue
        interp = 0.0
        for corner in np.ndindex(*[len(t) for t in taps]):
            w = 1.0
            where = []
            for d, c in enumerate(corner):
                where.append(taps[d][c][0])
                w *= taps[d][c][1]
            interp += w * float(ua[tuple(where)])
        c = float(ua[idx]) - interp
        sets = sub_sets[m]
        loc = [int(np.searchsorted(sets[d], idx[d])) for d in range(h.D)]
        pos = sub_off[m] + int(np.ravel_multi_index(loc, [len(x) for x in sets]))
        pos_out.append(pos)
        c_out.append(c)
    return np.asarray(pos_out, dtype=np.int64), np.asarray(c_out)
