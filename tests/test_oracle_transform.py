"""Pins of the oracle's multilevel transform against facts it does not compute.

* exact inversion: recompose(decompose(u)) = u (FP64, 1e-12);
* the correction equals a dense L2 projection whose Gram matrices come from
  Gauss quadrature of hat-function products evaluated with numpy.interp, and
  whose prolongation is the coarse hats sampled at the fine nodes;
* closed forms: multilinear data has zero coefficients; the nodal x^2 projects
  to x^2 - h^2/2; the sawtooth projects to 1/2 per axis;
* the adjoint is the transpose: dot-product test and dense R^T on small grids;
* hierarchy sizes worked out by hand from the coarsening rule;
* the one-by-one finest-level coefficient helper (used where the full
  decomposition would be too large) equals the finest level of decompose,
  positions included.
"""

import numpy as np
import pytest

import oracle
from oracle import Hierarchy
from oracle.transform import decompose_level, level_slices


def _coarse_idx(n):
    idx = list(range(0, n, 2))
    if n % 2 == 0:
        idx.append(n - 1)
    return np.array(idx)


# ---------------------------------------------------------------- hierarchy
@pytest.mark.parametrize("shape,L,coarsest", [
    ((513, 513, 513), 9, (2, 2, 2)),
    ((300, 400, 500), 9, (2, 2, 2)),
    ((33, 257, 65), 5, (2, 9, 3)),
    ((65, 65, 65), 6, (2, 2, 2)),
    ((8193, 8193), 13, (2, 2)),
    ((2, 7), 0, (2, 7)),
    ((1, 9, 1), 3, (2,)),
])
def test_hierarchy_levels(shape, L, coarsest):
    h = Hierarchy(shape)
    assert h.L == L
    assert h.sizes[0] == coarsest


def test_hierarchy_nonuniform_300():
    # 300 -> 151 -> 76 -> 39 -> 20 -> 11 -> 6 -> 4 -> 3 -> 2 by the rule
    # "keep even positions, plus the last node when the count is even"
    h = Hierarchy((300,))
    assert [s[0] for s in h.sizes[::-1]] == [300, 151, 76, 39, 20, 11, 6, 4, 3, 2]
    # level 8 (151 nodes) keeps original coordinates 0,2,...,298,299
    x = h.coords[8][0]
    assert x[0] == 0 and x[-2] == 298 and x[-1] == 299


# ---------------------------------------------------------------- inversion
@pytest.mark.parametrize("shape", [(65, 65, 65), (9, 5, 4), (6, 6, 6), (17,), (33, 20),
                                   (1, 7, 1), (2, 2, 2), (3, 5), (30, 41, 12), (100,)])
def test_roundtrip_exact(shape):
    rng = np.random.default_rng(11)
    u = rng.standard_normal(shape)
    h = Hierarchy(shape)
    c = oracle.decompose(u, h)
    assert c.shape == (h.N,)
    r = oracle.recompose(c, h)
    assert np.max(np.abs(r - u)) <= 1e-12 * np.max(np.abs(u))


# ---------------------------------------------------- dense L2 projection pin
def _hat_matrix(nodes, at):
    """hat_i(at_j) for the piecewise linear hats on ``nodes`` (via numpy.interp)."""
    return np.stack([np.interp(at, nodes, np.eye(len(nodes))[i]) for i in range(len(nodes))])


def _gram_by_quadrature(nodes_a, nodes_b, fine_nodes):
    """int hat^a_i hat^b_j over the axis: 2-point Gauss per fine cell (exact)."""
    g = np.zeros((len(nodes_a), len(nodes_b)))
    for lo, hi in zip(fine_nodes[:-1], fine_nodes[1:]):
        mid, half = (lo + hi) / 2, (hi - lo) / 2
        pts = np.array([mid - half / np.sqrt(3), mid + half / np.sqrt(3)])
        A = _hat_matrix(nodes_a, pts)
        B = _hat_matrix(nodes_b, pts)
        g += half * (A @ B.T)
    return g


def _kron_all(mats):
    out = np.ones((1, 1))
    for m in mats:
        out = np.kron(out, m)
    return out


@pytest.mark.parametrize("shape", [(9, 9, 9), (6, 6, 6), (9, 5, 4), (7, 6), (5,), (8,)])
def test_correction_is_dense_l2_projection(shape):
    rng = np.random.default_rng(3)
    u = rng.standard_normal(shape)
    h = Hierarchy(shape)
    l = h.L
    x_f = [np.arange(n, dtype=float) for n in shape]
    x_c = [x[_coarse_idx(len(x))] for x in x_f]
    # prolongation: coarse hats sampled at the fine nodes
    P = _kron_all([_hat_matrix(xc, xf).T for xc, xf in zip(x_c, x_f)])
    Gc_mass = _kron_all([_gram_by_quadrature(xc, xc, xf) for xc, xf in zip(x_c, x_f)])
    cross = _kron_all([_gram_by_quadrature(xc, xf, xf) for xc, xf in zip(x_c, x_f)])
    cidx = np.ix_(*[_coarse_idx(n) for n in shape])
    Gc = u[cidx].ravel()
    c = u.ravel() - P @ Gc
    z = np.linalg.solve(Gc_mass, cross @ c)
    G_prev, coeffs = decompose_level(u, h, l)
    assert np.max(np.abs(G_prev.ravel() - (Gc + z))) < 1e-12
    # the coefficients are c at the new nodes (any order: compare sorted)
    new_mask = np.ones(shape, bool)
    new_mask[cidx] = False
    assert np.allclose(np.sort(coeffs), np.sort(c.reshape(shape)[new_mask]), atol=1e-13)


# ------------------------------------------------------------- closed forms
@pytest.mark.parametrize("shape", [(17, 9, 5), (12, 7), (10,)])
def test_multilinear_has_zero_coefficients(shape):
    grids = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    u = 1.5 + sum((d + 1) * 0.3 * g for d, g in enumerate(grids))
    if len(shape) > 1:
        u = u + 0.01 * grids[0] * grids[-1]       # bilinear term: still multilinear
    h = Hierarchy(shape)
    c, levels = oracle.decompose(u, h, keep_levels=True)
    sl = level_slices(h)
    assert np.max(np.abs(c[sl[0][1]:])) < 1e-12
    # and each coarse grid is the data restricted to its nodes
    for l in range(h.L):
        idx = np.ix_(*[h.coords[l][d].astype(int) for d in range(h.D)])
        assert np.max(np.abs(levels[l] - u[idx])) < 1e-11


@pytest.mark.parametrize("n", [9, 17, 65])
def test_parabola_projects_to_shifted_parabola(n):
    x = np.arange(n, dtype=float)
    h = Hierarchy((n,))
    G_prev, _ = decompose_level(x ** 2, h, h.L)
    assert np.max(np.abs(G_prev - (x[::2] ** 2 - 0.5))) < 1e-12


@pytest.mark.parametrize("shape", [(17,), (9, 9), (9, 5, 17)])
def test_sawtooth_projects_to_half_per_axis(shape):
    saw = [(np.arange(n) % 2).astype(float) for n in shape]
    u = saw[0]
    for s in saw[1:]:
        u = np.multiply.outer(u, s)
    h = Hierarchy(shape)
    G_prev, _ = decompose_level(u, h, h.L)
    assert np.max(np.abs(G_prev - 0.5 ** len(shape))) < 1e-14


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("shape", [(9, 9, 9), (6, 6, 6), (9, 5, 4), (33, 20), (17,)])
def test_adjoint_dot_product(shape):
    rng = np.random.default_rng(5)
    h = Hierarchy(shape)
    x = rng.standard_normal(h.N)
    y = rng.standard_normal(shape)
    lhs = np.vdot(oracle.recompose(x, h), y)
    rhs = np.vdot(x, oracle.recompose_adjoint(y, h))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0) * 10


@pytest.mark.parametrize("shape", [(5, 4, 3), (9, 5), (6,)])
def test_adjoint_equals_dense_transpose(shape):
    h = Hierarchy(shape)
    R = np.stack([oracle.recompose(e, h).ravel() for e in np.eye(h.N)], axis=1)
    rng = np.random.default_rng(2)
    y = rng.standard_normal(shape)
    assert np.max(np.abs(R.T @ y.ravel() - oracle.recompose_adjoint(y, h))) < 1e-12


def test_recompose_is_identity_plus_projection_complements():
    # R(delta) = delta_0 + sum_l (I - Q_{l-1}) delta_l: a single level-l unit
    # coefficient reconstructs to a function with zero L2 inner product with
    # every coarser hat (it is orthogonal to V_{l-1}).
    shape = (9, 9)
    h = Hierarchy(shape)
    sl = level_slices(h)
    e = np.zeros(h.N)
    e[sl[2][0] + 3] = 1.0
    g = oracle.recompose(e, h)
    x = np.arange(9.0)
    xc = np.array([0.0, 4.0, 8.0])      # the level-1 nodes of a 9-node axis
    M1 = _gram_by_quadrature(xc, x, x)
    assert np.max(np.abs(M1 @ g @ M1.T)) < 1e-13


# ------------------------------------------------- finest_coefficients_at
@pytest.mark.parametrize("shape", [(9, 5, 4), (6, 7, 5), (13, 10, 6), (17,), (12, 9), (1, 7, 1),
                                   (2, 6, 3)])
def test_finest_coefficients_at_equals_decompose(shape):
    """Every index of the grid: coarse nodes are skipped, new nodes give the
    coefficient and stream position that decompose writes."""
    rng = np.random.default_rng(8)
    u = rng.standard_normal(shape)
    h = Hierarchy(shape)
    full = oracle.decompose(u, h)
    a, b = level_slices(h)[h.L]
    idx = np.arange(u.size)
    pos, c = oracle.transform.finest_coefficients_at(u, h, idx)
    assert len(pos) == b - a                      # one per new node
    assert np.array_equal(np.sort(pos), np.arange(a, b))
    assert np.max(np.abs(c - full[pos])) <= 1e-14 * max(1.0, float(np.max(np.abs(u))))


@pytest.mark.parametrize("shape", [(17, 9, 13), (33, 33, 33), (65, 40), (100,), (5, 1, 7), (2, 3)])
def test_finest_coefficients_at_equals_the_decomposition(shape):
    # the one-by-one sampler the full-size GPU checks use: at every input
    # index it must return the finest level's coefficient (value minus the
    # multilinear interpolant of the coarse corners) at its stream position,
    # exactly as the level-by-level decomposition stores it
    rng = np.random.default_rng(len(shape) * 7 + shape[0])
    u = rng.standard_normal(shape)
    u += np.cumsum(np.cumsum(u, axis=0), axis=-1) * 0.1
    h = Hierarchy(shape)
    stream = oracle.decompose(u, h)
    pos, c = oracle.transform.finest_coefficients_at(u, h, np.arange(u.size))
    lo, hi = level_slices(h)[h.L]
    if h.L == 0:
        assert np.array_equal(pos, np.arange(u.size))
    else:
        assert np.array_equal(np.sort(pos), np.arange(lo, hi))   # every new node once
    scale = float(np.max(np.abs(u)))
    assert np.max(np.abs(stream[pos] - c)) <= 1e-13 * scale
