"""Pins of the oracle's error control.

* worst case over every admissible quantisation error: for L-inf the exact
  maximum of |R delta| over the box |delta_j| <= q_j/2 is the weighted row sum
  of the dense recomposition matrix R; for L2 the maximum of ||R delta||_2 is
  found by brute force over all sign vectors (a convex function of delta peaks
  at a vertex of the box);
* the quantiser's rounding bound |c - k q| <= q/2 (1 + 2^-50) and the symbol /
  escape mapping at the dictionary edges;
* the per-axis transfer norm kappa = ||M_c^{-1} P^T M||_inf behind the L-inf
  bins: hand-derived on three nodes (3/2), the infinite uniform grid's closed
  form 1 + sqrt(3)/2 (derived below), the same operator assembled
  independently from quadrature of hat-function products and sampled coarse
  hats, and the diagonal-dominance bound kappa <= 3 on random spacings;
* the level-wise L-inf bins in closed form on 3 and 3x3 nodes, and the
  budget they spend (sum_l A_l q_l / 2 = tau') on larger grids;
* the end-to-end bound on reconstructed data for both norms and both types.
"""
import numpy as np
import pytest

import oracle
import synthetic
from oracle import Hierarchy
from oracle.operators import transfer_norm
from oracle.quantize import level_bins, to_symbols, from_symbols
from oracle.transform import level_slices


def _dense_R(h):
    return np.stack([oracle.recompose(e, h).ravel() for e in np.eye(h.N)], axis=1)


def _half_bins(h, q):
    w = np.empty(h.N)
    for l, (a, b) in enumerate(level_slices(h)):
        w[a:b] = q[l] / 2
    return w


@pytest.mark.parametrize("shape", [(9, 9, 9), (6, 6, 6), (9, 5, 4), (17, 12), (33,),
                                   (2, 2, 2), (3, 4, 5)])
def test_linf_worst_case_within_budget(shape):
    h = Hierarchy(shape)
    tau_eff = 1.0
    q = level_bins(h, tau_eff, "linf")
    R = _dense_R(h)
    worst = np.max(np.abs(R) @ _half_bins(h, q))
    assert worst <= tau_eff
    # exact transfer norms make the bound tight to within a small factor
    # (the slack left is that of bounding each level's term separately)
    assert worst > 0.3 * tau_eff


@pytest.mark.parametrize("shape", [(5, 4), (3, 3, 2), (17,), (3, 6)])
def test_l2_worst_case_within_budget(shape):
    h = Hierarchy(shape)
    assert h.N <= 20
    q = level_bins(h, 1.0, "l2")
    RD = _dense_R(h) * _half_bins(h, q)[None, :]
    G = RD.T @ RD
    best = 0.0
    n = h.N
    for start in range(0, 1 << n, 1 << 14):
        idx = np.arange(start, min(start + (1 << 14), 1 << n))
        S = 1.0 - 2.0 * ((idx[:, None] >> np.arange(n)[None, :]) & 1)
        best = max(best, float(np.max(np.einsum("ij,jk,ik->i", S, G, S))))
    assert np.sqrt(best) <= 1.0


def test_quantizer_rounding_bound():
    rng = np.random.default_rng(0)
    h = Hierarchy((33, 17))
    c = rng.standard_normal(h.N) * 10
    q = level_bins(h, 1e-3, "linf")
    k = oracle.quantize(c, h, q)
    back = oracle.dequantize(k, h, q)
    assert np.all(np.abs(c - back) <= _half_bins(h, q) * (1 + 2.0 ** -50))


def test_symbol_mapping_edges():
    k = np.array([0, 1, -1, 32767, -32767, 32768, -32768, 10 ** 12, -(10 ** 12)])
    sym, pos, vals = to_symbols(k)
    assert sym.tolist() == [32768, 32769, 32767, 65535, 1, 0, 0, 0, 0]
    assert pos.tolist() == [5, 6, 7, 8]
    assert vals.tolist() == [32768, -32768, 10 ** 12, -(10 ** 12)]
    assert np.array_equal(from_symbols(sym, pos, vals), k)


def test_linf_bins_closed_form():
    # q_l = 2 tau' sqrt(m_l) / (A_l S), S = sum_j sqrt(m_j), A_0 = 1,
    # A_l = 1 + prod_d kappa, kappa = 3/2 on three nodes.
    # 3 nodes: m = (2, 1), A_1 = 5/2, S = 1 + sqrt 2 ->
    # q = (4 - 2 sqrt 2, (4/5)(sqrt 2 - 1)); A_0 q_0 / 2 + A_1 q_1 / 2 = 1.
    r2, r5 = np.sqrt(2.0), np.sqrt(5.0)
    q = level_bins(Hierarchy((3,)), 1.0, "linf")
    assert abs(q[0] - (4.0 - 2.0 * r2)) <= 1e-15 and abs(q[1] - 0.8 * (r2 - 1.0)) <= 1e-15
    # 3x3: m = (4, 5), A_1 = 1 + 9/4 = 13/4, S = 2 + sqrt 5 ->
    # q = (4 (sqrt 5 - 2), (8/13)(5 - 2 sqrt 5))
    q = level_bins(Hierarchy((3, 3)), 1.0, "linf")
    assert abs(q[0] - 4.0 * (r5 - 2.0)) <= 1e-15
    assert abs(q[1] - 8.0 / 13.0 * (5.0 - 2.0 * r5)) <= 1e-15
    # the whole budget is spent: sum_l A_l q_l / 2 = tau'
    for shape in [(9, 9, 9), (17, 12), (33,), (6, 6, 6)]:
        h = Hierarchy(shape)
        from oracle.quantize import linf_amplification
        A = linf_amplification(h)
        q = level_bins(h, 1.0, "linf")
        assert abs(sum(a * b / 2 for a, b in zip(A, q)) - 1.0) <= 1e-14


# ---------------------------------------------------------- transfer norm
def test_transfer_norm_three_nodes_by_hand():
    # nodes 0, 1, 2 -> coarse 0, 2.  P^T M = [[5/12, 1/2, 1/12], [1/12, 1/2, 5/12]],
    # M_c = [[2/3, 1/3], [1/3, 2/3]], M_c^{-1} = [[2, -1], [-1, 2]], so
    # M_c^{-1} P^T M = [[3/4, 1/2, -1/4], [-1/4, 1/2, 3/4]]: row sums 3/2.
    assert transfer_norm(np.arange(3.0)) == 1.5


def test_transfer_norm_uniform_limit():
    # Infinite uniform grid: M_c = (1/3) tridiag(1, 4, 1) whose inverse has
    # entries 3 c (-r)^|k|, r = 2 - sqrt(3), c = 1/(2 sqrt 3).  The row of
    # M_c^{-1} P^T M at a coarse node has entries 3/2 t_k + [k=0]/4 at the
    # even fine nodes and 3/2 (t_k + t_{k-1}) at the odd ones (t_k = c(-r)^|k|),
    # whose absolute values sum to 1/4 + 9c/2 + 3 c r/(1 - r) = 1 + sqrt(3)/2.  Far from the ends a long axis attains it.
    limit = 1.0 + np.sqrt(3.0) / 2.0
    expect = np.ceil(limit * 2.0 ** 20) / 2.0 ** 20
    for n in (33, 65, 513, 300):
        assert transfer_norm(np.arange(float(n))) == expect


def _hat(xs, k, t):
    e = np.zeros(len(xs))
    e[k] = 1.0
    return np.interp(t, xs, e)


def _gram(xa, xb, xq):
    """Gram matrix of the hats on nodes xa against those on xb, by 2-point
    Gauss quadrature on every cell of the union grid xq (exact: products of
    two linear pieces)."""
    g = np.array([-1.0, 1.0]) / np.sqrt(3.0)
    G = np.zeros((len(xa), len(xb)))
    for lo, hi in zip(xq[:-1], xq[1:]):
        t = (lo + hi) / 2 + (hi - lo) / 2 * g
        fa = np.stack([_hat(xa, k, t) for k in range(len(xa))])
        fb = np.stack([_hat(xb, k, t) for k in range(len(xb))])
        G += (hi - lo) / 2 * fa @ fb.T
    return G


@pytest.mark.parametrize("x", [np.arange(9.0), np.arange(6.0), np.array([0.0, 1.0, 2.0, 4.0, 5.0, 8.0, 9.0]),
                               np.cumsum(np.r_[0.0, np.random.default_rng(3).uniform(0.2, 3.0, 10)])])
def test_transfer_norm_matches_quadrature_projection(x):
    # the L2 projection onto the coarse hats, built without P or M: the
    # coarse Gram matrix and the coarse-vs-fine Gram matrix by quadrature
    xc = x[oracle.hierarchy.coarse_positions(len(x))]
    Gc = _gram(xc, xc, x)
    Gcf = _gram(xc, x, x)
    X = np.linalg.solve(Gc, Gcf)
    kappa = float(np.max(np.sum(np.abs(X), axis=1)))
    assert abs(transfer_norm(x) - kappa) <= 2.0 ** -20
    assert transfer_norm(x) >= kappa


def test_transfer_norm_at_most_three():
    rng = np.random.default_rng(9)
    for _ in range(20):
        n = int(rng.integers(3, 40))
        x = np.cumsum(np.r_[0.0, rng.uniform(0.01, 5.0, n - 1)])
        assert 1.0 <= transfer_norm(x) <= 3.0


@pytest.mark.parametrize("norm", ["linf", "l2"])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(65, 65, 65), (30, 41, 12), (257,), (40, 33)])
def test_end_to_end_bound(norm, dtype, shape):
    u = synthetic.bumps(shape, 1, dtype=dtype) if len(shape) == 3 else \
        synthetic.grf(shape, 2, dtype=dtype)
    for rel in (1e-2, 1e-4):
        b = oracle.compress(u, rel, norm)
        v = oracle.decompress(b)
        assert v.dtype == u.dtype and v.shape == u.shape
        e = v.astype(np.float64) - u.astype(np.float64)
        x = u.astype(np.float64)
        if norm == "linf":
            assert np.max(np.abs(e)) <= rel * (x.max() - x.min())
        else:
            assert np.sqrt(np.sum(e * e)) <= rel * np.sqrt(np.sum(x * x))


def test_absolute_mode_bound():
    u = synthetic.grf((33, 33, 33), 4)
    b = oracle.compress(u, 0.05, "linf", "abs")
    assert np.max(np.abs(oracle.decompress(b).astype(np.float64) - u)) <= 0.05
