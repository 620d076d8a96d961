"""Pins of the oracle's error control.

* worst case over every admissible quantisation error: for L-inf the exact
  maximum of |R delta| over the box |delta_j| <= q_j/2 is the weighted row sum
  of the dense recomposition matrix R; for L2 the maximum of ||R delta||_2 is
  found by brute force over all sign vectors (a convex function of delta peaks
  at a vertex of the box);
* the quantiser's rounding bound |c - k q| <= q/2 (1 + 2^-50) and the symbol /
  escape mapping at the dictionary edges;
* the end-to-end bound on reconstructed data for both norms and both types.
"""
import numpy as np
import pytest

import oracle
import synthetic
from oracle import Hierarchy
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
    # the bound is rigorous but not tight: record how loose (sanity, > 1%)
    assert worst > 0.01 * tau_eff


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
    assert np.all(np.abs(c - back) <= q[0] / 2 * (1 + 2.0 ** -50))


def test_symbol_mapping_edges():
    k = np.array([0, 1, -1, 32767, -32767, 32768, -32768, 10 ** 12, -(10 ** 12)])
    sym, pos, vals = to_symbols(k)
    assert sym.tolist() == [32768, 32769, 32767, 65535, 1, 0, 0, 0, 0]
    assert pos.tolist() == [5, 6, 7, 8]
    assert vals.tolist() == [32768, -32768, 10 ** 12, -(10 ** 12)]
    assert np.array_equal(from_symbols(sym, pos, vals), k)


def test_linf_bins_closed_form():
    # 3D, L = 6: q = 2 tau' / (1 + 6 * 28) = 2 tau' / 169 on every level
    h = Hierarchy((65, 65, 65))
    q = level_bins(h, 1.0, "linf")
    assert np.all(q == 2.0 / 169.0)


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
