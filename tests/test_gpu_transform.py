"""GPU multilevel transform vs the FP64 oracle (coefficients, recomposition).

Arithmetic is FP64 on both sides (FP32 inputs are read exactly), so the
coefficients must agree to 1e-12 of max|u| per entry.
"""
import numpy as np
import pytest

import oracle
import synthetic
from oracle import Hierarchy
from tests.gpu_common import gpu

pytestmark = pytest.mark.gpu

SHAPES = [(65, 65, 65), (9, 5, 4), (6, 6, 6), (30, 41, 12), (33, 20), (17,), (1, 7, 1), (17, 17, 17),
          (2, 2, 2), (3, 5), (100, 3), (40, 33, 17), (257,), (5, 129)]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", SHAPES)
def test_decompose_matches_oracle(shape, dtype):
    torch, mgc = gpu()
    u = synthetic.grf(shape, 7, dtype=dtype) if np.prod(shape) > 1 else np.ones(shape, dtype)
    h = Hierarchy(shape)
    ref = oracle.decompose(u.astype(np.float64), h)
    got = mgc.decompose(torch.from_numpy(u).cuda()).cpu().numpy()
    scale = float(np.max(np.abs(u)))
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale


@pytest.mark.parametrize("shape", SHAPES)
def test_recompose_matches_oracle(shape):
    torch, mgc = gpu()
    h = Hierarchy(shape)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(h.N)
    ref = oracle.recompose(c, h)
    got = mgc.recompose(torch.from_numpy(c).cuda(), shape, torch.float64).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, float(np.max(np.abs(ref))))


@pytest.mark.parametrize("shape", [(129, 129, 129), (300, 40, 50)])
def test_roundtrip_on_gpu(shape):
    torch, mgc = gpu()
    u = synthetic.grf(shape, 9, dtype=np.float64)
    x = torch.from_numpy(u).cuda()
    back = mgc.recompose(mgc.decompose(x), shape, torch.float64)
    assert torch.max(torch.abs(back - x)).item() <= 1e-12 * float(np.max(np.abs(u)))


def test_decompose_513_sampled_finest_coefficients():
    torch, mgc = gpu()
    shape = (513, 513, 513)
    u = synthetic.grf(shape, 2)
    h = Hierarchy(shape)
    got = mgc.decompose(torch.from_numpy(u).cuda())
    idx = np.random.default_rng(0).choice(u.size, 3000, replace=False)
    pos, c = oracle.transform.finest_coefficients_at(u.astype(np.float64), h, idx)
    g = got[torch.from_numpy(pos).cuda()].cpu().numpy()
    assert np.max(np.abs(g - c)) <= 1e-12 * float(np.max(np.abs(u)))
    # exact inversion at full size
    back = mgc.recompose(got, shape, torch.float64)
    assert torch.max(torch.abs(back - torch.from_numpy(u).cuda().double())).item() <= \
        1e-11 * float(np.max(np.abs(u)))


@pytest.mark.parametrize("shape", [(65, 513, 1025), (300, 400, 500), (513, 513, 513)])
def test_partitioned_sweeps_match_serial_sweeps(shape):
    """Coarse grids above 2^22 points solve in partitioned sweeps (segments
    in registers, carries chained between segments); the serial sweeps
    (forced candidate 1) must give the same coefficients and recompositions
    up to rounding.  The shapes reach the strided-axis kernel with one to
    eight segments per line and the row kernel with 4 to 16 values per lane."""
    torch, mgc = gpu()
    u = synthetic.grf(shape, 11, dtype=np.float64)
    x = torch.from_numpy(u).cuda()
    del u
    scale = torch.max(torch.abs(x)).item()
    part = mgc.decompose(x)
    rec_part = mgc.recompose(part, shape, torch.float64)
    mgc.set_tuning("thomas_strided", 1)
    mgc.set_tuning("thomas_rows", 1)
    try:
        serial = mgc.decompose(x)
        rec_serial = mgc.recompose(part, shape, torch.float64)
    finally:
        mgc.set_tuning("thomas_strided", -1)
        mgc.set_tuning("thomas_rows", -1)
    d = torch.max(torch.abs(part - serial)).item()
    r = torch.max(torch.abs(rec_part - rec_serial)).item()
    print("%s: decompose %.3g, recompose %.3g of max|u|" % (shape, d / scale, r / scale))
    assert d <= 1e-13 * scale
    assert r <= 1e-13 * scale
    assert torch.max(torch.abs(rec_part - x)).item() <= 1e-12 * scale
