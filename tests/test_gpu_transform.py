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
