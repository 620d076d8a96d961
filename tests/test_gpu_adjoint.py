"""Differentiation form: the GPU adjoint of recomposition.

* equals the FP64 oracle's transpose (oracle.recompose_adjoint) entry by entry;
* dot-product test <R x, y> = <x, R^T y> on the GPU;
* the 257^3 quantity-of-interest check: J(c) = mean over a random 64^3
  sub-box of u^2, u = R c.  J is quadratic in c, so central differences are
  exact for any step; the autograd gradient must match them (and the
  oracle's transpose of dJ/du) to 1e-5 relative;
* the per-level checkpoints of the forward pass equal the oracle's grids.
"""
import numpy as np
import pytest

import oracle
import synthetic
from oracle import Hierarchy
from tests.gpu_common import gpu

pytestmark = pytest.mark.gpu

SHAPES = [(65, 65, 65), (9, 5, 4), (17, 17, 17), (30, 41, 12), (33, 20), (17,), (2, 2, 2),
          (40, 33, 17), (5, 129), (1, 7, 1)]


@pytest.mark.parametrize("shape", SHAPES)
def test_adjoint_matches_oracle(shape):
    torch, mgc = gpu()
    rng = np.random.default_rng(3)
    y = rng.standard_normal(shape)
    ref = oracle.recompose_adjoint(y, Hierarchy(shape))
    got = mgc.recompose_adjoint(torch.from_numpy(y).cuda()).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, float(np.max(np.abs(ref))))


@pytest.mark.parametrize("shape", [(129, 129, 129), (300, 40, 50), (1025, 513)])
def test_dot_product_on_gpu(shape):
    torch, mgc = gpu()
    g = torch.Generator(device="cuda").manual_seed(7)
    N = int(np.prod(shape))
    x = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    y = torch.randn(shape, dtype=torch.float64, device="cuda", generator=g)
    lhs = torch.sum(mgc.recompose(x, shape) * y).item()
    rhs = torch.sum(x * mgc.recompose_adjoint(y)).item()
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0) * np.sqrt(N)


def test_qoi_gradient_257():
    torch, mgc = gpu()
    shape = (257, 257, 257)
    u0 = synthetic.grf(shape, 6)
    rng = np.random.default_rng(6)
    o = rng.integers(0, 194, size=3)
    box = tuple(slice(int(a), int(a) + 64) for a in o)
    c = mgc.decompose(torch.from_numpy(u0).cuda())
    c.requires_grad_(True)
    u = mgc.Recompose.apply(c, shape, True)
    J = torch.mean(u[box] ** 2)
    J.backward()
    grad = c.grad.detach()
    # the gradient equals R^T dJ/du computed by the oracle's transpose
    du = np.zeros(shape)
    ub = u.detach()[box].cpu().numpy()
    du[box] = 2.0 * ub / ub.size
    ref = oracle.recompose_adjoint(du, Hierarchy(shape))
    scale = float(np.max(np.abs(ref)))
    assert np.max(np.abs(grad.cpu().numpy() - ref)) <= 1e-5 * scale
    # central differences on 100 random coefficients (exact for quadratic J)
    idx = rng.choice(c.numel(), 100, replace=False)
    h = float(torch.max(torch.abs(c)).item())
    cd = c.detach()
    fd = []
    for i in idx:
        e = torch.zeros_like(cd)
        e[int(i)] = h
        jp = torch.mean(mgc.recompose(cd + e, shape)[box] ** 2).item()
        jm = torch.mean(mgc.recompose(cd - e, shape)[box] ** 2).item()
        fd.append((jp - jm) / (2 * h))
    fd = np.asarray(fd)
    g_i = grad[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert np.max(np.abs(fd - g_i)) <= 1e-5 * max(float(np.max(np.abs(g_i))), 1e-30)


@pytest.mark.parametrize("shape", [(65, 65, 65), (33, 20), (17,)])
def test_level_checkpoints_match_oracle(shape):
    torch, mgc = gpu()
    h = Hierarchy(shape)
    rng = np.random.default_rng(8)
    c = rng.standard_normal(h.N)
    ref_u, ref_levels = oracle.recompose(c, h, keep_levels=True)
    u, levels = mgc.recompose_levels(torch.from_numpy(c).cuda(), shape)
    assert np.max(np.abs(u.cpu().numpy() - ref_u)) <= 1e-12 * float(np.max(np.abs(ref_u)))
    flat = np.concatenate([np.asarray(g).ravel() for g in ref_levels[:-1]]) if h.L else np.zeros(0)
    got = levels.cpu().numpy()[: len(flat)]
    assert np.max(np.abs(got - flat), initial=0.0) <= 1e-12 * float(np.max(np.abs(flat), initial=1.0))
