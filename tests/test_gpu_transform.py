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


def _leave_nan_in_lds(torch):
    """Runs library kernels of torch's that stage NaN doubles in LDS on every
    CU (a block scan and a row softmax over NaN inputs), so that the next
    kernels start with NaN bit patterns in whatever LDS they do not write."""
    torch.cumsum(torch.full((1 << 24,), float("nan"), dtype=torch.float64, device="cuda"), 0)
    torch.softmax(torch.full((4096, 4096), float("nan"), dtype=torch.float64, device="cuda"), 1)
    torch.cuda.synchronize()


@pytest.mark.parametrize("shape", [(30, 41, 12), (40, 33, 17), (300, 400, 500), (64, 64),
                                   (16, 21, 7), (66,), (9, 5, 4), (65, 65, 65)])
def test_results_do_not_depend_on_stale_lds(shape):
    """Every LDS value a kernel reads, also with a zero weight, must be one it
    wrote: decomposition, recomposition (raw coefficients and quantised
    symbols) and the adjoint give bit for bit the same results after kernels
    that leave NaN in LDS as without them, and (small grids) the oracle's.
    (Axes of even length end in two adjacent coarse nodes; a recomposition
    tile starting at the last of them once read a fine node no cell had
    written.)"""
    torch, mgc = gpu()
    u = synthetic.grf(shape, 13, dtype=np.float64)
    h = Hierarchy(shape)
    x = torch.from_numpy(u).cuda()
    g = torch.from_numpy(np.random.default_rng(3).standard_normal(shape)).cuda()
    scale = float(np.max(np.abs(u)))

    def run(poisoned):
        out = {}
        if poisoned:
            _leave_nan_in_lds(torch)
        out["c"] = mgc.decompose(x)
        if poisoned:
            _leave_nan_in_lds(torch)
        out["y"] = mgc.recompose(out["c"], shape, torch.float64)
        if poisoned:
            _leave_nan_in_lds(torch)
        blob = mgc.compress(x, 1e-4)
        out["blob"] = blob.clone()
        if poisoned:
            _leave_nan_in_lds(torch)
        out["v"] = mgc.decompress(blob)
        if poisoned:
            _leave_nan_in_lds(torch)
        out["ga"] = mgc.recompose_adjoint(g)
        torch.cuda.synchronize()
        return out

    clean, dirty = run(False), run(True)
    for k in clean:
        assert not bool(torch.isnan(dirty[k].double() if k != "blob" else dirty[k].double()).any()), k
        assert clean[k].shape == dirty[k].shape and bool(torch.equal(clean[k], dirty[k])), k
    assert torch.max(torch.abs(clean["y"] - x)).item() <= 1e-12 * scale
    tau = 1e-4 * (float(u.max()) - float(u.min()))
    assert torch.max(torch.abs(clean["v"] - x)).item() <= tau
    if h.N <= 300_000:
        ref = oracle.decompose(u, h)
        assert np.max(np.abs(clean["c"].cpu().numpy() - ref)) <= 1e-12 * scale
        gref = oracle.recompose_adjoint(g.cpu().numpy(), h)
        assert np.max(np.abs(clean["ga"].cpu().numpy() - gref)) <= \
            1e-12 * max(1.0, float(np.max(np.abs(gref))))


# The smallest levels of a hierarchy (fine grids up to 17^3) run in one
# workgroup with their grids in LDS; with per-level checkpoints requested,
# every level runs as its own launches instead.  Both forms take the same
# operations in the same order, so the outputs must agree bit for bit.
TAIL_SHAPES = [(17, 17, 17), (33, 33, 33), (65, 65, 65), (9, 5, 4), (30, 41, 12), (65, 129),
               (255,), (1, 7, 1), (2, 2, 2), (40, 33, 17)]


@pytest.mark.parametrize("shape", TAIL_SHAPES)
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_small_levels_in_one_workgroup_equal_per_level_launches(shape, dtype):
    torch, mgc = gpu()
    h = Hierarchy(shape)
    rng = np.random.default_rng(5)
    c = torch.from_numpy(rng.standard_normal(h.N)).cuda()
    dt = getattr(torch, dtype)
    one = mgc.recompose(c, shape, dt)
    per_level, _ = mgc.recompose_levels(c, shape, dt)
    assert torch.equal(one, per_level)
