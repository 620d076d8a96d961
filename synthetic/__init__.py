"""Seeded synthetic scientific fields.

This module is the only code shared by the CPU oracle, the GPU tests and the
benchmark.  It draws random numbers and shapes signals; it holds none of the
compressor's arithmetic.  The paper evaluates on NYX (512^3 FP32), XGC (4D
FP64) and E3SM (2880x240x960 FP32) fields (Section VI-A, "Datasets" table);
those files are not available, so these generators stand in for their shapes:

* ``bumps``      a sum of Gaussian bumps plus white noise (smooth field);
* ``grf``        an isotropic Gaussian random field with power ~ |k|^-3;
* ``sinusoids``  a 2D sum of plane waves with amplitudes decaying as 1/k;
* ``zipf_bytes`` / ``laplace_ints``  byte and integer streams for the
  standalone Huffman codec: Zipf-like bytes, and Laplacian integers around
  zero (the shape of quantised multilevel coefficients) with a fraction of
  arbitrary values.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and draws its
random numbers in the order stated in its docstring, so the same seed gives
the same field on every machine running the same NumPy.
"""
from __future__ import annotations

import numpy as np

__all__ = ["bumps", "grf", "sinusoids", "batch_specs", "field_from_spec", "zipf_bytes",
           "laplace_ints"]


def _axis_coords(n: int) -> np.ndarray:
    # unit-box coordinates x_i = i / (n - 1) (a single node sits at 0)
    if n == 1:
        return np.zeros(1)
    return np.arange(n, dtype=np.float64) / (n - 1)


def bumps(shape, seed: int, n_bumps: int = 8, noise: float = 1e-3,
          dtype=np.float32) -> np.ndarray:
    """Sum of ``n_bumps`` isotropic Gaussian bumps plus N(0, noise^2) noise.

    Draw order: centres U[0,1]^(n_bumps x ndim), widths U(0.05, 0.2),
    amplitudes N(0, 1), then the noise field.  Each bump is separable, so it is
    evaluated as an outer product of per-axis factors.
    """
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    nd = len(shape)
    centres = rng.uniform(0.0, 1.0, size=(n_bumps, nd))
    widths = rng.uniform(0.05, 0.2, size=n_bumps)
    amps = rng.normal(0.0, 1.0, size=n_bumps)
    axes = [_axis_coords(n) for n in shape]
    u = np.zeros(shape, dtype=np.float64)
    for b in range(n_bumps):
        term = np.array(amps[b], dtype=np.float64)
        for d in range(nd):
            f = np.exp(-((axes[d] - centres[b, d]) ** 2) / (2.0 * widths[b] ** 2))
            term = np.multiply.outer(term, f)
        u += term
    u += rng.normal(0.0, noise, size=shape)
    return u.astype(dtype)


def grf(shape, seed: int, slope: float = -3.0, dtype=np.float32) -> np.ndarray:
    """Gaussian random field with isotropic power spectrum ~ |k|^slope.

    Draw order: one white N(0,1) field of ``shape``.  It is transformed with a
    real FFT, multiplied by |k|^(slope/2) with k the integer frequency index
    (the k = 0 mode set to zero), transformed back, then shifted to zero mean
    and scaled to unit standard deviation.
    """
    import scipy.fft as sfft

    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(size=shape)
    spec = sfft.rfftn(white, workers=-1)
    del white
    k2 = np.zeros(spec.shape, dtype=np.float64)
    nd = len(shape)
    for d, n in enumerate(shape):
        if d == nd - 1:
            kd = np.arange(spec.shape[d], dtype=np.float64)
        else:
            kd = np.fft.fftfreq(n, d=1.0 / n)
        sh = [1] * nd
        sh[d] = -1
        k2 = k2 + (kd.reshape(sh) ** 2)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)
    del k2
    spec *= amp
    del amp
    u = sfft.irfftn(spec, s=shape, workers=-1)
    del spec
    u -= u.mean()
    sd = u.std()
    if sd > 0:
        u /= sd
    return u.astype(dtype)


def sinusoids(shape, seed: int, n_waves: int = 64, kmax: int = 200,
              dtype=np.float64) -> np.ndarray:
    """2D sum of ``n_waves`` plane waves (1/k) sin(2 pi k (cos t x + sin t y) + phi).

    Draw order: wavenumbers k ~ U{1..kmax}, directions t ~ U[0, 2 pi), phases
    phi ~ U[0, 2 pi).  Coordinates are the unit box.  Each wave is evaluated
    separably with sin(a + b) = sin a cos b + cos a sin b.
    """
    ny, nx = (int(s) for s in shape)
    rng = np.random.default_rng(seed)
    ks = rng.integers(1, kmax + 1, size=n_waves)
    th = rng.uniform(0.0, 2 * np.pi, size=n_waves)
    ph = rng.uniform(0.0, 2 * np.pi, size=n_waves)
    y = _axis_coords(ny)
    x = _axis_coords(nx)
    a = 2 * np.pi * ks[None, :] * np.cos(th)[None, :] * y[:, None] + ph[None, :]
    b = 2 * np.pi * ks[None, :] * np.sin(th)[None, :] * x[:, None]
    amp = 1.0 / ks
    # sum_m amp_m (sin a_m cos b_m + cos a_m sin b_m) as one matrix product
    left = np.concatenate([np.sin(a) * amp, np.cos(a) * amp], axis=1)
    right = np.concatenate([np.cos(b), np.sin(b)], axis=1)
    return (left @ right.T).astype(dtype)


def batch_specs(n_arrays: int = 256, seed: int = 5,
                sizes=(33, 65, 129, 257), bounds=(1e-2, 1e-3, 1e-4)):
    """Shapes, field kinds, bounds and sub-seeds for a batch of uneven arrays.

    Draw order per array i (one generator seeded with ``seed``): three axis
    lengths from ``sizes``, then one bound from ``bounds``.  Even i is a bump
    field, odd i a |k|^-3 random field; array i uses sub-seed 1000*seed + i.
    """
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_arrays):
        shp = tuple(int(sizes[j]) for j in rng.integers(0, len(sizes), size=3))
        eb = float(bounds[int(rng.integers(0, len(bounds)))])
        specs.append({"shape": shp, "kind": "bumps" if i % 2 == 0 else "grf",
                      "bound": eb, "seed": 1000 * seed + i})
    return specs


def field_from_spec(spec, dtype=np.float32) -> np.ndarray:
    if spec["kind"] == "bumps":
        return bumps(spec["shape"], spec["seed"], dtype=dtype)
    return grf(spec["shape"], spec["seed"], dtype=dtype)


def zipf_bytes(n: int, seed: int, s: float = 1.2) -> np.ndarray:
    """n bytes with P(b) proportional to (b + 1)^-s.  Draws n 16-bit uniform
    integers and maps each through the inverse CDF sampled at 65536 points."""
    p = 1.0 / np.arange(1, 257, dtype=np.float64) ** s
    cdf = np.cumsum(p) / p.sum()
    table = np.minimum(np.searchsorted(cdf, (np.arange(65536) + 0.5) / 65536), 255).astype(np.uint8)
    rng = np.random.default_rng(seed)
    return table[rng.integers(0, 65536, size=n, dtype=np.uint16)]


def laplace_ints(n: int, seed: int, dtype=np.int32, scale: float = 8.0,
                 wild: float = 1e-3) -> np.ndarray:
    """n integers: Laplace(0, scale) rounded to the nearest integer, then a
    fraction ``wild`` of positions (uniform draws below wild) replaced by
    uniform values over the whole type.  Draw order: the n Laplace variates,
    the n selection uniforms, then the replacement values."""
    rng = np.random.default_rng(seed)
    info = np.iinfo(dtype)
    v = np.round(rng.laplace(0.0, scale, size=n)).astype(dtype)
    m = rng.random(n) < wild
    v[m] = rng.integers(info.min, info.max, size=int(m.sum()), dtype=dtype, endpoint=True)
    return v
