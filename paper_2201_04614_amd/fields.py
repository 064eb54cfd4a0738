"""Seeded synthetic fp32 fields.

These generators are the only code shared by the CPU oracle's tests and the
HIP path's tests and benchmark. They hold none of the compression method's
arithmetic: they only produce input arrays (numpy fp64 synthesis, cast to fp32,
C order, slowest axis first).

The workloads stand in for the SDRBench fields of Table II (HACC, CESM-ATM,
Hurricane, NYX, QMCPACK), which are not available here. The paper evaluates
smooth, multi-scale simulation output; the stand-ins are smooth spectral
fields (sums of sinusoids, power-law Gaussian random fields) with optional
sharp features (planar steps, spherical shocks) and an optional constant
offset (a field with few near-zero values, the case Section IV singles out as
the one where zero padding produces border outliers).
"""

from __future__ import annotations

import numpy as np

try:  # scipy's pocketfft is multi-threaded; numpy's is not
    import scipy.fft as _sfft
except Exception:  # pragma: no cover - scipy is present in this image
    _sfft = None


def _rfftn(a, workers):
    if _sfft is not None:
        return _sfft.rfftn(a, workers=workers)
    return np.fft.rfftn(a)


def _irfftn(a, shape, workers):
    if _sfft is not None:
        return _sfft.irfftn(a, s=shape, workers=workers)
    return np.fft.irfftn(a, s=shape)


def sinusoid_field(shape=(512, 512), n_waves=8, seed=1, noise=1e-3):
    """Sum of ``n_waves`` random plane sinusoids plus white noise.

    Wave s has integer wavenumbers k_a in [1, 16] with a random sign per axis,
    amplitude U(0.1, 1) and phase U(0, 2*pi); the noise is N(0, noise).
    """
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) / n for n in shape],
                        indexing="ij", sparse=True)
    f = np.zeros(shape, dtype=np.float64)
    for _ in range(n_waves):
        k = [int(rng.integers(1, 17)) * int(rng.choice([-1, 1])) for _ in shape]
        amp = rng.uniform(0.1, 1.0)
        phase = rng.uniform(0.0, 2.0 * np.pi)
        arg = sum(ki * g for ki, g in zip(k, grids))
        f += amp * np.sin(2.0 * np.pi * arg + phase)
    if noise:
        f += rng.normal(0.0, noise, size=shape)
    return np.ascontiguousarray(f.astype(np.float32))


def power_law_grf(shape=(256, 256, 256), slope=3.0, seed=2, workers=-1):
    """Gaussian random field with power spectrum proportional to |k|^-slope.

    White N(0,1) noise is transformed with a real FFT, each mode is scaled by
    |k|^(-slope/2) using integer wavenumbers, the k = 0 mode is zeroed, and the
    inverse transform is normalised to zero mean and unit standard deviation.
    """
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    spec = _rfftn(white, workers)
    del white
    k2 = np.zeros(spec.shape, dtype=np.float64)
    nd = len(shape)
    for ax, n in enumerate(shape):
        if ax == nd - 1:
            k = np.fft.rfftfreq(n) * n
        else:
            k = np.fft.fftfreq(n) * n
        view = [1] * nd
        view[ax] = k.size
        k2 += (k * k).reshape(view)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (-slope / 4.0), 0.0)
    spec *= amp
    del amp, k2
    f = _irfftn(spec, shape, workers)
    del spec
    f -= f.mean()
    sd = f.std()
    if sd > 0:
        f /= sd
    return np.ascontiguousarray(f.astype(np.float32))


def sharp_feature_field(shape=(512, 1024, 1024), seed=5, n_planes=25,
                        n_spheres=25, slope=3.0, workers=-1):
    """k^-slope background plus planar step discontinuities and spherical shocks.

    A planar step adds a * H(n . (p - c)) with a random unit normal n, a centre c
    uniform in the box and a = +-U(0.5, 2) (the background has unit standard
    deviation); a spherical shock adds a * H(rho - |p - c|) with
    rho = U(0.05, 0.3) * max(shape). Built slab by slab along axis 0 so the
    peak memory stays a small multiple of the field itself.
    """
    shape = tuple(int(s) for s in shape)
    assert len(shape) == 3
    f = power_law_grf(shape, slope=slope, seed=seed, workers=workers)
    rng = np.random.default_rng([seed, 0x5EED])
    nz, ny, nx = shape
    zc = np.arange(nz, dtype=np.float32)
    yc = np.arange(ny, dtype=np.float32)
    xc = np.arange(nx, dtype=np.float32)
    slab = max(1, (1 << 24) // (ny * nx))
    for _ in range(n_planes):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        c = rng.uniform(0.0, 1.0, 3) * np.array(shape, dtype=np.float64)
        a = np.float32(rng.choice([-1.0, 1.0]) * rng.uniform(0.5, 2.0))
        ty = (n[1] * (yc - c[1])).astype(np.float32)[:, None]
        tx = (n[2] * (xc - c[2])).astype(np.float32)[None, :]
        tyx = ty + tx
        for z0 in range(0, nz, slab):
            z1 = min(nz, z0 + slab)
            tz = (n[0] * (zc[z0:z1] - c[0])).astype(np.float32)[:, None, None]
            f[z0:z1] += a * ((tz + tyx[None]) > 0)
    L = max(shape)
    for _ in range(n_spheres):
        c = rng.uniform(0.0, 1.0, 3) * np.array(shape, dtype=np.float64)
        rho = rng.uniform(0.05, 0.3) * L
        a = np.float32(rng.choice([-1.0, 1.0]) * rng.uniform(0.5, 2.0))
        lo = [max(0, int(np.floor(c[i] - rho))) for i in range(3)]
        hi = [min(shape[i], int(np.ceil(c[i] + rho)) + 1) for i in range(3)]
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        dy2 = ((yc[lo[1]:hi[1]] - c[1]) ** 2)[:, None]
        dx2 = ((xc[lo[2]:hi[2]] - c[2]) ** 2)[None, :]
        dyx2 = (dy2 + dx2).astype(np.float32)
        for z0 in range(lo[0], hi[0], slab):
            z1 = min(hi[0], z0 + slab)
            dz2 = ((zc[z0:z1] - c[0]) ** 2)[:, None, None]
            inside = (dz2 + dyx2[None]) < np.float32(rho * rho)
            f[z0:z1, lo[1]:hi[1], lo[2]:hi[2]] += a * inside
    return f


def field_range(x):
    """max - min of a field, in fp64 (used to state eb = c * range)."""
    return float(np.float64(x.max()) - np.float64(x.min()))


# ---------------------------------------------------------------- test fields


def uniform_field(shape, seed, lo=-1.0, hi=1.0):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(lo, hi, size=tuple(shape)).astype(np.float32))


def integer_field(shape, seed, amp):
    """Random integers in [-amp, amp] stored as fp32 (exact below 2^24)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(
        rng.integers(-amp, amp + 1, size=tuple(shape)).astype(np.float32))


def affine_integer_field(shape, offset, slopes):
    """x[u] = offset + sum_a slopes[a] * u_a, an exactly representable integer grid."""
    shape = tuple(int(s) for s in shape)
    f = np.full(shape, float(offset), dtype=np.float64)
    for ax, (n, s) in enumerate(zip(shape, slopes)):
        view = [1] * len(shape)
        view[ax] = n
        f = f + s * np.arange(n, dtype=np.float64).reshape(view)
    assert np.abs(f).max() < 2 ** 24
    return np.ascontiguousarray(f.astype(np.float32))


def constant_field(shape, value):
    return np.full(tuple(shape), np.float32(value), dtype=np.float32)
