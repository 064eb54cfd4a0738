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


def power_law_grf(shape=(256, 256, 256), slope=3.0, seed=2, workers=-1, dtype=np.float64):
    """Gaussian random field with power spectrum proportional to |k|^-slope.

    White N(0,1) noise is transformed with a real FFT, each mode is scaled by
    |k|^(-slope/2) using integer wavenumbers, the k = 0 mode is zeroed, and the
    inverse transform is normalised to zero mean and unit standard deviation.
    dtype is the synthesis precision: fp64 (default) or fp32 for very large
    fields (half the memory and time; the spectrum is scaled slab by slab).
    """
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    if dtype == np.float32:
        white = rng.standard_normal(shape, dtype=np.float32)
    else:
        white = rng.standard_normal(shape)
    spec = _rfftn(white, workers)
    del white
    nd = len(shape)
    ks = []
    for ax, n in enumerate(shape):
        k = (np.fft.rfftfreq(n) if ax == nd - 1 else np.fft.fftfreq(n)) * n
        ks.append(k * k)
    rdt = np.float32 if dtype == np.float32 else np.float64
    # |k|^2 of the trailing axes, then one slab of the leading axis at a time
    tail = np.zeros(spec.shape[1:], dtype=np.float64)
    for ax in range(1, nd):
        view = [1] * (nd - 1)
        view[ax - 1] = ks[ax].size
        tail += ks[ax].reshape(view)
    for i0 in range(spec.shape[0]):
        k2 = tail + ks[0][i0]
        with np.errstate(divide="ignore"):
            amp = np.where(k2 > 0, k2 ** (-slope / 4.0), 0.0).astype(rdt)
        spec[i0] *= amp
    del tail
    f = _irfftn(spec, shape, workers)
    del spec
    f -= f.mean(dtype=np.float64)
    sd = f.std(dtype=np.float64)
    if sd > 0:
        f /= f.dtype.type(sd)
    return np.ascontiguousarray(f.astype(np.float32))


def sharp_feature_field(shape=(512, 1024, 1024), seed=5, n_planes=25,
                        n_spheres=25, slope=3.0, workers=-1):
    """k^-slope background (fp32 synthesis) plus planar step discontinuities
    and spherical shocks.

    A planar step adds a * H(n . (p - c)) with a random unit normal n, a centre c
    uniform in the box and a = +-U(0.5, 2) (the background has unit standard
    deviation); a spherical shock adds a * H(rho - |p - c|) with
    rho = U(0.05, 0.3) * max(shape). Built slab by slab along axis 0 so the
    peak memory stays a small multiple of the field itself.
    """
    shape = tuple(int(s) for s in shape)
    assert len(shape) == 3
    f = power_law_grf(shape, slope=slope, seed=seed, workers=workers, dtype=np.float32)
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


def sharp_feature_field_device(shape=(512, 1024, 1024), seed=5, n_planes=25, n_spheres=25, slope=3.0,
                               device="cuda"):
    """The recipe of sharp_feature_field synthesised on a GPU with torch (for
    the 2 GiB configuration, where host synthesis takes minutes): the white
    noise comes from a seeded torch generator on the device, the spectrum is
    scaled by |k|^(-slope/2) with torch.fft, the result is normalised to zero
    mean and unit standard deviation, and the same planar steps and spherical
    shocks are added, their parameters drawn from the same numpy stream as the
    host version. Returns an fp32 device tensor (C order). Deterministic for a
    given seed, device and library build; the background differs from the
    host version's (another random stream), the recipe is the same.
    """
    import torch

    shape = tuple(int(s) for s in shape)
    assert len(shape) == 3
    nz, ny, nx = shape
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    white = torch.randn(shape, generator=gen, device=device, dtype=torch.float32)
    spec = torch.fft.rfftn(white)
    del white
    kz = torch.fft.fftfreq(nz, d=1.0 / nz, device=device, dtype=torch.float64) ** 2
    ky = torch.fft.fftfreq(ny, d=1.0 / ny, device=device, dtype=torch.float64) ** 2
    kx = torch.fft.rfftfreq(nx, d=1.0 / nx, device=device, dtype=torch.float64) ** 2
    tail = (ky[:, None] + kx[None, :])
    for i0 in range(nz):
        k2 = tail + kz[i0]
        amp = torch.where(k2 > 0, k2.clamp_min(1e-300) ** (-slope / 4.0), torch.zeros_like(k2))
        spec[i0] *= amp.to(torch.float32)
    f = torch.fft.irfftn(spec, s=shape)
    del spec
    mean = f.mean(dtype=torch.float64)
    sd = f.std(correction=0)
    f -= mean.to(torch.float32)
    if float(sd) > 0:
        f /= sd
    rng = np.random.default_rng([seed, 0x5EED])
    zc = torch.arange(nz, device=device, dtype=torch.float32)
    yc = torch.arange(ny, device=device, dtype=torch.float32)
    xc = torch.arange(nx, device=device, dtype=torch.float32)
    for _ in range(n_planes):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        c = rng.uniform(0.0, 1.0, 3) * np.array(shape, dtype=np.float64)
        a = float(np.float32(rng.choice([-1.0, 1.0]) * rng.uniform(0.5, 2.0)))
        t = ((float(n[0]) * (zc - float(c[0])))[:, None, None] + (float(n[1]) * (yc - float(c[1])))[None, :, None]
             + (float(n[2]) * (xc - float(c[2])))[None, None, :])
        f += a * (t > 0).to(torch.float32)
        del t
    L = max(shape)
    for _ in range(n_spheres):
        c = rng.uniform(0.0, 1.0, 3) * np.array(shape, dtype=np.float64)
        rho = rng.uniform(0.05, 0.3) * L
        a = float(np.float32(rng.choice([-1.0, 1.0]) * rng.uniform(0.5, 2.0)))
        lo = [max(0, int(np.floor(c[i] - rho))) for i in range(3)]
        hi = [min(shape[i], int(np.ceil(c[i] + rho)) + 1) for i in range(3)]
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        d2 = (((zc[lo[0]:hi[0]] - float(c[0])) ** 2)[:, None, None] + ((yc[lo[1]:hi[1]] - float(c[1])) ** 2)[None, :, None]
              + ((xc[lo[2]:hi[2]] - float(c[2])) ** 2)[None, None, :])
        f[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += a * (d2 < float(np.float32(rho * rho))).to(torch.float32)
        del d2
    return f.contiguous()


def power_law_grf_device(shape, slope=3.0, seed=0, device="cuda"):
    """Gaussian random field with power spectrum |k|^-slope of any dimension
    (1-3), synthesised on a GPU with torch: seeded white noise, rfftn, the
    spectrum scaled by |k|^(-slope/2) with integer wavenumbers (k = 0
    removed), irfftn, zero mean and unit standard deviation. fp32 device
    tensor, C order; the recipe of power_law_grf on another random stream."""
    import torch

    shape = tuple(int(s) for s in shape)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    spec = torch.fft.rfftn(torch.randn(shape, generator=gen, device=device, dtype=torch.float32))
    k2 = None
    for a, n in enumerate(shape):
        f = (torch.fft.rfftfreq(n, d=1.0 / n, device=device) if a == len(shape) - 1
             else torch.fft.fftfreq(n, d=1.0 / n, device=device)).to(torch.float32) ** 2
        view = [1] * len(shape)
        view[a] = f.numel()
        f = f.reshape(view)
        k2 = f if k2 is None else k2 + f
    amp = torch.where(k2 > 0, k2.clamp_min(1e-30) ** (-slope / 4.0), torch.zeros_like(k2))
    spec *= amp
    del amp, k2
    x = torch.fft.irfftn(spec, s=shape)
    del spec
    x -= x.mean()
    sd = x.std(correction=0)
    if float(sd) > 0:
        x /= sd
    return x.contiguous()


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
