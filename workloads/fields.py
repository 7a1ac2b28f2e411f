"""Initial velocity fields. Arrays are (nz, ny, nx) with x fastest; vector
fields are (3, nz, ny, nx) with components (ux, uy, uz)."""
from __future__ import annotations

import os

import numpy as np


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64),
                          np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def tgv_field(nx, ny, nz, u0=0.05, k=None):
    """3-D Taylor-Green vortex: u = u0 sin kx cos ky cos kz,
    v = -u0 cos kx sin ky cos kz, w = 0, uniform density 1."""
    if k is None:
        k = 2.0 * np.pi / nx
    x, y, z = _grid(nx, ny, nz)
    u = np.zeros((3, nz, ny, nx))
    u[0] = u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    u[1] = -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    return np.ones((nz, ny, nx)), u


def shear_wave_field(nx, ny, nz, u0=1e-3, m=1):
    """Decaying shear wave u_x = u0 sin(2 pi m y / ny)."""
    x, y, z = _grid(nx, ny, nz)
    u = np.zeros((3, nz, ny, nx))
    u[0] = u0 * np.sin(2.0 * np.pi * m * y / ny)
    return np.ones((nz, ny, nx)), u


def random_phase_field(n, seed=0, k_peak=8.0, u_rms=0.03, dtype=np.float64):
    """Divergence-free random-phase field on a periodic n^3 box with shell
    spectrum E(k) ~ k^4 exp(-2 (k/k_peak)^2), scaled so that the
    per-component rms velocity is u_rms. Returns (rho=1, u).

    Recipe: on the half-spectrum (rfft layout, x last) draw a complex
    Gaussian vector xi per wavenumber from default_rng(seed) (float32
    normals: real parts of x, y, z, then imaginary parts), project it onto
    the plane normal to k, scale by |k| exp(-(|k|/k_peak)^2), inverse-FFT."""
    import scipy.fft as sfft

    rng = np.random.default_rng(seed)
    kz = np.fft.fftfreq(n, 1.0 / n).astype(np.float32)[:, None, None]
    ky = np.fft.fftfreq(n, 1.0 / n).astype(np.float32)[None, :, None]
    kx = np.fft.rfftfreq(n, 1.0 / n).astype(np.float32)[None, None, :]
    shape = (n, n, n // 2 + 1)
    k2 = kx * kx + ky * ky + kz * kz
    kk = np.sqrt(k2)
    amp = kk * np.exp(-(kk / np.float32(k_peak)) ** 2)
    amp[0, 0, 0] = 0.0
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0).astype(np.float32)
    del kk
    xi = np.empty((3,) + shape, dtype=np.complex64)
    for c in range(3):
        xi[c].real = rng.standard_normal(shape, dtype=np.float32)
    for c in range(3):
        xi[c].imag = rng.standard_normal(shape, dtype=np.float32)
    kdx = xi[0] * kx
    kdx += xi[1] * ky
    kdx += xi[2] * kz
    kdx *= inv
    del inv
    for c, kc in enumerate((kx, ky, kz)):
        xi[c] -= kc * kdx
        xi[c] *= amp
    del kdx, amp, k2
    workers = os.cpu_count() or 1
    u = np.empty((3, n, n, n), dtype=dtype)
    for c in range(3):
        u[c] = sfft.irfftn(xi[c], s=(n, n, n), axes=(0, 1, 2), workers=workers)
    del xi
    for c in range(3):
        u[c] -= u[c].mean()
    rms = np.sqrt(sum(float(np.mean(np.square(u[c], dtype=np.float64))) for c in range(3)) / 3.0)
    u *= u_rms / rms
    return np.ones((n, n, n), dtype=dtype), u


def shell_spectrum(u):
    """Shell-summed energy spectrum E(k), k = 0..n/2, of a periodic cube."""
    n = u.shape[-1]
    uh = np.fft.fftn(u, axes=(1, 2, 3)) / n ** 3
    e = 0.5 * (np.abs(uh) ** 2).sum(axis=0)
    k = np.fft.fftfreq(n, 1.0 / n)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    kk = np.rint(np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)).astype(int)
    E = np.bincount(kk.ravel(), weights=e.ravel())
    return E[: n // 2 + 1]
