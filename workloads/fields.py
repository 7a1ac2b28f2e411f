"""Initial velocity fields. Arrays are (nz, ny, nx) with x fastest; vector
fields are (3, nz, ny, nx) with components (ux, uy, uz)."""
from __future__ import annotations

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
    per-component rms velocity is u_rms. Returns (rho=1, u)."""
    rng = np.random.default_rng(seed)
    kz = np.fft.fftfreq(n, 1.0 / n)
    ky = np.fft.fftfreq(n, 1.0 / n)
    kx = np.fft.rfftfreq(n, 1.0 / n)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    k2 = KX * KX + KY * KY + KZ * KZ
    kk = np.sqrt(k2)
    # shell spectrum E(k) ~ 4 pi k^2 |u_hat|^2 / 2  =>  |u_hat| ~ k exp(-(k/kp)^2)
    amp = kk * np.exp(-(kk / k_peak) ** 2)
    amp[0, 0, 0] = 0.0
    shape = KX.shape
    xi = [(rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) for _ in range(3)]
    # solenoidal projection (I - k k^T / k^2) xi
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    kdx = (KX * xi[0] + KY * xi[1] + KZ * xi[2]) * inv
    uh = [amp * (xi[0] - KX * kdx), amp * (xi[1] - KY * kdx), amp * (xi[2] - KZ * kdx)]
    del xi, kdx
    u = np.empty((3, n, n, n), dtype=dtype)
    for c in range(3):
        u[c] = np.fft.irfftn(uh[c], s=(n, n, n), axes=(0, 1, 2))
    u -= u.reshape(3, -1).mean(axis=1)[:, None, None, None]
    rms = np.sqrt((u.astype(np.float64) ** 2).mean() )
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
