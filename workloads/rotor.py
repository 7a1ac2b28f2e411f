"""Synthetic rotor geometry and airfoil polars (the paper's test rotor data
is not available; these are the stand-in rotors of the benchmark cases)."""
from __future__ import annotations

import numpy as np


def synthetic_polars(step_deg=0.1, clip_deg=12.0):
    """Tabulated polars on a uniform angle grid over [-180, 180] degrees:
    C_L = 2 pi alpha with alpha clipped at +-clip_deg, C_D = 0.01 + 0.02 alpha^2
    (alpha in radians, unclipped)."""
    n = int(round(360.0 / step_deg)) + 1
    a_deg = np.linspace(-180.0, 180.0, n)
    a = np.deg2rad(a_deg)
    ac = np.clip(a, -np.deg2rad(clip_deg), np.deg2rad(clip_deg))
    return {"alpha_deg": a_deg, "cl": 2.0 * np.pi * ac, "cd": 0.01 + 0.02 * a * a}


def make_rotor(hub, radius, n_blades, n_points, tsr, u_ref, eps=2.0,
               chord_root=0.25, chord_tip=0.10, twist_root_deg=20.0,
               azimuth0=0.0, pitch_deg=0.0, polar_step_deg=0.1):
    """Rigid rotor turning about +x. Elements are n_points equal segments of
    [0, R] with centres r_j = (j + 1/2) R / n_points; chord falls linearly
    from chord_root*R at the hub to chord_tip*R at the tip; twist falls
    linearly from twist_root_deg to 0; Omega = tsr * u_ref / R."""
    R = float(radius)
    r = (np.arange(n_points) + 0.5) * R / n_points
    s = r / R
    return {
        "hub": [float(h) for h in hub],
        "radius": R,
        "omega_rot": tsr * u_ref / R,
        "azimuth0": azimuth0,
        "eps": float(eps),
        "pitch_deg": pitch_deg,
        "n_blades": int(n_blades),
        "r": r,
        "chord": R * (chord_root + (chord_tip - chord_root) * s),
        "twist_deg": twist_root_deg * (1.0 - s),
        "dl": np.full(n_points, R / n_points),
        "polar": synthetic_polars(polar_step_deg),
    }


def single_turbine_rotor():
    """One 3-blade rotor of diameter 32 cells at x = 64, centred in y/z of a
    256 x 128 x 128 box, 32 points per blade, TSR 7 at u = 0.05, eps = 2."""
    return make_rotor(hub=(64.0, 63.5, 63.5), radius=16.0, n_blades=3,
                      n_points=32, tsr=7.0, u_ref=0.05, eps=2.0)


def turbine_row_rotors():
    """Three rotors of diameter 48 cells, 5D apart in x, hub height 128 above
    the ground wall, 3 blades x 48 points, TSR 7 at the hub wind 0.05."""
    return [make_rotor(hub=(x, 127.5, 127.5), radius=24.0, n_blades=3,
                       n_points=48, tsr=7.0, u_ref=0.05, eps=2.0)
            for x in (128.0, 368.0, 608.0)]


def turbine_row_inflow(ny=256, nz=256, u_hub=0.05, hub_height=128.0, alpha=0.14,
                       ti=0.05, seed=100, lt=256):
    """Sheared inlet u(z) = u_hub ((z + 1/2) / hub_height)^alpha (height above
    a ground wall at z = -1/2) plus a frozen random-phase turbulence box of
    per-component rms ti * u_hub (same spectrum recipe, given seed), laid out
    as box[3, lt, nz, ny] with lt the convected direction. Returns
    (mean[3, nz, ny], box)."""
    from .fields import random_phase_field
    z = np.arange(nz, dtype=np.float64)
    mean = np.zeros((3, nz, ny))
    mean[0] = (u_hub * ((z + 0.5) / hub_height) ** alpha)[:, None]
    n = max(lt, ny, nz)
    _, u = random_phase_field(n, seed=seed, u_rms=ti * u_hub)
    box = np.ascontiguousarray(u[:, :nz, :ny, :lt].transpose(0, 3, 1, 2))  # [3, x=lt, z, y]
    return mean, box
