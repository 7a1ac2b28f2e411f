"""Synthetic turbine trees: components in a parent-child hierarchy (Sec. 3.3
of the waLBerla-wind paper), as plain dicts read by both the library binding
and the oracle. Geometry and operating points only; the stand-ins for the
configurations the paper's framework is built for (a horizontal-axis turbine
with tower and nacelle, a vertical-axis turbine, a floating horizontal-axis
turbine, an actuator disk), since the paper's turbine data are not available.

Node dict keys: parent, kind ("frame" | "line" | "disk"), force ("none" |
"blade" | "drag"), pos, rot (3x3), axis, omega, angle0, amp, freq, phase,
disp, dir, normal, coef, pitch_deg, tip_loss, n_azimuth, and the per-point
arrays s, width, chord, twist.
"""
from __future__ import annotations

import numpy as np

from .rotor import synthetic_polars


def rot_x(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _blades(parent, rotor, n_blades):
    """Blade lines of a rotor turning about the parent's +x: blade b is fixed
    at angle 2 pi b / B about x, spans +y, with the rotor axis +x as the
    blade-element normal."""
    out = []
    for b in range(n_blades):
        out.append({"parent": parent, "kind": "line", "force": "blade",
                    "rot": rot_x(2.0 * np.pi * b / n_blades),
                    "dir": (0.0, 1.0, 0.0), "normal": (1.0, 0.0, 0.0),
                    "pitch_deg": rotor.get("pitch_deg", 0.0),
                    "tip_loss": rotor.get("tip_loss", False),
                    "s": np.asarray(rotor["r"], dtype=np.float64),
                    "width": np.asarray(rotor["dl"], dtype=np.float64),
                    "chord": np.asarray(rotor["chord"], dtype=np.float64),
                    "twist": np.asarray(rotor["twist_deg"], dtype=np.float64)})
    return out


def rotor_tree(rotor):
    """The tree form of a workloads.rotor rotor: a hub frame at the hub
    turning about +x at omega_rot from azimuth0, with one blade line per
    blade. Same points, same forces."""
    hub = {"parent": -1, "kind": "frame", "pos": tuple(rotor["hub"]),
           "axis": (1.0, 0.0, 0.0), "omega": rotor["omega_rot"],
           "angle0": rotor.get("azimuth0", 0.0)}
    return {"nodes": [hub] + _blades(0, rotor, rotor["n_blades"]),
            "kernel": rotor.get("kernel", "gauss"), "eps": rotor["eps"],
            "n_blades": rotor["n_blades"], "radius": rotor["radius"],
            "polar": rotor["polar"]}


def hawt(rotor, base_z=8.0, overhang=3.0, tower_diameter=2.0, tower_spacing=2.0, cd_tower=1.0,
         nacelle_radius=2.0, nacelle_rings=2, nacelle_azimuth=8, cd_nacelle=0.8, yaw_rate=0.0,
         pitch_amp=0.0, surge_amp=0.0, wave_freq=0.0, kernel=None):
    """Horizontal-axis turbine: tower base (root) -> tower line (drag) and
    nacelle frame at the tower top (optionally yawing about +z) -> nacelle
    face (a drag disk at the hub) and hub (turning about +x) -> blades. The
    tower stands overhang cells downstream of the hub. pitch_amp / surge_amp
    with wave_freq make the root a floating platform: pitch about +y and
    surge along +x, both sinusoidal."""
    hub = np.asarray(rotor["hub"], dtype=np.float64)
    H = hub[2] - base_z
    nt = max(2, int(round(H / tower_spacing)))
    ts = (np.arange(nt) + 0.5) * H / nt
    rn = (np.arange(nacelle_rings) + 0.5) * nacelle_radius / nacelle_rings
    nodes = [
        {"parent": -1, "kind": "frame", "pos": (hub[0] + overhang, hub[1], base_z),
         "axis": (0.0, 1.0, 0.0), "amp": pitch_amp, "freq": wave_freq,
         "disp": (surge_amp, 0.0, 0.0)},
        {"parent": 0, "kind": "line", "force": "drag", "dir": (0.0, 0.0, 1.0), "coef": cd_tower,
         "s": ts, "width": np.full(nt, H / nt), "chord": np.full(nt, tower_diameter)},
        {"parent": 0, "kind": "frame", "pos": (0.0, 0.0, H), "axis": (0.0, 0.0, 1.0),
         "omega": yaw_rate},
        {"parent": 2, "kind": "disk", "force": "drag", "pos": (-overhang, 0.0, 0.0),
         "coef": cd_nacelle, "n_azimuth": nacelle_azimuth, "s": rn,
         "width": np.full(nacelle_rings, nacelle_radius / nacelle_rings)},
        {"parent": 2, "kind": "frame", "pos": (-overhang, 0.0, 0.0), "axis": (1.0, 0.0, 0.0),
         "omega": rotor["omega_rot"], "angle0": rotor.get("azimuth0", 0.0)},
    ]
    nodes += _blades(4, rotor, rotor["n_blades"])
    return {"nodes": nodes, "kernel": kernel or rotor.get("kernel", "gauss"), "eps": rotor["eps"],
            "n_blades": rotor["n_blades"], "radius": rotor["radius"], "polar": rotor["polar"]}


def vawt(center, radius=12.0, height=24.0, n_blades=3, n_points=16, tsr=3.0, u_ref=0.05,
         chord=2.0, twist_deg=0.0, eps=2.0, tower_diameter=1.5, cd_tower=1.0, kernel="gauss"):
    """Vertical-axis turbine: rotor frame at the rotor centre (root) turning
    about +z at Omega = tsr u_ref / radius, with straight blades parallel to
    the axis at the radius (spanning +z over the height, centred), and a
    static central shaft (a drag line). The blade-element normal points to the
    axis, so that the blade's motion direction is e_n x e_s = +e_theta."""
    cx, cy, cz = (float(v) for v in center)
    om = tsr * u_ref / radius
    zs = (np.arange(n_points) + 0.5) * height / n_points
    nodes = [{"parent": -1, "kind": "frame", "pos": (cx, cy, cz), "axis": (0.0, 0.0, 1.0),
              "omega": om}]
    for b in range(n_blades):
        beta = 2.0 * np.pi * b / n_blades
        nodes.append({"parent": 0, "kind": "line", "force": "blade",
                      "pos": (radius * np.cos(beta), radius * np.sin(beta), -0.5 * height),
                      "rot": rot_z(beta), "dir": (0.0, 0.0, 1.0), "normal": (-1.0, 0.0, 0.0),
                      "s": zs, "width": np.full(n_points, height / n_points),
                      "chord": np.full(n_points, chord), "twist": np.full(n_points, twist_deg)})
    ns = max(2, n_points // 2)
    nodes.append({"parent": -1, "kind": "line", "force": "drag",
                  "pos": (cx, cy, cz - 0.5 * height), "dir": (0.0, 0.0, 1.0), "coef": cd_tower,
                  "s": (np.arange(ns) + 0.5) * height / ns, "width": np.full(ns, height / ns),
                  "chord": np.full(ns, tower_diameter)})
    return {"nodes": nodes, "kernel": kernel, "eps": eps, "n_blades": n_blades,
            "radius": radius, "polar": synthetic_polars()}


def actuator_disk(center, radius=16.0, n_rings=8, n_azimuth=16, ct_prime=4.0 / 3.0, eps=2.0,
                  kernel="gauss"):
    """Non-rotating actuator disk facing +x: n_rings equal-width rings,
    thrust coefficient ct_prime on the local normal velocity (4/3 is
    C_T' for the Betz-optimal induction a = 1/4 in momentum theory)."""
    r = (np.arange(n_rings) + 0.5) * radius / n_rings
    return {"nodes": [{"parent": -1, "kind": "disk", "force": "drag",
                       "pos": tuple(float(c) for c in center), "coef": ct_prime,
                       "n_azimuth": n_azimuth, "s": r,
                       "width": np.full(n_rings, radius / n_rings)}],
            "kernel": kernel, "eps": eps, "n_blades": 0, "radius": radius}
