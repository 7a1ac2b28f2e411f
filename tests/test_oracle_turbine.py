"""Pins of the oracle's turbine topology tree (Sec. 3.3, Alg. 1 and 2):
the tree form of a rotor reproduces the oracle's closed-form rotor, point
kinematics match closed forms and the finite-difference time derivative of
the positions, frames stay orthonormal, and the force models of towers and
disks give their closed forms in uniform flow; the spread force conserves
momentum."""
import numpy as np
import pytest

import workloads
from workloads import turbines as TB


def _small_rotor(hub=(20.0, 23.5, 24.0), R=8.0, omega_rot=0.02, **kw):
    rot = workloads.make_rotor(hub=hub, radius=R, n_blades=3, n_points=8,
                               tsr=omega_rot * R / 0.05, u_ref=0.05, **kw)
    return rot


def _uniform_grid(orc, n, U, omega=1.8, shape=None):
    nx, ny, nz = shape or (n, n, n)
    g = orc.Grid(nx, ny, nz, omega=omega)
    u = np.zeros((3, nz, ny, nx))
    for a in range(3):
        u[a] = U[a]
    g.init_fields(np.ones((nz, ny, nx)), u)
    return g


def _random_grid(orc, n, seed):
    rng = np.random.default_rng(seed)
    g = orc.Grid(n, n, n, omega=1.8)
    u = 0.05 * np.array([1.0, 0.0, 0.0])[:, None, None, None] + rng.normal(0, 0.01, (3, n, n, n))
    g.init_fields(1.0 + rng.normal(0, 0.002, (n, n, n)), u)
    return g


@pytest.mark.parametrize("kernel,tip", [("gauss", False), ("roma3", True)])
def test_tree_of_a_rotor_matches_the_closed_form_rotor(orc, kernel, tip):
    """Composed rotation matrices (tree) against the azimuth formula (rotor):
    same points, forces, spread field and flow after several steps."""
    rot = _small_rotor()
    rot["kernel"], rot["tip_loss"], rot["azimuth0"] = kernel, tip, 0.3
    a, b = _random_grid(orc, 40, 5), _random_grid(orc, 40, 5)
    a.set_rotor(0, rot)
    b.set_turbine(0, TB.rotor_tree(rot))
    for _ in range(3):
        a.step(1)
        b.step(1)
        _, pf = a.rotor_loads(0, with_points=True)
        nl, pts = b.turbine_loads(0)
        np.testing.assert_allclose(pts[:, 0:3], a.rotor_points(0), rtol=0, atol=1e-12)
        np.testing.assert_allclose(pts[:, 6:9], pf, rtol=0, atol=1e-12 * np.abs(pf).max())
    np.testing.assert_allclose(b.force(), a.force(), rtol=0, atol=1e-12 * np.abs(a.force()).max())
    np.testing.assert_allclose(b.get_pops(), a.get_pops(), rtol=0, atol=1e-13)
    # per-node loads: the blades' force sums, moments about the hub and power
    loads = a.rotor_loads(0)
    Fx = nl[1:, 0].sum()
    Mx = nl[1:, 3].sum()
    assert Fx == pytest.approx(loads[0], rel=1e-11)
    assert Mx == pytest.approx(loads[1], rel=1e-10)
    assert nl[1:, 6].sum() == pytest.approx(loads[2], rel=1e-10)


def test_vawt_points_follow_the_closed_form(orc):
    c = (30.0, 31.0, 32.0)
    vt = TB.vawt(c, radius=10.0, height=12.0, n_blades=3, n_points=4)
    om = vt["nodes"][0]["omega"]
    zs = vt["nodes"][1]["s"]
    for t in (0.0, 7.0, 123.0):
        x, v, _ = orc.turbine_kinematics(vt, t)
        for b in range(3):
            th = 2.0 * np.pi * b / 3 + om * t
            xe = np.stack([c[0] + 10.0 * np.cos(th) + 0 * zs, c[1] + 10.0 * np.sin(th) + 0 * zs,
                           c[2] - 6.0 + zs], 1)
            ve = np.tile([-om * 10.0 * np.sin(th), om * 10.0 * np.cos(th), 0.0], (len(zs), 1))
            np.testing.assert_allclose(x[4 * b:4 * b + 4], xe, atol=1e-12)
            np.testing.assert_allclose(v[4 * b:4 * b + 4], ve, atol=1e-15)
        # the shaft does not move
        np.testing.assert_allclose(v[12:], 0.0, atol=0)


def test_hawt_points_follow_the_closed_form(orc):
    rot = _small_rotor(hub=(30.0, 40.0, 44.0), R=10.0)
    tr = TB.hawt(rot, base_z=6.0, overhang=3.0, tower_spacing=4.0)
    nt = len(tr["nodes"][1]["s"])
    nn = len(tr["nodes"][3]["s"]) * tr["nodes"][3]["n_azimuth"]
    for t in (0.0, 11.0, 250.0):
        x, v, fr = orc.turbine_kinematics(tr, t)
        base = np.array([33.0, 40.0, 6.0])
        np.testing.assert_allclose(x[:nt], base + np.outer(tr["nodes"][1]["s"], [0, 0, 1]), atol=1e-12)
        hub = np.array(rot["hub"])
        np.testing.assert_allclose(fr[4, 9:12], hub, atol=1e-12)
        off = nt + nn
        for b in range(3):
            th = rot["omega_rot"] * t + 2.0 * np.pi * b / 3
            xe = hub + np.outer(rot["r"], [0, np.cos(th), np.sin(th)])
            ve = rot["omega_rot"] * np.outer(rot["r"], [0, -np.sin(th), np.cos(th)])
            np.testing.assert_allclose(x[off + 8 * b:off + 8 * b + 8], xe, atol=1e-12)
            np.testing.assert_allclose(v[off + 8 * b:off + 8 * b + 8], ve, atol=1e-14)


def test_point_velocity_is_the_time_derivative_of_position(orc):
    """Floating, yawing turbine (platform pitch and surge, nacelle yaw, hub
    spin): the velocities equal central differences of the positions."""
    rot = _small_rotor(hub=(40.0, 40.0, 50.0), R=10.0)
    tr = TB.hawt(rot, base_z=10.0, yaw_rate=0.003, pitch_amp=0.08, surge_amp=1.5,
                 wave_freq=2.0 * np.pi / 400.0)
    h = 1e-3
    for t in (3.0, 77.0, 301.5):
        _, v, _ = orc.turbine_kinematics(tr, t)
        xp, _, _ = orc.turbine_kinematics(tr, t + h)
        xm, _, _ = orc.turbine_kinematics(tr, t - h)
        fd = (xp - xm) / (2 * h)
        assert np.abs(fd - v).max() < 1e-8 * max(1.0, np.abs(v).max()) + 1e-9
        assert np.abs(v).max() > 0.1  # the blades do move


def test_frames_stay_orthonormal(orc):
    rot = _small_rotor(hub=(40.0, 40.0, 50.0), R=10.0)
    tr = TB.hawt(rot, base_z=10.0, yaw_rate=0.01, pitch_amp=0.3, wave_freq=0.05)
    for t in (0.0, 1234.5, 98765.0):
        _, _, fr = orc.turbine_kinematics(tr, t)
        for k in range(len(tr["nodes"])):
            T = fr[k, :9].reshape(3, 3)
            np.testing.assert_allclose(T @ T.T, np.eye(3), atol=1e-13)
            assert np.linalg.det(T) == pytest.approx(1.0, abs=1e-13)


def _tower(height=20.0, n=5, d=2.0, cd=1.1, base=(16.0, 16.0, 6.0)):
    return {"nodes": [{"parent": -1, "kind": "line", "force": "drag", "pos": base,
                       "dir": (0.0, 0.0, 1.0), "coef": cd,
                       "s": (np.arange(n) + 0.5) * height / n, "width": np.full(n, height / n),
                       "chord": np.full(n, d)}], "kernel": "gauss", "eps": 2.0}


def test_tower_drag_closed_form(orc):
    """Uniform cross flow: 1/2 rho C_D d l U^2 along the flow at every point;
    flow along the tower axis gives no force."""
    U = (0.04, -0.03, 0.0)
    g = _uniform_grid(orc, 32, U)
    g.set_turbine(0, _tower())
    g.step(1)
    nl, pts = g.turbine_loads(0)
    speed = np.hypot(U[0], U[1])
    Fe = 0.5 * 1.1 * 2.0 * 4.0 * speed * np.array(U)
    np.testing.assert_allclose(pts[:, 6:9], np.tile(Fe, (5, 1)), rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(nl[0, :3], 5 * Fe, rtol=1e-13)
    # along the axis: only the cross-flow part counts
    g = _uniform_grid(orc, 32, (0.0, 0.0, 0.05))
    g.set_turbine(0, _tower())
    g.step(1)
    _, pts = g.turbine_loads(0)
    assert np.abs(pts[:, 6:9]).max() < 1e-30  # round-off of the sampled cross flow only


def test_actuator_disk_thrust_closed_form(orc):
    """Uniform axial flow: total thrust 1/2 rho C_T' U^2 pi R^2 (the rings
    tile the disk), no side force, no moment about the centre, and the
    reaction on the fluid equals minus the thrust."""
    U = 0.05
    n = 40
    g = _uniform_grid(orc, n, (U, 0.0, 0.0))
    ad = TB.actuator_disk((20.0, 20.0, 20.0), radius=6.0, n_rings=4, n_azimuth=12, ct_prime=4.0 / 3.0)
    g.set_turbine(0, ad)
    g.step(1)
    nl, pts = g.turbine_loads(0)
    T = 0.5 * (4.0 / 3.0) * U * U * np.pi * 36.0
    assert nl[0, 0] == pytest.approx(T, rel=1e-13)
    assert abs(nl[0, 1]) < 1e-16 and abs(nl[0, 2]) < 1e-16
    assert np.abs(nl[0, 3:6]).max() < 1e-15
    assert nl[0, 6] == 0.0  # a fixed disk does no work
    Fsum = g.force().reshape(3, -1).sum(1)
    np.testing.assert_allclose(Fsum, -nl[0, :3], rtol=1e-12, atol=1e-17)


def test_frozen_tree_blade_matches_hand_formula(orc):
    """Omega = 0 blade line along +y in uniform axial flow U: W = U e_x,
    phi = 90 deg, alpha = 90 - twist, force = 1/2 rho U^2 c l (C_L e_L +
    C_D e_D) with e_L along +e_t = -z... in the blade's (e_n, e_t) plane."""
    rot = _small_rotor(hub=(16.0, 12.0, 16.0), R=8.0, omega_rot=0.0)
    tr = TB.rotor_tree(rot)
    tr["nodes"] = tr["nodes"][:2]  # hub + blade 0
    U = 0.05
    g = _uniform_grid(orc, 32, (U, 0.0, 0.0))
    g.set_turbine(0, tr)
    g.step(1)
    _, pts = g.turbine_loads(0)
    pol = workloads.synthetic_polars()
    for k in range(8):
        a = np.deg2rad(90.0 - rot["twist_deg"][k])
        CL = np.interp(np.rad2deg(a), pol["alpha_deg"], pol["cl"])
        CD = np.interp(np.rad2deg(a), pol["alpha_deg"], pol["cd"])
        q = 0.5 * U * U * rot["chord"][k] * rot["dl"][k]
        # W_n = U, W_t = 0: e_L = e_t, e_D = e_n; e_t = e_x x e_y = +z
        np.testing.assert_allclose(pts[k, 6:9], [q * CD, 0.0, q * CL], rtol=1e-12, atol=1e-18)


def test_turbine_momentum_budget(orc):
    """Tower, nacelle disk and turning blades together in a periodic box:
    the fluid momentum changes by minus the total force on the structure."""
    rot = _small_rotor(hub=(18.0, 20.0, 24.0), R=6.0)
    tr = TB.hawt(rot, base_z=8.0, tower_spacing=4.0)
    g = _random_grid(orc, 40, 9)
    g.set_turbine(3, tr)
    C27 = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)])
    for _ in range(2):
        P0 = np.einsum("ia,in->a", C27, g.get_pops().reshape(27, -1))
        g.step(1)
        P1 = np.einsum("ia,in->a", C27, g.get_pops().reshape(27, -1))
        nl, pts = g.turbine_loads(3)
        # round-off of the FP64 momentum sums over 27 x 64000 populations: ~1e-11
        np.testing.assert_allclose(P1 - P0, -pts[:, 6:9].sum(0), rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(nl[:, :3].sum(0), pts[:, 6:9].sum(0), rtol=1e-12, atol=1e-18)
