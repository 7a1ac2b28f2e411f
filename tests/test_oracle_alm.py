"""Pins of the oracle's actuator-line model: exactness of trilinear sampling
on affine fields, force conservation and centring of the spreading kernel,
hand-derived blade-element forces, rotor kinematics and the momentum budget
of a rotor in a periodic box."""
import json
import os

import numpy as np
import pytest

import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_trilinear_exact_on_affine_fields(orc):
    nx, ny, nz = 10, 8, 6
    g = orc.Grid(nx, ny, nz)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    field = np.stack([0.3 + 0.01 * x - 0.02 * y + 0.005 * z, 2.0 - 0.1 * x + 0.07 * z])
    rng = np.random.default_rng(0)
    for _ in range(20):
        p = rng.uniform([1, 1, 1], [nx - 2, ny - 2, nz - 2])
        got = g.trilinear(field, p)
        assert got[0] == pytest.approx(0.3 + 0.01 * p[0] - 0.02 * p[1] + 0.005 * p[2], abs=1e-14)
        assert got[1] == pytest.approx(2.0 - 0.1 * p[0] + 0.07 * p[2], abs=1e-14)


def test_spread_conserves_force_and_is_centred(orc):
    n = 32
    g = orc.Grid(n, n, n)
    rng = np.random.default_rng(1)
    for _ in range(5):
        xp = rng.uniform(10, 22, 3)
        Fp = rng.normal(0, 1, 3)
        F = g.spread_point(xp, Fp, 2.0)
        assert np.allclose(F.reshape(3, -1).sum(1), -Fp, rtol=1e-13, atol=1e-15)
        w = -F[0] / Fp[0]
        z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        cen = np.array([(w * x).sum(), (w * y).sum(), (w * z).sum()]) / w.sum()
        assert np.abs(cen - xp).max() < 5e-5
        # Gaussian shape: weight ratio of two support nodes
        c0 = np.floor(xp + 0.5).astype(int)
        a, b = c0, c0 + np.array([2, -1, 3])
        ra = np.sum((a - xp) ** 2)
        rb = np.sum((b - xp) ** 2)
        assert w[b[2], b[1], b[0]] / w[a[2], a[1], a[0]] == pytest.approx(
            np.exp(-(rb - ra) / 4.0), rel=1e-12)
        # nothing outside the 13^3 support
        assert np.count_nonzero(w) == 13 ** 3


def test_blade_element_hand_derived_cases(orc):
    """values derived by hand in golden/blade_element_cases.json"""
    with open(os.path.join(GOLD, "blade_element_cases.json")) as fh:
        cases = json.load(fh)["cases"]
    polar = workloads.synthetic_polars()
    for c in cases:
        fn, ft, al = orc.blade_element(c["rho"], c["wn"], c["wt"], c["chord"], c["dl"],
                                       c["twist_deg"], 0.0, polar)
        assert al == pytest.approx(c["alpha_deg"], abs=1e-12)
        assert fn == pytest.approx(c["Fn"], rel=2e-6)
        assert ft == pytest.approx(c["Ft"], rel=2e-6)


def _box_with_rotor(orc, n=48, R=8.0, omega_rot=0.02):
    rot = workloads.make_rotor(hub=(20.0, 23.5, 24.0), radius=R, n_blades=3,
                               n_points=8, tsr=omega_rot * R / 0.05, u_ref=0.05)
    g = orc.Grid(n, n, n, omega=1.8)
    u = np.zeros((3, n, n, n))
    u[0] = 0.05
    g.init_fields(np.ones((n, n, n)), u)
    g.set_rotor(0, rot)
    return g, rot


def test_rotor_kinematics_right_handed(orc):
    g, rot = _box_with_rotor(orc)
    g.step(1)
    pos = g.rotor_points(0)
    hub = np.array(rot["hub"])
    np.testing.assert_allclose(pos[: len(rot["r"])] - hub,
                               np.outer(rot["r"], [0, 1, 0]), atol=1e-14)
    g.step(1)  # second step: blade 0 turned by Omega towards +z
    th = rot["omega_rot"]
    pos = g.rotor_points(0)
    np.testing.assert_allclose(pos[: len(rot["r"])] - hub,
                               np.outer(rot["r"], [0, np.cos(th), np.sin(th)]), atol=1e-14)
    # blade 1 sits 120 degrees further
    th1 = th + 2 * np.pi / 3
    np.testing.assert_allclose(pos[len(rot["r"]): 2 * len(rot["r"])] - hub,
                               np.outer(rot["r"], [0, np.cos(th1), np.sin(th1)]), atol=1e-13)


def test_rotor_momentum_budget_and_loads(orc):
    """In a periodic box the fluid momentum changes each step by exactly the
    spread force, which is minus the total blade force; thrust and torque are
    the axial force sum and the r-weighted tangential force sum."""
    g, rot = _box_with_rotor(orc)
    C27 = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)])
    for _ in range(3):
        f0 = g.get_pops().reshape(27, -1)
        P0 = np.einsum("ia,in->a", C27, f0)
        g.step(1)
        f1 = g.get_pops().reshape(27, -1)
        P1 = np.einsum("ia,in->a", C27, f1)
        loads, pf = g.rotor_loads(0, with_points=True)
        np.testing.assert_allclose(P1 - P0, -pf.sum(0), rtol=1e-9, atol=1e-9)
        Fsum = g.force().reshape(3, -1).sum(1)
        np.testing.assert_allclose(Fsum, -pf.sum(0), rtol=1e-12, atol=1e-16)
        pos = g.rotor_points(0)
        hub = np.array(rot["hub"])
        rvec = pos - hub
        r = np.linalg.norm(rvec, axis=1)
        et = np.stack([np.zeros_like(r), -rvec[:, 2] / r, rvec[:, 1] / r], 1)
        assert loads[0] == pytest.approx(pf[:, 0].sum(), rel=1e-12)
        assert loads[1] == pytest.approx(np.sum(r * (pf * et).sum(1)), rel=1e-10)
        assert loads[2] == pytest.approx(loads[1] * rot["omega_rot"], rel=1e-12)
    # a turning rotor in axial wind produces positive thrust
    assert loads[0] > 0


# ---------------------------------------------------------------- Roma delta
def test_roma_phi_node_values(orc):
    """Values fixed by the closed form at the nodes and half-nodes, and the
    continuity of the two branches at |r| = 1/2."""
    assert orc.roma_phi(0.0) == pytest.approx(2.0 / 3.0, abs=1e-15)
    assert orc.roma_phi(1.0) == pytest.approx(1.0 / 6.0, abs=1e-15)
    assert orc.roma_phi(-1.0) == pytest.approx(1.0 / 6.0, abs=1e-15)
    assert orc.roma_phi(0.5) == pytest.approx(0.5, abs=1e-15)
    assert orc.roma_phi(0.5 + 1e-12) == pytest.approx(0.5, abs=1e-9)
    assert orc.roma_phi(1.5) == 0.0 and orc.roma_phi(-2.0) == 0.0
    assert orc.roma_phi(1.5 - 1e-9) == pytest.approx(0.0, abs=1e-8)


def test_roma_phi_defining_moment_conditions(orc):
    """Roma, Peskin and Berger define the 3-point delta by three conditions at
    every offset r: the shifts sum to one, their first moment vanishes and
    their squares sum to one half."""
    rng = np.random.default_rng(7)
    for r in np.concatenate([rng.uniform(0.0, 1.0, 50), [0.0, 0.25, 0.5, 0.75]]):
        w = np.array([orc.roma_phi(r - j) for j in range(-2, 4)])
        d = r - np.arange(-2, 4)
        assert w.sum() == pytest.approx(1.0, abs=1e-14)
        assert (d * w).sum() == pytest.approx(0.0, abs=1e-14)
        assert (w * w).sum() == pytest.approx(0.5, abs=1e-14)
        assert np.count_nonzero(w) <= 3


def test_roma_spread_conserves_force_and_centre(orc):
    n = 16
    g = orc.Grid(n, n, n)
    rng = np.random.default_rng(8)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    for _ in range(6):
        xp = rng.uniform(4, 12, 3)
        Fp = rng.normal(0, 1, 3)
        F = g.spread_point(xp, Fp, 0.0, kernel="roma3")
        assert np.allclose(F.reshape(3, -1).sum(1), -Fp, rtol=1e-14, atol=1e-15)
        w = -F[1] / Fp[1]
        # zero first moment per axis: the centre of the weights is the point
        cen = np.array([(w * x).sum(), (w * y).sum(), (w * z).sum()])
        assert np.abs(cen - xp).max() < 1e-12
        assert np.count_nonzero(w) == 27
        assert (w >= 0).all()


# ---------------------------------------------------------------- tip loss
def test_tip_loss_closed_forms(orc):
    """exp(-f) = 1/2 gives arccos(1/2) = pi/3, i.e. F = 2/3; exp(-f) = 1/sqrt(2)
    gives F = 1/2. With f = B (R - r) / (2 r |sin phi|) the radius R that
    makes f a chosen value is R = r + 2 r |sin phi| f / B."""
    B, r, phi = 3, 10.0, 0.3
    for f, F in [(np.log(2.0), 2.0 / 3.0), (0.5 * np.log(2.0), 0.5)]:
        R = r + 2.0 * r * abs(np.sin(phi)) * f / B
        assert orc.tip_loss(B, R, r, phi) == pytest.approx(F, abs=1e-14)
        assert orc.tip_loss(B, R, r, -phi) == pytest.approx(F, abs=1e-14)
    # zero at the tip, one far inboard, one for wind in the rotor plane
    assert orc.tip_loss(3, 20.0, 20.0, 0.3) == 0.0
    assert orc.tip_loss(3, 20.0, 0.5, 0.3) == pytest.approx(1.0, abs=1e-12)
    assert orc.tip_loss(3, 20.0, 15.0, 0.0) == 1.0
    # decreasing towards the tip; more blades, less loss
    rs = np.linspace(1.0, 19.9, 40)
    Fs = np.array([orc.tip_loss(3, 20.0, rr, 0.2) for rr in rs])
    assert (np.diff(Fs) <= 0).all()
    assert (np.diff(Fs[Fs < 1.0 - 1e-15]) < 0).all() and Fs[-1] < 0.5
    assert orc.tip_loss(5, 20.0, 18.0, 0.2) > orc.tip_loss(3, 20.0, 18.0, 0.2)


def test_tip_loss_and_roma_in_the_rotor_step(orc):
    """Same rotor and flow: with the tip-loss factor every point force is
    scaled by a factor in (0, 1], smallest at the outermost point; with the
    Roma delta the momentum budget of the box still closes exactly."""
    base = workloads.make_rotor(hub=(12.0, 15.5, 15.5), radius=8.0, n_blades=3, n_points=8,
                                tsr=6.0, u_ref=0.05)
    res = {}
    for name, extra in [("plain", {}), ("tip", {"tip_loss": True}), ("roma", {"kernel": "roma3"})]:
        rot = dict(base, **extra)
        g = orc.Grid(32, 32, 32, omega=1.8)
        rho = np.ones((32, 32, 32))
        u = np.zeros((3, 32, 32, 32))
        u[0] = 0.05
        g.init_fields(rho, u)
        g.set_rotor(0, rot)
        C27 = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)])
        f0 = g.get_pops().reshape(27, -1)
        g.step(1)
        f1 = g.get_pops().reshape(27, -1)
        res[name] = g.rotor_loads(0, with_points=True)
        dP = np.einsum("ia,in->a", C27, f1 - f0)
        np.testing.assert_allclose(dP, -res[name][1].sum(0), rtol=1e-9, atol=1e-12)
    # the first step samples the same initial field in every case
    ratio = np.linalg.norm(res["tip"][1], axis=1) / np.linalg.norm(res["plain"][1], axis=1)
    ratio = ratio.reshape(3, -1)
    assert (ratio > 0).all() and (ratio <= 1 + 1e-12).all()
    assert (np.diff(ratio, axis=1) < 0).all()
    assert res["tip"][0][0] < res["plain"][0][0]
    # the kernel does not change the first step's blade forces
    np.testing.assert_allclose(res["roma"][1], res["plain"][1], rtol=1e-12, atol=1e-18)
