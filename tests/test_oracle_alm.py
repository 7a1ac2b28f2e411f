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
