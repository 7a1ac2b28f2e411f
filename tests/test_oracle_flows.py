"""Pins of the oracle's streaming, boundaries and whole-domain behaviour
against exact flow solutions, fixed points and conservation laws."""
import numpy as np
import pytest

import workloads


def nu_of(om):
    return (1.0 / om - 0.5) / 3.0


@pytest.mark.parametrize("om", [1.0, 1.9])
def test_shear_wave_decays_at_lattice_viscosity(orc, om):
    """u_x = u0 sin(k y) is an exact Navier-Stokes solution decaying as
    exp(-nu k^2 t) with nu = (1/omega - 1/2)/3."""
    ny = 64
    g = orc.Grid(4, ny, 4, omega=om)
    g.init_fields(*workloads.shear_wave_field(4, ny, 4, 1e-3))
    s = np.sin(2 * np.pi * np.arange(ny) / ny)[None, :, None]
    amp = []
    for _ in range(200):
        g.step(1)
        amp.append(np.sum(g.fields()[1][0] * s))
    t = np.arange(1, 201)
    slope = np.polyfit(t[20:], np.log(np.abs(amp[20:])), 1)[0]
    k = 2 * np.pi / ny
    assert -slope / (k * k) == pytest.approx(nu_of(om), rel=5e-3)


def test_tgv_energy_mass_momentum(orc):
    """Taylor-Green vortex on 64^3: E(0) = N u0^2 / 8 exactly, energy decay at
    the lattice viscosity (rate 6 nu k^2 in the linear limit; 3 % band at
    u0 = 0.05), exact mass and momentum conservation."""
    n, u0 = 64, 0.05
    g = orc.Grid(n, n, n, omega=1.9)
    g.init_fields(*workloads.tgv_field(n, n, n, u0))
    m0, p0, e0 = g.global_moments()
    assert e0 == pytest.approx(n ** 3 * u0 ** 2 / 8, rel=1e-12)
    E = [e0]
    for _ in range(50):
        g.step(1)
        m, p, e = g.global_moments()
        E.append(e)
        assert abs(m - m0) <= 1e-13 * m0
        assert np.abs(p).max() <= 1e-10 * n ** 3 * u0
    t = np.arange(51)
    k = 2 * np.pi / n
    slope = np.polyfit(t[10:], np.log(E[10:]), 1)[0]
    assert -slope / (6 * k * k) == pytest.approx(nu_of(1.9), rel=0.03)


def test_tgv_linear_regime(orc):
    """u0 = 1e-3: fit after the (1 - omega)^t non-hydrodynamic transient"""
    n, u0 = 32, 1e-3
    g = orc.Grid(n, n, n, omega=1.9)
    g.init_fields(*workloads.tgv_field(n, n, n, u0))
    E = [g.global_moments()[2]]
    for _ in range(120):
        g.step(1)
        E.append(g.global_moments()[2])
    t = np.arange(121)
    k = 2 * np.pi / n
    slope = np.polyfit(t[40:], np.log(E[40:]), 1)[0]
    assert -slope / (6 * k * k) == pytest.approx(nu_of(1.9), rel=0.01)


def _poiseuille_error(orc, H, om):
    nu, F = nu_of(om), 1e-6
    g = orc.Grid(4, 4, H, omega=om, bc_zlo=orc.NOSLIP, bc_zhi=orc.NOSLIP,
                 body_force=(F, 0, 0))
    g.init_fields(np.ones((H, 4, 4)), np.zeros((3, H, 4, 4)))
    g.step(int(8 * H * H / nu))
    ux = g.fields()[1][0, :, 0, 0]
    z = np.arange(H)
    ua = F / (2 * nu) * (z + 0.5) * (H - 0.5 - z)   # walls at z = -1/2, H - 1/2
    return np.sqrt(np.sum((ux - ua) ** 2) / np.sum(ua ** 2))


@pytest.mark.parametrize("om", [1.0, 1.6])
def test_poiseuille_second_order(orc, om):
    e = [_poiseuille_error(orc, H, om) for H in (8, 16, 32)]
    assert e[2] < 0.01
    assert np.log2(e[0] / e[1]) >= 1.8 and np.log2(e[1] / e[2]) >= 1.8


def test_kolmogorov_flow(orc):
    """steady u_x = F0 sin(kz) / (nu k^2) under F_x = F0 sin(kz)"""
    N, om, F0 = 32, 1.0, 1e-6
    nu, k = nu_of(om), 2 * np.pi / N
    g = orc.Grid(4, 4, N, omega=om)
    z = np.arange(N)
    F = np.zeros((3, N, 4, 4))
    F[0] = F0 * np.sin(k * z)[:, None, None]
    g.set_force_field(F)
    g.init_fields(np.ones((N, 4, 4)), np.zeros((3, N, 4, 4)))
    g.step(int(40 / (nu * k * k)))
    ua = F0 * np.sin(k * z) / (nu * k * k)
    assert np.abs(g.fields()[1][0, :, 0, 0] - ua).max() <= 5e-3 * np.abs(ua).max()


@pytest.mark.parametrize("walls", [(0, 0), (3, 3), (3, 0)])
def test_uniform_inflow_is_fixed_point(orc, walls):
    """Uniform flow entering at the inlet equilibrium and leaving through the
    zero-gradient outlet, with periodic or free-slip z sides, stays exact."""
    nx, ny, nz = 12, 6, 8
    uin = (0.05, 0.0, 0.0)
    g = orc.Grid(nx, ny, nz, omega=1.9, bc_x=orc.INOUT, bc_zlo=walls[0],
                 bc_zhi=walls[1], u_in=uin)
    u = np.zeros((3, nz, ny, nx))
    u[0] = uin[0]
    g.init_fields(np.ones((nz, ny, nx)), u)
    f0 = g.get_pops()
    g.step(10)
    assert np.abs(g.get_pops() - f0).max() < 1e-15


def test_free_slip_channel_keeps_tangential_flow(orc):
    nx, ny, nz = 6, 6, 8
    g = orc.Grid(nx, ny, nz, omega=1.5, bc_zlo=orc.FREESLIP, bc_zhi=orc.FREESLIP)
    u = np.zeros((3, nz, ny, nx))
    u[0], u[1] = 0.05, -0.02
    g.init_fields(np.ones((nz, ny, nx)), u)
    f0 = g.get_pops()
    g.step(10)
    assert np.abs(g.get_pops() - f0).max() < 1e-15


@pytest.mark.parametrize("walls", [(2, 2), (2, 3), (3, 3)])
def test_closed_walls_conserve_mass(orc, walls):
    nx, ny, nz = 8, 6, 10
    g = orc.Grid(nx, ny, nz, omega=1.8, bc_zlo=walls[0], bc_zhi=walls[1])
    rng = np.random.default_rng(0)
    u = rng.uniform(-0.03, 0.03, (3, nz, ny, nx))
    g.init_fields(1.0 + rng.uniform(-0.01, 0.01, (nz, ny, nx)), u)
    m0 = g.global_moments()[0]
    g.step(30)
    assert g.global_moments()[0] == pytest.approx(m0, rel=1e-14)


def test_inflow_channel_steady_state_matches_inlet_populations(orc):
    """From rest, the channel settles to a uniform state (rho, u e_x) whose
    nine incoming (c_x = +1) equilibrium populations equal those of the inlet
    state (1, u_in e_x): rho (1/3 + u^2 + u) = 1/3 + u_in^2 + u_in."""
    nx, ny, nz, uin = 24, 4, 4, 0.04
    g = orc.Grid(nx, ny, nz, omega=1.2, bc_x=orc.INOUT, u_in=(uin, 0, 0))
    g.init_fields(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    g.step(1200)
    rho, u = g.fields()
    assert np.ptp(rho) < 1e-9 and np.ptp(u[0]) < 1e-9
    assert np.abs(u[1:]).max() < 1e-12
    r, ux = rho.mean(), u[0].mean()
    assert r * (1 / 3 + ux * ux + ux) == pytest.approx(1 / 3 + uin * uin + uin, rel=1e-9)
