"""Degenerate and empty cases of the stream-collide path against the oracle:
the smallest boxes (2 cells along an axis, where the left and right periodic
neighbours coincide and an open box is all inlet and outlet), the rest state
(an exact fixed point: every stored deviation stays exactly zero), a zero-step
call, an empty sample, and relaxation rates near both ends of (0, 2)."""
import numpy as np
import pytest

import oracle
from test_gpu_parity import make_pair, random_field, _need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,case", [
    ((2, 2, 2), dict()),
    ((2, 3, 2), dict(bc_x="inout", bc_z=("noslip", "freeslip"), u_in=(0.05, 0.01, 0.0))),
    ((3, 2, 4), dict(bc_z=("noslip", "noslip"), body_force=(1e-5, 0, 0))),
    ((2, 5, 3), dict(bc_x="inout", u_in=(0.04, 0.0, 0.0))),
], ids=["2x2x2", "2x3x2-open-walls", "3x2x4-walls", "2x5x3-open"])
@pytest.mark.parametrize("general_path", [False, True], ids=["auto", "general"])
def test_smallest_boxes_match_oracle(shape, case, general_path):
    _need_gpu()
    nx, ny, nz = shape
    sim, ref = make_pair(nx, ny, nz, omega=1.6, general_path=general_path, **case)
    rho, u = random_field(nx, ny, nz, seed=21)
    sim.init_fields(rho, u)
    ref.init_fields(rho, u)
    for steps in (1, 1, 4):
        sim.step(steps)
        ref.step(steps)
        assert np.abs(sim.pops() - ref.get_pops()).max() <= 2e-7 * sim.time, (shape, sim.time)


def test_smallest_box_with_learned_closure():
    """2 x 3 x 2: 62 of every 64 lanes of a wave have no cell of their own and
    recompute a neighbour for the matrix-core instructions."""
    _need_gpu()
    from paper_2402_13171_amd.lbm import Lbm
    from test_gpu_mlp import make_blob
    nx, ny, nz = 2, 3, 2
    blob = make_blob(12)
    sim = Lbm(nx, ny, nz, omega=1.95, closure="mlp")
    sim.set_closure_weights(blob)
    ref = oracle.Grid(nx, ny, nz, omega=1.95, closure=oracle.CLOSURE_MLP, mlp_emulate_bf16=True)
    ref.set_mlp(blob)
    rho, u = random_field(nx, ny, nz, seed=22)
    sim.init_fields(rho, u)
    ref.init_fields(rho, u)
    sim.step(5)
    ref.step(5)
    assert np.abs(sim.pops() - ref.get_pops()).max() <= 2e-6


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("case", [dict(), dict(bc_x="inout", bc_z=("noslip", "freeslip"))], ids=["periodic", "open"])
def test_rest_state_is_preserved(storage, case):
    """rho = 1, u = 0: all deviations are 0. In a periodic box they stay
    exactly 0 through both AA parities (the collision maps zero to zero). A
    resting inlet feeds phi(0)^3 - w evaluated in FP32, which is zero only up
    to rounding (a few 1e-10 here), so the open box stays at rest to that
    level through the inflow/outflow and wall rules. FP16 storage rounds
    stochastically: a residue of 1e-11 is stored as 0 or, rarely, as the
    smallest FP16 step 2^-24 (6e-8), so there the bound is that step."""
    _need_gpu()
    from paper_2402_13171_amd.lbm import Lbm
    nx, ny, nz = 37, 9, 6
    sim = Lbm(nx, ny, nz, omega=1.7, storage=storage, **case)
    sim.init_fields(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    w = sim.pops().copy()
    sim.step(7)
    rho, u = sim.fields()
    if not case:
        assert np.array_equal(sim.pops(), w)
        assert not np.any(u)
        assert np.abs(rho - 1.0).max() <= 1e-15  # FP64 sum of the 27 weights
    else:
        tol = 2.0 ** -24 if storage == "f16" else 1e-8
        assert np.abs(sim.pops() - w).max() <= tol
        assert np.abs(u).max() <= 27 * tol and np.abs(rho - 1.0).max() <= 27 * tol


def test_zero_steps_and_empty_sample():
    _need_gpu()
    sim, _ = make_pair(10, 6, 4, omega=1.7)
    rho, u = random_field(10, 6, 4, seed=23)
    sim.init_fields(rho, u)
    sim.step(3)
    s0 = np.asarray(sim.get_state()).copy()
    sim.step(0)
    assert sim.time == 3
    assert np.array_equal(np.asarray(sim.get_state()), s0)
    assert sim.sample_pops(np.zeros(0, dtype=np.uint64)).shape == (0, 27)


@pytest.mark.parametrize("omega", [0.3, 1.999])
def test_extreme_relaxation_rates_match_oracle(omega):
    _need_gpu()
    n = 12
    sim, ref = make_pair(n, n, n, omega=omega)
    rho, u = random_field(n, n, n, seed=24, amp=0.02)
    sim.init_fields(rho, u)
    ref.init_fields(rho, u)
    sim.step(8)
    ref.step(8)
    assert np.abs(sim.pops() - ref.get_pops()).max() <= 2e-6
