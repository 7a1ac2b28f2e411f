"""Long GPU <-> oracle runs, opt-in (set LBM_LONG_TESTS=1): the single-turbine
case over 2000 steps (about seven rotor revolutions), thrust, torque and
power time series against the FP64 oracle. About four minutes of oracle time
on 16 host cores."""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not os.environ.get("LBM_LONG_TESTS"),
                                 reason="long run (~4 min of FP64 oracle time); set LBM_LONG_TESTS=1")]


def test_single_turbine_loads_over_2000_steps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2402_13171_amd.lbm import Lbm
    nx, ny, nz = 256, 128, 128
    rot = workloads.single_turbine_rotor()
    sim = Lbm(nx, ny, nz, omega=1.9, bc_x="inout", u_in=(0.05, 0, 0))
    ref = oracle.Grid(nx, ny, nz, omega=1.9, bc_x=oracle.INOUT, u_in=(0.05, 0, 0))
    u = np.zeros((3, nz, ny, nx))
    u[0] = 0.05
    rho = np.ones((nz, ny, nx))
    sim.init_fields(rho, u)
    ref.init_fields(rho, u)
    sim.set_rotor(0, rot)
    ref.set_rotor(0, rot)
    lg, lr = [], []
    for s in range(2000):
        sim.step(1)
        ref.step(1)
        lg.append(sim.rotor_loads(0))
        lr.append(ref.rotor_loads(0))
        if (s + 1) % 250 == 0:
            e = (np.abs(np.array(lg) - np.array(lr)) / np.abs(np.array(lr)).max(axis=0)).max()
            print(f"step {s + 1}: worst relative load error so far {e:.2e}", flush=True)
    lg, lr = np.array(lg), np.array(lr)
    err = (np.abs(lg - lr) / np.abs(lr).max(axis=0)).max()
    _, ug = sim.fields()
    _, ur = ref.fields()
    ferr = np.linalg.norm(ug - ur, axis=0).max() / np.linalg.norm(ur, axis=0).max()
    print(f"2000 steps: worst relative load error {err:.2e}, field eps_max {ferr:.2e}; "
          f"last-step thrust {lg[-1, 0]:.5f} (oracle {lr[-1, 0]:.5f}), power {lg[-1, 2]:.6f} "
          f"(oracle {lr[-1, 2]:.6f})")
    assert err <= 1e-3
