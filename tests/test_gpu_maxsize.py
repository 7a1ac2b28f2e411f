"""Parity at the largest boxes (FP32, 113-116 GB of populations in the
blocked store, far past 2^32 bytes): the fast path, whose lane offsets are
32-bit within a z plane of blocks (113 MB here) and whose z-plane bases are
64-bit, on 1024 x 1024 x 1016 and 1024^3, and the 64-bit general path forced
on 1024^3.
Taylor-Green initial state on the device; after one (even) and two (even +
odd) AA steps, sampled cells (corners and the highest linear indices
included) are compared with the FP64 oracle run on a 9^3 periodic window cut
around each cell from the same closed-form initial field."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
HALF = 4
U0 = 0.05


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def tgv_window(shape, k, xyz):
    nx, ny, nz = shape
    x, y, z = xyz
    ix = np.arange(x - HALF, x + HALF + 1) % nx
    iy = np.arange(y - HALF, y + HALF + 1) % ny
    iz = np.arange(z - HALF, z + HALF + 1) % nz
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    u = np.zeros((3,) + Z.shape)
    u[0] = U0 * np.sin(k * X) * np.cos(k * Y) * np.cos(k * Z)
    u[1] = -U0 * np.cos(k * X) * np.sin(k * Y) * np.cos(k * Z)
    return np.ones(Z.shape), u


def oracle_cell(shape, k, xyz, steps):
    rho, u = tgv_window(shape, k, xyz)
    w = 2 * HALF + 1
    g = oracle.Grid(w, w, w, omega=1.9)
    g.init_fields(rho, u)
    g.step(steps)
    return g.get_pops()[:, HALF, HALF, HALF]


@pytest.mark.parametrize("shape,general", [((1024, 1024, 1016), False), ((1024, 1024, 1024), False),
                                           ((1024, 1024, 1024), True)],
                         ids=["fast-1016", "fast-1024", "general-1024"])
def test_largest_planes_match_oracle(shape, general):
    _need_gpu()
    import torch
    from paper_2402_13171_amd.lbm import Lbm
    nx, ny, nz = shape
    n = nx * ny * nz
    k = 2 * np.pi / nx
    rng = np.random.default_rng(5)
    pts = np.stack([rng.integers(0, nx, 30), rng.integers(0, ny, 30), rng.integers(0, nz, 30)], 1)
    corners = np.array([[0, 0, 0], [nx - 1, ny - 1, nz - 1], [nx - 2, ny - 1, nz - 1], [0, ny - 1, nz - 1],
                        [nx - 1, 0, nz - 1], [nx - 1, ny - 1, 0], [5, 7, nz - 2]])
    cells = np.vstack([pts, corners])
    lin = cells[:, 0] + nx * (cells[:, 1] + ny * cells[:, 2])
    assert lin.max() == n - 1
    sim = Lbm(nx, ny, nz, omega=1.9, storage="f32", general_path=general)
    try:
        sim.init_tgv(u0=U0, k=k)
        got = {}
        for steps in (1, 2):
            sim.step(1)
            got[steps] = sim.sample_pops(lin)
    finally:
        sim.close()
        del sim
        torch.cuda.empty_cache()
    worst = 0.0
    for j, xyz in enumerate(cells):
        for steps in (1, 2):
            ref = oracle_cell(shape, k, xyz, steps)
            worst = max(worst, np.abs(got[steps][j] - ref).max())
    print(f"{shape}: worst population error over {len(cells)} cells after 1 and 2 steps = {worst:.3e}")
    assert worst <= 1e-7
