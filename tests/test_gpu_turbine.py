"""GPU <-> oracle parity of the turbine topology tree (Sec. 3.3, Alg. 1 and
Alg. 2) through the C ABI: a rotor given as a tree against the same rotor in
a rotor slot and against the oracle; a horizontal-axis turbine with tower
and nacelle; a vertical-axis turbine; a floating (pitching and surging) and
a yawing turbine; an actuator disk; FP16 storage; argument validation."""
import numpy as np
import pytest

import oracle
import workloads
from workloads import turbines as TB

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _uniform(shape, U=0.05):
    nx, ny, nz = shape
    u = np.zeros((3, nz, ny, nx))
    u[0] = U
    return np.ones((nz, ny, nx)), u


def _rotor(hub, R=8.0, omega_rot=0.02, n_points=8, **kw):
    rot = workloads.make_rotor(hub=hub, radius=R, n_blades=3, n_points=n_points,
                               tsr=omega_rot * R / 0.05, u_ref=0.05)
    rot.update(kw)
    return rot


def run_tree(shape, turbine, steps, storage="f32", omega=1.8, open_domain=False):
    from paper_2402_13171_amd.lbm import Lbm
    nx, ny, nz = shape
    print(f"turbine case {shape} {storage} nodes={len(turbine['nodes'])} open={open_domain}", flush=True)
    if open_domain:
        # inflow / zero-gradient outflow in x, ground wall (bounce-back) and
        # free-slip top in z
        sim = Lbm(nx, ny, nz, omega=omega, storage=storage, bc_x="inout", bc_z=("noslip", "freeslip"),
                  u_in=(0.05, 0.0, 0.0))
        ref = oracle.Grid(nx, ny, nz, omega=omega, bc_x=oracle.INOUT, bc_zlo=oracle.NOSLIP,
                          bc_zhi=oracle.FREESLIP, u_in=(0.05, 0.0, 0.0))
    else:
        sim = Lbm(nx, ny, nz, omega=omega, storage=storage)
        ref = oracle.Grid(nx, ny, nz, omega=omega)
    rho, u = _uniform(shape)
    sim.init_fields(rho, u)
    ref.init_fields(rho, u)
    sim.set_turbine(2, turbine)
    ref.set_turbine(2, turbine)
    hist = []
    for s in range(steps):
        sim.step(1)
        ref.step(1)
        hist.append((s, sim.turbine_loads(2), ref.turbine_loads(2)))
    return sim, ref, hist


def check_tree(hist, ftol, xtol=1e-11):
    """Per-point positions and velocities (FP64 kinematics on both sides),
    forces relative to the largest force, node loads relative to the largest
    load of each kind; returns the worst force error."""
    worst = 0.0
    for s, (nlg, pg), (nlr, pr) in hist:
        np.testing.assert_allclose(pg[:, 0:3], pr[:, 0:3], rtol=0, atol=xtol * max(1.0, np.abs(pr[:, 0:3]).max()))
        np.testing.assert_allclose(pg[:, 3:6], pr[:, 3:6], rtol=0, atol=xtol)
        fs = np.abs(pr[:, 6:9]).max()
        assert fs > 0
        e = np.abs(pg[:, 6:9] - pr[:, 6:9]).max() / fs
        worst = max(worst, e)
        assert e <= ftol, (s, e)
        # scales: the largest node force; for moments at least that force on a
        # one-cell lever, for power that force at the fastest point's speed
        # (a moment or power that cancels by symmetry is round-off on both sides)
        fmax = np.abs(nlr[:, 0:3]).max()
        vmax = np.abs(pr[:, 3:6]).max()
        for cols, floor in ((slice(0, 3), 0.0), (slice(3, 6), fmax), (slice(6, 7), fmax * vmax)):
            sc = max(np.abs(nlr[:, cols]).max(), floor)
            if sc > 0:
                assert np.abs(nlg[:, cols] - nlr[:, cols]).max() <= ftol * sc, (s, cols)
    return worst


def check_fields(sim, ref, tol):
    _, ug = sim.fields()
    _, ur = ref.fields()
    err = np.linalg.norm(ug - ur, axis=0).max() / np.linalg.norm(ur, axis=0).max()
    assert err <= tol, err
    return err


@pytest.mark.parametrize("kernel", ["gauss", "roma3"])
def test_rotor_as_tree_matches_rotor_slot_and_oracle(kernel):
    """The tree form of a rotor (hub frame + blade lines) gives the same
    points and forces as the closed-form rotor slot, and matches the oracle."""
    _need_gpu()
    from paper_2402_13171_amd.lbm import Lbm
    shape = (48, 48, 48)
    rot = _rotor((20.0, 23.5, 24.0), kernel=kernel, tip_loss=True, azimuth0=0.4)
    sim, ref, hist = run_tree(shape, TB.rotor_tree(rot), 6)
    w = check_tree(hist, 2e-5)
    e = check_fields(sim, ref, 1e-5)
    print(f"rotor tree ({kernel}): worst force error {w:.2e}, field {e:.2e}")
    # the same rotor in a rotor slot
    a = Lbm(*shape, omega=1.8)
    rho, u = _uniform(shape)
    a.init_fields(rho, u)
    a.set_rotor(0, rot)
    a.step(6)
    _, pf = a.rotor_loads(0, with_points=True)
    _, pts = hist[-1][1]
    assert np.abs(pts[:, 6:9] - pf).max() <= 1e-6 * np.abs(pf).max()
    loads = a.rotor_loads(0)
    nl, _ = hist[-1][1]
    assert nl[1:, 0].sum() == pytest.approx(loads[0], rel=1e-6)
    assert nl[1:, 3].sum() == pytest.approx(loads[1], rel=1e-6)


@pytest.mark.parametrize("kernel", ["gauss", "roma3"])
def test_hawt_with_tower_and_nacelle(kernel):
    _need_gpu()
    rot = _rotor((16.0, 23.5, 36.0))
    tr = TB.hawt(rot, base_z=8.0, overhang=3.0, tower_spacing=4.0, kernel=kernel)
    sim, ref, hist = run_tree((48, 48, 56), tr, 9)
    w = check_tree(hist, 2e-5)
    e = check_fields(sim, ref, 1e-5)
    nl, pts = hist[-1][1]
    assert nl[1, 0] > 0 and nl[3, 0] > 0  # tower and nacelle drag downstream
    print(f"HAWT + tower + nacelle ({kernel}): worst force error {w:.2e}, field {e:.2e}")


@pytest.mark.parametrize("kernel,base_z", [("gauss", 7.0), ("roma3", 1.5)])
def test_hawt_on_the_ground_in_an_open_domain(kernel, base_z):
    """Tower standing on the bounce-back ground of an inflow/outflow domain
    with a free-slip top (the Roma delta lets the tower reach one cell above
    the wall)."""
    _need_gpu()
    rot = _rotor((16.0, 23.5, 30.0))
    tr = TB.hawt(rot, base_z=base_z, overhang=3.0, tower_spacing=3.0, kernel=kernel)
    sim, ref, hist = run_tree((48, 48, 48), tr, 9, open_domain=True)
    w = check_tree(hist, 2e-5)
    e = check_fields(sim, ref, 1e-5)
    print(f"HAWT on the ground, open domain ({kernel}): worst force error {w:.2e}, field {e:.2e}")


def test_vawt():
    _need_gpu()
    vt = TB.vawt((24.0, 24.0, 24.0), radius=8.0, height=12.0, n_points=8, tsr=2.5)
    sim, ref, hist = run_tree((48, 48, 48), vt, 9)
    w = check_tree(hist, 2e-5)
    e = check_fields(sim, ref, 1e-5)
    print(f"VAWT: worst force error {w:.2e}, field {e:.2e}")


@pytest.mark.parametrize("case", ["floating", "yawing"])
def test_moving_platforms(case):
    """Pitching and surging platform (sinusoidal), or a yawing nacelle: the
    conservative spreading box holds every support node (the fields match
    the oracle, which spreads into the whole domain)."""
    _need_gpu()
    if case == "floating":
        rot = _rotor((24.0, 31.5, 40.0))
        tr = TB.hawt(rot, base_z=12.0, pitch_amp=0.05, surge_amp=1.0, wave_freq=2.0 * np.pi / 50.0,
                     tower_spacing=4.0)
        shape = (64, 64, 64)
    else:
        rot = _rotor((32.0, 32.0, 32.0), R=6.0)
        tr = TB.hawt(rot, base_z=10.0, overhang=2.0, yaw_rate=0.01, tower_spacing=4.0)
        shape = (64, 64, 64)
    sim, ref, hist = run_tree(shape, tr, 12)
    w = check_tree(hist, 2e-5)
    e = check_fields(sim, ref, 1e-5)
    print(f"{case}: worst force error {w:.2e}, field {e:.2e}")


def test_actuator_disk():
    _need_gpu()
    ad = TB.actuator_disk((16.0, 24.0, 24.0), radius=8.0, n_rings=4, n_azimuth=16)
    sim, ref, hist = run_tree((48, 48, 48), ad, 9)
    w = check_tree(hist, 2e-5)
    e = check_fields(sim, ref, 1e-5)
    nl, _ = hist[0][1]
    T = 0.5 * (4.0 / 3.0) * 0.05 ** 2 * np.pi * 64.0
    assert nl[0, 0] == pytest.approx(T, rel=1e-6)  # uniform inflow at the first step
    print(f"actuator disk: worst force error {w:.2e}, field {e:.2e}")


def test_hawt_fp16_storage():
    _need_gpu()
    rot = _rotor((16.0, 23.5, 36.0))
    tr = TB.hawt(rot, base_z=8.0, overhang=3.0, tower_spacing=4.0)
    sim, ref, hist = run_tree((48, 48, 56), tr, 9, storage="f16")
    # FP16 storage gate of the method (max velocity error 1e-3 of the largest
    # velocity); the forces inherit the sampled velocity's error
    w = check_tree(hist, 2e-3)
    e = check_fields(sim, ref, 1e-3)
    print(f"HAWT FP16 storage: worst force error {w:.2e}, field {e:.2e}")


def test_turbine_argument_validation():
    _need_gpu()
    from paper_2402_13171_amd.lbm import Lbm, LbmError
    sim = Lbm(32, 32, 32)
    rot = _rotor((12.0, 16.0, 16.0), R=6.0)
    good = TB.rotor_tree(rot)

    def bad(mutate):
        tr = {k: v for k, v in good.items()}
        tr["nodes"] = [dict(n) for n in good["nodes"]]
        mutate(tr)
        with pytest.raises(LbmError):
            sim.set_turbine(0, tr)

    bad(lambda t: t["nodes"][1].update(parent=1))                 # parent must precede
    bad(lambda t: t["nodes"][1].update(rot=2.0 * np.eye(3)))       # not orthonormal
    bad(lambda t: t["nodes"][1].update(rot=np.diag([1.0, 1.0, -1.0])))  # reflection
    bad(lambda t: t["nodes"][0].update(axis=(1.0, 1.0, 0.0)))      # axis not a unit vector
    bad(lambda t: t["nodes"][1].update(kind="disk", n_azimuth=4))  # blade elements on a disk
    bad(lambda t: t["nodes"][1].update(normal=(0.0, 1.0, 0.0)))    # normal along the span
    bad(lambda t: t["nodes"][0].update(pos=(3.0, 16.0, 16.0)))     # box leaves the domain
    bad(lambda t: t.update(kernel="roma3") or t["nodes"][1].update(s=np.linspace(0, 6, 600),
                                                                   width=np.ones(600),
                                                                   chord=np.ones(600),
                                                                   twist=np.zeros(600)))
    bad(lambda t: t["nodes"][0].update(pos=(np.nan, 16.0, 16.0)))  # non-finite pose
    bad(lambda t: t["nodes"][1].update(chord=np.full(8, np.inf)))    # non-finite point data
    sim.set_turbine(0, good)  # and the good one is accepted
    # arguments are checked before the slot is touched: a rejected call
    # leaves the earlier turbine in place
    bad(lambda t: t["nodes"][1].update(parent=1))
    sim.init_tgv(u0=0.01)
    sim.step(2)
    nl, pts = sim.turbine_loads(0)
    assert pts.shape == (24, 9) and np.isfinite(nl).all() and np.abs(pts[:, 6:9]).max() > 0


def test_rotors_and_a_turbine_in_one_box():
    """Two rotor slots and a turbine-tree slot in one periodic box (one
    spreading launch covers every slot's box): per-slot loads and the flow
    against the oracle."""
    _need_gpu()
    from paper_2402_13171_amd.lbm import Lbm
    shape = (64, 48, 48)
    ra = _rotor((14.0, 23.5, 24.0), R=6.0)
    rb = _rotor((52.0, 23.5, 24.0), R=6.0, kernel="roma3", azimuth0=1.0)
    disk = TB.actuator_disk((34.0, 24.0, 24.0), radius=6.0, n_rings=3, n_azimuth=12)
    sim = Lbm(*shape, omega=1.8)
    ref = oracle.Grid(*shape, omega=1.8)
    rho, u = _uniform(shape)
    sim.init_fields(rho, u)
    ref.init_fields(rho, u)
    for g in (sim, ref):
        g.set_rotor(0, ra)
        g.set_turbine(1, disk)
        g.set_rotor(2, rb)
    worst = 0.0
    for s in range(8):
        sim.step(1)
        ref.step(1)
        for rid in (0, 2):
            lg, lr = sim.rotor_loads(rid), ref.rotor_loads(rid)
            worst = max(worst, np.abs(lg - lr).max() / np.abs(lr).max())
        nlg, _ = sim.turbine_loads(1)
        nlr, _ = ref.turbine_loads(1)
        worst = max(worst, np.abs(nlg[:, 0] - nlr[:, 0]).max() / np.abs(nlr[:, 0]).max())
    e = check_fields(sim, ref, 1e-5)
    print(f"two rotors + a disk: worst load error {worst:.2e}, field {e:.2e}")
    assert worst <= 2e-5


def test_checkpoint_resume_with_rotor_and_turbine_is_bitwise():
    """A run resumed from a checkpoint repeats the uninterrupted run bit for
    bit, rotor and turbine loads included: the state carries the slots'
    spread force of the last step, which the next step's sampling uses. A
    context without the same slots refuses the state."""
    _need_gpu()
    from paper_2402_13171_amd.lbm import Lbm, LbmError
    shape = (64, 48, 48)
    ra = _rotor((14.0, 23.5, 24.0), R=6.0)
    tr = TB.hawt(_rotor((40.0, 23.5, 28.0), R=6.0), base_z=8.0, overhang=2.0, tower_spacing=4.0)
    sim = Lbm(*shape, omega=1.8, bc_x="inout", bc_z=("noslip", "freeslip"), u_in=(0.05, 0.0, 0.0))
    rho, u = _uniform(shape)
    sim.init_fields(rho, u)
    sim.set_rotor(0, ra)
    sim.set_turbine(1, tr)
    sim.step(5)
    state = sim.get_state()

    def run(k):
        out = []
        for _ in range(k):
            sim.step(1)
            out.append((sim.rotor_loads(0).copy(), sim.turbine_loads(1)[0].copy()))
        return out, sim.pops()

    a, pa = run(3)
    sim.set_state(state)
    assert sim.time == 5
    b, pb = run(3)
    assert np.array_equal(pa, pb)
    for (ra_, ta), (rb_, tb_) in zip(a, b):
        assert np.array_equal(ra_, rb_) and np.array_equal(ta, tb_)
    other = Lbm(*shape, omega=1.8, bc_x="inout", bc_z=("noslip", "freeslip"), u_in=(0.05, 0.0, 0.0))
    other.init_fields(rho, u)
    other.set_rotor(0, ra)
    with pytest.raises(LbmError):
        other.set_state(state)  # the turbine slot is missing


def test_hawt_tree_in_the_single_turbine_box_200_steps():
    """The run_turbine tree case at full size (256 x 128 x 128, inflow /
    outflow, the D = 32 rotor with tower and nacelle face, 140 points) for 200
    steps: node loads within 1e-3 of the largest load of each kind every
    10 steps, and the flow within 1e-4 at the end."""
    _need_gpu()
    from paper_2402_13171_amd.lbm import Lbm
    shape = (256, 128, 128)
    tr = TB.hawt(workloads.single_turbine_rotor(), base_z=8.0, overhang=3.0)
    print("HAWT tree, 256x128x128, 200 steps (FP64 oracle on the host: ~30 s)", flush=True)
    sim = Lbm(*shape, omega=1.9, bc_x="inout", u_in=(0.05, 0.0, 0.0))
    ref = oracle.Grid(*shape, omega=1.9, bc_x=oracle.INOUT, u_in=(0.05, 0.0, 0.0))
    rho, u = _uniform(shape)
    sim.init_fields(rho, u)
    ref.init_fields(rho, u)
    sim.set_turbine(0, tr)
    ref.set_turbine(0, tr)
    worst = 0.0
    for s in range(20):
        sim.step(10)
        ref.step(10)
        nlg, _ = sim.turbine_loads(0)
        nlr, _ = ref.turbine_loads(0)
        for cols in (slice(0, 3), slice(3, 6), slice(6, 7)):
            sc = np.abs(nlr[:, cols]).max()
            worst = max(worst, np.abs(nlg[:, cols] - nlr[:, cols]).max() / sc)
    e = check_fields(sim, ref, 1e-4)
    print(f"HAWT tree 200 steps: worst node-load error {worst:.2e}, field {e:.2e}")
    assert worst <= 1e-3
