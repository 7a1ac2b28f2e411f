"""The spreading box of a turbine tree (host logic of the library,
lbm_turbine_box, no device): it holds every point's spreading support at every
time, checked against the oracle's kinematics at many times, and it is tight
for a rigid rotor turning about a fixed axis (the bound there is the exact
bounding box of the blade circles)."""
import numpy as np
import pytest

import oracle
import workloads
from workloads import turbines as TB


def _lbm():
    from paper_2402_13171_amd import lbm
    try:
        lbm.lib()
    except RuntimeError:
        pytest.fail("liblbm.so is not built (run __graft_entry__.build())")
    return lbm


def _rotor(hub, R=10.0, omega_rot=0.02):
    return workloads.make_rotor(hub=hub, radius=R, n_blades=3, n_points=8,
                                tsr=omega_rot * R / 0.05, u_ref=0.05)


CASES = {
    "rotor": TB.rotor_tree(_rotor((40.0, 40.5, 41.0))),
    "hawt": TB.hawt(_rotor((40.0, 40.5, 50.0)), base_z=10.0, tower_spacing=4.0),
    "hawt-roma": TB.hawt(_rotor((40.0, 40.5, 50.0)), base_z=10.0, tower_spacing=4.0, kernel="roma3"),
    "floating": TB.hawt(_rotor((40.0, 40.5, 50.0)), base_z=10.0, pitch_amp=0.08, surge_amp=1.5,
                        wave_freq=2.0 * np.pi / 300.0, tower_spacing=4.0),
    "yawing": TB.hawt(_rotor((40.0, 40.5, 50.0), R=6.0), base_z=10.0, overhang=2.0, yaw_rate=0.01,
                      tower_spacing=4.0),
    "vawt": TB.vawt((40.0, 40.0, 40.0), radius=9.0, height=14.0, n_points=6),
    "disk": TB.actuator_disk((40.0, 40.0, 40.0), radius=8.0, n_rings=3, n_azimuth=8),
}


def _supports(tb, t):
    half = 1 if tb.get("kernel") == "roma3" else 6
    x, _, _ = oracle.turbine_kinematics(tb, t)
    c = np.floor(x + 0.5).astype(int)
    return c - half, c + half


@pytest.mark.parametrize("name", sorted(CASES))
def test_box_holds_every_support_at_every_time(name):
    lbm = _lbm()
    tb = CASES[name]
    lo, hi = lbm.turbine_box(tb)
    rng = np.random.default_rng(1)
    for t in np.concatenate([np.arange(0.0, 400.0, 1.0), rng.uniform(0.0, 1e6, 300)]):
        a, b = _supports(tb, t)
        assert (a >= np.array(lo)).all() and (b <= np.array(hi)).all(), (name, t)


def test_box_of_a_rotor_is_tight():
    """Rotor about +x: the box is the union of the supports over one turn
    (within one node: the sampled turn misses the circles' extreme points by
    less than a cell)."""
    lbm = _lbm()
    tb = CASES["rotor"]
    lo, hi = lbm.turbine_box(tb)
    om = tb["nodes"][0]["omega"]
    ts = np.linspace(0.0, 2.0 * np.pi / om, 2000)
    slo = np.min([_supports(tb, t)[0].min(axis=0) for t in ts], axis=0)
    shi = np.max([_supports(tb, t)[1].max(axis=0) for t in ts], axis=0)
    assert (np.abs(slo - np.array(lo)) <= 1).all() and (np.abs(shi - np.array(hi)) <= 1).all(), (lo, hi, slo, shi)


def test_invalid_turbines_are_rejected_without_a_device():
    lbm = _lbm()
    bad = TB.rotor_tree(_rotor((40.0, 40.5, 41.0)))
    bad["nodes"] = [dict(n) for n in bad["nodes"]]
    bad["nodes"][2]["parent"] = 3
    with pytest.raises(lbm.LbmError):
        lbm.turbine_box(bad)
