"""Wind-turbine runs of the actuator-line path.

    python -m paper_2402_13171_amd.run_turbine single --kernel gauss --out results/single_turbine_gauss.json
    python -m paper_2402_13171_amd.run_turbine row --weights results/closure_weights.npy \
        --out results/turbine_row.json

single: 256 x 128 x 128, FP32, uniform inflow 0.05 at x = 0, zero-gradient
outflow, periodic y/z, one 3-blade rotor (diameter 32, TSR 7, 3 x 32 points,
Gaussian eps = 2, or --kernel roma3 for the Roma 3-point delta, --tip-loss
for the Prandtl factor) at x = 64, 2000 steps. Reports MLUPS with the rotor and
without it (the paper's way of isolating the turbine overhead, Sec. 4.3,
Table 1), the thrust/torque/power time series, and the final normal and
tangential force per blade point.

tree: the single-turbine box with a turbine given as a component tree
(Sec. 3.3): --config hawt (tower, nacelle face and rotor), floating (the same
on a pitching and surging platform), vawt (vertical-axis rotor, D = 32, with
its shaft) or disk (actuator disk, D = 32, C_T' = 4/3). Reports MLUPS with
and without it and per-component loads over the last rotor revolution.

row: 1024 x 256 x 256, FP16 storage (--storage f32 for the FP32 comparison
run), learned closure, three rotors of diameter 48 spaced 5 D apart, ground
wall (bounce-back) and free-slip top,
sheared inflow u = 0.05 ((z + 1/2)/128)^0.14 plus a convected frozen
turbulence box (5 % intensity), 5000 steps; per-rotor thrust and power.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

import workloads
from .lbm import Lbm


def timed_steps(sim, n):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(sim.stream)
    sim.step(n)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def single(args, log):
    nx, ny, nz = 256, 128, 128
    rot = dict(workloads.single_turbine_rotor(), kernel=args.kernel, tip_loss=args.tip_loss)
    u0 = np.zeros((3, nz, ny, nx))
    u0[0] = 0.05
    spread = "eps 2 Gaussian" if args.kernel == "gauss" else "Roma 3-point delta"
    out = {"workload": f"single turbine 256x128x128 FP32, inflow 0.05, rotor D=32 TSR 7, {spread}"
                       + (", Prandtl tip loss" if args.tip_loss else ""),
           "kernel": args.kernel, "tip_loss": args.tip_loss}
    # without the rotor
    sim = Lbm(nx, ny, nz, omega=args.omega, bc_x="inout", u_in=(0.05, 0, 0))
    sim.init_fields(np.ones((nz, ny, nx)), u0)
    sim.step(10)
    ms0 = timed_steps(sim, 200)
    sim.close()
    # with the rotor
    sim = Lbm(nx, ny, nz, omega=args.omega, bc_x="inout", u_in=(0.05, 0, 0))
    sim.init_fields(np.ones((nz, ny, nx)), u0)
    sim.set_rotor(0, rot)
    series = []
    t0 = time.time()
    chunk = 10
    ms_rot = []
    while sim.time < args.steps:
        ms_rot.append(timed_steps(sim, chunk))
        T, Q, P = sim.rotor_loads(0)
        series.append([sim.time, T, Q, P])
        if sim.time % 500 == 0:
            log(f"single turbine: step {sim.time}, T {T:.4e}, P {P:.4e}")
    loads, pts = sim.rotor_loads(0, with_points=True)
    n = nx * ny * nz
    per_rev = int(round(2 * np.pi / rot["omega_rot"]))
    s = np.array(series)
    last = s[s[:, 0] > s[-1, 0] - per_rev]
    # normal (axial) and tangential force per point along blade 0
    npb = len(rot["r"])
    th = rot["azimuth0"] + rot["omega_rot"] * (sim.time - 1)
    et = np.array([0.0, -np.sin(th), np.cos(th)])
    out.update({
        "steps": sim.time, "mlups_without_rotor": n / (ms0 * 1e-3) / 1e6,
        "mlups_with_rotor": n / (np.median(ms_rot) * 1e-3) / 1e6,
        "turbine_overhead_pct": 100.0 * (np.median(ms_rot) - ms0) / ms0,
        "mean_last_revolution": {"thrust": float(last[:, 1].mean()), "torque": float(last[:, 2].mean()),
                                 "power": float(last[:, 3].mean())},
        "series_every_10_steps": s.tolist(),
        "blade0_points": {"r": list(map(float, rot["r"])), "normal": pts[:npb, 0].tolist(),
                          "tangential": (pts[:npb] @ et).tolist()},
        "wall_s": time.time() - t0,
    })
    sim.close()
    return out


def tree(args, log):
    from workloads import turbines as TB
    nx, ny, nz = 256, 128, 128
    hub = (64.0, 63.5, 63.5)
    rot = dict(workloads.single_turbine_rotor(), kernel=args.kernel, tip_loss=args.tip_loss)
    if args.config == "hawt":
        tb = TB.hawt(rot, base_z=8.0, overhang=3.0)
        names = ["platform", "tower", "nacelle", "nacelle face", "hub", "blade 0", "blade 1", "blade 2"]
    elif args.config == "floating":
        tb = TB.hawt(rot, base_z=8.0, overhang=3.0, pitch_amp=0.05, surge_amp=1.0,
                     wave_freq=2.0 * np.pi / 400.0)
        names = ["platform", "tower", "nacelle", "nacelle face", "hub", "blade 0", "blade 1", "blade 2"]
    elif args.config == "vawt":
        tb = TB.vawt(hub, radius=16.0, height=32.0, n_points=32, tsr=3.0, chord=2.0, kernel=args.kernel)
        names = ["rotor", "blade 0", "blade 1", "blade 2", "shaft"]
    else:
        tb = TB.actuator_disk(hub, radius=16.0, n_rings=8, n_azimuth=16, kernel=args.kernel)
        names = ["disk"]
    npts = sum(len(n["s"]) * n.get("n_azimuth", 1) if n["kind"] == "disk" else len(n.get("s", []))
               for n in tb["nodes"] if n["kind"] != "frame")
    u0 = np.zeros((3, nz, ny, nx))
    u0[0] = 0.05
    out = {"workload": f"turbine tree '{args.config}' in the single-turbine box 256x128x128 FP32, inflow 0.05, "
                       f"{npts} points, {args.kernel} spreading", "config": args.config, "points": npts}
    sim = Lbm(nx, ny, nz, omega=args.omega, bc_x="inout", u_in=(0.05, 0, 0))
    sim.init_fields(np.ones((nz, ny, nx)), u0)
    sim.step(10)
    ms0 = timed_steps(sim, 200)
    sim.close()
    sim = Lbm(nx, ny, nz, omega=args.omega, bc_x="inout", u_in=(0.05, 0, 0))
    sim.init_fields(np.ones((nz, ny, nx)), u0)
    sim.set_turbine(0, tb)
    t0 = time.time()
    chunk, ms_t, series = 10, [], []
    while sim.time < args.steps:
        ms_t.append(timed_steps(sim, chunk))
        nl, _ = sim.turbine_loads(0)
        series.append([sim.time] + nl.reshape(-1).tolist())
        if sim.time % 500 == 0:
            log(f"tree {args.config}: step {sim.time}, total force x {nl[:, 0].sum():.4e}, power {nl[:, 6].sum():.4e}")
    n = nx * ny * nz
    s = np.array(series)
    per_rev = int(round(2 * np.pi / rot["omega_rot"])) if args.config != "vawt" else \
        int(round(2 * np.pi / tb["nodes"][0]["omega"]))
    last = s[s[:, 0] > s[-1, 0] - per_rev][:, 1:].reshape(-1, len(tb["nodes"]), 7).mean(0)
    out.update({
        "steps": sim.time, "mlups_without_turbine": n / (ms0 * 1e-3) / 1e6,
        "mlups_with_turbine": n / (np.median(ms_t) * 1e-3) / 1e6,
        "turbine_overhead_pct": 100.0 * (np.median(ms_t) - ms0) / ms0,
        "mean_last_revolution_per_node": {names[k]: {"force": last[k, 0:3].tolist(), "moment": last[k, 3:6].tolist(),
                                                     "power": float(last[k, 6])}
                                          for k in range(len(tb["nodes"]))},
        "total_force_x": float(last[:, 0].sum()), "total_power": float(last[:, 6].sum()),
        "wall_s": time.time() - t0,
    })
    sim.close()
    return out


def row(args, log):
    nx, ny, nz = 1024, 256, 256
    rots = workloads.turbine_row_rotors()
    mean, box = workloads.turbine_row_inflow(ny=ny, nz=nz)
    blob = np.load(args.weights).astype(np.float64) if args.weights else None
    closure = "mlp" if blob is not None else "smag"
    sim = Lbm(nx, ny, nz, omega=args.omega, storage=args.storage, closure=closure, cs_smag=0.1, bc_x="inout",
              bc_z=("noslip", "freeslip"), check_every=500)
    if blob is not None:
        sim.set_closure_weights(blob)
    u0 = np.broadcast_to(mean[:, :, :, None], (3, nz, ny, nx)).astype(np.float64)
    sim.init_fields(np.ones((nz, ny, nx)), u0)
    del u0
    sim.set_inflow(mean, box, advect=0.05)
    for k, r in enumerate(rots):
        sim.set_rotor(k, r)
    series = []
    ms = []
    t0 = time.time()
    while sim.time < args.steps:
        ms.append(timed_steps(sim, 50))
        series.append([sim.time] + [float(v) for k in range(3) for v in sim.rotor_loads(k)])
        if sim.time % 500 == 0:
            log(f"turbine row: step {sim.time}, thrusts " + " ".join(f"{series[-1][1 + 3 * k]:.3e}" for k in range(3)))
    s = np.array(series)
    per_rev = int(round(2 * np.pi / rots[0]["omega_rot"]))
    last = s[s[:, 0] > s[-1, 0] - 2 * per_rev]
    n = nx * ny * nz
    out = {
        "workload": f"turbine row 1024x256x256 {args.storage.upper()} + " + closure
                    + " closure, 3 rotors D=48, sheared turbulent inflow",
        "storage": args.storage, "rounding": "stochastic" if args.storage != "f32" else None,
        "weights": args.weights,
        "steps": sim.time, "mlups": n / (np.median(ms) * 1e-3) / 1e6,
        "per_rotor_mean_last_two_revolutions": [
            {"thrust": float(last[:, 1 + 3 * k].mean()), "torque": float(last[:, 2 + 3 * k].mean()),
             "power": float(last[:, 3 + 3 * k].mean())} for k in range(3)],
        "series_every_50_steps": s.tolist(), "wall_s": time.time() - t0,
    }
    sim.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=["single", "row", "tree"])
    ap.add_argument("--config", choices=["hawt", "floating", "vawt", "disk"], default="hawt",
                    help="turbine tree (tree case)")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--omega", type=float, default=1.9)
    ap.add_argument("--weights", default=None)
    ap.add_argument("--kernel", choices=["gauss", "roma3"], default="gauss",
                    help="force spreading kernel (single case)")
    ap.add_argument("--tip-loss", action="store_true", help="Prandtl tip-loss factor (single case)")
    ap.add_argument("--storage", choices=["f16", "bf16", "f32"], default="f16", help="population storage (row case)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.steps is None:
        a.steps = 2000 if a.case == "single" else 5000
    t_start = time.time()
    log = lambda *m: print(f"[{time.time() - t_start:7.1f}s]", *m, flush=True)
    res = {"single": single, "row": row, "tree": tree}[a.case](a, log)
    default = {"single": f"results/single_turbine_{a.kernel}{'_tiploss' if a.tip_loss else ''}.json",
               "row": f"results/turbine_row{'' if a.storage == 'f16' else '_' + a.storage}.json",
               "tree": f"results/tree_{a.config}.json"}
    out = a.out or default[a.case]
    os.makedirs(os.path.dirname(out) or ".", exist_ok=True)
    with open(out, "w") as fh:
        json.dump(res, fh)
    log("written", out, {k: v for k, v in res.items() if not isinstance(v, (list, dict))})
    return res


if __name__ == "__main__":
    main(sys.argv[1:])
