"""Train the learned closure on filtered fine runs and evaluate it in a coarse
LES against no model and Smagorinsky (see closure_training.py).

    python -m paper_2402_13171_amd.train_closure --out results/closure_les.json

Defaults: fine 512^3, omega 1.9, training seeds 0-6 with snapshots at fine
steps 2000/4000/6000/8000, hold-out seed 7. Each filter width w (default 4
and 8: 128^3 and 64^3 coarse grids) gets its own training set (every
8 (4/w)^3-th coarse cell of every snapshot, about 7 M cells at w = 4), its
own network and its own coarse LES: the
coarse run is compared with the filtered fine run at fine steps
2000/4000/8000 (coarse steps 2000/w, 4000/w, 8000/w) through shell spectra
over k in [1, min(42, n_c/2 - 2)] (also over the lower half of that range)
and through the resolved kinetic energy. The gain of the network is the
ratio of an error of no model (or Smagorinsky) to the network's at the last
compared step: above 1, the network is closer to the reference.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import closure_training as ct


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-fine", type=int, default=512)
    ap.add_argument("--w", default="4,8", help="filter widths (coarse grid = n_fine / w)")
    ap.add_argument("--omega", type=float, default=1.9)
    ap.add_argument("--train-seeds", default="0,1,2,3,4,5,6")
    ap.add_argument("--test-seed", type=int, default=7)
    ap.add_argument("--snaps", default="2000,4000,6000,8000")
    ap.add_argument("--eval-fine-steps", default="2000,4000,8000")
    ap.add_argument("--subsample", type=int, default=8, help="keep every n-th coarse cell at w = 4 (scaled by (4/w)^3)")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--out", default="results/closure_les.json")
    ap.add_argument("--weights", default="results/closure_weights.npy",
                    help="weights of the first width's network (the others: _w<width> before the suffix)")
    ap.add_argument("--throughput", action="store_true",
                    help="only measure training and inference samples/s (writes --out)")
    a = ap.parse_args(argv)
    if a.throughput:
        res = {"workload": "closure network 6-32-32-1, synthetic features, forward + backward + Adam per iteration",
               "batches": ct.training_throughput()}
        os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
        print(json.dumps(res))
        return res

    t_start = time.time()
    log = lambda *m: print(f"[{time.time() - t_start:7.1f}s]", *m, flush=True)
    widths = [int(x) for x in a.w.split(",")]
    om = a.omega
    snaps = [int(s) for s in a.snaps.split(",")]
    evals = [int(s) for s in a.eval_fine_steps.split(",")]
    train_seeds = [int(s) for s in a.train_seeds.split(",")]

    feats = {w: [] for w in widths}
    targets = {w: [] for w in widths}
    rng = np.random.default_rng(0)
    for seed in train_seeds:
        filt = ct.fine_run(a.n_fine, seed, om, widths, snaps, log=log)
        for w in widths:
            sub = max(1, int(round(a.subsample * (4.0 / w) ** 3)))
            for s in snaps:
                F, T = ct.targets_and_features(filt[w][s], ct.coarse_omega(om, w))
                pick = rng.choice(F.shape[0], F.shape[0] // sub, replace=False) if sub > 1 else np.arange(F.shape[0])
                feats[w].append(F[pick])
                targets[w].append(T[pick])
        del filt
    # hold-out seed: reference filtered fields at every width
    ref = ct.fine_run(a.n_fine, a.test_seed, om, widths, sorted(set([0] + evals + snaps)), log=log)

    import torch
    from .lbm import MlpTrainer
    by_width = {}
    for wi, w in enumerate(widths):
        om_c = ct.coarse_omega(om, w)
        nc = a.n_fine // w
        kmax = min(42, nc // 2 - 2)
        Fw, Tw = np.concatenate(feats[w]), np.concatenate(targets[w])
        feats[w] = targets[w] = None
        log(f"w = {w}: training set {Fw.shape[0]} cells, nu_t* mean {Tw.mean():.3e} rms "
            f"{np.sqrt((Tw ** 2).mean()):.3e}")
        ncells = int(Fw.shape[0])
        blob0 = ct.make_initial_blob(Fw, Tw)
        blob, losses = ct.train(Fw, Tw, blob0, epochs=a.epochs, log=log)
        del Fw, Tw
        Fh, Th = ct.targets_and_features(ref[w][snaps[-1]], om_c)
        tr = MlpTrainer(blob)
        pred = tr.forward(torch.from_numpy(Fh).cuda()).cpu().numpy().astype(np.float64)
        tr.close()
        smag = Fh[:, 5].astype(np.float64)
        corr_mlp = float(np.corrcoef(pred, Th)[0, 1])
        corr_smag = float(np.corrcoef(smag, Th)[0, 1])
        log(f"w = {w}: a priori (hold-out seed) corr(nu_mlp, nu*) {corr_mlp:.3f}, corr(nu_smag, nu*) {corr_smag:.3f}")
        Eref = {s: ct.shell_spectrum(ref[w][s][1:4]) for s in evals}
        coarse_steps = [s // w for s in evals]
        les = {}
        for closure in ("none", "smag", "mlp"):
            spec = ct.les_run(ref[w][0], om_c, closure, coarse_steps, blob=blob, log=log)
            errs = {}
            for s in evals:
                E = spec.get(s // w)
                errs[str(s // w)] = (ct.spectrum_error(E, Eref[s], kmax)
                                     if E is not None and np.all(np.isfinite(E)) else None)
            ke = {str(s // w): float(spec[s // w][1:].sum()) if s // w in spec else None for s in evals}
            les[closure] = {"spectrum_log_error": errs, "resolved_ke": ke,
                            "spectra": {str(k): v[:kmax + 1].tolist() for k, v in spec.items()}}
            log(f"w = {w}: LES {closure}: log-spectrum error {errs}")
        last = str(coarse_steps[-1])
        ke_ref = {str(s // w): float(Eref[s][1:].sum()) for s in evals}
        for c in les:
            # resolved kinetic energy against the reference, and the log-spectrum
            # error over the lower half of the compared range (the scales an
            # eddy viscosity acts on most, away from the grid-scale deficit)
            les[c]["resolved_ke_rel_error"] = {k: (abs(v / ke_ref[k] - 1.0) if v is not None else None)
                                               for k, v in les[c]["resolved_ke"].items()}
            les[c]["spectrum_log_error_lower_half"] = {
                str(s // w): (ct.spectrum_error(np.array(les[c]["spectra"][str(s // w)]), Eref[s], kmax // 2)
                              if str(s // w) in les[c]["spectra"] else None) for s in evals}
        gain = {}
        for other in ("none", "smag"):
            e_m, e_o = les["mlp"]["spectrum_log_error"][last], les[other]["spectrum_log_error"][last]
            gain[f"mlp_vs_{other}"] = (e_o / e_m) if (e_m and e_o) else None
            k_m, k_o = les["mlp"]["resolved_ke_rel_error"][last], les[other]["resolved_ke_rel_error"][last]
            gain[f"mlp_vs_{other}_resolved_ke"] = (k_o / k_m) if (k_m and k_o) else None
            h_m, h_o = les["mlp"]["spectrum_log_error_lower_half"][last], les[other]["spectrum_log_error_lower_half"][last]
            gain[f"mlp_vs_{other}_lower_half"] = (h_o / h_m) if (h_m and h_o) else None
        wpath = a.weights if wi == 0 else a.weights.replace(".npy", f"_w{w}.npy")
        os.makedirs(os.path.dirname(wpath) or ".", exist_ok=True)
        np.save(wpath, blob.astype(np.float32))
        by_width[str(w)] = {
            "coarse_grid": nc, "omega_c": om_c, "kmax": kmax, "weights": wpath,
            "training_cells": ncells,
            "loss_per_epoch": losses, "a_priori_corr": {"mlp": corr_mlp, "smag": corr_smag},
            "les": les, "reference_resolved_ke": ke_ref,
            "reference_spectra": {str(s // w): Eref[s][:kmax + 1].tolist() for s in evals},
            "last_coarse_step": int(last),
            "spectrum_log_error_at_last_step": {c: les[c]["spectrum_log_error"][last] for c in les},
            "resolved_ke_rel_error_at_last_step": {c: les[c]["resolved_ke_rel_error"][last] for c in les},
            "spectrum_log_error_lower_half_at_last_step": {c: les[c]["spectrum_log_error_lower_half"][last]
                                                           for c in les},
            "a_priori_gain": corr_mlp / corr_smag if corr_smag else None,
            "gain_error_ratio_at_last_step": gain,
        }
        log(f"w = {w}: gain (error of the other / error of the network) {json.dumps(gain)}")
    out = {
        "workload": f"{a.n_fine}^3 fine runs, omega {om}, box filters {widths} -> coarse LES",
        "train_seeds": a.train_seeds, "test_seed": a.test_seed, "snapshots_fine": snaps,
        "epochs": a.epochs, "by_width": by_width, "wall_s": time.time() - t_start,
    }
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    log("done")
    return out


if __name__ == "__main__":
    main(sys.argv[1:])
