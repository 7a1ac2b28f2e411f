"""Train the learned closure on filtered fine runs and evaluate it in a coarse
LES against no model and Smagorinsky (see closure_training.py).

    python -m paper_2402_13171_amd.train_closure --out results/closure_les128.json

Defaults: fine 512^3, omega 1.9, filter width 4 (coarse 128^3), training
seeds 0-3 with snapshots at fine steps 2000/4000/6000/8000 (every 8th coarse
cell), hold-out seed 7; coarse LES for 2000 steps compared with the filtered
fine run at fine steps 2000/4000/8000 (coarse 500/1000/2000), k in [1, 42].
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
    ap.add_argument("--w", type=int, default=4)
    ap.add_argument("--omega", type=float, default=1.9)
    ap.add_argument("--train-seeds", default="0,1,2,3")
    ap.add_argument("--test-seed", type=int, default=7)
    ap.add_argument("--fine-steps", type=int, default=8000)
    ap.add_argument("--snaps", default="2000,4000,6000,8000")
    ap.add_argument("--eval-fine-steps", default="2000,4000,8000")
    ap.add_argument("--subsample", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--out", default="results/closure_les128.json")
    ap.add_argument("--weights", default="results/closure_weights.npy")
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
    w, om = a.w, a.omega
    om_c = ct.coarse_omega(om, w)
    snaps = [int(s) for s in a.snaps.split(",")]
    evals = [int(s) for s in a.eval_fine_steps.split(",")]
    nc = a.n_fine // w
    kmax = min(42, nc // 2 - 2)

    feats, targets = [], []
    rng = np.random.default_rng(0)
    for seed in [int(s) for s in a.train_seeds.split(",")]:
        filt = ct.fine_run(a.n_fine, seed, om, w, snaps, log=log)
        for s in snaps:
            F, T = ct.targets_and_features(filt[s], om_c)
            pick = rng.choice(F.shape[0], F.shape[0] // a.subsample, replace=False)
            feats.append(F[pick])
            targets.append(T[pick])
        del filt
    feats = np.concatenate(feats)
    targets = np.concatenate(targets)
    log(f"training set: {feats.shape[0]} cells, nu_t* mean {targets.mean():.3e} rms "
        f"{np.sqrt((targets ** 2).mean()):.3e}")
    blob0 = ct.make_initial_blob(feats, targets)
    blob, losses = ct.train(feats, targets, blob0, epochs=a.epochs, log=log)

    # hold-out seed: reference filtered fields and a-priori error
    ref = ct.fine_run(a.n_fine, a.test_seed, om, w, sorted(set([0] + evals + snaps)), log=log)
    Fh, Th = ct.targets_and_features(ref[snaps[-1]], om_c)
    import torch
    from .lbm import MlpTrainer
    tr = MlpTrainer(blob)
    pred = tr.forward(torch.from_numpy(Fh).cuda()).cpu().numpy().astype(np.float64)
    tr.close()
    smag = Fh[:, 5].astype(np.float64)
    corr_mlp = float(np.corrcoef(pred, Th)[0, 1])
    corr_smag = float(np.corrcoef(smag, Th)[0, 1])
    log(f"a priori (hold-out seed): corr(nu_mlp, nu*) {corr_mlp:.3f}, corr(nu_smag, nu*) {corr_smag:.3f}")

    Eref = {s: ct.shell_spectrum(ref[s][1:4]) for s in evals}
    coarse_steps = [s // w for s in evals]
    results = {}
    for closure in ("none", "smag", "mlp"):
        spec = ct.les_run(ref[0], om_c, closure, coarse_steps, blob=blob, log=log)
        errs = {}
        for s in evals:
            E = spec.get(s // w)
            errs[str(s // w)] = ct.spectrum_error(E, Eref[s], kmax) if E is not None and np.all(np.isfinite(E)) else None
        ke = {str(s // w): float(spec[s // w][1:].sum()) if s // w in spec else None for s in evals}
        results[closure] = {"spectrum_log_error": errs, "resolved_ke": ke,
                            "spectra": {str(k): v[:kmax + 1].tolist() for k, v in spec.items()}}
        log(f"LES {closure}: log-spectrum error {errs}")
    ke_ref = {str(s // w): float(Eref[s][1:].sum()) for s in evals}
    last = str(coarse_steps[-1])
    gain = {}
    for other in ("none", "smag"):
        e_m, e_o = results["mlp"]["spectrum_log_error"][last], results[other]["spectrum_log_error"][last]
        gain[f"mlp_vs_{other}"] = (e_o / e_m) if (e_m and e_o) else None
    out = {
        "workload": f"{a.n_fine}^3 fine runs, omega {om}, {w}^3 box filter -> {nc}^3 LES, omega_c {om_c:.5f}",
        "train_seeds": a.train_seeds, "test_seed": a.test_seed, "snapshots_fine": snaps,
        "training_cells": int(feats.shape[0]), "epochs": a.epochs,
        "loss_per_epoch": losses, "a_priori_corr": {"mlp": corr_mlp, "smag": corr_smag},
        "kmax": kmax, "les": results, "reference_resolved_ke": ke_ref,
        "reference_spectra": {str(s // w): Eref[s][:kmax + 1].tolist() for s in evals},
        "gain_error_ratio_at_last_step": gain, "wall_s": time.time() - t_start,
    }
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    np.save(a.weights, blob.astype(np.float32))
    log("done:", json.dumps(gain))
    return out


if __name__ == "__main__":
    main(sys.argv[1:])
