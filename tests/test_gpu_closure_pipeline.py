"""End-to-end run of the closure pipeline at a small size: fine runs ->
device box filter at two widths -> targets/features -> device training ->
coarse LES with no model, Smagorinsky and the network, whose a-posteriori
errors and gain ratios are printed and stored (the full-size run is the
committed results/closure_les.json)."""
import json
import math
import os

import pytest

pytestmark = pytest.mark.gpu


def test_small_pipeline_runs_end_to_end(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2402_13171_amd import train_closure
    out = tmp_path / "c.json"
    res = train_closure.main(["--n-fine", "64", "--w", "4,2", "--train-seeds", "0,1",
                              "--test-seed", "2", "--snaps", "100,200", "--eval-fine-steps", "100,200",
                              "--subsample", "1", "--epochs", "3", "--out", str(out),
                              "--weights", str(tmp_path / "w.npy")])
    assert os.path.exists(out) and os.path.exists(tmp_path / "w.npy") and os.path.exists(tmp_path / "w_w2.npy")
    stored = json.loads(out.read_text())
    # every (4 / w)^3-th cell at width w: the same number of samples per width
    for w, cells in (("4", 2 * 2 * 16 ** 3), ("2", 2 * 2 * 32 ** 3 // 8)):
        r = res["by_width"][w]
        assert r["training_cells"] == cells
        assert r["loss_per_epoch"][-1] < r["loss_per_epoch"][0]
        errs = r["spectrum_log_error_at_last_step"]
        gain = r["gain_error_ratio_at_last_step"]
        print(f"w = {w}: log-spectrum error at coarse step {r['last_coarse_step']}: no model {errs['none']:.3f}, "
              f"Smagorinsky {errs['smag']:.3f}, network {errs['mlp']:.3f}; gain vs no model "
              f"{gain['mlp_vs_none']:.3f}, vs Smagorinsky {gain['mlp_vs_smag']:.3f}")
        for closure in ("none", "smag", "mlp"):
            assert errs[closure] is not None and math.isfinite(errs[closure])
        for k in ("mlp_vs_none", "mlp_vs_smag"):
            assert math.isfinite(gain[k]) and gain[k] > 0
            assert stored["by_width"][w]["gain_error_ratio_at_last_step"][k] == pytest.approx(gain[k])
