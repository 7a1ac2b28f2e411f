"""End-to-end run of the closure pipeline at a small size: fine runs ->
device box filter -> targets/features -> device training -> coarse LES with
no model, Smagorinsky and the network (the full-size run is the committed
results/closure_les128.json)."""
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
    res = train_closure.main(["--n-fine", "64", "--w", "4", "--train-seeds", "0,1",
                              "--test-seed", "2", "--snaps", "100,200", "--eval-fine-steps", "100,200",
                              "--subsample", "1", "--epochs", "3", "--out", str(out),
                              "--weights", str(tmp_path / "w.npy")])
    assert os.path.exists(out)
    assert res["training_cells"] == 2 * 2 * 16 ** 3
    assert res["loss_per_epoch"][-1] < res["loss_per_epoch"][0]
    for closure in ("none", "smag", "mlp"):
        for v in res["les"][closure]["spectrum_log_error"].values():
            assert v is not None and math.isfinite(v)
    json.loads(out.read_text())
