"""The no-allocation gradient entry point (lbm_mlp_loss_grad_noalloc) against
the allocating one (lbm_mlp_loss_grad), through the C ABI: same kernels and
the same fixed-order reduction, so gradient, loss and the Adam update that
follows agree bit for bit. Two calls in a row, the maximum batch (65536
samples) and then a smaller, ragged one (stale partials of the first call
stay in the shared scratch and must not leak into the second); a batch over
the limit is refused before any device work."""
import numpy as np
import pytest

from oracle import mlp_ref

pytestmark = pytest.mark.gpu


def _blob(seed):
    rng = np.random.default_rng(seed)
    blob = mlp_ref.init_blob(seed=seed, mu=rng.normal(0, 1e-3, 6), sigma=rng.uniform(0.5, 2.0, 6) * 1e-3,
                             nu_scale=2e-3)
    return blob.astype(np.float32).astype(np.float64)


def test_noalloc_gradient_matches_allocating_entry_point():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2402_13171_amd.lbm import MlpTrainer, LbmError, EINVAL
    blob = _blob(11)
    rng = np.random.default_rng(12)
    batches = []
    for m in (65536, 1000 + 37):
        feats = torch.from_numpy(rng.normal(0, 2e-3, (m, 6)).astype(np.float32)).cuda()
        tgt = torch.from_numpy(rng.uniform(0.2, 2.0, m).astype(np.float32)).cuda()
        batches.append((feats, tgt))
    ref_tr = MlpTrainer(blob)
    ref = []
    for feats, tgt in batches:
        g = ref_tr.loss_grad(feats, tgt, want_grad=True)
        ref.append((g, ref_tr.take_loss()))
    tr = MlpTrainer(blob)
    got = []
    for feats, tgt in batches:  # two calls in a row, the second smaller
        g = tr.loss_grad_noalloc(feats, tgt, want_grad=True)
        got.append((g, tr.take_loss()))
    for (gr, lr), (gg, lg), (feats, _) in zip(ref, got, batches):
        print(f"batch {feats.shape[0]}: loss {lg:.9e} (allocating entry point {lr:.9e}), "
              f"max |grad difference| {np.abs(gg - gr).max():.1e}", flush=True)
        assert np.array_equal(gg, gr)
        assert lg == lr
        assert np.isfinite(gg).all() and np.abs(gg).max() > 0
    # the gradient left on the device by the no-allocation call drives Adam
    # exactly as the allocating call's does
    ref_tr.adam_step(1e-3)
    tr.adam_step(1e-3)
    assert np.array_equal(tr.get_params(), ref_tr.get_params())
    # over the limit: refused, nothing launched, the trainer still usable
    big = torch.zeros((65537, 6), dtype=torch.float32, device="cuda")
    bigt = torch.zeros(65537, dtype=torch.float32, device="cuda")
    with pytest.raises(LbmError) as ei:
        tr.loss_grad_noalloc(big, bigt)
    assert ei.value.code == EINVAL
    feats, tgt = batches[1]
    g = tr.loss_grad_noalloc(feats, tgt, want_grad=True)
    g_ref = ref_tr.loss_grad(feats, tgt, want_grad=True)
    assert np.array_equal(g, g_ref)
    tr.close()
    ref_tr.close()
