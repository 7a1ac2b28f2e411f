"""GPU <-> oracle parity of the learned closure: matrix-core inference (on
given features and fused in the lattice kernel), loss/gradient kernels and
the Adam update, against the FP64 NumPy/C oracle in its bfloat16-emulating
mode (same operands rounded to bfloat16, FP64 arithmetic)."""
import numpy as np
import pytest

import oracle
from oracle import mlp_ref

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def make_blob(seed=0):
    rng = np.random.default_rng(seed)
    mu = rng.normal(0, 1e-3, 6)
    sigma = rng.uniform(0.5, 2.0, 6) * 1e-3
    blob = mlp_ref.init_blob(seed=seed, mu=mu, sigma=sigma, nu_scale=2e-3)
    return blob.astype(np.float32).astype(np.float64)  # representable in float32


def make_feats(rng, m):
    return (rng.normal(0, 2e-3, (m, 6))).astype(np.float32)


def test_forward_matches_emulated_oracle():
    _need_gpu()
    import torch
    from paper_2402_13171_amd.lbm import MlpTrainer
    blob = make_blob(1)
    rng = np.random.default_rng(2)
    m = 5000 + 37  # ragged against the 64-cell waves
    feats = make_feats(rng, m)
    tr = MlpTrainer(blob)
    got = tr.forward(torch.from_numpy(feats).cuda()).cpu().numpy().astype(np.float64)
    ref, _ = mlp_ref.forward(blob, feats.astype(np.float64), emulate_bf16=True)
    rel = np.abs(got - ref) / np.abs(ref)
    print(f"mlp forward: median rel {np.median(rel):.2e}, p99 {np.percentile(rel, 99):.2e}, max {rel.max():.2e}")
    assert np.percentile(rel, 99) <= 1e-4
    assert rel.max() <= 5e-3
    # the C oracle agrees with the NumPy oracle on the same inputs
    c_ref = np.array([oracle.mlp_nu_t(blob, f, True) for f in feats[:64].astype(np.float64)])
    assert np.allclose(c_ref, ref[:64], rtol=1e-12)


def test_gradient_matches_emulated_oracle():
    _need_gpu()
    import torch
    from paper_2402_13171_amd.lbm import MlpTrainer
    blob = make_blob(3)
    rng = np.random.default_rng(4)
    m = 1000
    feats = make_feats(rng, m)
    tgt = rng.uniform(0.2, 2.0, m).astype(np.float32)
    tr = MlpTrainer(blob)
    g = tr.loss_grad(torch.from_numpy(feats).cuda(), torch.from_numpy(tgt).cuda(), want_grad=True)
    L, gref = mlp_ref.loss_and_grad(blob, feats.astype(np.float64), tgt.astype(np.float64), emulate_bf16=True)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    _, gexact = mlp_ref.loss_and_grad(blob, feats.astype(np.float64), tgt.astype(np.float64))
    rel_exact = np.linalg.norm(g - gexact) / np.linalg.norm(gexact)
    print(f"mlp gradient: rel norm error {rel:.2e} (emulated), {rel_exact:.2e} (exact FP64)")
    # The network is specified with bfloat16 weights and activations on the
    # matrix cores: the oracle of that arithmetic is the FP64 oracle with the
    # same operands rounded to bfloat16, held to 1e-4 here (the 1e-3 bar on
    # gradients with a margin). Against the network with unrounded FP64
    # operands the difference is the bfloat16 rounding itself: 2^-9 relative
    # per operand through products of several rounded factors, about 1e-2 in
    # norm; that gate only checks the size of the effect.
    assert rel <= 1e-4
    assert rel_exact <= 3e-2
    assert tr.take_loss() == pytest.approx(L, rel=1e-5)


def test_adam_step_matches_oracle():
    _need_gpu()
    import torch
    from paper_2402_13171_amd.lbm import MlpTrainer
    blob = make_blob(5)
    rng = np.random.default_rng(6)
    feats = make_feats(rng, 256)
    tgt = rng.uniform(0.2, 2.0, 256).astype(np.float32)
    tr = MlpTrainer(blob)
    g = tr.loss_grad(torch.from_numpy(feats).cuda(), torch.from_numpy(tgt).cuda(), want_grad=True)
    tr.adam_step(lr=1e-3)
    got = tr.get_params()
    p0 = blob[:1313]
    ref, _, _ = mlp_ref.adam_step(p0, g.astype(np.float64), np.zeros(1313), np.zeros(1313), 1, lr=1e-3)
    assert np.abs(got[:1313] - ref).max() <= 2e-6 * max(1.0, np.abs(p0).max())
    assert np.array_equal(got[1313:], blob[1313:].astype(np.float32))


def test_training_reduces_loss():
    """Fit a teacher network's output: the loss of the trained student falls
    below a tenth of the untrained student's loss on the same samples."""
    _need_gpu()
    import torch
    from paper_2402_13171_amd.lbm import MlpTrainer
    rng = np.random.default_rng(7)
    teacher = make_blob(8)
    student = make_blob(9)
    m = 1 << 15
    feats = make_feats(rng, m)
    y, _ = mlp_ref.forward(teacher, feats.astype(np.float64))
    y = (y / teacher[1325]).astype(np.float32)
    tr = MlpTrainer(student)
    F = torch.from_numpy(feats).cuda()
    Y = torch.from_numpy(y).cuda()
    for b in range(0, m, 4096):  # loss of the untrained student (no update)
        tr.loss_grad(F[b:b + 4096], Y[b:b + 4096])
    loss0 = tr.take_loss()
    losses = []
    for epoch in range(40):
        perm = torch.randperm(m, device="cuda", generator=torch.Generator(device="cuda").manual_seed(epoch))
        Fp, Yp = F[perm].contiguous(), Y[perm].contiguous()
        for b in range(0, m, 4096):
            tr.loss_grad(Fp[b:b + 4096], Yp[b:b + 4096])
            tr.adam_step(lr=3e-3)
        losses.append(tr.take_loss())
    print(f"untrained loss {loss0:.3e}; training loss per epoch:", " ".join(f"{v:.3e}" for v in losses[::5]),
          f"last {losses[-1]:.3e}")
    assert losses[-1] < loss0 / 10


def test_fused_closure_in_lattice_matches_oracle():
    _need_gpu()
    from paper_2402_13171_amd.lbm import Lbm
    n = 24
    blob = make_blob(10)
    rng = np.random.default_rng(11)
    u = rng.uniform(-0.05, 0.05, (3, n, n, n))
    rho = 1.0 + rng.uniform(-0.01, 0.01, (n, n, n))
    sim = Lbm(n, n, n, omega=1.95, closure="mlp")
    sim.set_closure_weights(blob)
    sim.init_fields(rho, u)
    ref = oracle.Grid(n, n, n, omega=1.95, closure=oracle.CLOSURE_MLP, mlp_emulate_bf16=True)
    ref.set_mlp(blob)
    ref.init_fields(rho, u)
    sim.step(7)
    ref.step(7)
    err = np.abs(sim.pops() - ref.get_pops()).max()
    print(f"fused closure: max population error after 7 steps {err:.2e}")
    assert err <= 2e-6
