"""Training and a-posteriori evaluation of the learned eddy-viscosity closure.

Pipeline (an extension beyond the paper, whose LES names no subgrid model):
  1. fine runs of this solver on a periodic n_f^3 box (random-phase initial
     field, seeds), box-filtered on the device (lbm_get_filtered) to the
     coarse n_c^3 grid at chosen steps;
  2. on the coarse grid: resolved strain S from central differences of the
     filtered velocity, subgrid stress tau = mean(u u) - mean(u) mean(u),
     target nu_t* = max(0, -dev(tau):S / (2 S:S));
  3. closure inputs as the coarse LES will see them: the pre-collision
     non-equilibrium stress per unit density is -(2/3)[tau_s dev(S) +
     tau_b tr(S)/3 I] with tau_s = 3 (nu0 + nu_t*) + 1/2 and tau_b = 1, and
     the inputs are its invariants, the norm of its deviator, rho - 1 and the
     Smagorinsky viscosity for Cs = 0.1;
  4. training on the device (lbm_mlp_* kernels, Adam);
  5. coarse LES (lbm_step with no model / Smagorinsky / the network) from the
     filtered initial field, compared with the filtered fine run through shell
     energy spectra at matched times (acoustic scaling: the coarse time step is
     w fine steps).
Steps 2-3 are offline data preparation on the host (NumPy); every step of
the solver and of the network runs in the HIP library.
"""
from __future__ import annotations

import numpy as np

import workloads
from .lbm import Lbm, MlpTrainer

NU_CS = 0.1


def nu_of(omega):
    return (1.0 / omega - 0.5) / 3.0


def coarse_omega(omega_fine, w):
    """acoustic scaling: dx and dt both grow by w, so nu (lattice units) / w"""
    return 1.0 / (3.0 * nu_of(omega_fine) / w + 0.5)


def _grad(u):
    """periodic central differences: g[a][b] = d u_a / d x_b, u is (3, z, y, x)"""
    g = np.empty((3, 3) + u.shape[1:])
    for a in range(3):
        for b, ax in enumerate((2, 1, 0)):  # x, y, z axes of the (z, y, x) array
            g[a, b] = 0.5 * (np.roll(u[a], -1, axis=ax) - np.roll(u[a], 1, axis=ax))
    return g


def targets_and_features(filt, omega_c):
    """filt: [10, z, y, x] block means (rho, u, uu). Returns (features [m, 6]
    float32, nu_t* [m] float64)."""
    rho = filt[0]
    u = filt[1:4]
    uu = {(0, 0): filt[4], (1, 1): filt[5], (2, 2): filt[6], (0, 1): filt[7], (0, 2): filt[8], (1, 2): filt[9]}
    tau = np.empty((3, 3) + rho.shape)
    for (a, b), v in uu.items():
        tau[a, b] = v - u[a] * u[b]
        tau[b, a] = tau[a, b]
    g = _grad(u)
    S = 0.5 * (g + g.transpose(1, 0, 2, 3, 4))
    trS = S[0, 0] + S[1, 1] + S[2, 2]
    trT = tau[0, 0] + tau[1, 1] + tau[2, 2]
    eye = np.eye(3)[:, :, None, None, None]
    Sd = S - eye * (trS / 3.0)
    Td = tau - eye * (trT / 3.0)
    SS = np.einsum("ab...,ab...->...", Sd, Sd)
    TS = np.einsum("ab...,ab...->...", Td, Sd)
    nu_t = np.maximum(0.0, -TS / (2.0 * np.maximum(SS, 1e-30)))
    tau_s = 3.0 * (nu_of(omega_c) + nu_t) + 0.5
    A = -(2.0 / 3.0) * (tau_s * Sd + eye * (trS / 3.0))
    feats = invariant_features(A, rho, omega_c)
    return np.ascontiguousarray(feats.reshape(6, -1).T, dtype=np.float32), nu_t.reshape(-1)


def invariant_features(A, rho, omega_c):
    """(I1, I2, I3 of A, |dev A|, rho - 1, Smagorinsky nu_t for Cs = 0.1)"""
    i1 = A[0, 0] + A[1, 1] + A[2, 2]
    tr2 = np.einsum("ab...,ba...->...", A, A)
    i2 = 0.5 * (i1 * i1 - tr2)
    i3 = (A[0, 0] * (A[1, 1] * A[2, 2] - A[1, 2] * A[2, 1])
          - A[0, 1] * (A[1, 0] * A[2, 2] - A[1, 2] * A[2, 0])
          + A[0, 2] * (A[1, 0] * A[2, 1] - A[1, 1] * A[2, 0]))
    eye = np.eye(3)[:, :, None, None, None]
    Ad = A - eye * (i1 / 3.0)
    q = np.sqrt(np.einsum("ab...,ab...->...", Ad, Ad))
    tau0 = 1.0 / omega_c
    tau = 0.5 * (tau0 + np.sqrt(tau0 * tau0 + 18.0 * np.sqrt(2.0) * NU_CS ** 2 * q))
    return np.stack([i1, i2, i3, q, rho - 1.0, (tau - tau0) / 3.0])


def shell_spectrum(u):
    return workloads.shell_spectrum(u)


def fine_run(n_fine, seed, omega, widths, snap_steps, log=print, storage="f32"):
    """Fine run; returns {w: {step: filtered [10, n/w...]}} for the requested
    filter widths and steps (one run serves every width)."""
    sim = Lbm(n_fine, n_fine, n_fine, omega=omega, storage=storage)
    rho, u = workloads.random_phase_field(n_fine, seed=seed)
    sim.init_fields(rho, u)
    del rho, u
    out = {w: {} for w in widths}
    for s in sorted(snap_steps):
        sim.step(s - sim.time)
        for w in widths:
            out[w][s] = sim.filtered(w)
        log(f"fine run seed {seed}: step {s} filtered ({', '.join(str(w) for w in widths)})")
    sim.close()
    return out


def train(feats, targets, blob0, epochs=8, batch=4096, lr=2e-3, seed=0, log=print):
    """Adam on the device; returns (trained blob, loss per epoch)."""
    import torch
    tr = MlpTrainer(blob0)
    F = torch.from_numpy(np.ascontiguousarray(feats, dtype=np.float32)).cuda()
    Y = torch.from_numpy(np.ascontiguousarray(targets / blob0[-1], dtype=np.float32)).cuda()
    m = F.shape[0]
    gen = torch.Generator(device="cuda").manual_seed(seed)
    losses = []
    for e in range(epochs):
        perm = torch.randperm(m, device="cuda", generator=gen)
        Fp, Yp = F[perm].contiguous(), Y[perm].contiguous()
        lr_e = lr * (0.5 ** (e // 5))
        for b in range(0, m - batch + 1, batch):
            tr.loss_grad(Fp[b:b + batch], Yp[b:b + batch])
            tr.adam_step(lr=lr_e)
        losses.append(tr.take_loss())
        log(f"training epoch {e}: loss {losses[-1]:.4e}")
    blob = tr.get_params().astype(np.float64)
    tr.close()
    return blob, losses


def training_throughput(batches=(4096, 65536), iters=200, seed=0, log=print):
    """Samples per second of one training iteration (forward + backward on
    the device, loss and gradient, then one Adam update) and of inference,
    on seeded synthetic features (the kernels' cost does not depend on the
    values), timed with HIP events on the trainer's stream."""
    import torch
    rng = np.random.default_rng(seed)
    feats = rng.standard_normal((max(batches), 6))
    targets = np.abs(rng.standard_normal(max(batches)))
    tr = MlpTrainer(make_initial_blob(feats, targets, seed))
    F = torch.from_numpy(feats.astype(np.float32)).cuda()
    Y = torch.from_numpy((targets / np.sqrt(np.mean(targets ** 2))).astype(np.float32)).cuda()
    out = {}
    for b in batches:
        fb, yb = F[:b].contiguous(), Y[:b].contiguous()
        for _ in range(10):
            tr.loss_grad(fb, yb)
            tr.adam_step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(tr.stream)
        for _ in range(iters):
            tr.loss_grad(fb, yb)
            tr.adam_step()
        e1.record(tr.stream)
        torch.cuda.synchronize()
        ms_train = e0.elapsed_time(e1) / iters
        tr.forward(fb)
        torch.cuda.synchronize()
        e0.record(tr.stream)
        for _ in range(iters):
            tr.forward(fb)
        e1.record(tr.stream)
        torch.cuda.synchronize()
        ms_inf = e0.elapsed_time(e1) / iters
        out[str(b)] = {"train_ms_per_iteration": ms_train, "train_samples_per_s": b / (ms_train * 1e-3),
                       "inference_ms": ms_inf, "inference_samples_per_s": b / (ms_inf * 1e-3)}
        log(f"closure training batch {b}: {b / (ms_train * 1e-3):.3e} samples/s "
            f"({ms_train * 1e3:.1f} us per iteration), inference {b / (ms_inf * 1e-3):.3e} samples/s")
    tr.take_loss()
    tr.close()
    return out


def make_initial_blob(feats, targets, seed=0):
    """He-initialised network with the training set's feature statistics and
    the target rms as output scale."""
    rng = np.random.default_rng(seed)
    blob = np.zeros(1326)
    blob[0:192] = rng.standard_normal(192) * np.sqrt(2.0 / 6.0)
    blob[224:1248] = rng.standard_normal(1024) * np.sqrt(2.0 / 32.0)
    blob[1280:1312] = rng.standard_normal(32) * np.sqrt(1.0 / 32.0)
    blob[192:224] = 0.01
    blob[1248:1280] = 0.01
    blob[1313:1319] = feats.mean(axis=0)
    blob[1319:1325] = np.maximum(feats.std(axis=0), 1e-30)
    blob[1325] = max(float(np.sqrt(np.mean(targets ** 2))), 1e-12)
    return blob.astype(np.float32).astype(np.float64)


def les_run(filt0, omega_c, closure, steps_list, blob=None, log=print):
    """Coarse LES from a filtered field; returns {step: shell spectrum}."""
    n = filt0.shape[-1]
    sim = Lbm(n, n, n, omega=omega_c, closure=closure, cs_smag=NU_CS, check_every=0)
    if closure == "mlp":
        sim.set_closure_weights(blob)
    sim.init_fields(filt0[0], filt0[1:4])
    spectra = {}
    for s in sorted(steps_list):
        sim.step(s - sim.time)
        _, u = sim.fields()
        spectra[s] = shell_spectrum(u)
        if not np.all(np.isfinite(spectra[s])):
            log(f"LES {closure}: non-finite field at step {s}")
            break
        log(f"LES {closure}: step {s}")
    sim.close()
    return spectra


def spectrum_error(E, Eref, kmax):
    k = np.arange(1, kmax + 1)
    return float(np.mean(np.abs(np.log(E[k]) - np.log(Eref[k]))))
