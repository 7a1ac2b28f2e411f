"""FP64 NumPy reference of the learned eddy-viscosity closure: forward pass,
analytic backward pass and Adam update.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py). The paper runs an LES but
names no subgrid model; this per-cell network (6 -> 32 -> 32 -> 1, ReLU,
softplus output scaled by nu_scale) is an extension beyond the paper.

Parameter blob layout (1326 values, row-major matrices):
    W1[32][6] b1[32] W2[32][32] b2[32] w3[32] b3 | mu[6] sigma[6] nu_scale
The first 1313 entries are trainable; the normalisation and scale are not.

Training loss (per batch of B cells with targets y = nu_t / nu_scale):
    L = (1/B) sum_b (softplus(z_b) - y_b)^2
"""
from __future__ import annotations

import numpy as np

NPARAM = 1313
NBLOB = NPARAM + 13
SL = {
    "W1": (slice(0, 192), (32, 6)),
    "b1": (slice(192, 224), (32,)),
    "W2": (slice(224, 1248), (32, 32)),
    "b2": (slice(1248, 1280), (32,)),
    "w3": (slice(1280, 1312), (32,)),
    "b3": (slice(1312, 1313), (1,)),
    "mu": (slice(1313, 1319), (6,)),
    "sigma": (slice(1319, 1325), (6,)),
    "nu_scale": (slice(1325, 1326), (1,)),
}


def unpack(blob):
    blob = np.asarray(blob, dtype=np.float64)
    return {k: blob[s].reshape(sh) for k, (s, sh) in SL.items()}


def bf16(x):
    """Round to float32, then to bfloat16 (round to nearest even)."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    finite = (b & 0x7F800000) != 0x7F800000
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = np.where(finite, r, b.astype(np.uint32)).astype(np.uint32)
    return out.view(np.float32).astype(np.float64)


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def normalise(blob, feats, emulate_bf16=False):
    p = unpack(blob)
    if emulate_bf16:
        d = feats.astype(np.float32) - p["mu"].astype(np.float32)
        inv = (1.0 / p["sigma"]).astype(np.float32)
        return bf16((d * inv).astype(np.float32))
    return (feats - p["mu"]) / p["sigma"]


def forward(blob, feats, emulate_bf16=False):
    """feats: (B, 6). Returns (nu_t (B,), cache)."""
    p = unpack(blob)
    e = emulate_bf16
    r = bf16 if e else (lambda a: np.asarray(a, dtype=np.float64))
    f32 = (lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)) if e else r
    xh = normalise(blob, np.asarray(feats, dtype=np.float64), e)
    W1, W2 = r(p["W1"]), r(p["W2"])
    a1 = xh @ W1.T + f32(p["b1"])
    h1 = r(np.maximum(a1, 0.0))
    a2 = h1 @ W2.T + f32(p["b2"])
    h2 = np.maximum(a2, 0.0)
    z = h2 @ f32(p["w3"]) + f32(p["b3"])[0]
    nu = f32(p["nu_scale"])[0] * softplus(z)
    cache = {"xh": xh, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "z": z,
             "W1": W1, "W2": W2, "w3": f32(p["w3"])}
    return nu, cache


def loss_and_grad(blob, feats, target_scaled, emulate_bf16=False):
    """MSE loss on softplus(z) against target_scaled = nu_t/nu_scale and the
    gradient with respect to the 1313 trainable entries of the blob."""
    _, c = forward(blob, feats, emulate_bf16)
    B = feats.shape[0]
    sp = softplus(c["z"])
    diff = sp - target_scaled
    L = float(np.mean(diff * diff))
    dz = 2.0 * diff * sigmoid(c["z"]) / B                 # (B,)
    g = np.zeros(NPARAM)
    g[SL["w3"][0]] = c["h2"].T @ dz
    g[SL["b3"][0]] = dz.sum()
    da2 = np.outer(dz, c["w3"]) * (c["a2"] > 0)          # (B, 32)
    g[SL["W2"][0]] = (da2.T @ c["h1"]).reshape(-1)
    g[SL["b2"][0]] = da2.sum(axis=0)
    # with the bf16 emulation the backward data product takes da2 in bfloat16
    # (as the matrix cores do); the weight sums keep it in full precision
    da2_mm = bf16(da2) if emulate_bf16 else da2
    da1 = (da2_mm @ c["W2"]) * (c["a1"] > 0)             # (B, 32)
    g[SL["W1"][0]] = (da1.T @ c["xh"]).reshape(-1)
    g[SL["b1"][0]] = da1.sum(axis=0)
    return L, g


def adam_step(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) of the trainable entries; returns
    new (params, m, v). t is the 1-based step count."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    params = params - lr * mh / (np.sqrt(vh) + eps)
    return params, m, v


def init_blob(seed=0, mu=None, sigma=None, nu_scale=1e-3):
    """He-initialised weights, zero biases, given normalisation."""
    rng = np.random.default_rng(seed)
    blob = np.zeros(NBLOB)
    blob[SL["W1"][0]] = rng.standard_normal(192) * np.sqrt(2.0 / 6.0)
    blob[SL["W2"][0]] = rng.standard_normal(1024) * np.sqrt(2.0 / 32.0)
    blob[SL["w3"][0]] = rng.standard_normal(32) * np.sqrt(1.0 / 32.0)
    blob[SL["b1"][0]] = 0.01
    blob[SL["b2"][0]] = 0.01
    blob[SL["mu"][0]] = 0.0 if mu is None else mu
    blob[SL["sigma"][0]] = 1.0 if sigma is None else sigma
    blob[SL["nu_scale"][0]] = nu_scale
    return blob
