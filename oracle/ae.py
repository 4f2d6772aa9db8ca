"""Autoencoder oracle for the learned pre-screen (FP64 numpy).

TEST INFRASTRUCTURE ONLY (never imported by the product package).

The learned pre-screen is not part of the paper; the network and its training
are a plain reading of a small dense autoencoder:
  64 -> 128 -> 32 -> 128 -> 64, ReLU after the three hidden layers, linear
  output, loss = mean over rows and features of (y - x)^2, Adam with bias
  correction (Kingma & Ba 2015), Xavier-uniform initial weights (Glorot &
  Bengio 2010), zero biases.
Inputs are per-rank iteration profiles: x[r, i, :] = (T[r, i, :] - mu) / sigma
with per-region mean and standard deviation over the training tensors' valid
cells.  Rank score = max over regions of the mean over the rank's valid
iterations of the squared reconstruction error.

`bf16=True` rounds every matrix-product operand (activations, weights and the
back-propagated errors) to bfloat16 (round to nearest even) at the points
where the GPU kernels do, keeping FP64 accumulation; `bf16=False` is plain
FP64.
"""
from __future__ import annotations

import numpy as np

DIMS = (64, 128, 32, 128, 64)
N_LAYERS = 4


# ---------------------------------------------------------------------------
# bfloat16 rounding (round to nearest, ties to even) of FP32 values
# ---------------------------------------------------------------------------

def to_bf16(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) through FP32; returns FP64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


# ---------------------------------------------------------------------------
# SplitMix64 counter draws, the same definition the GPU initialiser uses
# ---------------------------------------------------------------------------

_M = np.uint64(0xFFFFFFFFFFFFFFFF)


def _mix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z + np.uint64(0x9E3779B97F4A7C15)) & _M
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M
        return z ^ (z >> np.uint64(31))


def init_params(seed: int) -> dict:
    """Xavier-uniform weights W_l[out, in] ~ U(-a, a), a = sqrt(6/(in+out)),
    drawn as u = SplitMix64(seed-mixed counter) -> (u >> 11 + 0.5) / 2^53,
    w = (2u - 1) * a in FP64, stored as FP32.  Biases are zero."""
    p = {}
    s = _mix64(np.array([seed], dtype=np.uint64))[0]
    for l in range(N_LAYERS):
        fin, fout = DIMS[l], DIMS[l + 1]
        idx = np.arange(fout * fin, dtype=np.uint64)
        with np.errstate(over="ignore"):
            key = (s ^ _mix64(np.array([l + 1], dtype=np.uint64))[0])
            z = _mix64((key + idx * np.uint64(0x9E3779B97F4A7C15)) & _M)
        u = ((z >> np.uint64(11)).astype(np.float64) + 0.5) / 9007199254740992.0
        a = np.sqrt(6.0 / (fin + fout))
        p[f"W{l + 1}"] = ((2.0 * u - 1.0) * a).astype(np.float32).astype(np.float64).reshape(fout, fin)
        p[f"b{l + 1}"] = np.zeros(fout)
    return p


def gaussian_noise(key: int, rows, n_features: int = 64) -> np.ndarray:
    """Standard normal draws N_key(j, c) for row ids `rows` and features
    c < n_features: base = M(key ^ M(64 j + c)), z1 = M(base),
    z2 = M(base ^ 0xD1B54A32D192ED03), u1 = ((z1 >> 40) + 1/2) / 2^24,
    u2 = (z2 >> 40) / 2^24, N = sqrt(-2 ln u1) cos(2 pi u2) (Box & Muller
    1958), M the SplitMix64 finaliser; in FP64."""
    j = np.asarray(rows, dtype=np.uint64)[:, None]
    c = np.arange(n_features, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        ctr = (j * np.uint64(n_features) + c) & _M
        base = _mix64(np.uint64(key) ^ _mix64(ctr))
        z1 = _mix64(base)
        z2 = _mix64(base ^ np.uint64(0xD1B54A32D192ED03))
    u1 = ((z1 >> np.uint64(40)).astype(np.float64) + 0.5) / 16777216.0
    u2 = (z2 >> np.uint64(40)).astype(np.float64) / 16777216.0
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


# ---------------------------------------------------------------------------
# Normalisation
# ---------------------------------------------------------------------------

def fit_norm(tensors, iters_list):
    """Per-region mean and (population) standard deviation over the valid
    cells of all training tensors, accumulated in FP64; returned as FP32."""
    G = tensors[0].shape[2]
    s = np.zeros(G)
    q = np.zeros(G)
    n = 0
    for T, it in zip(tensors, iters_list):
        R, I, _ = T.shape
        valid = np.arange(I)[None, :] < np.asarray(it)[:, None]
        x = T[valid].astype(np.float64)
        s += x.sum(0)
        n += x.shape[0]
    mu = s / n
    for T, it in zip(tensors, iters_list):
        R, I, _ = T.shape
        valid = np.arange(I)[None, :] < np.asarray(it)[:, None]
        x = T[valid].astype(np.float64)
        q += ((x - mu) ** 2).sum(0)
    sd = np.sqrt(q / n)
    sd[sd == 0] = 1.0
    return mu.astype(np.float32), sd.astype(np.float32)


def normalize(T, mu, sd):
    """x = ((float)T - mu) * (1 / sd), in FP32 as the GPU does."""
    inv = (np.float32(1.0) / np.asarray(sd, np.float32)).astype(np.float32)
    return ((T.astype(np.float32) - np.asarray(mu, np.float32)) * inv).astype(np.float32)


# ---------------------------------------------------------------------------
# Forward / backward
# ---------------------------------------------------------------------------

def forward(p: dict, X: np.ndarray, bf16: bool = False):
    """X [B, 64] -> (pre-activations z_l, activations a_l); a_0 = X."""
    rnd = to_bf16 if bf16 else (lambda v: np.asarray(v, np.float64))
    a = [np.asarray(X, np.float64)]
    z = []
    for l in range(N_LAYERS):
        W, b = p[f"W{l + 1}"], p[f"b{l + 1}"]
        zl = rnd(a[-1]) @ rnd(W).T + b
        if bf16:
            zl = zl.astype(np.float32).astype(np.float64)
        z.append(zl)
        a.append(np.maximum(zl, 0.0) if l < N_LAYERS - 1 else zl)
    return z, a


def loss_and_grads(p: dict, X: np.ndarray, bf16: bool = False, X_in=None):
    """Mean squared reconstruction error and its gradients.  X_in (default X)
    is what the network sees; the error is taken against X (a denoising step
    when X_in is a corrupted copy of X)."""
    rnd = to_bf16 if bf16 else (lambda v: np.asarray(v, np.float64))
    X = np.asarray(X, np.float64)
    B = X.shape[0]
    z, a = forward(p, X if X_in is None else np.asarray(X_in, np.float64), bf16)
    y = a[-1]
    diff = y - X
    loss = float((diff ** 2).sum() / (B * DIMS[-1]))
    g = {}
    d = 2.0 * diff / (B * DIMS[-1])                  # dL/dz_4
    for l in range(N_LAYERS - 1, -1, -1):
        W = p[f"W{l + 1}"]
        g[f"W{l + 1}"] = rnd(d).T @ rnd(a[l])
        g[f"b{l + 1}"] = d.sum(0)
        if l > 0:
            da = rnd(d) @ rnd(W)
            d = da * (z[l - 1] > 0)
    return loss, g


def adam_update(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1) on FP64 copies of the parameters."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def robust_z(v: np.ndarray) -> np.ndarray:
    """Robust z-score of a sample: (v - median) / (1.4826 * MAD); when MAD is 0,
    1.253314 * mean absolute deviation replaces the denominator; when that is
    0 too, every z is 0.  Medians of an even count average the two middle
    values (the same rule as the exact scan's second stage)."""
    v = np.asarray(v, np.float64)
    if v.size == 0:
        return v.copy()
    med = np.median(v)
    dev = np.abs(v - med)
    mad = np.median(dev)
    if mad > 0:
        return (v - med) / (1.4826 * mad)
    mean_ad = dev.mean()
    if mean_ad > 0:
        return (v - med) / (1.253314 * mean_ad)
    return np.zeros_like(v)


def robust_z32(v) -> np.ndarray:
    """robust_z in IEEE FP32, one operation at a time: med = (a + b) * 0.5 of
    the two middle values (a for an odd count), MAD likewise over |v - med|,
    scale = 1.4826 * MAD, else 1.253314 * mean |v - med| (the mean summed in
    FP64, then rounded), else 0; z = (v - med) / scale."""
    v = np.asarray(v, np.float32)
    n = v.size
    if n == 0:
        return v.copy()
    f = np.float32
    s = np.sort(v)
    med = s[(n - 1) // 2] if n % 2 else f((s[n // 2 - 1] + s[n // 2]) * f(0.5))
    dev = np.abs(v - med).astype(np.float32)
    d = np.sort(dev)
    mad = d[(n - 1) // 2] if n % 2 else f((d[n // 2 - 1] + d[n // 2]) * f(0.5))
    if mad > 0:
        scale = f(f(1.4826) * mad)
    else:
        mean_ad = dev.astype(np.float64).sum() / n
        scale = f(1.253314 * mean_ad) if mean_ad > 0 else f(0)
    if scale == 0:
        return np.zeros(n, np.float32)
    return ((v - med) / scale).astype(np.float32)


def rank_scores(p: dict, T: np.ndarray, iters, mu, sd, bf16: bool = False,
                kind: int = 0) -> np.ndarray:
    """kind 0: score[r] = max_g mean_{i < iters[r]} (y - x)^2 (reconstruction
    error); kind 1: score[r] = max_g |m(r,g)| with m(r,g) = mean_{i < iters[r]}
    (y - x) (persistent residual of a region over the rank's iterations);
    kind 2: score[r] = max_g |robust_z32 over ranks with iterations of
    m(., g) rounded to FP32| (the second stage in FP32).  Ranks without
    iterations score 0 and take no part in kind 2."""
    R, I, G = T.shape
    X = normalize(T, mu, sd)
    err = np.zeros((R, G))
    m = np.zeros((R, G))
    active = np.zeros(R, bool)
    for r in range(R):
        n = int(min(iters[r], I)) if iters is not None else I
        if n <= 0:
            continue
        active[r] = True
        _, a = forward(p, X[r, :n], bf16)
        res = a[-1] - X[r, :n].astype(np.float64)
        err[r] = (res ** 2).mean(0)
        m[r] = res.mean(0)
    if kind == 0:
        return np.where(active, err.max(1), 0.0)
    if kind == 1:
        return np.where(active, np.abs(m).max(1), 0.0)
    out = np.zeros(R)
    for g in range(G):
        z = robust_z32(m[active, g].astype(np.float32))
        out[active] = np.maximum(out[active], np.abs(z).astype(np.float64))
    return out
