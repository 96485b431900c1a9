"""CPU oracle of the learned surrogate (float64 numpy, bf16 rounding at storage points).

TEST INFRASTRUCTURE ONLY (see the package docstring): the plain definition the GPU
surrogate kernels are checked against. It shares no code with the HIP library.

The network (a small learned stand-in for the hybrid filter, trained on pairs that the
plain method produces; the paper itself has no learned component):
  x = g / M (float), six 3x3 convolutions with zero padding, 32 channels,
  Z_l[p, co] = sum_t sum_ci X[p + off_t, ci] * W_l[t, co, ci] + b_l[co]   (t = ky*3 + kx,
  off_t = (ky - 1, kx - 1)), A_l = relu(Z_l) for l = 1..5, y = x + Z_6.
Parameter shapes: W1 (9, 32) [t, co], b1 (32); W2..W5 (9, 32, 32) [t, co, ci], b (32);
W6 (9, 32) [t, ci], b6 (1). Flat order: W1, b1, W2, b2, ..., W5, b5, W6, b6 (37601 values).

Precision as the GPU path defines it: weights used by the layers are bf16-rounded master
weights; the activations A_1..A_5 and the back-propagated gradients dZ_1..dZ_5 are stored
as bf16; x, y, the loss gradient and all accumulations are wider (float64 here).
Loss: mean over pixels of (y - target)^2. Optimizer: Adam with float32-style master
weights (float64 here), bias-corrected moments.
"""
from __future__ import annotations

import numpy as np

C = 32
TAPS = [(ky - 1, kx - 1) for ky in range(3) for kx in range(3)]

SHAPES = [("W1", (9, C)), ("b1", (C,))] + sum(
    ([(f"W{l}", (9, C, C)), (f"b{l}", (C,))] for l in range(2, 6)), []) + [("W6", (9, C)), ("b6", (1,))]
N_PARAMS = int(sum(np.prod(s) for _, s in SHAPES))


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) and return as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def unflatten(flat: np.ndarray) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == N_PARAMS
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = flat[o:o + n].reshape(shp)
        o += n
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SHAPES])


def _shift(a: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """out[b, y, x, ...] = a[b, y + dy, x + dx, ...], zero outside the image."""
    out = np.zeros_like(a)
    H, W = a.shape[1], a.shape[2]
    ys0, ys1 = max(0, -dy), min(H, H - dy)
    xs0, xs1 = max(0, -dx), min(W, W - dx)
    if ys0 < ys1 and xs0 < xs1:
        out[:, ys0:ys1, xs0:xs1] = a[:, ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx]
    return out


def _identity(a):
    return np.asarray(a, np.float64)


def forward(g: np.ndarray, max_value: float, flat_params: np.ndarray, keep: bool = False,
            exact: bool = False):
    """Forward pass on a batch g (B, H, W) of integer images.

    Returns y (B, H, W) float64 and, with keep=True, the cache of stored activations.
    exact=True drops every bf16 rounding (plain float64 network, for derivative checks).
    """
    rnd = _identity if exact else bf16
    P = {k: (rnd(v) if k.startswith("W") else v) for k, v in unflatten(flat_params).items()}
    x = np.asarray(g, np.float64) / float(max_value)
    acts = []
    z = np.zeros(x.shape + (C,))
    for t, (dy, dx) in enumerate(TAPS):
        z += _shift(x, dy, dx)[..., None] * P["W1"][t][None, None, None, :]
    a = rnd(np.maximum(z + P["b1"], 0.0))
    acts.append(a)
    for l in range(2, 6):
        z = np.zeros(a.shape)
        for t, (dy, dx) in enumerate(TAPS):
            z += _shift(a, dy, dx) @ P[f"W{l}"][t].T
        a = rnd(np.maximum(z + P[f"b{l}"], 0.0))
        acts.append(a)
    z6 = np.zeros(x.shape)
    for t, (dy, dx) in enumerate(TAPS):
        z6 += _shift(a, dy, dx) @ P["W6"][t]
    y = x + z6 + P["b6"][0]
    if keep:
        return y, {"x": x, "acts": acts, "P": P, "rnd": rnd}
    return y


def layer(l: int, inp: np.ndarray, flat_params: np.ndarray, x: np.ndarray = None) -> np.ndarray:
    """One layer of the forward pass on a given input, as forward() computes it: l = 1 takes
    x = g / M (B, H, W) and returns A_1; l = 2..5 take A_{l-1} (B, H, W, 32) and return A_l
    (bf16-rounded ReLU outputs); l = 6 takes A_5 and returns y = x + Z_6 (x required). Used to
    check each GPU layer on the GPU's own stored input (teacher forcing)."""
    P = {k: (bf16(v) if k.startswith("W") else v) for k, v in unflatten(flat_params).items()}
    a = np.asarray(inp, np.float64)
    if l == 1:
        z = np.zeros(a.shape + (C,))
        for t, (dy, dx) in enumerate(TAPS):
            z += _shift(a, dy, dx)[..., None] * P["W1"][t][None, None, None, :]
        return bf16(np.maximum(z + P["b1"], 0.0))
    if 2 <= l <= 5:
        z = np.zeros(a.shape)
        for t, (dy, dx) in enumerate(TAPS):
            z += _shift(a, dy, dx) @ P[f"W{l}"][t].T
        return bf16(np.maximum(z + P[f"b{l}"], 0.0))
    if l == 6:
        z6 = np.zeros(a.shape[:3])
        for t, (dy, dx) in enumerate(TAPS):
            z6 += _shift(a, dy, dx) @ P["W6"][t]
        return np.asarray(x, np.float64) + z6 + P["b6"][0]
    raise ValueError(f"layer {l}")


def loss_and_grad(g, max_value, flat_params, target, exact: bool = False):
    """MSE loss and its gradient w.r.t. the flat parameters (backward pass by hand)."""
    y, cache = forward(g, max_value, flat_params, keep=True, exact=exact)
    x, acts, P, rnd = cache["x"], cache["acts"], cache["P"], cache["rnd"]
    npx = y.size
    loss = float(np.mean((y - target) ** 2))
    dy_ = 2.0 * (y - target) / npx
    G = {}
    # layer 6: y = x + sum_t shift(A5, t) @ W6[t] + b6
    a5 = acts[4]
    G["b6"] = np.array([dy_.sum()])
    G["W6"] = np.stack([np.einsum("byx,byxc->c", dy_, _shift(a5, dy, dx)) for dy, dx in TAPS])
    da = np.zeros(a5.shape)
    for t, (dy, dx) in enumerate(TAPS):
        da += _shift(dy_, -dy, -dx)[..., None] * P["W6"][t][None, None, None, :]
    dz = rnd(da * (a5 > 0))
    for l in range(5, 1, -1):
        a_prev = acts[l - 2]
        G[f"b{l}"] = dz.sum(axis=(0, 1, 2))
        G[f"W{l}"] = np.stack([np.einsum("byxo,byxi->oi", dz, _shift(a_prev, dy, dx)) for dy, dx in TAPS])
        da = np.zeros(a_prev.shape)
        for t, (dy, dx) in enumerate(TAPS):
            da += _shift(dz, -dy, -dx) @ P[f"W{l}"][t]
        dz = rnd(da * (a_prev > 0))
    G["b1"] = dz.sum(axis=(0, 1, 2))
    G["W1"] = np.stack([np.einsum("byxc,byx->c", dz, _shift(x, dy, dx)) for dy, dx in TAPS])
    return loss, flatten(G)


class Adam:
    """Adam with bias-corrected moments (beta1 0.9, beta2 0.999, eps 1e-8)."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, w, grad):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad
        self.v = self.b2 * self.v + (1 - self.b2) * grad * grad
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return w - self.lr * mh / (np.sqrt(vh) + self.eps)


# ---- per-tile check and fallback ------------------------------------------------------
def tile_stats(g: np.ndarray, y: np.ndarray, max_value: float, tile: int = 64):
    """Per tile: impulse fraction (pixels at 0 or max_value) and the mean squared residual
    (x - y)^2 over the other pixels (0 when the tile has none)."""
    H, W = g.shape
    ty, tx = -(-H // tile), -(-W // tile)
    frac = np.zeros((ty, tx))
    res = np.zeros((ty, tx))
    x = g / float(max_value)
    for i in range(ty):
        for j in range(tx):
            gs = g[i * tile:(i + 1) * tile, j * tile:(j + 1) * tile]
            d = (x - y)[i * tile:(i + 1) * tile, j * tile:(j + 1) * tile]
            imp = (gs == 0) | (gs == max_value)
            frac[i, j] = imp.mean()
            ok = ~imp
            res[i, j] = float(np.mean(d[ok] ** 2)) if ok.any() else 0.0
    return frac, res


def tile_deviation(y: np.ndarray, proxy: np.ndarray, tile: int = 64):
    """Per tile: mean squared deviation (y - proxy)^2 of the surrogate output from a proxy
    of the plain output, over every pixel of the tile."""
    H, W = y.shape
    ty, tx = -(-H // tile), -(-W // tile)
    dev = np.zeros((ty, tx))
    d2 = (np.asarray(y, np.float64) - np.asarray(proxy, np.float64)) ** 2
    for i in range(ty):
        for j in range(tx):
            dev[i, j] = float(d2[i * tile:(i + 1) * tile, j * tile:(j + 1) * tile].mean())
    return dev


def tile_scores(frac, res, p_max, r_lo, r_hi, dev=None, d_hi=0.0):
    """Distance of each tile from the calibrated band: max(frac / p_max, res / r_hi,
    r_lo / res) and, with a deviation bound d_hi > 0, dev / d_hi^2 (dev: the tile's mean
    squared deviation from the plain-output proxy); a tile passes when its score is below
    the threshold."""
    with np.errstate(divide="ignore"):
        s_lo = np.where(res > 0, r_lo / np.where(res > 0, res, 1.0), np.inf)
    sc = np.maximum(np.maximum(frac / p_max, res / r_hi), s_lo)
    if dev is not None and d_hi > 0:
        sc = np.maximum(sc, dev / (d_hi * d_hi))
    return sc

