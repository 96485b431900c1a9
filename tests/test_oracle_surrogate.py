"""Pins for the CPU oracle of the conv surrogate (no GPU).

  * each layer against scipy.signal.correlate2d (zero padding, 'same');
  * the hand-written backward pass against central finite differences of the float64
    forward (bf16 rounding off, so the loss is smooth);
  * Adam against torch.optim.Adam on the CPU in float64;
  * bf16 rounding against torch's bfloat16 conversion;
  * tile statistics on hand-made tiles.
"""
import numpy as np
import pytest
import scipy.signal as sig
import torch

import oracle.surrogate as S
from phantoms import noisy_phantom, surrogate_params


def _params(seed=1):
    return surrogate_params(seed, scale_last=1.0).astype(np.float64)


def test_bf16_matches_torch():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-30, 100), [0.0, -0.0, 1.0, 3.0e38]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16(a), ref)


def test_layers_match_scipy_correlate():
    g = noisy_phantom(23, 31, 255, 15, 0.2, seed=2)[None]
    p = _params()
    P = S.unflatten(p)
    y, cache = S.forward(g, 255, p, keep=True, exact=True)
    x = g[0] / 255.0
    # layer 1
    for co in range(S.C):
        k = P["W1"][:, co].reshape(3, 3)
        ref = np.maximum(sig.correlate2d(x, k, mode="same") + P["b1"][co], 0)
        np.testing.assert_allclose(cache["acts"][0][0, :, :, co], ref, rtol=0, atol=1e-12)
    # layer 3 from layer 2
    a2 = cache["acts"][1][0]
    for co in (0, 7, 31):
        z = sum(sig.correlate2d(a2[:, :, ci], P["W3"][:, co, ci].reshape(3, 3), mode="same")
                for ci in range(S.C))
        np.testing.assert_allclose(cache["acts"][2][0, :, :, co], np.maximum(z + P["b3"][co], 0),
                                   rtol=0, atol=1e-10)
    # output layer and the residual
    a5 = cache["acts"][4][0]
    z6 = sum(sig.correlate2d(a5[:, :, ci], P["W6"][:, ci].reshape(3, 3), mode="same") for ci in range(S.C))
    np.testing.assert_allclose(y[0], x + z6 + P["b6"][0], rtol=0, atol=1e-10)


def test_single_layers_compose_to_forward():
    """oracle.surrogate.layer, applied layer by layer to its own outputs, is forward() bit for
    bit (it serves the per-layer GPU checks, which feed it the GPU's stored activations)."""
    g = np.stack([noisy_phantom(13, 17, 4095, 60, 0.3, seed=5 + i) for i in range(2)])
    p = _params(4)
    y, cache = S.forward(g, 4095, p, keep=True)
    x = g / 4095.0
    a = S.layer(1, x, p)
    np.testing.assert_array_equal(a, cache["acts"][0])
    for l in range(2, 6):
        a = S.layer(l, cache["acts"][l - 2], p)
        np.testing.assert_array_equal(a, cache["acts"][l - 1])
    np.testing.assert_array_equal(S.layer(6, cache["acts"][4], p, x=x), y)


def test_backward_matches_finite_differences():
    g = noisy_phantom(2 * 9, 11, 255, 20, 0.3, seed=3).reshape(2, 9, 11)
    p = _params(4)
    target = np.random.default_rng(5).uniform(0, 1, g.shape)
    loss, grad = S.loss_and_grad(g, 255, p, target, exact=True)
    rng = np.random.default_rng(6)
    offsets = np.cumsum([0] + [int(np.prod(s)) for _, s in S.SHAPES])
    idx = [int(offsets[i] + rng.integers(0, offsets[i + 1] - offsets[i])) for i in range(len(S.SHAPES))
           for _ in range(3)]
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        lp = float(np.mean((S.forward(g, 255, pp, exact=True) - target) ** 2))
        lm = float(np.mean((S.forward(g, 255, pm, exact=True) - target) ** 2))
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, grad[i])


def test_adam_matches_torch():
    rng = np.random.default_rng(7)
    w0 = rng.normal(0, 1, 50)
    opt = S.Adam(50, lr=1e-2)
    tw = torch.tensor(w0.copy(), dtype=torch.float64, requires_grad=True)
    topt = torch.optim.Adam([tw], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    w = w0.copy()
    for step in range(5):
        grad = rng.normal(0, 1, 50)
        w = opt.step(w, grad)
        topt.zero_grad()
        tw.grad = torch.tensor(grad)
        topt.step()
        np.testing.assert_allclose(w, tw.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_identity_when_last_layer_zero():
    g = noisy_phantom(16, 16, 255, 10, 0.1, seed=8)[None]
    p = _params()
    P = S.unflatten(p)
    P["W6"][:] = 0
    P["b6"][:] = 0
    y = S.forward(g, 255, S.flatten(P))
    np.testing.assert_array_equal(y, g / 255.0)


def test_tile_stats_and_scores():
    g = np.full((128, 70), 100, np.int32)
    g[:64, :64] = 0                      # tile (0,0): all impulses
    g[64:, :64][::2] = 255               # tile (1,0): half impulses
    y = g / 255.0
    y[64:, 64:] += 0.1                   # tile (1,1): residual 0.01 on every pixel
    frac, res = S.tile_stats(g, y, 255)
    assert frac.shape == (2, 2)
    assert frac[0, 0] == 1.0 and res[0, 0] == 0.0
    assert frac[1, 0] == 0.5 and res[1, 0] == 0.0
    assert frac[1, 1] == 0.0 and abs(res[1, 1] - 0.01) < 1e-12
    sc = S.tile_scores(frac, res, p_max=0.5, r_lo=0.001, r_hi=0.02)
    assert sc[0, 0] == np.inf            # no residual: below the band
    assert abs(sc[1, 1] - 0.5) < 1e-9    # inside the band: max(0, 0.01/0.02, 0.001/0.01)
