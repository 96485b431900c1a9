"""Training, calibration and checkpointing of the learned surrogate.

The surrogate learns to reproduce the plain hybrid filter (AMF + adaptive Wiener) from
(noisy, plain output) pairs that the plain path itself produces on seeded phantoms. All
network arithmetic (forward, backward, Adam) runs in the library's HIP kernels; this
module only orders the work: data, mini-batches, epochs, the tile-check calibration and
checkpoint files.

Calibration of the per-tile check: on the training set, for every 64 x 64 tile of the
PLAIN output, take frac = share of impulse-valued pixels (0 or max) and res = mean of
(x - plain)^2 over the other pixels; p_max = max frac, (r_lo, r_hi) = the (q, 1 - q)
quantiles of res. With a proxy of the plain output (the plain hybrid with the AMF stopped
at window check_smax), d_hi = the (1 - q) quantile of the tiles' root-mean-square distance
between the plain output and the proxy. At inference a surrogate tile passes while its own
(frac, res) stays inside that band and its distance from the proxy stays within d_hi
(score < threshold, 1.0 = the band itself): its distance from the plain output is then at
most about 2 d_hi for all but a fraction q of tiles.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import asdict, dataclass
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _binding as B


@dataclass
class TrainConfig:
    n_train: int = 2000
    size: int = 256
    batch: int = 16
    epochs: int = 8
    lr: float = 2e-3
    seed: int = 0
    smax: int = 9
    win: int = 5
    quantile: float = 0.005
    max_value: int = 255
    check_smax: int = 3


def make_training_pairs(n: int, size: int, smax: int, win: int, device="cuda", like=None, proxy_smax: int = 0):
    """Seeded noisy phantoms and their plain hybrid outputs, both on the GPU. `like` (a
    phantoms.Workload) sets the dtype, max value and noise of the images (default: the
    64 x 1024^2 8-bit surrogate workload's). With proxy_smax > 0 also returns the plain
    output's proxy (the plain hybrid with the AMF stopped at window proxy_smax)."""
    from phantoms import surrogate_train_set, training_set_like
    wl = surrogate_train_set(n, size) if like is None else training_set_like(like, n, size)
    noisy = np.stack([wl.make_slice(i).noisy for i in range(n)])
    x = torch.from_numpy(noisy).to(device)
    target = torch.empty((n, size, size), dtype=torch.float32, device=device)
    proxy = torch.empty_like(target) if proxy_smax else None
    chunk = 256
    for s in range(0, n, chunk):
        ins = [x[i] for i in range(s, min(n, s + chunk))]
        outs = [target[i] for i in range(s, min(n, s + chunk))]
        B.hybrid_denoise_batched(ins, smax, win, wl.max_value, outs=outs)
        if proxy is not None:
            B.hybrid_denoise_batched(ins, proxy_smax, win, wl.max_value,
                                     outs=[proxy[i] for i in range(s, min(n, s + chunk))])
    torch.cuda.synchronize()
    if proxy is not None:
        return x, target, proxy
    return x, target


def calibrate(noisy: np.ndarray, plain: np.ndarray, max_value: int, quantile: float = 0.005,
              tile: int = 64, proxy: Optional[np.ndarray] = None):
    """(p_max, r_lo, r_hi) from the plain outputs' per-tile statistics, and with `proxy`
    also d_hi (see module doc): (p_max, r_lo, r_hi, d_hi)."""
    fr, rs, ds = [], [], []
    for k, (g, y) in enumerate(zip(noisy, plain)):
        x = g.astype(np.float64) / max_value
        H, W = g.shape
        for i in range(0, H, tile):
            for j in range(0, W, tile):
                gs = g[i:i + tile, j:j + tile]
                imp = (gs == 0) | (gs == max_value)
                fr.append(float(imp.mean()))
                ok = ~imp
                if ok.any():
                    d = (x - y)[i:i + tile, j:j + tile][ok]
                    rs.append(float(np.mean(d * d)))
                if proxy is not None:
                    e = (np.asarray(y, np.float64) - proxy[k])[i:i + tile, j:j + tile]
                    ds.append(float(np.sqrt(np.mean(e * e))))
    rs = np.asarray(rs)
    out = (float(max(fr)), float(np.quantile(rs, quantile)), float(np.quantile(rs, 1 - quantile)))
    if proxy is not None:
        # a floor keeps the bound positive where the proxy equals the plain output
        out = out + (max(float(np.quantile(np.asarray(ds), 1 - quantile)), 0.5 / max_value),)
    return out


def save_checkpoint(path: str, net: "B.Surrogate", epoch: int, cfg: TrainConfig,
                    calib=None, history: Optional[List[float]] = None):
    st = net.get_state()
    tmp = path + ".tmp.npz"
    np.savez(tmp, params=st["params"], m=st["m"], v=st["v"], step=np.int64(st["step"]),
             epoch=np.int64(epoch), config=json.dumps(asdict(cfg)),
             calib=np.asarray(calib if calib is not None else [np.nan] * 3, np.float64),
             history=np.asarray(history or [], np.float64))
    os.replace(tmp, path)


def load_checkpoint(path: str, net: Optional["B.Surrogate"] = None):
    """Restore parameters, Adam moments and step into `net` (created if None)."""
    with np.load(path, allow_pickle=False) as z:
        st = {k: z[k] for k in z.files}
    net = net or B.Surrogate()
    net.set_state(st["params"], st["m"], st["v"], int(st["step"]))
    cfg = TrainConfig(**json.loads(str(st["config"])))
    return net, int(st["epoch"]), cfg, st["calib"], list(st["history"])


def train(net: "B.Surrogate", x: torch.Tensor, target: torch.Tensor, cfg: TrainConfig,
          start_epoch: int = 0, ckpt_path: Optional[str] = None, log=print) -> Dict:
    """Mini-batch training; the batch order of epoch e is a permutation seeded by
    (cfg.seed, e), so a resumed run replays exactly the batches it would have seen."""
    n = x.shape[0]
    history = []
    t0 = time.perf_counter()
    for ep in range(start_epoch, cfg.epochs):
        order = np.random.default_rng([cfg.seed, ep]).permutation(n)
        losses = []
        for s in range(0, n - cfg.batch + 1, cfg.batch):
            idx = torch.from_numpy(order[s:s + cfg.batch]).to(x.device)
            xb = x.index_select(0, idx).contiguous()
            tb = target.index_select(0, idx).contiguous()
            loss, _ = net.train_step(xb, tb, lr=cfg.lr, max_value=cfg.max_value)
            losses.append(loss)
        ep_loss = float(torch.stack(losses).mean().item())
        history.append(ep_loss)
        log(f"epoch {ep + 1}/{cfg.epochs} loss {ep_loss:.3e} ({time.perf_counter() - t0:.1f} s)")
        if ckpt_path:
            save_checkpoint(ckpt_path, net, ep + 1, cfg, history=history)
    torch.cuda.synchronize()
    return {"history": history, "seconds": time.perf_counter() - t0}
