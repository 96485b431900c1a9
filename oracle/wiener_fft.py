"""Oracle of the paper's frequency-domain Wiener step (Alg. 1, step d: wnrFn(adapOnly,
original); Sec. III places the Wiener step in the Fourier domain).

TEST INFRASTRUCTURE ONLY (see the package docstring). The paper names the function and
its two arguments only. Reading: with A = DFT2(a) of the AMF output and F = DFT2(f) of the
clean original (both H x W, the image's own size, so the filter acts on the periodic
image), the noise spectrum is N = A - F and every frequency is weighted by the Wiener gain
|F|^2 / (|F|^2 + |N|^2) (0 where both vanish, where A is 0 too); the output is
real(IDFT2(gain A)) / M. Plain float64 numpy DFTs (numpy.fft), no windowing or padding.
"""
from __future__ import annotations

import numpy as np


def wiener_fft(a: np.ndarray, original: np.ndarray, max_value: float) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    f = np.asarray(original, dtype=np.float64)
    A = np.fft.fft2(a)
    F = np.fft.fft2(f)
    N = A - F
    pf = np.abs(F) ** 2
    den = pf + np.abs(N) ** 2
    gain = np.divide(pf, den, out=np.zeros_like(pf), where=den > 0)
    return np.real(np.fft.ifft2(gain * A)) / max_value


def dft2_brute(x: np.ndarray) -> np.ndarray:
    """The 2-D DFT written out as its double sum (small images only)."""
    x = np.asarray(x, dtype=np.complex128)
    h, w = x.shape
    ky = np.arange(h).reshape(h, 1)
    kx = np.arange(w).reshape(w, 1)
    ey = np.exp(-2j * np.pi * ky * np.arange(h) / h)   # [k, y]
    ex = np.exp(-2j * np.pi * kx * np.arange(w) / w)   # [k, x]
    return ey @ x @ ex.T
