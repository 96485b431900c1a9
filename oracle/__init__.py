"""CPU oracle of the hybrid AMF + adaptive Wiener de-noiser, and of the conv surrogate.

TEST INFRASTRUCTURE ONLY: the slow, plain definitions that the HIP library is checked
against. Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package. It imports nothing from the GPU package and shares no
code with it; the product path never calls it.

The AMF / Wiener definitions live in ``hybrid_oracle.c`` (plain C, int64 / double),
built here with gcc and loaded through ctypes. The surrogate network's oracle is
``oracle.surrogate`` (numpy float64).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hybrid_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

ERRORS = {-1: "SMAX must be an odd integer > 1", -2: "bad dimensions", -3: "bad window",
          -4: "out of memory"}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP) into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ci = ctypes.c_int
        lib.oracle_mirror.argtypes = [ctypes.c_long, ctypes.c_long]
        lib.oracle_mirror.restype = ctypes.c_long
        lib.oracle_amf.argtypes = [i32p, i32p, ctypes.c_void_p, ci, ci, ci, ci, ci]
        lib.oracle_amf.restype = ci
        lib.oracle_noise_estimate.argtypes = [i32p, ci, ci, ci, ci, ci]
        lib.oracle_noise_estimate.restype = ctypes.c_double
        lib.oracle_wiener.argtypes = [i32p, f64p, ci, ci, ci, ci, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_void_p, ci]
        lib.oracle_wiener.restype = ci
        _lib = lib
    return _lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def mirror(i: int, n: int) -> int:
    """Symmetric-padding index of i in [0, n) (period 2n)."""
    return int(_load().oracle_mirror(int(i), int(n)))


def _check(rc: int):
    if rc != 0:
        raise ValueError(ERRORS.get(rc, f"oracle error {rc}"))


def amf(g: np.ndarray, smax: int, keep: bool = False, threads: Optional[int] = None,
        return_level: bool = False):
    """Adaptive median filter of a 2-D integer image (returns int32; optionally the level map).

    ``level[y, x]`` is the window size at which stage A passed, 0 if it never did.
    """
    g = np.ascontiguousarray(g, dtype=np.int32)
    if g.ndim != 2:
        raise ValueError("image must be 2-D")
    h, w = g.shape
    out = np.empty_like(g)
    level = np.empty_like(g) if return_level else None
    lp = level.ctypes.data_as(ctypes.c_void_p) if level is not None else None
    _check(_load().oracle_amf(g, out, lp, h, w, int(smax), int(bool(keep)),
                              threads or default_threads()))
    return (out, level) if return_level else out


def noise_estimate(a: np.ndarray, win: Tuple[int, int], threads: Optional[int] = None) -> float:
    a = np.ascontiguousarray(a, dtype=np.int32)
    v = _load().oracle_noise_estimate(a, a.shape[0], a.shape[1], int(win[0]), int(win[1]),
                                      threads or default_threads())
    if v < 0:
        raise MemoryError("oracle noise estimate failed")
    return float(v)


def wiener(a: np.ndarray, win, max_value: float, noise_var: float = -1.0,
           threads: Optional[int] = None, return_nu2: bool = False):
    """Adaptive Wiener filter of an integer image, float64 output divided by max_value."""
    if np.isscalar(win):
        win = (int(win), int(win))
    a = np.ascontiguousarray(a, dtype=np.int32)
    h, w = a.shape
    out = np.empty((h, w), dtype=np.float64)
    nu2 = np.zeros(1, dtype=np.float64)
    _check(_load().oracle_wiener(a, out, h, w, int(win[0]), int(win[1]), float(noise_var),
                                 float(max_value), nu2.ctypes.data_as(ctypes.c_void_p),
                                 threads or default_threads()))
    return (out, float(nu2[0])) if return_nu2 else out


def hybrid(g: np.ndarray, smax: int, win, max_value: float, noise_var: float = -1.0,
           keep: bool = False, threads: Optional[int] = None):
    """Hybrid de-noiser: Wiener(AMF(g)). Returns (float64 output / max_value, AMF int32, nu2)."""
    a = amf(g, smax, keep=keep, threads=threads)
    out, nu2 = wiener(a, win, max_value, noise_var, threads=threads, return_nu2=True)
    return out, a, nu2


def contrast_stretch(y: np.ndarray) -> np.ndarray:
    """Post-processing step of the hybrid (Alg. 1, step e; Sec. III): linear min-max
    contrast stretch of one slice, (y - min) / (max - min) in float64, so the slice spans
    [0, 1]. The paper names the step only; reading: per slice, over all pixels; a constant
    slice (max == min) is returned unchanged."""
    y = np.asarray(y, dtype=np.float64)
    lo, hi = float(y.min()), float(y.max())
    if hi == lo:
        return y.copy()
    return (y - lo) / (hi - lo)


def strip_bounds(h: int, parts: int):
    """Row bounds of the paper's image partitions (Alg. 1, procedure parallelAdapMedian,
    imgSpliter; Fig. 5). Reading: `parts` horizontal strips, strip i = rows
    [floor(i h / parts), floor((i + 1) h / parts)); empty strips when parts > h."""
    return [(i * h // parts, (i + 1) * h // parts) for i in range(parts)]


def amf_partitioned(g: np.ndarray, smax: int, parts: int, keep: bool = False,
                    threads: Optional[int] = None) -> np.ndarray:
    """Partitioned AMF as in the paper's parallel procedure: every strip filtered as an
    image of its own (no halo: windows mirror at the strip's own borders), strips stacked
    back. Differs from the whole-image AMF near the cuts."""
    g = np.asarray(g)
    out = np.empty(g.shape, dtype=np.int32)
    for r0, r1 in strip_bounds(g.shape[0], parts):
        if r1 > r0:
            out[r0:r1] = amf(g[r0:r1], smax, keep=keep, threads=threads)
    return out


def level_histogram(level: np.ndarray, smax: int) -> dict:
    """Fraction of pixels resolved at each window size (key 0 = never resolved)."""
    n = level.size
    keys = [k for k in range(3, smax + 1, 2)] + [0]
    return {k: float(np.count_nonzero(level == k)) / n for k in keys}


def window_elements_per_pixel(level: np.ndarray, smax: int) -> float:
    """Mean number of window elements the method visits per pixel: sum of k^2 over the
    levels a pixel is tested at (all levels up to its resolving one, all of them if
    it never resolves)."""
    total = 0.0
    n = level.size
    for k in range(3, smax + 1, 2):
        # a pixel is tested at level k if it resolves at >= k or never resolves
        tested = np.count_nonzero((level >= k) | (level == 0))
        total += tested * k * k
    return total / n
