"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, without a GPU.

1. The CPU oracle's C functions (gcc, -fsanitize=address,undefined) on ragged, 1 x 1,
   single-row / single-column images, windows far wider than the image, 16-bit extremes
   and a dense 12-bit impulse image; their outputs must equal the regular build's bit for
   bit.
2. The C-ABI library with its host code instrumented (hipcc, the sanitizers on the host
   side only): every entry point's argument validation, driven from C with fake pointers
   that the checks reject before anything is enqueued.
The sanitizers abort on the first error they report. Builds are cached under
tests/sanitize/_build, keyed by the sources and flags.
"""
import hashlib
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from phantoms import noisy_phantom

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
BUILD = os.path.join(HERE, "_build")
CSRC = os.path.join(ROOT, "paper_2005_05371_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=86",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=87")


def _key(paths, flags):
    h = hashlib.sha256()
    for p in sorted(paths):
        h.update(p.encode())
        with open(p, "rb") as f:
            h.update(f.read())
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)} failed ({r.returncode}):\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}")
    return r


def build_oracle_checks() -> str:
    srcs = [os.path.join(ROOT, "oracle", "hybrid_oracle.c"), os.path.join(HERE, "oracle_checks.c")]
    flags = ["-O1", "-g", "-std=c11", "-fopenmp", *SAN]
    exe = os.path.join(BUILD, f"oracle_checks-{_key(srcs, flags)}")
    if not os.path.exists(exe):
        os.makedirs(BUILD, exist_ok=True)
        _run(["gcc", *flags, *srcs, "-o", exe + ".tmp"])
        os.replace(exe + ".tmp", exe)
    return exe


def build_abi_checks() -> str:
    lib_srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".h")))
    hdrs = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    drv = os.path.join(HERE, "abi_checks.c")
    # host side instrumented; every -fsanitize option applies to the host pass only
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    hip_flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san]
    exe = os.path.join(BUILD, f"abi_checks-{_key(lib_srcs + hdrs + [drv], hip_flags)}")
    if os.path.exists(exe):
        return exe
    obj_dir = exe + ".objs"
    os.makedirs(obj_dir, exist_ok=True)
    hips = [s for s in lib_srcs if s.endswith(".hip")]
    procs = []
    for s in hips:
        o = os.path.join(obj_dir, os.path.basename(s)[:-4] + ".o")
        procs.append((s, subprocess.Popen([HIPCC, *hip_flags, "-c", s, "-o", o], stdout=subprocess.PIPE,
                                          stderr=subprocess.STDOUT, text=True)))
    for s, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed for {s}:\n{out[-4000:]}")
    drv_o = os.path.join(obj_dir, "abi_checks.o")
    _run([CLANG, "-O1", "-g", "-std=c11", "-Wno-incompatible-pointer-types-discards-qualifiers", *SAN,
          "-I", os.path.join(ROOT, "include"), "-c", drv, "-o", drv_o])
    objs = [drv_o] + [os.path.join(obj_dir, os.path.basename(s)[:-4] + ".o") for s in hips]
    _run([CLANGXX, *SAN, *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
          "-o", exe + ".tmp"])
    os.replace(exe + ".tmp", exe)
    shutil.rmtree(obj_dir, ignore_errors=True)
    return exe


# name, image, smax, keep, Wiener window, max_value, threads
def _cases():
    rng = np.random.default_rng(2005)
    u16 = rng.integers(0, 65536, size=(20, 17)).astype(np.int32)
    u16[rng.random(u16.shape) < 0.3] = 65535
    u16[rng.random(u16.shape) < 0.2] = 0
    return [
        ("ragged", noisy_phantom(37, 53, 255, 15, 0.2, seed=1), 7, 0, (3, 3), 255, 2),
        ("one", np.array([[200]], np.int32), 3, 0, (3, 3), 255, 1),
        ("row", noisy_phantom(1, 40, 255, 10, 0.3, seed=2), 9, 0, (5, 5), 255, 1),
        ("col", noisy_phantom(29, 1, 255, 10, 0.3, seed=3), 5, 1, (7, 3), 255, 1),
        ("wide", noisy_phantom(3, 5, 255, 10, 0.4, seed=4), 31, 1, (15, 15), 255, 1),
        ("wide_zmed", noisy_phantom(4, 6, 255, 10, 0.6, seed=5), 31, 0, (15, 1), 255, 1),
        ("u16_extremes", u16, 11, 0, (15, 15), 65535, 2),
        ("dense_12bit", noisy_phantom(64, 48, 4095, 60, 0.5, seed=6), 15, 0, (7, 7), 4095, 3),
    ]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = build_oracle_checks()
    cases = _cases()
    with open(tmp_path / "cases.txt", "w") as f:
        for name, g, smax, keep, (wh, ww), maxv, thr in cases:
            np.ascontiguousarray(g, np.int32).tofile(tmp_path / f"{name}.in")
            f.write(f"{name} {g.shape[0]} {g.shape[1]} {smax} {keep} {wh} {ww} {maxv} {thr}\n")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, f"sanitized oracle failed ({r.returncode}):\n{r.stdout}\n{r.stderr[-6000:]}"
    assert f"oracle checks: {len(cases)} cases" in r.stdout
    for name, g, smax, keep, (wh, ww), maxv, thr in cases:
        h, w = g.shape
        a, level = oracle.amf(g, smax, keep=bool(keep), return_level=True)
        out, _, nu2 = oracle.hybrid(g, smax, (wh, ww), maxv, keep=bool(keep))
        np.testing.assert_array_equal(np.fromfile(tmp_path / f"{name}.amf", np.int32).reshape(h, w), a)
        np.testing.assert_array_equal(np.fromfile(tmp_path / f"{name}.level", np.int32).reshape(h, w), level)
        got = np.fromfile(tmp_path / f"{name}.out", np.float64).reshape(h, w)
        np.testing.assert_array_equal(got.view(np.uint64), out.view(np.uint64), err_msg=name)
        assert np.fromfile(tmp_path / f"{name}.nu2", np.float64)[0] == nu2, name


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs hipcc")
def test_abi_validation_under_sanitizers():
    import torch
    if torch.cuda.is_available():
        pytest.skip("fake device pointers are only passed where no GPU is present")
    exe = build_abi_checks()
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, f"sanitized ABI checks failed ({r.returncode}):\n{r.stdout}\n{r.stderr[-6000:]}"
    assert ", 0 unexpected" in r.stdout, r.stdout
