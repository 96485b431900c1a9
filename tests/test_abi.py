"""The C-ABI library loads, exports every symbol its headers declare, and rejects bad
arguments on the host before anything is enqueued (no GPU needed)."""
import ctypes
import glob
import os
import re

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DECL = re.compile(r"^\s*(?:const\s+)?[A-Za-z_][\w]*\s*\**\s*\b([A-Za-z_]\w*)\s*\(")


def declared_functions():
    names = []
    for hdr in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        text = open(hdr).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = "\n".join(l for l in text.splitlines() if not l.strip().startswith("#"))
        for stmt in text.split(";"):
            s = " ".join(stmt.split())
            if not s or s.startswith("#") or "typedef" in s or "}" in s and "(" not in s:
                continue
            s = s.split("}")[-1].strip()
            m = DECL.match(s)
            if m and not s.startswith("#"):
                names.append(m.group(1))
    return names


def test_header_declares_core_entry_points():
    names = declared_functions()
    for fn in ("amf_filter", "wiener_filter", "hybrid_denoise", "hd_last_error", "hd_version"):
        assert fn in names, names


def test_library_exports_every_declared_symbol():
    from paper_2005_05371_amd import _binding
    lib = ctypes.CDLL(_binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps every declared function
    assert set(declared_functions()) <= set(_binding.SIGNATURES), \
        set(declared_functions()) - set(_binding.SIGNATURES)


def test_version():
    from paper_2005_05371_amd import _binding
    assert _binding.load().hd_version() >= 100


# Fake (never dereferenced) device addresses: every call below fails host-side checks.
# Skipped where a GPU is present, so that a regression in the checks can never launch a
# kernel on them; the GPU suite repeats these checks with real buffers.
FAKE_IN, FAKE_OUT = 0x10000, 0x800000
nogpu = pytest.mark.skipif(torch.cuda.is_available(), reason="fake pointers only off-GPU")


@nogpu
@pytest.mark.parametrize("smax,expect", [(1, 4), (0, 4), (-3, 4), (4, 4), (10, 4), (33, 4)])
def test_amf_bad_smax(smax, expect):
    from paper_2005_05371_amd import _binding as b
    rc = b.load().amf_filter(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 1, smax, 0, None)
    assert rc == expect
    assert b"SMAX" in b.load().hd_last_error() or b"Smax" in b.load().hd_last_error()


@nogpu
def test_amf_bad_args():
    from paper_2005_05371_amd import _binding as b
    L = b.load()
    assert L.amf_filter(None, FAKE_OUT, 16, 16, 16, 16, 1, 5, 0, None) == 1
    assert L.amf_filter(FAKE_IN, FAKE_OUT, 0, 16, 16, 16, 1, 5, 0, None) == 2
    assert L.amf_filter(FAKE_IN, FAKE_OUT, 16, 16, 8, 16, 1, 5, 0, None) == 2
    assert L.amf_filter(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 3, 5, 0, None) == 3
    assert L.amf_filter(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 1, 5, 0x10, None) == 10
    assert L.amf_filter(FAKE_IN, FAKE_IN + 8, 16, 16, 16, 16, 1, 5, 0, None) == 7


@nogpu
def test_wiener_and_hybrid_bad_args():
    from paper_2005_05371_amd import _binding as b
    L = b.load()
    assert L.wiener_filter(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 1, 255, 4, 3, -1.0, None, None) == 5
    assert L.wiener_filter(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 1, 255, 17, 17, -1.0, None, None) == 5
    assert L.wiener_filter(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 1, 256, 3, 3, -1.0, None, None) == 6
    assert L.wiener_filter(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 2, 0, 3, 3, -1.0, None, None) == 6
    assert L.hybrid_denoise(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 1, 255, 6, 3, 3, -1.0, 0, None, 0,
                            None, None) == 4
    assert L.hybrid_denoise(FAKE_IN, FAKE_IN, 16, 16, 16, 16, 1, 255, 5, 3, 3, -1.0, 0, None, 0,
                            None, None) == 7
    # amf_out overlapping the output
    assert L.hybrid_denoise(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 1, 255, 5, 3, 3, -1.0, 0, FAKE_OUT,
                            16, None, None) == 7


@pytest.mark.parametrize("args", [(99, 9, 5, 5, -1), (1, 8, 5, 5, -1), (1, 9, 4, 5, -1), (2, 9, 5, 5, 7),
                                  (1, 33, 5, 5, 0), (1, 9, 17, 17, 0)])
def test_resident_capacity_rejects_bad_keys(args):
    """Invalid keys return 0 before any device query."""
    from paper_2005_05371_amd import _binding
    lib = _binding.load()
    assert lib.hd_resident_capacity(*args) == 0


@nogpu
def test_parts_and_stretch_bad_args():
    from paper_2005_05371_amd import _binding as b
    L = b.load()
    # parts out of range: 0, above the height, above the limit
    assert L.amf_filter_parts(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 1, 5, 0, 0, None) == 10
    assert L.amf_filter_parts(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 1, 5, 17, 0, None) == 10
    assert L.amf_filter_parts(FAKE_IN, FAKE_OUT, 4096, 16, 16, 16, 1, 5, 257, 0, None) == 10
    assert L.amf_filter_parts(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 1, 6, 2, 0, None) == 4
    assert L.amf_filter_parts(FAKE_IN, FAKE_IN + 8, 16, 16, 16, 16, 1, 5, 2, 0, None) == 7
    assert L.contrast_stretch(None, 16, 16, 16, None) == 1
    assert L.contrast_stretch(FAKE_OUT, 16, 0, 16, None) == 2
    # unknown hybrid flag bits
    assert L.hybrid_denoise(FAKE_IN, FAKE_OUT, 16, 16, 16, 16, 1, 255, 5, 3, 3, -1.0, 0x8, None, 0,
                            None, None) == 10
