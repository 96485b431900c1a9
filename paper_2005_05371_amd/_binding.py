"""ctypes binding of libhybrid_denoise.so (argument marshalling only).

Every function takes torch tensors that live on the GPU, passes their device pointers,
sizes and row pitches, plus the current HIP stream, to the C ABI declared in
``include/hybrid_denoise.h``. All computation happens in the library's HIP kernels;
there is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhybrid_denoise.so")

HD_U8, HD_U16 = 1, 2
HD_CONTRAST_STRETCH = 2
HD_AMF_UNRESOLVED_KEEP = 1
STATUS = {0: "HD_OK", 1: "HD_ERR_NULL", 2: "HD_ERR_DIMS", 3: "HD_ERR_DTYPE", 4: "HD_ERR_SMAX",
          5: "HD_ERR_WINDOW", 6: "HD_ERR_MAXVAL", 7: "HD_ERR_ALIAS", 8: "HD_ERR_NOMEM",
          9: "HD_ERR_HIP", 10: "HD_ERR_ARG", 11: "HD_ERR_TIMEOUT"}


class HDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


_lib = None

c_i32, c_i64, c_u32, c_dbl, c_vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                    ctypes.c_double, ctypes.c_void_p)

# name -> (argtypes, restype); mirrors include/hybrid_denoise.h
SIGNATURES = {
    "hd_version": ([], c_i32),
    "hd_last_error": ([], ctypes.c_char_p),
    "hd_check_errors": ([c_vp], c_i32),
    "amf_filter": ([c_vp, c_vp, c_i32, c_i32, c_i64, c_i64, c_i32, c_i32, c_u32, c_vp], c_i32),
    "contrast_stretch": ([c_vp, c_i32, c_i32, c_i64, c_vp], c_i32),
    "wiener_fft": ([c_vp, c_vp, c_vp, c_i32, c_i32, c_i64, c_i64, c_i64, c_i32, c_i32, c_vp], c_i32),
    "degrade_image": ([c_vp, c_vp, c_i32, c_i32, c_i64, c_i64, c_i32, c_i32, c_dbl, c_dbl,
                       ctypes.c_uint64, c_u32, c_vp], c_i32),
    "amf_filter_parts": ([c_vp, c_vp, c_i32, c_i32, c_i64, c_i64, c_i32, c_i32, c_i32, c_u32, c_vp],
                         c_i32),
    "wiener_filter": ([c_vp, c_vp, c_i32, c_i32, c_i64, c_i64, c_i32, c_i32, c_i32, c_i32, c_dbl,
                       c_vp, c_vp], c_i32),
    "hybrid_denoise": ([c_vp, c_vp, c_i32, c_i32, c_i64, c_i64, c_i32, c_i32, c_i32, c_i32, c_i32,
                        c_dbl, c_u32, c_vp, c_i64, c_vp, c_vp], c_i32),
    "hybrid_denoise_noalloc": ([c_vp, c_vp, c_i32, c_i32, c_i64, c_i64, c_i32, c_i32, c_i32, c_i32, c_i32,
                                c_dbl, c_u32, c_vp, c_i64, c_vp, c_vp], c_i32),
    "hybrid_denoise_batched": ([c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_dbl, c_u32, c_vp],
                               c_i32),
    "hybrid_denoise_batched_timed": ([c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_dbl, c_u32, c_vp,
                                      c_vp], c_i32),
    "hd_release_plans": ([], None),
    "hd_set_option": ([c_i32, c_i32], c_i32),
    "hd_resident_capacity": ([c_i32, c_i32, c_i32, c_i32, c_i32], c_i32),
    "hd_autotune_hybrid": ([c_vp, c_i32, c_i32, c_i64, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32,
                            c_vp, c_vp, c_vp, c_vp], c_i32),
    "hd_autotune_batched": ([c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp], c_i32),
    "surrogate_num_params": ([], c_i32),
    "surrogate_create": ([c_vp, c_vp], c_i32),
    "surrogate_destroy": ([c_vp], None),
    "surrogate_get_state": ([c_vp, c_vp, c_vp, c_vp, c_vp], c_i32),
    "surrogate_set_state": ([c_vp, c_vp, c_vp, c_vp, c_i32], c_i32),
    "surrogate_get_activation": ([c_vp, c_i32, c_vp, c_i64], c_i32),
    "surrogate_forward": ([c_vp, c_vp, c_i32, c_i32, c_i32, c_i64, c_i64, c_i32, c_i32, c_vp, c_i64,
                           c_i64, c_vp], c_i32),
    "surrogate_train_step": ([c_vp, c_vp, c_i32, c_i32, c_i32, c_i64, c_i64, c_i32, c_i32, c_vp,
                              ctypes.c_float, c_vp, c_vp, c_i32, c_vp], c_i32),
    "surrogate_denoise": ([c_vp, c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, ctypes.c_float,
                           ctypes.c_float, ctypes.c_float, ctypes.c_float, c_i32, ctypes.c_float, c_vp, c_vp,
                           c_vp], c_i32),
}

HD_OPT_SELECT, HD_OPT_FUSE_MOMENTS, HD_OPT_GRAPHS, HD_OPT_RESIDENT = 1, 2, 3, 4
HD_OPT_WAIT_LIMIT_US, HD_OPT_FAIL_ALLOC, HD_OPT_SURROGATE_FUSED, HD_OPT_TILE_ROWS = 5, 6, 7, 8


class HDSlice(ctypes.Structure):
    """Mirror of hd_slice in include/hybrid_denoise.h."""
    _fields_ = [("in_", c_vp), ("out", c_vp), ("h", c_i32), ("w", c_i32), ("in_pitch", c_i64),
                ("out_pitch", c_i64)]


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} not found: build it with `python -m paper_2005_05371_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != 0:
        raise HDError(rc, load().hd_last_error().decode(errors="replace"))


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.uint8:
        return HD_U8
    if t.dtype == torch.uint16:
        return HD_U16
    raise HDError(3, f"unsupported dtype {t.dtype}")


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _img(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit column stride")
    return t.data_ptr(), t.shape[0], t.shape[1], t.stride(0)


def default_max_value(t: torch.Tensor) -> int:
    return 255 if t.dtype == torch.uint8 else 4095


def amf_filter(inp: torch.Tensor, smax: int, out: Optional[torch.Tensor] = None,
               keep: bool = False, parts: int = 1, stream=None) -> torch.Tensor:
    """Adaptive median filter; ``out`` has the input's dtype and shape. With parts > 1 the
    image is filtered as `parts` independent horizontal strips (the paper's partitions)."""
    if out is None:
        out = torch.empty_like(inp)
    pi, h, w, ip = _img(inp, "input")
    po, ho, wo, op = _img(out, "output")
    if (ho, wo) != (h, w) or out.dtype != inp.dtype:
        raise ValueError("output must match the input's shape and dtype")
    flags = HD_AMF_UNRESOLVED_KEEP if keep else 0
    if parts == 1:
        _check(load().amf_filter(pi, po, h, w, ip, op, _dtype_code(inp), int(smax), flags,
                                 _stream(stream)))
    else:
        _check(load().amf_filter_parts(pi, po, h, w, ip, op, _dtype_code(inp), int(smax),
                                       int(parts), flags, _stream(stream)))
    return out


def hybrid_partitioned(inp: torch.Tensor, smax: int, win, max_value: Optional[int] = None,
                       parts: int = 2, stretch: bool = False, out: Optional[torch.Tensor] = None,
                       stream=None) -> torch.Tensor:
    """The paper's parallel hybrid (Alg. 1, procedure parallelHybrid): partitioned AMF over
    `parts` strips, then the Wiener filter (noise power estimated) of the whole image, then
    optionally the contrast stretch. Two library calls on `stream`."""
    a = amf_filter(inp, smax, parts=parts, stream=stream)
    mv = default_max_value(inp) if max_value is None else int(max_value)
    y = wiener_filter(a, win, mv, out=out, stream=stream)
    if stretch:
        contrast_stretch(y, stream=stream)
    return y


def degrade_image(clean: torch.Tensor, sigma: float, density: float, seed: int, stream_id: int = 0,
                  max_value: Optional[int] = None, out: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """Gaussian + salt-and-pepper degradation on the device (Philox4x32-10 counter-based
    random numbers; `out` may be `clean` for in place)."""
    if out is None:
        out = torch.empty_like(clean)
    pc, h, w, cp = _img(clean, "clean")
    po, ho, wo, op = _img(out, "noisy")
    if (ho, wo) != (h, w) or out.dtype != clean.dtype:
        raise ValueError("noisy must match the clean image's shape and dtype")
    mv = default_max_value(clean) if max_value is None else int(max_value)
    _check(load().degrade_image(pc, po, h, w, cp, op, _dtype_code(clean), mv, float(sigma),
                                float(density), int(seed) & 0xFFFFFFFFFFFFFFFF, int(stream_id),
                                _stream(stream)))
    return out


def wiener_fft(inp: torch.Tensor, original: torch.Tensor, max_value: Optional[int] = None,
               out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The paper's frequency-domain Wiener step wnrFn(inp, original); float32 / max_value."""
    if out is None:
        out = torch.empty(inp.shape, dtype=torch.float32, device=inp.device)
    pi, h, w, ip = _img(inp, "input")
    pf, hf, wf, fp = _img(original, "original")
    po, ho, wo, op = _img(out, "output")
    if (hf, wf) != (h, w) or original.dtype != inp.dtype or (ho, wo) != (h, w):
        raise ValueError("original and output must match the input's shape (original: and dtype)")
    mv = default_max_value(inp) if max_value is None else int(max_value)
    _check(load().wiener_fft(pi, pf, po, h, w, ip, fp, op, _dtype_code(inp), mv, _stream(stream)))
    return out


def hybrid_paper(noisy: torch.Tensor, original: torch.Tensor, smax: int, parts: int = 1,
                 max_value: Optional[int] = None, stretch: bool = True,
                 out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Alg. 1, procedure parallelHybrid as printed: partitioned AMF (parts strips), the
    frequency-domain Wiener step with the clean original, the contrast stretch."""
    a = amf_filter(noisy, smax, parts=parts, stream=stream)
    y = wiener_fft(a, original, max_value, out=out, stream=stream)
    if stretch:
        contrast_stretch(y, stream=stream)
    return y


def contrast_stretch(img: torch.Tensor, stream=None) -> torch.Tensor:
    """In-place min-max contrast stretch of a float32 GPU image (Alg. 1, step e)."""
    if img.dtype != torch.float32:
        raise ValueError("contrast_stretch takes a float32 image")
    p, h, w, pitch = _img(img, "image")
    _check(load().contrast_stretch(p, h, w, pitch, _stream(stream)))
    return img


def wiener_filter(inp: torch.Tensor, win, max_value: Optional[int] = None,
                  noise_var: float = -1.0, out: Optional[torch.Tensor] = None,
                  nu2_out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Adaptive Wiener filter of an integer image; float32 output / max_value."""
    wh, ww = (win, win) if isinstance(win, int) else win
    if out is None:
        out = torch.empty(inp.shape, dtype=torch.float32, device=inp.device)
    pi, h, w, ip = _img(inp, "input")
    po, _, _, op = _img(out, "output")
    mv = default_max_value(inp) if max_value is None else int(max_value)
    nu = nu2_out.data_ptr() if nu2_out is not None else None
    _check(load().wiener_filter(pi, po, h, w, ip, op, _dtype_code(inp), mv, int(wh), int(ww),
                                float(noise_var), nu, _stream(stream)))
    return out


def _flags(keep: bool, stretch: bool) -> int:
    return (HD_AMF_UNRESOLVED_KEEP if keep else 0) | (HD_CONTRAST_STRETCH if stretch else 0)


def hybrid_denoise(inp: torch.Tensor, smax: int, win, max_value: Optional[int] = None,
                   noise_var: float = -1.0, keep: bool = False,
                   out: Optional[torch.Tensor] = None, amf_out: Optional[torch.Tensor] = None,
                   nu2_out: Optional[torch.Tensor] = None, stretch: bool = False,
                   stream=None) -> torch.Tensor:
    """Wiener(AMF(inp)); float32 output / max_value (contrast-stretched with `stretch`)."""
    wh, ww = (win, win) if isinstance(win, int) else win
    if out is None:
        out = torch.empty(inp.shape, dtype=torch.float32, device=inp.device)
    pi, h, w, ip = _img(inp, "input")
    po, _, _, op = _img(out, "output")
    mv = default_max_value(inp) if max_value is None else int(max_value)
    pa, ap = (None, 0)
    if amf_out is not None:
        pa, _, _, ap = _img(amf_out, "amf_out")
    nu = nu2_out.data_ptr() if nu2_out is not None else None
    _check(load().hybrid_denoise(pi, po, h, w, ip, op, _dtype_code(inp), mv, int(smax), int(wh),
                                 int(ww), float(noise_var), _flags(keep, stretch), pa, ap, nu,
                                 _stream(stream)))
    return out


def hybrid_denoise_noalloc(inp: torch.Tensor, smax: int, win, max_value: Optional[int] = None,
                           noise_var: float = -1.0, keep: bool = False, out: Optional[torch.Tensor] = None,
                           stretch: bool = False, stream=None) -> torch.Tensor:
    """hybrid_denoise whose scratch is the library's static device array (no allocation in
    the library; `out` must be given by a caller that cannot allocate either)."""
    wh, ww = (win, win) if isinstance(win, int) else win
    if out is None:
        out = torch.empty(inp.shape, dtype=torch.float32, device=inp.device)
    pi, h, w, ip = _img(inp, "input")
    po, _, _, op = _img(out, "output")
    mv = default_max_value(inp) if max_value is None else int(max_value)
    _check(load().hybrid_denoise_noalloc(pi, po, h, w, ip, op, _dtype_code(inp), mv, int(smax), int(wh),
                                         int(ww), float(noise_var), _flags(keep, stretch), None, 0, None,
                                         _stream(stream)))
    return out


def hybrid_denoise_batched(inputs, smax: int, win, max_value: Optional[int] = None,
                           noise_var: float = -1.0, keep: bool = False, outs=None,
                           stretch: bool = False, stream=None):
    """Wiener(AMF(x)) for every image of `inputs` (GPU tensors of one dtype, any sizes),
    in one batched call (captured graph, replayed on later calls with the same buffers)."""
    wh, ww = (win, win) if isinstance(win, int) else win
    if not inputs:
        raise ValueError("no slices")
    if outs is None:
        outs = [torch.empty(x.shape, dtype=torch.float32, device=x.device) for x in inputs]
    arr = (HDSlice * len(inputs))()
    for i, (x, o) in enumerate(zip(inputs, outs)):
        pi, h, w, ip = _img(x, f"input {i}")
        po, ho, wo, op = _img(o, f"output {i}")
        if (ho, wo) != (h, w) or o.dtype != torch.float32:
            raise ValueError(f"output {i} must be float32 of the input's shape")
        arr[i] = HDSlice(pi, po, h, w, ip, op)
    code = _dtype_code(inputs[0])
    if any(_dtype_code(x) != code for x in inputs):
        raise ValueError("all slices must share one dtype")
    mv = default_max_value(inputs[0]) if max_value is None else int(max_value)
    _check(load().hybrid_denoise_batched(ctypes.cast(arr, c_vp), len(inputs), code, mv, int(smax),
                                         int(wh), int(ww), float(noise_var),
                                         _flags(keep, stretch), _stream(stream)))
    return outs


HD_STAGES = 5
STAGE_NAMES = ("amf_stage", "noise_sums", "noise_reduce", "wiener_apply", "contrast_stretch")


def _slice_array(inputs, outs):
    arr = (HDSlice * len(inputs))()
    for i, (x, o) in enumerate(zip(inputs, outs)):
        pi, h, w, ip = _img(x, f"input {i}")
        po, ho, wo, op = _img(o, f"output {i}")
        if (ho, wo) != (h, w) or o.dtype != torch.float32:
            raise ValueError(f"output {i} must be float32 of the input's shape")
        arr[i] = HDSlice(pi, po, h, w, ip, op)
    code = _dtype_code(inputs[0])
    if any(_dtype_code(x) != code for x in inputs):
        raise ValueError("all slices must share one dtype")
    return arr, code


def hybrid_denoise_batched_timed(inputs, smax: int, win, max_value: Optional[int] = None,
                                 noise_var: float = -1.0, keep: bool = False, outs=None,
                                 stretch: bool = False, stream=None):
    """One batched step with each stage kernel timed by HIP events on `stream`; returns
    (outs, {stage name: milliseconds}) for the stages the step runs."""
    wh, ww = (win, win) if isinstance(win, int) else win
    if not inputs:
        raise ValueError("no slices")
    if outs is None:
        outs = [torch.empty(x.shape, dtype=torch.float32, device=x.device) for x in inputs]
    arr, code = _slice_array(inputs, outs)
    mv = default_max_value(inputs[0]) if max_value is None else int(max_value)
    ms = (ctypes.c_float * HD_STAGES)()
    _check(load().hybrid_denoise_batched_timed(ctypes.cast(arr, c_vp), len(inputs), code, mv, int(smax),
                                               int(wh), int(ww), float(noise_var), _flags(keep, stretch),
                                               ctypes.cast(ms, c_vp), _stream(stream)))
    return outs, {STAGE_NAMES[i]: float(ms[i]) for i in range(HD_STAGES) if ms[i] > 0.0}


def release_plans():
    load().hd_release_plans()


def check_errors(stream=None):
    """Synchronise `stream`; raise HDError (HD_ERR_TIMEOUT) if a wait of the single-launch
    exchange gave up on the current device since the last check."""
    _check(load().hd_check_errors(_stream(stream)))


def set_option(key: int, value: int):
    _check(load().hd_set_option(int(key), int(value)))


def autotune_hybrid(inp: torch.Tensor, smax: int, win, max_value: Optional[int] = None,
                    iters: int = 10, stream=None):
    """Time every strategy on `inp`; returns (select_mode, fuse, tile_rows) chosen for this key."""
    wh, ww = (win, win) if isinstance(win, int) else win
    pi, h, w, ip = _img(inp, "input")
    mv = default_max_value(inp) if max_value is None else int(max_value)
    sel, fuse, rows = ctypes.c_int32(-1), ctypes.c_int32(-1), ctypes.c_int32(-1)
    _check(load().hd_autotune_hybrid(pi, h, w, ip, _dtype_code(inp), mv, int(smax), int(wh), int(ww),
                                     int(iters), ctypes.addressof(sel), ctypes.addressof(fuse),
                                     ctypes.addressof(rows), _stream(stream)))
    return sel.value, fuse.value, rows.value


def autotune_batched(inputs, smax: int, win, max_value: Optional[int] = None, iters: int = 3,
                     outs=None, stream=None):
    """Time every strategy on the batch itself (writes the outputs); returns (select, fuse,
    tile_rows)."""
    wh, ww = (win, win) if isinstance(win, int) else win
    if outs is None:
        outs = [torch.empty(x.shape, dtype=torch.float32, device=x.device) for x in inputs]
    arr, code = _slice_array(inputs, outs)
    mv = default_max_value(inputs[0]) if max_value is None else int(max_value)
    sel, fuse, rows = ctypes.c_int32(-1), ctypes.c_int32(-1), ctypes.c_int32(-1)
    _check(load().hd_autotune_batched(ctypes.cast(arr, c_vp), len(inputs), code, mv, int(smax), int(wh), int(ww),
                                      int(iters), ctypes.addressof(sel), ctypes.addressof(fuse),
                                      ctypes.addressof(rows), _stream(stream)))
    return sel.value, fuse.value, rows.value


def resident_capacity(dtype, smax: int, win, select_mode: int = -1) -> int:
    """Largest tile count (64 x 32 tiles, summed over a call's slices) that runs as one
    resident launch on the current device; `dtype` is a torch dtype (uint8 / uint16)."""
    wh, ww = (win, win) if isinstance(win, int) else win
    code = HD_U8 if dtype == torch.uint8 else HD_U16
    return int(load().hd_resident_capacity(code, int(smax), int(wh), int(ww), int(select_mode)))


def tiles_of(h: int, w: int) -> int:
    """Number of 64 x 32 output tiles of an h x w image."""
    return ((w + 63) // 64) * ((h + 31) // 32)


def _batch(t: torch.Tensor, name: str):
    """(B, H, W) GPU tensor with unit column stride -> (ptr, B, H, W, pitch, image stride)."""
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3 or t.stride(2) != 1:
        raise ValueError(f"{name} must be (B, H, W) with unit column stride")
    return t.data_ptr(), t.shape[0], t.shape[1], t.shape[2], t.stride(1), t.stride(0)


class Surrogate:
    """Handle on a device-resident surrogate network (parameters, Adam state, workspace)."""

    def __init__(self, params=None):
        import numpy as np
        self._h = ctypes.c_void_p()
        arr = None
        if params is not None:
            arr = np.ascontiguousarray(params, dtype=np.float32)
            if arr.size != self.num_params():
                raise ValueError("wrong parameter count")
        _check(load().surrogate_create(ctypes.byref(self._h),
                                       arr.ctypes.data_as(c_vp) if arr is not None else None))

    @staticmethod
    def num_params() -> int:
        return int(load().surrogate_num_params())

    def close(self):
        if self._h:
            load().surrogate_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_state(self):
        import numpy as np
        n = self.num_params()
        p, m, v = (np.empty(n, np.float32) for _ in range(3))
        step = ctypes.c_int32(0)
        _check(load().surrogate_get_state(self._h, p.ctypes.data_as(c_vp), m.ctypes.data_as(c_vp),
                                          v.ctypes.data_as(c_vp), ctypes.addressof(step)))
        return {"params": p, "m": m, "v": v, "step": int(step.value)}

    def set_state(self, params=None, m=None, v=None, step: int = 0):
        import numpy as np
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32) for a in (params, m, v)]
        ptrs = [None if a is None else a.ctypes.data_as(c_vp) for a in arrs]
        _check(load().surrogate_set_state(self._h, *ptrs, int(step)))

    def forward(self, x: torch.Tensor, max_value: Optional[int] = None, out=None, stream=None):
        pi, B, H, W, ip, istr = _batch(x, "input")
        if out is None:
            out = torch.empty((B, H, W), dtype=torch.float32, device=x.device)
        po, Bo, Ho, Wo, op, ostr = _batch(out, "output")
        mv = default_max_value(x) if max_value is None else int(max_value)
        _check(load().surrogate_forward(self._h, pi, B, H, W, ip, istr, _dtype_code(x), mv, po, op, ostr,
                                        _stream(stream)))
        self._last_shape = (B, H, W)
        return out

    def activation(self, layer: int):
        """Host copy of the stored activation A_layer (1..5) of the last forward or training
        step: float32 array (B, H, W, 32) holding the bf16 values."""
        import numpy as np
        B, H, W = getattr(self, "_last_shape", (0, 0, 0))
        bits = np.empty((B, H, W, 32), np.uint16)
        _check(load().surrogate_get_activation(self._h, int(layer), bits.ctypes.data_as(c_vp), bits.size))
        return (bits.astype(np.uint32) << 16).view(np.float32)

    def train_step(self, x: torch.Tensor, target: torch.Tensor, lr: float = 1e-3,
                   max_value: Optional[int] = None, apply: bool = True, want_grad: bool = False,
                   stream=None):
        """One step; returns (loss tensor [1], gradient tensor or None) on the GPU."""
        pi, B, H, W, ip, istr = _batch(x, "input")
        t = target.reshape(B, H, W)
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("target must be a contiguous float32 GPU tensor (B, H, W)")
        loss = torch.zeros(1, dtype=torch.float32, device=x.device)
        grad = torch.empty(self.num_params(), dtype=torch.float32, device=x.device) if want_grad else None
        mv = default_max_value(x) if max_value is None else int(max_value)
        self._last_shape = (B, H, W)
        _check(load().surrogate_train_step(self._h, pi, B, H, W, ip, istr, _dtype_code(x), mv, t.data_ptr(),
                                           float(lr), loss.data_ptr(),
                                           grad.data_ptr() if grad is not None else None,
                                           1 if apply else 0, _stream(stream)))
        return loss, grad

    def denoise(self, inputs, smax: int, win, calib, threshold: float, max_value: Optional[int] = None,
                outs=None, want_scores: bool = False, check_smax: int = 3, stream=None):
        """Surrogate + per-tile check + plain fallback. calib = (p_max, r_lo, r_hi) or
        (p_max, r_lo, r_hi, d_hi) with the deviation bound against the plain output's proxy
        (the plain hybrid with the AMF stopped at check_smax). Returns (outs, n_fallback
        work tiles (int), scores tensor or None)."""
        wh, ww = (win, win) if isinstance(win, int) else win
        if outs is None:
            outs = [torch.empty(x.shape, dtype=torch.float32, device=x.device) for x in inputs]
        arr = (HDSlice * len(inputs))()
        n_check = 0
        for i, (x, o) in enumerate(zip(inputs, outs)):
            pi, h, w, ip = _img(x, f"input {i}")
            po, _, _, op = _img(o, f"output {i}")
            arr[i] = HDSlice(pi, po, h, w, ip, op)
            n_check += ((h + 63) // 64) * ((w + 63) // 64)
        mv = default_max_value(inputs[0]) if max_value is None else int(max_value)
        nfb = torch.zeros(1, dtype=torch.int32, device=inputs[0].device)
        scores = torch.empty(n_check, dtype=torch.float32, device=inputs[0].device) if want_scores else None
        p_max, r_lo, r_hi = (float(c) for c in calib[:3])
        d_hi = float(calib[3]) if len(calib) > 3 else 0.0
        _check(load().surrogate_denoise(self._h, ctypes.cast(arr, c_vp), len(inputs), _dtype_code(inputs[0]), mv,
                                        int(smax), int(wh), int(ww), p_max, r_lo, r_hi, d_hi, int(check_smax),
                                        float(threshold), nfb.data_ptr(),
                                        scores.data_ptr() if scores is not None else None, _stream(stream)))
        return outs, int(nfb.item()), scores
