"""Python binding of ``libbdis.so`` (ctypes), argument marshalling only.

PyTorch supplies device memory and streams; every step of the computation
runs in the library's HIP kernels.  If the library is not built this module
raises on first use: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbdis.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bdis.h")

OK, E_ARG, E_SIZE, E_CAPACITY, E_HIP, E_NOMEM, E_STATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_SIZE", -3: "E_CAPACITY", -4: "E_HIP", -5: "E_NOMEM",
                -6: "E_STATE"}
DBG = dict(left=0, right=1, uinit=2, pipar=3, u=4, ssd0=5, dssd=6, rho=7, acc=8, hess=9, dens=10,
           ubar=11, qmap=12, scal=13)


class Params(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32), ("finest_level", ctypes.c_int32), ("patch", ctypes.c_int32),
        ("stride", ctypes.c_int32), ("iters", ctypes.c_int32), ("sigma_r_dynamic", ctypes.c_int32),
        ("variance", ctypes.c_int32), ("float_pyramid", ctypes.c_int32),
        ("sigma_s", ctypes.c_float), ("sigma_r", ctypes.c_float), ("valid_ratio", ctypes.c_float),
        ("var_fail_sigma", ctypes.c_float), ("var_fit_thresh", ctypes.c_float),
        ("prob_thresh", ctypes.c_float), ("level_weight", ctypes.c_float * 8),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "level_weight"}
        d["level_weight"] = list(self.level_weight)
        return d


class Pair(ctypes.Structure):
    _fields_ = [("left", ctypes.c_void_p), ("right", ctypes.c_void_p), ("w", ctypes.c_int32),
                ("h", ctypes.c_int32), ("pitch", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("disparity", ctypes.c_void_p), ("variance", ctypes.c_void_p),
                ("confidence", ctypes.c_void_p)]


class BdisError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load ``libbdis.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run paper_2205_03133_amd.build.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int
        pp = ctypes.POINTER(Params)
        L.bdis_params_default.argtypes = [pp]
        L.bdis_params_check.argtypes = [pp]
        L.bdis_create.argtypes = [ctypes.POINTER(vp), pp, i32, i32, i32, ctypes.c_uint]
        L.bdis_set_params.argtypes = [vp, pp]
        L.bdis_compute.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp, vp]
        L.bdis_compute_batch.argtypes = [vp, i32, ctypes.POINTER(Pair), vp]
        L.bdis_debug_dump.argtypes = [vp, i32, i32, vp, ctypes.c_size_t, vp]
        L.bdis_level_dims.argtypes = [pp, i32, i32, i32] + [ctypes.POINTER(i32)] * 4
        L.bdis_destroy.argtypes = [vp]
        L.bdis_destroy.restype = None
        L.bdis_last_error.argtypes = [vp]
        L.bdis_last_error.restype = ctypes.c_char_p
        L.bdis_version.restype = ctypes.c_char_p
        L.bdis_timing_enable.argtypes = [vp, i32]
        L.bdis_timing_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_long)]
        for name in ("bdis_params_default", "bdis_params_check", "bdis_create", "bdis_set_params",
                     "bdis_compute", "bdis_compute_batch", "bdis_debug_dump", "bdis_level_dims",
                     "bdis_timing_enable", "bdis_timing_read"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def header_functions():
    """Names of the functions ``include/bdis.h`` declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bdis_[a-z0-9_]+)\s*\(", txt)))


def params(**overrides):
    """Library defaults (Sec. IV-A values where the paper gives them), with overrides."""
    p = Params()
    st = lib().bdis_params_default(ctypes.byref(p))
    assert st == OK
    for k, v in overrides.items():
        if k == "level_weight":
            lw = list(v) + [0.0] * (8 - len(v))
            p.level_weight = (ctypes.c_float * 8)(*lw[:8])
        elif not hasattr(p, k):
            raise KeyError(k)
        else:
            setattr(p, k, v)
    return p


def check(p):
    return lib().bdis_params_check(ctypes.byref(p))


def level_dims(p, w, h, level):
    out = [ctypes.c_int() for _ in range(4)]
    st = lib().bdis_level_dims(ctypes.byref(p), w, h, level, *[ctypes.byref(o) for o in out])
    if st:
        raise BdisError(st, "level_dims")
    return tuple(o.value for o in out)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _image_arg(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.uint8 or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D uint8 CUDA tensor")
    if t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    return t.data_ptr(), t.shape[1], t.shape[0], t.stride(0)


class Context:
    """Owns a ``bdis_ctx`` (device workspace sized for max_w x max_h x max_batch)."""

    def __init__(self, p, max_w, max_h, max_batch=1):
        self._h = ctypes.c_void_p()
        self.params = p
        st = lib().bdis_create(ctypes.byref(self._h), ctypes.byref(p), max_w, max_h, max_batch, 0)
        if st:
            raise BdisError(st, lib().bdis_last_error(None).decode())
        self.max_w, self.max_h, self.max_batch = max_w, max_h, max_batch

    def _err(self, st):
        return BdisError(st, lib().bdis_last_error(self._h).decode())

    def close(self):
        if self._h:
            lib().bdis_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_params(self, p):
        st = lib().bdis_set_params(self._h, ctypes.byref(p))
        if st:
            raise self._err(st)
        self.params = p

    def compute(self, left, right, *, variance=None, confidence=True, out=None, stream=None):
        """Disparity (and variance / confidence) of one uint8 pair on the GPU.

        Returns ``dict(disp, var, conf)`` of float32 CUDA tensors (``var``/``conf``
        None when not requested).  ``out`` may hold preallocated tensors.
        """
        import torch
        lp, w, h, pitch = _image_arg(left, "left")
        rp, w2, h2, pitch2 = _image_arg(right, "right")
        if (w, h, pitch) != (w2, h2, pitch2):
            raise ValueError("left and right must have the same shape and row stride")
        if variance is None:
            variance = bool(self.params.variance)
        out = dict(out or {})
        dev = left.device
        disp = out.get("disp")
        if disp is None:
            disp = torch.empty((h, w), dtype=torch.float32, device=dev)
        var = out.get("var") if variance else None
        if variance and var is None:
            var = torch.empty((h, w), dtype=torch.float32, device=dev)
        conf = out.get("conf") if confidence else None
        if confidence and conf is None:
            conf = torch.empty((h, w), dtype=torch.float32, device=dev)
        st = lib().bdis_compute(self._h, lp, rp, w, h, pitch, disp.data_ptr(),
                                var.data_ptr() if var is not None else None,
                                conf.data_ptr() if conf is not None else None, _stream_ptr(stream))
        if st:
            raise self._err(st)
        self._last_wh = (w, h)
        return dict(disp=disp, var=var, conf=conf)

    def compute_batch(self, lefts, rights, levels=None, *, variance=None, confidence=True, outs=None,
                      stream=None):
        """A batch of uint8 pairs (lists of 2-D tensors, sizes may differ) in one call."""
        import torch
        n = len(lefts)
        if variance is None:
            variance = bool(self.params.variance)
        arr = (Pair * max(n, 1))()
        results = []
        for i in range(n):
            lp, w, h, pitch = _image_arg(lefts[i], "left")
            rp, w2, h2, pitch2 = _image_arg(rights[i], "right")
            if (w, h, pitch) != (w2, h2, pitch2):
                raise ValueError("left and right must match")
            o = outs[i] if outs is not None else {}
            dev = lefts[i].device
            disp = o.get("disp")
            if disp is None:
                disp = torch.empty((h, w), dtype=torch.float32, device=dev)
            var = o.get("var") if variance else None
            if variance and var is None:
                var = torch.empty((h, w), dtype=torch.float32, device=dev)
            conf = o.get("conf") if confidence else None
            if confidence and conf is None:
                conf = torch.empty((h, w), dtype=torch.float32, device=dev)
            lv = 0 if levels is None else int(levels[i])
            arr[i] = Pair(lp, rp, w, h, pitch, lv, disp.data_ptr(),
                          var.data_ptr() if var is not None else None,
                          conf.data_ptr() if conf is not None else None)
            results.append(dict(disp=disp, var=var, conf=conf))
        st = lib().bdis_compute_batch(self._h, n, arr, _stream_ptr(stream))
        if st:
            raise self._err(st)
        return results

    KERNELS = ("pyramid", "search", "prob", "fuse", "reduce")

    def timing(self, enable):
        """Start (clearing totals) or stop per-kernel HIP-event timing."""
        st = lib().bdis_timing_enable(self._h, 1 if enable else 0)
        if st:
            raise self._err(st)

    def timing_read(self):
        """{kernel: (total_ms, launches)} since timing was enabled (synchronises)."""
        out = {}
        for k, name in enumerate(self.KERNELS):
            ms, n = ctypes.c_double(), ctypes.c_long()
            st = lib().bdis_timing_read(self._h, k, ctypes.byref(ms), ctypes.byref(n))
            if st:
                raise self._err(st)
            out[name] = (ms.value, n.value)
        return out

    def debug(self, level, what, stream=None):
        """Intermediate array of the last single-pair compute, copied to the host."""
        p = self.params
        w, h, nx, ny = self._last_dims(level)
        if what in ("left", "right"):
            shape, dt = (h, w), np.uint8
        elif what in ("ubar", "qmap"):
            shape, dt = (h, w), np.float64
        elif what in ("dssd", "dens"):
            shape, dt = (ny, nx, 4), np.float64
        elif what == "acc":
            shape, dt = (ny, nx), np.int32
        elif what == "scal":
            shape, dt = (2,), np.float64
        elif what in ("rho", "hess"):
            shape, dt = (ny, nx), np.float32
        else:
            shape, dt = (ny, nx), np.float64
        buf = np.empty(shape, dt)
        st = lib().bdis_debug_dump(self._h, level, DBG[what], buf.ctypes.data, buf.nbytes,
                                   _stream_ptr(stream))
        if st:
            raise self._err(st)
        return buf

    def _last_dims(self, level):
        w, h = self._last_wh
        return level_dims(self.params, w, h, level)


def compute(left, right, p, **kw):
    """One-shot helper: create a context for this pair, compute, destroy."""
    h, w = left.shape
    with Context(p, w, h) as ctx:
        res = ctx.compute(left, right, **kw)
        import torch
        torch.cuda.current_stream().synchronize()
        return res
