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
        ("fusion", ctypes.c_int32), ("propagate", ctypes.c_int32),
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


class PairF32(ctypes.Structure):
    _fields_ = [("left", ctypes.c_void_p), ("right", ctypes.c_void_p), ("w", ctypes.c_int32),
                ("h", ctypes.c_int32), ("pitch", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("disparity", ctypes.c_void_p), ("variance", ctypes.c_void_p),
                ("confidence", ctypes.c_void_p)]


class PairGrad(ctypes.Structure):
    _fields_ = [("grad_disparity", ctypes.c_void_p), ("grad_variance", ctypes.c_void_p),
                ("grad_left", ctypes.c_void_p), ("grad_right", ctypes.c_void_p)]


TRAIN = 1
KEEP = 2


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
        L.bdis_compute_static.argtypes = [pp, vp, vp, i32, i32, i32, vp, vp, vp, vp]
        L.bdis_debug_dump.argtypes = [vp, i32, i32, vp, ctypes.c_size_t, vp]
        L.bdis_level_dims.argtypes = [pp, i32, i32, i32] + [ctypes.POINTER(i32)] * 4
        L.bdis_destroy.argtypes = [vp]
        L.bdis_destroy.restype = None
        L.bdis_last_error.argtypes = [vp]
        L.bdis_last_error.restype = ctypes.c_char_p
        L.bdis_version.restype = ctypes.c_char_p
        L.bdis_compute_f32.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp, vp]
        L.bdis_compute_f32_batch.argtypes = [vp, i32, ctypes.POINTER(PairF32), vp]
        L.bdis_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.bdis_backward_batch.argtypes = [vp, i32, ctypes.POINTER(PairGrad), vp, vp]
        L.bdis_timing_enable.argtypes = [vp, i32]
        L.bdis_timing_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_long)]
        L.bdis_setup_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.bdis_timing_read_level.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_long)]
        L.bdis_depth.argtypes = [vp, vp, vp, i32, i32, i32, ctypes.c_float, vp, vp, vp]
        L.bdis_flow.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp]
        L.bdis_coverage.argtypes = [vp, vp, vp, vp, vp, i32, i32, i32, ctypes.c_float, vp, vp]
        for name in ("bdis_params_default", "bdis_params_check", "bdis_create", "bdis_set_params",
                     "bdis_compute", "bdis_compute_batch", "bdis_compute_static", "bdis_debug_dump", "bdis_level_dims",
                     "bdis_timing_enable", "bdis_timing_read", "bdis_timing_read_level", "bdis_setup_time", "bdis_compute_f32", "bdis_compute_f32_batch",
                     "bdis_backward", "bdis_backward_batch"):
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


def _image_arg(t, name, dtype=None):
    import torch
    dtype = torch.uint8 if dtype is None else dtype
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D {dtype} CUDA tensor")
    if t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    return t.data_ptr(), t.shape[1], t.shape[0], t.stride(0)


def compute_static(p, left, right, *, variance=None, confidence=True, out=None, stream=None):
    """One uint8 pair through ``bdis_compute_static`` (no context, no allocation
    inside the library: its workspace is a static device array).  Output
    tensors are allocated here unless ``out`` holds them.  Returns
    ``dict(disp, var, conf)`` as ``Context.compute``."""
    import torch
    lp, w, h, pitch = _image_arg(left, "left")
    rp, w2, h2, pitch2 = _image_arg(right, "right")
    if (w, h, pitch) != (w2, h2, pitch2) or left.device != right.device:
        raise ValueError("left and right must have the same shape, row stride and device")
    if variance is None:
        variance = bool(p.variance)
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
    with torch.cuda.device(dev):
        st = lib().bdis_compute_static(ctypes.byref(p), lp, rp, w, h, pitch, disp.data_ptr(),
                                       var.data_ptr() if var is not None else None,
                                       conf.data_ptr() if conf is not None else None, _stream_ptr(stream))
    if st:
        raise BdisError(st, lib().bdis_last_error(None).decode())
    return dict(disp=disp, var=var, conf=conf)


class Context:
    """Owns a ``bdis_ctx`` (device workspace sized for max_w x max_h x max_batch).
    ``keep`` stores every per-patch intermediate for ``debug`` (BDIS_KEEP)."""

    def __init__(self, p, max_w, max_h, max_batch=1, train=False, keep=False):
        self._h = ctypes.c_void_p()
        self.params = p
        self.train = train
        st = lib().bdis_create(ctypes.byref(self._h), ctypes.byref(p), max_w, max_h, max_batch,
                               (TRAIN if train else 0) | (KEEP if keep else 0))
        if st:
            raise BdisError(st, lib().bdis_last_error(None).decode())
        self.max_w, self.max_h, self.max_batch = max_w, max_h, max_batch
        import torch
        self.device = torch.device("cuda", torch.cuda.current_device())

    def _on_device(self, *tensors):
        for t in tensors:
            if t is not None and t.device != self.device:
                raise ValueError(f"tensor on {t.device}; this context lives on {self.device}")

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
        self._on_device(left, right)
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
            self._on_device(lefts[i], rights[i])
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

    def flow(self, i0, i1, stream=None):
        """Optical flow (u, v) between two uint8 frames (2-D CUDA tensors, same shape)."""
        import torch
        self._on_device(i0, i1)
        p0, w, h, pitch = _image_arg(i0, "i0")
        p1, w2, h2, pitch2 = _image_arg(i1, "i1")
        if (w, h, pitch) != (w2, h2, pitch2):
            raise ValueError("frames must have the same shape and row stride")
        u = torch.empty((h, w), dtype=torch.float32, device=i0.device)
        v = torch.empty((h, w), dtype=torch.float32, device=i0.device)
        st = lib().bdis_flow(self._h, p0, p1, w, h, pitch, u.data_ptr(), v.data_ptr(), _stream_ptr(stream))
        if st:
            raise self._err(st)
        self._last_wh = (w, h)
        return u, v

    def depth(self, disp, fb, var=None, stream=None):
        """Depth fb / d (and its variance (fb)^2 / d^4 var) of a disparity map
        (float32 CUDA tensor, contiguous rows).  Returns (depth, depth_var or None)."""
        import torch
        dp, w, h, pitch = _image_arg(disp, "disparity", torch.float32)
        vp = None
        if var is not None:
            vp, w2, h2, pitch2 = _image_arg(var, "variance", torch.float32)
            if (w2, h2, pitch2) != (w, h, pitch):
                raise ValueError("variance must match the disparity map")
        depth = torch.empty((h, w), dtype=torch.float32, device=disp.device)
        dvar = torch.empty((h, w), dtype=torch.float32, device=disp.device) if var is not None else None
        st = lib().bdis_depth(self._h, dp, vp, w, h, pitch, float(fb), depth.data_ptr(),
                              dvar.data_ptr() if dvar is not None else None, _stream_ptr(stream))
        if st:
            raise self._err(st)
        return depth, dvar

    def coverage(self, disp, var, ref, k=1.96, valid=None, stream=None):
        """Variance coverage of one frame: (covered, considered) pixel counts of
        |d - ref| <= k sqrt(var) (float32 CUDA maps, shared row stride; `valid`
        an optional uint8 mask).  Synchronises the stream to return the counts."""
        import torch
        dp, w, h, pitch = _image_arg(disp, "disparity", torch.float32)
        vp_, w2, h2, p2 = _image_arg(var, "variance", torch.float32)
        rp, w3, h3, p3 = _image_arg(ref, "reference", torch.float32)
        if not (w == w2 == w3 and h == h2 == h3 and pitch == p2 == p3):
            raise ValueError("disparity, variance and reference must share shape and row stride")
        mp = None
        if valid is not None:
            mp, w4, h4, p4 = _image_arg(valid, "valid", torch.uint8)
            if (w4, h4, p4) != (w, h, pitch):
                raise ValueError("valid must share shape and row stride")
        counts = torch.empty(2, dtype=torch.int64, device=disp.device)
        st = lib().bdis_coverage(self._h, dp, vp_, rp, mp, w, h, pitch, float(k), counts.data_ptr(),
                                 _stream_ptr(stream))
        if st:
            raise self._err(st)
        c = counts.cpu()
        return int(c[0]), int(c[1])

    KERNELS = ("pyramid", "search", "prob", "fuse", "reduce", "backward", "top")

    def timing(self, enable):
        """Start (clearing totals) or stop per-kernel HIP-event timing."""
        st = lib().bdis_timing_enable(self._h, 1 if enable else 0)
        if st:
            raise self._err(st)

    def setup_time(self):
        """(tune_ms, capture_ms): host time the last compute call spent tuning and
        capturing its graph (0 when it did neither)."""
        t, c = ctypes.c_double(), ctypes.c_double()
        st = lib().bdis_setup_time(self._h, ctypes.byref(t), ctypes.byref(c))
        if st:
            raise self._err(st)
        return t.value, c.value

    def timing_read(self, level=-1):
        """{kernel: (total_ms, launches)} since timing was enabled (synchronises);
        one pyramid level's launches when ``level`` >= 0."""
        out = {}
        for k, name in enumerate(self.KERNELS):
            ms, n = ctypes.c_double(), ctypes.c_long()
            st = lib().bdis_timing_read_level(self._h, k, level, ctypes.byref(ms), ctypes.byref(n))
            if st:
                raise self._err(st)
            out[name] = (ms.value, n.value)
        return out

    def compute_f32(self, lefts, rights, *, variance=None, confidence=True, stream=None):
        """Float path on a batch: lefts/rights are (B, H, W) or (H, W) float32 CUDA tensors
        (contiguous rows).  Returns dict(disp, var, conf) shaped like the input."""
        import torch
        single = lefts.dim() == 2
        self._on_device(lefts, rights)
        L = lefts[None] if single else lefts
        R = rights[None] if single else rights
        if L.dtype != torch.float32 or R.dtype != torch.float32 or not L.is_cuda or L.shape != R.shape:
            raise TypeError("float path needs equal float32 CUDA tensors")
        if L.stride(-1) != 1 or R.stride(-1) != 1 or L.stride(-2) != R.stride(-2):
            raise ValueError("rows must be contiguous with equal pitch")
        if variance is None:
            variance = bool(self.params.variance)
        B, h, w = L.shape
        disp = torch.empty((B, h, w), dtype=torch.float32, device=L.device)
        var = torch.empty((B, h, w), dtype=torch.float32, device=L.device) if variance else None
        conf = torch.empty((B, h, w), dtype=torch.float32, device=L.device) if confidence else None
        arr = (PairF32 * B)()
        for b in range(B):
            arr[b] = PairF32(L[b].data_ptr(), R[b].data_ptr(), w, h, L.stride(-2), 0, disp[b].data_ptr(),
                             var[b].data_ptr() if var is not None else None,
                             conf[b].data_ptr() if conf is not None else None)
        st = lib().bdis_compute_f32_batch(self._h, B, arr, _stream_ptr(stream))
        if st:
            raise self._err(st)
        self._last_f32 = (B, h, w, L.device)
        # backward differentiates the latest float call only: callers that keep
        # several calls' graphs check this counter (see the autograd Function)
        self.f32_generation = getattr(self, "f32_generation", 0) + 1
        if single:
            return dict(disp=disp[0], var=var[0] if var is not None else None,
                        conf=conf[0] if conf is not None else None)
        return dict(disp=disp, var=var, conf=conf)

    def backward(self, grad_disp, grad_var=None, stream=None):
        """Reverse mode through the last compute_f32: returns (grad_left, grad_right, grad_hyper)
        with grad_hyper = [sigma_s, sigma_r (alpha_r when dynamic), omega_0 .. omega_{L-1}]."""
        import torch
        B, h, w, dev = self._last_f32
        gd = grad_disp.reshape(B, h, w).to(device=dev, dtype=torch.float32).contiguous()
        gv = (grad_var.reshape(B, h, w).to(device=dev, dtype=torch.float32).contiguous()
              if grad_var is not None else None)
        gl = torch.empty((B, h, w), dtype=torch.float32, device=dev)
        gr = torch.empty((B, h, w), dtype=torch.float32, device=dev)
        gh = torch.zeros(2 + self.params.levels, dtype=torch.float64, device=dev)
        arr = (PairGrad * B)()
        for b in range(B):
            arr[b] = PairGrad(gd[b].data_ptr(), gv[b].data_ptr() if gv is not None else None,
                              gl[b].data_ptr(), gr[b].data_ptr())
        st = lib().bdis_backward_batch(self._h, B, arr, gh.data_ptr(), _stream_ptr(stream))
        if st:
            raise self._err(st)
        return gl, gr, gh

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


def _set_hyper(ctx, sigma_s, sigma_r, omega):
    p = ctx.params
    q = params(**{k: v for k, v in p.as_dict().items()})
    q.sigma_s = float(sigma_s)
    q.sigma_r = float(sigma_r)
    lw = list(q.level_weight)
    for n, v in enumerate(omega):
        lw[n] = float(v)
    q.level_weight = (ctypes.c_float * 8)(*lw)
    ctx.set_params(q)


def _autograd_function():
    import torch

    class BDISFunction(torch.autograd.Function):
        """Disparity (and variance) of float stereo pairs on the GPU with a hand-written
        backward: gradients with respect to both images and the hyperparameters
        sigma_s, sigma_r (alpha_r in the dynamic mode) and the level weights omega."""

        @staticmethod
        def forward(fctx, left, right, sigma_s, sigma_r, omega, bctx):
            _set_hyper(bctx, sigma_s.item(), sigma_r.item(), omega.detach().cpu().tolist())
            out = bctx.compute_f32(left.detach().contiguous(), right.detach().contiguous())
            fctx.bctx = bctx
            fctx.generation = bctx.f32_generation
            fctx.shapes = (left.shape, omega.shape, sigma_s.dtype, omega.dtype, sigma_s.device, sigma_r.device,
                           omega.device)
            var = out["var"] if out["var"] is not None else torch.zeros_like(out["disp"])
            fctx.has_var = out["var"] is not None
            return out["disp"], var

        @staticmethod
        def backward(fctx, g_disp, g_var):
            import torch
            if fctx.bctx.f32_generation != fctx.generation:
                # the library keeps the saved state of its latest float call only
                raise RuntimeError("BDIS backward: the context has run another forward since this node's; "
                                   "use one context per pending node (or call backward before the next forward)")
            g_disp = torch.nan_to_num(g_disp) if g_disp is not None else None
            g_var = torch.nan_to_num(g_var) if (g_var is not None and fctx.has_var) else None
            if g_disp is None:
                g_disp = torch.zeros(fctx.shapes[0], dtype=torch.float32, device=g_var.device)
            gl, gr, gh = fctx.bctx.backward(g_disp, g_var)
            shape, oshape, sdt, odt, sdev, rdev, odev = fctx.shapes
            L = oshape[0]
            return (gl.reshape(shape), gr.reshape(shape), gh[0].to(device=sdev, dtype=sdt),
                    gh[1].to(device=rdev, dtype=sdt), gh[2:2 + L].to(device=odev, dtype=odt), None)

    return BDISFunction


_BDISFunction = None


def bdis_function():
    """The torch.autograd.Function of the differentiable path (created on first use)."""
    global _BDISFunction
    if _BDISFunction is None:
        _BDISFunction = _autograd_function()
    return _BDISFunction
