"""ctypes wrapper of the FP64 CPU oracle (``libbdis_ref.so``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg.  The product path never imports this
module, and this module imports nothing from the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbdis_ref.so")
SOURCES = [os.path.join(HERE, "bdis_ref.c")]

NWIN = 5
WHAT = dict(left=0, right=1, grad=2, uinit=3, pipar=4, u=5, ssd=6, rho=7, acc=8, post=9,
            pi=10, sigk2=11, hess=12, ubar=13, qmap=14, valid=15, odisp=16, ovar=17, oconf=18,
            fv=19, vbar=20, gy=21)
SCALAR = dict(sigma_r2=0, tau=1, nacc=2, gamma=3)
PER_PATCH = {"uinit", "pipar", "u", "ssd", "rho", "acc", "post", "pi", "sigk2", "hess", "fv"}


class RefParams(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32), ("finest_level", ctypes.c_int32), ("patch", ctypes.c_int32),
        ("stride", ctypes.c_int32), ("iters", ctypes.c_int32), ("sigma_r_dynamic", ctypes.c_int32),
        ("variance", ctypes.c_int32), ("float_pyramid", ctypes.c_int32),
        ("sigma_s", ctypes.c_double), ("sigma_r", ctypes.c_double), ("valid_ratio", ctypes.c_double),
        ("var_fail_sigma", ctypes.c_double), ("var_fit_thresh", ctypes.c_double),
        ("prob_thresh", ctypes.c_double), ("level_weight", ctypes.c_double * 8),
        ("fusion", ctypes.c_int32), ("propagate", ctypes.c_int32),
    ]


def default_params(**overrides):
    """The paper's parameter choices (Sec. IV-A) where it gives them."""
    p = dict(levels=5, finest_level=0, patch=8, stride=4, iters=12, sigma_r_dynamic=1,
             variance=0, float_pyramid=0, sigma_s=4.0, sigma_r=1.0, valid_ratio=0.75,
             var_fail_sigma=0.0, var_fit_thresh=0.1, prob_thresh=0.0,
             level_weight=[float(2 ** n) for n in range(8)], fusion=0, propagate=1)
    for k, v in overrides.items():
        if k not in p:
            raise KeyError(k)
        p[k] = v
    return p


def _to_struct(p):
    s = RefParams()
    for name, _ in RefParams._fields_:
        if name == "level_weight":
            lw = list(p["level_weight"]) + [0.0] * (8 - len(p["level_weight"]))
            s.level_weight = (ctypes.c_double * 8)(*lw[:8])
        else:
            setattr(s, name, p[name])
    return s


def build(force=False):
    """Compile the oracle with the system C compiler (plain C11, FP64, no FMA contraction)."""
    if not force and os.path.exists(LIB_PATH) and all(
            os.path.getmtime(LIB_PATH) >= os.path.getmtime(s) for s in SOURCES):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp] + SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.bdis_ref_compute_u8.argtypes = [ctypes.POINTER(RefParams), ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp,
                                          ctypes.POINTER(ctypes.c_void_p)]
        L.bdis_ref_compute_f64.argtypes = L.bdis_ref_compute_u8.argtypes
        L.bdis_ref_trace_dims.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 4
        L.bdis_ref_trace_get.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, dp, ctypes.c_long]
        L.bdis_ref_trace_get.restype = ctypes.c_long
        L.bdis_ref_trace_scalar.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.bdis_ref_trace_scalar.restype = ctypes.c_double
        L.bdis_ref_trace_free.argtypes = [ctypes.c_void_p]
        L.bdis_ref_trace_hash.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.bdis_ref_trace_hash.restype = ctypes.c_uint64
        L.bdis_ref_grid.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        L.bdis_ref_mask.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.bdis_ref_parent_init.argtypes = [dp, dp] + [ctypes.c_int] * 6 + [dp, dp]
        L.bdis_ref_depth.argtypes = [dp, dp, ctypes.c_long, ctypes.c_double, dp, dp]
        L.bdis_ref_flow.argtypes = [ctypes.POINTER(RefParams), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, dp, dp, ctypes.POINTER(ctypes.c_void_p)]
        L.bdis_ref_coverage.argtypes = [dp, dp, dp, ctypes.c_void_p, ctypes.c_long, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned status {code}")
        self.code = code


class Trace:
    """Per-level intermediates of one oracle run."""

    def __init__(self, handle, levels):
        self._h = handle
        self.levels = levels

    def __del__(self):
        if getattr(self, "_h", None):
            lib().bdis_ref_trace_free(self._h)
            self._h = None

    def dims(self, level):
        w, h, nx, ny = (ctypes.c_int() for _ in range(4))
        st = lib().bdis_ref_trace_dims(self._h, level, ctypes.byref(w), ctypes.byref(h),
                                       ctypes.byref(nx), ctypes.byref(ny))
        if st:
            raise OracleError(st)
        return w.value, h.value, nx.value, ny.value

    def get(self, level, what):
        w, h, nx, ny = self.dims(level)
        if what in PER_PATCH:
            shape = (ny, nx, NWIN) if what == "ssd" else (ny, nx)
        else:
            shape = (h, w)
        out = np.empty(shape, dtype=np.float64)
        n = lib().bdis_ref_trace_get(self._h, level, WHAT[what],
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size)
        if n < 0:
            raise OracleError(n)
        return out

    def scalar(self, level, what):
        return lib().bdis_ref_trace_scalar(self._h, level, SCALAR[what])

    def decision_hash(self):
        """Hashes of the discrete decisions of every level (tuple)."""
        return tuple(int(lib().bdis_ref_trace_hash(self._h, n)) for n in range(self.levels))


def compute(left, right, params, trace=False):
    """Run the oracle on one pair.  uint8 inputs take the integer path, float inputs the float path.

    Returns ``dict(disp, var, conf[, trace])`` with float64 ``H x W`` arrays.
    """
    left = np.ascontiguousarray(left)
    right = np.ascontiguousarray(right)
    if left.shape != right.shape or left.ndim != 2:
        raise ValueError("left/right must be equal 2-D arrays")
    h, w = left.shape
    s = _to_struct(params)
    disp = np.empty((h, w), np.float64)
    var = np.empty((h, w), np.float64)
    conf = np.empty((h, w), np.float64)
    handle = ctypes.c_void_p()
    dp = ctypes.POINTER(ctypes.c_double)
    if left.dtype == np.uint8:
        fn = lib().bdis_ref_compute_u8
        if right.dtype != np.uint8:
            raise ValueError("both images must be uint8")
    else:
        left = left.astype(np.float64)
        right = right.astype(np.float64)
        fn = lib().bdis_ref_compute_f64
    st = fn(ctypes.byref(s), left.ctypes.data, right.ctypes.data, w, h, w,
            disp.ctypes.data_as(dp), var.ctypes.data_as(dp), conf.ctypes.data_as(dp),
            ctypes.byref(handle) if trace else None)
    if st:
        raise OracleError(st)
    out = dict(disp=disp, var=var, conf=conf)
    if trace:
        out["trace"] = Trace(handle.value, params["levels"])
    return out


def mask(patch, sigma_s):
    out = np.empty((patch, patch), np.float64)
    st = lib().bdis_ref_mask(patch, sigma_s, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if st:
        raise OracleError(st)
    return out


def parent_init(ubar, qmap, w, h, patch, stride):
    """Start displacement and propagated probability of every patch of a w x h
    level from the parent level's fused maps (ny x nx arrays each)."""
    ubar = np.ascontiguousarray(ubar, dtype=np.float64)
    qmap = np.ascontiguousarray(qmap, dtype=np.float64)
    if ubar.shape != qmap.shape or ubar.ndim != 2:
        raise ValueError("parent maps must be equal 2-D arrays")
    ph, pw = ubar.shape
    ny, nx = len(grid(h, patch, stride)), len(grid(w, patch, stride))
    dp = ctypes.POINTER(ctypes.c_double)
    u0 = np.empty((ny, nx), np.float64)
    pi = np.empty((ny, nx), np.float64)
    st = lib().bdis_ref_parent_init(ubar.ctypes.data_as(dp), qmap.ctypes.data_as(dp), pw, ph, w, h, patch,
                                    stride, u0.ctypes.data_as(dp), pi.ctypes.data_as(dp))
    if st:
        raise OracleError(st)
    return u0, pi


def grid(n, patch, stride):
    """Patch-grid origins along an axis of length ``n``."""
    cnt = lib().bdis_ref_grid(n, patch, stride, None, 0)
    if cnt < 0:
        raise OracleError(cnt)
    out = (ctypes.c_int * cnt)()
    lib().bdis_ref_grid(n, patch, stride, out, cnt)
    return np.array(out[:], dtype=np.int64)


def depth(disp, var, fb):
    """Depth and depth variance from disparity and its variance (Eq. 14, 18)."""
    disp = np.ascontiguousarray(disp, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    out = np.empty_like(disp)
    ov = None
    vp = None
    if var is not None:
        var = np.ascontiguousarray(var, dtype=np.float64)
        ov = np.empty_like(disp)
        vp = var.ctypes.data_as(dp)
    st = lib().bdis_ref_depth(disp.ctypes.data_as(dp), vp, disp.size, fb, out.ctypes.data_as(dp),
                              ov.ctypes.data_as(dp) if ov is not None else None)
    if st:
        raise OracleError(st)
    return out, ov


def coverage(disp, var, ref, k=1.96, valid=None):
    """(covered, total): pixels with |d - ref| <= k sqrt(var) among the usable ones."""
    dp = ctypes.POINTER(ctypes.c_double)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (disp, var, ref)]
    vm = None if valid is None else np.ascontiguousarray(valid, dtype=np.uint8)
    c, t = ctypes.c_long(), ctypes.c_long()
    st = lib().bdis_ref_coverage(*(a.ctypes.data_as(dp) for a in arrs),
                                 vm.ctypes.data if vm is not None else None, arrs[0].size, k,
                                 ctypes.byref(c), ctypes.byref(t))
    if st:
        raise OracleError(st)
    return c.value, t.value


def flow(i0, i1, params, trace=False):
    """2-D dense inverse search between two uint8 frames: dict(u, v[, trace]), H x W float64."""
    i0 = np.ascontiguousarray(i0, dtype=np.uint8)
    i1 = np.ascontiguousarray(i1, dtype=np.uint8)
    if i0.shape != i1.shape or i0.ndim != 2:
        raise ValueError("frames must be equal 2-D arrays")
    h, w = i0.shape
    u = np.empty((h, w), np.float64)
    v = np.empty((h, w), np.float64)
    handle = ctypes.c_void_p()
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib().bdis_ref_flow(ctypes.byref(_to_struct(params)), i0.ctypes.data, i1.ctypes.data, w, h, w,
                             u.ctypes.data_as(dp), v.ctypes.data_as(dp), ctypes.byref(handle) if trace else None)
    if st:
        raise OracleError(st)
    out = dict(u=u, v=v)
    if trace:
        out["trace"] = Trace(handle.value, params["levels"])
    return out

