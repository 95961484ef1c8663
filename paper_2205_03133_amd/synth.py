"""Seeded synthetic rectified stereo pairs with ground-truth disparity.

The paper measures on surgical datasets (a Unity3D colon, Hamlyn, SCARED,
SERV-CT; Sec. IV-A) that are not available here.  This module stands in for
them: it produces pairs with the same image shapes and with the nuisances the
paper names (textureless tissue, dark illumination, non-Lambertian highlights;
Sec. I and Sec. III-B), plus a known disparity field so that accuracy can be
measured.

This module holds input generation only (texture synthesis, warping, noise).
It contains none of the stereo method's arithmetic and is shared, read-only,
by the oracle tests, the GPU parity tests and the benchmark.

Recipe (all draws from ``numpy.random.default_rng(SeedSequence([2205, 3133,
cfg, pair]))``):

* texture: white N(0,1) noise on a canvas ``H x (W + dmax + 8)``, filtered in
  the Fourier domain by ``1/max(|k|, 1/256)`` (1/f spectrum), standardised to
  mean 128 / std 40 and clipped to [0, 255];
* textureless regions: a very-low-frequency noise field thresholded at the
  quantile giving the target area; inside, the canvas is replaced by its
  Gaussian blur (sigma 16 px);
* the disparity field ``d_R`` lives on the right grid; the right image is the
  backward linear warp ``R(x', y) = gain * canvas(x' + d_R(x', y), y)`` and
  the left image is ``canvas[:, :W]``, so left pixel ``x`` matches right
  pixel ``x - d``;
* ground truth on the left grid solves ``d_L(x) = d_R(x - d_L(x))`` by 30
  fixed-point steps; a pixel is valid when the iteration converged to 1e-6,
  and ``x - d_L`` lies inside the right image;
* illumination gain, specular blobs (added after warping at positions that
  differ by U(-8, 8) px between the views, saturated at 255), Gaussian noise,
  round-half-even and clip to uint8.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import ndimage

__all__ = ["Workload", "WORKLOADS", "make_pair", "method_params", "c3_sizes", "c3_levels"]


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape and nuisance recipe of one synthetic workload."""

    name: str
    width: int
    height: int
    field: str               # "bumps" (smooth Gaussian bumps) or "planes" (piecewise-smooth)
    dmax: float              # largest disparity in px
    textureless: float       # fraction of the area made textureless
    specular: bool
    gain_lo: float           # right-view gain range
    gain_hi: float
    dark_lo: float           # illumination gain range applied to both views
    dark_hi: float
    noise: float             # Gaussian noise sigma (intensity units)
    noise_left: bool         # noise on the left view as well as the right
    quantize: bool = True


WORKLOADS = {
    # one 320x240 pair: 1/f texture, bumps 0-32 px, N(0,1) noise on the right view
    1: Workload("c1", 320, 240, "bumps", 32.0, 0.0, False, 1.0, 1.0, 1.0, 1.0, 1.0, False),
    # one 640x480 pair: planes + bumps 0-64 px, 20% textureless, highlights,
    # right gain U(0.8, 1.2), noise sigma 2 on both views
    2: Workload("c2", 640, 480, "planes", 64.0, 0.20, True, 0.8, 1.2, 1.0, 1.0, 2.0, True),
    # 640x480 pairs with the config-1 field, used by the differentiable form
    4: Workload("c4", 640, 480, "bumps", 32.0, 0.0, False, 1.0, 1.0, 1.0, 1.0, 1.0, False),
    # 1920x1080 pairs: planes + bumps 0-192 px, 30% textureless, dark gain U(0.2, 0.5), noise 3
    5: Workload("c5", 1920, 1080, "planes", 192.0, 0.30, False, 1.0, 1.0, 0.2, 0.5, 3.0, True),
}

# The mixed-resolution batch: 8 pairs at each of these sizes, generated with the
# config-2 recipe and disparity up to 10% of the width.
_C3_SIZES = [(320, 240), (360, 288), (640, 480), (720, 576),
             (1024, 768), (1280, 720), (1600, 900), (1920, 1080)]


def c3_sizes():
    """Sizes (w, h) of the 64 pairs of the mixed-resolution batch, in order."""
    return [s for s in _C3_SIZES for _ in range(8)]


def c3_levels(w, h):
    """Pyramid depth for a pair of the mixed batch: clamp(floor(log2(min/30)) + 1, 4, 6)."""
    return int(min(6, max(4, math.floor(math.log2(min(w, h) / 30.0)) + 1)))


def _workload(cfg, pair_idx):
    if cfg == 3:
        w, h = c3_sizes()[pair_idx % 64]
        base = WORKLOADS[2]
        return dataclasses.replace(base, name="c3", width=w, height=h, dmax=0.1 * w)
    return WORKLOADS[cfg]


def method_params(cfg, pair_idx=0):
    """Method parameters of each workload (pyramid depth, patch, stride, iterations, variance)."""
    if cfg == 1:
        return dict(levels=3, patch=8, stride=4, iters=8, variance=0)
    if cfg == 2:
        return dict(levels=5, patch=8, stride=3, iters=16, variance=1)
    if cfg == 3:
        w, h = c3_sizes()[pair_idx % 64]
        return dict(levels=c3_levels(w, h), patch=8, stride=3, iters=16, variance=1)
    if cfg == 4:
        return dict(levels=4, patch=8, stride=4, iters=8, variance=0, float_pyramid=1)
    if cfg == 5:
        return dict(levels=6, patch=12, stride=4, iters=16, variance=1)
    raise ValueError(f"unknown workload {cfg}")


def _rng(cfg, pair_idx):
    return np.random.default_rng(np.random.SeedSequence([2205, 3133, int(cfg), int(pair_idx)]))


def _texture(rng, h, w):
    """1/f noise texture, mean 128, std 40, clipped to [0, 255]."""
    white = rng.standard_normal((h, w))
    ky = np.fft.fftfreq(h)[:, None]
    kx = np.fft.rfftfreq(w)[None, :]
    k = np.sqrt(kx * kx + ky * ky)
    spec = np.fft.rfft2(white) / np.maximum(k, 1.0 / 256.0)
    tex = np.fft.irfft2(spec, s=(h, w))
    tex = (tex - tex.mean()) / tex.std() * 40.0 + 128.0
    return np.clip(tex, 0.0, 255.0)


def _textureless(rng, canvas, area):
    if area <= 0:
        return canvas
    h, w = canvas.shape
    # white noise low-passed by a periodic Gaussian of sigma max(h, w)/12 px (in the Fourier domain)
    sig = max(h, w) / 12.0
    ky = np.fft.fftfreq(h)[:, None]
    kx = np.fft.rfftfreq(w)[None, :]
    lp = np.exp(-2.0 * (np.pi * sig) ** 2 * (kx * kx + ky * ky))
    field = np.fft.irfft2(np.fft.rfft2(rng.standard_normal((h, w))) * lp, s=(h, w))
    mask = field > np.quantile(field, 1.0 - area)
    blurred = ndimage.gaussian_filter(canvas, sigma=16.0, mode="reflect")
    return np.where(mask, blurred, canvas)


def _bumps(rng, h, w, count, amp_lo, amp_hi):
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    out = np.zeros((h, w))
    for _ in range(count):
        cx, cy = rng.uniform(0, w), rng.uniform(0, h)
        sb = rng.uniform(w / 12.0, w / 4.0)
        a = rng.uniform(amp_lo, amp_hi)
        out += a * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2.0 * sb * sb))
    return out


def _field(rng, wl):
    h, w = wl.height, wl.width
    if wl.field == "bumps":
        f = _bumps(rng, h, w, 6, 0.3, 1.0)
        lo, hi = f.min(), f.max()
        return (f - lo) / max(hi - lo, 1e-12) * wl.dmax
    # piecewise-smooth: eight Voronoi cells, each a slanted plane, plus four bumps of <= 8 px
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    seeds = np.stack([rng.uniform(0, w, 8), rng.uniform(0, h, 8)], axis=1)
    d2 = (xx[None] - seeds[:, 0, None, None]) ** 2 + (yy[None] - seeds[:, 1, None, None]) ** 2
    cell = np.argmin(d2, axis=0)
    base = rng.uniform(0.15 * wl.dmax, 0.85 * wl.dmax, 8)
    sx = rng.uniform(-0.05, 0.05, 8)
    sy = rng.uniform(-0.05, 0.05, 8)
    d = base[cell] + sx[cell] * (xx - seeds[cell, 0]) + sy[cell] * (yy - seeds[cell, 1])
    bumps = _bumps(rng, h, w, 4, 0.0, 1.0)
    d = d + bumps / max(bumps.max(), 1e-12) * min(8.0, 0.25 * wl.dmax)
    return np.clip(d, 0.0, wl.dmax)


def _warp_rows(src, pos):
    """Linear interpolation of each row of ``src`` at fractional columns ``pos``
    (positions outside the row take the end values)."""
    h, wc = src.shape
    p = np.clip(pos, 0.0, wc - 1.0)
    i0 = np.minimum(np.floor(p).astype(np.int64), wc - 2)
    f = p - i0
    rows = np.arange(h)[:, None]
    return src[rows, i0] * (1.0 - f) + src[rows, i0 + 1] * f


def _ground_truth(d_right):
    """Disparity on the left grid: d_L(x) = d_R(x - d_L(x)), 30 fixed-point steps."""
    h, w = d_right.shape
    xs = np.arange(w, dtype=np.float64)
    d = d_right.copy()
    prev = d
    for _ in range(30):
        prev = d
        d = _warp_rows(d_right, np.clip(xs[None, :] - d, 0.0, w - 1.0))
    xr = xs[None, :] - d
    valid = (np.abs(d - prev) <= 1e-6) & (xr >= 0.0) & (xr <= w - 1.0)
    return d, valid


def _speculars(rng, h, w):
    n = rng.poisson(6.0 * (w * h) / 0.3e6)
    blobs = []
    for _ in range(n):
        blobs.append((rng.uniform(0, w), rng.uniform(0, h), rng.uniform(4, 16),
                      rng.uniform(60, 160), rng.uniform(-8, 8)))
    return blobs


def _add_blobs(img, blobs, shift):
    h, w = img.shape
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    out = img.copy()
    for cx, cy, r, a, off in blobs:
        cxx = cx + (off if shift else 0.0)
        out += a * np.exp(-((xx - cxx) ** 2 + (yy - cy) ** 2) / (2.0 * r * r))
    return np.minimum(out, 255.0)


def make_pair(cfg, pair_idx=0, *, quantize=True):
    """Return ``(left, right, gt_disp, gt_valid)`` for workload ``cfg``.

    ``left``/``right`` are uint8 ``H x W`` arrays (float64 when ``quantize`` is
    False: the same values before rounding).  ``gt_disp`` is float32 on the
    left grid with ``d = x_left - x_right`` and ``gt_valid`` is boolean.
    """
    wl = _workload(cfg, pair_idx)
    rng = _rng(cfg, pair_idx)
    h, w = wl.height, wl.width
    wc = w + int(math.ceil(wl.dmax)) + 8
    canvas = _texture(rng, h, wc)
    canvas = _textureless(rng, canvas, wl.textureless)
    d_r = _field(rng, wl)
    gain = rng.uniform(wl.gain_lo, wl.gain_hi)
    dark = rng.uniform(wl.dark_lo, wl.dark_hi)
    xs = np.arange(w, dtype=np.float64)
    right = gain * _warp_rows(canvas, xs[None, :] + d_r)
    left = canvas[:, :w].copy()
    left *= dark
    right *= dark
    if wl.specular:
        blobs = _speculars(rng, h, w)
        left = _add_blobs(left, blobs, False)
        right = _add_blobs(right, blobs, True)
    right = right + rng.standard_normal((h, w)) * wl.noise
    if wl.noise_left:
        left = left + rng.standard_normal((h, w)) * wl.noise
    gt, valid = _ground_truth(d_r)
    if quantize:
        left = np.clip(np.rint(left), 0, 255).astype(np.uint8)
        right = np.clip(np.rint(right), 0, 255).astype(np.uint8)
    else:
        left = np.clip(left, 0.0, 255.0)
        right = np.clip(right, 0.0, 255.0)
    return left, right, gt.astype(np.float32), valid


def make_flow_pair(idx=0, w=640, h=480, max_flow=12.0, noise=2.0):
    """Two frames with a known smooth 2-D flow (optical-flow form of the search).

    Recipe (draws from ``SeedSequence([2205, 3133, 99, idx])``): a 1/f texture
    ``I1`` on an ``H x W`` canvas; a flow field ``(u, v)`` on the first frame's
    grid made of six Gaussian bumps per component scaled to ``[-max_flow,
    max_flow]``; ``I0(x, y) = I1(x + u, y + v)`` by bilinear interpolation with
    edge clamping (so ``I1(x + u) = I0(x)`` holds exactly before noise);
    Gaussian noise ``noise`` on both frames, round-half-even, clip to uint8.
    Returns ``(I0, I1, u, v, valid)`` with ``valid`` where ``x + u`` stays in
    the frame.
    """
    rng = np.random.default_rng(np.random.SeedSequence([2205, 3133, 99, int(idx)]))
    i1 = _texture(rng, h, w)

    def comp():
        f = _bumps(rng, h, w, 6, -1.0, 1.0)
        return f / max(np.abs(f).max(), 1e-12) * max_flow

    u, v = comp(), comp()
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    i0 = ndimage.map_coordinates(i1, [yy + v, xx + u], order=1, mode="nearest")
    i0 = i0 + rng.standard_normal((h, w)) * noise
    i1 = i1 + rng.standard_normal((h, w)) * noise
    q = lambda a: np.clip(np.rint(a), 0, 255).astype(np.uint8)
    valid = (xx + u >= 0) & (xx + u <= w - 1) & (yy + v >= 0) & (yy + v <= h - 1)
    return q(i0), q(i1), u.astype(np.float32), v.astype(np.float32), valid
