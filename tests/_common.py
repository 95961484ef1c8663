"""Helpers shared by the GPU tests: device transfer and parity statistics."""
import numpy as np

DISP_TOL = 1e-3        # px, on >= 99.9% of pixels
VAR_RTOL = 1e-3        # relative
PASS_FRAC = 0.999
# Variance: relative 1e-3 on >= 99.9% of pixels overall (the disparity bar),
# and also away from patches whose accept / fit decision differs, where a
# rounding-level change of the level-wide tau can flip a threshold decision of
# Eq. 17 (fit residual <= 0.1, kappa > 0).
VAR_FLOOR = PASS_FRAC
MAX_FLIP_FRAC = 5e-4   # patches whose accept / fit decision differs
# Patches whose search differs and is shown ill-conditioned (chaotic in exact
# arithmetic): a near-textureless patch takes huge steps, so a rounding-level
# change of its start (the parent map's summation order, or the level scalars
# once an acceptance differs above) moves its result by pixels.
MAX_ILL_FRAC = 2e-3


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def parity(gpu, ref, tol, rel=False):
    """Fraction of pixels where GPU and oracle agree (mask disagreements count as misses).

    Returns dict(frac, max_err, p999, mask_mismatch, n).
    """
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    gv, rv = np.isfinite(gpu), np.isfinite(ref)
    both = gv & rv
    err = np.abs(gpu - ref)
    lim = tol * np.maximum(np.abs(ref), 1e-30) if rel else np.full(ref.shape, tol)
    ok = (both & (err <= lim)) | (~gv & ~rv)
    e = err[both] / (np.maximum(np.abs(ref[both]), 1e-30) if rel else 1.0)
    return dict(frac=float(ok.mean()), max_err=float(e.max()) if e.size else 0.0,
                p999=float(np.quantile(e, 0.999)) if e.size else 0.0,
                mask_mismatch=int((gv != rv).sum()), n=int(ok.size))


def oracle_params(oracle, bp):
    """Oracle parameters equal to the library's (float32 values widened exactly)."""
    d = bp.as_dict()
    return oracle.default_params(
        levels=d["levels"], finest_level=d["finest_level"], patch=d["patch"], stride=d["stride"],
        iters=d["iters"], sigma_r_dynamic=d["sigma_r_dynamic"], variance=d["variance"],
        float_pyramid=d["float_pyramid"], sigma_s=float(d["sigma_s"]), sigma_r=float(d["sigma_r"]),
        valid_ratio=float(d["valid_ratio"]), var_fail_sigma=float(d["var_fail_sigma"]),
        var_fit_thresh=float(d["var_fit_thresh"]), prob_thresh=float(d["prob_thresh"]),
        level_weight=[float(x) for x in d["level_weight"]], fusion=d["fusion"], propagate=d["propagate"])


def footprint(mask_patches, w, h, P, S):
    """Pixels covered by the flagged patches of a level (grid origins min(i*S, n-P))."""
    ny, nx = mask_patches.shape
    ox = np.minimum(np.arange(nx) * S, w - P)
    oy = np.minimum(np.arange(ny) * S, h - P)
    out = np.zeros((h, w), bool)
    for j, i in np.argwhere(mask_patches):
        out[oy[j]:oy[j] + P, ox[i]:ox[i] + P] = True
    return out


def variance_parity(gpu_var, ref_var, g_acc, g_sig, r_acc, r_sig, P, S, f=0, level_wh=None, exclude=None):
    """Variance agreement overall and away from patches whose decisions differ.

    A decision differs when acceptance differs, or when exactly one side
    failed the variance fit (sigma_k^2 == P^2 with the default failure sigma).
    With a finest level f > 0 the patches live on the level-f grid (size
    level_wh); their footprint grows by the one level-f pixel that bilinear
    upsampling reaches and is mapped to full resolution.  `exclude` adds
    pixels to leave out (the footprint of searches that differ).
    """
    h, w = ref_var.shape
    fail_g = g_acc & np.isclose(g_sig, P * P, rtol=0, atol=0)
    fail_r = r_acc & np.isclose(r_sig, P * P, rtol=0, atol=0)
    flip = (g_acc != r_acc) | (fail_g != fail_r)
    st = parity(gpu_var, ref_var, VAR_RTOL, rel=True)
    if f == 0:
        fp = footprint(flip, w, h, P, S)
    else:
        from scipy import ndimage
        lw, lh = level_wh
        fp = ndimage.binary_dilation(footprint(flip, lw, lh, P, S), np.ones((3, 3), bool))
        fp = np.kron(fp, np.ones((2 ** f, 2 ** f), bool))[:h, :w]
    if exclude is not None:
        fp = fp | exclude
    st_away = parity(np.where(fp, 0.0, gpu_var), np.where(fp, 0.0, ref_var), VAR_RTOL, rel=True)
    # pixels excluded above are counted as agreeing; report the fraction over the rest
    n_rest = int((~fp).sum())
    frac_rest = 1.0 - (1.0 - st_away["frac"]) * st_away["n"] / max(n_rest, 1)
    return dict(overall=st, away_frac=frac_rest, flip_patches=int(flip.sum()),
                flip_frac=float(flip.mean()))


def exact_lk(left, right, ox, oy, P, K, u0):
    """The patch search of Eq. 1 in exact rational arithmetic, from start u0.

    Written from the definition, independently of both implementations:
    J = Sobel-x / 8 of the integer left level image (reflect-101 borders) minus
    its patch mean, H = sum J^2, K updates u <- u - sum J (I_w(u) - T) / H with
    the linear warp I_w (indices clamped to the row) while H >= 1e-3, then the
    search-threshold reset (|u - u0| > P: back to u0).  Returns a Fraction.
    The trajectory of a patch with a small Hessian can be chaotic: a change of
    its start or of one rounding then moves the result by whole pixels, and no
    FP64 evaluation order determines it to 1e-3 px.
    """
    from fractions import Fraction
    import math
    L = np.asarray(left, np.int64)
    R = np.asarray(right, np.int64)
    h, w = L.shape

    def refl(x, n):
        x = -x if x < 0 else x
        return 2 * (n - 1) - x if x >= n else x

    G = [[0] * P for _ in range(P)]
    for a in range(P):
        y = oy + a
        ym, yp = refl(y - 1, h), refl(y + 1, h)
        for c in range(P):
            x = ox + c
            xm, xp = refl(x - 1, w), refl(x + 1, w)
            G[a][c] = int((L[ym, xp] - L[ym, xm]) + 2 * (L[y, xp] - L[y, xm]) + (L[yp, xp] - L[yp, xm]))
    gbar = Fraction(sum(map(sum, G)), 8 * P * P)
    J = [[Fraction(G[a][c], 8) - gbar for c in range(P)] for a in range(P)]
    H = sum(j * j for row in J for j in row)
    u0 = Fraction(float(u0))
    u = u0
    if H >= Fraction(1, 1000):
        rows = [[int(v) for v in R[oy + a]] for a in range(P)]
        T = [[int(L[oy + a, ox + c]) for c in range(P)] for a in range(P)]
        for _ in range(K):
            m = math.floor(u)
            f = u - m
            b = Fraction(0)
            for a in range(P):
                ra = rows[a]
                for c in range(P):
                    i0 = min(max(ox + c + m, 0), w - 1)
                    i1 = min(max(ox + c + m + 1, 0), w - 1)
                    b += J[a][c] * ((1 - f) * ra[i0] + f * ra[i1] - T[a][c])
            u = u - b / H
    return u0 if abs(u - u0) > P else u


def _up2(mask, w, h):
    """A level mask on the next finer level's grid (w x h), dilated by one pixel."""
    from scipy import ndimage
    up = np.kron(mask, np.ones((2, 2), bool))[:h, :w]
    if up.shape != (h, w):
        up = np.pad(up, ((0, h - up.shape[0]), (0, w - up.shape[1])), mode="edge")
    return ndimage.binary_dilation(up, np.ones((3, 3), bool))


def divergence_analysis(ctx, tr, p, max_exact=40):
    """Every patch whose search differs between the GPU and the oracle
    (acceptance differs or |u_gpu - u_oracle| > DISP_TOL) must be explained:

    * inherited: its pixels meet the footprint, scaled down one level and
      dilated, of the disagreements at the parent level (which reach it through
      the bilinear start and the parent-filled holes);
    * a window tie: the displacements agree but the acceptance differs at the
      margin that their difference allows (the centre SSD within 1e-9 relative,
      plus the window slope times that difference, of a neighbour's), or the
      in-bounds ratio sits at the threshold;
    * ill-conditioned, shown by exact rational trajectories independently of
      the GPU's result: from the oracle's start the exact result differs from
      the oracle's FP64 result by more than DISP_TOL / 2, or the two sides'
      starts (which differ by the rounding of the parent level's fused map, or
      by the level scalars once an acceptance differs above) or the oracle's
      start moved by 1e-9 px lead to exact results further apart than that.

    The ill-conditioned class is checked exactly on an evenly spaced sample of
    at most `max_exact` patches per level, every one of which must pass.
    Returns (per-level counts, the level-f footprint of all disagreements,
    per-level class counts); raises AssertionError for an unexplained patch.
    """
    P, S, K = p.patch, p.stride, p.iters
    f = p.finest_level
    fp_parent = None  # affected pixels of the parent level's map, on the parent grid
    counts, how = {}, {}
    for n in range(p.levels - 1, f - 1, -1):
        lw, lh, nx, ny = tr.dims(n)
        ag, ar = ctx.debug(n, "acc") > 0, tr.get(n, "acc") > 0
        ug, ur = ctx.debug(n, "u"), tr.get(n, "u")
        div = (ag != ar) | (np.abs(ug - ur) > DISP_TOL)
        counts[n] = int(div.sum())
        inherited_px = _up2(fp_parent, lw, lh) if fp_parent is not None else np.zeros((lh, lw), bool)
        ox = np.minimum(np.arange(nx) * S, lw - P)
        oy = np.minimum(np.arange(ny) * S, lh - P)
        h = dict(inherited=0, window_tie=0, searched=0, checked_exactly=0)
        uig, uir = ctx.debug(n, "uinit"), tr.get(n, "uinit")
        left, right = tr.get(n, "left"), tr.get(n, "right")
        ssd, rho = tr.get(n, "ssd"), tr.get(n, "rho")
        cand = []
        for j, i in np.argwhere(div):
            if inherited_px[oy[j]:oy[j] + P, ox[i]:ox[i] + P].any():
                h["inherited"] += 1
                continue
            if abs(ug[j, i] - ur[j, i]) <= DISP_TOL:
                s0 = ssd[j, i, 2]
                margin = min(abs(ssd[j, i, d] - s0) for d in (0, 1, 3, 4))
                # SSD moves by at most about its window slope times the displacement difference
                slope = max(abs(ssd[j, i, d] - s0) for d in (1, 3)) / 0.5
                bound = 1e-9 * max(abs(s0), 1.0) + 4.0 * slope * abs(ug[j, i] - ur[j, i])
                assert margin <= bound or abs(rho[j, i] - p.valid_ratio) < 1e-12, \
                    f"level {n} patch ({j}, {i}): acceptance differs at margin {margin:.3g} (SSD0 {s0:.6g})"
                h["window_tie"] += 1
                continue
            cand.append((int(j), int(i)))
        h["searched"] = len(cand)
        pick = cand if len(cand) <= max_exact else [cand[k] for k in np.linspace(0, len(cand) - 1, max_exact).astype(int)]
        for j, i in pick:
            def ex(u0):
                return exact_lk(left, right, int(ox[i]), int(oy[j]), P, K, u0)
            er = ex(uir[j, i])
            eg = er if uig[j, i] == uir[j, i] else ex(uig[j, i])
            # the oracle's own FP64 error and the sensitivity of the exact map to its start
            spread = max(abs(float(er) - ur[j, i]), abs(float(er - eg)),
                         abs(float(ex(uir[j, i] + 1e-9) - er)), abs(float(ex(uir[j, i] - 1e-9) - er)))
            assert spread > DISP_TOL / 2, (
                f"level {n} patch ({j}, {i}): GPU u {ug[j, i]!r}, oracle u {ur[j, i]!r}, exact from the oracle's "
                f"start {float(er)!r}, from the GPU's {float(eg)!r}: a well-conditioned patch that disagrees")
            h["checked_exactly"] += 1
        how[n] = h
        fp = footprint(div, lw, lh, P, S)
        fp_parent = fp | inherited_px
    return counts, fp_parent, how
