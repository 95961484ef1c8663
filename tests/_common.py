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


def variance_parity(gpu_var, ref_var, g_acc, g_sig, r_acc, r_sig, P, S, f=0, level_wh=None):
    """Variance agreement overall and away from patches whose decisions differ.

    A decision differs when acceptance differs, or when exactly one side
    failed the variance fit (sigma_k^2 == P^2 with the default failure sigma).
    With a finest level f > 0 the patches live on the level-f grid (size
    level_wh); their footprint grows by the one level-f pixel that bilinear
    upsampling reaches and is mapped to full resolution.
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
    st_away = parity(np.where(fp, 0.0, gpu_var), np.where(fp, 0.0, ref_var), VAR_RTOL, rel=True)
    # pixels excluded above are counted as agreeing; report the fraction over the rest
    n_rest = int((~fp).sum())
    frac_rest = 1.0 - (1.0 - st_away["frac"]) * st_away["n"] / max(n_rest, 1)
    return dict(overall=st, away_frac=frac_rest, flip_patches=int(flip.sum()),
                flip_frac=float(flip.mean()))
