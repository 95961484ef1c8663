"""Helpers shared by the GPU tests: device transfer and parity statistics."""
import numpy as np

DISP_TOL = 1e-3        # px, on >= 99.9% of pixels
VAR_RTOL = 1e-3        # relative, on >= 99.9% of pixels
PASS_FRAC = 0.999


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
        level_weight=[float(x) for x in d["level_weight"]])
