"""The allocation-free entry point (bdis_compute_static) against bdis_compute.

Both run the same kernels; the static one keeps its workspace and job table in
a static device array shared by every call on the device, so two calls in a
row (the second smaller) must each give what a context gives on the same pair,
with nothing left over from the earlier call.  Also checked: the pass runs
against the oracle's tolerance, device memory does not change across calls, and
a pair too large for the array is refused with a clear message.
"""
import numpy as np
import pytest

from _common import DISP_TOL, PASS_FRAC, parity, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2205_03133_amd import bdis
    bdis.lib()
    return bdis


def _same(a, b):
    """Bitwise equal float maps (NaN where the other is NaN)."""
    a, b = np.asarray(a), np.asarray(b)
    na, nb = np.isnan(a), np.isnan(b)
    return bool(np.array_equal(na, nb) and np.array_equal(a[~na], b[~nb]))


def _context_result(B, p, left, right):
    import torch
    h, w = left.shape
    with B.Context(p, w, h) as ctx:
        out = ctx.compute(left, right)
        torch.cuda.synchronize()
        return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def test_static_entry_matches_compute_on_two_calls(B):
    import torch
    from paper_2205_03133_amd.synth import make_pair, method_params
    cases = [("640x480 (5 levels, P8 S3 K16, variance)", 2), ("320x240 (3 levels, P8 S4 K8)", 1)]
    data = []
    for name, cfg in cases:
        left, right, _, _ = make_pair(cfg, 0)
        p = B.params(**method_params(cfg))
        data.append((name, p, to_gpu(left), to_gpu(right)))
    expected = [_context_result(B, p, l, r) for _, p, l, r in data]
    # outputs allocated up front, so the device memory reading below sees only the library
    outs = []
    for _, p, l, r in data:
        h, w = l.shape
        o = dict(disp=torch.empty((h, w), dtype=torch.float32, device=l.device),
                 conf=torch.empty((h, w), dtype=torch.float32, device=l.device))
        if p.variance:
            o["var"] = torch.empty((h, w), dtype=torch.float32, device=l.device)
        outs.append(o)
    # a first call on the small pair places the library's device code (and the
    # array) on the device; then the large pair and the small one again
    _, p1, l1, r1 = data[1]
    print("[gpu] bdis_compute_static warm-up on the small pair", flush=True)
    B.compute_static(p1, l1, r1)
    torch.cuda.synchronize()
    free_before = torch.cuda.mem_get_info()[0]
    for (name, p, l, r), o, exp in zip(data, outs, expected):
        print(f"[gpu] bdis_compute_static {name}", flush=True)
        got = B.compute_static(p, l, r, out=o)
        torch.cuda.synchronize()
        for k in ("disp", "var", "conf"):
            if exp[k] is None:
                assert got[k] is None
                continue
            g = got[k].cpu().numpy()
            st = parity(g, exp[k], DISP_TOL)
            print(f"  {k}: frac={st['frac']:.6f} max={st['max_err']:.3g} mask_mismatch={st['mask_mismatch']}",
                  flush=True)
            assert st["frac"] >= PASS_FRAC
            assert _same(g, exp[k]), f"{name}: {k} differs from bdis_compute"
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free_before, "device memory changed across the calls"


def test_static_entry_refuses_what_does_not_fit(B):
    import torch
    p = B.params(levels=6, patch=8, stride=3, iters=16, variance=1)
    left = torch.zeros((2160, 3840), dtype=torch.uint8, device="cuda")
    with pytest.raises(B.BdisError) as e:
        B.compute_static(p, left, left.clone())
    assert e.value.code == B.E_CAPACITY
    assert "static scratch" in str(e.value)
    bad = B.params(levels=3, patch=8, stride=4, iters=8)
    small = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    with pytest.raises(B.BdisError) as e:
        B.compute_static(bad, small, small.clone())
    assert e.value.code == B.E_SIZE
