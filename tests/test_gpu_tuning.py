"""The launch-shape tuner and its cache file: the choices persist across
contexts, a context that finds its shapes in the file does not tune, and every
choice the file can force (fusion tile height, pyramid form, search
configuration, the coarsest level in one workgroup or in per-phase launches,
one launch for the chained small pyramid levels or one each) gives the same
bits."""
import json
import os

import pytest

from _common import to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2205_03133_amd import bdis
    bdis.lib()
    return bdis


def _run(B, p, l, r):
    import torch
    h, w = l.shape
    with B.Context(p, w, h) as ctx:
        out = ctx.compute(l, r)
        torch.cuda.synchronize()
        tune_ms, cap_ms = ctx.setup_time()
        res = {k: v.clone() for k, v in out.items() if v is not None}
    return res, tune_ms, cap_ms


def _equal(a, b):
    import torch
    return all(torch.equal(torch.nan_to_num(a[k], nan=-7.0), torch.nan_to_num(b[k], nan=-7.0)) for k in a)


@pytest.mark.parametrize("cfg", [2, 5], ids=["640x480", "1080p"])
def test_tune_cache_and_forced_choices(B, tmp_path, monkeypatch, cfg):
    from paper_2205_03133_amd.synth import make_pair, method_params
    path = str(tmp_path / "tune.json")
    monkeypatch.setenv("BDIS_TUNE_CACHE", path)
    left, right, _, _ = make_pair(cfg, 0)
    l, r = to_gpu(left), to_gpu(right)
    p = B.params(**method_params(cfg))
    print(f"[gpu] tuning cache, workload {cfg}: first context", flush=True)
    ref, tune_ms, cap_ms = _run(B, p, l, r)
    assert tune_ms > 0.0 and cap_ms > 0.0
    text = open(path).read()
    doc = json.loads(text)
    entries = doc["entries"]
    assert len(entries) == p.levels
    for key, v in entries.items():
        assert key.startswith("gfx950") and set(v) == {"search", "fuse_ty", "pyr_tall", "top", "chain"}
    top_entries = [v for v in entries.values() if v["top"] >= 0]
    assert len(top_entries) == 1  # the coarsest level, timed both ways
    print(f"  tuned in {tune_ms:.1f} ms, captured in {cap_ms:.1f} ms", flush=True)
    out, tune2, cap2 = _run(B, p, l, r)
    assert tune2 == 0.0 and cap2 > 0.0  # the file's choices: no tuning
    assert _equal(out, ref)
    # every choice forced through the file gives the same bits
    variants = [("fuse_ty", 4), ("fuse_ty", 16), ("fuse_ty", 32), ("pyr_tall", 0), ("pyr_tall", 1),
                ("search", 0), ("search", 5), ("search", 10), ("top", 0), ("top", 1), ("chain", 0), ("chain", 1)]
    for field, val in variants:
        forced = {k: dict(v) for k, v in entries.items()}
        for k, v in forced.items():
            if field == "pyr_tall" and v["pyr_tall"] < 0:
                continue  # level 0 has no pyramid step
            if field in ("top", "chain") and v[field] < 0:
                continue  # only the coarsest level / the chain's top level has the choice
            v[field] = val
        # one entry per line, as the library writes it
        with open(path, "w") as f:
            f.write('{\n"bdis_tune_cache": 1,\n"entries": {\n')
            f.write(",\n".join(f'"{k}": {{"search": {v["search"]}, "fuse_ty": {v["fuse_ty"]}, '
                               f'"pyr_tall": {v["pyr_tall"]}, "top": {v["top"]}, "chain": {v["chain"]}}}'
                               for k, v in forced.items()))
            f.write("\n}\n}\n")
        print(f"  forced {field} = {val}", flush=True)
        out, t3, _ = _run(B, p, l, r)
        assert t3 == 0.0
        assert _equal(out, ref), (field, val)


def test_no_cache_file_when_disabled(B, tmp_path, monkeypatch):
    from paper_2205_03133_amd.synth import make_pair, method_params
    monkeypatch.setenv("BDIS_TUNE_CACHE", "")
    monkeypatch.setenv("HOME", str(tmp_path))
    left, right, _, _ = make_pair(1, 0)
    _run(B, B.params(**method_params(1)), to_gpu(left), to_gpu(right))
    assert not os.path.exists(tmp_path / ".cache")
