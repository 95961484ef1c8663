"""Throughput of the BDIS hot path on one MI355X.

Headline: one step = one full coarse-to-fine pass (pyramid, patch search,
probability, fusion, variance) over one 640x480 synthetic pair (5 levels, 8x8
patches, stride 3, 16 iterations, variance on), inputs resident in HBM, through
the library's default path (the captured launch graph).  A second timed region
of the same K steps runs eagerly with per-kernel HIP events that each kernel
dispatch records itself (the library's timing mode) and gives the roofline of
the dominant kernel (the patch search), overall and per pyramid level.  The
oracle's result on the same pair gives the parity figures of the line.

Also reported: the 1920x1080 batch stream (6 levels, 12x12 patches, stride 4,
16 iterations, variance on) on one GPU's share of 64 pairs, and the FP64 CPU
oracle on the host cores as a baseline.
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X vector peaks: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz = 78.6
# TFLOP/s for non-packed 32-bit and for FP64 operations (the rate the search's
# int32 / dot4 / FP64 code issues at: packed FP32 is disabled for all device
# code of this build), 157.3 TFLOP/s with packed FP32 (reported beside it).
VALU_PEAK_TFLOPS = 78.6
FP32_PACKED_PEAK_TFLOPS = 157.3
WIN = 5


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def search_flops(bdis, p, w, h, levels=None, skip=()):
    """Algorithmic flops of the patch search of one pass: per patch 4P^2 (template
    setup) + 5KP^2 (K warped-patch iterations) + 8sP^2 (s-sample window), FMA = 2.
    Levels in `skip` (searched inside the fused coarsest-level kernel) are left out."""
    tot = 0
    P2 = p.patch * p.patch
    for n in range(levels or p.levels):
        if n in skip:
            continue
        _, _, nx, ny = bdis.level_dims(p, w, h, n)
        tot += nx * ny * (4 * P2 + 5 * p.iters * P2 + 8 * WIN * P2)
    return tot


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "search_hbm_traffic_640x480_1080p_batch64_mixed64.md")
# the search kernel's sources: the kernel, its per-patch body and the header
# that fixes its layouts and launch shapes
SEARCH_SRC = [os.path.join(ROOT, "paper_2205_03133_amd", "csrc", "k_search.hip"),
              os.path.join(ROOT, "paper_2205_03133_amd", "csrc", "search_common.h"),
              os.path.join(ROOT, "paper_2205_03133_amd", "csrc", "bdis_internal.h")]


def search_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for p in SEARCH_SRC:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def measured_traffic(workload, levels):
    """HBM bytes per search launch from the committed FETCH_SIZE/WRITE_SIZE counter
    runs (per level, scaled by the copy-kernel calibration): the mean over the
    levels this run's pass searched, so that it matches the timed launches
    whichever structure the tuner picked for the coarsest level.  None when a
    level was not counted or the kernel source differs from the one the
    counters were taken on."""
    try:
        text = open(TRAFFIC_FILE).read()
        src = search_source_sha256()
    except OSError:
        return None
    sha, per_level = None, {}
    for ln in text.splitlines():
        f = ln.split()
        if len(f) == 3 and f[0] == "source_sha256":
            sha = f[2]
        if len(f) == 4 and f[0] == "traffic_bytes_level" and f[1] == workload:
            per_level[int(f[2])] = int(f[3])
    levels = list(levels)
    if sha != src or not levels or any(n not in per_level for n in levels):
        return None
    return sum(per_level[n] for n in levels) // len(levels)


HBM_PEAK_GBS = 8000.0   # MI355X published HBM3E bandwidth


def search_bytes(bdis, p, w, h, levels=None, skip=()):
    """Algorithmic HBM bytes of the patch search of one pass: both level images
    (1 B per pixel each), per patch what the later phases read (displacement,
    propagated probability, four window SSD differences as FP64, acceptance:
    52 B written) and the 4-tap reads of the parent maps (64 B, every level but
    the coarsest)."""
    L = levels or p.levels
    tot = 0
    for n in range(p.finest_level, L):
        if n in skip:
            continue
        lw, lh, nx, ny = bdis.level_dims(p, w, h, n)
        tot += 2 * lw * lh + nx * ny * (52 + (64 if n + 1 < L else 0))
    return tot


def roofline(flops_per_step, steps, timing, kernel_name, workload, levels, bytes_per_step=None):
    s_ms, s_n = timing["search"]
    achieved = flops_per_step * steps / (s_ms * 1e-3) / 1e12
    out = dict(bound="alu", achieved=round(achieved, 3), peak=VALU_PEAK_TFLOPS, unit="TFLOP/s",
               frac=round(achieved / VALU_PEAK_TFLOPS, 5), traffic=measured_traffic(workload, levels),
               frac_of_packed_fp32_peak=round(achieved / FP32_PACKED_PEAK_TFLOPS, 5),
               traffic_unit="bytes per launch", kernel=kernel_name,
               avg_launch_us=round(s_ms * 1e3 / max(s_n, 1), 3), launches=s_n)
    launch_s = s_ms * 1e-3 / max(s_n, 1)
    if bytes_per_step is not None:
        per_launch = bytes_per_step * steps / max(s_n, 1)
        out["hbm_frac_algorithmic"] = round(per_launch / launch_s / 1e9 / HBM_PEAK_GBS, 5)
    if out["traffic"] is not None:
        out["hbm_frac_counters"] = round(out["traffic"] / launch_s / 1e9 / HBM_PEAK_GBS, 5)
    return out


def kernel_table(tk):
    return {k: dict(total_ms=round(v[0], 4), launches=v[1], avg_us=round(v[0] * 1e3 / max(v[1], 1), 3))
            for k, v in tk.items()}


# A GPU's share of the host: at most this many oracle threads (one GPU of a
# node gets 16 cores, whatever the node's core count).
HOST_CORE_SHARE = 16


def host_info():
    """Cores the process may use, the node's count and the CPU model."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(nproc=os.cpu_count(), usable=usable, threads=max(1, min(HOST_CORE_SHARE, usable)), model=model)


def oracle_throughput(jobs, threads, keep_first=False):
    """Runs the oracle on every (left, right, params) job over `threads` threads
    (ctypes releases the GIL); returns (wall seconds, output pixels, the first
    job's result if keep_first)."""
    from oracle import ref

    def job(j):
        return ref.compute(j[0], j[1], j[2])

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(job, jobs))
    dt = time.perf_counter() - t0
    return dt, sum(j[0].shape[0] * j[0].shape[1] for j in jobs), (res[0] if keep_first else None)


def cpu_baseline(left, right, params, budget_s=16.0):
    """The FP64 oracle on the host cores on a bounded sample of the headline
    workload: one pass on one core (also kept for the parity figures), then
    copies of the pair one per thread.  Returns (baseline dict, oracle result)."""
    from oracle import ref
    ref.build(force=False)
    hi = host_info()
    threads = hi["threads"]
    t0 = time.perf_counter()
    res = ref.compute(left, right, params)
    t1 = time.perf_counter() - t0
    reps = max(1, int(round(budget_s / (t1 * threads))))
    n = threads * reps
    dt, px, _ = oracle_throughput([(left, right, params)] * n, threads)
    h, w = left.shape
    return dict(value=round(px / dt / 1e6, 4), unit="Mpixel/s", cores=threads, kind="oracle",
                sample=f"{n} oracle passes over the 640x480 pair ({threads} threads x {reps}), "
                       f"{dt:.1f} s wall, {n * t1:.1f} s of CPU work",
                one_core=dict(value=round(w * h / t1 / 1e6, 4), unit="Mpixel/s", seconds_per_pair=round(t1, 4)),
                host=hi, note=f"{threads} threads: the host-core share of one GPU (the node shows {hi['nproc']})"), res


def accuracy(d, gt, valid):
    """Median end-point error and bad-1px over ground-truth-valid pixels with an
    estimate, and the fraction of ground-truth-valid pixels with an estimate."""
    import numpy as np
    ok = np.isfinite(d) & valid
    e = np.abs(d[ok] - gt[ok])
    return dict(epe_median_px=round(float(np.median(e)), 4), bad1px=round(float((e > 1.0).mean()), 5),
                density=round(float(ok.sum() / max(valid.sum(), 1)), 4))


def parity_block(disp, var, ref_res, tol=1e-3, rtol=1e-3):
    """GPU outputs against the FP64 oracle on the same pair: fraction of pixels
    within tol px (a validity-mask disagreement counts as a miss), p99.9 and max
    error, mask mismatches; variance at relative rtol likewise."""
    import numpy as np

    def stats(g, r, rel):
        g = np.asarray(g, np.float64)
        r = np.asarray(r, np.float64)
        gv, rv = np.isfinite(g), np.isfinite(r)
        both = gv & rv
        err = np.abs(g - r)
        if rel:
            err = err / np.maximum(np.abs(r), 1e-30)
        lim = rtol if rel else tol
        ok = (both & (err <= lim)) | (~gv & ~rv)
        e = err[both]
        return dict(frac=round(float(ok.mean()), 6), p999=float(f"{np.quantile(e, 0.999):.3g}") if e.size else 0.0,
                    max=float(f"{e.max():.3g}") if e.size else 0.0, mask_mismatch=int((gv != rv).sum()))
    out = dict(disparity=dict(tol_px=tol, **stats(disp, ref_res["disp"], False)))
    if var is not None and ref_res.get("var") is not None:
        out["variance"] = dict(rtol=rtol, **stats(var, ref_res["var"], True))
    return out


def top_levels(ctx, levels):
    """Levels of the timed region that ran in the fused coarsest-level kernel."""
    return {n for n in range(levels) if ctx.timing_read(n)["top"][1] > 0}


def search_per_level(bdis, ctx, p, w, h, steps, npairs=1, levels=None, shapes=None):
    """Per-level search launches of the event region: patches, mean launch time
    and the algorithmic rate against the vector peak.  `shapes` (a list of
    (w, h, levels) per pair) replaces npairs copies of w x h for mixed batches."""
    out = []
    P2 = p.patch * p.patch
    shapes = shapes or [(w, h, levels or p.levels)] * npairs
    for n in range(p.finest_level, max(s[2] for s in shapes)):
        ms, k = ctx.timing_read(n)["search"]
        if k == 0:
            continue
        patches = 0
        for (sw, sh, sl) in shapes:
            if n < sl:
                _, _, nx, ny = bdis.level_dims(p, sw, sh, n)
                patches += nx * ny
        flops = patches * (4 * P2 + 5 * p.iters * P2 + 8 * WIN * P2)
        per = ms * 1e-3 / k
        out.append(dict(level=n, patches=patches, avg_us=round(per * 1e6, 3),
                        tflops=round(flops / per / 1e12, 3), frac=round(flops / per / 1e12 / VALU_PEAK_TFLOPS, 5)))
    return out


def bench_single(bdis, torch, args):
    import numpy as np
    from paper_2205_03133_amd.synth import make_pair, method_params
    dev = torch.device("cuda:0")
    left, right, gt, valid = make_pair(2, 0)
    h, w = left.shape
    p = bdis.params(**method_params(2))
    ctx = bdis.Context(p, w, h)
    lt = torch.from_numpy(left).to(dev)
    rt = torch.from_numpy(right).to(dev)
    out = {k: torch.empty((h, w), dtype=torch.float32, device=dev) for k in ("disp", "var", "conf")}
    log(f"640x480 pair, L={p.levels} P={p.patch} S={p.stride} K={p.iters}: warmup {args.warmup}")
    t0 = time.perf_counter()
    ctx.compute(lt, rt, out=out)
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    tune_ms, cap_ms = ctx.setup_time()
    for _ in range(args.warmup):
        ctx.compute(lt, rt, out=out)
    torch.cuda.synchronize()
    log(f"timed region: {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.compute(lt, rt, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"per-kernel event region: {args.steps} steps")
    ctx.timing(True)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        ctx.compute(lt, rt, out=out)
    torch.cuda.synchronize()
    dt_ev = time.perf_counter() - t1
    tk = ctx.timing_read()
    per_level = search_per_level(bdis, ctx, p, w, h, args.steps)
    top = top_levels(ctx, p.levels)
    ctx.timing(False)
    d = out["disp"].cpu().numpy()
    var = out["var"].cpu().numpy()
    acc = accuracy(d, gt, valid)
    ctx.close()
    # single-call latency: host call to finished outputs, one call at a time
    ctx = bdis.Context(p, w, h)
    ctx.compute(lt, rt, out=out)
    torch.cuda.synchronize()
    lat = []
    for _ in range(min(args.steps, 50)):
        t0 = time.perf_counter()
        ctx.compute(lt, rt, out=out)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    tune2, cap2 = ctx.setup_time()
    ctx.close()
    lat.sort()
    setup = dict(first_call_ms=round(first_ms, 2), tune_ms=round(tune_ms, 2), capture_ms=round(cap_ms, 2),
                 note="first call of a new shape tunes the launch shapes (cached per shape and in the tuning "
                      "file) and captures the graph; both outside the timed regions")
    return dict(w=w, h=h, p=p, dt=dt, dt_ev=dt_ev, tk=tk, top=top, acc=acc, left=left, right=right, disp=d, var=var,
                mp=method_params(2), per_level=per_level, setup=setup,
                latency_ms=dict(median=round(lat[len(lat) // 2], 4), p90=round(lat[int(len(lat) * 0.9)], 4),
                                calls=len(lat)))


def bench_c1(bdis, torch, args):
    """The small workload: one 320x240 pair (3 levels, P 8, S 4, K 8), one call
    per step; throughput over the steps and single-call latency."""
    from paper_2205_03133_amd.synth import make_pair, method_params
    dev = torch.device("cuda:0")
    left, right, gt, valid = make_pair(1, 0)
    h, w = left.shape
    p = bdis.params(**method_params(1))
    lt, rt = torch.from_numpy(left).to(dev), torch.from_numpy(right).to(dev)
    out = {k: torch.empty((h, w), dtype=torch.float32, device=dev) for k in ("disp", "conf")}
    with bdis.Context(p, w, h) as ctx:
        for _ in range(args.warmup):
            ctx.compute(lt, rt, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.compute(lt, rt, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        lat = []
        for _ in range(min(args.steps, 50)):
            t1 = time.perf_counter()
            ctx.compute(lt, rt, out=out)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t1) * 1e3)
    lat.sort()
    return dict(ms_per_pair=round(dt * 1e3, 4), mpx_s=round(w * h / dt / 1e6, 2),
                latency_ms=dict(median=round(lat[len(lat) // 2], 4), p90=round(lat[int(len(lat) * 0.9)], 4)),
                **accuracy(out["disp"].cpu().numpy(), gt, valid),
                config="320x240 pair (bumps 0-32 px, noise 1 on the right), L=3 P=8 S=4 K=8, variance off")


def bench_batch(bdis, torch, args):
    """One GPU's share (64 pairs) of the 512-pair 1920x1080 stream, one call per step."""
    import numpy as np
    from paper_2205_03133_amd.synth import make_pair, method_params
    dev = torch.device("cuda:0")
    uniq = args.batch_unique
    log(f"1080p batch: generating {uniq} pairs")
    base = [make_pair(5, i) for i in range(uniq)]
    p = bdis.params(**method_params(5))
    n = args.batch_pairs
    lefts = [torch.from_numpy(base[i % uniq][0]).to(dev) for i in range(n)]
    rights = [torch.from_numpy(base[i % uniq][1]).to(dev) for i in range(n)]
    ctx = bdis.Context(p, 1920, 1080, max_batch=n)
    outs = [{k: torch.empty((1080, 1920), dtype=torch.float32, device=dev) for k in ("disp", "var", "conf")}
            for _ in range(n)]
    log(f"1080p batch of {n}: warmup (includes tuning and graph capture)")
    t0 = time.perf_counter()
    ctx.compute_batch(lefts, rights, outs=outs)
    torch.cuda.synchronize()
    setup = dict(first_call_ms=round((time.perf_counter() - t0) * 1e3, 2))
    setup["tune_ms"], setup["capture_ms"] = (round(x, 2) for x in ctx.setup_time())
    ctx.compute_batch(lefts, rights, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        ctx.compute_batch(lefts, rights, outs=outs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing(True)
    for _ in range(max(1, args.batch_steps // 2)):
        ctx.compute_batch(lefts, rights, outs=outs)
    torch.cuda.synchronize()
    tk = ctx.timing_read()
    per_level = search_per_level(bdis, ctx, p, 1920, 1080, max(1, args.batch_steps // 2), npairs=n)
    top = top_levels(ctx, p.levels)
    ctx.timing(False)
    nu = min(n, uniq)
    dd = [outs[i]["disp"].cpu().numpy() for i in range(nu)]
    acc = accuracy(np.stack(dd), np.stack([base[i][2] for i in range(nu)]), np.stack([base[i][3] for i in range(nu)]))
    d0 = dd[0]
    v0 = outs[0]["var"].cpu().numpy()
    ctx.close()
    # the plain form: the same pairs one call each (single-pair context)
    log("1080p pairs one at a time (plain form)")
    one = bdis.Context(p, 1920, 1080)
    o1 = {k: torch.empty((1080, 1920), dtype=torch.float32, device=dev) for k in ("disp", "var", "conf")}
    for i in range(2):
        one.compute(lefts[i], rights[i], out=o1)
    torch.cuda.synchronize()
    reps = max(uniq, 8)
    t0 = time.perf_counter()
    for i in range(reps):
        one.compute(lefts[i % n], rights[i % n], out=o1)
    torch.cuda.synchronize()
    dt1 = (time.perf_counter() - t0) / reps
    one.compute(lefts[0], rights[0], out=o1)
    torch.cuda.synchronize()
    same0 = bool(torch.equal(torch.nan_to_num(o1["disp"], nan=-7.0), torch.nan_to_num(outs[0]["disp"], nan=-7.0)))
    one.close()
    steps_ev = max(1, args.batch_steps // 2)
    mpx = 1920 * 1080 * n * args.batch_steps / dt / 1e6
    flops = search_flops(bdis, p, 1920, 1080, skip=top) * n
    res = dict(metric="disparity Mpixel/s (1080p batch)", value=round(mpx, 2), unit="Mpixel/s",
               pairs_per_step=n, unique_pairs=uniq, steps=args.batch_steps,
               ms_per_step=round(dt * 1e3 / args.batch_steps, 3),
               config=dict(workload="1920x1080 synthetic pairs (planes+bumps 0-192 px, 30% textureless, "
                                    "dark gain U(0.2,0.5), noise 3), L=6 P=12 S=4 K=16 variance on",
                           share="64 of the 512-pair stream"),
               roofline=roofline(flops, steps_ev, tk, "k_search_u8<12>", "1080p_batch64",
                                 [m for m in range(p.finest_level, p.levels) if m not in top],
                                 search_bytes(bdis, p, 1920, 1080, skip=top) * n),
               search_per_level=per_level, kernels=kernel_table(tk), setup=setup, **acc,
               plain_single=dict(ms_per_pair=round(dt1 * 1e3, 4), mpx_s=round(1920 * 1080 / dt1 / 1e6, 2),
                                 same_bits_as_batch_pair0=same0,
                                 note="one bdis_compute per pair on a single-pair context, same pairs and method"))
    return res, dict(left=base[0][0], right=base[0][1], disp=d0, var=v0, base=base, p=p)


def bench_mixed(bdis, torch, args):
    """Mixed-resolution batch: 64 pairs from 320x240 to 1920x1080 (8 per size,
    4-6 levels by size, P 8, S 3, K 16, variance on) in one call per step."""
    import numpy as np
    from paper_2205_03133_amd.synth import c3_sizes, make_pair, method_params
    dev = torch.device("cuda:0")
    sizes = c3_sizes()
    log("mixed batch: generating one pair per size")
    base = {}
    for i, wh in enumerate(sizes):
        if wh not in base:
            base[wh] = (i, make_pair(3, i))
    mp = [method_params(3, i) for i in range(len(sizes))]
    p = bdis.params(**{k: v for k, v in mp[0].items() if k != "levels"}, levels=6)
    lefts = [torch.from_numpy(base[wh][1][0]).to(dev) for wh in sizes]
    rights = [torch.from_numpy(base[wh][1][1]).to(dev) for wh in sizes]
    levels = [m["levels"] for m in mp]
    outs = [{k: torch.empty((h, w), dtype=torch.float32, device=dev) for k in ("disp", "var", "conf")}
            for (w, h) in sizes]
    ctx = bdis.Context(p, 1920, 1080, max_batch=len(sizes))
    for _ in range(2):
        ctx.compute_batch(lefts, rights, levels=levels, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        ctx.compute_batch(lefts, rights, levels=levels, outs=outs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing(True)
    steps_ev = max(1, args.batch_steps // 2)
    for _ in range(steps_ev):
        ctx.compute_batch(lefts, rights, levels=levels, outs=outs)
    torch.cuda.synchronize()
    tk = ctx.timing_read()
    top = top_levels(ctx, max(levels))
    per_level = search_per_level(bdis, ctx, p, 0, 0, steps_ev,
                                 shapes=[(w, h, levels[i]) for i, (w, h) in enumerate(sizes)])
    ctx.timing(False)
    errs, bad, dens = [], [], []
    for wh, (i, pr) in base.items():
        k = sizes.index(wh)
        d = outs[k]["disp"].cpu().numpy()
        ok = np.isfinite(d) & pr[3]
        errs.append(np.abs(d[ok] - pr[2][ok]))
        dens.append(ok.sum() / max(pr[3].sum(), 1))
    ctx.close()
    ae = np.concatenate(errs)
    px = sum(w * h for (w, h) in sizes)
    flops = sum(search_flops(bdis, p, w, h, levels[i], skip=top) for i, (w, h) in enumerate(sizes))
    nbytes = sum(search_bytes(bdis, p, w, h, levels[i], skip=top) for i, (w, h) in enumerate(sizes))
    return dict(metric="disparity Mpixel/s (mixed batch)", value=round(px * args.batch_steps / dt / 1e6, 2),
                unit="Mpixel/s", pairs_per_step=len(sizes), megapixels_per_step=round(px / 1e6, 3),
                unique_pairs=len(base), steps=args.batch_steps, ms_per_step=round(dt * 1e3 / args.batch_steps, 3),
                config=dict(workload="64 synthetic pairs, 8 each of 320x240 .. 1920x1080, disparity up to 10% of "
                                     "the width, L=4..6 by size, P=8 S=3 K=16 variance on"),
                roofline=roofline(flops, steps_ev, tk, "k_search_u8<8>", "mixed64",
                                  [m for m in range(p.finest_level, max(levels)) if m not in top], nbytes),
                search_per_level=per_level, kernels=kernel_table(tk), epe_median_px=round(float(np.median(ae)), 4),
                bad1px=round(float((ae > 1.0).mean()), 5), density=round(float(np.mean(dens)), 4),
                _oracle_jobs=[(base[wh][1][0], base[wh][1][1], mp[sizes.index(wh)]) for wh in sizes])


def bench_preset(bdis, torch, args):
    """The paper's preset on the 640x480 pair: levels 5..1 searched, P 10,
    overlap 0.55 (S 4), 12 iterations, gamma 0.75, pixel threshold 0.15; the
    level-1 maps upsampled to full resolution.  Without and with variance."""
    import numpy as np
    from paper_2205_03133_amd.synth import make_pair
    dev = torch.device("cuda:0")
    left, right, gt, valid = make_pair(2, 0)
    lt, rt = torch.from_numpy(left).to(dev), torch.from_numpy(right).to(dev)
    out = {}
    for var in (0, 1):
        p = bdis.params(levels=6, finest_level=1, patch=10, stride=4, iters=12, valid_ratio=0.75,
                        sigma_s=4.0, prob_thresh=0.15, variance=var)
        ctx = bdis.Context(p, 640, 480)
        res = None
        for _ in range(args.warmup):
            res = ctx.compute(lt, rt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = ctx.compute(lt, rt)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        d = res["disp"].cpu().numpy()
        ok = np.isfinite(d) & valid
        out["variance_on" if var else "variance_off"] = dict(
            ms_per_pair=round(dt * 1e3, 4), mpx_s=round(640 * 480 / dt / 1e6, 2),
            valid_frac=round(float(np.isfinite(d).mean()), 4), **accuracy(d, gt, valid))
        ctx.close()
    out["config"] = "640x480 pair (planes+bumps 0-64 px), levels 5..1, P=10 S=4 K=12, gamma 0.75, prob 0.15"
    out["paper_cpu_s"] = dict(variance_off=0.064, variance_on=0.072,
                              note="one i5-9400 core, synthetic colon data (context)")
    return out


ABLATIONS = [("bdis", {}), ("no_sgmm", dict(fusion=2)), ("no_coarse_to_fine", dict(propagate=0)),
             ("no_dynamic_sigma", dict(sigma_r_dynamic=0, sigma_r=8.0)), ("dis_weights_eq2", dict(fusion=1))]


def bench_ablation(bdis, torch, args):
    """Accuracy of the ablations of Sec. V (and the DIS weighting of Eq. 2) on
    synthetic 640x480 pairs with ground truth: median / mean absolute disparity
    error over valid pixels, and each normalised by the full method's."""
    import numpy as np
    from paper_2205_03133_amd.synth import make_pair, method_params
    dev = torch.device("cuda:0")
    pairs = [make_pair(2, 100 + i) for i in range(args.ablation_pairs)]
    out = {}
    for name, kw in ABLATIONS:
        mp = dict(method_params(2))
        mp.update(kw)
        ctx = bdis.Context(bdis.params(**mp), 640, 480)
        med, mean, cov, bad = [], [], [], []
        for left, right, gt, valid in pairs:
            d = ctx.compute(torch.from_numpy(left).to(dev), torch.from_numpy(right).to(dev))["disp"].cpu().numpy()
            ok = np.isfinite(d) & valid
            e = np.abs(d[ok] - gt[ok])
            med.append(float(np.median(e)))
            mean.append(float(e.mean()))
            cov.append(float(ok.sum() / valid.sum()))
            bad.append(float((e > 1.0).mean()))
        ctx.close()
        out[name] = dict(median_px=round(float(np.mean(med)), 4), mean_px=round(float(np.mean(mean)), 4),
                         bad1px=round(float(np.mean(bad)), 5), valid_frac=round(float(np.mean(cov)), 4))
    for name in out:
        out[name]["median_norm"] = round(out[name]["median_px"] / out["bdis"]["median_px"], 4)
        out[name]["mean_norm"] = round(out[name]["mean_px"] / out["bdis"]["mean_px"], 4)
    out["config"] = (f"{args.ablation_pairs} synthetic 640x480 pairs (planes+bumps 0-64 px), L=5 P=8 S=3 K=16; "
                     "errors averaged over pairs")
    return out


def bench_coverage(bdis, torch, args):
    """Variance coverage per frame (the Table 6 check on synthetic ground truth):
    fraction of valid pixels with |d - d_gt| <= 1.96 sqrt(Var), on the 640x480
    workload and on the paper preset (levels 5..1, variance upsampled)."""
    import numpy as np
    from paper_2205_03133_amd.synth import make_pair, method_params
    dev = torch.device("cuda:0")
    pairs = [make_pair(2, 200 + i) for i in range(args.ablation_pairs)]
    presets = dict(workload_640x480=dict(method_params(2)),
                   paper_preset=dict(levels=6, finest_level=1, patch=10, stride=4, iters=12, valid_ratio=0.75,
                                     sigma_s=4.0, prob_thresh=0.15, variance=1))
    out = {}
    for name, mp in presets.items():
        ctx = bdis.Context(bdis.params(**mp), 640, 480)
        fr = []
        for left, right, gt, valid in pairs:
            o = ctx.compute(torch.from_numpy(left).to(dev), torch.from_numpy(right).to(dev))
            c, t = ctx.coverage(o["disp"], o["var"], torch.from_numpy(gt.astype(np.float32)).to(dev), 1.96,
                                valid=torch.from_numpy(valid.astype(np.uint8)).to(dev))
            fr.append(c / max(t, 1))
        ctx.close()
        out[name] = dict(per_frame=[round(x, 4) for x in fr], mean=round(float(np.mean(fr)), 4),
                         ideal=0.95)
    return out


def bench_flow(bdis, torch, args):
    """Optical-flow form: one 640x480 pair of frames with a smooth 2-D flow up to
    12 px (L=4 P=8 S=4 K=12), one call per step."""
    import numpy as np
    from paper_2205_03133_amd.synth import make_flow_pair
    dev = torch.device("cuda:0")
    i0, i1, gu, gv, valid = make_flow_pair(0, 640, 480, 12.0)
    a, b = torch.from_numpy(i0).to(dev), torch.from_numpy(i1).to(dev)
    ctx = bdis.Context(bdis.params(levels=4, patch=8, stride=4, iters=12), 640, 480)
    for _ in range(args.warmup):
        u, v = ctx.flow(a, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        u, v = ctx.flow(a, b)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ctx.timing(True)
    for _ in range(max(1, args.steps // 4)):
        ctx.flow(a, b)
    tk = ctx.timing_read()
    ctx.timing(False)
    epe = np.hypot(u.cpu().numpy() - gu, v.cpu().numpy() - gv)[valid]
    ctx.close()
    return dict(ms_per_pair=round(dt * 1e3, 4), mpx_s=round(640 * 480 / dt / 1e6, 2),
                epe_median_px=round(float(np.median(epe)), 4), epe_mean_px=round(float(epe.mean()), 4),
                bad1px=round(float((epe > 1.0).mean()), 5),
                kernels=kernel_table({k: tk[k] for k in ("pyramid", "search", "fuse")}),
                config="640x480 frames, smooth 2-D flow up to 12 px, noise 2; L=4 P=8 S=4 K=12, Eq. 2 fusion")


def bench_diff(bdis, torch, args):
    """Differentiable form: a batch of 16 float 640x480 pairs, forward and backward
    (K = 8 unrolled, 4 levels, P 8, S 4), and the plain uint8 form on the same pairs."""
    import numpy as np
    from paper_2205_03133_amd.synth import make_pair, method_params
    dev = torch.device("cuda:0")
    n, uniq = args.diff_pairs, min(args.diff_pairs, 4)
    log(f"differentiable form: {n} pairs 640x480 ({uniq} unique)")
    base = [make_pair(4, i, quantize=False) for i in range(uniq)]
    L = torch.stack([torch.from_numpy(base[i % uniq][0].astype(np.float32)) for i in range(n)]).to(dev)
    R = torch.stack([torch.from_numpy(base[i % uniq][1].astype(np.float32)) for i in range(n)]).to(dev)
    mp = method_params(4)
    p = bdis.params(**mp)
    ctx = bdis.Context(p, 640, 480, max_batch=n, train=True)
    g = torch.randn((n, 480, 640), generator=torch.Generator().manual_seed(0)).to(dev)
    for _ in range(2):
        ctx.compute_f32(L, R)
        ctx.backward(g)
    torch.cuda.synchronize()
    reps = args.diff_steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_f = t_b = 0.0
    for _ in range(reps):
        ev[0].record()
        out = ctx.compute_f32(L, R)
        ev[1].record()
        ctx.backward(g)
        ev[2].record()
        torch.cuda.synchronize()
        t_f += ev[0].elapsed_time(ev[1])
        t_b += ev[1].elapsed_time(ev[2])
    d = out["disp"].cpu().numpy()
    epe_f = [np.abs(d[i][np.isfinite(d[i]) & base[i][3]] - base[i][2][np.isfinite(d[i]) & base[i][3]])
             for i in range(uniq)]
    ctx.close()
    # the plain form on the same pairs, quantised to uint8
    pu = bdis.params(**{k: v for k, v in mp.items() if k != "float_pyramid"})
    ctxu = bdis.Context(pu, 640, 480, max_batch=n)
    Lu = [torch.from_numpy(np.clip(np.rint(base[i % uniq][0]), 0, 255).astype(np.uint8)).to(dev) for i in range(n)]
    Ru = [torch.from_numpy(np.clip(np.rint(base[i % uniq][1]), 0, 255).astype(np.uint8)).to(dev) for i in range(n)]
    for _ in range(2):
        outs = ctxu.compute_batch(Lu, Ru)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        outs = ctxu.compute_batch(Lu, Ru)
    ev[1].record()
    torch.cuda.synchronize()
    t_u = ev[0].elapsed_time(ev[1]) / reps
    du = [outs[i]["disp"].cpu().numpy() for i in range(uniq)]
    epe_u = [np.abs(du[i][np.isfinite(du[i]) & base[i][3]] - base[i][2][np.isfinite(du[i]) & base[i][3]])
             for i in range(uniq)]
    ctxu.close()
    fwd, bwd = t_f / reps, t_b / reps
    return dict(pairs=n, unique_pairs=uniq, fwd_ms=round(fwd, 3), bwd_ms=round(bwd, 3),
                bwd_fwd_ratio=round(bwd / fwd, 3), fwd_mpx_s=round(640 * 480 * n / fwd / 1e3, 2),
                plain_u8_ms=round(t_u, 3), plain_u8_mpx_s=round(640 * 480 * n / t_u / 1e3, 2),
                epe_median_px_float=round(float(np.median(np.concatenate(epe_f))), 4),
                epe_median_px_plain=round(float(np.median(np.concatenate(epe_u))), 4),
                bad1px_float=round(float((np.concatenate(epe_f) > 1.0).mean()), 5),
                bad1px_plain=round(float((np.concatenate(epe_u) > 1.0).mean()), 5),
                config="16 x 640x480 float pairs (bumps 0-32 px), L=4 P=8 S=4 K=8, FP64 state; "
                       "loss gradient = random field")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batch-pairs", type=int, default=64)
    ap.add_argument("--batch-unique", type=int, default=4)
    ap.add_argument("--batch-steps", type=int, default=6)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--diff-pairs", type=int, default=16)
    ap.add_argument("--diff-steps", type=int, default=5)
    ap.add_argument("--no-diff", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ablation-pairs", type=int, default=4, help="pairs of the accuracy ablation (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain float32 copy kernel over MIB MiB (reference for HBM counters)")
    ap.add_argument("--only", default="", metavar="LEGS",
                    help="comma-separated legs to run besides the headline pair (c1, batch, mixed, preset, flow, "
                         "ablation, diff); default all.  For profiling one workload at a time.")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU form "
              "(pairs would shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2205_03133_amd import bdis

    bdis.lib()
    torch.cuda.set_device(0)
    s = bench_single(bdis, torch, args)
    w, h, p = s["w"], s["h"], s["p"]
    value = w * h * args.steps / s["dt"] / 1e6
    line = dict(metric="disparity Mpixel/s (640x480)", value=round(value, 3), unit="Mpixel/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=round(s["dt"] * 1e3 / args.steps, 4),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="int32+f64",
                data="synthetic",
                config=dict(workload="640x480 synthetic stereo pair (planes+bumps 0-64 px, 20% textureless, "
                                     "highlights, gain U(0.8,1.2), noise 2), L=5 P=8 S=3 K=16 variance on",
                            global_batch=1, pairs_per_step=1),
                roofline=roofline(search_flops(bdis, p, w, h, skip=s["top"]), args.steps, s["tk"], "k_search_u8<8>",
                                  "640x480", [m for m in range(p.finest_level, p.levels) if m not in s["top"]],
                                  search_bytes(bdis, p, w, h, skip=s["top"])),
                kernels=kernel_table(s["tk"]),
                ms_per_step_with_kernel_events=round(s["dt_ev"] * 1e3 / args.steps, 4),
                latency_ms=s["latency_ms"], setup=s["setup"], **s["acc"])
    line["roofline"]["per_level"] = s["per_level"]
    legs = set(x.strip() for x in args.only.split(",") if x.strip())
    run = lambda name: not legs or name in legs  # noqa: E731
    if run("c1"):
        line["c1_320x240"] = bench_c1(bdis, torch, args)
    batch_extra, mixed_jobs = None, None
    if not args.no_batch and run("batch"):
        line["batch_1080p"], batch_extra = bench_batch(bdis, torch, args)
    if not args.no_batch and run("mixed"):
        line["batch_mixed"] = bench_mixed(bdis, torch, args)
        mixed_jobs = line["batch_mixed"].pop("_oracle_jobs")
    if run("preset"):
        line["paper_preset"] = bench_preset(bdis, torch, args)
    if run("flow"):
        line["optical_flow"] = bench_flow(bdis, torch, args)
    if args.ablation_pairs > 0 and run("ablation"):
        line["ablation"] = bench_ablation(bdis, torch, args)
        line["variance_coverage"] = bench_coverage(bdis, torch, args)
    if not args.no_diff and run("diff"):
        line["differentiable_c4"] = bench_diff(bdis, torch, args)
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)  # reads and writes exactly 4n bytes
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = 4 * n
    if not args.no_cpu_baseline:
        from oracle import ref
        from paper_2205_03133_amd.synth import method_params
        log("cpu baseline (FP64 oracle) and parity of the 640x480 pair")
        line["cpu_baseline"], ores = cpu_baseline(s["left"], s["right"], ref.default_params(**s["mp"]))
        line["parity"] = parity_block(s["disp"], s["var"], ores)
        threads = line["cpu_baseline"]["cores"]
        if batch_extra is not None:
            log("oracle on 16 of the 1080p pairs (parity of pair 0, throughput)")
            base = batch_extra["base"]
            op = ref.default_params(**method_params(5))
            jobs = [(base[i % len(base)][0], base[i % len(base)][1], op) for i in range(16)]
            dt, px, r0 = oracle_throughput(jobs, threads, keep_first=True)
            line["batch_1080p"]["parity_pair0"] = parity_block(batch_extra["disp"], batch_extra["var"], r0)
            line["batch_1080p"]["cpu_oracle"] = dict(
                value=round(px / dt / 1e6, 4), unit="Mpixel/s", cores=threads, kind="oracle",
                sample=f"16 oracle passes over the 1080p pairs ({len(base)} unique), {dt:.1f} s wall",
                seconds_for_512_pairs_extrapolated=round(dt * 512 / 16, 1))
        if mixed_jobs is not None:
            log("oracle on the 64 mixed pairs")
            jobs = [(l, r, ref.default_params(**m)) for (l, r, m) in mixed_jobs]
            dt, px, _ = oracle_throughput(jobs, threads)
            line["batch_mixed"]["cpu_oracle"] = dict(
                value=round(px / dt / 1e6, 4), unit="Mpixel/s", cores=threads, kind="oracle",
                sample=f"all 64 pairs ({len(set(id(j[0]) for j in jobs))} unique), {dt:.1f} s wall")
    line["paper_context"] = "17 Hz (0.064 s) at 640x480 on one i5-9400 core, levels 5..1, P=10, K=12"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
