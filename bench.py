"""Throughput of the BDIS hot path on one MI355X.

One step = one full coarse-to-fine pass (pyramid, patch search, probability,
fusion, variance) over one 640x480 synthetic pair (5 levels, 8x8 patches,
stride 3, 16 iterations, variance on), inputs resident in HBM.  Prints one
JSON line with the throughput in output Mpixel/s, the roofline of the
dominant kernel (the patch search) measured with HIP events over the timed
region, and the FP64 CPU oracle's throughput on the host cores as a baseline.
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published fp32 vector peak
HBM_PEAK_GBS = 8000.0
WIN = 5


def search_flops(bdis, p, w, h):
    """Algorithmic flops of the patch search per pass: per patch 4P^2 (template
    setup) + 5KP^2 (K warped-patch iterations) + 8sP^2 (s-sample window), FMA = 2."""
    tot = 0
    for n in range(p.levels):
        _, _, nx, ny = bdis.level_dims(p, w, h, n)
        P2 = p.patch * p.patch
        tot += nx * ny * (4 * P2 + 5 * p.iters * P2 + 8 * WIN * P2)
    return tot


def cpu_baseline(left, right, params, budget_s=16.0):
    """The FP64 oracle, one pair per thread on the host cores, on a bounded sample."""
    from oracle import ref
    ref.build(force=False)
    threads = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    ref.compute(left, right, params)
    t1 = time.perf_counter() - t0
    reps = max(1, int(round(budget_s / (t1 * threads))))
    n = threads * reps

    def job(_):
        ref.compute(left, right, params)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(job, range(n)))
    dt = time.perf_counter() - t0
    h, w = left.shape
    return dict(value=round(w * h * n / dt / 1e6, 4), unit="Mpixel/s", cores=threads, kind="oracle",
                sample=f"{n} oracle passes over the 640x480 pair ({threads} threads x {reps}), "
                       f"{dt:.1f} s wall")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path has no multi-GPU form here "
              "(pairs shard across GPUs with no communication; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2205_03133_amd import bdis
    from paper_2205_03133_amd.synth import make_pair, method_params

    bdis.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    left, right, gt, valid = make_pair(2, 0)
    h, w = left.shape
    mp = method_params(2)
    p = bdis.params(**mp)
    ctx = bdis.Context(p, w, h)
    lt = torch.from_numpy(left).to(dev)
    rt = torch.from_numpy(right).to(dev)
    out = dict(disp=torch.empty((h, w), dtype=torch.float32, device=dev),
               var=torch.empty((h, w), dtype=torch.float32, device=dev),
               conf=torch.empty((h, w), dtype=torch.float32, device=dev))
    print(f"[bench] 640x480 pair, L={p.levels} P={p.patch} S={p.stride} K={p.iters}, "
          f"warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        ctx.compute(lt, rt, out=out)
    torch.cuda.synchronize()

    ctx.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.compute(lt, rt, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tk = ctx.timing_read()
    ctx.timing(False)

    # accuracy of this run's output vs the synthetic ground truth (context only)
    d = out["disp"].cpu().numpy()
    ok = np.isfinite(d) & valid
    epe = float(np.median(np.abs(d[ok] - gt[ok])))

    ms = dt * 1e3 / args.steps
    value = w * h * args.steps / dt / 1e6
    s_ms, s_n = tk["search"]
    flops = search_flops(bdis, p, w, h)
    achieved = flops * args.steps / (s_ms * 1e-3) / 1e12
    roof = dict(bound="alu", achieved=round(achieved, 3), peak=FP32_VECTOR_PEAK_TFLOPS,
                unit="TFLOP/s", frac=round(achieved / FP32_VECTOR_PEAK_TFLOPS, 5), traffic=None,
                kernel="k_search_u8<8>", avg_launch_us=round(s_ms * 1e3 / max(s_n, 1), 3),
                launches=s_n)
    kernels = {k: dict(total_ms=round(v[0], 4), launches=v[1],
                       avg_us=round(v[0] * 1e3 / max(v[1], 1), 3)) for k, v in tk.items()}
    line = dict(metric="disparity Mpixel/s (640x480)", value=round(value, 3), unit="Mpixel/s",
                n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=round(ms, 4),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="int32+f64+f32",
                data="synthetic",
                config=dict(workload="640x480 synthetic stereo pair (planes+bumps 0-64 px, 20% textureless, "
                                     "highlights, gain U(0.8,1.2), noise 2), L=5 P=8 S=3 K=16 variance on",
                            global_batch=1, pairs_per_step=1),
                roofline=roof, kernels=kernels, epe_median_px=round(epe, 4))
    if not args.no_cpu_baseline:
        from oracle import ref
        rp = ref.default_params(**mp)
        line["cpu_baseline"] = cpu_baseline(left, right, rp)
    line["paper_context"] = "17 Hz (0.064 s) at 640x480 on one i5-9400 core, levels 5..1, P=10, K=12"
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
