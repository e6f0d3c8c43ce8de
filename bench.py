"""Benchmark: path-steps/s for price + full vol-grid adjoint on one MI355X.

A step is one pass of the whole path over one batch: the per-step vol table,
Philox normals, LDS vol lookup, log-Euler stepping with stored states, payoff and
FP64 reductions, the reverse sweep (over the paths whose adjoint is not zero) with
the fixed-point LDS gradient histogram, and the fixed-order merge -- for the
workload of the paper's timing run: one call, 2^19 paths (the paper's 500K), 156
weekly steps, a 60 x 30 = 1800-node grid, FP32 stepping.

Prints one JSON line.  Also reports the FP64 GPU variant, the forward-only,
checkpointed and every-path-reverse variants, their accuracy against each other,
the roofline of the dominant kernel and the CPU oracle timed on a bounded sample.
"""
import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz issue 3.93e13 vector lane-slots/s
# (the 157.3 TFLOP/s FP32 figure counts an FMA as 2 and packed FP32 as 2 lanes; the
# kernels are built without packed FP32).  HBM3E 8 TB/s.
PEAK_HBM_GBS = 8000.0
PEAK_SLOTS_T = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic work per path-step on the log-spot axis, in VALU issue slots: each
# operation of the method weighted by its issue cost on gfx950 (full rate 1;
# 32x32->64 multiply 2.4; transcendental 3.1), as itemised below.
SLOTS_FWD = 37.7    # Philox/4 17 + uniforms 3 + Box-Muller 7.7 + lookup 7 + Euler 2 + store 1
SLOTS_REV = 26.1    # per live path-step: load 1 + lookup 7 + slope 4 + c_n 6.1 + adjoint 2 + scatter 6
BYTES_FWD = 4.0     # one FP32 state written per path-step
BYTES_REV = 4.0     # one FP32 state read per live path-step


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_call_60x30.json")
    src = os.path.join(ROOT, "paper_2002_02481_amd", "csrc", "lv_kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    return rec.get("bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the FP64/forward/checkpoint variants")
    ap.add_argument("--launch", default="", metavar="BLOCK,COPIES,WINDOW,BPC,FWD_BLOCK,FWD_BPC",
                    help="fix the launch shape instead of autotuning it")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def copy_probe(mib: int):
    import torch
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": a.numel() * 4}), flush=True)


def settle(fn, min_steps, min_ms=40.0):
    """Call fn at least min_steps times and for at least min_ms of GPU time: the first
    milliseconds of work after idle run slower while the GPU's clocks settle."""
    import torch
    torch.cuda.synchronize()
    t0, n = time.perf_counter(), 0
    while n < min_steps or (time.perf_counter() - t0) * 1e3 < min_ms:
        fn()
        n += 1
        if n % 8 == 0 or n >= min_steps:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return n


def other_workloads(lv, W, ctx, dev):
    """The 64-option book and the 32-surface checkpointed batch at full size, each with
    its autotuned launch shape: path-steps/s of price + grid adjoint (FP32)."""
    import numpy as np
    import torch
    out = {}
    wl = W.book_60x30()
    s, b = wl.surface, wl.book
    sig = torch.tensor(s.sigma, dtype=torch.float64, device=dev)
    kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, is_put=b.is_put, weights=b.weight, ctx=ctx,
              autotune=True)
    o = lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, wl.seed, **kw)
    settle(lambda: lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, wl.seed,
                                       out=o, **kw), 10)
    t0 = time.perf_counter()
    for _ in range(20):
        lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, wl.seed, out=o, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / 20
    out[wl.name] = {"ms_per_step": ms, "value": wl.n_paths * wl.n_steps / (ms * 1e-3), "options": b.n,
                    "adjoint": "stored, live paths"}
    wl = W.surface_batch()
    s, b = wl.surface, wl.book
    sig = torch.tensor(np.stack([x.sigma for x in wl.surfaces]), dtype=torch.float64, device=dev)
    kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, ctx=ctx, adjoint="checkpoint", ckpt_every=16,
              autotune=True)
    o = lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, wl.seed, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, wl.seed, out=o, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    n_s = len(wl.surfaces)
    out[wl.name] = {"ms_per_step": ms, "value": n_s * wl.n_paths * wl.n_steps / (ms * 1e-3), "surfaces": n_s,
                    "adjoint": "checkpoint every 16"}
    return out


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for {args.gpus}); across GPUs the path "
              "would shard by Philox path range, each GPU sweeping its own paths", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2002_02481_amd as lv
    import workloads as W

    wl = W.single_call_60x30()
    s = wl.surface
    P, N = wl.n_paths, wl.n_steps
    dev = torch.device("cuda:0")
    sig = torch.tensor(s.sigma, dtype=torch.float64, device=dev)
    ctx = lv.Context(0)
    kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, ctx=ctx)
    strikes, mats = wl.book.strike, wl.book.maturity

    def base_run(out=None, **opts):
        return lv.price_and_grad_dev(sig, 100.0, strikes, mats, P, N, wl.seed, out=out, **kw, **opts)

    if args.launch:
        bl, k, w, c, fb, fc = (int(x) for x in args.launch.split(","))
        out = [t for t in base_run(block=bl, copies=k, window=w, blocks_per_cu=c, fwd_block=fb,
                                   fwd_blocks_per_cu=fc)]
    else:
        first = [t for t in base_run()]                 # default shape: clocks up before tuning
        settle(lambda: base_run(out=first), 5)
        out = [t for t in base_run(autotune=True)]      # first tuned call tunes the launch shape
    torch.cuda.synchronize()
    info = ctx.run_info()
    shape = dict(block=info["block"], copies=info["copies"], window=info["window"],
                 blocks_per_cu=info["blocks_per_cu"], fwd_block=info["fwd_block"],
                 fwd_blocks_per_cu=info["fwd_blocks_per_cu"])

    def run(out=None, **opts):
        for k, v in shape.items():
            opts.setdefault(k, v)
        return base_run(out=out, **opts)

    # fraction of paths the reverse sweep visits: those ending in the money
    _, _, states = lv.forward_dev(sig, 100.0, strikes, mats, P, N, wl.seed, spot_axis=s.spot_axis,
                                  time_axis=s.time_axis, ctx=ctx)
    y_last = states.view(torch.float32).view(N, P)[N - 1]
    live_frac = float((100.0 * torch.exp(y_last) > float(strikes[0])).double().mean())
    del states, y_last
    torch.cuda.synchronize()

    # no Python garbage collection while GPU work is timed (a collection stalls the
    # host for milliseconds); it runs again before the CPU baseline
    gc.collect()
    gc.disable()
    # warmup: every kernel timed with HIP events, to find the dominant kernel
    settle(lambda: run(out=out, profile=True), args.warmup)
    warm = ctx.kernel_times(reset=True)
    warm_avg = {k: (ms / n if n else 0.0) for k, (ms, n) in warm.items()}
    dom = max(("fwd", "rev"), key=lambda k: warm_avg[k])
    dom_bit = 1 << lv._lib.KERNEL_KINDS.index(dom)

    # timed region: events on the dominant kernel only (a timed dispatch waits for its
    # timestamp, so timing every kernel would slow the step it measures)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run(out=out, profile=True, profile_kinds=dom_bit)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = P * N / (ms_per_step * 1e-3)
    times = ctx.kernel_times(reset=True)
    avg = dict(warm_avg)
    avg[dom] = times[dom][0] / times[dom][1]

    # roofline of the dominant kernel: algorithmic slots per launch / its mean duration
    units = P * N * (1.0 if dom == "fwd" else live_frac)     # path-steps of work per launch
    slots = (SLOTS_FWD if dom == "fwd" else SLOTS_REV) * units
    byts = (BYTES_FWD if dom == "fwd" else BYTES_REV) * units
    achieved = slots / (avg[dom] * 1e-3) / 1e12
    frac_of = {k: round((SLOTS_FWD * P * N if k == "fwd" else SLOTS_REV * P * N * live_frac)
                        / (avg[k] * 1e-3) / 1e12 / PEAK_SLOTS_T, 4) for k in ("fwd", "rev")}
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3),
                "peak": round(PEAK_SLOTS_T, 3), "unit": "Tops/s", "frac": round(achieved / PEAK_SLOTS_T, 4),
                "traffic": measured_traffic(dom),
                "slots_per_path_step": SLOTS_FWD if dom == "fwd" else SLOTS_REV,
                "path_steps_per_launch": units, "live_fraction": round(live_frac, 5),
                "frac_by_kernel": frac_of,
                "hbm_achieved_GBs": round(byts / (avg[dom] * 1e-3) / 1e9, 1),
                "hbm_frac": round(byts / (avg[dom] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                "avg_ms": {k: round(v, 5) for k, v in avg.items() if v},
                "avg_ms_from": f"{dom}: HIP events over the timed region; others: events over the warmup steps"}

    price32, se32, grad32, delta32 = [t.cpu().numpy().copy() for t in out]
    result = {
        "metric": "path-steps/s for price + full vol-grid adjoint, FP32 vs FP64 GPU at fixed error",
        "value": value, "unit": "path-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded 60x30 local-vol surface, Philox streams)",
        "config": {"workload": wl.name, "paths": P, "steps": N, "grid": list(s.sigma.shape),
                   "options": 1, "adjoint": "stored, live paths", "parallelism": "none", "launch": shape},
        "roofline": roofline,
    }

    if not args.no_variants:
        variants = {}
        def timed(n, **opts):
            """Mean step of the fastest of three runs of n steps (a host stall in one run
            does not count)."""
            o = [t for t in base_run(autotune=True, **opts)]     # tunes this variant's shape
            settle(lambda: base_run(out=o, autotune=True, **opts), 5)
            best = float("inf")
            for _ in range(3):
                t0 = time.perf_counter()
                for _ in range(n):
                    base_run(out=o, autotune=True, **opts)
                torch.cuda.synchronize()
                best = min(best, (time.perf_counter() - t0) * 1e3 / n)
            return best, o
        ms64, o64 = timed(max(3, args.steps // 4), precision=64)
        p64, g64 = o64[0].cpu().numpy(), o64[2].cpu().numpy()
        variants["fp64_gpu"] = {"ms_per_step": ms64, "value": P * N / (ms64 * 1e-3)}
        msf, _ = timed(args.steps, adjoint="none", want_grad=False)
        variants["fp32_forward_only"] = {"ms_per_step": msf, "value": P * N / (msf * 1e-3)}
        msc, oc = timed(max(3, args.steps // 2), adjoint="checkpoint")
        variants["fp32_checkpoint"] = {"ms_per_step": msc, "value": P * N / (msc * 1e-3),
                                       "max_bucket_err_vs_stored": float(np.abs(oc[2].cpu().numpy() - grad32).max() / np.abs(grad32).max())}
        mse, oe = timed(args.steps, scheme="euler_x")
        variants["fp32_euler_step_on_price"] = {"ms_per_step": mse, "value": P * N / (mse * 1e-3),
                                                "price": float(oe[0].cpu().numpy().ravel()[0])}
        msec, oec = timed(max(3, args.steps // 2), scheme="euler_x", adjoint="checkpoint")
        variants["fp32_euler_step_on_price_checkpoint"] = {
            "ms_per_step": msec, "value": P * N / (msec * 1e-3),
            "max_bucket_err_vs_stored": float(np.abs(oec[2].cpu().numpy() - oe[2].cpu().numpy()).max()
                                              / np.abs(oe[2].cpu().numpy()).max())}
        # the TPU runs' mixed precision held sigma in bfloat16 for the interpolation
        # (Sec. IV-D); the same rounding of the nodes here, with its effect on the
        # estimates next to FP32's own distance from FP64 on the same paths
        msh, oh = timed(args.steps, sigma_bf16=True)
        ph, gh = oh[0].cpu().numpy(), oh[2].cpu().numpy()
        gscale = np.abs(g64).max()
        variants["fp32_sigma_nodes_bf16"] = {
            "ms_per_step": msh, "value": P * N / (msh * 1e-3),
            "price_diff_vs_fp64": float(np.abs(ph - p64).max()),
            "max_bucket_diff_vs_fp64": float(np.abs(gh - g64).max() / gscale),
            "fp32_price_diff_vs_fp64": float(np.abs(price32 - p64).max()),
            "fp32_max_bucket_diff_vs_fp64": float(np.abs(grad32 - g64).max() / gscale),
            "price_std_err": float(se32.max())}
        msd, od = timed(max(3, args.steps // 2), dense_adjoint=True)
        variants["fp32_every_path_reverse"] = {
            "ms_per_step": msd, "value": P * N / (msd * 1e-3),
            "max_bucket_diff_vs_live": float(np.abs(od[2].cpu().numpy() - grad32).max() / np.abs(grad32).max())}
        # bumping (Sec. III), the estimator the adjoint replaces: 2 I J forward pricings of
        # bumped surfaces on the same paths, timed once after one untimed run
        gb = torch.empty_like(sig)
        bump = lambda: lv.bump_grad_dev(sig, 100.0, strikes, mats, P, N, wl.seed, spot_axis=s.spot_axis,
                                        time_axis=s.time_axis, eps=1e-3, batch=512, out=gb, ctx=ctx, **shape)
        bump()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bump()
        torch.cuda.synchronize()
        msb = (time.perf_counter() - t0) * 1e3
        variants["fp32_bump_and_reprice"] = {
            "ms_per_gradient": msb, "surfaces_priced": 2 * int(sig.numel()), "eps": 1e-3,
            "slower_than_adjoint_step": msb / ms_per_step,
            "max_bucket_diff_vs_adjoint": float(np.abs(gb.cpu().numpy() - grad32).max() / np.abs(grad32).max())}
        # the host-buffer entry point: surface in, prices and grid out through PCIe (not `value`)
        settle(lambda: lv.price_and_grad(s, 100.0, strikes, mats, P, N, wl.seed, ctx=ctx, **shape), 5)
        t0 = time.perf_counter()
        for _ in range(10):
            lv.price_and_grad(s, 100.0, strikes, mats, P, N, wl.seed, ctx=ctx, **shape)
        msh = (time.perf_counter() - t0) * 1e3 / 10
        variants["fp32_host_buffers_pcie"] = {"ms_per_step": msh, "value": P * N / (msh * 1e-3)}
        result["variants"] = variants
        result["workloads"] = other_workloads(lv, W, ctx, dev)
        result["accuracy"] = {
            "fp32_vs_fp64_gpu_price_abs": float(abs(price32.ravel()[0] - p64.ravel()[0])),
            "fp32_vs_fp64_gpu_max_bucket_err_rel_maxg": float(np.abs(grad32 - g64).max() / np.abs(g64).max()),
            "price": float(price32.ravel()[0]), "stderr": float(se32.ravel()[0]),
            # FP32's own error is far below the Monte Carlo error of the same paths, so at
            # a fixed error both precisions need the same paths and the speed ratio is
            # the ratio of step times
            "fp32_error_over_stderr": float(abs(price32.ravel()[0] - p64.ravel()[0]) / se32.ravel()[0]),
            "fp32_speedup_over_fp64_at_fixed_error": float(ms64 / ms_per_step),
        }

    gc.enable()
    if not args.no_cpu:
        import oracle
        o = oracle.default()
        n_threads = oracle.default_threads()
        sample = 32768
        t0 = time.perf_counter()
        o.price_and_grad(s, wl.book, sample, N, wl.seed, n_threads=n_threads)
        dt = time.perf_counter() - t0
        # scale the sample up to a budget of about 10 s of CPU work
        reps = max(1, int(10.0 / max(dt, 1e-3)))
        if reps > 1:
            t0 = time.perf_counter()
            o.price_and_grad(s, wl.book, sample * reps, N, wl.seed, n_threads=n_threads)
            dt = time.perf_counter() - t0
            sample *= reps
        result["cpu_baseline"] = {"value": sample * N / dt, "unit": "path-steps/s", "cores": n_threads,
                                  "kind": "oracle",
                                  "sample": f"{sample} paths x {N} steps of {wl.name}, FP64, price + grid adjoint"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
