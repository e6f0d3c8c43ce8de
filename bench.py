"""Benchmark: path-steps/s for price + full vol-grid adjoint on one MI355X.

A step is one pass of the whole path over one batch of the largest single-GPU
workload: 32 perturbed 100 x 50 local-vol surfaces priced and differentiated on the
same 2^24 Philox paths of 260 weekly steps each (one call, T = 5y) -- the per-step
vol table, Philox normals, LDS vol lookup, log-Euler stepping with checkpoints every
16 steps, payoff and FP64 reductions, the re-simulation and reverse sweep of the
paths whose adjoint is not zero with the fixed-point LDS gradient histogram, and the
fixed-order merge, for every surface.  FP32 stepping and adjoint, FP64 cross-path
sums.

Prints one JSON line.  Also reports the all-FP64 GPU variant on the same paths (the
"fixed error" pair), the roofline of the dominant kernel, the 60 x 30 single-call
workload (the paper's timing run) with its variants, the 64-option book
(hipGraph-captured), the precision study (FP32 against FP64 on the GPU, and a flat
surface against Black-Scholes), and the CPU oracle timed on a bounded sample of the
headline workload.
"""
import argparse
import gc
import hashlib
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
PEAK_FP32_TFLOPS = 157.3

# Algorithmic work in VALU issue slots: each operation of the method weighted by its
# issue cost on gfx950 (full rate 1; 32x32->64 multiply 2.4; transcendental 3.1).  A
# Philox round is two multiplies and two three-input XORs (one instruction each on
# gfx950); a uniform is a funnel shift and a subtraction; the lookup's cell fraction is
# one instruction.
# Log-spot axis, per path-step:
SLOTS_FWD = 35.7    # Philox/4 17 + uniforms 2 + Box-Muller 7.7 + lookup 6 + Euler 2 + store 1
SLOTS_REV = 25.1    # per live path-step: load 1 + lookup 6 + slope 4 + c_n 6.1 + adjoint 2 + scatter 6
# Linear spot axis, checkpointed (fused) kernel: e^y for the lookup costs 4.1 (a multiply
# and an exp; the spot is folded into the axis scale) wherever a forward lookup is made.
SLOTS_FUSED_ALL = 38.9    # every path-step: forward 35.7 - store 1 + exp 4.1 + checkpoint 1/16
SLOTS_FUSED_LIVE = 56.8   # every live path-step: re-simulation 38.9 - 1/16 + c_n 1, and the
                          # reverse: lookup 6 + slope 3 + adjoint 2 + scatter 6 (the segment
                          # keeps the re-simulation's e^y, so no exp)
BYTES_FWD = 4.0     # one FP32 state written per path-step
BYTES_REV = 4.0     # one FP32 state read per live path-step

METRIC = "path-steps/s for price + full vol-grid adjoint, FP32 vs FP64 GPU at fixed error"


KERNEL_SOURCES = {"fused": "lv_k_fused.hip", "fwd": "lv_k_fwd.hip", "rev": "lv_k_rev.hip", "opt": "lv_k_opt.hip"}


def source_sha(kernel: str):
    """sha256 over the sources a kernel is compiled from: its own file and the shared
    device header and declarations."""
    h = hashlib.sha256()
    for name in (KERNEL_SOURCES[kernel], "lv_device.h", "lv_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2002_02481_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != source_sha(kernel):
        return None
    return rec.get("bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true",
                    help="headline only: no FP64 pair, other workloads or precision study")
    ap.add_argument("--launch", default="", metavar="BLOCK,COPIES,BPC",
                    help="fix the headline's launch shape instead of autotuning it")
    ap.add_argument("--only-call-60x30", default="", metavar="BLOCK,COPIES,WINDOW,BPC,FBLOCK,FBPC",
                    help="only time the 60 x 30 call's stored adjoint at this launch shape (for profiling)")
    ap.add_argument("--tuning", default="", metavar="FILE",
                    help="take saved launch shapes from FILE (if it exists) and save the tuned ones to it")
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


def best_of(fn, n, reps=3):
    """Mean step of the fastest of `reps` runs of n steps (a host stall in one run
    does not count)."""
    import torch
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) * 1e3 / n)
    return best


def cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    quota = None
    try:
        q, period = open("/sys/fs/cgroup/cpu.max").read().split()
        if q != "max":
            quota = float(q) / float(period)
    except (OSError, ValueError):
        pass
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(nproc=os.cpu_count(), affinity=affinity, cgroup_cpus=quota, model=model)


def live_fraction(lv, sig, wl, ctx, n_sample):
    """Fraction of paths whose adjoint is not zero (the call ends in the money), per
    surface, from the first n_sample paths of the same Philox streams."""
    import torch
    s, b = wl.surface, wl.book
    out = []
    states = None
    for k in range(sig.shape[0]):
        _, _, states = lv.forward_dev(sig[k], 100.0, b.strike, b.maturity, n_sample, wl.n_steps, wl.seed,
                                      spot_axis=s.spot_axis, time_axis=s.time_axis, states=states, ctx=ctx)
        last = states.view(torch.float32)[(wl.n_steps - 1) * n_sample: wl.n_steps * n_sample]
        out.append(float((100.0 * torch.exp(last.double()) > float(b.strike[0])).double().mean()))
    del states
    torch.cuda.synchronize()
    return out


def headline(lv, W, ctx, args):
    """The 32-surface batch, FP32 checkpointed adjoint: value, timing and roofline."""
    import numpy as np
    import torch
    wl = W.surface_batch()
    s, b = wl.surface, wl.book
    P, N, S = wl.n_paths, wl.n_steps, len(wl.surfaces)
    dev = torch.device("cuda:0")
    sig = torch.tensor(np.stack([x.sigma for x in wl.surfaces]), dtype=torch.float64, device=dev)
    kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, ctx=ctx, adjoint="checkpoint",
              ckpt_every=wl.ckpt_every)

    def run(out=None, **opts):
        return lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, P, N, wl.seed, out=out, **{**kw, **opts})

    if args.launch:
        bl, k, c = (int(x) for x in args.launch.split(","))
        shape = dict(block=bl, copies=k, blocks_per_cu=c)
        out = [t for t in run(**shape)]
    else:
        out = [t for t in run()]                         # default shape: clocks up before tuning
        torch.cuda.synchronize()
        out = [t for t in run(autotune=True, out=out)]   # tunes on the first surface
        torch.cuda.synchronize()
        info = ctx.run_info()
        shape = dict(block=info["block"], copies=info["copies"], blocks_per_cu=info["blocks_per_cu"])
    torch.cuda.synchronize()

    fused_bit = 1 << lv._lib.KERNEL_KINDS.index("fused")
    gc.collect()
    gc.disable()
    for _ in range(args.warmup):
        run(out=out, profile=True, **shape)
    torch.cuda.synchronize()
    warm = ctx.kernel_times(reset=True)
    # timed region: events on the dominant kernel only
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run(out=out, profile=True, profile_kinds=fused_bit, **shape)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc.enable()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = S * P * N / (ms_per_step * 1e-3)
    times = ctx.kernel_times(reset=True)
    fused_ms = times["fused"][0] / times["fused"][1]
    warm_avg = {k: (ms / n if n else 0.0) for k, (ms, n) in warm.items()}

    live = live_fraction(lv, sig, wl, ctx, 1 << 20)
    live_mean = float(np.mean(live))
    units = P * N                                       # path-steps per launch (one surface)
    slots = SLOTS_FUSED_ALL * units + SLOTS_FUSED_LIVE * units * live_mean
    achieved = slots / (fused_ms * 1e-3) / 1e12
    step_slots = S * slots
    roofline = {"bound": "alu", "kernel": "fused", "achieved": round(achieved, 3),
                "peak": round(PEAK_SLOTS_T, 3), "unit": "Tops/s", "frac": round(achieved / PEAK_SLOTS_T, 4),
                "traffic": measured_traffic("fused", "batch32"),
                "slots_per_path_step": {"all": SLOTS_FUSED_ALL, "live": SLOTS_FUSED_LIVE},
                "path_steps_per_launch": units, "live_fraction": round(live_mean, 5),
                "live_fraction_sample": "first 2^20 paths of each surface",
                "whole_step_frac": round(step_slots / (ms_per_step * 1e-3) / 1e12 / PEAK_SLOTS_T, 4),
                "launches_per_step": S,
                "avg_ms": {"fused": round(fused_ms, 4),
                           **{k: round(v, 4) for k, v in warm_avg.items() if v and k != "fused"}},
                "avg_ms_from": "fused: HIP events over the timed region; others: events over the warmup steps",
                "checkpoint_bytes_per_path_step": round(2 * 4.0 / wl.ckpt_every, 4)}
    p32, se32, g32, d32 = [t.cpu().numpy().copy() for t in out]
    res = {
        "metric": METRIC, "value": value, "unit": "path-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (32 seeded 100x50 local-vol surfaces, Philox streams)",
        "config": {"workload": wl.name, "surfaces": S, "paths": P, "steps": N, "grid": list(s.sigma.shape),
                   "options": b.n, "adjoint": f"checkpoint every {wl.ckpt_every}, live paths",
                   "parallelism": "none", "launch": shape},
        "roofline": roofline,
    }
    return res, dict(wl=wl, sig=sig, run=run, shape=shape, p32=p32, se32=se32, g32=g32, kw=kw)


def headline_fp64(lv, W, ctx, h, args):
    """The all-FP64 GPU variant on the same surfaces and paths: its step time and the
    FP32 result's distance from it."""
    import numpy as np
    import torch
    wl, run = h["wl"], h["run"]
    o = [t for t in run(precision=64, autotune=True)]
    torch.cuda.synchronize()
    ms64 = best_of(lambda: run(out=o, precision=64, autotune=True), 1, reps=2)
    p64, se64, g64 = [t.cpu().numpy() for t in o[:3]]
    S, P, N = len(wl.surfaces), wl.n_paths, wl.n_steps
    gmax = np.abs(g64).reshape(S, -1).max(axis=1)
    err = np.abs(h["g32"] - g64).reshape(S, -1).max(axis=1) / gmax
    # Monte Carlo standard error of every bucket of the last surface, from the spread of
    # the FP64 call's per-block partial sums (blocks take interleaved path tiles)
    G = g64[-1].size
    blocks = ctx.block_grads(G)
    B = blocks.shape[0]
    se_b = blocks.std(axis=0, ddof=1) * np.sqrt(B) / P
    d_last = np.abs(h["g32"][-1] - g64[-1]).ravel()
    ratio = d_last[se_b > 0] / se_b[se_b > 0]
    return {"ms_per_step": ms64, "value": S * P * N / (ms64 * 1e-3), "launch": ctx.run_info()["block"]}, {
        "fp32_vs_fp64_gpu_price_abs_max": float(np.abs(h["p32"] - p64).max()),
        "fp32_price_err_over_stderr_max": float((np.abs(h["p32"] - p64) / se64).max()),
        "fp32_vs_fp64_gpu_max_bucket_err_rel_maxg": {"max": float(err.max()), "median": float(np.median(err)),
                                                     "per_surface": [round(float(x), 6) for x in err]},
        "fp32_vs_fp64_bucket_err_over_mc_stderr_last_surface": {
            "max": float(ratio.max()), "q99": float(np.quantile(ratio, 0.99)),
            "median": float(np.median(ratio)), "blocks": int(B)},
        "stderr_price_mean": float(se64.mean()),
    }


def headline_stored(lv, ctx, h):
    """The same 32 surfaces with every state stored (17 GB per surface in FP32) and
    swept back by the stored reverse kernel instead of checkpoints and recompute."""
    import numpy as np
    import torch
    wl, run = h["wl"], h["run"]
    o = [t for t in run(adjoint="stored", autotune=True)]
    torch.cuda.synchronize()
    ms = best_of(lambda: run(out=o, adjoint="stored", autotune=True), 1, reps=2)
    S, P, N = len(wl.surfaces), wl.n_paths, wl.n_steps
    g = o[2].cpu().numpy()
    gmax = np.abs(h["g32"]).reshape(S, -1).max(axis=1)
    diff = np.abs(g - h["g32"]).reshape(S, -1).max(axis=1) / gmax
    info = ctx.run_info()
    r = {"ms_per_step": ms, "value": S * P * N / (ms * 1e-3),
         "state_bytes_per_surface": lv.states_bytes(32, P, N),
         "launch": {k: info[k] for k in ("block", "copies", "window", "blocks_per_cu", "fwd_block",
                                         "fwd_blocks_per_cu")},
         "max_bucket_diff_vs_checkpointed_rel_maxg": float(diff.max())}
    del o
    torch.cuda.empty_cache()
    return r


def call_60x30_fixed(lv, W, ctx, dev, args):
    """The 60 x 30 call's stored adjoint at a fixed launch shape, warm-up then timed
    steps with every kernel's events: the run its rocprofv3 summaries come from."""
    import torch
    wl = W.single_call_60x30()
    s = wl.surface
    sig = torch.tensor(s.sigma, dtype=torch.float64, device=dev)
    b, k, w, c, fb, fc = (int(x) for x in args.only_call_60x30.split(","))
    shape = dict(block=b, copies=k, window=w, blocks_per_cu=c, fwd_block=fb, fwd_blocks_per_cu=fc)
    run = lambda out=None, **o: lv.price_and_grad_dev(sig, 100.0, wl.book.strike, wl.book.maturity, wl.n_paths,
                                                      wl.n_steps, wl.seed, spot_axis=s.spot_axis,
                                                      time_axis=s.time_axis, ctx=ctx, out=out, **shape, **o)
    out = [t for t in run()]
    settle(lambda: run(out=out), max(args.warmup, 1))
    ctx.kernel_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run(out=out, profile=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    kt = ctx.kernel_times(reset=True)
    return {"workload": wl.name, "launch": shape, "steps": args.steps, "ms_per_step_with_events": ms,
            "avg_ms": {k: round(v / n, 5) for k, (v, n) in kt.items() if n}}


def call_60x30(lv, W, ctx, dev):
    """The paper's timing-run shape (2^19 paths, 156 steps, 60 x 30): FP32 stored adjoint
    and its variants, with the kernel roofline of its two kernels."""
    import numpy as np
    import torch
    wl = W.single_call_60x30()
    s = wl.surface
    P, N = wl.n_paths, wl.n_steps
    sig = torch.tensor(s.sigma, dtype=torch.float64, device=dev)
    kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, ctx=ctx)
    strikes, mats = wl.book.strike, wl.book.maturity

    def base(out=None, **opts):
        return lv.price_and_grad_dev(sig, 100.0, strikes, mats, P, N, wl.seed, out=out, **kw, **opts)

    first = [t for t in base()]
    settle(lambda: base(out=first), 5)
    out = [t for t in base(autotune=True)]
    torch.cuda.synchronize()
    info = ctx.run_info()
    shape = dict(block=info["block"], copies=info["copies"], window=info["window"],
                 blocks_per_cu=info["blocks_per_cu"], fwd_block=info["fwd_block"],
                 fwd_blocks_per_cu=info["fwd_blocks_per_cu"])

    def run(out=None, **opts):
        for k, v in shape.items():
            opts.setdefault(k, v)
        return base(out=out, **opts)

    _, _, states = lv.forward_dev(sig, 100.0, strikes, mats, P, N, wl.seed, spot_axis=s.spot_axis,
                                  time_axis=s.time_axis, ctx=ctx)
    y_last = states.view(torch.float32).view(N, P)[N - 1]
    live = float((100.0 * torch.exp(y_last) > float(strikes[0])).double().mean())
    del states, y_last
    gc.collect()
    gc.disable()
    settle(lambda: run(out=out, profile=True), 30)
    kt = ctx.kernel_times(reset=True)
    avg = {k: (ms / n if n else 0.0) for k, (ms, n) in kt.items()}
    ms = best_of(lambda: run(out=out), 50)
    gc.enable()
    frac = {"fwd": SLOTS_FWD * P * N / (avg["fwd"] * 1e-3) / 1e12 / PEAK_SLOTS_T,
            "rev": SLOTS_REV * P * N * live / (avg["rev"] * 1e-3) / 1e12 / PEAK_SLOTS_T}
    whole = (SLOTS_FWD + SLOTS_REV * live) * P * N / (ms * 1e-3) / 1e12 / PEAK_SLOTS_T
    p32, se32, g32 = [t.cpu().numpy().copy() for t in out[:3]]
    res = {"ms_per_step": ms, "value": P * N / (ms * 1e-3), "launch": shape, "live_fraction": round(live, 5),
           "roofline": {"frac_by_kernel": {k: round(v, 4) for k, v in frac.items()},
                        "whole_step_frac": round(whole, 4),
                        "avg_ms": {k: round(v, 5) for k, v in avg.items() if v},
                        "traffic": {k: measured_traffic(k, "call_60x30") for k in ("fwd", "rev")},
                        "hbm_GBs": {"fwd": round(BYTES_FWD * P * N / (avg["fwd"] * 1e-3) / 1e9, 1),
                                    "rev": round(BYTES_REV * P * N * live / (avg["rev"] * 1e-3) / 1e9, 1)}}}

    def timed(n, **opts):
        o = [t for t in base(autotune=True, **opts)]
        settle(lambda: base(out=o, autotune=True, **opts), 5)
        return best_of(lambda: base(out=o, autotune=True, **opts), n), o

    v = {}
    ms64, o64 = timed(12, precision=64)
    p64, g64 = o64[0].cpu().numpy(), o64[2].cpu().numpy()
    gscale = np.abs(g64).max()
    v["fp64_gpu"] = {"ms_per_step": ms64, "value": P * N / (ms64 * 1e-3)}
    msf, _ = timed(50, adjoint="none", want_grad=False)
    v["fp32_forward_only"] = {"ms_per_step": msf, "value": P * N / (msf * 1e-3)}
    msc, oc = timed(25, adjoint="checkpoint")
    v["fp32_checkpoint"] = {"ms_per_step": msc, "value": P * N / (msc * 1e-3),
                            "max_bucket_diff_vs_stored": float(np.abs(oc[2].cpu().numpy() - g32).max() / np.abs(g32).max())}
    mse, oe = timed(50, scheme="euler_x")
    v["fp32_euler_step_on_price"] = {"ms_per_step": mse, "value": P * N / (mse * 1e-3)}
    msh, oh = timed(50, sigma_bf16=True)
    v["fp32_sigma_nodes_bf16"] = {"ms_per_step": msh, "value": P * N / (msh * 1e-3),
                                  "price_diff_vs_fp64": float(np.abs(oh[0].cpu().numpy() - p64).max()),
                                  "max_bucket_diff_vs_fp64": float(np.abs(oh[2].cpu().numpy() - g64).max() / gscale)}
    msd, od = timed(25, dense_adjoint=True)
    v["fp32_every_path_reverse"] = {"ms_per_step": msd, "value": P * N / (msd * 1e-3)}
    gb = torch.empty_like(sig)
    bump = lambda: lv.bump_grad_dev(sig, 100.0, strikes, mats, P, N, wl.seed, spot_axis=s.spot_axis,
                                    time_axis=s.time_axis, eps=1e-3, batch=512, out=gb, ctx=ctx, **shape)
    bump()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bump()
    torch.cuda.synchronize()
    msb = (time.perf_counter() - t0) * 1e3
    v["fp32_bump_and_reprice"] = {"ms_per_gradient": msb, "surfaces_priced": 2 * int(sig.numel()), "eps": 1e-3,
                                  "slower_than_adjoint_step": msb / ms,
                                  "max_bucket_diff_vs_adjoint": float(np.abs(gb.cpu().numpy() - g32).max() / np.abs(g32).max())}
    settle(lambda: lv.price_and_grad(s, 100.0, strikes, mats, P, N, wl.seed, ctx=ctx, **shape), 5)
    t0 = time.perf_counter()
    for _ in range(10):
        lv.price_and_grad(s, 100.0, strikes, mats, P, N, wl.seed, ctx=ctx, **shape)
    mshb = (time.perf_counter() - t0) * 1e3 / 10
    v["fp32_host_buffers_pcie"] = {"ms_per_step": mshb, "value": P * N / (mshb * 1e-3)}
    res["variants"] = v
    res["accuracy"] = {"fp32_vs_fp64_gpu_price_abs": float(abs(p32[0] - p64[0])),
                       "fp32_vs_fp64_gpu_max_bucket_err_rel_maxg": float(np.abs(g32 - g64).max() / gscale),
                       "price": float(p32[0]), "stderr": float(se32[0]),
                       "fp32_speedup_over_fp64": float(ms64 / ms)}
    return wl.name, res


def book64(lv, W, ctx, dev):
    """64 calls/puts of uneven maturity on 2^20 shared paths: the fused persistent
    (checkpointed) kernel captured in a hipGraph, and the stored-state pair."""
    import torch
    wl = W.book_60x30()
    s, b = wl.surface, wl.book
    sig = torch.tensor(s.sigma, dtype=torch.float64, device=dev)
    out = {"options": b.n}
    for name, opts in (("checkpoint_graph", dict(adjoint="checkpoint", use_graph=True)),
                       ("stored_graph", dict(adjoint="stored", use_graph=True)),
                       ("stored_eager", dict(adjoint="stored"))):
        kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, is_put=b.is_put, weights=b.weight, ctx=ctx,
                  autotune=True, **opts)
        o = lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, wl.seed, **kw)
        f = lambda: lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, wl.seed,
                                          out=o, **kw)
        settle(f, 10)
        ms = best_of(f, 20)
        out[name] = {"ms_per_step": ms, "value": wl.n_paths * wl.n_steps / (ms * 1e-3),
                     "graph_replayed": bool(ctx.run_info()["graph_replayed"])}
    out["per_option_grids"] = per_option_cost(lv, wl, sig, ctx)
    return wl.name, out


def per_option_cost(lv, wl, sig, ctx):
    """Every option's own grid (64 grids) from one stored forward: the reverse sweep
    that serves up to 8 options at a time, against one reverse pass per option (a
    one-hot cotangent each) on the same stored states."""
    import numpy as np
    import torch
    s, b = wl.surface, wl.book
    P, N = wl.n_paths, wl.n_steps
    kw = dict(spot_axis=s.spot_axis, time_axis=s.time_axis, is_put=b.is_put, ctx=ctx)
    one_sweep = lambda: lv.per_option_grads_dev(sig, 100.0, b.strike, b.maturity, P, N, wl.seed, **kw)
    res = one_sweep()
    settle(one_sweep, 3)
    ms_sweep = best_of(one_sweep, 5)
    _, _, states = lv.forward_dev(sig, 100.0, b.strike, b.maturity, P, N, wl.seed, **kw)
    eye = torch.eye(b.n, dtype=torch.float64, device=sig.device)

    def passes():
        lv.forward_dev(sig, 100.0, b.strike, b.maturity, P, N, wl.seed, states=states, **kw)
        return [lv.backward_dev(sig, 100.0, b.strike, b.maturity, P, N, wl.seed, states, eye[k], **kw)[0]
                for k in range(b.n)]

    g_passes = passes()
    settle(passes, 2)
    ms_passes = best_of(passes, 2)
    g_sweep = res[2].cpu().numpy()
    diff = max(float(np.abs(g_sweep[k] - g_passes[k].cpu().numpy()).max() / max(np.abs(g_sweep[k]).max(), 1e-300))
               for k in range(b.n))
    del states
    torch.cuda.empty_cache()
    return {"options": b.n, "ms_forward_and_sweeps_of_up_to_8": ms_sweep,
            "ms_forward_and_one_pass_per_option": ms_passes, "speedup": ms_passes / ms_sweep,
            "max_grid_diff_rel_maxg_k": diff}


def bs_call_and_vega(spot, strike, sigma, T):
    """Black-Scholes call price and vega at zero rates."""
    v = sigma * math.sqrt(T)
    d1 = math.log(spot / strike) / v + 0.5 * v
    N = lambda x: 0.5 * (1.0 + math.erf(x / math.sqrt(2.0)))
    price = spot * N(d1) - strike * N(d1 - v)
    vega = spot * math.exp(-0.5 * d1 * d1) / math.sqrt(2.0 * math.pi) * math.sqrt(T)
    return price, vega


def precision_study(lv, W, ctx):
    """2^22 paths x 52 steps on the 21 x 13 surface and on a flat 0.2 one: FP32 against
    the all-FP64 GPU variant on the same streams; the flat case also against the
    Black-Scholes price and vega (log-Euler is exact in law for a flat vol, and the sum
    of the grid gradient is the sensitivity to a parallel shift of the surface).  The
    comparison with the FP64 CPU oracle is in the test-suite."""
    import numpy as np
    res = {}
    for flat in (False, True):
        wl = W.precision_study(flat)
        s, b = wl.surface, wl.book
        out = {}
        for prec in (32, 64):
            p, se, g, d = lv.price_and_grad(s, 100.0, b.strike, b.maturity, wl.n_paths, wl.n_steps, 0,
                                            precision=prec, ctx=ctx)
            out[prec] = (p[0], se[0], g)
        gm = np.abs(out[64][2]).max()
        rec = {"fp32_vs_fp64_price_abs": float(abs(out[32][0] - out[64][0])),
               "fp32_vs_fp64_max_bucket_err_rel_maxg": float(np.abs(out[32][2] - out[64][2]).max() / gm),
               "price": float(out[32][0]), "stderr": float(out[32][1]), "sum_grad": float(out[32][2].sum())}
        if flat:
            bs, vega = bs_call_and_vega(100.0, 100.0, 0.2, 1.0)
            rec["black_scholes"] = {"price": bs, "vega": vega,
                                    "fp32_price_minus_bs_over_stderr": (rec["price"] - bs) / rec["stderr"],
                                    "fp32_sum_grad_over_vega": rec["sum_grad"] / vega}
        res[wl.name] = rec
    return res


def cpu_threads():
    info = cpu_info()
    n = info["affinity"] or 1
    if info["cgroup_cpus"]:
        n = min(n, max(1, int(math.ceil(info["cgroup_cpus"]))))
    return n


def cpu_baseline(W, budget_s=12.0):
    """The oracle as it stands on the host: the headline workload's first surface on a
    bounded sample of its paths, all usable host threads, and one thread."""
    import oracle
    o = oracle.default()
    wl = W.surface_batch(1)
    s, b, N = wl.surface, wl.book, wl.n_steps
    threads = cpu_threads()

    def rate(n_paths, n_threads):
        t0 = time.perf_counter()
        o.price_and_grad(s, b, n_paths, N, wl.seed, n_threads=n_threads)
        return n_paths * N / (time.perf_counter() - t0)

    probe = 1 << 14
    r = rate(probe, threads)
    sample = max(probe, int(r * budget_s / N) // 4096 * 4096)
    r = rate(sample, threads)
    r1_sample = max(4096, int(rate(4096, 1) * budget_s / 4 / N) // 4096 * 4096)
    r1 = rate(r1_sample, 1)
    info = cpu_info()
    return {"value": r, "unit": "path-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample} paths x {N} steps of surface 1 of {wl.name}, FP64, price + grid adjoint "
                      f"(the batch's 32 surfaces would take 32 x as long)",
            "one_thread": {"value": r1, "sample": f"{r1_sample} paths x {N} steps"},
            "host": info}


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for {args.gpus}); across GPUs the path "
              "would shard by Philox path range (or by surface), each GPU sweeping its own paths",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2002_02481_amd as lv
    import workloads as W

    dev = torch.device("cuda:0")
    ctx = lv.Context(0)
    if args.only_call_60x30:
        print(json.dumps(call_60x30_fixed(lv, W, ctx, dev, args)), flush=True)
        return
    if args.tuning and os.path.exists(args.tuning):
        ctx.load_tuning(args.tuning)
    result, h = headline(lv, W, ctx, args)
    if not args.no_variants:
        fp64, acc = headline_fp64(lv, W, ctx, h, args)
        result["variants"] = {"fp64_gpu": fp64, "fp32_stored_states": headline_stored(lv, ctx, h)}
        acc["fp32_speedup_over_fp64_at_fixed_error"] = fp64["ms_per_step"] / result["ms_per_step"]
        result["accuracy"] = acc
        del h
        gc.collect()
        torch.cuda.empty_cache()
        w = {}
        name, r = call_60x30(lv, W, ctx, dev)
        w[name] = r
        name, r = book64(lv, W, ctx, dev)
        w[name] = r
        result["workloads"] = w
        result["precision_study"] = precision_study(lv, W, ctx)
    if args.tuning:
        ctx.save_tuning(args.tuning)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
