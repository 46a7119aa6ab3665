"""Throughput of rotational OMP encoding on one MI355X.

A step is one pass of the whole coding path over the batch: rsc_project (hat
coordinates) then rsc_omp_encode (K pursuit steps), inputs resident in HBM.
Default workload: 1,000,000 synthetic 11x11 patches, each 1-4 atoms of a random
unit-norm 64-atom dictionary at continuous angles with Laplace(0,1) weights plus
N(0, 0.05^2) noise; K=4 atoms per patch over R=64 angles.

Prints one JSON line.  The CPU baseline leg times the FP64 reference on a
bounded sample of the same workload and checks the device codes of that sample
against it (selection match and MSE).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1806_04374_amd import workloads as wl  # noqa: E402

METRIC = "patches encoded/sec (rotational OMP, K atoms, R angles) at matched MSE; p50/p99"
FP32_MFMA_PEAK = 157.3e12
HALF_MFMA_PEAK = 2.5e15          # dense BF16 / FP16 matrix peak
DTYPE = {"fp32": "f32", "bf16": "bf16 (FP32 accumulation, FP32 re-score)",
         "fp16": "f16 (FP32 accumulation, FP32 re-score)"}

# HBM bytes per encoder launch from rocprofv3 FETCH_SIZE and WRITE_SIZE counters, each
# scaled by the factor a plain 1 GiB copy gives (reads x2.0, writes x1.0), measured on the
# same kernel and workload (profiles/encode32_scale-fp32_counters.md and
# profiles/encode16_ragged-images_kernel_trace.md).  Valid for the encoder as of those
# counter runs; a workload missing here reports null.
TRAFFIC = {
    "scale-fp32": {"read": 226.9e6, "write": 55.1e6},      # algorithmic 220.0e6 / 52.0e6
    "ragged-images": {"read": 12.95e9, "write": 2.222e9},  # algorithmic 12.21e9 / 2.21e9
    "rotate-steer-11": {"read": 880.1e6, "write": 880.0e6},  # algorithmic 880e6 / 880e6 (4M x 55 x 4 B)
}


def traffic(name: str):
    t = TRAFFIC.get(name)
    return None if t is None else t["read"] + t["write"]


def encode_flops_per_patch(M: int, R: int, S: int, T: int, K: int, split: bool = False) -> float:
    """Flops of the pursuit for one patch doing all K steps.

    Correlation (per step): per-harmonic inner products 2*M*S*(1+4T) plus the angle DFT
    2*M*R*(2T+1).  With split=True the DFT is counted as the FP32 encoder computes it for
    even R: split once by harmonic parity, the even and odd partial sums are formed for R/2
    angle rows only, M*R*(2T+1).  Least squares and residual (step k): 2*(2*k*B + k^2).
    """
    B = S * (2 * T + 1)
    dft = 2.0 * M * R * (2 * T + 1) * (0.5 if split else 1.0)
    corr = 2.0 * M * S * (1 + 4 * T) + dft
    ls = sum(2.0 * (2 * k * B + k * k) for k in range(1, K + 1))
    return K * corr + ls


def encoder_roofline(h, prec: str, M: int, R: int, S: int, T: int, K: int, P: int, enc_s: float,
                     traffic_bytes=None) -> dict:
    """Roofline of one encoder launch over P patches that took enc_s seconds.

    frac counts the arithmetic the encoder itself performs: the FP32 encoder splits the
    angle DFT by harmonic parity for even R; the 16-bit encoder forms the whole DFT in 16-bit
    (its FP32 re-score of candidates is data-dependent and not counted).  Beside it: the same
    work with the direct R-angle DFT (what the split saves is counted as if done), and the
    matrix-core work actually executed (padding and recomputation included).
    """
    from paper_1806_04374_amd import rsc
    split = prec == "fp32" and R % 2 == 0
    own = encode_flops_per_patch(M, R, S, T, K, split=split) * P
    direct = encode_flops_per_patch(M, R, S, T, K, split=False) * P
    tile_used, mfma_pp = rsc.rsc_encode_info(h, K)
    peak = FP32_MFMA_PEAK if prec == "fp32" else HALF_MFMA_PEAK
    out = {"kernel": "encode_kernel" if prec == "fp32" else "encode_lp_kernel", "bound": "mfma",
           "achieved": own / enc_s / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s", "frac": own / enc_s / peak,
           "traffic": traffic_bytes, "algorithmic_flops_per_launch": own, "dft_split": split,
           "launch_ms": enc_s * 1e3,
           "frac_direct_dft_equivalent": direct / enc_s / peak,
           "executed_mfma_tflops": mfma_pp * P / enc_s / 1e12, "executed_mfma_frac": mfma_pp * P / enc_s / peak,
           "tile": tile_used}
    if prec != "fp32":
        # the 16-bit matrix work is a small part of the launch: the per-atom maxima over the
        # angles (vector instructions) and the FP32 re-score of candidates bound it
        out["limited_by"] = "vector issue (per-atom angle maxima) and the FP32 re-score, not the 16-bit matrix peak"
    return out


def make_inputs(h, w, P, dev):
    """Synthesize the workload's patches on the device from the seeded draws."""
    import torch
    from paper_1806_04374_amd import rsc
    g = w["geom"]
    X = torch.empty((P, g.N, g.N), dtype=torch.float32, device=dev)
    step = 1 << 18
    for lo in range(0, P, step):
        n = min(step, P - lo)
        if w["name"] == "small-fp32":
            _, d = wl.small_draw(P=n, start=lo)
        else:
            _, d = wl.scale_draw(P=n, start=lo)
        rsc.rsc_synthesize(h, torch.from_numpy(d.atom.astype(np.int32)).to(dev),
                           torch.from_numpy(d.angle.astype(np.float32)).to(dev),
                           torch.from_numpy(d.weight.astype(np.float32)).to(dev),
                           torch.from_numpy(d.noise.astype(np.float32)).to(dev), out=X[lo:lo + n])
    torch.cuda.synchronize()
    return X


def host_info() -> dict:
    """CPU model and logical core count of the host the reference is timed on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu": model, "nproc": os.cpu_count()}


def oracle_rate_one_thread(run, X, target_s: float) -> dict:
    """The reference's rate with its BLAS pools held to one thread, on a prefix of X sized
    from a 1,024-patch pilot to take about target_s seconds."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        n0 = min(1024, len(X))
        t0 = time.perf_counter()
        run(X[:n0].astype(np.float64))
        dt0 = time.perf_counter() - t0
        n = int(min(len(X), max(n0, n0 * target_s / max(dt0, 1e-3))))
        t0 = time.perf_counter()
        run(X[:n].astype(np.float64))
        dt = time.perf_counter() - t0
    return {"value": n / dt, "cores": 1, "sample": f"first {n} patches of the same sample ({dt:.1f} s)"}


def cpu_baseline(h, w, D, target_s: float, dev):
    """Time the FP64 reference (as it stands) on a bounded sample of the workload."""
    import torch
    from threadpoolctl import threadpool_info
    from oracle import rsc_oracle as orc
    from paper_1806_04374_amd import rsc
    g = w["geom"]
    basis = orc.build_basis(g.N, g.S, g.T)

    def sample(n):
        if w["name"] == "small-fp32":
            _, d = wl.small_draw(P=n)
        else:
            _, d = wl.scale_draw(P=n)
        return orc.synthesize(basis, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32)

    # the sample is sized from a pilot of a few thousand patches: a smaller pilot is dominated
    # by the reference's fixed costs and would size the sample well short of target_s
    n0 = 2048
    X0 = sample(n0)
    t0 = time.perf_counter()
    orc.encode(basis, D, w["R"], X0.astype(np.float64), w["K"])
    dt0 = time.perf_counter() - t0
    n = int(min(200_000, max(n0, n0 * target_s / max(dt0, 1e-3))))
    X = sample(n)
    t0 = time.perf_counter()
    _, code = orc.encode(basis, D, w["R"], X.astype(np.float64), w["K"])
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    one = oracle_rate_one_thread(lambda Xs: orc.encode(basis, D, w["R"], Xs, w["K"]), X, target_s=8.0)
    ref = {"X": X, "code": code, "mse": orc.mse(basis, X, orc.reconstruct(basis, D, w["R"], code)),
           "basis": basis}
    return {
        "value": n / dt, "unit": "patches/s", "cores": int(threads), "kind": "oracle",
        "sample": f"first {n} patches of the same workload (FP64 reference, {dt:.1f} s)",
        "one_thread": one, "host": host_info(),
        "check": device_check(h, ref, D, w["R"], w["K"], dev),
    }, ref


def device_check(h, ref, D, R, K, dev) -> dict:
    """Device codes of the reference's sample: selection match, coefficient error of the
    matched patches and matched MSE against the FP64 reference."""
    import torch
    from oracle import rsc_oracle as orc
    from paper_1806_04374_amd import rsc
    from tests.parity import compare_codes
    X, code, basis = ref["X"], ref["code"], ref["basis"]
    xh = rsc.rsc_project(h, torch.from_numpy(X).to(dev))
    atom, angle, coef, _ = rsc.rsc_omp_encode(h, xh, K)
    rec = rsc.rsc_reconstruct(h, atom, angle, coef)
    torch.cuda.synchronize()
    rep = compare_codes(atom.cpu().numpy(), angle.cpu().numpy(), coef.cpu().numpy(), code)
    mse_dev = orc.mse(basis, X, rec.cpu().numpy().astype(np.float64))
    # the floor under any code's MSE: the part of the patches outside span(Phi) (Sec. III-A)
    span = orc.span_error(basis, X.astype(np.float64))
    return {"patches": int(len(X)), "selection_match": rep.match_rate, "coef_rel_err_max": rep.coef_err_max,
            "coef_bad": rep.coef_bad, "mse_device": mse_dev, "mse_oracle": ref["mse"],
            "mse_rel_diff": abs(mse_dev - ref["mse"]) / ref["mse"], "span_error": span}


def run_ragged(args, dev):
    """256 texture images of uneven sizes; all stride-1 15x15 windows, K=6, R=64, M=128.

    Inputs are synthesized on the device from the seeded stamp draws.  One step =
    one replay of a HIP graph holding the image projection and the encoder.
    """
    import torch
    from paper_1806_04374_amd import autotune, rsc
    w = wl.RAGGED
    g = w["geom"]
    K = w["K"]
    D = wl.draw_dictionary(w["M"], g.B)
    h = rsc.rsc_create(g.N, g.S, g.T, prec=args.prec)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), w["R"])
    draws = wl.ragged_draws(args.images or None)
    batch = rsc.ImageBatch([(d.H, d.W) for d in draws], g.N, dev)
    pix = torch.from_numpy(np.concatenate([d.noise.ravel() for d in draws]).astype(np.float32)).to(dev)
    cat = lambda f, dt: torch.from_numpy(np.concatenate([f(d) for d in draws]).astype(dt)).to(dev)
    rsc.rsc_synthesize_images(
        h, batch, cat(lambda d: d.atom, np.int32), cat(lambda d: d.angle, np.float32),
        cat(lambda d: d.amplitude, np.float32),
        cat(lambda d: d.centre.reshape(-1, 2), np.int32).reshape(-1, 2).contiguous(),
        torch.from_numpy(np.concatenate([np.full(len(d.atom), i) for i, d in enumerate(draws)])
                         .astype(np.int32)).to(dev),
        pix)
    n_stamps = int(sum(len(d.atom) for d in draws))
    del draws
    P = batch.P_total
    xh = torch.empty((P, g.B), dtype=torch.float32, device=dev)
    outs = (torch.empty((P, K), dtype=torch.int32, device=dev), torch.empty((P, K), dtype=torch.int32, device=dev),
            torch.empty((P, K), dtype=torch.float32, device=dev), torch.empty((P,), dtype=torch.float32, device=dev))
    rsc.rsc_project_images(h, pix, batch, xhat=xh)
    torch.cuda.synchronize()
    tuned = autotune.tune(h, xh[: min(P, 1 << 18)], K, reps=3)

    def step(stream=None):
        rsc.rsc_project_images(h, pix, batch, xhat=xh, stream=stream)
        rsc.rsc_omp_encode(h, xh, K, out=outs, stream=stream)

    step()
    torch.cuda.synchronize()
    cs = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=cs):
        step(stream=cs)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        graph.replay()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])
    # kernel durations from eager launches with events on the launch stream
    kp, ke = [], []
    for _ in range(3):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        rsc.rsc_project_images(h, pix, batch, xhat=xh, stream=stream)
        e1.record(stream)
        rsc.rsc_omp_encode(h, xh, K, out=outs, stream=stream)
        e2.record(stream)
        torch.cuda.synchronize()
        kp.append(e0.elapsed_time(e1))
        ke.append(e1.elapsed_time(e2))
    ms = wall * 1e3 / args.steps
    out = {
        "metric": METRIC, "value": P / (ms * 1e-3), "unit": "patches/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "p50_ms": float(np.percentile(step_ms, 50)), "p99_ms": float(np.percentile(step_ms, 99)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.prec],
        "data": "synthetic",
        "config": {"workload": f"{w['name']}: {batch.n} images, sides log-uniform {w['side']}, "
                               f"{P} 15x15 windows, M={w['M']}, K={K}, R={w['R']}, one HIP graph per step",
                   "P": P, "images": batch.n, "stamps": n_stamps, "N": g.N, "S": g.S, "T": g.T,
                   "M": w["M"], "K": K, "R": w["R"], "launch": {k: tuned[k] for k in ("tile", "blocks_per_cu")},
                   "precision": args.prec},
        "autotune": tuned,
        "kernels_ms": {"project_images_mean": float(np.mean(kp)), "encode_mean": float(np.mean(ke))},
        "roofline": encoder_roofline(h, args.prec, w["M"], w["R"], g.S, g.T, K, P, np.mean(ke) * 1e-3,
                                     traffic(w["name"]) if args.prec == "fp32" else None),
        "cpu_baseline": None,
    }
    if args.prec != "fp32":
        out["precision_stats"] = rsc.rsc_precision_stats(h)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_ragged(h, w, D, args.cpu_seconds, dev)
    return out


def run_serving(args, dev):
    """Open-loop Poisson trace of encode requests (square images, sides log-uniform
    32..2048, 15x15 windows, M=128, K=6, R=64): continuous batching against
    one-request-at-a-time encoding of the same trace."""
    import torch
    from paper_1806_04374_amd import autotune, rsc, serve
    w = wl.SERVING
    g = w["geom"]
    K = w["K"]
    D = wl.draw_dictionary(w["M"], g.B)
    h = rsc.rsc_create(g.N, g.S, g.T, prec=args.prec)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), w["R"])
    arrivals, sides = wl.serving_trace(args.duration, args.rate)
    n = len(arrivals)
    sizes = sides.astype(np.int64) ** 2
    offs = np.concatenate([[0], np.cumsum(sizes)])
    host = torch.empty(int(offs[-1]), dtype=torch.float32, pin_memory=True)
    gen = torch.Generator(device=dev)
    t_gen = time.perf_counter()
    for i in range(n):           # request images: seeded device noise plus stamps
        if i % 500 == 0:
            print(f"serving: generating request {i}/{n}", file=sys.stderr, flush=True)
        sd = int(sides[i])
        gen.manual_seed(1_000_003 * 7 + i)
        pix = torch.randn(sd * sd, generator=gen, device=dev) * w["sigma"]
        centre, atom, angle, amp = wl.request_stamps(i, sd, sd, w["M"], w["density"])
        if len(atom):
            b1 = rsc.ImageBatch([(sd, sd)], g.N, dev)
            rsc.rsc_synthesize_images(
                h, b1, torch.from_numpy(atom.astype(np.int32)).to(dev),
                torch.from_numpy(angle.astype(np.float32)).to(dev), torch.from_numpy(amp.astype(np.float32)).to(dev),
                torch.from_numpy(centre.astype(np.int32)).to(dev), torch.zeros(len(atom), dtype=torch.int32, device=dev),
                pix)
        host[int(offs[i]):int(offs[i + 1])].copy_(pix)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    total_windows = int(((sides - g.N + 1).clip(0) ** 2).sum())
    # tune the encoder launch shape on one large image before the trace
    big = int(np.argmax(sides))
    b1 = rsc.ImageBatch([(int(sides[big]), int(sides[big]))], g.N, dev)
    xs = rsc.rsc_project_images(h, host[int(offs[big]):int(offs[big + 1])].to(dev), b1)
    tuned = autotune.tune(h, xs[: min(len(xs), 1 << 18)], K, reps=3)
    del xs

    def make(i):
        sd = int(sides[i])
        return serve.Request(i, float(arrivals[i]), host[int(offs[i]):int(offs[i + 1])].view(sd, sd), sd, sd)

    keep = lambda r: r.rid % 50 == 0
    if args.budget_gib > 0:
        budget = int(args.budget_gib * (1 << 30))
    else:
        # free HBM minus 8 GiB, less the step slots the backend allocates next to the pool
        free, _ = torch.cuda.mem_get_info()
        slot_bytes = 2 * args.step_windows * (g.B + 3 * K) * 4
        budget = max(1 << 30, free - (8 << 30) - slot_bytes)
    be = serve.DeviceBackend(h, K, budget, args.step_windows, keep_codes=keep)
    sch = serve.Scheduler(be, budget // 4, args.step_windows)
    served = [make(i) for i in range(n)]
    print(f"serving: replaying {n} requests over {args.duration:g} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    serve.replay(sch, served, realtime=True)
    span = time.perf_counter() - t0
    rep = serve.latency_report(served, warmup=5.0 if args.duration > 10 else 0.0)
    print(f"serving: continuous batching done in {span:.1f} s", file=sys.stderr, flush=True)
    # baseline: one request at a time through an FP32 handle, same trace
    if args.prec == "fp32":
        h_base = h
    else:
        h_base = rsc.rsc_create(g.N, g.S, g.T)
        rsc.rsc_set_dictionary(h_base, D.astype(np.float32), w["R"])
    if args.no_baseline:
        span1, rep1 = None, None
    else:
        alone = [make(i) for i in range(n)]
        t1 = time.perf_counter()
        serve.encode_one_at_a_time(h_base, K, alone, realtime=True, keep_codes=lambda r: False)
        span1 = time.perf_counter() - t1
        rep1 = serve.latency_report(alone, warmup=5.0 if args.duration > 10 else 0.0)
        print(f"serving: one-at-a-time baseline done in {span1:.1f} s", file=sys.stderr, flush=True)
    # batching invariance: sampled requests encoded alone (untimed) with the serving handle
    sampled = [make(r.rid) for r in served if r.codes is not None and r.windows]
    serve.encode_one_at_a_time(h, K, sampled, realtime=False)
    by_id = {r.rid: r for r in served}
    same = [all(np.array_equal(a, b) for a, b in zip(by_id[r.rid].codes, r.codes)) for r in sampled]
    out = {
        "metric": METRIC, "value": total_windows / span, "unit": "patches/s", "n_gpus": 1,
        "steps": sch.steps, "warmup": 0, "ms_per_step": span * 1e3 / max(sch.steps, 1),
        "p50_ms": rep.get("p50_s", float("nan")) * 1e3, "p99_ms": rep.get("p99_s", float("nan")) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.prec],
        "data": "synthetic",
        "config": {"workload": f"{w['name']}: Poisson {args.rate:g} req/s for {args.duration:g} s, square sides "
                               f"log-uniform {w['side']}, 15x15 windows, M={w['M']}, K={K}, R={w['R']}",
                   "requests": n, "windows": total_windows, "budget_gib": budget / (1 << 30),
                   "step_windows": args.step_windows, "launch": {k: tuned[k] for k in ("tile", "blocks_per_cu")},
                   "precision": args.prec},
        "serving": {"continuous_batching": dict(rep, makespan_s=span, patches_per_s=total_windows / span,
                                                max_active=sch.max_active, rejected=len(sch.rejected)),
                    "one_at_a_time": None if rep1 is None else dict(rep1, makespan_s=span1,
                                                                      patches_per_s=total_windows / span1),
                    "speedup_throughput": None if span1 is None else span1 / span,
                    "codes_identical_alone_vs_mix": f"{sum(same)}/{len(same)} sampled requests",
                    "offered_patches_per_s": total_windows / args.duration,
                    "input_generation_s": t_gen},
    }
    return out


def _timed_runs(h, X, xh, outs, K, n, warmup, stream):
    """n timed (project + encode) runs on one stream; per-run ms from HIP events."""
    import torch
    from paper_1806_04374_amd import rsc
    for _ in range(warmup):
        rsc.rsc_project(h, X, xh, stream=stream)
        rsc.rsc_omp_encode(h, xh, K, out=outs, stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record(stream)
        rsc.rsc_project(h, X, xh, stream=stream)
        rsc.rsc_omp_encode(h, xh, K, out=outs, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev])


def run_precision(args, dev):
    """FP32, BF16 and FP16 encoders on the same inputs: the small plain workload
    (2,000 patches, latency over >= 100 runs) and the 10^6-patch scale workload
    (throughput), with each form's codes checked against the FP64 reference in the
    CPU baseline leg."""
    import torch
    from paper_1806_04374_amd import rsc
    precs = ["fp32", "bf16", "fp16"]
    res = {"small": {}, "scale": {}}
    codes = {"small": {}, "scale": {}}
    inputs = {}
    stream = torch.cuda.current_stream()
    for name, w, runs in (("small", wl.SMALL, max(args.steps, 100)), ("scale", wl.SCALE, max(args.steps, 20))):
        g = w["geom"]
        K = w["K"]
        D = wl.draw_dictionary(w["M"], g.B)
        P = w["P"]
        X = None
        for prec in precs:
            h = rsc.rsc_create(g.N, g.S, g.T, prec=prec)
            rsc.rsc_set_dictionary(h, D.astype(np.float32), w["R"])
            if X is None:
                X = make_inputs(h, w, P, dev)
            xh = torch.empty((P, g.B), dtype=torch.float32, device=dev)
            outs = (torch.empty((P, K), dtype=torch.int32, device=dev), torch.empty((P, K), dtype=torch.int32, device=dev),
                    torch.empty((P, K), dtype=torch.float32, device=dev), torch.empty((P,), dtype=torch.float32, device=dev))
            ms = _timed_runs(h, X, xh, outs, K, runs, args.warmup, stream)
            p50 = float(np.percentile(ms, 50))
            res[name][prec] = {"p50_ms": p50, "p99_ms": float(np.percentile(ms, 99)), "runs": int(runs),
                               "patches_per_s_p50": P / (p50 * 1e-3)}
            if prec != "fp32":
                st = rsc.rsc_precision_stats(h)
                res[name][prec]["stats_per_run"] = {k: (v if k == "max_candidates" else v / (runs + args.warmup))
                                                    for k, v in st.items()}
            n_check = P if name == "small" else min(P, args.check_patches)
            rec = rsc.rsc_reconstruct(h, outs[0][:n_check], outs[1][:n_check], outs[2][:n_check])
            torch.cuda.synchronize()
            codes[name][prec] = tuple(t[:n_check].cpu().numpy() for t in outs[:3]) + (rec.cpu().numpy(),)
            h.close()
        inputs[name] = (w, D, X[: (w["P"] if name == "small" else min(w["P"], args.check_patches))].cpu().numpy())
        for prec in precs:
            res[name][prec]["speedup_vs_fp32"] = res[name]["fp32"]["p50_ms"] / res[name][prec]["p50_ms"]
    best = max(("bf16", "fp16"), key=lambda q: res["scale"][q]["patches_per_s_p50"])
    out = {
        "metric": METRIC, "value": res["scale"][best]["patches_per_s_p50"], "unit": "patches/s", "n_gpus": 1,
        "steps": int(res["scale"][best]["runs"]), "warmup": args.warmup, "ms_per_step": res["scale"][best]["p50_ms"],
        "p50_ms": res["scale"][best]["p50_ms"], "p99_ms": res["scale"][best]["p99_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[best], "data": "synthetic",
        "config": {"workload": f"precision forms: scale-fp32 inputs (10^6 11x11 patches, M=64, K=4, R=64) in "
                               f"{best}; small-fp32 inputs (2,000 patches, M=16, K=2, R=32) for latency",
                   "precision": best},
        "precision": res,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["errors_vs_oracle"] = cpu_baseline_precision(inputs, codes)
    print(json.dumps(out), flush=True)


def cpu_baseline_precision(inputs, codes):
    """FP64 reference on the small inputs (all 2,000) and a prefix of the scale inputs:
    its time, and each precision form's errors against it."""
    from threadpoolctl import threadpool_info
    from oracle import rsc_oracle as orc
    from tests.parity import compare_codes
    errors = {}
    timing = {}
    for name, (w, D, X) in inputs.items():
        g = w["geom"]
        basis = orc.build_basis(g.N, g.S, g.T)
        t0 = time.perf_counter()
        _, code = orc.encode(basis, D, w["R"], X.astype(np.float64), w["K"])
        timing[name] = (len(X), time.perf_counter() - t0)
        mse_ref = orc.mse(basis, X, orc.reconstruct(basis, D, w["R"], code))
        errors[name] = {}
        for prec, (atom, angle, coef, rec) in codes[name].items():
            rep = compare_codes(atom, angle, coef, code, 1e-4)
            errs = []
            for p in range(len(X)):
                o = {(int(a), int(r)): float(c) for a, r, c in zip(code.atom[p], code.angle[p], code.coef[p]) if a >= 0}
                gg = {(int(a), int(r)): float(c) for a, r, c in zip(atom[p], angle[p], coef[p]) if a >= 0}
                if set(o) == set(gg) and o:
                    sc = max(abs(v) for v in o.values())
                    errs.append(max(abs(gg[k] - v) / max(abs(v), 1e-3 * sc) for k, v in o.items()))
            errs = np.array(errs) if errs else np.zeros(1)
            mse_dev = orc.mse(basis, X, rec.astype(np.float64))
            errors[name][prec] = {"patches": len(X), "selection_match": rep.match_rate,
                                  "coef_rel_err_median": float(np.median(errs)),
                                  "coef_rel_err_p99": float(np.percentile(errs, 99)),
                                  "coef_rel_err_max": float(errs.max()),
                                  "mse_device": mse_dev, "mse_oracle": mse_ref,
                                  "mse_rel_diff": abs(mse_dev - mse_ref) / mse_ref}
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    n, dt = timing["scale"]
    base = {"value": n / dt, "unit": "patches/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {n} patches of the scale inputs (FP64 reference, {dt:.1f} s); "
                      f"small inputs: {timing['small'][0]} patches in {timing['small'][1]:.2f} s"}
    return base, errors


FP64_VECTOR_PEAK = 78.6e12


def run_rksvd(args, dev):
    """R-K-SVD learning on the scale workload: 10^6 patches, M=64, K=4, R=64, from the
    generating dictionary perturbed by N(0, 0.1^2) and renormalised.  Times whole
    iterations (pursuit + dictionary update + table rebuild) and their parts."""
    import torch
    from paper_1806_04374_amd import rsc
    w = wl.SCALE
    g = w["geom"]
    K, R = w["K"], w["R"]
    P = args.patches or w["P"]
    D = wl.draw_dictionary(w["M"], g.B)
    D0 = D + 0.1 * np.random.default_rng(31).standard_normal(D.shape)
    D0 = (D0 / np.linalg.norm(D0, axis=1, keepdims=True)).astype(np.float32)
    h = rsc.rsc_create(g.N, g.S, g.T, prec=args.prec)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), R)
    X = make_inputs(h, w, P, dev)
    xh = rsc.rsc_project(h, X)
    torch.cuda.synchronize()
    n_iter = max(args.steps, 1)
    # warm-up: one iteration (compiles nothing, but touches every kernel and allocation)
    rsc.rsc_rksvd_train(h, xh, D0, R, K, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Dn, codes, hist = rsc.rsc_rksvd_train(h, xh, D0, R, K, n_iter)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # one iteration's parts, events on the launch stream
    stream = torch.cuda.current_stream()
    rsc.rsc_set_dictionary(h, D0, R)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ws = torch.empty(rsc.rsc_rksvd_workspace_size(h, P, K), dtype=torch.uint8, device=dev)
    enc_ms, upd_ms = [], []
    for _ in range(3):
        ev[0].record(stream)
        atom, angle, coef, r2 = rsc.rsc_omp_encode(h, xh, K, stream=stream)
        ev[1].record(stream)
        d_new, usage, _ = rsc.rsc_rksvd_update(h, xh, atom, angle, coef, r2, workspace=ws, stream=stream)
        ev[2].record(stream)
        torch.cuda.synchronize()
        enc_ms.append(ev[0].elapsed_time(ev[1]))
        upd_ms.append(ev[1].elapsed_time(ev[2]))
    host = d_new.cpu().numpy()
    host /= np.linalg.norm(host, axis=1, keepdims=True)
    t1 = time.perf_counter()
    rsc.rsc_set_dictionary(h, host, R)
    load_ms = (time.perf_counter() - t1) * 1e3
    pairs = int((usage.cpu().numpy()).sum())
    # algorithmic FP64 work of the update: per (patch, atom) pair the outer product y y^T
    # (2 B^2) and the K - 1 steered atoms and the upright turn (about 6 B (K - 1) + 6 B)
    upd_flops = pairs * (2.0 * g.B * g.B + 6.0 * g.B * K)
    per_iter = wall / (n_iter + 1)          # n_iter updates and n_iter + 1 pursuits
    out = {
        "metric": "patches per second per R-K-SVD iteration (pursuit + dictionary update)",
        "value": P / per_iter, "unit": "patches/s", "n_gpus": 1, "steps": n_iter, "warmup": 1,
        "ms_per_step": per_iter * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.prec] + "; update in f64", "data": "synthetic",
        "config": {"workload": f"rksvd: {P} 11x11 patches, M={w['M']}, K={K}, R={R}, {n_iter} iterations "
                               "from the generating dictionary perturbed by N(0, 0.1^2)", "precision": args.prec},
        "parts_ms": {"pursuit": float(np.median(enc_ms)), "update": float(np.median(upd_ms)),
                     "dictionary_reload_host": load_ms},
        "coding_error_history": [float(x) for x in hist],
        "update_pairs": pairs,
        "roofline": {"kernel": "whole update (sort, rk_accum_kernel, reduce, rk_eig_kernel, reset)", "bound": "alu", "unit": "TFLOP/s",
                     "achieved": upd_flops / (np.median(upd_ms) * 1e-3) / 1e12, "peak": FP64_VECTOR_PEAK / 1e12,
                     "frac": upd_flops / (np.median(upd_ms) * 1e-3) / FP64_VECTOR_PEAK,
                     "algorithmic_flops_per_launch": upd_flops, "traffic": None},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_rksvd(w, D0, xh[: min(P, 2000)].cpu().numpy(), K, R)
    print(json.dumps(out), flush=True)


def cpu_baseline_rksvd(w, D0, X, K, R):
    """FP64 reference: one R-K-SVD iteration (pursuit + update) on the first patches."""
    from threadpoolctl import threadpool_info
    from oracle import rsc_oracle as orc
    g = w["geom"]
    t0 = time.perf_counter()
    orc.rksvd(D0.astype(np.float64), R, g.S, g.T, X.astype(np.float64), K, 1)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    # rksvd(n_iter=1) runs two pursuits and one update; count it as one iteration
    return {"value": len(X) / dt, "unit": "patches/s", "cores": int(threads), "kind": "oracle",
            "sample": f"one iteration (two pursuits and one update) on the first {len(X)} patches, {dt:.1f} s"}


def run_texture(args, dev):
    """Texture classification (Sec. III-B): 24 synthetic band-pass texture classes, 20
    upright 128x128 training images per class, 20 test images per class at each of 8
    rotations.  Setup (untimed): image draws uploaded, one R-K-SVD dictionary per class
    (M=100, K=1, R=64, from 4,000 windows per training image), training histograms.
    One timed step = one test rotation: projection of every window of its 480 images,
    labels against all 24 dictionaries, histograms and chi^2 1-NN."""
    import torch
    from paper_1806_04374_amd import rsc
    from paper_1806_04374_amd import texture as tx
    w = wl.TEXTURE
    g = w["geom"]
    C, side, K, R = w["C"], w["side"], w["K"], w["R"]
    n_train = w["n_train"]
    n_test = args.images or w["n_test"]
    rots = w["test_rot_deg"]
    annular = args.basis == "annular"
    if annular and args.prec != "fp32":
        sys.exit("the annular basis is FP32 only")
    t_setup = time.perf_counter()
    proj = rsc.rsc_create_annular(g.N) if annular else rsc.rsc_create(g.N, g.S, g.T)
    tr_images = [wl.draw_texture_image(c, i, side, w["sigma"]) for c in range(C) for i in range(n_train)]
    tb, tpix = tx.upload_batch(tr_images, g.N, dev)
    del tr_images
    xh_train = rsc.rsc_project_images(proj, tpix, tb)
    clf, learn_s = texture_learn(args, dev, xh_train, tb, R)
    torch.cuda.synchronize()
    print(f"texture: setup {time.perf_counter() - t_setup:.1f} s (learning {learn_s:.1f} s)", file=sys.stderr,
          flush=True)
    train_class = clf.train_class
    # test batches, one per rotation
    batches = []
    for j, deg in enumerate(rots):
        te = [wl.draw_texture_image(c, n_train + j * n_test + i, side, w["sigma"], np.deg2rad(deg))
              for c in range(C) for i in range(n_test)]
        b, pix = tx.upload_batch(te, g.N, dev)
        batches.append((b, pix, tx.window_offsets(b, dev)))
    P = batches[0][0].P_total
    xh = torch.empty((P, proj.B), dtype=torch.float32, device=dev)
    ws = torch.empty(rsc.rsc_classify_workspace_size(P, K), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    test_class = np.repeat(np.arange(C), n_test)

    def step(j, ev=None):
        b, pix, off = batches[j]
        if ev:
            ev[0].record(stream)
        rsc.rsc_project_images(proj, pix, b, xhat=xh, stream=stream)
        if ev:
            ev[1].record(stream)
        label, _ = rsc.rsc_classify(clf.handles, xh, K, workspace=ws, stream=stream)
        if ev:
            ev[2].record(stream)
        hist = rsc.rsc_label_histogram(label, off, C, stream=stream)
        nearest, _ = clf.predict(hist, stream=stream)
        if ev:
            ev[3].record(stream)
        return nearest

    for _ in range(args.warmup):
        step(0)
    torch.cuda.synchronize()
    n_steps = args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(n_steps)]
    preds = []
    t0 = time.perf_counter()
    for k in range(n_steps):
        preds.append(step(k % len(rots), evs[k]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    acc = {}
    for k, p in enumerate(preds):
        acc.setdefault(rots[k % len(rots)], float(np.mean(train_class[p.cpu().numpy()] == test_class)))
    parts = {"project": [], "classify": [], "histogram_nn": []}
    for e in evs:
        parts["project"].append(e[0].elapsed_time(e[1]))
        parts["classify"].append(e[1].elapsed_time(e[2]))
        parts["histogram_nn"].append(e[2].elapsed_time(e[3]))
    # dominant kernel: the encoder, C launches per step (events around rsc_classify)
    cls_ms = float(np.median(parts["classify"]))
    if annular:
        Sk = [sum(1 for t in proj.Ts if t >= k) for k in range(max(proj.Ts) + 1)]
        flops = annular_flops_per_patch(Sk, w["M"], R, K) * P * C
    else:
        flops = encode_flops_per_patch(w["M"], R, g.S, g.T, K, split=args.prec == "fp32" and R % 2 == 0) * P * C
    peak = FP32_MFMA_PEAK if args.prec == "fp32" else HALF_MFMA_PEAK
    images = batches[0][0].n
    out = {
        "metric": "texture windows classified per second (each coded against all C class dictionaries)",
        "value": P * n_steps / wall, "unit": "windows/s", "n_gpus": 1, "steps": n_steps, "warmup": args.warmup,
        "ms_per_step": wall / n_steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.prec], "data": "synthetic",
        "config": {"workload": f"texture: {C} band-pass classes, {images} test images of {side}x{side} per step "
                               f"({P} 15x15 windows), one step per rotation {list(rots)} deg; R-K-SVD "
                               f"dictionaries M={w['M']}, K={K}, R={R} learned from {n_train} upright images "
                               "per class", "precision": args.prec,
                   "basis": (f"the paper's annular basis, B={proj.B}" if annular
                             else f"Gaussian profiles S={g.S}, T={g.T}, B={g.B}")},
        "images_per_s": images * n_steps / wall,
        "accuracy": {"per_rotation_deg": {str(k): v for k, v in acc.items()}, "mean": float(np.mean(list(acc.values())))},
        "parts_ms": {k: float(np.median(v)) for k, v in parts.items()},
        "learning_s": learn_s,
        "roofline": {"kernel": f"encoder x {C} classes (rsc_classify)", "bound": "mfma",
                     "achieved": flops / (cls_ms * 1e-3) / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": flops / (cls_ms * 1e-3) / peak, "algorithmic_flops_per_launch": flops / C,
                     "traffic": None},
        "cpu_baseline": None,
    }
    del xh_train
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_texture(clf, proj, xh, batches[0], args.cpu_seconds, dev)
    print(json.dumps(out), flush=True)
    clf.close()


def texture_learn(args, dev, xh_train, tb, R):
    """One dictionary per class from 4,000 random windows of each of its training images
    (R = 1: plain K-SVD), then the training histograms.  Returns (classifier, seconds)."""
    import torch
    from paper_1806_04374_amd import rsc
    from paper_1806_04374_amd import texture as tx
    w = wl.TEXTURE
    g = w["geom"]
    C, K, n_train = w["C"], w["K"], w["n_train"]
    rng = np.random.default_rng(7)
    per = int(tb.patches_per_image[0])
    cls_windows = []
    for c in range(C):
        idx = np.concatenate([(c * n_train + j) * per + np.sort(rng.choice(per, min(per, w["train_windows"]),
                                                                           replace=False))
                              for j in range(n_train)])
        cls_windows.append(xh_train.index_select(0, torch.from_numpy(idx).to(dev)).contiguous())
    clf = tx.TextureClassifier(g.N, g.S, g.T, R, K, prec=args.prec, annular=args.basis == "annular")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    clf.learn(cls_windows, w["M"], w["n_iter"])
    torch.cuda.synchronize()
    learn_s = time.perf_counter() - t0
    del cls_windows
    ws = torch.empty(rsc.rsc_classify_workspace_size(xh_train.shape[0], K), dtype=torch.uint8, device=dev)
    clf.fit(clf.features(xh_train, tx.window_offsets(tb, dev), workspace=ws), np.repeat(np.arange(C), n_train))
    return clf, learn_s


def annular_flops_per_patch(Sk, M: int, R: int, K: int) -> float:
    """Arithmetic of the pursuit on a ragged (annular) layout, one patch, all K steps: stage
    1 forms C_k over the Sk[k] annuli of harmonic k (2 Sk[0] flops for k = 0, 8 Sk[k] per
    complex product sum for k >= 1), the angle DFT split by parity (M R (2T + 1) for even
    R), and the least squares as for the grid."""
    T = len(Sk) - 1
    B = Sk[0] + 2 * sum(Sk[1:])
    stage1 = 2.0 * M * (Sk[0] + 4 * sum(Sk[1:]))
    dft = M * R * (2 * T + 1) * (1.0 if R % 2 == 0 else 2.0)
    ls = sum(2.0 * (2 * k * B + k * k) for k in range(1, K + 1))
    return K * (stage1 + dft) + ls


def annular_inputs(h, w, N, P, dev):
    """The scale workload's draws (1-4 atoms at continuous angles, Laplace weights,
    N(0, 0.05^2) noise) as N x N patches, synthesized on the device in the handle's basis."""
    import torch
    from paper_1806_04374_amd import rsc
    X = torch.empty((P, N, N), dtype=torch.float32, device=dev)
    step = 1 << 18
    for lo in range(0, P, step):
        n = min(step, P - lo)
        d = wl.draw_mixtures(n, N, w["M"], w["J"], w["sigma"], 0, lo)
        rsc.rsc_synthesize(h, torch.from_numpy(d.atom.astype(np.int32)).to(dev),
                           torch.from_numpy(d.angle.astype(np.float32)).to(dev),
                           torch.from_numpy(d.weight.astype(np.float32)).to(dev),
                           torch.from_numpy(d.noise.astype(np.float32)).to(dev), out=X[lo:lo + n])
    torch.cuda.synchronize()
    return X


def run_annular(args, dev):
    """The pursuit on the paper's annular basis (eq. (5)-(8)): the scale workload's draws
    (10^6 patches, 1-4 atoms at continuous angles, Laplace weights, N(0, 0.05^2) noise) at
    N = 11 (B = 81) or 15 (B = 153, --annular-n 15) with a 64-atom dictionary in the annular
    coordinates, K = 4, R = 64."""
    import torch
    from paper_1806_04374_amd import rsc
    w = wl.SCALE
    N, M, K, R = args.annular_n, w["M"], w["K"], w["R"]
    P = args.patches or w["P"]
    h = rsc.rsc_create_annular(N)
    D = wl.draw_dictionary(M, h.B, seed=7)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), R)
    X = make_inputs(h, w, P, dev) if N == 11 else annular_inputs(h, w, N, P, dev)
    xh = torch.empty((P, h.B), dtype=torch.float32, device=dev)
    outs = (torch.empty((P, K), dtype=torch.int32, device=dev), torch.empty((P, K), dtype=torch.int32, device=dev),
            torch.empty((P, K), dtype=torch.float32, device=dev), torch.empty((P,), dtype=torch.float32, device=dev))
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        rsc.rsc_project(h, X, xh, stream=stream)
        rsc.rsc_omp_encode(h, xh, K, out=outs, stream=stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b, c in ev:
        a.record(stream)
        rsc.rsc_project(h, X, xh, stream=stream)
        b.record(stream)
        rsc.rsc_omp_encode(h, xh, K, out=outs, stream=stream)
        c.record(stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    step_ms = np.array([a.elapsed_time(c) for a, _, c in ev])
    enc = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    Ts = h.Ts
    Sk = [sum(1 for t in Ts if t >= k) for k in range(max(Ts) + 1)]
    own = annular_flops_per_patch(Sk, M, R, K) * P
    tile_used, mfma_pp = rsc.rsc_encode_info(h, K)
    out = {
        "metric": METRIC, "value": P / (ms * 1e-3), "unit": "patches/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"annular: {P} {N}x{N} patches in the paper's annular basis (T_s = {Ts}, B = {h.B}), "
                               f"M={M}, K={K}, R={R}", "P": P, "N": N, "B": h.B, "M": M, "K": K, "R": R},
        "kernels_ms": {"project_mean": float(np.mean([a.elapsed_time(b) for a, b, _ in ev])), "encode_mean": enc},
        "roofline": {"kernel": "encode16_kernel (annular layout)", "bound": "mfma",
                     "achieved": own / (enc * 1e-3) / 1e12, "peak": FP32_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": own / (enc * 1e-3) / FP32_MFMA_PEAK, "algorithmic_flops_per_launch": own,
                     "executed_mfma_frac": mfma_pp * P / (enc * 1e-3) / FP32_MFMA_PEAK, "tile": tile_used,
                     "traffic": None},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_annular(h, w, D, args.cpu_seconds, dev)
    print(json.dumps(out), flush=True)


def cpu_baseline_annular(h, w, D, target_s, dev):
    """The FP64 reference on a prefix of the annular workload, and the device's codes of that
    prefix against it."""
    from threadpoolctl import threadpool_info
    from oracle import rsc_oracle as orc
    ab = orc.build_annular_basis(h.N)

    def sample(n):
        if h.N == 11:
            _, d = wl.scale_draw(P=n)
        else:
            d = wl.draw_mixtures(n, h.N, w["M"], w["J"], w["sigma"], 0, 0)
        return orc.synthesize(ab, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32)

    X0 = sample(128)
    t0 = time.perf_counter()
    orc.encode(ab, D, w["R"], X0.astype(np.float64), w["K"])
    dt0 = time.perf_counter() - t0
    n = int(min(100_000, max(128, 128 * target_s / max(dt0, 1e-3))))
    X = sample(n)
    t0 = time.perf_counter()
    _, code = orc.encode(ab, D, w["R"], X.astype(np.float64), w["K"])
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    ref = {"X": X, "code": code, "mse": orc.mse(ab, X, orc.reconstruct(ab, D, w["R"], code)), "basis": ab}
    return {"value": n / dt, "unit": "patches/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {n} patches of the same workload (FP64 reference, {dt:.1f} s)", "host": host_info(),
            "check": device_check(h, ref, D, w["R"], w["K"], dev)}


def run_rotate(args, dev):
    """Rotation speed (Sec. III-C): random N x N patches turned by 100 + sqrt(2) degrees with
    the nearest and bicubic rotation matrices (R x) and by steering precomputed hat
    coordinates (S x_hat), at N = 11 and 15 and for the paper's 50,000 patches and a
    4,000,000-patch batch; also steering with the low-pass basis (T halved) and the full
    steering rotation (project, steer, synthesize).  Each method: median of 20 event-timed
    runs."""
    import torch
    from paper_1806_04374_amd import rsc
    theta = np.deg2rad(100 + np.sqrt(2))
    stream = torch.cuda.current_stream()
    reps = 20

    def timed(fn):
        for _ in range(3):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    results = {}
    for geom in (wl.GEOM11, wl.GEOM15):
        N = geom.N
        h = rsc.rsc_create(N, geom.S, geom.T)
        hl = rsc.rsc_create(N, geom.S, geom.T // 2)
        ha = rsc.rsc_create_annular(N)            # the paper's annular basis and its low-pass form
        hal = rsc.rsc_create_annular(N, lowpass=True)
        plans = {m: rsc.RotationPlan(N, theta, m) for m in ("nearest", "bicubic")}
        if N == 11:   # Phi S_theta Phi^+ as one operator on the matrix cores
            plans["steer_one_pass"] = rsc.RotationPlan.steer(h, theta)
        for P in (50_000, 4_000_000):
            rng = torch.Generator(device=dev)
            rng.manual_seed(P + N)
            X = torch.randn((P, N, N), generator=rng, device=dev, dtype=torch.float32)
            Y = torch.empty_like(X)
            xh = rsc.rsc_project(h, X)
            xo = torch.empty_like(xh)
            xl = rsc.rsc_project(hl, X)
            xlo = torch.empty_like(xl)
            r = {}
            for m, plan in plans.items():
                r[m] = timed(lambda: rsc.rsc_rotate_interp(plan, X, out=Y, stream=stream))
            r["steer"] = timed(lambda: rsc.rsc_steer(h, xh, theta, out=xo, stream=stream))
            r["copy_of_xhat"] = timed(lambda: xo.copy_(xh))          # achievable-bandwidth reference
            r["steer_low"] = timed(lambda: rsc.rsc_steer(hl, xl, theta, out=xlo, stream=stream))
            r["steer_full"] = timed(lambda: rsc.rsc_synthesize_hat(
                h, rsc.rsc_steer(h, rsc.rsc_project(h, X, xh, stream=stream), theta, out=xo, stream=stream),
                out=Y, stream=stream))
            del xl, xlo
            xa = rsc.rsc_project(ha, X)
            xao = torch.empty_like(xa)
            r["steer_annular"] = timed(lambda: rsc.rsc_steer(ha, xa, theta, out=xao, stream=stream))
            del xa, xao
            xa = rsc.rsc_project(hal, X)
            xao = torch.empty_like(xa)
            r["steer_annular_low"] = timed(lambda: rsc.rsc_steer(hal, xa, theta, out=xao, stream=stream))
            del xa, xao
            results[f"N{N}_P{P}"] = {
                "ms": r, "B": h.B, "B_low": hl.B, "B_annular": ha.B, "B_annular_low": hal.B,
                "bicubic_over_steer_annular": r["bicubic"] / r["steer_annular"],
                "steer_annular_GBps": 2 * 4 * ha.B * P / (r["steer_annular"] * 1e-3) / 1e9,
                "bicubic_over_steer": r["bicubic"] / r["steer"], "nearest_over_steer": r["nearest"] / r["steer"],
                "steer_GBps": 2 * 4 * h.B * P / (r["steer"] * 1e-3) / 1e9,
                "bicubic_GBps": 2 * 4 * N * N * P / (r["bicubic"] * 1e-3) / 1e9,
                "copy_GBps": 2 * 4 * h.B * P / (r["copy_of_xhat"] * 1e-3) / 1e9,
            }
            print(f"rotate N={N} P={P}: {json.dumps(r)}", file=sys.stderr, flush=True)
            del X, Y, xh, xo
            torch.cuda.empty_cache()
        for plan in plans.values():
            plan.close()
        h.close()
        hl.close()
        ha.close()
        hal.close()
    main = results["N11_P4000000"]
    bytes_steer = 2 * 4 * 55 * 4_000_000
    out = {
        "metric": "patch rotations per second by steering hat coordinates (S x_hat), 100 + sqrt(2) degrees",
        "value": 4_000_000 / (main["ms"]["steer"] * 1e-3), "unit": "patches/s", "n_gpus": 1, "steps": reps,
        "warmup": 3, "ms_per_step": main["ms"]["steer"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "rotate: 4,000,000 random 11x11 patches (B = 55); also 50,000 (the paper's "
                               "count) and 15x15; nearest / bicubic rotation matrices, steering, low-pass "
                               "steering (T halved), steering in the paper's annular basis and its "
                               "low-pass form, full steering rotation"},
        "results": results,
        "roofline": {"kernel": "steer_stream_kernel", "bound": "hbm", "achieved": main["steer_GBps"], "peak": 8000.0,
                     "unit": "GB/s", "frac": main["steer_GBps"] / 8000.0, "traffic": traffic("rotate-steer-11"),
                     "algorithmic_bytes_per_launch": bytes_steer},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_rotate(theta, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline_rotate(theta, target_s):
    """FP64 reference: bicubic rotation matrix product and steering on 11x11 patches."""
    from threadpoolctl import threadpool_info
    from oracle import rsc_oracle as orc
    g = wl.GEOM11
    basis = orc.build_basis(g.N, g.S, g.T)
    n = 50_000
    X = np.random.default_rng(0).standard_normal((n, g.N, g.N))
    xh = orc.project(basis, X)
    t0 = time.perf_counter()
    orc.steer(xh, theta, g.S, g.T)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    orc.rotate_interp(X, theta, "bicubic")
    dtb = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": n / dt, "unit": "patches/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} random 11x11 patches: steering {dt:.2f} s; bicubic matrix product {dtb:.2f} s "
                      f"({n / dtb:.0f} patches/s)"}


def cpu_baseline_texture(clf, proj, xh, batch0, target_s, dev):
    """FP64 reference classifier (labels of windows against all class dictionaries) on the
    first windows of the first test batch; also the device labels of the same windows."""
    import torch
    from threadpoolctl import threadpool_info
    from oracle import rsc_oracle as orc
    from paper_1806_04374_amd import rsc
    w = wl.TEXTURE
    g = w["geom"]
    b, pix, _ = batch0
    rsc.rsc_project_images(proj, pix, b, xhat=xh)
    D = [d.astype(np.float64) for d in clf.dictionaries]
    if clf.annular:
        ab = orc.build_annular_basis(g.N)

        def classify(X):   # the reference classifier's rule with the annular basis' steering
            sse = np.stack([orc.omp(orc.augmented_dictionary_basis(ab, Dc, w["R"]), X, w["K"], Dc.shape[0]).resid2
                            for Dc in D], axis=1)
            return np.argmin(sse, axis=1), sse
    else:
        def classify(X):
            return orc.classify(D, w["R"], g.S, g.T, X, w["K"])
    n0 = 96
    X0 = xh[:n0].cpu().numpy().astype(np.float64)
    t0 = time.perf_counter()
    classify(X0)
    dt0 = time.perf_counter() - t0
    n = int(min(20_000, max(n0, n0 * target_s / max(dt0, 1e-3))))
    X = xh[:n].cpu().numpy().astype(np.float64)
    t0 = time.perf_counter()
    ref_label, ref_sse = classify(X)
    dt = time.perf_counter() - t0
    label, _ = rsc.rsc_classify(clf.handles, xh[:n].contiguous(), w["K"])
    torch.cuda.synchronize()
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": n / dt, "unit": "windows/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {n} windows of the first test batch against all {len(D)} dictionaries ({dt:.1f} s)",
            "check": {"label_match": float(np.mean(label.cpu().numpy() == ref_label))}}


def cpu_baseline_ragged(h, w, D, target_s, dev):
    """FP64 reference on windows of the first image (reference-synthesized pixels)."""
    import torch
    from threadpoolctl import threadpool_info
    from oracle import rsc_oracle as orc
    from paper_1806_04374_amd import rsc
    g = w["geom"]
    basis = orc.build_basis(g.N, g.S, g.T)
    d = wl.ragged_draws(1)[0]
    img = orc.synthesize_image(basis, D, d.H, d.W, d.centre, d.atom, d.angle, d.amplitude, d.noise).astype(np.float32)
    wins = orc.image_patches(img.astype(np.float64), g.N)
    t0 = time.perf_counter()
    orc.encode(basis, D, w["R"], wins[:64], w["K"])
    dt0 = time.perf_counter() - t0
    n = int(min(len(wins), max(64, 64 * target_s / max(dt0, 1e-3))))
    t0 = time.perf_counter()
    _, code = orc.encode(basis, D, w["R"], wins[:n], w["K"])
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    batch = rsc.ImageBatch([(d.H, d.W)], g.N, dev)
    xh = rsc.rsc_project_images(h, torch.from_numpy(img.ravel()).to(dev), batch)
    atom, angle, coef, _ = rsc.rsc_omp_encode(h, xh[:n].contiguous(), w["K"])
    torch.cuda.synchronize()
    a, r = atom.cpu().numpy(), angle.cpu().numpy()
    match = np.mean([{(x, y) for x, y in zip(a[p], r[p]) if x >= 0} ==
                     {(int(x), int(y)) for x, y in zip(code.atom[p], code.angle[p]) if x >= 0} for p in range(n)])
    return {"value": n / dt, "unit": "patches/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {n} windows of image 0 ({d.H}x{d.W}), FP64 reference, {dt:.1f} s",
            "check": {"selection_match": float(match)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=["scale", "small", "ragged", "serving", "precision", "rksvd", "texture", "rotate",
                                           "annular"],
                    default="scale")
    ap.add_argument("--check-patches", type=int, default=50_000,
                    help="precision: scale-workload patches checked against the reference")
    ap.add_argument("--duration", type=float, default=30.0, help="serving: trace length (s)")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: mean requests per second")
    ap.add_argument("--budget-gib", type=float, default=64.0,
                    help="serving: HBM budget for request pixels (<= 0: free HBM minus 8 GiB)")
    ap.add_argument("--no-baseline", action="store_true", help="serving: skip the one-at-a-time leg")
    ap.add_argument("--step-windows", type=int, default=1 << 22, help="serving: windows per device step")
    ap.add_argument("--images", type=int, default=0,
                    help="ragged: use the first n images; texture: test images per class and rotation (testing only)")
    ap.add_argument("--patches", type=int, default=0, help="override P (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="scale: skip the BF16 / FP16 forms and the small-workload latency")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tile", choices=["auto", "16", "32"], default="auto")
    ap.add_argument("--annular-n", type=int, choices=[11, 15], default=11,
                    help="annular: patch side (B = 81 or 153)")
    ap.add_argument("--basis", choices=["grid", "annular"], default="grid",
                    help="texture: the classes' basis (the paper's annular basis is FP32)")
    ap.add_argument("--prec", choices=["fp32", "bf16", "fp16"], default="fp32",
                    help="encoder correlation precision (16-bit forms re-score candidates in FP32)")
    ap.add_argument("--mode", choices=["encode", "copy"], default="encode",
                    help="copy: only a plain 1 GiB device copy, to calibrate byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU (asked for --gpus {args.gpus}); the coding path has no "
              "cross-GPU step: patches, images or requests shard over independent per-GPU processes.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1806_04374_amd import rsc
    dev = torch.device("cuda:0")
    if args.mode == "copy":
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                          "launches": 3}), flush=True)
        return
    if args.workload == "ragged":
        print(json.dumps(run_ragged(args, dev)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps(run_serving(args, dev)), flush=True)
        return
    if args.workload == "precision":
        run_precision(args, dev)
        return
    if args.workload == "rksvd":
        run_rksvd(args, dev)
        return
    if args.workload == "texture":
        run_texture(args, dev)
        return
    if args.workload == "rotate":
        run_rotate(args, dev)
        return
    if args.workload == "annular":
        run_annular(args, dev)
        return
    w = wl.SCALE if args.workload == "scale" else wl.SMALL
    g = w["geom"]
    P = args.patches or w["P"]
    D = wl.draw_dictionary(w["M"], g.B)
    h = rsc.rsc_create(g.N, g.S, g.T, prec=args.prec)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), w["R"])
    rsc.rsc_set_tile(h, args.tile)
    X = make_inputs(h, w, P, dev)
    K = w["K"]
    xh = torch.empty((P, g.B), dtype=torch.float32, device=dev)
    outs = (torch.empty((P, K), dtype=torch.int32, device=dev),
            torch.empty((P, K), dtype=torch.int32, device=dev),
            torch.empty((P, K), dtype=torch.float32, device=dev),
            torch.empty((P,), dtype=torch.float32, device=dev))
    stream = torch.cuda.current_stream()

    def step():
        rsc.rsc_project(h, X, xh, stream=stream)
        rsc.rsc_omp_encode(h, xh, K, out=outs, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s0, s1, s2 in ev:
        s0.record(stream)
        rsc.rsc_project(h, X, xh, stream=stream)
        s1.record(stream)
        rsc.rsc_omp_encode(h, xh, K, out=outs, stream=stream)
        s2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([a.elapsed_time(c) for a, _, c in ev])
    proj_ms = np.array([a.elapsed_time(b) for a, b, _ in ev])
    enc_ms = np.array([b.elapsed_time(c) for _, b, c in ev])
    ms = wall * 1e3 / args.steps
    out = {
        "metric": METRIC,
        "value": P / (ms * 1e-3),
        "unit": "patches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "patches_per_s_p50": P / (np.percentile(step_ms, 50) * 1e-3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.prec],
        "data": "synthetic",
        "config": {"workload": f"{w['name']}: {P} {g.N}x{g.N} patches, M={w['M']}, K={K}, R={w['R']}, "
                               f"S={g.S}, T={g.T}, B={g.B}",
                   "P": P, "N": g.N, "S": g.S, "T": g.T, "M": w["M"], "K": K, "R": w["R"],
                   "tile": args.tile, "precision": args.prec},
        "kernels_ms": {"project_mean": float(proj_ms.mean()), "encode_mean": float(enc_ms.mean())},
        "roofline": encoder_roofline(h, args.prec, w["M"], w["R"], g.S, g.T, K, P, enc_ms.mean() * 1e-3,
                                     traffic(w["name"]) if args.prec == "fp32" else None),
        "cpu_baseline": None,
    }
    if args.prec != "fp32":
        out["precision_stats"] = rsc.rsc_precision_stats(h)
    ref = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"], ref = cpu_baseline(h, w, D, args.cpu_seconds, dev)
    if w["name"] == "scale-fp32" and args.prec == "fp32" and not args.no_extras and not args.patches:
        out["precision_forms"] = precision_forms(D, w, X, ref, ms, args, dev)
        out["small_latency"] = small_latency(dev)
        del X, xh, outs
        out["ragged_batch"] = _extra(lambda: ragged_batch_summary(dev))
        out["serving_trace"] = _extra(lambda: serving_trace_summary(dev))
    print(json.dumps(out), flush=True)


def _extra(fn):
    """An extra section of the default line; a failure is reported in its place, so that the
    line still carries the headline measurement."""
    import torch
    try:
        return fn()
    except Exception as e:      # noqa: BLE001 -- reported in the JSON line
        return {"error": f"{type(e).__name__}: {e}"}
    finally:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


def ragged_batch_summary(dev) -> dict:
    """The ragged batch (256 images, all stride-1 15x15 windows, FP32) in the default line:
    two timed graph replays after one warm-up."""
    import types
    a = types.SimpleNamespace(prec="fp32", images=0, steps=2, warmup=1, no_cpu_baseline=True, cpu_seconds=0.0)
    r = run_ragged(a, dev)
    return {"workload": r["config"]["workload"], "windows_per_s": r["value"], "ms_per_step": r["ms_per_step"],
            "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"], "kernels_ms": r["kernels_ms"],
            "launch": r["config"]["launch"], "roofline": r["roofline"]}


def serving_trace_summary(dev) -> dict:
    """A short serving trace in the default line: Poisson 200 req/s for 4 s against the BF16
    server (HBM budget 64 GiB), latencies from arrival to codes on the host."""
    import types
    a = types.SimpleNamespace(prec="bf16", duration=4.0, rate=200.0, budget_gib=64.0, no_baseline=True,
                              step_windows=1 << 22)
    r = run_serving(a, dev)
    cb = r["serving"]["continuous_batching"]
    return {"workload": r["config"]["workload"], "precision": "bf16", "requests": r["config"]["requests"],
            "windows_per_s": r["value"], "offered_windows_per_s": r["serving"]["offered_patches_per_s"],
            "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"], "admit_wait_p99_s": cb.get("admit_wait_p99_s"),
            "codes_identical_alone_vs_mix": r["serving"]["codes_identical_alone_vs_mix"]}


def precision_forms(D, w, X, ref, fp32_ms: float, args, dev) -> dict:
    """The BF16 and FP16 forms of the encoder on the same input as the FP32 line: step time,
    speedup over FP32 and, on the reference's sample, selection match and MSE."""
    import torch
    from paper_1806_04374_amd import rsc
    g, K, P = w["geom"], w["K"], X.shape[0]
    res = {}
    for prec in ("bf16", "fp16"):
        h = rsc.rsc_create(g.N, g.S, g.T, prec=prec)
        rsc.rsc_set_dictionary(h, D.astype(np.float32), w["R"])
        xh = torch.empty((P, g.B), dtype=torch.float32, device=dev)
        outs = (torch.empty((P, K), dtype=torch.int32, device=dev), torch.empty((P, K), dtype=torch.int32, device=dev),
                torch.empty((P, K), dtype=torch.float32, device=dev), torch.empty((P,), dtype=torch.float32, device=dev))
        stream = torch.cuda.current_stream()
        for _ in range(3):
            rsc.rsc_project(h, X, xh, stream=stream)
            rsc.rsc_omp_encode(h, xh, K, out=outs, stream=stream)
        n = max(10, args.steps)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b, c in ev:
            a.record(stream)
            rsc.rsc_project(h, X, xh, stream=stream)
            b.record(stream)
            rsc.rsc_omp_encode(h, xh, K, out=outs, stream=stream)
            c.record(stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / n
        enc = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
        r = {"ms_per_step": ms, "patches_per_s": P / (ms * 1e-3), "speedup_vs_fp32": fp32_ms / ms,
             "encode_mean_ms": enc,
             "roofline": encoder_roofline(h, prec, w["M"], w["R"], g.S, g.T, K, P, enc * 1e-3)}
        if ref is not None:
            r["check"] = device_check(h, ref, D, w["R"], K, dev)
        r["precision_stats"] = rsc.rsc_precision_stats(h)
        res[prec] = r
        h.close()
    return res


def small_latency(dev, runs: int = 100) -> dict:
    """The small workload (2,000 11x11 patches, M=16, K=2, R=32): latency of one project +
    encode over `runs` runs, HIP events on the launch stream, called eagerly and replayed
    from a HIP graph, and its codes against the FP64 reference (all 2,000 patches)."""
    import torch
    from oracle import rsc_oracle as orc
    from paper_1806_04374_amd import rsc
    w = wl.SMALL
    g, K = w["geom"], w["K"]
    D, draw = wl.small_draw()
    basis = orc.build_basis(g.N, g.S, g.T)
    X = orc.synthesize(basis, D, draw.atom, draw.angle, draw.weight, draw.noise).astype(np.float32)
    _, code = orc.encode(basis, D, w["R"], X.astype(np.float64), K)
    ref = {"X": X, "code": code, "mse": orc.mse(basis, X, orc.reconstruct(basis, D, w["R"], code)), "basis": basis}
    res = {"workload": f"{w['name']}: {w['P']} 11x11 patches, M={w['M']}, K={K}, R={w['R']}", "runs": runs}
    for prec in ("fp32", "bf16", "fp16"):
        h = rsc.rsc_create(g.N, g.S, g.T, prec=prec)
        rsc.rsc_set_dictionary(h, D.astype(np.float32), w["R"])
        x = torch.from_numpy(X).to(dev)
        xh = torch.empty((len(X), g.B), dtype=torch.float32, device=dev)
        outs = (torch.empty((len(X), K), dtype=torch.int32, device=dev),
                torch.empty((len(X), K), dtype=torch.int32, device=dev),
                torch.empty((len(X), K), dtype=torch.float32, device=dev), None)
        stream = torch.cuda.current_stream()
        lat = []
        for i in range(runs + 5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            rsc.rsc_project(h, x, xh, stream=stream)
            rsc.rsc_omp_encode(h, xh, K, out=outs, stream=stream)
            b.record(stream)
            b.synchronize()
            if i >= 5:
                lat.append(a.elapsed_time(b) * 1e3)
        eager = outs[0].clone()
        # the same two launches captured once in a HIP graph and replayed: what a serving loop
        # that replays a graph sees, without the host's per-call work between the launches
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            cs = torch.cuda.current_stream()
            rsc.rsc_project(h, x, xh, stream=cs)
            rsc.rsc_omp_encode(h, xh, K, out=outs, stream=cs)
        glat = []
        for i in range(runs + 5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            graph.replay()
            b.record(stream)
            b.synchronize()
            if i >= 5:
                glat.append(a.elapsed_time(b) * 1e3)
            if not torch.equal(outs[0], eager):
                raise RuntimeError("graph replay changed the codes")
        res[prec] = {"p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
                     "graph_p50_us": float(np.percentile(glat, 50)), "graph_p99_us": float(np.percentile(glat, 99)),
                     "check": device_check(h, ref, D, w["R"], K, dev)}
        del graph
        h.close()
    return res


if __name__ == "__main__":
    main()
