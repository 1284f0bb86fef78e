"""Benchmark: one extrapolated single+double-layer evaluation per step on the ellipsoid workload.

Workload (one step = one call evaluating u and v at all targets, densities resident in HBM):
ellipsoid semi-axes (1, 0.8, 0.6), h = 1/64 grid-line quadrature (N = 42342 points), targets = all
quadrature points + 20000 points within +-3h of the surface (M = 62342), rho = (2, 3, 4), cut-off 6,
direct far field.  The headline runs the mixed path (far field FP32 with FP64 accumulation, near
field and extrapolation FP64); the FP64 path is reported beside it.

Prints ONE JSON line.  Metric: target-source interactions per second = 2 M N / t (each target-source
pair counted once for the single layer and once for the double layer per extrapolated evaluation).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work of one far-field pair in the combined single+double layer pass (FMA = 2 flops,
# the reciprocal square root counted as 1): d = y - x (3), r^2 (5), rsqrt (1), r^-2 and r^-3 (2),
# single layer g = fw - c nw (6), d.g (5), scale (1), accumulate g/r + d s (12); double layer
# a = q - q0 (3), d.a (5), d.m (5), r^-5 (1), coefficient (2), accumulate (6).
FAR_FLOPS_PER_PAIR_SLDL = 57
# Per-lane VALU issue: 256 CUs x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz.  Packed FP32 is not
# used by this build, so FP32 and FP64 FMAs issue at the same rate.
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12  # 78.6
PEAK_FP32_PUBLISHED_TFLOPS = 157.3  # with packed FP32 (dual-issue per lane)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU work for the oracle baseline")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a device-to-device copy of 256 MiB (calibrates the FETCH_SIZE / WRITE_SIZE "
                         "counters against known bytes) and exit")
    return ap.parse_args()


def copy_probe():
    import torch

    n = 256 * 1024 * 1024 // 8
    a = torch.arange(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 3}))


def time_eval(P, ev, args_dev, steps, warmup, profile):
    import torch

    stream = torch.cuda.current_stream()
    u, v = ev.eval(P.SR_SL | P.SR_DL, *args_dev)
    out = (u, v, None, None)
    for _ in range(warmup):
        ev.eval(P.SR_SL | P.SR_DL, *args_dev, out=out)
    torch.cuda.synchronize()
    if profile:
        P.sr_get_profile(ev.ctx)  # clear
        P.sr_set_profiling(ev.ctx, True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        ev.eval(P.SR_SL | P.SR_DL, *args_dev, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    phases = None
    if profile:
        P.sr_set_profiling(ev.ctx, False)
        tot, ne = P.sr_get_profile(ev.ctx)
        phases = [x / max(ne, 1) for x in tot]
    return ms, wall, phases, out


def cpu_baseline(cfg, target_seconds):
    """The FP64 oracle (three full regularized sums per target, then the 3x3 solve) on a bounded,
    evenly spaced sample of the same targets; scaled to interactions/s."""
    import oracle

    t = cfg["targets"]
    n = cfg["surf"].n
    # calibrate on a small sample, then size the timed sample to about target_seconds
    idx = np.linspace(0, t.m - 1, 64).astype(np.int64)
    t0 = time.perf_counter()
    oracle.sl_cfg(cfg, idx)
    oracle.dl_cfg(cfg, idx)
    dt = time.perf_counter() - t0
    k = int(np.clip(64 * target_seconds / max(dt, 1e-3), 64, t.m))
    idx = np.linspace(0, t.m - 1, k).astype(np.int64)
    t0 = time.perf_counter()
    oracle.sl_cfg(cfg, idx)
    oracle.dl_cfg(cfg, idx)
    dt = time.perf_counter() - t0
    return {"value": 2.0 * k * n / dt, "unit": "interactions/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{k} of {t.m} targets (evenly spaced), single+double layer, {dt:.1f} s"}


def main():
    a = parse()
    if a.copy_probe:
        copy_probe()
        return
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {a.gpus} is not supported "
              "(the multi-GPU sharding is described in the design notes, not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2507_00156_amd as P
    import workload

    cfg = workload.build_config("c2")
    s, t = cfg["surf"], cfg["targets"]
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()  # noqa: E731
    args_dev = [dev(t.y), dev(t.x0), dev(t.n0), dev(t.b), dev(cfg["f0"]), dev(cfg["q0"])]
    N, M = s.n, t.m
    res = {}
    for prec_name, prec in (("mixed", P.SR_MIXED), ("fp64", P.SR_FP64)):
        ev = P.Evaluator(cfg["h"], cfg["rho"], precision=prec)
        ev.set_surface(dev(s.x), dev(s.normal), dev(s.w))
        ev.set_density(P.SR_SL, dev(cfg["f"]))
        ev.set_density(P.SR_DL, dev(cfg["q"]))
        steps = a.steps if prec_name == a.precision else max(3, a.steps // 4)
        ms, wall, phases, _ = time_eval(P, ev, args_dev, steps, a.warmup, profile=True)
        res[prec_name] = dict(ms=ms, wall=wall, phases=phases, steps=steps)
        print(f"[bench] {prec_name}: {ms:.3f} ms/step, far {phases[0]:.3f} ms, near+extrap {phases[1]:.3f} ms",
              file=sys.stderr, flush=True)
        ev.close()

    head = res[a.precision]
    ms = head["ms"]
    value = 2.0 * M * N / (ms / 1e3)
    far_ms = head["phases"][0]
    achieved = FAR_FLOPS_PER_PAIR_SLDL * M * N / (far_ms / 1e3) / 1e12
    out = {
        "metric": "target-source interactions/s (extrapolated single+double layer evaluation)",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if a.precision == "mixed" else "f64",
        "data": "synthetic (seeded ellipsoid quadrature, degree-4 harmonic densities, near targets)",
        "config": {
            "workload": "ellipsoid (1,0.8,0.6), h=1/64: N=42342 sources, M=62342 targets "
                        "(42342 on-surface + 20000 within 3h), single+double layer, rho=(2,3,4), cutoff 6, "
                        "direct far field",
            "precision": a.precision,
            "n_sources": N,
            "n_targets": M,
            "s_per_sl_dl_eval": ms / 1e3,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "far_direct_kernel (far-field pair sum)",
            "achieved": achieved,
            "peak": PEAK_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_VALU_TFLOPS,
            "traffic": None,
            "flops_per_pair": FAR_FLOPS_PER_PAIR_SLDL,
            "pairs_per_launch": M * N,
            "kernel_ms": far_ms,
            "frac_of_packed_fp32_published": achieved / PEAK_FP32_PUBLISHED_TFLOPS,
        },
        "phases_ms": {"far": far_ms, "near_extrap": head["phases"][1]},
        "other_precision": {k: {"ms_per_step": v["ms"], "value": 2.0 * M * N / (v["ms"] / 1e3),
                                "far_ms": v["phases"][0], "near_ms": v["phases"][1]}
                            for k, v in res.items() if k != a.precision},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
