"""Benchmark: one extrapolated single+double-layer evaluation per step on the ellipsoid workload.

Workload (one step = one call evaluating u and v at all targets, densities resident in HBM):
ellipsoid semi-axes (1, 0.8, 0.6), h = 1/64 grid-line quadrature (N = 42342 points), targets = all
quadrature points + 20000 points within +-3h of the surface (M = 62342), rho = (2, 3, 4), cut-off 6,
direct far field.  The headline runs the FP64 path (every sum in double precision, as the paper's
code); the mixed path (far field FP32 with FP64 accumulation, near field and extrapolation FP64) is
reported beside it.

Prints ONE JSON line.  Metric: target-source interactions per second = 2 M N / t (each target-source
pair counted once for the single layer and once for the double layer per extrapolated evaluation),
with the seconds per SL+DL evaluation, single-layer-only and double-layer-only rates, the maximum and
L2 relative errors of both paths against the FP64 oracle on the oracle's timed sample of targets, and
the GMRES iterations and seconds of the two-sphere solve (zero start, FP64 relative residual 1e-8) at
gaps 0.1, 0.05, 0.02.

Other workloads (--workload; each prints its own JSON line):
  tree       ellipsoid (1, 0.8, 0.6), h = 1/128 (N = 169342, M = 189342), treecode far field (degree 8,
             theta 0.7, leaf 2000), mixed precision; the direct sum timed beside it and the treecode's
             error against the FP64 direct sum.
  gmres      two unit spheres, h = 1/64 (136332 points), gaps 0.1, 0.05, 0.02, random rigid motions:
             refined GMRES (mixed operator, FP64 residuals) to an FP64 relative residual of 1e-8.
  mlp        the warm-start network at its real shape (width 256, 102420 outputs, batch 64): time of
             a training step by phase, and of one inference.
  warmstart  the learned warm start end to end: solves at h = 1/64 kept at the h = 1/32 points train
             the network on the interaction part of the density (less the isolated spheres'); held-out
             (gap, motion) pairs are solved from zero, from the isolated spheres' density, from the
             network's prediction and from the training data interpolated in log(gap) (--ws-eval).
  table1     the paper's Table 1 workload: prolate spheroid x1^2 + 4 x2^2 + 4 x3^2 = 1, grid targets
             within h outside, single layer, rho = (3, 4, 5), h = 1/32 ... 1/256, direct far field.
  sweep      treecode parameters (theta, leaf size N0, degree p) at the h = 1/128 spheroid: time and
             error against the FP64 direct sum.
  drops      the paper's two drops nearly touching (section 4.3): GMRES to 1e-10 at h = 1/16 ... 1/128,
             iterations, times and the self-convergence errors of Table 2.
  peak       vector-ALU issue rates of the GPU (FP32 FMA with a scalar or only vector operands, FP64 FMA, FP32 rsq).
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

# Algorithmic work per far-field pair, per layer (FMA = 2 flops; the reciprocal square root counted
# separately): single layer 34 = d = y - x (3), r^2 (5), r^-2 and r^-3 (2), g = fw - c nw (6), d.g (5),
# scale (1), accumulate g/r + d (d.g)/r^3 (12); double layer 32 = d (3), r^2 (5), r^-2, r^-3, r^-5 (3),
# a = q - q0 (3), d.a (5), d.m (5), coefficient (2), accumulate (6).  An SL+DL evaluation is one SL pair
# and one DL pair per far target-source pair: 66 flops.
FAR_FLOPS_SL, FAR_FLOPS_DL = 34, 32
FAR_FLOPS_PER_PAIR_SLDL = FAR_FLOPS_SL + FAR_FLOPS_DL
# MI355X published peaks (AMD): FP64 vector 78.6 TFLOP/s, FP32 vector 157.3 TFLOP/s.  This build uses no
# packed FP32 instructions; plain FP32 instructions whose operands are all vector registers issue at about
# twice the rate of those with a scalar operand, which --workload peak measures (about 140 TFLOP/s) and the
# line reports beside the published figure.
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_PUBLISHED_TFLOPS = 157.3
PEAK_VALU_TFLOPS = PEAK_FP64_TFLOPS
TREE_FLOPS_PER_PROXY_PAIR = 75  # SL 24 + DL 40 + d, r^2, rsqrt, 1/r^2, 1/r^3 (11); FMA = 2

# HBM bytes per launch of the far-field kernels at this workload (FP64 and mixed), from rocprofv3
# FETCH_SIZE and WRITE_SIZE runs scaled by a copy calibration (profiles/far_near_c2_ellipsoid_h64.txt).
# Valid only for the kernel sources they were measured on: reported as null once a source's hash differs.
FAR_TRAFFIC = {"bytes": {"fp64": 1.074e8, "mixed": 9.786e7},
               "sources": {"paper_2507_00156_amd/csrc/sr_far.hip":
                           "5f769e32b82e18b25269dc80e51b0771830f5c67136ac01102e174866ce8632a",
                           "paper_2507_00156_amd/csrc/sr_internal.h":
                           "a38c60466ccaff6e83f185cb5e6994014831aad5b9554f5b1a89adbe6fde6f22"}}


def far_traffic(precision):
    import hashlib

    for rel, digest in FAR_TRAFFIC["sources"].items():
        try:
            with open(os.path.join(ROOT, rel), "rb") as f:
                if digest is None or hashlib.sha256(f.read()).hexdigest() != digest:
                    return None
        except OSError:
            return None
    return FAR_TRAFFIC["bytes"][precision]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU work for the oracle baseline")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="fp64", help="c2: the headline path")
    ap.add_argument("--workload", choices=["c2", "tree", "gmres", "mlp", "warmstart", "table1", "sweep", "drops",
                                           "peak"], default="c2")
    ap.add_argument("--no-gmres", action="store_true", help="c2: leave out the two-sphere GMRES solves")
    ap.add_argument("--drops-max", type=int, default=128, help="drops: finest 1/h")
    ap.add_argument("--train-solves", type=int, default=2004, help="warmstart: training solves")
    ap.add_argument("--train-steps", type=int, default=20000, help="warmstart: optimizer steps")
    ap.add_argument("--ws-batch", type=int, default=0, help="warmstart: Adam batch (0: every training solve)")
    ap.add_argument("--ws-passes", type=int, default=6, choices=(1, 3, 6),
                    help="warmstart: BF16 pieces products per matrix product of the network (6: FP32 accuracy)")
    ap.add_argument("--ws-no-readout", action="store_true",
                    help="warmstart: keep the output layers from Adam (no least-squares fit of them)")
    ap.add_argument("--ws-data-tol", type=float, default=1e-7, help="warmstart: relative residual of the training solves")
    ap.add_argument("--heldout", type=int, default=200, help="warmstart: held-out solves")
    ap.add_argument("--heldout-stride", type=int, default=1,
                    help="warmstart: solve every k-th of the held-out samples (the samples stay those of --heldout)")
    ap.add_argument("--ws-design", choices=("unit-log", "unit", "random"), default="unit",
                    help="warmstart: the 12 unit motions per gap at log-spaced or random gaps, or 4 random "
                         "motions per random gap")
    ap.add_argument("--ws-eval", default="zero,iso,net,basis",
                    help="warmstart: the starts solved for each held-out sample, comma-separated: zero, iso (the "
                         "isolated spheres' density), net (network + isolated part), basis (the training data "
                         "interpolated in log(gap) + isolated part)")
    ap.add_argument("--ws-net", choices=("pod", "full"), default="pod",
                    help="warmstart: the network predicts the coefficients of the training data's principal "
                         "directions (pod) or every coarse value (full)")
    ap.add_argument("--ws-save", default="", help="warmstart: write the trained model (and the training data's "
                                                   "coefficients) to this directory")
    ap.add_argument("--ws-load", default="", help="warmstart: evaluate a model written by --ws-save (no data, no training)")
    ap.add_argument("--ws-no-iso", action="store_true",
                    help="warmstart: train the network on the whole density (no isolated-sphere part)")
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
    """Time `steps` evaluations with profiling off: the library runs the near-field kernel concurrently
    with the far field.  With `profile`, time the same number again with profiling on: the library then
    runs the phases one after the other and records HIP events around each on the evaluation stream,
    which gives each kernel's own duration.  Returns (ms, wall, phases, out, serial_ms)."""
    import torch

    stream = torch.cuda.current_stream()
    u, v = ev.eval(P.SR_SL | P.SR_DL, *args_dev)
    out = (u, v, None, None)
    for _ in range(warmup):
        ev.eval(P.SR_SL | P.SR_DL, *args_dev, out=out)
    torch.cuda.synchronize()

    def timed():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            ev.eval(P.SR_SL | P.SR_DL, *args_dev, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, time.perf_counter() - t0

    ms, wall = timed()
    phases = serial_ms = None
    if profile:
        P.sr_get_profile(ev.ctx)  # clear
        P.sr_set_profiling(ev.ctx, True)
        serial_ms, _ = timed()
        P.sr_set_profiling(ev.ctx, False)
        tot, ne = P.sr_get_profile(ev.ctx)
        phases = [x / max(ne, 1) for x in tot]
    return ms, wall, phases, out, serial_ms


def cpu_baseline(cfg, target_seconds):
    """The FP64 oracle (three full regularized sums per target, then the 3x3 solve) on all host threads,
    on a bounded, evenly spaced sample of the same targets; scaled to interactions/s.  Returns the
    baseline record, the sample's indices and the oracle's (u, v) there."""
    import oracle

    t = cfg["targets"]
    n = cfg["surf"].n
    # calibrate on a small sample, then size the timed sample to about target_seconds
    k0 = 512  # large enough that the thread start-up does not dominate the estimate
    idx = np.linspace(0, t.m - 1, k0).astype(np.int64)
    t0 = time.perf_counter()
    oracle.sl_cfg(cfg, idx)
    oracle.dl_cfg(cfg, idx)
    dt = time.perf_counter() - t0
    k = int(np.clip(k0 * target_seconds / max(dt, 1e-3), k0, t.m))
    idx = np.linspace(0, t.m - 1, k).astype(np.int64)
    t0 = time.perf_counter()
    uo = oracle.sl_cfg(cfg, idx)
    vo = oracle.dl_cfg(cfg, idx)
    dt = time.perf_counter() - t0
    rec = {"value": 2.0 * k * n / dt, "unit": "interactions/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"{k} of {t.m} targets (evenly spaced), single+double layer, {dt:.1f} s",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    return rec, idx, (uo, vo)


def cpu_baseline_1thread(cfg, target_seconds):
    """The oracle on one thread, on a smaller evenly spaced sample."""
    import oracle

    t, n = cfg["targets"], cfg["surf"].n
    nt = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        k0 = 16
        idx = np.linspace(0, t.m - 1, k0).astype(np.int64)
        t0 = time.perf_counter()
        oracle.sl_cfg(cfg, idx)
        oracle.dl_cfg(cfg, idx)
        dt = time.perf_counter() - t0
        k = int(np.clip(k0 * target_seconds / max(dt, 1e-3), k0, t.m))
        idx = np.linspace(0, t.m - 1, k).astype(np.int64)
        t0 = time.perf_counter()
        oracle.sl_cfg(cfg, idx)
        oracle.dl_cfg(cfg, idx)
        dt = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(nt)
    return {"value": 2.0 * k * n / dt, "unit": "interactions/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} of {t.m} targets (evenly spaced), single+double layer, {dt:.1f} s, one thread",
            "cpu_model": cpu_model()}


def cpu_localized_baseline(cfg, target_seconds, gpu_fp64):
    """The paper-style localized CPU evaluation (far pairs once, near pairs at three deltas; gcc -O2,
    OpenMP over targets) on all host threads and on one, on evenly spaced samples; its error against the
    GPU FP64 result is reported for information (it is not a checker)."""
    import cpu_localized as L

    t, n = cfg["targets"], cfg["surf"].n
    out = {"kind": "paper-style localized CPU evaluation (not the oracle)", "unit": "interactions/s",
           "cpu_model": cpu_model()}
    nt = L.num_threads()
    for label, threads in (("all_threads", nt), ("one_thread", 1)):
        L.set_num_threads(threads)
        try:
            k0 = 512 if threads > 1 else 64
            idx = np.linspace(0, t.m - 1, k0).astype(np.int64)
            t0 = time.perf_counter()
            L.evaluate(cfg, idx)
            dt = time.perf_counter() - t0
            k = int(np.clip(k0 * (target_seconds / 2) / max(dt, 1e-3), k0, t.m))
            idx = np.linspace(0, t.m - 1, k).astype(np.int64)
            t0 = time.perf_counter()
            u, v = L.evaluate(cfg, idx)
            dt = time.perf_counter() - t0
        finally:
            L.set_num_threads(nt)
        out[label] = {"value": 2.0 * k * n / dt, "cores": threads,
                      "sample": f"{k} of {t.m} targets (evenly spaced), single+double layer, {dt:.1f} s"}
        if label == "all_threads":
            out["max_rel_diff_vs_gpu_fp64"] = {"sl": errors_vs(u, gpu_fp64[0][idx])["max_rel"],
                                                "dl": errors_vs(v, gpu_fp64[1][idx])["max_rel"]}
    return out


def cpu_baseline_tree(cfg, target_seconds, p=8, theta=0.7, leaf=2000):
    """The oracle treecode (its own octree, proxies and modified weights, built per call) on an evenly
    spaced sample of the targets; scaled to equivalent target-source interactions/s."""
    import oracle

    t, n = cfg["targets"], cfg["surf"].n

    def run(k):
        idx = np.linspace(0, t.m - 1, k).astype(np.int64)
        t0 = time.perf_counter()
        oracle.tree_cfg(cfg, idx, p=p, theta=theta, leaf=leaf)
        return time.perf_counter() - t0

    # every call builds the tree (a fixed cost a) and then pays b per target: fit both on two sizes and
    # size the sample so that the whole call takes about target_seconds
    k0 = 256
    t1, t2 = run(k0), run(4 * k0)
    b = max((t2 - t1) / (3 * k0), 1e-6)
    a = max(t1 - b * k0, 0.0)
    k = int(np.clip((target_seconds - a) / b, k0, t.m))
    idx = np.linspace(0, t.m - 1, k).astype(np.int64)
    t0 = time.perf_counter()
    oracle.tree_cfg(cfg, idx, p=p, theta=theta, leaf=leaf)
    dt = time.perf_counter() - t0
    return {"value": 2.0 * k * n / dt, "unit": "interactions/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{k} of {t.m} targets (evenly spaced), single+double layer, treecode degree {p}, theta {theta}, "
                      f"leaf {leaf}, tree set-up included, {dt:.1f} s", "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def cpu_baseline_rigid(h, gap, q, matvecs, target_seconds):
    """The oracle's rigid-sphere operator (FP64, direct sums) on an evenly spaced sample of rows, scaled
    to one matrix-vector product and multiplied by the number of products the GPU solve used."""
    import oracle
    import workload
    from oracle.rigid import RigidProblem, Sphere

    cen, rad, surfs = workload.two_spheres(h, gap)
    prob = RigidProblem([Sphere(sf, c, a, h) for sf, c, a in zip(surfs, cen, rad)], h, full=False)
    k0 = 64
    rows = np.linspace(0, prob.ntot - 1, k0).astype(np.int64)
    t0 = time.perf_counter()
    prob.matvec_rows(q, rows)
    dt0 = time.perf_counter() - t0
    k = int(np.clip(k0 * target_seconds / max(dt0, 1e-3), k0, prob.ntot))
    rows = np.linspace(0, prob.ntot - 1, k).astype(np.int64)
    t0 = time.perf_counter()
    prob.matvec_rows(q, rows)
    dt = time.perf_counter() - t0
    mv = dt * prob.ntot / k
    return {"value": mv * matvecs, "unit": "s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"oracle operator on {k} of {prob.ntot} rows ({dt:.1f} s), scaled to one product ({mv:.1f} s) "
                      f"x the {matvecs} products of the GPU solve at gap {gap}", "matvec_s": mv,
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def cpu_baseline_mlp(width, nout, batch, target_seconds):
    """The oracle network (numpy FP64: forward, gradients, Adam) at the same shape; training steps/s."""
    import workload
    from oracle import mlp as omlp

    p = workload.mlp_init(width, nout, 5)
    rng = np.random.default_rng(2)
    g, m = workload.warmstart_samples(batch, 3)
    m = m.reshape(batch, 12)
    y = rng.standard_normal((batch, nout))
    opt = omlp.Adam(lr=1e-4)
    steps, t0 = 0, time.perf_counter()
    while True:
        o, cache = omlp.forward(p, g, m, -2.760730458931123, 1.151292546497023)
        gr = omlp.backward(p, cache, o, y)
        opt.step(p, gr)
        steps += 1
        dt = time.perf_counter() - t0
        if dt >= target_seconds or steps >= 200:
            break
    return {"value": steps / dt, "unit": "steps/s", "cores": os.cpu_count(), "kind": "oracle",
            "sample": f"{steps} training steps (batch {batch}) of the numpy FP64 oracle, {dt:.1f} s; cores = the "
                      "threads numpy's BLAS may use", "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def base_line(metric, value, unit, steps, warmup, ms, higher, dtype, data, config):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": data, "config": config}


def bench_tree(a):
    """Treecode far field at the ellipsoid h = 1/128 workload."""
    import torch

    import paper_2507_00156_amd as P
    import workload

    cfg = workload.build_config("c3")
    s, t = cfg["surf"], cfg["targets"]
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()  # noqa: E731
    args_dev = [dev(t.y), dev(t.x0), dev(t.n0), dev(t.b), dev(cfg["f0"]), dev(cfg["q0"])]
    N, M = s.n, t.m
    res, outs = {}, {}
    for name, prec, far in (("tree", P.SR_MIXED, P.SR_TREE), ("direct", P.SR_MIXED, P.SR_DIRECT),
                            ("direct_fp64", P.SR_FP64, P.SR_DIRECT)):
        ev = P.Evaluator(cfg["h"], cfg["rho"], precision=prec, far_method=far, tree_degree=8, tree_theta=0.7,
                         tree_leaf=2000)
        ev.set_surface(dev(s.x), dev(s.normal), dev(s.w))
        ev.set_density(P.SR_SL, dev(cfg["f"]))
        ev.set_density(P.SR_DL, dev(cfg["q"]))
        steps = a.steps if name == "tree" else max(2, a.steps // 5)
        ms, wall, phases, out, _ = time_eval(P, ev, args_dev, steps, 1, profile=True)
        res[name] = dict(ms=ms, phases=phases, steps=steps)
        outs[name] = [o.clone() for o in out[:2]]
        log(f"[bench tree] {name}: {ms:.3f} ms/step, far {phases[0]:.3f} ms, near+extrap {phases[1]:.3f} ms")
        if name == "tree":
            work = ev.tree_work(t.y)  # (target-proxy interactions, leaf pairs, points in accepted clusters)
        ev.close()
    ref = outs["direct_fp64"]

    def rel(x, r):
        return ((x - r).norm(dim=1).max() / r.norm(dim=1).max()).item()

    ms = res["tree"]["ms"]
    out = base_line("target-source interactions/s (extrapolated single+double layer, treecode far field)",
                    2.0 * M * N / (ms / 1e3), "interactions/s", res["tree"]["steps"], 1, ms, True, "f32+f64",
                    "synthetic (seeded ellipsoid quadrature, degree-4 harmonic densities, near targets)",
                    {"workload": "ellipsoid (1,0.8,0.6), h=1/128: N=169342 sources, M=189342 targets, single+double "
                                 "layer, rho=(2,3,4), cutoff 6, treecode degree 8, theta 0.7, leaf 2000, mixed",
                     "n_sources": N, "n_targets": M})
    far_ms = res["tree"]["phases"][0]
    flops = TREE_FLOPS_PER_PROXY_PAIR * work[0] + FAR_FLOPS_PER_PAIR_SLDL * work[1]
    achieved = flops / (far_ms / 1e3) / 1e12
    out["roofline"] = {"bound": "alu", "kernel": "tree_far_kernel (treecode far field; the target Morton sort "
                       "runs before the timed phases)", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / PEAK_VALU_TFLOPS, "traffic": None,
                       "flops_per_proxy_pair": TREE_FLOPS_PER_PROXY_PAIR, "flops_per_leaf_pair": FAR_FLOPS_PER_PAIR_SLDL,
                       "proxy_pairs_per_launch": work[0], "leaf_pairs_per_launch": work[1], "kernel_ms": far_ms}
    out["phases_ms"] = {"far_tree": far_ms, "near_extrap": res["tree"]["phases"][1]}
    out["direct_mixed_ms"] = res["direct"]["ms"]
    out["direct_fp64_ms"] = res["direct_fp64"]["ms"]
    out["speedup_vs_direct_mixed"] = res["direct"]["ms"] / ms
    out["error_vs_fp64_direct"] = {"sl": rel(outs["tree"][0], ref[0]), "dl": rel(outs["tree"][1], ref[1])}
    out["error_direct_mixed_vs_fp64_direct"] = {"sl": rel(outs["direct"][0], ref[0]),
                                                "dl": rel(outs["direct"][1], ref[1])}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_tree(cfg, a.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_gmres(a):
    """Refined GMRES for two spheres at h = 1/64, one random rigid motion per gap."""
    import torch

    import workload
    from paper_2507_00156_amd import warmstart as W

    h = 1 / 64
    tree_kw = dict(far_method=1, tree_degree=6, tree_theta=0.6, tree_leaf=4000)
    per_gap, per_gap_tree = {}, {}
    mv_ms = None
    for gap in (0.1, 0.05, 0.02):
        sysm = W.TwoSpheres(h, gap, precision=1, **tree_kw)
        motion = workload.rigid_motion(np.random.default_rng(int(round(gap * 1000))))
        b = sysm.R.rhs(motion)
        sysm.R.solve_refined(b, tol=1e-8, restart=100)  # set-up (untimed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, it, nout, rr = sysm.R.solve_refined(b, tol=1e-8, restart=100)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        per_gap_tree[str(gap)] = {"seconds": dt, "inner_iterations": it, "fp64_corrections": nout, "fp64_relres": rr}
        log(f"[bench gmres] treecode gap {gap}: {dt:.2f} s, {it} inner iterations, {nout} passes, residual {rr:.1e}")
        sysm.close()
    for gap in (0.1, 0.05, 0.02):
        sysm = W.TwoSpheres(h, gap, precision=1)
        motion = workload.rigid_motion(np.random.default_rng(int(round(gap * 1000))))
        b = sysm.R.rhs(motion)
        if mv_ms is None:  # operator timing: mixed matrix-vector products
            q = b.clone()
            for _ in range(2):
                sysm.R.matvec(q)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(max(3, a.steps // 4)):
                sysm.R.matvec(q)
            e1.record()
            torch.cuda.synchronize()
            mv_ms = e0.elapsed_time(e1) / max(3, a.steps // 4)
        sysm.R.solve_refined(b, tol=1e-8, restart=100)  # builds the FP64 evaluators (set-up, untimed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, it, nout, rr = sysm.R.solve_refined(b, tol=1e-8, restart=100)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        per_gap[str(gap)] = {"seconds": dt, "inner_iterations": it, "fp64_corrections": nout, "fp64_relres": rr}
        log(f"[bench gmres] gap {gap}: {dt:.2f} s, {it} inner iterations, {nout} passes, residual {rr:.1e}")
        sysm.close()
    # the same operator with the on-surface modified smoothing for each sphere's own points
    sysm = W.TwoSpheres(h, 0.1, precision=1, surface_sharp=True)
    q = sysm.R.rhs(workload.rigid_motion(np.random.default_rng(100)))
    for _ in range(2):
        sysm.R.matvec(q)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(max(3, a.steps // 4)):
        sysm.R.matvec(q)
    e1.record()
    torch.cuda.synchronize()
    mv_sharp_ms = e0.elapsed_time(e1) / max(3, a.steps // 4)
    log(f"[bench gmres] matvec mixed {mv_ms:.2f} ms; with on-surface modified smoothing {mv_sharp_ms:.2f} ms")
    sysm.close()
    ntot, nsph = 136332, 68166
    mean_s = float(np.mean([v["seconds"] for v in per_gap_tree.values()]))
    out = base_line("seconds per two-sphere GMRES solve to FP64 relative residual 1e-8", mean_s, "s", 3, 1,
                    mean_s * 1e3, False, "f32+f64",
                    "synthetic (two unit spheres, grid-line quadrature, seeded random rigid motions)",
                    {"workload": "two unit spheres, h=1/64 (136332 points, 408996 unknowns), gaps 0.1/0.05/0.02, "
                                 "completed double layer; inner operator mixed precision with the treecode far field "
                                 "(degree 6, theta 0.6, leaf 4000), outer residuals FP64 with the direct far field; "
                                 "restart 100"})
    out["roofline"] = None
    out["per_gap"] = per_gap_tree
    out["per_gap_direct_far_field"] = per_gap
    out["seconds_direct_far_field_mean"] = float(np.mean([v["seconds"] for v in per_gap.values()]))
    out["matvec_ms_mixed"] = mv_ms
    out["matvec_interactions_per_s"] = 2 * nsph * ntot / (mv_ms / 1e3)
    out["matvec_ms_mixed_surface_sharp"] = mv_sharp_ms
    if not a.no_cpu_baseline:
        # matrix-vector products per solve: the inner iterations plus one FP64 residual per correction and
        # the initial one; the operator's cost hardly depends on the gap, so it is timed at the first gap
        nmv = float(np.mean([v["inner_iterations"] + v["fp64_corrections"] + 1 for v in per_gap_tree.values()]))
        ntot_cpu = sum(sf.n for sf in workload.two_spheres(h, 0.1)[2])
        qs = np.random.default_rng(11).standard_normal((ntot_cpu, 3))
        out["cpu_baseline"] = cpu_baseline_rigid(h, 0.1, qs, round(nmv), a.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_mlp(a):
    """Training step and inference of the warm-start network at its real shape."""
    import torch

    import paper_2507_00156_amd as P
    import workload

    W_, nout, batch, n = 256, 102420, 64, 256
    net = P.WarmStartNet(W_, nout, max_batch=batch, passes=3)
    net.set_params(np.concatenate([v.ravel() for v in workload.mlp_init(W_, nout, 5).values()]).astype(np.float32))
    rng = np.random.default_rng(1)
    g, m = workload.warmstart_samples(n, 2)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()  # noqa: E731
    gd, md, yd = dev(g), dev(m.reshape(n, 12)), dev(rng.standard_normal((n, nout)))
    net.fit_output_scale(yd)
    idxs = [torch.from_numpy(rng.integers(0, n, batch)).cuda() for _ in range(16)]
    steps = max(50, a.steps * 10)
    for i in range(a.warmup + 5):
        net.train_step(gd, md, yd, 1e-4, idx=idxs[i % 16], batch=batch, want_loss=False)
    torch.cuda.synchronize()
    net.get_profile()
    net.set_profiling(True)
    t0 = time.perf_counter()
    for i in range(steps):
        net.train_step(gd, md, yd, 1e-4, idx=idxs[i % 16], batch=batch, want_loss=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    net.set_profiling(False)
    ph, ns = net.get_profile()
    ph = [x / max(ns, 1) for x in ph]
    # inference: one prediction
    g1, m1 = gd[:1].contiguous(), md[:1].contiguous()
    for _ in range(5):
        net.predict(g1, m1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(50):
        net.predict(g1, m1)
    e1.record()
    torch.cuda.synchronize()
    inf_ms = e0.elapsed_time(e1) / 50
    nparam = net.nparam
    adam_bytes = 28 * nparam  # theta, m, v read + written (24 B) and the gradient read (4 B)
    achieved = adam_bytes / (ph[2] / 1e3) / 1e9
    out = base_line("warm-start network training steps/s (batch 64)", 1e3 / (wall * 1e3 / steps), "steps/s", steps,
                    a.warmup + 5, wall * 1e3 / steps, True, "bf16 (hi/lo, 3 products) + f32",
                    "synthetic (random targets at the real shape)",
                    {"workload": f"warm-start network: width 256, 4 layers, {nout} outputs, {nparam} parameters, "
                                 "batch 64"})
    out["roofline"] = {"bound": "hbm", "kernel": "adam_kernel (parameter update)", "achieved": achieved,
                       "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0, "traffic": None,
                       "bytes_per_launch": adam_bytes, "kernel_ms": ph[2]}
    out["phases_ms_per_step"] = {"forward": ph[0], "backward": ph[1], "adam": ph[2], "weight_copies": ph[3]}
    out["inference_ms_batch1"] = inf_ms
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_mlp(W_, nout, batch, a.cpu_seconds)
    print(json.dumps(out), flush=True)
    net.close()


def bench_warmstart(a):
    """Data from the library's own solves, training, and held-out solves from zero, from the learned
    warm start and from two warm starts without learning (the isolated spheres' density; the training
    data interpolated in log(gap))."""
    import torch

    import paper_2507_00156_amd as P
    import workload
    from paper_2507_00156_amd import warmstart as W

    h_c, h_f, width = 1 / 32, 1 / 64, 256
    methods = [m for m in a.ws_eval.split(",") if m]
    bad = set(methods) - {"zero", "iso", "net", "basis"}
    if bad:
        raise SystemExit(f"--ws-eval: unknown {sorted(bad)}")
    learned = "net" in methods or "basis" in methods
    use_iso = not a.ws_no_iso
    out_extra = {}
    t0 = time.perf_counter()
    iso = W.IsolatedSphere(h_f) if (use_iso or "iso" in methods) else None
    if iso is not None:
        out_extra["isolated_basis_seconds"] = time.perf_counter() - t0
        log(f"[bench warmstart] isolated-sphere basis: {iso.iterations} iterations, {time.perf_counter() - t0:.1f} s")
    starters = {"zero": None}
    if "iso" in methods:
        starters["iso"] = W.WarmStarter(None, h_c, iso)
    net = None
    if learned and a.ws_load:
        net, pod, gaps, motions, T, meta = W.load_model(a.ws_load)
        out_extra.update(meta)
        out_extra["loaded_from"] = os.path.basename(os.path.normpath(a.ws_load))
        if "net" in methods:
            starters["net"] = W.WarmStarter(W.network_predictor(net, pod), h_c, iso if use_iso else None)
        if "basis" in methods:
            starters["basis"] = W.WarmStarter(W.BasisInterpolator(gaps, T @ pod.V.T), h_c, iso if use_iso else None)
        log(f"[bench warmstart] loaded {meta.get('training_solves')} training solves' model: {pod.r} modes")
    elif learned:
        if a.ws_design in ("unit", "unit-log"):
            gaps, motions = workload.warmstart_unit_dataset(max(1, a.train_solves // 12), seed=21,
                                                             spacing="log" if a.ws_design == "unit-log" else "random",
                                                             ends=True)
        else:
            gaps, motions = workload.warmstart_dataset(max(1, a.train_solves // 4), 4, seed=21)
        t0 = time.perf_counter()
        Y, its = W.generate(h_f, gaps, motions, tol=a.ws_data_tol, log=log, keep=lambda g: W.restriction(h_c, h_f, g))
        t_data = time.perf_counter() - t0
        log(f"[bench warmstart] data: {len(gaps)} solves in {t_data:.0f} s (mean {its.mean():.1f} iterations)")
        out_extra.update({"data_seconds": t_data, "data_iterations_mean": float(its.mean()),
                          "training_solves": int(len(gaps))})
        if use_iso:
            for c0 in range(0, len(gaps), 256):
                Y[c0:c0 + 256] -= W.coarse_isolated(iso, h_c, motions[c0:c0 + 256])
        if "net" in methods:
            pod, T, scale = None, Y, None
            if a.ws_net == "pod":
                t0 = time.perf_counter()
                pod = W.PodDecoder(Y, rel=1e-7, rmax=width)
                T = pod.encode(Y)
                scale = torch.full((pod.r,), float(T.pow(2).mean().sqrt()), dtype=torch.float64, device="cuda")
                out_extra.update({"pod_modes": pod.r, "pod_energy_tail": pod.energy_tail,
                                  "pod_seconds": time.perf_counter() - t0})
                log(f"[bench warmstart] principal directions: {pod.r} modes, energy beyond them {pod.energy_tail:.1e} "
                    f"({time.perf_counter() - t0:.1f} s)")
            bs = min(4096, len(gaps)) if a.ws_batch <= 0 else a.ws_batch
            net = P.WarmStartNet(width, T.shape[1], max_batch=bs, passes=a.ws_passes)
            net.set_params(np.concatenate([v.ravel() for v in workload.mlp_init(width, T.shape[1], 5).values()])
                           .astype(np.float32))
            t0 = time.perf_counter()
            hist = W.train(net, gaps, motions, T, steps=a.train_steps, batch=bs, lr=1e-3, lr_min=1e-6, seed=3,
                           log=log, log_every=max(1, a.train_steps // 10), scale=scale)
            torch.cuda.synchronize()
            out_extra.update({"train_seconds": time.perf_counter() - t0, "final_train_loss": hist[-1][1],
                              "train_steps": a.train_steps, "train_batch": bs, "network_outputs": int(T.shape[1]),
                              "network_passes": a.ws_passes})
            if not a.ws_no_readout:
                if a.ws_design == "random" or scale is None:
                    raise SystemExit("the least-squares output layers need the unit-motion data and --ws-net pod")
                t0 = time.perf_counter()
                lam, loo, fit = W.fit_readout(net, gaps, T, scale, log=log)
                out_extra.update({"readout_lambda": lam, "readout_leave_one_gap_out_rms": loo,
                                  "readout_train_rms": fit, "readout_seconds": time.perf_counter() - t0})
                log(f"[bench warmstart] least-squares output layers: lambda {lam:.1e}, leave-one-gap-out RMS {loo:.2e}, "
                    f"training RMS {fit:.2e} (standardized)")
            starters["net"] = W.WarmStarter(W.network_predictor(net, pod), h_c, iso if use_iso else None)
            if a.ws_save:
                W.save_model(a.ws_save, net, pod, gaps, motions, T,
                             {k: out_extra[k] for k in ("training_solves", "data_seconds", "data_iterations_mean",
                                                        "train_seconds", "final_train_loss", "train_steps", "train_batch",
                                                        "network_outputs", "network_passes", "pod_modes",
                                                        "pod_energy_tail", "readout_lambda",
                                                        "readout_leave_one_gap_out_rms", "readout_train_rms")
                              if k in out_extra} | {"passes": a.ws_passes, "ws_design": a.ws_design,
                                                    "iso": use_iso, "data_tol": a.ws_data_tol})
                log(f"[bench warmstart] model written to {a.ws_save}")
        if "basis" in methods:
            if a.ws_design == "random":
                raise SystemExit("--ws-eval basis needs the unit-motion data (--ws-design unit or unit-log)")
            starters["basis"] = W.WarmStarter(W.BasisInterpolator(gaps, Y), h_c, iso if use_iso else None)
        if "basis" not in methods:
            del Y
    tg, tm = workload.warmstart_samples(a.heldout, 77)
    sel = list(range(0, len(tg), max(1, a.heldout_stride)))
    rows = {m: [] for m in methods}
    for c, i in enumerate(sel):
        g, m = tg[i], tm[i]
        fine = W.TwoSpheres(h_f, g, precision=1)
        b = fine.R.rhs(m)
        try:  # builds the FP64 evaluators (set-up, untimed); 3 iterations do not converge
            fine.R.solve_refined(b, tol=1e-8, restart=100, maxit=3)
        except P.SrError:
            pass
        msg, guesses, xs = [], {}, None
        for name in methods:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x0 = None if starters[name] is None else starters[name].guess(fine, m)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, it, _, rr = fine.R.solve_refined(b, x0=x0, tol=1e-8, restart=100)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            guesses[name] = x0
            xs = x if xs is None else xs
            rows[name].append([g, it, t2 - t0, t1 - t0, rr, 0.0])
            msg.append(f"{name} {it} ({t2 - t0:.2f} s)")
        for name in methods:  # the start's distance from the solution, relative
            x0 = guesses[name]
            rows[name][-1][5] = 1.0 if x0 is None else ((x0 - xs).norm() / xs.norm()).item()
        msg.append("start errors " + " ".join(f"{k} {rows[k][-1][5]:.1e}" for k in methods))
        log(f"[bench warmstart] held-out {c + 1}/{len(sel)} (sample {i}) gap {g:.4f}: " + ", ".join(msg))
        fine.close()
    R = {k: np.array(v) for k, v in rows.items()}
    summary = {k: {"iterations_mean": float(v[:, 1].mean()), "seconds_mean": float(v[:, 2].mean()),
                   "start_ms_mean": float(v[:, 3].mean() * 1e3), "max_final_residual": float(v[:, 4].max()),
                   "start_error_median": float(np.median(v[:, 5])), "start_error_max": float(v[:, 5].max())}
               for k, v in R.items()}
    if "zero" in R:
        for k, v in summary.items():
            v["iteration_ratio_vs_zero"] = summary["zero"]["iterations_mean"] / v["iterations_mean"]
            v["time_ratio_vs_zero"] = summary["zero"]["seconds_mean"] / v["seconds_mean"]
    head = "net" if "net" in summary else methods[-1]
    ratio = summary[head].get("iteration_ratio_vs_zero")
    for k, v in summary.items():
        log(f"[bench warmstart] {k}: mean {v['iterations_mean']:.1f} iterations, {v['seconds_mean']:.2f} s, start error "
            f"median {v['start_error_median']:.1e}"
            + (f", {v['iteration_ratio_vs_zero']:.2f}x fewer iterations than zero start" if "iteration_ratio_vs_zero" in v else ""))
    ntr = out_extra.get("training_solves", 0)
    out = base_line("GMRES iterations from zero / from the learned warm start (FP64 residual 1e-8)", ratio,
                    "x", len(sel), 0, summary[head]["seconds_mean"] * 1e3, True, "bf16 (hi/lo) network + f32/f64 solve",
                    "synthetic (two unit spheres, seeded gaps U[0.02,0.2] and N(0,1) rigid motions)",
                    {"workload": f"warm start: {ntr} training solves at h=1/64 kept at the h=1/32 points "
                                 + {"unit": "(the 12 unit motions at each of uniformly drawn gaps) ",
                                    "unit-log": "(the 12 unit motions at each of log-spaced gaps) ",
                                    "random": "(4 random motions at each of uniformly drawn gaps) "}[a.ws_design]
                                 + ("network on the interaction part (density less the isolated spheres') "
                                    if use_iso else "network on the whole density ")
                                 + ("predicting the coefficients of the data's principal directions "
                                    if a.ws_net == "pod" else "")
                                 + f"(102420 coarse values), width 256, {a.train_steps} Adam steps"
                                 + ("" if a.ws_no_readout else " then least-squares output layers")
                                 + f", {a.ws_passes}-product BF16 matrix products; {len(sel)} held-out "
                                 "solves at h=1/64 to FP64 residual 1e-8; starts: " + ", ".join(methods)})
    out["roofline"] = None
    out["starts"] = summary
    out.update(out_extra)
    out["iterations_by_sample"] = [[float(R[methods[0]][j, 0])] + [int(R[k][j, 1]) for k in methods]
                                   for j in range(len(sel))]
    out["iterations_by_sample_columns"] = ["gap"] + methods
    print(json.dumps(out), flush=True)
    if net is not None:
        net.close()


def _sl_setup(P, cfg, **kw):
    import torch

    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()  # noqa: E731
    s, t = cfg["surf"], cfg["targets"]
    ev = P.Evaluator(cfg["h"], cfg["rho"], **kw)
    ev.set_surface(dev(s.x), dev(s.normal), dev(s.w))
    ev.set_density(P.SR_SL, dev(cfg["f"]))
    args = [dev(t.y), dev(t.x0), dev(t.n0), dev(t.b), dev(cfg["f0"]), None]
    return ev, args


def _time_sl(P, ev, args, steps):
    import torch

    (u,) = [ev.eval(P.SR_SL, *args)[0]]
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        ev.eval(P.SR_SL, *args, out=(u, None, None, None))
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, u


def bench_table1(a):
    """The paper's Table 1 workload (single layer near the prolate spheroid) on the GPU."""
    import paper_2507_00156_amd as P
    import workload

    paper_4thread_s = {32: 1.0, 64: 11.0, 128: 155.0, 256: 2461.0}
    rows = {}
    for inv_h in (32, 64, 128, 256):
        log(f"[bench table1] generating the spheroid workload at h=1/{inv_h}")
        cfg = workload.build_config("table1", h=1 / inv_h)
        N, M = cfg["surf"].n, cfg["targets"].m
        r = {"n_quads": N, "n_targets": M}
        for name, prec in (("mixed", P.SR_MIXED), ("fp64", P.SR_FP64)):
            ev, args = _sl_setup(P, cfg, precision=prec)
            ms, u = _time_sl(P, ev, args, max(2, a.steps // (1 if inv_h < 256 else 4)))
            r[name + "_ms"] = ms
            r[name + "_pairs_per_s"] = M * N / (ms / 1e3)
            if name == "fp64":
                ref = u.clone()
            else:
                um = u.clone()
            ev.close()
        r["mixed_vs_fp64"] = ((um - ref).norm(dim=1).max() / ref.norm(dim=1).max()).item()
        r["paper_4thread_cpu_s"] = paper_4thread_s[inv_h]
        r["speedup_vs_paper_4thread_fp64"] = paper_4thread_s[inv_h] / (r["fp64_ms"] / 1e3)
        rows[str(inv_h)] = r
        log(f"[bench table1] h=1/{inv_h}: N={N} M={M} mixed {r['mixed_ms']:.2f} ms, fp64 {r['fp64_ms']:.2f} ms, "
            f"mixed vs fp64 {r['mixed_vs_fp64']:.1e}")
    top = rows["256"]
    out = base_line("target-source interactions/s (extrapolated single layer, Table 1 workload h=1/256)",
                    top["n_quads"] * top["n_targets"] / (top["mixed_ms"] / 1e3), "interactions/s", max(2, a.steps // 4),
                    1, top["mixed_ms"], True, "f32+f64",
                    "synthetic (the paper's spheroid and grid targets; density f1 = 1/sqrt(1 - 3 x1^2/4))",
                    {"workload": "prolate spheroid x1^2+4x2^2+4x3^2=1, targets = grid points within h outside, single "
                                 "layer, rho=(3,4,5), cutoff 6, direct far field; h = 1/32 .. 1/256"})
    out["roofline"] = None
    out["per_h"] = rows
    out["note"] = "paper times: 4-thread Intel Core i7 2.3 GHz, FP64, context only"
    print(json.dumps(out), flush=True)


def bench_sweep(a):
    """Treecode parameter sweeps on the h = 1/128 spheroid (the paper's treecode study)."""
    import paper_2507_00156_amd as P
    import workload

    cfg = workload.build_config("table1", h=1 / 128)
    N, M = cfg["surf"].n, cfg["targets"].m
    ev, args = _sl_setup(P, cfg, precision=P.SR_FP64)
    ref_ms, ref = _time_sl(P, ev, args, 2)
    ref = ref.clone()
    ev.close()
    ev, args = _sl_setup(P, cfg, precision=P.SR_MIXED)
    dmix_ms, _ = _time_sl(P, ev, args, 3)
    ev.close()
    base = dict(theta=0.6, leaf=2000, p=8)
    grid = [dict(base, theta=th) for th in (0.4, 0.5, 0.6, 0.7, 0.8)]
    grid += [dict(base, leaf=n0) for n0 in (500, 1000, 4000, 8000, 16000)]
    grid += [dict(base, p=p) for p in (4, 6, 10, 12)]
    res = []
    for g in grid:
        ev, args = _sl_setup(P, cfg, precision=P.SR_MIXED, far_method=P.SR_TREE, tree_degree=g["p"],
                             tree_theta=g["theta"], tree_leaf=g["leaf"])
        ev.eval(P.SR_SL, *args)  # tree set-up and modified weights
        ms, u = _time_sl(P, ev, args, 3)
        err = ((u - ref).norm(dim=1).max() / ref.norm(dim=1).max()).item()
        res.append(dict(g, ms=ms, err=err))
        log(f"[bench sweep] theta {g['theta']} N0 {g['leaf']} p {g['p']}: {ms:.2f} ms, error {err:.2e}")
        ev.close()
    out = base_line("treecode parameter sweep (single layer, spheroid h=1/128): time and error vs FP64 direct",
                    float(min(r["ms"] for r in res)), "ms", 3, 1, float(min(r["ms"] for r in res)), False, "f32+f64",
                    "synthetic (the paper's spheroid, grid targets within h)",
                    {"workload": f"prolate spheroid h=1/128 (N={N}, M={M}), single layer, rho=(3,4,5); sweeps of "
                                 "theta, N0, p around theta 0.6, N0 2000, p 8"})
    out["roofline"] = None
    out["direct_fp64_ms"] = ref_ms
    out["direct_mixed_ms"] = dmix_ms
    out["sweep"] = res
    print(json.dumps(out), flush=True)


def bench_drops(a):
    """Two drops nearly touching (eq. (IE-2Surf)): FP64 GMRES from zero to 1e-10, Table 2's columns."""
    import torch

    from paper_2507_00156_amd import drops

    paper = {16: (13, 3.17e-3, 1.19e-4), 32: (12, 1.07e-4, 6.11e-6), 64: (12, 4.06e-6, 2.11e-7),
             128: (12, 1.02e-7, 6.37e-9), 256: (12, None, None)}
    levels = [n for n in (16, 32, 64, 128, 256) if n <= a.drops_max]
    us, rows = {}, {}
    for inv_h in levels:
        T = drops.TwoDrops(1 / inv_h, precision=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, it, rr = T.solve(tol=1e-10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        us[inv_h] = u.cpu().numpy()
        rows[str(inv_h)] = {"n_points": int(sum(T.counts)), "iterations": it, "relres": rr, "seconds": dt,
                            "paper_iterations": paper[inv_h][0]}
        log(f"[bench drops] h=1/{inv_h}: {sum(T.counts)} points, {it} iterations (paper {paper[inv_h][0]}), "
            f"relres {rr:.1e}, {dt:.2f} s")
        T.close()
    prev = None
    for inv_h in levels[:-1]:
        emax, el2 = drops.self_convergence(us[inv_h], us[2 * inv_h], 1 / inv_h)
        r = rows[str(inv_h)]
        r.update(max_err=emax, l2_err=el2, paper_max_err=paper[inv_h][1], paper_l2_err=paper[inv_h][2])
        if prev is not None:
            r["max_order"] = float(np.log2(prev[0] / emax))
            r["l2_order"] = float(np.log2(prev[1] / el2))
        prev = (emax, el2)
        log(f"[bench drops] e_{inv_h}: max {emax:.3e} (paper {paper[inv_h][1]}), L2 {el2:.3e} (paper {paper[inv_h][2]})")
    fin = rows[str(levels[-1])]
    out = base_line("seconds per two-drop GMRES solve to relative residual 1e-10 (FP64)", fin["seconds"], "s", 1, 0,
                    fin["seconds"] * 1e3, False, "f64",
                    "synthetic (the paper's two drops: unit spheres at 0 and (2,0,1/16^3), surface tension 1+(x1-xc)^2)",
                    {"workload": f"two drops nearly touching, lambda=2, h=1/16..1/{levels[-1]}, own-surface modified "
                                 "smoothing delta=3h, cross-surface extrapolation delta=3h,4h,5h, direct far field"})
    out["roofline"] = None
    out["per_h"] = rows
    print(json.dumps(out), flush=True)


def near_pair_count(cfg):
    """Target-source pairs within the near radius cutoff * max delta (FP64 distances), for the far-pair
    count of the roofline: far pairs = M N - this."""
    from scipy.spatial import cKDTree

    s, t = cfg["surf"], cfg["targets"]
    rnear = 6.0 * max(cfg["rho"]) * cfg["h"]
    return int(cKDTree(s.x).query_ball_point(t.y, rnear, return_length=True).sum())


def peak_rates():
    """Measured vector-ALU rates from bench_peak.so (TFLOP/s, an FMA counting 2; rsq and add in Tops/s):
    FP32 FMA with a scalar operand and with vector operands only, FP64 FMA, FP32 rsq, FP32 and FP64 add
    (no packed FP32); 2048 workgroups of 256 lanes (8 wavefronts per SIMD), best of 4 launches."""
    import ctypes as C

    path = os.path.join(ROOT, "bench_peak.so")
    if not os.path.exists(path):
        return None
    L = C.CDLL(path)
    L.pk_run.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_float)]
    L.pk_run.restype = C.c_double
    out = {}
    for kind, name, iters in ((0, "fp32_fma_scalar_operand", 4096), (1, "fp64_fma", 2048), (2, "fp32_rsq", 2048),
                              (3, "fp32_add_scalar_operand", 4096), (4, "fp32_fma_vector_operands", 4096),
                              (5, "fp64_add", 2048)):
        best = 0.0
        for _ in range(4):
            ms = C.c_float()
            ops = L.pk_run(kind, iters, 2048, C.byref(ms))
            if ops < 0:
                return None
            best = max(best, ops / (ms.value / 1e3) / 1e12)
        out[name] = best
    return out


def bench_peak(a):
    r = peak_rates()
    out = base_line("vector ALU issue rate (microbenchmark)", r["fp32_fma_vector_operands"], "TFLOP/s", 4, 0, None,
                    True, "f32", "synthetic (register-resident FMA / rsq chains)",
                    {"workload": "2048 workgroups x 256 lanes, 8 or 16 independent chains per lane"})
    out["roofline"] = None
    out["rates"] = r
    out["published"] = {"fp64_vector": PEAK_FP64_TFLOPS, "fp32_vector_packed": PEAK_FP32_PUBLISHED_TFLOPS}
    print(json.dumps(out), flush=True)


def errors_vs(got, ref):
    """Max and L2 relative errors (Euclidean norm per target) of got against ref."""
    d = np.linalg.norm(got - ref, axis=1)
    nr = np.linalg.norm(ref, axis=1)
    return {"max_rel": float(d.max() / nr.max()), "l2_rel": float(np.sqrt((d ** 2).sum() / (nr ** 2).sum()))}


def gmres_summary(log_prefix="[bench]"):
    """Two spheres at h = 1/64, gaps 0.1, 0.05, 0.02, one seeded rigid motion per gap: refined GMRES from
    zero to an FP64 relative residual of 1e-8 (inner operator mixed with the treecode far field, degree 6,
    theta 0.6, leaf 4000; outer residuals FP64 with the direct far field); iterations and seconds."""
    import torch

    import workload
    from paper_2507_00156_amd import warmstart as W

    h = 1 / 64
    tree_kw = dict(far_method=1, tree_degree=6, tree_theta=0.6, tree_leaf=4000)
    per_gap = {}
    for gap in (0.1, 0.05, 0.02):
        sysm = W.TwoSpheres(h, gap, precision=1, **tree_kw)
        motion = workload.rigid_motion(np.random.default_rng(int(round(gap * 1000))))
        b = sysm.R.rhs(motion)
        sysm.R.solve_refined(b, tol=1e-8, restart=100)  # set-up: trees, FP64 evaluators (untimed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, it, nout, rr = sysm.R.solve_refined(b, tol=1e-8, restart=100)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        per_gap[str(gap)] = {"gmres_iterations": it, "fp64_corrections": nout, "fp64_relres": rr, "seconds": dt}
        log(f"{log_prefix} gmres gap {gap}: {it} iterations, {nout} FP64 corrections, residual {rr:.1e}, {dt:.2f} s")
        sysm.close()
    return per_gap


def host_buffer_eval(P, ev, cfg, steps, device_out):
    """sr_eval with the target arrays and the outputs in pinned host memory (SR_HOST: the call stages
    them to the device and back and synchronizes): wall time per evaluation including the host-device
    copies (in: y, x0, n0, f0, q0 and b, 128 B per target; out: u and v, 48 B per target)."""
    import torch

    from paper_2507_00156_amd.binding import sr_eval_host

    t = cfg["targets"]
    keep = []

    def pinned(x, shape=None):
        ten = (torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)) if x is not None
               else torch.empty(shape, dtype=torch.float64)).pin_memory()
        keep.append(ten)
        return ten.numpy()

    hin = [pinned(x) for x in (t.y, t.x0, t.n0, t.b, cfg["f0"], cfg["q0"])]
    u, v = pinned(None, (t.m, 3)), pinned(None, (t.m, 3))
    lay = P.SR_SL | P.SR_DL
    sr_eval_host(ev.ctx, lay, *hin, u, v)  # first call: the staging buffer
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sr_eval_host(ev.ctx, lay, *hin, u, v)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    # against the device-pointer evaluation of the same targets (which ran with the phases one after the
    # other: the far sum enters in another order, so the two agree to rounding, not bit for bit)
    diff = max(float(np.abs(u - device_out[0]).max() / np.abs(device_out[0]).max()),
               float(np.abs(v - device_out[1]).max() / np.abs(device_out[1]).max()))
    return {"ms_per_eval": ms, "interactions_per_s": 2.0 * t.m * cfg["surf"].n / (ms / 1e3), "steps": steps,
            "bytes_host_to_device": 128 * t.m, "bytes_device_to_host": 48 * t.m,
            "max_rel_diff_vs_device_pointer_outputs": diff}


def bench_c2(a):
    import torch

    import paper_2507_00156_amd as P
    import workload

    cfg = workload.build_config("c2")
    s, t = cfg["surf"], cfg["targets"]
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()  # noqa: E731
    args_dev = [dev(t.y), dev(t.x0), dev(t.n0), dev(t.b), dev(cfg["f0"]), dev(cfg["q0"])]
    N, M = s.n, t.m
    res, setup, outs = {}, {}, {}
    for prec_name, prec in (("fp64", P.SR_FP64), ("mixed", P.SR_MIXED)):
        ev = P.Evaluator(cfg["h"], cfg["rho"], precision=prec)
        xs, ns, ws, fd, qd = dev(s.x), dev(s.normal), dev(s.w), dev(cfg["f"]), dev(cfg["q"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev.set_surface(xs, ns, ws)  # geometry ingest (copies, host spatial index)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ev.set_density(P.SR_SL, fd)
        ev.set_density(P.SR_DL, qd)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ev.eval(P.SR_SL | P.SR_DL, *args_dev)  # first evaluation: cell list, packed records, then the sums
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        setup[prec_name] = {"set_surface_ms": 1e3 * (t1 - t0), "set_density_ms": 1e3 * (t2 - t1),
                            "first_eval_ms": 1e3 * (t3 - t2)}
        steps = a.steps if prec_name == a.precision else max(3, a.steps // 2)
        ms, wall, phases, out, serial_ms = time_eval(P, ev, args_dev, steps, a.warmup, profile=True)
        outs[prec_name] = (out[0].cpu().numpy(), out[1].cpu().numpy())
        # each layer alone (same targets, the other layer's work left out)
        one = {}
        for name, lay in (("sl", P.SR_SL), ("dl", P.SR_DL)):
            o = ev.eval(lay, *args_dev)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            k = max(3, steps // 2)
            e0.record()
            for _ in range(k):
                ev.eval(lay, *args_dev, out=(o[0], o[1], None, None))
            e1.record()
            torch.cuda.synchronize()
            one[name] = e0.elapsed_time(e1) / k
        ev.check()
        hostbuf = host_buffer_eval(P, ev, cfg, max(3, steps // 2), outs[prec_name])
        res[prec_name] = dict(ms=ms, wall=wall, phases=phases, steps=steps, serial_ms=serial_ms, sl_ms=one["sl"],
                              dl_ms=one["dl"], host=hostbuf)
        log(f"[bench] {prec_name}: {ms:.3f} ms/step (phases one after the other: {serial_ms:.3f} ms, far "
            f"{phases[0]:.3f} ms, near+extrap {phases[1]:.3f} ms); SL alone {one['sl']:.3f} ms, DL alone "
            f"{one['dl']:.3f} ms; with host buffers (PCIe-inclusive) {hostbuf['ms_per_eval']:.3f} ms")
        ev.close()

    near_pairs = near_pair_count(cfg)
    far_pairs = M * N - near_pairs
    peaks = peak_rates()

    def roofline(prec_name, peak, peak_name):
        far_ms = res[prec_name]["phases"][0]
        achieved = FAR_FLOPS_PER_PAIR_SLDL * far_pairs / (far_ms / 1e3) / 1e12
        return {"bound": "alu", "kernel": ("far_direct_kernel<double>" if prec_name == "fp64" else "far_lds_kernel "
                "(single precision)") + " (far-field pair sum, single+double layer)", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "peak_is": peak_name, "traffic": far_traffic(prec_name),
                "traffic_unit": "bytes per launch (HBM, counters scaled by a copy calibration)",
                "flops_per_pair": FAR_FLOPS_PER_PAIR_SLDL, "far_pairs_per_launch": far_pairs,
                "near_pairs_per_launch": near_pairs, "kernel_ms": far_ms,
                "kernel_ms_from": "second pass of this run with profiling on: the phases run one after the other "
                                  "and HIP events on the evaluation stream time each; the timed steps run the far "
                                  "and near kernels concurrently"}

    head = res[a.precision]
    ms = head["ms"]
    out = base_line("target-source interactions/s (extrapolated single+double layer evaluation)", 2.0 * M * N / (ms / 1e3),
                    "interactions/s", head["steps"], a.warmup, ms, True, "f64" if a.precision == "fp64" else "f32+f64",
                    "synthetic (seeded ellipsoid quadrature, degree-4 harmonic densities, near targets)",
                    {"workload": "ellipsoid (1,0.8,0.6), h=1/64: N=42342 sources, M=62342 targets "
                                 "(42342 on-surface + 20000 within 3h), single+double layer, rho=(2,3,4), cutoff 6, "
                                 "direct far field", "precision": a.precision, "n_sources": N, "n_targets": M,
                     "s_per_sl_dl_eval": ms / 1e3})
    out["roofline"] = (roofline("fp64", PEAK_FP64_TFLOPS, "published FP64 vector") if a.precision == "fp64"
                       else roofline("mixed", PEAK_FP32_PUBLISHED_TFLOPS, "published FP32 vector (packed)"))
    for name, r in res.items():
        out[name] = {"ms_per_step": r["ms"], "interactions_per_s": 2.0 * M * N / (r["ms"] / 1e3),
                     "s_per_sl_dl_eval": r["ms"] / 1e3, "sl_only_ms": r["sl_ms"], "dl_only_ms": r["dl_ms"],
                     "sl_interactions_per_s": M * N / (r["sl_ms"] / 1e3),
                     "dl_interactions_per_s": M * N / (r["dl_ms"] / 1e3),
                     "far_ms": r["phases"][0], "near_extrap_ms": r["phases"][1],
                     "ms_per_step_phases_serial": r["serial_ms"], "setup_ms": setup[name],
                     "host_buffers_pcie_inclusive": r["host"]}
    mixed_rf = roofline("mixed", PEAK_FP32_PUBLISHED_TFLOPS, "published FP32 vector (packed)")
    if peaks:
        mixed_rf["frac_of_measured_fp32_vector_operands"] = mixed_rf["achieved"] / peaks["fp32_fma_vector_operands"]
    out["mixed"]["roofline"] = mixed_rf
    out["vector_alu_measured_tflops"] = peaks
    if not a.no_gmres:
        out["gmres_two_spheres_h64"] = gmres_summary()
    if not a.no_cpu_baseline:
        cb, idx, (uo, vo) = cpu_baseline(cfg, a.cpu_seconds)
        out["cpu_baseline"] = cb
        out["error_vs_oracle"] = {"sample": cb["sample"]}
        for name, (u, v) in outs.items():
            out["error_vs_oracle"][name] = {"sl": errors_vs(u[idx], uo), "dl": errors_vs(v[idx], vo)}
        out["cpu_baseline_1thread"] = cpu_baseline_1thread(cfg, a.cpu_seconds / 2)
        out["cpu_localized"] = cpu_localized_baseline(cfg, a.cpu_seconds / 2, outs["fp64"])
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.copy_probe:
        copy_probe()
        return
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {a.gpus} is not supported "
              "(the multi-GPU sharding is described in the design notes, not implemented)", file=sys.stderr)
        sys.exit(2)
    if a.workload != "c2":
        import torch

        torch.cuda.init()  # the HIP runtime is initialized through torch before the library loads
        import paper_2507_00156_amd as P

        P.load_library()
        {"tree": bench_tree, "gmres": bench_gmres, "mlp": bench_mlp, "warmstart": bench_warmstart,
         "table1": bench_table1, "sweep": bench_sweep, "drops": bench_drops, "peak": bench_peak}[a.workload](a)
        return
    import torch

    torch.cuda.init()
    import paper_2507_00156_amd as P

    P.load_library()
    bench_c2(a)


if __name__ == "__main__":
    main()
