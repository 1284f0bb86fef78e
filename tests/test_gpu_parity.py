"""GPU library (through the C ABI) against the FP64 CPU oracle, element by element.

Bars: FP64 path <= 1e-10 and mixed path <= 1e-7 in max_y |u_gpu - u_oracle| / max_y |u_oracle|
(Euclidean norm per target).  Sizes: whole workloads the oracle finishes in seconds (several
workgroup tiles plus a ragged tail), and the full 42342-point ellipsoid workload in the benchmark's
launch configuration, checked on sampled targets.
"""
import numpy as np
import pytest

import oracle
import workload
from tests.gpu_helpers import gpu_eval, rel_err, to_dev

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-7}  # SR_FP64, SR_MIXED


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2507_00156_amd as P

    P.load_library()
    return P


@pytest.fixture(scope="module")
def c1():
    cfg = workload.build_config("c1")
    u, ud = oracle.sl_cfg(cfg, want_delta=True)
    v, vd = oracle.dl_cfg(cfg, want_delta=True)
    return cfg, (u, v, ud, vd)


@pytest.fixture(scope="module")
def small():
    cfg = workload.build_config("small")
    u, ud = oracle.sl_cfg(cfg, want_delta=True)
    v, vd = oracle.dl_cfg(cfg, want_delta=True)
    return cfg, (u, v, ud, vd)


@pytest.mark.parametrize("precision", [0, 1])
def test_c1_full(P, c1, precision):
    cfg, (u, v, ud, vd) = c1
    gu, gv, gud, gvd = gpu_eval(cfg, P.SR_SL | P.SR_DL, precision, want_delta=True)
    print(f"c1 prec={precision}: SL {rel_err(gu, u):.3e} DL {rel_err(gv, v):.3e}", flush=True)
    assert rel_err(gu, u) <= TOL[precision]
    assert rel_err(gv, v) <= TOL[precision]
    for j in range(3):
        assert rel_err(gud[:, j], ud[:, j]) <= TOL[precision]
        assert rel_err(gvd[:, j], vd[:, j]) <= TOL[precision]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("layers", [1, 2, 3])
def test_small_full(P, small, precision, layers):
    cfg, (u, v, ud, vd) = small
    gu, gv = gpu_eval(cfg, layers, precision)
    if layers & 1:
        assert rel_err(gu, u) <= TOL[precision]
    if layers & 2:
        assert rel_err(gv, v) <= TOL[precision]


def test_layers_separately_equal_combined(P, small):
    cfg, _ = small
    gu, gv = gpu_eval(cfg, 3, 0)
    su, _ = gpu_eval(cfg, 1, 0)
    _, sv = gpu_eval(cfg, 2, 0)
    # the same pair arithmetic in the same order; only the compiler's fma contraction may differ
    assert rel_err(su, gu) <= 1e-13
    assert rel_err(sv, gv) <= 1e-13


def test_deterministic(P, small):
    cfg, _ = small
    a = gpu_eval(cfg, 3, 1)
    b = gpu_eval(cfg, 3, 1)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


@pytest.fixture(scope="module")
def c2_sample():
    # the benchmark workload (ellipsoid 1, 0.8, 0.6; h = 1/64; N = 42342, M = 62342): 1000 surface and
    # 1000 near targets sampled, plus the first and last of each kind; the oracle recomputes them one by one
    cfg = workload.build_config("c2")
    t = cfg["targets"]
    n = cfg["surf"].n
    rng = np.random.default_rng(42)
    idx = np.concatenate([rng.choice(n, 1000, replace=False), n + rng.choice(t.m - n, 1000, replace=False),
                          [0, n - 1, n, t.m - 1]])
    return cfg, idx, oracle.sl_cfg(cfg, idx), oracle.dl_cfg(cfg, idx)


@pytest.mark.parametrize("precision", [0, 1])
def test_c2_full_size_sampled(P, c2_sample, precision):
    """Evaluated in full on the GPU, in the benchmark's launch configuration; compared on 2004 sampled
    targets."""
    cfg, idx, u, v = c2_sample
    gu, gv = gpu_eval(cfg, 3, precision)
    e1, e2 = rel_err(gu[idx], u), rel_err(gv[idx], v)
    print(f"c2 prec={precision}: SL {e1:.3e} DL {e2:.3e}", flush=True)
    assert e1 <= TOL[precision] and e2 <= TOL[precision]


def test_table1_spheroid_rho345(P):
    # the paper's Table 1 workload at 1/h = 32 (spheroid, grid targets within h, rho = 3, 4, 5)
    cfg = workload.build_config("table1", h=1 / 32)
    gu, _ = gpu_eval(cfg, 1, 0)
    u = oracle.sl_cfg(cfg)
    assert rel_err(gu, u) <= 1e-10


def test_far_and_inside_targets(P):
    # targets farther than the near radius (no smoothing; extrapolation weight (1, 0, 0)) and deep inside
    cfg = workload.build_config("tiny")
    ax = cfg["axes"]
    y = np.array([[1.9, 0.2, -0.1], [0.05, -0.02, 0.03], [0.3, 0.1, -0.2], [-0.4, 1.3, 0.9], [0.0, 0.0, 1.2]])
    x0, b = workload.closest_point_ellipsoid(ax, y)
    n0 = workload.ellipsoid_normal(ax, x0)
    f0 = workload.harmonic_field(cfg["coeffs"], x0)
    tt = workload.Targets(y, x0, n0, b, np.full(len(b), -1))
    c2 = dict(cfg, targets=tt, f0=f0, q0=f0.copy())
    for prec in (0, 1):
        gu, gv = gpu_eval(c2, 3, prec)
        assert rel_err(gu, oracle.sl_cfg(c2)) <= TOL[prec]
        assert rel_err(gv, oracle.dl_cfg(c2)) <= TOL[prec]


def test_single_target_and_ragged(P, small):
    cfg, (u, v, _, _) = small
    for m in (1, 3, 65, 257, 513):
        idx = np.arange(m) * 7 % cfg["targets"].m
        gu, gv = gpu_eval(cfg, 3, 0, idx=idx)
        assert rel_err(gu, u[idx]) <= 1e-10
        assert rel_err(gv, v[idx]) <= 1e-10


def test_tiny_surface(P):
    # fewer sources than far-field source splits: empty splits must contribute zero
    cfg = workload.build_config("tiny")
    s = cfg["surf"]
    keep = np.arange(0, s.n, 200)  # 6 points
    s2 = workload.Surface(s.x[keep], s.normal[keep], s.w[keep], s.family[keep], s.axes, s.center, s.h)
    t = cfg["targets"]
    sel = np.concatenate([keep, [s.n, s.n + 1, s.n + 2]])
    c2 = dict(cfg, surf=s2, f=cfg["f"][keep], q=cfg["q"][keep], targets=t.subset(sel), f0=cfg["f0"][sel],
              q0=cfg["q0"][sel])
    gu, gv = gpu_eval(c2, 3, 0)
    assert rel_err(gu, oracle.sl_cfg(c2)) <= 1e-10
    assert rel_err(gv, oracle.dl_cfg(c2)) <= 1e-10


def test_empty_target_set_is_noop(P):
    import torch

    cfg = workload.build_config("tiny")
    s = cfg["surf"]
    ev = P.Evaluator(cfg["h"], cfg["rho"])
    ev.set_surface(to_dev(s.x), to_dev(s.normal), to_dev(s.w))
    ev.set_density(P.SR_SL, to_dev(cfg["f"]))
    z3 = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    z1 = torch.zeros((0,), dtype=torch.float64, device="cuda")
    u, v = ev.eval(P.SR_SL, z3, z3, z3, z1, z3, None)
    torch.cuda.synchronize()
    assert u.shape == (0, 3) and v is None
    ev.close()


def test_error_paths(P):
    cfg = workload.build_config("tiny")
    s, t = cfg["surf"], cfg["targets"]
    ev = P.Evaluator(cfg["h"], cfg["rho"])
    y = to_dev(t.y)
    with pytest.raises(P.SrError) as ei:  # surface not set
        ev.eval(P.SR_SL, y, to_dev(t.x0), to_dev(t.n0), to_dev(t.b), to_dev(cfg["f0"]))
    assert ei.value.status == -4
    ev.set_surface(to_dev(s.x), to_dev(s.normal), to_dev(s.w))
    with pytest.raises(P.SrError) as ei:  # density not set
        ev.eval(P.SR_DL, y, to_dev(t.x0), to_dev(t.n0), to_dev(t.b), None, to_dev(cfg["q0"]))
    assert ei.value.status == -4
    with pytest.raises(P.SrError) as ei:  # bad parameters
        ev.set_params(rho=(2.0, 2.0, 4.0))
    assert ei.value.status == -1
    bad_w = s.w.copy()
    bad_w[3] = np.nan
    with pytest.raises(P.SrError) as ei:
        ev.set_surface(to_dev(s.x), to_dev(s.normal), to_dev(bad_w))
    assert ei.value.status == -1
    ev.close()


def test_params_change_rebuilds_index(P, small):
    # changing rho changes the near radius; the cell grid must be rebuilt
    cfg, _ = small
    s, t = cfg["surf"], cfg["targets"]
    ev = P.Evaluator(cfg["h"], (2.0, 3.0, 4.0))
    ev.set_surface(to_dev(s.x), to_dev(s.normal), to_dev(s.w))
    ev.set_density(P.SR_SL, to_dev(cfg["f"]))
    idx = np.arange(0, t.m, 37)
    args = [to_dev(a[idx]) for a in (t.y, t.x0, t.n0, t.b, cfg["f0"])]
    ev.eval(P.SR_SL, *args)
    ev.set_params(rho=(3.0, 4.0, 5.0))
    u, _ = ev.eval(P.SR_SL, *args)
    ref = oracle.sl(s.x, s.normal, s.w, cfg["f"], t.y[idx], t.x0[idx], t.n0[idx], t.b[idx], cfg["f0"][idx],
                    cfg["h"], (3.0, 4.0, 5.0))
    assert rel_err(u.cpu().numpy(), ref) <= 1e-10
    ev.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("far", ["direct", "tree"])
def test_concurrent_phases_equal_serial(P, small, precision, far):
    # With no per-delta outputs and profiling off, the near-field kernel runs on the context's own
    # stream concurrently with the far field, and the far sum is added afterwards; with profiling on,
    # the phases run one after the other and the near kernel adds the far sum itself.  The two differ
    # only in rounding: (far + near) / (8 pi) against near / (8 pi) + far / (8 pi).  Three
    # evaluations with densities scaled by 2^k are enqueued back to back on a non-default stream, each
    # with its outputs copied right after on the same stream, and each is compared with a serial
    # evaluation of the same densities: a copy taken before the near kernel or the far addition
    # finished, or a kernel reading the previous call's records, would differ at the 1e-1 level.  (The
    # serial results are not assumed to scale exactly with 2^k: in single precision, products with
    # the tiny quadrature weights near the partition-of-unity cut-off underflow, and gradual
    # underflow is not homogeneous.)
    import torch

    cfg, (u_or, v_or, _, _) = small
    s, t = cfg["surf"], cfg["targets"]
    kw = dict(far_method=P.SR_TREE, tree_degree=6, tree_theta=0.6, tree_leaf=64) if far == "tree" else {}
    ev = P.Evaluator(cfg["h"], cfg["rho"], precision=precision, **kw)
    ev.set_surface(to_dev(s.x), to_dev(s.normal), to_dev(s.w))
    f, q, f0, q0 = (to_dev(cfg[k]) for k in ("f", "q", "f0", "q0"))
    y, x0, n0, b = (to_dev(a) for a in (t.y, t.x0, t.n0, t.b))
    tol = TOL[precision] if far == "direct" else 1e-3  # the treecode's own error against the direct oracle
    serial = []
    for k in range(3):
        c = float(2**k)
        ev.set_density(P.SR_SL, f * c)
        ev.set_density(P.SR_DL, q * c)
        torch.cuda.synchronize()
        P.sr_set_profiling(ev.ctx, True)
        us, vs = ev.eval(3, y, x0, n0, b, f0 * c, q0 * c)
        torch.cuda.synchronize()
        P.sr_set_profiling(ev.ctx, False)
        P.sr_get_profile(ev.ctx)
        serial.append((us.cpu().numpy(), vs.cpu().numpy()))
        assert rel_err(serial[-1][0], c * u_or) <= tol and rel_err(serial[-1][1], c * v_or) <= tol

    st = torch.cuda.Stream()
    snaps, keep = [], []
    with torch.cuda.stream(st):
        for k in range(3):
            c = float(2**k)
            fk, qk, f0k, q0k = f * c, q * c, f0 * c, q0 * c
            ev.set_density(P.SR_SL, fk)
            ev.set_density(P.SR_DL, qk)
            uk, vk = ev.eval(3, y, x0, n0, b, f0k, q0k)
            snaps.append((uk.clone(), vk.clone()))
            keep += [fk, qk, f0k, q0k, uk, vk]
    torch.cuda.synchronize()
    ev.close()
    for k, (uk, vk) in enumerate(snaps):
        e1 = rel_err(uk.cpu().numpy(), serial[k][0])
        e2 = rel_err(vk.cpu().numpy(), serial[k][1])
        print(f"concurrent {far} prec={precision} k={k}: SL {e1:.2e} DL {e2:.2e}", flush=True)
        assert e1 <= 1e-13 and e2 <= 1e-13


@pytest.mark.parametrize("precision", [0, 1])
def test_surface_table_equals_closed_forms(P, small, precision):
    """Targets on the surface (b = 0) take the smoothing table in the combined mode and the closed forms
    of eqs. (s1)-(s3) when the per-delta values are asked for; the extrapolated values agree to the
    table's accuracy in double precision (1e-12 relative) and, on the mixed path, to that of the closed
    forms' degree-11 erfcx interpolant (|erfc error| <= 1.6e-11, so <= 2e-9 in u)."""
    cfg, _ = small
    on = np.nonzero(cfg["targets"].b == 0.0)[0]
    assert len(on) > 100
    u1, v1 = gpu_eval(cfg, P.SR_SL | P.SR_DL, precision)[:2]
    u2, v2 = gpu_eval(cfg, P.SR_SL | P.SR_DL, precision, want_delta=True)[:2]
    e1, e2 = rel_err(u1[on], u2[on]), rel_err(v1[on], v2[on])
    print(f"table vs closed forms prec={precision}: SL {e1:.2e} DL {e2:.2e}", flush=True)
    bar = 1e-12 if precision == 0 else 2e-9
    assert e1 <= bar and e2 <= bar


def test_surface_targets_without_table_match_oracle(P, small):
    """With rho = 1 : 2 : 4 the smoothing table misses its accuracy check (the smallest delta is h, the
    range 24 h) and the surface targets take the closed forms in the combined mode; parity with the
    oracle."""
    cfg, _ = small
    rho = (1.0, 2.0, 4.0)
    with pytest.raises(P.SrError) as ei:  # the table the evaluation would build: refused
        P.sr_near_table(rho, 6.0, 6.0 * 4.0 * (1.0 + 1e-5))
    assert ei.value.status == -6
    cfg = dict(cfg, rho=rho)
    u = oracle.sl_cfg(cfg)
    v = oracle.dl_cfg(cfg)
    for precision in (0, 1):
        gu, gv = gpu_eval(cfg, P.SR_SL | P.SR_DL, precision)[:2]
        e1, e2 = rel_err(gu, u), rel_err(gv, v)
        print(f"rho 1:2:4 prec={precision}: SL {e1:.3e} DL {e2:.3e}", flush=True)
        assert e1 <= TOL[precision] and e2 <= TOL[precision]
