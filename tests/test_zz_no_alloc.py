"""sr_eval_noalloc (static scratch array, no device allocation) against sr_eval through the C ABI:
two calls in a row, the second with fewer targets, at both precisions; the same kernels run on the
same inputs, so the results agree to the last bit."""
import numpy as np
import pytest

import workload
from tests.gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _ctx(cfg, precision):
    from paper_2507_00156_amd import binding as B

    p = B.sr_default_params()
    p.h = cfg["h"]
    p.rho[:] = cfg["rho"]
    p.precision = precision
    c = B.sr_create(0)
    B.sr_set_params(c, p)
    s = cfg["surf"]
    B.sr_set_surface(c, to_dev(s.x), to_dev(s.normal), to_dev(s.w))
    B.sr_set_density(c, B.SR_SL, to_dev(cfg["f"]))
    B.sr_set_density(c, B.SR_DL, to_dev(cfg["q"]))
    return c


def _targets(cfg, sel):
    t = cfg["targets"]
    return [to_dev(a[sel]) for a in (t.y, t.x0, t.n0)] + [to_dev(t.b[sel]), to_dev(cfg["f0"][sel]),
                                                         to_dev(cfg["q0"][sel])]


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_sr_eval(precision):
    import torch

    from paper_2507_00156_amd import binding as B

    cfg = workload.build_config("small")
    m = cfg["targets"].y.shape[0]
    print(f"[noalloc] small config, m={m}, precision={precision}", flush=True)
    c = _ctx(cfg, precision)
    try:
        rng = np.random.default_rng(7)
        first = np.arange(m)
        second = np.sort(rng.choice(m, m // 3, replace=False))  # smaller, a ragged count
        for sel in (first, second):
            y, x0, n0, b, f0, q0 = _targets(cfg, sel)
            k = len(sel)
            u_ref = torch.zeros((k, 3), dtype=torch.float64, device="cuda")
            v_ref = torch.zeros_like(u_ref)
            B.sr_eval(c, B.SR_SL | B.SR_DL, y, x0, n0, b, f0, q0, u_ref, v_ref)
            u = torch.full((k, 3), np.nan, dtype=torch.float64, device="cuda")
            v = torch.full_like(u, np.nan)
            B.sr_eval_noalloc(c, B.SR_SL | B.SR_DL, y, x0, n0, b, f0, q0, u, v)
            torch.cuda.synchronize()
            for name, got, ref in (("SL", u, u_ref), ("DL", v, v_ref)):
                got, ref = got.cpu().numpy(), ref.cpu().numpy()
                assert np.isfinite(got).all(), name
                err = np.abs(got - ref).max() / np.abs(ref).max()
                print(f"[noalloc] m={k} {name}: max |noalloc - sr_eval| / max |sr_eval| = {err:.1e}", flush=True)
                assert err <= (1e-10 if precision == 0 else 1e-7), (name, k, err)
                assert np.array_equal(got, ref), (name, k, err)
        # a density change is packed into the existing records without allocation
        B.sr_set_density(c, B.SR_SL, to_dev(2.0 * cfg["f"]))
        y, x0, n0, b, f0, q0 = _targets(cfg, second)
        f0 = 2.0 * f0
        k = len(second)
        u_ref = torch.zeros((k, 3), dtype=torch.float64, device="cuda")
        u = torch.full_like(u_ref, np.nan)
        B.sr_eval(c, B.SR_SL, y, x0, n0, b, f0, None, u_ref, None)
        B.sr_eval_noalloc(c, B.SR_SL, y, x0, n0, b, f0, None, u, None)
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), u_ref.cpu().numpy())
    finally:
        B.sr_destroy(c)


def test_noalloc_rejects_oversize_and_unbuilt_context():
    import torch

    from paper_2507_00156_amd import binding as B

    cfg = workload.build_config("tiny")
    c = _ctx(cfg, 0)
    try:
        y, x0, n0, b, f0, q0 = _targets(cfg, np.arange(cfg["targets"].y.shape[0]))
        u = torch.zeros_like(y)
        # no sr_eval yet: the cell list and records are not built, and building them would allocate
        with pytest.raises(B.SrError) as ei:
            B.sr_eval_noalloc(c, B.SR_SL, y, x0, n0, b, f0, None, u, None)
        assert ei.value.status == B.SR_ESTATE
        big = B.SR_NOALLOC_MAX_TARGETS + 1
        z = torch.zeros((big, 3), dtype=torch.float64, device="cuda")
        zb = torch.zeros(big, dtype=torch.float64, device="cuda")
        with pytest.raises(B.SrError) as ei:
            B.sr_eval_noalloc(c, B.SR_SL, z, z, z, zb, z, None, z, None)
        assert ei.value.status == B.SR_EINVAL and "out of range" in str(ei.value)
    finally:
        B.sr_destroy(c)
