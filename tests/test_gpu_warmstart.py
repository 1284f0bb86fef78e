"""The learned warm start at a small scale, end to end on the GPU: what the trained network gains over
the method without it.

Solves at h = 1/32 (24 gaps x 4 motions), kept at the h = 1/16 points, train the network; for
held-out (gap, motion) pairs the refined GMRES at h = 1/32 to an FP64 residual of 1e-8 is run from
zero and from the prediction interpolated to h = 1/32.  Both must converge; the warm start must
save iterations.
"""
import numpy as np
import pytest

import workload

pytestmark = pytest.mark.gpu


def test_warm_start_saves_iterations():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2507_00156_amd as P
    from paper_2507_00156_amd import warmstart as W

    P.load_library()
    h_c, h_f = 1 / 16, 1 / 32
    gaps, motions = workload.warmstart_dataset(24, 4, seed=21)
    Y, its = W.generate(h_f, gaps, motions, tol=1e-6, log=lambda s: print(s, flush=True),
                        keep=lambda g: W.restriction(h_c, h_f, g))
    print(f"data: {len(gaps)} solves, mean iterations {its.mean():.1f}", flush=True)
    net = P.WarmStartNet(128, Y.shape[1], max_batch=32, passes=3)
    net.set_params(np.concatenate([v.ravel() for v in workload.mlp_init(128, Y.shape[1], 5).values()]).astype(np.float32))
    hist = W.train(net, gaps, motions, Y, steps=3000, batch=32, lr=1e-3, seed=3, log=lambda s: print(s, flush=True))
    assert hist[-1][1] <= 0.01 * hist[0][1]
    ws = W.WarmStarter(net, h_c)
    tg, tm = workload.warmstart_samples(4, 77)
    zero_it, warm_it = [], []
    for g, m in zip(tg, tm):
        fine = W.TwoSpheres(h_f, g, precision=1)
        f64 = W.TwoSpheres(h_f, g, precision=0)
        b = fine.R.rhs(m)
        _, i0, n0, r0 = fine.R.solve_refined(b, tol=1e-8, restart=100)
        x0 = ws.guess(fine, m)
        g0 = (b - f64.R.matvec(x0)).norm().item() / b.norm().item()
        _, i1, n1, r1 = fine.R.solve_refined(b, x0=x0, tol=1e-8, restart=100)
        print(f"gap {g:.4f}: zero start {i0} iterations ({n0} passes), warm start {i1} ({n1} passes) from an "
              f"initial residual {g0:.1e} (final residuals {r0:.1e}, {r1:.1e})", flush=True)
        f64.close()
        assert r0 <= 1e-8 and r1 <= 1e-8
        zero_it.append(i0)
        warm_it.append(i1)
        fine.close()
    print(f"mean iterations: zero {np.mean(zero_it):.1f}, warm {np.mean(warm_it):.1f}", flush=True)
    assert np.mean(warm_it) <= 0.8 * np.mean(zero_it)
    net.close()
