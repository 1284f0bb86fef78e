"""The benchmark's localized CPU baseline (far pairs once, near pairs at three smoothing lengths) computes
the same extrapolated values as the oracle.  The baseline is timed by the benchmark only; this test
checks it against the oracle, never the other way round."""
import numpy as np

import oracle
import workload


def _rel(a, b):
    return np.linalg.norm(a - b, axis=1).max() / np.linalg.norm(b, axis=1).max()


def test_localized_baseline_equals_oracle():
    import cpu_localized as L

    cfg = workload.build_config("small")
    idx = np.arange(0, cfg["targets"].m, 5)
    u, v = L.evaluate(cfg, idx)
    assert _rel(u, oracle.sl_cfg(cfg, idx)) < 1e-12
    assert _rel(v, oracle.dl_cfg(cfg, idx)) < 1e-12
