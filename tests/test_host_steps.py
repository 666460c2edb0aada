"""Host-side optimiser steps of the library against the oracle (no GPU needed)."""
import os

import numpy as np
import pytest

from oracle import oracle as O

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2211_17263_amd", "libprdpt.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libprdpt.so not built")


def test_sigma_schedule_matches_oracle():
    from paper_2211_17263_amd import native as NV
    for t in range(0, 200, 7):
        assert NV.prdpt_sigma_schedule(1.0, 0.05, t, 200) == O.sigma_schedule(1.0, 0.05, t, 200)
    assert NV.prdpt_sigma_schedule(1.0, 0.05, 199, 200) == pytest.approx(0.05, abs=1e-15)


def test_adam_matches_oracle():
    from paper_2211_17263_amd import native as NV
    rng = np.random.default_rng(0)
    a, b = rng.normal(size=5), None
    b = a.copy()
    ma, va, mb, vb = (np.zeros(5) for _ in range(4))
    for t in range(1, 30):
        g = rng.normal(size=5)
        NV.prdpt_adam_step(a, g, ma, va, t, 0.01)
        O.adam_step(b, g, mb, vb, t, 0.01)
        np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-15)


def test_warm_started_schedule():
    # constant sigma_0 until half of the iterations, then linear to sigma_min at
    # the last one (Sec. 3.3 with the supplement's warm start)
    from paper_2211_17263_amd import optimize as OP
    steps = 101
    for t in range(steps):
        got = OP.sigma_at([0.5, 0.25], 0.01, t, steps, warm_start=0.5)
        first = 50
        want = [s0 if t <= first else O.sigma_schedule(s0, 0.01, t - first, steps - first)
                for s0 in (0.5, 0.25)]
        assert np.array_equal(got, np.array(want, np.float32)), t
    assert OP.sigma_at(0.5, 0.01, steps - 1, steps)[0] == np.float32(0.01)
    assert OP.sigma_at(1.0, 0.05, 0, 200, warm_start=0.0)[0] == np.float32(1.0)
    assert OP.sigma_at(1.0, 0.05, 199, 200, warm_start=0.0)[0] == np.float32(0.05)


def test_driver_checkpoint_round_trip(tmp_path):
    # the checkpoint holds the parameters, Adam's moments, the next iteration
    # and the run's settings bit for bit, in a file that loads without pickle
    import numpy as np
    from paper_2211_17263_amd import optimize as OP
    rng = np.random.default_rng(3)
    st = OP.DriverState(theta=rng.normal(size=5), m=rng.normal(size=5), v=rng.random(5), t=17,
                        steps=200, sigma0=np.array([1.0, 0.5, 0.25, 0.125, 0.0625]),
                        sigma_min=0.05, warm_start=0.5, lr=0.01, N=32, est=1, seed=2**40 + 7)
    path = str(tmp_path / "ckpt.npz")
    OP.save_state(path, st)
    back = OP.load_state(path)
    for f in ("theta", "m", "v", "sigma0"):
        assert np.array_equal(getattr(back, f).view(np.uint64), getattr(st, f).view(np.uint64))
    for f in ("t", "steps", "sigma_min", "warm_start", "lr", "N", "est", "seed"):
        assert getattr(back, f) == getattr(st, f)
    with np.load(path, allow_pickle=False) as z:
        assert all(z[k].dtype != object for k in z.files)
