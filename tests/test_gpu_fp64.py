"""The device's FP64 square root and division, as the step kernels compile them, against the
host's correctly rounded results (numpy) on 10^6 seeded inputs: the reading that both sides use
IEEE binary64 with round-to-nearest rests on these two operations (the pseudopotential's square
root, the velocity's division); the ulp differences are reported and must be at most 1."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def ulps(x, y):
    """|x - y| in units in the last place (same-sign finite doubles)."""
    ix = x.view(np.int64)
    iy = y.view(np.int64)
    return np.abs(ix - iy)


def test_device_sqrt_and_division_rounding(gpu):
    import torch
    from paper_1410_2569_amd.lbm import fp64_probe

    rng = np.random.default_rng(7)
    n = 1_000_000
    # magnitudes of the densities, pseudopotentials, velocities and forces the step sees, and
    # uniform values in [0, 1)
    a = np.concatenate([10.0 ** rng.uniform(-8, 4, n // 2), rng.uniform(0.0, 1.0, n - n // 2)])
    b = 10.0 ** rng.uniform(-8, 4, n) * rng.choice([-1.0, 1.0], n)
    sq, qt = fp64_probe(torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda"))
    sq, qt = sq.cpu().numpy(), qt.cpu().numpy()
    us = ulps(sq, np.sqrt(a))
    uq = ulps(np.abs(qt), np.abs(a / b))
    assert np.array_equal(np.sign(qt), np.sign(a / b))
    print(f"sqrt: {int((us > 0).sum())} of {n} differ, max {int(us.max())} ulp; "
          f"division: {int((uq > 0).sum())} differ, max {int(uq.max())} ulp")
    assert us.max() <= 1 and uq.max() <= 1


def test_probe_rejects_null_arrays(gpu):
    import ctypes as C

    rc = gpu.lib().lbm_fp64_probe(None, None, None, None, 4, None)
    assert rc == -1
    assert gpu.lib().lbm_fp64_probe(None, None, None, None, 0, None) == 0
