"""The device Boys function (the one every integral kernel uses) against
F_m(T) = 1F1(m + 1/2; m + 3/2; -T) / (2m + 1) evaluated by mpmath at 40
digits, for m = 0..7 and T in [0, 60]: the table grid points T = k/16, the
grid midpoints (the Taylor expansion's farthest points), both sides of the
T = 40 switch to the asymptotic form, T near 0 and random points.  Bar:
1e-14 relative per value (the table is built in long double and the
expansion truncates below 1e-16)."""
import sys

import mpmath
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MMAX = 7


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def boys_ref(m, T):
    with mpmath.workdps(40):
        if T == 0:
            return mpmath.mpf(1) / (2 * m + 1)
        return mpmath.hyp1f1(m + mpmath.mpf(1) / 2, m + mpmath.mpf(3) / 2, -mpmath.mpf(T)) / (2 * m + 1)


def test_device_boys_vs_mpmath():
    import ctypes
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_18233_amd import ris
    lib = ris.load_library()
    rng = np.random.default_rng(11)
    pts = [0.0, 1e-14, 1e-8, 1e-3, 0.5 / 16, 1.0 / 32]
    pts += [k / 16.0 for k in range(0, 641, 7)]                    # grid points
    pts += [k / 16.0 + 1.0 / 32 for k in range(0, 640, 5)]         # grid midpoints
    pts += [39.9, 39.96875, 39.999, 40.0, 40.001, 40.03125, 41.0, 45.0, 50.0, 59.99, 60.0]
    pts += list(rng.uniform(0.0, 60.0, 200))
    T = np.array(pts, dtype=np.float64)
    Td = torch.as_tensor(T, device="cuda")
    Fd = torch.empty((T.size, MMAX + 1), dtype=torch.float64, device="cuda")
    say(f"[gpu] Boys probe on {T.size} points")
    assert lib.ris_test_boys(T.size, ctypes.c_void_p(Td.data_ptr()), ctypes.c_void_p(Fd.data_ptr())) == 0
    F = Fd.cpu().numpy()
    worst = (0.0, None)
    for i, t in enumerate(T):
        for m in range(MMAX + 1):
            ref = float(boys_ref(m, float(t)))
            rel = abs(F[i, m] - ref) / ref
            if rel > worst[0]:
                worst = (rel, (m, float(t)))
    say(f"[gpu] worst relative error {worst[0]:.2e} at (m, T) = {worst[1]}")
    assert worst[0] <= 1e-14
    # the argument check refuses a negative count without touching the GPU
    assert lib.ris_test_boys(-1, ctypes.c_void_p(Td.data_ptr()), ctypes.c_void_p(Fd.data_ptr())) == 1
