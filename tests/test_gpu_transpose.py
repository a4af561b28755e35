"""The LDS-tiled transpose that forms the H_UO blocks from the H_OU blocks,
checked through the C ABI against numpy: ragged shapes (not multiples of the
32 x 32 tile), leading dimensions wider than the rows, more row tiles than the
y grid holds (its row loop), the empty case and the argument checks."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("R,C,padi,pado", [(1, 1, 0, 0), (33, 31, 0, 0), (391, 7820, 3, 5), (77, 64, 0, 9),
                                           (2_100_000, 2, 1, 0)])
def test_transpose_matches_numpy(R, C, padi, pado):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_18233_amd import ris
    lib = ris.load_library()
    rng = np.random.default_rng(R + 7 * C)
    ldi, ldo = C + padi, R + pado
    A = rng.standard_normal((R, ldi))
    sentinel = -12345.0
    din = torch.as_tensor(A, device="cuda")
    dout = torch.full((C, ldo), sentinel, dtype=torch.float64, device="cuda")
    say(f"[gpu] transpose R={R} C={C} ldi={ldi} ldo={ldo}")
    assert lib.ris_test_transpose(_p(din), ldi, _p(dout), ldo, R, C) == 0
    got = dout.cpu().numpy()
    assert np.array_equal(got[:, :R], A[:, :C].T)
    # the padding columns of out are not written
    assert np.all(got[:, R:] == sentinel)


def test_transpose_empty_and_invalid():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_18233_amd import ris
    lib = ris.load_library()
    x = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    y = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    assert lib.ris_test_transpose(_p(x), 4, _p(y), 4, 0, 4) == 0
    assert lib.ris_test_transpose(_p(x), 4, _p(x), 4, 4, 4) == 1   # in place
    assert lib.ris_test_transpose(_p(x), 3, _p(y), 4, 4, 4) == 1   # ldi < C
    assert lib.ris_test_transpose(_p(x), 4, _p(y), 3, 4, 4) == 1   # ldo < R
    assert lib.ris_test_transpose(None, 4, _p(y), 4, 4, 4) == 1
