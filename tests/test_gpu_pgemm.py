"""The split-BF16 product on pre-split operands (bf16 planes), through the
ris_test_pgemm entry: FP64 output with alpha / beta, plane output, the banded
K of the exchange weights, lower tiles, the two-product form A B^T + B A^T,
ragged M, N and K (K padded to a multiple of 32 with zero columns).  Reference: the same parts of fl32(x)
formed in numpy (round-to-nearest-even to bf16) and the same products summed
in FP64; the kernel sums in FP32, so the bar is 2e-5 of sum |A||B|^T (a wrong
index or part moves an element by O(1) of it)."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bf16(x32):
    """round-to-nearest-even float32 -> bf16, returned as float32"""
    b = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def parts(x, ns):
    f = np.asarray(x, dtype=np.float32)
    out = []
    for _ in range(ns):
        p = bf16(f)
        out.append(p)
        f = (f - p).astype(np.float32)
    return out


# parts of A and B in each product: ns = 2: hi.lo, lo.hi, hi.hi;
# ns = 3: hi.lo, lo.hi, mid.mid, hi.mid, mid.hi, hi.hi (part 1 = mid, 2 = lo)
PRODUCTS = {2: [(0, 1), (1, 0), (0, 0)], 3: [(0, 2), (2, 0), (1, 1), (0, 1), (1, 0), (0, 0)]}


def emulate(A, B, ns, alpha):
    pa, pb = parts(A, ns), parts(B, ns)
    acc = np.zeros((A.shape[0], B.shape[0]))
    for ia, ib in PRODUCTS[ns]:
        acc += pa[ia].astype(np.float64) @ pb[ib].astype(np.float64).T
    return alpha * acc


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def run(lib, ns, A, B, alpha, beta, C0, kband=0, lower=0, out_planes=0, sym2=0):
    import torch
    dA = torch.as_tensor(A, device="cuda")
    dB = torch.as_tensor(B, device="cuda")
    dC = torch.as_tensor(C0, device="cuda").clone()
    M, K = A.shape
    N = B.shape[0]
    say(f"[gpu] pgemm ns={ns} M={M} N={N} K={K} kband={kband} lower={lower} planes={out_planes} sym2={sym2}")
    st = lib.ris_test_pgemm(ns, M, N, K, alpha, _p(dA), K, _p(dB), K, beta, _p(dC), N, kband, lower, out_planes,
                            sym2)
    assert st == 0
    return dC.cpu().numpy()


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_18233_amd import ris
    return ris.load_library()


@pytest.mark.parametrize("ns", [2, 3])
@pytest.mark.parametrize("M,N,K", [(300, 200, 136), (131, 260, 45), (257, 129, 1173)])
def test_pgemm_fp64_out(lib, ns, M, N, K):
    rng = np.random.default_rng(M * 7 + N + K + ns)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((N, K)) * 1e-3
    C0 = rng.standard_normal((M, N))
    bound = 2e-5 * (np.abs(A) @ np.abs(B).T)
    got = run(lib, ns, A, B, -0.5, 0.0, C0)
    assert np.all(np.abs(got - emulate(A, B, ns, -0.5)) <= bound * 0.5)
    got = run(lib, ns, A, B, 0.3, 1.0, C0)
    assert np.all(np.abs(got - (emulate(A, B, ns, 0.3) + C0)) <= bound * 0.3 + 1e-15)
    # the split itself: products of the parts reproduce the FP64 product to
    # the split's relative order (2^-16 with three products, 2^-22 with six)
    exact = -0.5 * A @ B.T
    rel = 2.0 ** -15 if ns == 2 else 2.0 ** -21
    assert np.all(np.abs(emulate(A, B, ns, -0.5) - exact) <= rel * 0.5 * (np.abs(A) @ np.abs(B).T))


@pytest.mark.parametrize("ns", [2, 3])
def test_pgemm_kband(lib, ns):
    """B (3w x 3w) zero in its (1st row, 3rd k) and (3rd row, 1st k) blocks, as
    W^T of the exchange weights; column tiles wholly inside the first or the
    third block skip the zero k-blocks (w = 130 puts both cases in one call)"""
    rng = np.random.default_rng(3 + ns)
    w, M = 130, 200
    A = rng.standard_normal((M, 3 * w))
    B = rng.standard_normal((3 * w, 3 * w))
    B[:w, 2 * w:] = 0.0
    B[2 * w:, :w] = 0.0
    got = run(lib, ns, A, B, 1.0, 0.0, np.zeros((M, 3 * w)), kband=w)
    assert np.all(np.abs(got - emulate(A, B, ns, 1.0)) <= 2e-5 * (np.abs(A) @ np.abs(B).T))


@pytest.mark.parametrize("ns", [2, 3])
def test_pgemm_lower_tiles(lib, ns):
    rng = np.random.default_rng(9 + ns)
    n, K = 300, 64
    A = rng.standard_normal((n, K))
    B = rng.standard_normal((n, K))
    sentinel = 12345.0
    got = run(lib, ns, A, B, 1.0, 0.0, np.full((n, n), sentinel), lower=1)
    ref = emulate(A, B, ns, 1.0)
    bound = 2e-5 * (np.abs(A) @ np.abs(B).T)
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    tr, tc = r // 128, c // 128
    # every element on or below the diagonal is computed; tiles above the
    # diagonal tiles are untouched; the upper elements of a diagonal tile may
    # be either (its strictly upper 64 x 64 quarter is skipped)
    low = r >= c
    assert np.all(np.abs(got - ref)[low] <= bound[low])
    assert np.all(got[tr < tc] == sentinel)
    diag_up = (tr == tc) & (r < c)
    assert np.all((got[diag_up] == sentinel) | (np.abs(got - ref)[diag_up] <= bound[diag_up]))


@pytest.mark.parametrize("ns", [2, 3])
def test_pgemm_plane_output(lib, ns):
    """Plane output: the ns parts of the FP32 product, summed back in FP64"""
    rng = np.random.default_rng(21 + ns)
    M, N, K = 300, 141, 100
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((N, K))
    got = run(lib, ns, A, B, 1.0, 0.0, np.zeros((M, N)), out_planes=1)
    ref = emulate(A, B, ns, 1.0)
    keep = 2.0 ** -16 if ns == 2 else 0.0  # two parts hold 16 bits of the FP32 value, three all 24
    assert np.all(np.abs(got - ref) <= 2e-5 * (np.abs(A) @ np.abs(B).T) + keep * np.abs(ref))


@pytest.mark.parametrize("ns", [2, 3])
@pytest.mark.parametrize("lower", [0, 1])
def test_pgemm_sym2(lib, ns, lower):
    """C = alpha (A B^T + B A^T) in one launch (the exchange weights of a
    transition between two states): both products of the parts, summed in one
    set of FP32 accumulators; ragged n and K; with lower tiles the elements on
    or below the diagonal (the upper quarter of a diagonal tile may be
    written too, the rest is untouched)"""
    rng = np.random.default_rng(31 + ns + 2 * lower)
    n, K = 301, 117
    A = rng.standard_normal((n, K))
    B = rng.standard_normal((n, K)) * 3e-3
    sentinel = 12345.0
    got = run(lib, ns, A, B, -0.7, 0.0, np.full((n, n), sentinel), lower=lower, sym2=1)
    ref = emulate(A, B, ns, -0.7) + emulate(B, A, ns, -0.7)
    bound = 2e-5 * 0.7 * (np.abs(A) @ np.abs(B).T + np.abs(B) @ np.abs(A).T)
    # the two halves are not interchangeable: dropping either moves elements
    # by far more than the bar
    assert np.max(np.abs(emulate(A, B, ns, -0.7) - ref) - bound) > 0
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    if not lower:
        assert np.all(np.abs(got - ref) <= bound)
        return
    tr, tc = r // 128, c // 128
    low = r >= c
    assert np.all(np.abs(got - ref)[low] <= bound[low])
    assert np.all(got[tr < tc] == sentinel)
    diag_up = (tr == tc) & (r < c)
    assert np.all((got[diag_up] == sentinel) | (np.abs(got - ref)[diag_up] <= bound[diag_up]))


def test_pgemm_refuses_bad_arguments(lib):
    import torch
    d = torch.zeros(64, dtype=torch.float64, device="cuda")
    # ns outside {2, 3}; lower with M != N; plane output with beta; kband with K != 3w
    assert lib.ris_test_pgemm(4, 4, 4, 4, 1.0, _p(d), 4, _p(d), 4, 0.0, _p(d), 4, 0, 0, 0, 0) == 1
    assert lib.ris_test_pgemm(2, 4, 5, 4, 1.0, _p(d), 4, _p(d), 4, 0.0, _p(d), 5, 0, 1, 0, 0) == 1
    assert lib.ris_test_pgemm(2, 4, 4, 4, 1.0, _p(d), 4, _p(d), 4, 1.0, _p(d), 4, 0, 0, 1, 0) == 1
    assert lib.ris_test_pgemm(2, 4, 4, 6, 1.0, _p(d), 6, _p(d), 6, 0.0, _p(d), 4, 3, 0, 0, 0) == 1
    # the two-product form: M != N, beta, plane output
    assert lib.ris_test_pgemm(2, 4, 5, 4, 1.0, _p(d), 4, _p(d), 4, 0.0, _p(d), 5, 0, 0, 0, 1) == 1
    assert lib.ris_test_pgemm(2, 4, 4, 4, 1.0, _p(d), 4, _p(d), 4, 1.0, _p(d), 4, 0, 0, 0, 1) == 1
    assert lib.ris_test_pgemm(2, 4, 4, 4, 1.0, _p(d), 4, _p(d), 4, 0.0, _p(d), 4, 0, 0, 1, 1) == 1
