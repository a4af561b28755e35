"""GPU checks of the matrix-core FP64 GEMM building block (test entry points
of include/ris_test.h) against numpy: the v_mfma_f64_16x16x4f64 lane layout
and the tiled GEMM over ragged shapes, all transpose combinations and batches."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_18233_amd.ris import load_library
    return load_library()


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_mfma_lane_layout(lib):
    import torch
    rng = np.random.default_rng(0)
    a = rng.standard_normal(64)
    b = rng.standard_normal(64)
    da = torch.tensor(a, device="cuda")
    db = torch.tensor(b, device="cuda")
    out = torch.zeros(256, dtype=torch.float64, device="cuda")
    assert lib.ris_test_mfma_probe(_p(da), _p(db), _p(out)) == 0
    got = out.cpu().numpy().reshape(64, 4)
    # layout: A[l%16][l/16] = a[l], B[l/16][l%16] = b[l], out[l][e] = D[4e + l/16][l%16]
    A = np.zeros((16, 4))
    B = np.zeros((4, 16))
    for l in range(64):
        A[l % 16, l // 16] = a[l]
        B[l // 16, l % 16] = b[l]
    D = A @ B
    ref = np.array([[D[4 * e + l // 16, l % 16] for e in range(4)] for l in range(64)])
    print("mfma layout max err", np.abs(got - ref).max(), flush=True)
    assert np.abs(got - ref).max() < 1e-13


@pytest.mark.parametrize("M,N,K,tA,tB,batch", [
    (16, 16, 4, 0, 0, 1), (128, 128, 16, 0, 0, 1), (200, 77, 45, 0, 0, 2), (77, 200, 45, 1, 0, 3),
    (131, 129, 300, 0, 1, 1), (45, 45, 133, 1, 1, 2), (1, 500, 1, 1, 0, 1), (300, 2, 17, 0, 1, 1)])
def test_dgemm_vs_numpy(lib, M, N, K, tA, tB, batch):
    import torch
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    As = (K, M) if tA else (M, K)
    Bs = (N, K) if tB else (K, N)
    A = rng.standard_normal((batch,) + As)
    B = rng.standard_normal((batch,) + Bs)
    C0 = rng.standard_normal((batch, M, N))
    dA, dB = torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")
    dC = torch.tensor(C0, device="cuda")
    print(f"dgemm M={M} N={N} K={K} tA={tA} tB={tB} batch={batch}", flush=True)
    st = lib.ris_test_dgemm(M, N, K, tA, tB, 0.7, _p(dA), As[1], int(np.prod(As)), _p(dB), Bs[1], int(np.prod(Bs)),
                            -0.3, _p(dC), N, M * N, batch)
    assert st == 0
    opA = A.transpose(0, 2, 1) if tA else A
    opB = B.transpose(0, 2, 1) if tB else B
    ref = 0.7 * opA @ opB - 0.3 * C0
    err = np.abs(dC.cpu().numpy() - ref).max()
    print("  err", err, flush=True)
    assert err < 1e-12 * max(1.0, np.abs(ref).max())
