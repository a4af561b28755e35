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
    assert lib.ris_test_mfma_probe(0, _p(da), _p(db), _p(out)) == 0
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


def _probe_onehot(lib, kind, width):
    """Run the one-hot probe: for every (lane, slot) of A set a single 1, with
    distinct small integers in B; returns {(lane, slot): [(out_lane, e, value)]}."""
    import torch
    b = (np.arange(64 * width) % 97 + 1).astype(np.float64)
    db = torch.tensor(b, device="cuda")
    res = {}
    for la in range(64):
        for sl in range(width):
            a = np.zeros(64 * width)
            a[la * width + sl] = 1.0
            out = torch.zeros(256, dtype=torch.float64, device="cuda")
            assert lib.ris_test_mfma_probe(kind, _p(torch.tensor(a, device="cuda")), _p(db), _p(out)) == 0
            o = out.cpu().numpy().reshape(64, 4)
            res[(la, sl)] = [(int(l), int(e), o[l, e]) for (l, e) in np.argwhere(o != 0)]
    return b, res


@pytest.mark.parametrize("kind,width", [(1, 1), (2, 8)])
def test_mfma_f32_bf16_lane_layouts(lib, kind, width):
    """Lane l, slot s holds A[l % 16][width*(l // 16) + s] and B[width*(l // 16) + s][l % 16];
    out[l][e] = D[4 (l // 16) + e][l % 16] (rows in blocks of four, unlike FP64)."""
    b, res = _probe_onehot(lib, kind, width)
    for (la, sl), hits in res.items():
        i, k = la % 16, width * (la // 16) + sl
        # row i of D equals row k of B
        exp = {(16 * (i // 4) + j, i % 4): b[(16 * (k // width) + j) * width + (k % width)] for j in range(16)}
        got = {(l, e): v for (l, e, v) in hits}
        assert got == exp, (kind, la, sl)


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


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("M,N,K,tA,tB,batch", [(200, 77, 45, 0, 0, 2), (77, 200, 300, 1, 0, 1),
                                               (131, 129, 1000, 0, 1, 1), (45, 45, 133, 1, 1, 2)])
def test_reduced_precision_gemm(lib, mode, M, N, K, tA, tB, batch):
    """FP32 and split-BF16 products against numpy: the error of a K-term sum of
    products rounded to FP32 (2^-24), split BF16 with three products (~2^-16 per
    product) or with six (operands whole to 2^-24, dropped terms below 2^-24)
    stays below eps_mode * sqrt(K) * max|a| max|b| * 8."""
    import torch
    rng = np.random.default_rng(M + 13 * N + K + 1000 * mode)
    As = (K, M) if tA else (M, K)
    Bs = (N, K) if tB else (K, N)
    A = rng.standard_normal((batch,) + As)
    B = rng.standard_normal((batch,) + Bs)
    C0 = rng.standard_normal((batch, M, N))
    dA, dB, dC = (torch.tensor(x, device="cuda") for x in (A, B, C0))
    print(f"gemm mode={mode} M={M} N={N} K={K} tA={tA} tB={tB}", flush=True)
    st = lib.ris_test_gemm(mode, M, N, K, tA, tB, 1.3, _p(dA), As[1], int(np.prod(As)), _p(dB), Bs[1],
                           int(np.prod(Bs)), 0.5, _p(dC), N, M * N, batch)
    assert st == 0
    opA = A.transpose(0, 2, 1) if tA else A
    opB = B.transpose(0, 2, 1) if tB else B
    ref = 1.3 * opA @ opB + 0.5 * C0
    err = np.abs(dC.cpu().numpy() - ref).max()
    eps = 2.0 ** -16 if mode == 2 else 2.0 ** -24
    bound = 8 * eps * np.sqrt(K) * np.abs(A).max() * np.abs(B).max() * 1.3
    print("  err", err, "bound", bound, flush=True)
    assert err < bound


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("tB", [0, 1])
def test_gemm_long_rows_sliced(lib, tB, mode):
    """A k-fast operand whose rows are too far apart for 32-bit offsets across
    a 128-row tile (leading dimension 4.5e6 doubles, as (ai|P) at 500 atoms)
    is issued in row slices: untransposed A (tB = 0) or transposed B (tB = 1)."""
    import torch
    ld = 4_500_000
    rng = np.random.default_rng(77 + tB)
    if tB == 0:
        M, N, K = 140, 5, 24
        a = rng.standard_normal((M, K))
        b = rng.standard_normal((K, N))
        buf = torch.zeros((M - 1) * ld + K, dtype=torch.float64, device="cuda")
        buf.as_strided((M, K), (ld, 1)).copy_(torch.tensor(a))
        dA, lda = buf, ld
        dB, ldb = torch.tensor(b, device="cuda"), N
    else:
        M, N, K = 5, 140, 24
        a = rng.standard_normal((M, K))
        b = rng.standard_normal((N, K))
        buf = torch.zeros((N - 1) * ld + K, dtype=torch.float64, device="cuda")
        buf.as_strided((N, K), (ld, 1)).copy_(torch.tensor(b))
        dA, lda = torch.tensor(a, device="cuda"), K
        dB, ldb = buf, ld
    dC = torch.zeros((M, N), dtype=torch.float64, device="cuda")
    print(f"gemm long rows mode={mode} tB={tB} M={M} N={N} K={K} ld={ld}", flush=True)
    st = lib.ris_test_gemm(mode, M, N, K, 0, tB, 1.0, _p(dA), lda, 0, _p(dB), ldb, 0, 0.0, _p(dC), N, 0, 1)
    assert st == 0
    ref = a @ (b.T if tB else b)
    err = np.abs(dC.cpu().numpy() - ref).max()
    print("  err", err, flush=True)
    if mode == 0:
        assert err < 1e-12 * max(1.0, np.abs(ref).max())
    else:  # split BF16: the bound of test_reduced_precision_gemm
        assert err < 8 * 2.0 ** -16 * np.sqrt(K) * np.abs(a).max() * np.abs(b).max()
    del buf
    torch.cuda.empty_cache()
