"""TDA-ris excitation energies by block Davidson on the GPU against the
oracle's dense eigendecomposition (Sec. 2.1 eq. casida with B = 0, the ris
kernel in A), and the one-workgroup Jacobi eigensolver of its subspace
against numpy.

Bars: the Jacobi eigenvalues within 1e-12 of the largest magnitude and
A y = w y to 1e-12; Davidson with residual tolerance 1e-9: eigenvalues within
1e-10 Ha of the oracle's (the error is second order in the residual), each
vector parallel to the oracle's to 1e-9 (|<x, x_ref>| >= 1 - 1e-9; roots are
non-degenerate here, and the sign is free), and A x - w x <= 1e-8 with the
oracle's dense A."""
import ctypes
import sys

import numpy as np
import pytest

import molgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_18233_amd import RisContext
    c = RisContext(0)
    yield c
    c.close()


@pytest.mark.parametrize("m", [1, 2, 7, 32, 95, 256])
def test_jacobi_small_eigensolver(m):
    import torch
    from paper_2511_18233_amd import ris
    lib = ris.load_library()
    rng = np.random.default_rng(m)
    M = rng.standard_normal((m, m))
    M = M + M.T
    if m >= 7:  # a repeated eigenvalue
        Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
        ev = np.sort(rng.standard_normal(m))
        ev[1] = ev[0]
        M = (Q * ev) @ Q.T
        M = 0.5 * (M + M.T)
    A = torch.as_tensor(M.copy(), device="cuda")
    w = torch.zeros(m, dtype=torch.float64, device="cuda")
    say(f"[gpu] jacobi m={m}")
    assert lib.ris_test_sym_eig(m, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(w.data_ptr())) == 0
    wg, Y = w.cpu().numpy(), A.cpu().numpy()
    ref = np.linalg.eigvalsh(M)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(wg - ref).max() <= 1e-12 * scale
    assert np.all(np.diff(wg) >= -1e-12 * scale)
    assert np.abs(Y @ Y.T - np.eye(m)).max() <= 1e-12
    assert np.abs(M @ Y.T - Y.T * wg[None, :]).max() <= 1e-12 * scale


def _setup(ctx, prob, radii, jp):
    import torch
    m = prob.mol
    ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
    ctx.int3c(torch.as_tensor(prob.C, device=ctx.device), torch.as_tensor(prob.eps, device=ctx.device), prob.nocc,
              2.0, 0.25)


CASES = [("ring12", lambda: molgen.make_problem("ring12"), False, 3),
         ("chain12", lambda: molgen.make_chain_problem(12, 5, 3, tda=True), True, 4)]


@pytest.mark.parametrize("name,make,jp,nroots", CASES, ids=[c[0] for c in CASES])
def test_davidson_vs_oracle(ctx, radii, name, make, jp, nroots):
    from oracle import ris_oracle as O
    prob = make()
    say(f"[gpu] davidson {name}: aux_build + int3c")
    _setup(ctx, prob, radii, jp)
    say(f"[gpu] davidson {name}: nroots={nroots}")
    w, X, it = ctx.tda_davidson(nroots, tol=1e-9, maxit=200)
    X = X.cpu().numpy().reshape(nroots, -1)
    S = O.setup(prob.mol, radii, j_p_on_heavy=jp)
    wr, Xr = O.tda_eigen(S, prob.C, prob.eps, prob.nocc, nroots)
    A = O.dense_a(S, prob.C, prob.eps, prob.nocc)
    Xr = Xr.reshape(nroots, -1)
    dw = np.abs(w - wr).max()
    par = np.abs(np.sum(X * Xr, axis=1))
    res = max(np.abs(A @ X[k] - w[k] * X[k]).max() for k in range(nroots))
    say(f"[gpu]   {name}: {it} iterations, max|dw| {dw:.2e}, min|<x,xref>| {par.min():.12f}, residual {res:.2e}")
    assert dw <= 1e-10
    assert par.min() >= 1.0 - 1e-9
    assert res <= 1e-8
    assert np.abs(np.linalg.norm(X, axis=1) - 1.0).max() <= 1e-12


def test_davidson_edges_and_determinism(ctx, radii):
    from paper_2511_18233_amd.ris import RisError
    prob = molgen.make_problem("ring12")
    _setup(ctx, prob, radii, False)
    say("[gpu] davidson determinism, limits, errors")
    w1, X1, i1 = ctx.tda_davidson(2, tol=1e-8)
    w2, X2, i2 = ctx.tda_davidson(2, tol=1e-8)
    assert i1 == i2 and np.array_equal(w1, w2) and bool((X1 == X2).all())
    w3, X3, i3 = ctx.tda_davidson(2, tol=1e-12, maxit=1, allow_noconv=True)
    assert i3 == 1
    with pytest.raises(RisError, match="NOCONV"):
        ctx.tda_davidson(2, tol=1e-12, maxit=1)
    with pytest.raises(RisError, match="INVALID"):
        ctx.tda_davidson(0)
    with pytest.raises(RisError, match="INVALID"):
        ctx.tda_davidson(2, max_space=3)
