"""Allocation-free response matvec (ris_response_matvec_noalloc) through the C
ABI: its products equal those of ris_response_matvec on the same context, it
allocates no device memory (the context's held bytes do not move, also when
it is the first product of a fresh context), two calls in a row with the
second on a smaller input both match, and a request whose intermediates do
not fit the fixed scratch is refused with RIS_E_NOMEM while the allocating
entry point still serves it.  The same products are also held against the
FP64 oracle (1e-10 relative to the largest element, the matvec bar)."""
import sys

import numpy as np
import pytest

import molgen
from oracle import ris_oracle as O

pytestmark = pytest.mark.gpu

OPS = ("A", "B", "A+B", "A-B")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _context(prob, radii, jp):
    import torch
    from paper_2511_18233_amd import RisContext
    ctx = RisContext(0)
    m = prob.mol
    say(f"[noalloc] aux_build natm={m.natm} nao={m.nao} jp={jp}")
    ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
    C = torch.as_tensor(prob.C, device=ctx.device).contiguous()
    eps = torch.as_tensor(prob.eps, device=ctx.device).contiguous()
    ctx.int3c(C, eps, prob.nocc, 2.0, 0.25)
    torch.cuda.synchronize()
    return ctx


def _vectors(prob, nvec, seed):
    v = prob.C.shape[1] - prob.nocc
    return np.random.default_rng(seed).standard_normal((nvec, v, prob.nocc))


def _check(ctx, prob, radii, jp, V, label, oracle=True):
    import torch
    Vd = torch.as_tensor(V, device=ctx.device).contiguous()
    S = O.setup(prob.mol, radii, j_p_on_heavy=jp) if oracle else None
    for op in OPS:
        out = torch.full_like(Vd, float("nan"))
        held = ctx.bytes_held
        say(f"[noalloc] {label} op={op} nvec={V.shape[0]}")
        ctx.response_matvec_noalloc(op, Vd, out)
        torch.cuda.synchronize()
        assert ctx.bytes_held == held, "the allocation-free call changed the context's device memory"
        got = out.cpu().numpy()
        ref = ctx.response_matvec(op, Vd).cpu().numpy()
        scale = np.abs(ref).max()
        err = np.abs(got - ref).max()
        say(f"[noalloc] {label} op={op}: |noalloc - matvec| = {err:.3e} (max {scale:.3e})")
        assert np.isfinite(got).all()
        assert err <= 1e-13 * scale
        if oracle:
            o_ref = O.response_matvec(S, prob.C, prob.eps, prob.nocc, V, op)
            e2 = np.abs(got - o_ref).max()
            say(f"[noalloc] {label} op={op}: |noalloc - oracle| = {e2:.3e}")
            assert e2 <= 1e-10 * np.abs(o_ref).max()


def test_noalloc_matvec_two_calls(torch_dev, radii):
    # call 1: 30-atom chain, TDDFT, p auxiliary functions, 8 vectors; call 2: the
    # same context with 2 vectors; call 3: a smaller molecule (12-atom ring), 3 vectors
    big = molgen.make_chain_problem(30, seed=7, nstate=2, tda=False)
    ctx = _context(big, radii, True)
    held = ctx.bytes_held
    import torch
    Vd = torch.as_tensor(_vectors(big, 8, 1), device=ctx.device).contiguous()
    out = torch.empty_like(Vd)
    ctx.response_matvec_noalloc("A+B", Vd, out)      # first product of a fresh context
    torch.cuda.synchronize()
    assert ctx.bytes_held == held
    _check(ctx, big, radii, True, _vectors(big, 8, 1), "chain30 x8")
    _check(ctx, big, radii, True, _vectors(big, 2, 2), "chain30 x2")
    ctx.close()
    small = molgen.make_problem("ring12")
    ctx = _context(small, radii, False)
    _check(ctx, small, radii, False, _vectors(small, 3, 3), "ring12 x3")
    ctx.close()


def test_noalloc_matvec_refuses_oversized(torch_dev, radii):
    import torch
    from paper_2511_18233_amd.ris import RisError
    prob = molgen.make_chain_problem(110, seed=9, nstate=1, tda=True)
    ctx = _context(prob, radii, True)
    Vd = torch.as_tensor(_vectors(prob, 1, 4), device=ctx.device).contiguous()
    out = torch.empty_like(Vd)
    say(f"[noalloc] chain110 nocc={prob.nocc}: expecting RIS_E_NOMEM")
    with pytest.raises(RisError) as ei:
        ctx.response_matvec_noalloc("A", Vd, out)
    assert ei.value.code == 3 and "fixed scratch" in str(ei.value)
    ref = ctx.response_matvec("A", Vd)                 # the allocating entry point serves it
    torch.cuda.synchronize()
    assert torch.isfinite(ref).all()
    ctx.close()
