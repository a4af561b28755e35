"""ris terms of the Z-vector right-hand side on the GPU (Appendix A.3) against
the oracle's four-index construction, and the whole ris Z-vector step (these
terms' VO - OV^T block solved with the ris (A+B), Sec. 4.2) against the
oracle's dense solve.

Bars: |G_gpu - G_oracle| <= 1e-10 max|G| (FP64 products of integrals that
agree to 1e-12 relative, through two MO transforms and one product);
Z within 1e-8 max|Z| (the solve's own bar)."""
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


CASES = [("ring12", lambda: molgen.make_problem("ring12"), False, [(0, 0), (1, 1), (0, 1), (1, 2)]),
         ("chain12_tddft", lambda: molgen.make_chain_problem(12, 5, 3, tda=False), True, [(0, 0), (2, 2), (0, 1)])]


@pytest.mark.parametrize("block", [0, 5])
@pytest.mark.parametrize("name,make,jp,pairs", CASES, ids=[c[0] for c in CASES])
def test_zrhs_vs_oracle_and_zvector(ctx, radii, name, make, jp, pairs, block):
    """block > 0: the integrals recomputed in blocks of at most 5 auxiliary
    functions (whole shells), as at sizes whose (mu nu|P) does not fit."""
    import torch
    from oracle import ris_oracle as O
    prob = make()
    m = prob.mol
    dev = ctx.device
    ctx.set_blocking(block)
    say(f"[gpu] zrhs {name}: aux_build + int3c (block {block})")
    ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
    ctx.int3c(torch.as_tensor(prob.C, device=dev), torch.as_tensor(prob.eps, device=dev), prob.nocc, 2.0, 0.25)
    X = torch.as_tensor(prob.X, device=dev)
    Y = None if prob.Y is None else torch.as_tensor(prob.Y, device=dev)
    say(f"[gpu] zrhs {name}: pairs {pairs}")
    G = ctx.zrhs_contract(X, Y, pairs).cpu().numpy()
    S = O.setup(m, radii, j_p_on_heavy=jp)
    ref = O.zrhs_ris_terms(S, prob.C, prob.nocc, prob.X, prob.Y, pairs)
    err = np.abs(G - ref).max()
    say(f"[gpu]   {name}: max|dG| {err:.2e} (max|G| {np.abs(ref).max():.2e})")
    assert err <= 1e-10 * np.abs(ref).max()
    # the ris Z-vector step: rhs = VO block - OV block^T, solved with the ris (A+B)
    o = prob.nocc
    rhs_ref = ref[:, o:, :o] - ref[:, :o, o:].transpose(0, 2, 1)
    rhs = torch.as_tensor(np.ascontiguousarray(G[:, o:, :o] - G[:, :o, o:].transpose(0, 2, 1)), device=dev)
    Z, it, res = ctx.zvector_solve(rhs, tol=1e-12, maxit=2000)
    Zref = O.zvector_solve(S, prob.C, prob.eps, prob.nocc, rhs_ref)
    zerr = np.abs(Z.cpu().numpy() - Zref).max()
    say(f"[gpu]   {name}: Z-vector {it} iterations, max|dZ| {zerr:.2e} (max|Z| {np.abs(Zref).max():.2e})")
    assert zerr <= 1e-8 * np.abs(Zref).max()
    ctx.set_blocking(0)


def test_zrhs_errors(ctx, radii):
    import torch
    from paper_2511_18233_amd.ris import RisError
    prob = molgen.make_problem("ring12")
    m = prob.mol
    ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, False)
    ctx.int3c(torch.as_tensor(prob.C, device=ctx.device), torch.as_tensor(prob.eps, device=ctx.device), prob.nocc,
              2.0, 0.25)
    X = torch.as_tensor(prob.X, device=ctx.device)
    with pytest.raises(RisError, match="INVALID"):
        ctx.zrhs_contract(X, None, [(0, 5)])
    G = ctx.zrhs_contract(X, None, np.zeros((0, 2), dtype=np.int32))
    assert G.shape[0] == 0
