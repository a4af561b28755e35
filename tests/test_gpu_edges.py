"""Edge cases of the hot path on the GPU, each against the oracle where there
is something to compare: the smallest molecule (H2, one occupied orbital),
empty request lists, a pure functional (c_x = 0, no exchange part), a single
state, and the shell-pair screen switched off.
Bar: 1e-8 Ha/Bohr as for the main parity cases."""
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


def _run(ctx, prob, radii, jp, outs, cx=0.25):
    import torch
    m = prob.mol
    dev = ctx.device
    ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
    ctx.int3c(torch.as_tensor(prob.C, device=dev), torch.as_tensor(prob.eps, device=dev), prob.nocc, 2.0, cx)
    X = torch.as_tensor(prob.X, device=dev)
    Y = None if prob.Y is None else torch.as_tensor(prob.Y, device=dev)
    grads = [i for (i, j) in outs if i == j]
    pairs = [(i, j) for (i, j) in outs if i != j]
    g, n = ctx.grad_nac_contract(X, Y, grads, pairs)
    return g.cpu().numpy(), n.cpu().numpy()


def test_h2_single_occupied(ctx, radii):
    from oracle import ris_oracle as O
    prob = molgen.make_tiny_problem(21, natm=2, lmax=1, nstate=2, tda=False, elements=(1, 1))
    assert prob.nocc == 1
    say(f"[gpu] H2: nao={prob.mol.nao} nocc={prob.nocc}")
    outs = [(0, 0), (1, 1), (0, 1)]
    g, n = _run(ctx, prob, radii, False, outs)
    ref = O.grad_nac(prob, radii, outs, j_p_on_heavy=False)
    err = max(np.abs(g - ref[:2]).max(), np.abs(n - ref[2:]).max())
    say(f"[gpu]   H2 max|d| {err:.2e}")
    assert err <= 1e-8
    assert np.abs(g.sum(1)).max() <= 1e-10


def test_pure_functional_and_single_state(ctx, radii):
    from oracle import ris_oracle as O
    prob = molgen.make_tiny_problem(22, natm=3, lmax=2, nstate=1, tda=False)
    say("[gpu] c_x = 0, one state")
    g, n = _run(ctx, prob, radii, True, [(0, 0)], cx=0.0)
    ref = O.grad_nac(prob, radii, [(0, 0)], c_x=0.0)
    assert n.shape[0] == 0
    err = np.abs(g - ref).max()
    say(f"[gpu]   c_x=0 max|d| {err:.2e}")
    assert err <= 1e-8


def test_empty_lists_and_screen_off(ctx, radii):
    import torch
    prob = molgen.make_problem("ring12")
    say("[gpu] empty lists")
    g, n = _run(ctx, prob, radii, False, [])
    assert g.shape[0] == 0 and n.shape[0] == 0
    V = torch.zeros((0,) + prob.X.shape[1:], dtype=torch.float64, device=ctx.device)
    out = ctx.response_matvec("A+B", V)
    assert out.shape[0] == 0
    # the default screen drops only pairs with a product prefactor below 1e-15: switching it off
    # changes the 12-atom results by far less than the parity bar
    nsh = len(prob.mol.shell_l)
    g1, n1 = _run(ctx, prob, radii, False, [(0, 0), (0, 1)])
    try:
        kept = ctx.set_screening(0.0)
        assert kept == nsh * nsh
        g0, n0 = _run(ctx, prob, radii, False, [(0, 0), (0, 1)])
    finally:
        ctx.set_screening(1e-15)
    say(f"[gpu]   screen on/off max|d| {max(np.abs(g1 - g0).max(), np.abs(n1 - n0).max()):.2e}")
    assert np.abs(g1 - g0).max() <= 1e-12 and np.abs(n1 - n0).max() <= 1e-12
