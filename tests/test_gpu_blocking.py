"""Memory blocking over the auxiliary index on the GPU (ris_ctx_set_blocking).

The blocked (mu nu|P) and MO transforms and the blocked gradient + NAC
contraction are checked against the oracle (1e-8 Ha/Bohr, the FP64 bar) and
against the unblocked path of the same context, on block sizes that leave a
ragged last block, with p-type J shells beyond the exchange set (their
derivative shells carry the Coulomb part only), in FP64 and FP32."""
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
    c.set_blocking(0)
    c.close()


def _to(a, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device=dev)


def _run(ctx, prob, radii, block, outs, precision="fp64", dbg=False, jp=True):
    import torch
    m = prob.mol
    ctx.set_blocking(block)
    nJ, nK = ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
    dbg_t = torch.empty((nJ, m.nao, m.nao), dtype=torch.float64, device=ctx.device) if dbg else None
    ctx.int3c(_to(prob.C, ctx.device), _to(prob.eps, ctx.device), prob.nocc, 2.0, 0.25, precision=precision,
              dbg=dbg_t)
    rng = np.random.default_rng(11)
    V = rng.standard_normal((2,) + prob.X.shape[1:])
    mv = {op: ctx.response_matvec(op, _to(V, ctx.device)).cpu().numpy() for op in ("A+B", "A-B")}
    X = _to(prob.X, ctx.device)
    Y = None if prob.Y is None else _to(prob.Y, ctx.device)
    g, n = ctx.grad_nac_contract(X, Y, [i for (i, j) in outs if i == j], [(i, j) for (i, j) in outs if i != j])
    got = np.concatenate([g.cpu().numpy(), n.cpu().numpy()])
    return nJ, nK, got, mv, (dbg_t.cpu().numpy() if dbg else None)


def _outs(ns):
    return [(i, i) for i in range(ns)] + [(i, i + 1) for i in range(ns - 1)]


@pytest.mark.parametrize("block", [5, 7])
def test_blocked_fp64_vs_oracle_and_unblocked(ctx, radii, block):
    from oracle import ris_oracle as O
    prob = molgen.make_chain_problem(12, seed=5, nstate=3, tda=False)
    outs = _outs(prob.nstate)
    say(f"[gpu] blocking chain12_tddft block={block}: unblocked run")
    nJ, nK, ref_gpu, mv0, X0 = _run(ctx, prob, radii, 0, outs, dbg=True)
    say(f"[gpu]   nJ={nJ} nK={nK}; blocked run")
    assert nJ > nK > block  # several K blocks, p shells after the K set
    _, _, got, mv1, X1 = _run(ctx, prob, radii, block, outs, dbg=True)
    # the integrals themselves are computed block by block: identical
    assert np.array_equal(X0, X1)
    for op in mv0:
        d = np.abs(mv1[op] - mv0[op]).max()
        say(f"[gpu]   matvec {op} blocked - unblocked {d:.2e} (max {np.abs(mv0[op]).max():.2e})")
        assert d <= 1e-12 * np.abs(mv0[op]).max()
    ref = O.grad_nac(prob, radii, outs, j_p_on_heavy=True)
    e_or = np.abs(got - ref).max()
    e_un = np.abs(got - ref_gpu).max()
    say(f"[gpu]   grad/NAC blocked vs oracle {e_or:.2e}, vs unblocked {e_un:.2e} (max {np.abs(ref).max():.2e})")
    assert e_or <= 1e-8
    assert e_un <= 1e-12
    assert np.abs(got.sum(1)).max() <= 1e-10


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_blocked_reduced_precision_vs_unblocked(ctx, radii, precision):
    prob = molgen.make_chain_problem(30, seed=8, nstate=3, tda=False)
    outs = _outs(prob.nstate)
    say(f"[gpu] blocking chain30_tddft {precision}: unblocked run")
    _, nK, ref_gpu, _, _ = _run(ctx, prob, radii, 0, outs, precision=precision)
    blk = max(2, nK // 3 + 1)
    say(f"[gpu]   blocked run (block {blk} of nK={nK})")
    _, _, got, _, _ = _run(ctx, prob, radii, blk, outs, precision=precision)
    d = np.abs(got - ref_gpu).max()
    say(f"[gpu]   {precision} blocked vs unblocked {d:.2e} (max {np.abs(ref_gpu).max():.2e})")
    # FP32: the same roundings in both paths.  Split BF16: the blocked path
    # forms H_UO as the transpose of H_OU, which swaps the operands of the
    # hi*lo and lo*hi partial products and so their FP32 summation order; the
    # two results differ at the mode's own rounding level (its error against
    # FP64 is ~1e-7 Ha/Bohr here)
    assert d <= (1e-10 if precision == "fp32" else 1e-7)
    assert np.abs(got.sum(1)).max() <= 1e-9


def test_budget_forces_blocks(ctx, radii):
    """A context whose HBM budget holds only the blocked footprint that
    ris_plan_bytes gives for 4-function blocks completes the request (the
    calls choose blocks by themselves) with the unblocked results."""
    from paper_2511_18233_amd import RisContext
    from paper_2511_18233_amd.ris import request_bytes
    prob = molgen.make_chain_problem(12, seed=5, nstate=3, tda=False)
    outs = _outs(prob.nstate)
    m = prob.mol
    full = request_bytes(m.Z, m.shell_atom, m.shell_l, radii, m.nao, prob.nocc, prob.nstate, 2, len(outs),
                         xyz=m.xyz, shell_exp=m.shell_exp)
    plan = request_bytes(m.Z, m.shell_atom, m.shell_l, radii, m.nao, prob.nocc, prob.nstate, 2, len(outs),
                         aux_block=4, xyz=m.xyz, shell_exp=m.shell_exp)
    say(f"[gpu] budget-forced blocking: unblocked plan {full} B, 4-function blocks {plan} B")
    assert plan < full
    _, _, ref_gpu, mv0, _ = _run(ctx, prob, radii, 0, outs)
    small = RisContext(0, hbm_budget=plan)
    try:
        _, _, got, mv1, _ = _run(small, prob, radii, 0, outs)
        held = small.bytes_held
    finally:
        small.close()
    say(f"[gpu]   held {held} B of {plan}")
    assert held <= plan
    for op in mv0:
        assert np.abs(mv1[op] - mv0[op]).max() <= 1e-12 * np.abs(mv0[op]).max()
    d = np.abs(got - ref_gpu).max()
    say(f"[gpu]   budget-blocked vs unblocked {d:.2e}")
    assert d <= 1e-12


def test_blocked_tda_s_only_screen_off(ctx, radii):
    """TDA amplitudes (Y = NULL), an s-only auxiliary set (J = K: no
    Coulomb-only shells after the blocks) and the shell-pair screen off."""
    from oracle import ris_oracle as O
    prob = molgen.make_problem("ring12")
    outs = _outs(prob.nstate)
    try:
        ctx.set_screening(0.0)
        say("[gpu] blocking ring12 (TDA, s-only aux, screen off): unblocked run")
        nJ, nK, ref_gpu, _, _ = _run(ctx, prob, radii, 0, outs, jp=False)
        assert nJ == nK
        say("[gpu]   blocked run (block 5)")
        _, _, got, _, _ = _run(ctx, prob, radii, 5, outs, jp=False)
    finally:
        ctx.set_screening(1e-15)
    ref = O.grad_nac(prob, radii, outs, j_p_on_heavy=False)
    e_or, e_un = np.abs(got - ref).max(), np.abs(got - ref_gpu).max()
    say(f"[gpu]   blocked vs oracle {e_or:.2e}, vs unblocked {e_un:.2e}")
    assert e_or <= 1e-8
    assert e_un <= 1e-12
