"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.  Tolerances: the FP64 path must match the oracle
within 1e-8 Ha/Bohr on gradients and NAC numerators (absolute); integrals
within 1e-12 and matvecs within 1e-10 relative to the largest element (FP64
rounding of sums over ~1e3-1e5 terms, amplified by the auxiliary metric's
condition number of up to ~1e5 in M^-1)."""
import sys

import numpy as np
import pytest

import molgen
from oracle import ris_oracle as O

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def ctx(torch_dev):
    from paper_2511_18233_amd import RisContext
    c = RisContext(0)
    yield c
    c.close()


def _to(t, dev):
    import torch
    return None if t is None else torch.as_tensor(np.ascontiguousarray(t), device=dev)


def _setup(ctx, prob, radii, jp, dbg=False):
    import torch
    m = prob.mol
    say(f"[gpu] aux_build natm={m.natm} nao={m.nao} jp={jp}")
    nJ, nK = ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
    C = _to(prob.C, ctx.device)
    eps = _to(prob.eps, ctx.device)
    dbg_t = torch.empty((nJ, m.nao, m.nao), dtype=torch.float64, device=ctx.device) if dbg else None
    say(f"[gpu] int3c nJ={nJ} nK={nK} nocc={prob.nocc}")
    ctx.int3c(C, eps, prob.nocc, 2.0, 0.25, dbg=dbg_t)
    torch.cuda.synchronize()
    return dbg_t


CASES = {
    "ring12": (lambda: molgen.make_problem("ring12"), False),
    "tiny_mixed_tddft": (lambda: molgen.make_tiny_problem(21, natm=4, lmax=2, nstate=3, tda=False), True),
    "tiny_s_only": (lambda: molgen.make_tiny_problem(22, natm=3, lmax=0, nstate=2, tda=False), False),
    "chain12_tddft": (lambda: molgen.make_chain_problem(12, seed=5, nstate=3, tda=False), True),
}


@pytest.mark.parametrize("case", list(CASES))
def test_int3c_parity(ctx, radii, case):
    make, jp = CASES[case]
    prob = make()
    dbg = _setup(ctx, prob, radii, jp, dbg=True).cpu().numpy()
    S = O.setup(prob.mol, radii, j_p_on_heavy=jp)
    ref = S.int3J
    err = np.abs(dbg - ref).max()
    say(f"[gpu] int3c {case} max err {err:.3e} (max {np.abs(ref).max():.3e})")
    assert err <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("case", list(CASES))
def test_matvec_parity(ctx, radii, case):
    make, jp = CASES[case]
    prob = make()
    _setup(ctx, prob, radii, jp)
    S = O.setup(prob.mol, radii, j_p_on_heavy=jp)
    rng = np.random.default_rng(3)
    V = rng.standard_normal((3,) + prob.X.shape[1:])
    Vd = _to(V, ctx.device)
    for op in ("A", "B", "A+B", "A-B"):
        say(f"[gpu] matvec {case} {op}")
        got = ctx.response_matvec(op, Vd).cpu().numpy()
        ref = O.response_matvec(S, prob.C, prob.eps, prob.nocc, V, op)
        err = np.abs(got - ref).max()
        say(f"[gpu]   err {err:.3e} (max {np.abs(ref).max():.3e})")
        assert err <= 1e-10 * np.abs(ref).max(), op


def _outputs(ns):
    outs = [(i, i) for i in range(ns)] + [(i, i + 1) for i in range(ns - 1)]
    return outs


@pytest.mark.parametrize("case", list(CASES))
def test_grad_nac_parity(ctx, radii, case):
    make, jp = CASES[case]
    prob = make()
    _setup(ctx, prob, radii, jp)
    outs = _outputs(prob.nstate)
    X = _to(prob.X, ctx.device)
    Y = _to(prob.Y, ctx.device)
    say(f"[gpu] grad {case} nout={len(outs)}")
    g = ctx.grad_contract(X, Y, [i for (i, j) in outs if i == j]).cpu().numpy()
    n = ctx.nac_contract(X, Y, [(i, j) for (i, j) in outs if i != j]).cpu().numpy()
    got = np.concatenate([g, n])
    ref = O.grad_nac(prob, radii, outs, j_p_on_heavy=jp)
    err = np.abs(got - ref).max()
    say(f"[gpu]   max |dgrad| {err:.3e} (max |grad| {np.abs(ref).max():.3e})")
    assert err <= GRAD_TOL
    # translational invariance of the GPU result itself
    assert np.abs(got.sum(1)).max() <= 1e-10


MIXED_CASES = {
    "ring12": (CASES["ring12"][0], False),
    "chain12_tddft": (CASES["chain12_tddft"][0], True),
    "chain30_tddft": (lambda: molgen.make_chain_problem(30, seed=8, nstate=3, tda=False), True),
    # 4 atoms 1.7-3.5 Bohr apart (a compressed cluster, far from the chain
    # workloads): gradients up to 0.16 Ha/Bohr, ten times the chains'
    "tiny_cluster": (CASES["tiny_mixed_tddft"][0], True),
    # H2 with one occupied orbital: 3o = 3 against the 32 columns of a bf16
    # plane (nearly all padding) and one tile everywhere
    "h2": (lambda: molgen.make_tiny_problem(21, natm=2, lmax=1, nstate=2, tda=False, elements=(1, 1)), False),
}
# What each mode claims (reading A18): every mode holds 1e-6 Ha/Bohr on the
# workload-shaped molecules (ring, chains); on any input the error is relative
# to the largest output, |d| <= eps_mode max|g|, with eps = 2e-5 for FP32 and the
# six-product split (24-bit operands, FP32 accumulation, amplified about a
# hundredfold by the cancellation in the three-term derivative) and 1e-3 for the
# three-product split (16-bit operands).  The compressed cluster, with gradients
# ten times the chains', is held to the relative bound.
MIXED_BAR = {"fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 1e-6}
MIXED_REL_BAR = {"fp32": 2e-5, "bf16x6": 2e-5, "bf16x3": 1e-3}
REL_CASES = ("tiny_cluster", "h2")
# "+transforms" claims, relative to max|g| on the workload shapes: FP32 2e-4
# (measured 4-11e-5), split BF16 x3 1e-2 (measured 1.5-4e-3)
TRANSFORMS_REL_BAR = {"fp32": 2e-4, "bf16x3": 1e-2}


@pytest.mark.parametrize("precision", ["fp32", "bf16x6", "bf16x3", "fp32+transforms", "bf16x3+transforms"])
@pytest.mark.parametrize("case", list(MIXED_CASES))
def test_mixed_precision_error(ctx, radii, case, precision):
    """Reduced-precision exchange contractions against the FP64 oracle, the
    error of each case and mode printed.  "+transforms" also runs the MO
    transforms of (mu nu|P) in the mode: that costs about two digits (FP32: 1e-4
    of max|g| on the ring and the chains, 4e-3 on the compressed cluster), so the
    flag is opt-in, makes relative claims (TRANSFORMS_REL_BAR) and is checked on
    the workload shapes."""
    import torch
    make, jp = MIXED_CASES[case]
    if "+" in precision and case in REL_CASES:
        pytest.skip("the transforms flag makes no claim off the workload shapes (FP32: 4e-3 of max|g| on the "
                    "compressed cluster)")
    prob = make()
    m = prob.mol
    ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
    say(f"[gpu] int3c {case} precision={precision}")
    ctx.int3c(_to(prob.C, ctx.device), _to(prob.eps, ctx.device), prob.nocc, 2.0, 0.25, precision=precision)
    outs = _outputs(prob.nstate)
    X = _to(prob.X, ctx.device)
    Y = _to(prob.Y, ctx.device)
    g, n = ctx.grad_nac_contract(X, Y, [i for (i, j) in outs if i == j], [(i, j) for (i, j) in outs if i != j])
    got = np.concatenate([g.cpu().numpy(), n.cpu().numpy()])
    ref = O.grad_nac(prob, radii, outs, j_p_on_heavy=jp)
    err = np.abs(got - ref).max()
    gmax = np.abs(ref).max()
    say(f"[gpu]   {case} {precision}: max |dgrad| {err:.3e} Ha/Bohr (max |grad| {gmax:.3e}, rel {err / gmax:.2e})")
    base = precision.split("+")[0]
    if "+" in precision:
        assert err <= TRANSFORMS_REL_BAR[base] * gmax
        return
    assert err <= MIXED_REL_BAR[base] * gmax
    if case not in REL_CASES:
        assert err <= MIXED_BAR[base]
    torch.cuda.synchronize()


# Matvecs in the reduced modes (exchange products in the mode, the rest FP64):
# relative to the largest element, about ten times the operand rounding of the
# mode (2^-24 for FP32 and the six-product split, 2^-17 for the three-product
# split) to allow for FP32 accumulation over o or v terms; measured on these
# cases: at most 8e-8 (FP32, six products) and 1.9e-6 (three products)
MATVEC_REL_BAR = {"fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 2e-5}


@pytest.mark.parametrize("precision", ["fp32", "bf16x6", "bf16x3"])
@pytest.mark.parametrize("case", ["ring12", "chain12_tddft"])
def test_matvec_reduced_precision(ctx, radii, case, precision):
    """A, B, A+B and A-B matvecs with the exchange contractions in each
    reduced mode against the FP64 oracle, the error of each printed (in the
    split modes the per-vector products run on bf16 planes)."""
    import torch
    make, jp = CASES[case]
    prob = make()
    m = prob.mol
    ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
    say(f"[gpu] int3c {case} precision={precision}")
    ctx.int3c(_to(prob.C, ctx.device), _to(prob.eps, ctx.device), prob.nocc, 2.0, 0.25, precision=precision)
    S = O.setup(prob.mol, radii, j_p_on_heavy=jp)
    rng = np.random.default_rng(4)
    V = rng.standard_normal((3,) + prob.X.shape[1:])
    Vd = _to(V, ctx.device)
    for op in ("A", "B", "A+B", "A-B"):
        say(f"[gpu] matvec {case} {precision} {op}")
        got = ctx.response_matvec(op, Vd).cpu().numpy()
        ref = O.response_matvec(S, prob.C, prob.eps, prob.nocc, V, op)
        err = np.abs(got - ref).max()
        say(f"[gpu]   err {err:.3e} (max {np.abs(ref).max():.3e}, rel {err / np.abs(ref).max():.2e})")
        assert err <= MATVEC_REL_BAR[precision] * np.abs(ref).max(), op
    torch.cuda.synchronize()


def test_combined_call_matches_separate_calls(ctx, radii):
    prob = molgen.make_chain_problem(12, seed=5, nstate=3, tda=False)
    _setup(ctx, prob, radii, True)
    X = _to(prob.X, ctx.device)
    Y = _to(prob.Y, ctx.device)
    say("[gpu] combined grad+nac chain12")
    g1 = ctx.grad_contract(X, Y, [0, 2]).cpu().numpy()
    n1 = ctx.nac_contract(X, Y, [(0, 1), (2, 1)]).cpu().numpy()
    g2, n2 = ctx.grad_nac_contract(X, Y, [0, 2], [(0, 1), (2, 1)])
    assert np.array_equal(g1, g2.cpu().numpy())
    assert np.array_equal(n1, n2.cpu().numpy())


def test_determinism_and_tda(ctx, radii, torch_dev):
    import torch
    prob = molgen.make_problem("ring12")
    _setup(ctx, prob, radii, False)
    X = _to(prob.X, ctx.device)
    say("[gpu] determinism ring12")
    a = ctx.nac_contract(X, None, [(0, 1), (1, 2)]).cpu().numpy()
    b = ctx.nac_contract(X, None, [(0, 1), (1, 2)]).cpu().numpy()
    assert np.array_equal(a, b)
    c = ctx.nac_contract(X, torch.zeros_like(X), [(0, 1), (1, 2)]).cpu().numpy()
    assert np.array_equal(a, c)


def test_nac_division_and_degenerate(ctx, radii):
    from paper_2511_18233_amd import RisError
    prob = molgen.make_problem("ring12")
    _setup(ctx, prob, radii, False)
    X = _to(prob.X, ctx.device)
    num = ctx.nac_contract(X, None, [(0, 1)]).cpu().numpy()
    omega = np.array([0.20, 0.25, 0.30])
    d = ctx.nac_contract(X, None, [(0, 1)], omega=omega).cpu().numpy()
    assert np.allclose(d, num / 0.05, rtol=1e-14, atol=0)
    with pytest.raises(RisError) as e:
        ctx.nac_contract(X, None, [(0, 1)], omega=np.array([0.2, 0.2, 0.3]))
    assert e.value.code == 5
    keep = ctx.nac_contract(X, None, [(0, 1)], omega=np.array([0.2, 0.2, 0.3]), allow_degenerate=True)
    assert np.array_equal(keep.cpu().numpy(), num)


def test_error_paths(radii, torch_dev):
    from paper_2511_18233_amd import RisContext, RisError
    c = RisContext(0)
    prob = molgen.make_problem("ring12")
    X = _to(prob.X, c.device)
    with pytest.raises(RisError) as e:
        c.grad_contract(X, None, [0])
    assert e.value.code == 6  # order
    m = prob.mol
    # two atoms on the same spot: singular metric
    xyz = m.xyz.copy()
    xyz[1] = xyz[0]
    with pytest.raises(RisError) as e:
        c.aux_build(m.Z, xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, False)
    assert e.value.code == 4
    bad_l = m.shell_l.copy()
    bad_l[0] = 3
    with pytest.raises(RisError) as e:
        c.aux_build(m.Z, m.xyz, m.shell_atom, bad_l, m.shell_exp, radii, 0.2, False)
    assert e.value.code == 2
    c.close()
    # an HBM budget below even the smallest blocks is refused, not attempted
    # (chain30: its kept MO blocks alone exceed 1 MiB)
    prob = molgen.make_chain_problem(30, seed=8, nstate=2, tda=False)
    m = prob.mol
    small = RisContext(0, hbm_budget=1 << 20)
    small.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, True)
    with pytest.raises(RisError) as e:
        small.int3c(_to(prob.C, small.device), _to(prob.eps, small.device), prob.nocc)
    assert e.value.code == 3
    small.close()
