"""CPU-side checks of the C ABI: the library builds, loads and exports every
entry point that include/ris.h declares.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_symbols():
    syms = set()
    for h in sorted(os.listdir(INCLUDE)):
        if h.endswith(".h"):
            txt = open(os.path.join(INCLUDE, h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            syms |= set(re.findall(r"\b(ris_[a-z0-9_]+)\s*\(", txt))
    return sorted(syms)


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for name in ("ris_aux_build", "ris_int3c", "ris_response_matvec", "ris_grad_contract", "ris_nac_contract"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2511_18233_amd import ris
    if not os.path.exists(ris.LIB_PATH):
        pytest.skip("libris_hip.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(ris.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(ris.EXPORTS) == set(declared_symbols())


def test_binding_refuses_without_gpu():
    import torch
    from paper_2511_18233_amd import RisContext
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        RisContext(0)


def _plan(name, block):
    import numpy as np
    import molgen
    from paper_2511_18233_amd.ris import request_bytes
    kind, natm, basis, ns, _ = molgen.WORKLOADS[name]
    m = molgen.make_molecule(kind, natm, basis, np.random.default_rng(molgen.WORKLOAD_SEED[name]))
    nocc = m.nelec // 2
    return request_bytes(m.Z, m.shell_atom, m.shell_l, molgen.radii_bohr_table(), m.nao, nocc, ns, ns, 2 * ns - 1,
                         aux_block=block, xyz=m.xyz, shell_exp=m.shell_exp)


def test_hbm_planner_host_sizing():
    """ris_plan_bytes (host-only): blocking over the auxiliary index shrinks
    the footprint monotonically with the block size; the 500-atom request
    does not fit one 288 GB GPU unblocked but does with 100-function blocks."""
    from paper_2511_18233_amd import ris
    if not os.path.exists(ris.LIB_PATH):
        pytest.skip("libris_hip.so not built (run __graft_entry__.build())")
    full = _plan("chain200", 0)
    sizes = [_plan("chain200", b) for b in (8, 16, 32, 64, 128)]
    assert all(a <= b for a, b in zip(sizes, sizes[1:]))
    assert sizes[-1] < full
    assert 70e9 < full < 90e9
    assert _plan("chain500", 0) > 288e9
    assert _plan("chain500", 100) < 0.9 * 288e9
    assert _plan("chain500", -1) == 0


def test_plan_counts_the_screened_pairs():
    """ris_plan_bytes holds, per chunk of 4 outputs, the compact copy of the
    s-shell weights over the AO shell pairs the default screen keeps
    (prefactor exp(-ab/(a+b)|A-B|^2) >= 1e-15; diagonal blocks whole): with the
    geometry given, the 199-atom plan is smaller than the all-pairs bound by
    4 x (function pairs the screen drops) x nK x 8 bytes, counted here in numpy."""
    import numpy as np
    import molgen
    from paper_2511_18233_amd import ris
    if not os.path.exists(ris.LIB_PATH):
        pytest.skip("libris_hip.so not built (run __graft_entry__.build())")
    kind, natm, basis, ns, _ = molgen.WORKLOADS["chain200"]
    m = molgen.make_molecule(kind, natm, basis, np.random.default_rng(molgen.WORKLOAD_SEED["chain200"]))
    nocc = m.nelec // 2
    args = (m.Z, m.shell_atom, m.shell_l, molgen.radii_bohr_table(), m.nao, nocc, ns, ns, 2 * ns - 1)
    bound = ris.request_bytes(*args)
    plan = ris.request_bytes(*args, xyz=m.xyz, shell_exp=m.shell_exp)
    sl = np.asarray(m.shell_l)
    c = np.asarray(m.xyz)[np.asarray(m.shell_atom)]
    e = np.asarray(m.shell_exp)
    d2 = ((c[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    keep = np.exp(-e[:, None] * e[None, :] / (e[:, None] + e[None, :]) * d2) >= 1e-15
    nf = np.array([1, 3, 6])[sl]
    pairs = np.tril(np.ones_like(keep)) * nf[:, None] * nf[None, :]
    dropped = int((pairs * ~keep).sum())
    assert dropped > 0
    expect = 4 * dropped * len(m.Z) * 8  # nK = one s function per atom
    assert abs((bound - plan) - expect) <= 4096, (bound - plan, expect)
