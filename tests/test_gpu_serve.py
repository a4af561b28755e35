"""Serving loop on the GPU: requests that overlap on the device give the same
results as the same requests run alone (bitwise: each slot's work is the same
kernels with ordered reductions), the results match the FP64 oracle, and so
does the time-derivative coupling T_IJ = g_IJ . v the server returns."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_alone_equals_mixed_and_oracle(radii):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import ris_oracle as O
    from paper_2511_18233_amd.serve import GpuExecutor, Server, make_trace
    reqs = make_trace(6, 3, rate_hz=1e6, seed=4242, natm_range=(12, 24))
    print("[gpu] serve: alone", flush=True)
    alone = Server([GpuExecutor(0, 0, radii, "fp64")], 64 << 30)
    ra = alone.run_trace(reqs, realtime=False)
    alone.close()
    print("[gpu] serve: mixed", flush=True)
    mixed = Server([GpuExecutor(k, 0, radii, "fp64") for k in range(3)], 64 << 30)
    rm = mixed.run_trace(reqs, realtime=False)
    mixed.close()
    for r in reqs:
        a, m = ra[r.rid], rm[r.rid]
        assert a.error is None and m.error is None, (a.error, m.error)
        assert np.array_equal(a.grad, m.grad) and np.array_equal(a.nac, m.nac), r.rid
    # overlap happened: some request was admitted before an earlier one finished
    ends = sorted((x.admitted, x.done) for x in rm.values())
    assert any(ends[i + 1][0] < ends[i][1] for i in range(len(ends) - 1))
    # and the results are right
    r = reqs[0]
    import molgen
    prob = molgen.Problem(molgen.Molecule(r.Z, r.xyz, r.shell_atom, r.shell_l, r.shell_exp), r.C, r.eps, r.nocc,
                          r.X, r.Y)
    ref = O.grad_nac(prob, radii, [(0, 0), (1, 1), (0, 1)])
    got = np.concatenate([rm[0].grad, rm[0].nac])
    assert np.abs(got - ref).max() <= 1e-8
    # the time-derivative coupling the server returns, T_01 = g_01 . v (Sec. 5.4),
    # against the oracle's NAC numerator dotted with the request's velocities
    t_ref = float(np.sum(ref[2] * r.velocity))
    assert rm[0].tdc is not None and rm[0].tdc.shape == (1,)
    assert abs(rm[0].tdc[0] - t_ref) <= 1e-8 * np.abs(r.velocity).sum()


def test_served_phases_and_mecp_on_gpu_results(radii):
    """The surface-hopping consumers on what the GPU server returns (Sec. 3,
    last paragraph; Sec. 5.3): the trace draws an arbitrary sign per state at
    every step and aligns it to the previous step (md.phase_signs), so along a
    trajectory the amplitudes keep the first step's signs and consecutive
    served NAC numerators (geometry steps of 0.01 A) point the same way; every
    served result matches the oracle for the request's own amplitudes, and the
    MECP effective gradient built from the served gradients and NAC equals the
    one built from the oracle's."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import molgen
    from oracle import ris_oracle as O
    from paper_2511_18233_amd import md
    from paper_2511_18233_amd.serve import GpuExecutor, Server, make_trace
    ntraj, steps = 2, 3
    reqs = make_trace(ntraj * steps, ntraj, rate_hz=1e6, seed=777, natm_range=(10, 16), random_phase=True)
    print("[gpu] serve: phases", flush=True)
    srv = Server([GpuExecutor(0, 0, radii, "fp64")], 64 << 30)
    res = srv.run_trace(reqs, realtime=False)
    srv.close()
    first, prev = {}, {}
    for r in reqs:
        traj = r.rid % ntraj
        prob = molgen.Problem(molgen.Molecule(r.Z, r.xyz, r.shell_atom, r.shell_l, r.shell_exp), r.C, r.eps,
                              r.nocc, r.X, r.Y)
        ref = O.grad_nac(prob, radii, [(0, 0), (1, 1), (0, 1)])
        got = res[r.rid]
        assert got.error is None
        assert np.abs(np.concatenate([got.grad, got.nac]) - ref).max() <= 1e-8
        if traj in first:
            assert np.array_equal(r.X, first[traj]), "aligned amplitudes changed sign along the trajectory"
            assert np.sum(got.nac[0] * prev[traj]) > 0.0, "consecutive NACs flipped"
        else:
            first[traj] = r.X.copy()
        prev[traj] = got.nac[0]
        geff = md.mecp_effective_gradient(got.grad[0], got.grad[1], got.nac[0], -0.30, -0.28)
        gref = md.mecp_effective_gradient(ref[0], ref[1], ref[2], -0.30, -0.28)
        assert np.abs(geff - gref).max() <= 1e-7
