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
