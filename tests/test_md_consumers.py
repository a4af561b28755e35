"""Host-side consumers of gradients and NACs (Sec. 5.3 MECP effective
gradient, Sec. 5.4 time-derivative coupling, Sec. 3 phase determination):
properties that pin each formula."""
import numpy as np

import molgen
from paper_2511_18233_amd import md


def test_time_derivative_coupling():
    rng = np.random.default_rng(1)
    g = rng.standard_normal((7, 3))
    v = rng.standard_normal((7, 3))
    t = md.time_derivative_coupling(g, v)
    assert abs(t - sum(g[a] @ v[a] for a in range(7))) < 1e-13
    assert abs(md.time_derivative_coupling(g, 2.5 * v) - 2.5 * t) < 1e-12
    assert abs(md.time_derivative_coupling(-g, v) + t) < 1e-13      # g_JI = -g_IJ flips T
    try:
        md.time_derivative_coupling(g, v[:6])
        raise AssertionError("shape mismatch accepted")
    except ValueError:
        pass


def test_mecp_effective_gradient_projects_out_the_branching_plane():
    rng = np.random.default_rng(2)
    gi, gj, h = rng.standard_normal((3, 9, 3))
    ei, ej = -0.31, -0.27
    geff = md.mecp_effective_gradient(gi, gj, h, ei, ej)
    x1 = gj - gi
    f = (ej - ei) * x1 / np.linalg.norm(x1)
    pg = geff - f
    # the projected part is orthogonal to both plane vectors, and g_J - P g_J lies in the plane
    assert abs(np.sum(pg * x1)) < 1e-12 and abs(np.sum(pg * h)) < 1e-12
    B = md.branching_plane(x1, h)
    assert B.shape == (2, 27) and np.abs(B @ B.T - np.eye(2)).max() < 1e-13
    r = (gj - pg).ravel()
    assert np.linalg.norm(r - B.T @ (B @ r)) < 1e-12
    # a gradient already orthogonal to the plane passes unchanged (equal energies: f = 0)
    q = rng.standard_normal(27)
    q = (q - B.T @ (B @ q)).reshape(9, 3)
    out = md.mecp_effective_gradient(q - x1, q, h, 0.0, 0.0)   # x1 = q - (q - x1): same plane
    assert np.abs(out - q).max() < 1e-12
    # NAC parallel to x1: the plane has one direction
    assert md.branching_plane(x1, 3.0 * x1).shape[0] == 1


def test_phase_signs_recover_state_and_orbital_sign_flips():
    p = molgen.make_problem("ring12")
    S = molgen.overlap_matrix(p.mol)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4,) + p.X.shape[1:])
    # the next step: some MOs change sign, some states change sign
    d = np.where(rng.random(p.C.shape[1]) < 0.4, -1.0, 1.0)
    C2 = p.C * d[None, :]
    flips = np.array([1.0, -1.0, -1.0, 1.0])
    o = p.nocc
    X2 = flips[:, None, None] * X * d[o:][None, :, None] * d[:o][None, None, :]
    s = md.phase_signs(X, X2, p.C, C2, S, o)
    assert np.array_equal(s, flips)
    # applying the signs restores continuity: a second call gives +1 everywhere
    X3 = s[:, None, None] * X2
    assert np.array_equal(md.phase_signs(X, X3, p.C, C2, S, o), np.ones(4))


def test_trace_amplitudes_are_phase_aligned():
    """The serving trace draws an arbitrary sign per state at every step and
    aligns it to the previous step: along a trajectory the aligned amplitudes
    stay those of its first step, and every request carries velocities."""
    from paper_2511_18233_amd.serve import make_trace
    reqs = make_trace(12, 2, 1.0, seed=5, natm_range=(10, 14))
    for t in range(2):
        xs = [r.X for r in reqs if r.rid % 2 == t]
        assert all(np.array_equal(x, xs[0]) for x in xs)
    assert all(r.velocity is not None and r.velocity.shape == r.xyz.shape for r in reqs)
