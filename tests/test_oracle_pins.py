"""Pins of the CPU oracle against facts fixed outside it: closed forms, special
functions evaluated by mpmath, finite differences, invariances and algebraic
identities of the ris functional.  CPU only."""
import math

import mpmath as mp
import numpy as np
import pytest

import molgen
from oracle import ris_oracle as O

mp.mp.dps = 40


# ------------------------------------------------------------- Boys (P1/P2) --
def _boys_ref(m, T):
    if T == 0:
        return mp.mpf(1) / (2 * m + 1)
    return mp.hyp1f1(m + mp.mpf(1) / 2, m + mp.mpf(3) / 2, -mp.mpf(T)) / (2 * m + 1)


@pytest.mark.parametrize("T", [0.0, 1e-12, 1e-6, 0.01, 0.3, 1.0, 2.5, 7.0, 12.0, 20.0, 29.9,
                               34.99, 35.01, 45.0, 60.0, 120.0])
def test_boys_vs_mpmath(T):
    F = O.boys(7, T)
    for m in range(8):
        ref = float(_boys_ref(m, T))
        assert abs(F[m] - ref) <= 1e-14 * ref, (m, T, F[m], ref)


def test_boys_limits():
    # F_m(0) = 1/(2m+1); F_0 closed form with erf; large-T asymptote;
    # downward recursion identity.
    F = O.boys(7, 0.0)
    assert np.allclose(F, [1.0 / (2 * m + 1) for m in range(8)], rtol=0, atol=1e-16)
    for T in (0.5, 3.0, 17.0, 50.0):
        F = O.boys(7, T)
        assert abs(F[0] - 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))) < 1e-15
        for m in range(7):
            lhs = F[m]
            rhs = (2 * T * F[m + 1] + math.exp(-T)) / (2 * m + 1)
            assert abs(lhs - rhs) <= 1e-15 * lhs
    T = 200.0
    F = O.boys(7, T)
    for m in range(8):
        asym = math.prod(range(2 * m - 1, 0, -2)) / 2 ** (m + 1) * math.sqrt(math.pi / T ** (2 * m + 1))
        assert abs(F[m] - asym) <= 1e-13 * asym


# --------------------------------------------------------- integrals (P3/P4) --
def _norm(a, lx, ly, lz):
    return molgen.cart_norm(a, lx, ly, lz)


def _sss_closed(a, A, b, B, c, C):
    """Unnormalised (g_a g_b | g_c) for s Gaussians, closed form (mpmath)."""
    a, b, c = mp.mpf(a), mp.mpf(b), mp.mpf(c)
    A = [mp.mpf(x) for x in A]
    B = [mp.mpf(x) for x in B]
    C = [mp.mpf(x) for x in C]
    p = a + b
    P = [(a * A[k] + b * B[k]) / p for k in range(3)]
    AB2 = sum((A[k] - B[k]) ** 2 for k in range(3))
    PC2 = sum((P[k] - C[k]) ** 2 for k in range(3))
    T = p * c / (p + c) * PC2
    F0 = mp.mpf(1) if T == 0 else mp.sqrt(mp.pi / T) * mp.erf(mp.sqrt(T)) / 2
    return 2 * mp.pi ** mp.mpf(2.5) / (p * c * mp.sqrt(p + c)) * mp.exp(-a * b / p * AB2) * F0


def _shells(xyz, l, e, atom=None):
    n = len(l)
    return O.Shells(np.ascontiguousarray(np.array(xyz, dtype=float).reshape(n, 3)),
                    np.array(l, dtype=np.int32), np.array(e, dtype=float),
                    np.array(atom if atom is not None else list(range(n)), dtype=np.int32))


def test_sss_and_ss_closed_forms():
    rng = np.random.default_rng(3)
    for _ in range(5):
        A, B, C = rng.uniform(-1.5, 1.5, (3, 3))
        a, b, c = rng.uniform(0.1, 3.0, 3)
        ao = _shells([A, B], [0, 0], [a, b])
        aux = _shells([C], [0], [c])
        t = O.int3c(ao, aux)
        ref = float(_sss_closed(a, A, b, B, c, C)) * _norm(a, 0, 0, 0) * _norm(b, 0, 0, 0) * _norm(c, 0, 0, 0)
        assert abs(t[0, 0, 1] - ref) < 1e-14 * abs(ref)
        assert abs(t[0, 1, 0] - ref) < 1e-14 * abs(ref)
        # (a|b) two-centre: 2 pi^{5/2}/(ab sqrt(a+b)) F0(ab/(a+b) R^2)
        m = O.int2c(_shells([A, C], [0, 0], [a, c]))
        R2 = float(((A - C) ** 2).sum())
        T = a * c / (a + c) * R2
        F0 = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
        ref2 = 2 * math.pi ** 2.5 / (a * c * math.sqrt(a + c)) * F0 * _norm(a, 0, 0, 0) * _norm(c, 0, 0, 0)
        assert abs(m[0, 1] - ref2) < 1e-14 * abs(ref2)
        assert abs(m[0, 1] - m[1, 0]) < 1e-15 * abs(m[0, 1])


def _deriv_closed(a, A, b, B, c, C, da, db, dc):
    """Unnormalised (x^da.. | ..) from derivatives of the s closed form:
    x_A g_a = (1/2a) d g_a/dA_x;  x_A^2 g_a = (d^2/dA_x^2 + 2a) g_a / (4a^2);
    x_A y_A g_a = d^2 g_a /(dA_x dA_y) / (4a^2).  Same for B and C."""
    def powers_to_ops(e, l):
        # list of (coefficient, derivative multi-index) so that
        # x^lx y^ly z^lz g = sum coef * d^mi g
        e = mp.mpf(e)
        terms = [(mp.mpf(1), (0, 0, 0))]
        for k in range(3):
            if l[k] == 0:
                continue
            new = []
            for coef, mi in terms:
                mi1 = list(mi)
                mi1[k] += l[k]
                if l[k] == 1:
                    new.append((coef / (2 * e), tuple(mi1)))
                elif l[k] == 2:
                    new.append((coef / (4 * e * e), tuple(mi1)))
                    new.append((coef * 2 * e / (4 * e * e), mi))
            terms = new
        return terms

    ta, tb, tc = powers_to_ops(a, da), powers_to_ops(b, db), powers_to_ops(c, dc)
    total = mp.mpf(0)
    for ca, mia in ta:
        for cb, mib in tb:
            for cc, mic in tc:
                orders = list(mia) + list(mib) + list(mic)
                if sum(orders) == 0:
                    val = _sss_closed(a, A, b, B, c, C)
                else:
                    f = lambda *x: _sss_closed(a, x[0:3], b, x[3:6], c, x[6:9])
                    val = mp.diff(f, list(A) + list(B) + list(C), tuple(orders))
                total += ca * cb * cc * val
    return total


@pytest.mark.parametrize("la,lb,lc", [(1, 0, 0), (0, 1, 1), (2, 0, 0), (1, 2, 1), (2, 2, 1)])
def test_pd_integrals_by_gaussian_derivatives(la, lb, lc):
    rng = np.random.default_rng(10 * la + 3 * lb + lc)
    A, B, C = rng.uniform(-1.0, 1.0, (3, 3))
    a, b, c = rng.uniform(0.3, 1.5, 3)
    ao = _shells([A, B], [la, lb], [a, b])
    aux = _shells([C], [lc], [c])
    t = O.int3c(ao, aux)
    na = molgen.NCART[la]
    cart = molgen.CART
    # sample a few components (mpmath differentiation is slow)
    comps = [(0, 0, 0), (na - 1, len(cart[lb]) - 1, len(cart[lc]) - 1)]
    if la == 2:
        comps.append((1, 0, 0))
    for (ia, ib, ic) in comps:
        pa, pb, pc = cart[la][ia], cart[lb][ib], cart[lc][ic]
        ref = _deriv_closed(a, A, b, B, c, C, pa, pb, pc)
        ref = float(ref) * _norm(a, *pa) * _norm(b, *pb) * _norm(c, *pc)
        got = t[ic, ia, na + ib]
        assert abs(got - ref) < 1e-11 * max(1.0, abs(ref)), (pa, pb, pc, got, ref)


# ------------------------------------------------- derivative integrals (P5) --
def test_int3c_derivatives_fd_and_sum_rule():
    p = molgen.make_tiny_problem(5, natm=3, lmax=2)
    mol = p.mol
    rng = np.random.default_rng(1)
    ao = O.ao_shells(mol)
    aux = O.aux_build(mol, molgen.radii_bohr_table()).J
    nao, naux = ao.nfunc, aux.nfunc
    W = rng.standard_normal((1, naux, nao, nao))
    g = O.int3c_grad(ao, aux, mol.natm, W)[0]
    assert np.abs(g.sum(0)).max() < 1e-12 * np.abs(g).max()

    def f(xyz):
        return float(np.sum(W[0] * O.int3c(ao.at(xyz), aux.at(xyz))))

    h = 2e-3
    for (A, d) in [(0, 0), (1, 2), (2, 1)]:
        vals = {}
        for k in (-2, -1, 1, 2):
            x = mol.xyz.copy()
            x[A, d] += k * h
            vals[k] = f(x)
        fd = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * h)
        assert abs(fd - g[A, d]) < 1e-8 * max(1.0, abs(g[A, d])), (A, d, fd, g[A, d])


def test_int2c_derivatives_fd():
    p = molgen.make_tiny_problem(6, natm=3, lmax=1)
    mol = p.mol
    aux = O.aux_build(mol, molgen.radii_bohr_table()).J
    rng = np.random.default_rng(2)
    W = rng.standard_normal((1, aux.nfunc, aux.nfunc))
    g = O.int2c_grad(aux, mol.natm, W)[0]
    assert np.abs(g.sum(0)).max() < 1e-12 * np.abs(g).max()
    h = 2e-3
    for (A, d) in [(0, 1), (2, 0)]:
        vals = {}
        for k in (-2, -1, 1, 2):
            x = mol.xyz.copy()
            x[A, d] += k * h
            vals[k] = float(np.sum(W[0] * O.int2c(aux.at(x))))
        fd = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * h)
        assert abs(fd - g[A, d]) < 1e-8 * max(1.0, abs(g[A, d]))


# ---------------------------------------------------------- RI exact (P6) --
def test_ri_exact_when_aux_is_the_product():
    # one centre, one s AO exponent a, aux s exponent 2a: the AO product is the
    # aux function itself, so (ss|ss)_ris equals the exact 4-centre (ss|ss)
    a = 0.7
    ao = _shells([[0.1, -0.2, 0.3]], [0], [a])
    aux = _shells([[0.1, -0.2, 0.3]], [0], [2 * a])
    t = O.int3c(ao, aux)[0, 0, 0]
    M = O.int2c(aux)[0, 0]
    ris = t * t / M
    N = _norm(a, 0, 0, 0)
    p = q = 2 * a
    exact = N ** 4 * 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q))
    assert abs(ris - exact) < 1e-14 * exact


# ------------------------------------------------------ the ris functional --
@pytest.fixture(scope="module")
def ring():
    p = molgen.make_problem("ring12")
    rad = molgen.radii_bohr_table()
    S = O.setup(p.mol, rad, j_p_on_heavy=False)
    return p, rad, S


def _dense_AB(S, C, eps, nocc, alpha_J, c_x):
    """Dense A and B of the ris kernel from the explicit four-index RI tensor."""
    MJinv = np.linalg.inv(S.MJ)
    MKinv = np.linalg.inv(S.MK)
    eriJ = np.einsum("Pmn,PQ,Qls->mnls", S.int3J, MJinv, S.int3J, optimize=True)
    eriK = np.einsum("Pmn,PQ,Qls->mnls", S.int3K, MKinv, S.int3K, optimize=True)
    moJ = np.einsum("mnls,mp,nq,lr,st->pqrt", eriJ, C, C, C, C, optimize=True)
    moK = np.einsum("mnls,mp,nq,lr,st->pqrt", eriK, C, C, C, C, optimize=True)
    o = nocc
    v = C.shape[1] - o
    de = (eps[o:][:, None] - eps[:o][None, :]).ravel()
    # K_{ai,bj} = g_{ai,jb} = (ai|jb) - c_x (ab|ji);  B_{ai,bj} = g_{ai,bj}
    A = alpha_J * moJ[o:, :o, :o, o:].transpose(0, 1, 3, 2) - c_x * moK[o:, o:, :o, :o].transpose(0, 3, 1, 2)
    B = alpha_J * moJ[o:, :o, o:, :o] - c_x * moK[o:, :o, o:, :o].transpose(0, 3, 2, 1)
    A = A.reshape(v * o, v * o) + np.diag(de)
    B = B.reshape(v * o, v * o)
    return A, B


def test_matvec_vs_dense_ris_matrices(ring):
    p, rad, S = ring
    A, B = _dense_AB(S, p.C, p.eps, p.nocc, 2.0, 0.25)
    assert np.abs(A - A.T).max() < 1e-10 * np.abs(A).max()
    assert np.abs(B - B.T).max() < 1e-10 * np.abs(B).max()
    rng = np.random.default_rng(0)
    V = rng.standard_normal((2,) + p.X.shape[1:])
    for op, M in (("A", A), ("B", B), ("A+B", A + B), ("A-B", A - B)):
        got = O.response_matvec(S, p.C, p.eps, p.nocc, V, op)
        ref = np.array([(M @ v.ravel()).reshape(v.shape) for v in V])
        assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max(), op
    # (A - B) does not depend on the Coulomb factor
    amb1 = O.response_matvec(S, p.C, p.eps, p.nocc, V, "A-B", alpha_J=1.0)
    amb2 = O.response_matvec(S, p.C, p.eps, p.nocc, V, "A-B", alpha_J=2.0)
    assert np.abs(amb1 - amb2).max() < 1e-13
    # TDA eigenpairs of the dense A satisfy the matvec
    w, U = np.linalg.eigh(A)
    x = U[:, 0].reshape(p.X.shape[1:])
    Ax = O.response_matvec(S, p.C, p.eps, p.nocc, x[None], "A")[0]
    assert np.abs(Ax - w[0] * x).max() < 1e-11


def test_zvector_dense_solve(ring):
    """The ris Z-vector operator (A+B)^ris assembled from matvecs equals the
    brute-force four-index A+B and is symmetric; with model orbitals (random
    rotation, uniform orbital energies) it is indefinite but nonsingular, which
    is why the GPU path uses MINRES rather than conjugate gradients; the solve
    inverts it."""
    p, rad, S = ring
    A, B = _dense_AB(S, p.C, p.eps, p.nocc, 2.0, 0.25)
    M = O.dense_apb(S, p.C, p.eps, p.nocc)
    assert np.abs(M - (A + B)).max() < 1e-11 * np.abs(A + B).max()
    assert np.abs(M - M.T).max() < 1e-10 * np.abs(M).max()
    w = np.abs(np.linalg.eigvalsh(0.5 * (M + M.T)))
    assert w.min() > 1e-8 * w.max()
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2,) + p.X.shape[1:])
    rhs = np.array([((A + B) @ xi.ravel()).reshape(xi.shape) for xi in x])
    Z = O.zvector_solve(S, p.C, p.eps, p.nocc, rhs)
    cond = w.max() / w.min()
    assert np.abs(Z - x).max() < 1e-13 * cond * np.abs(x).max()
    # a zero right-hand side gives Z = 0
    assert np.abs(O.zvector_solve(S, p.C, p.eps, p.nocc, np.zeros_like(rhs[:1]))).max() == 0.0


def test_tda_eigen(ring):
    """TDA-ris eigenpairs from the matvec-assembled A are eigenpairs of the
    brute-force four-index A, ascending, orthonormal, and the lowest ones."""
    p, rad, S = ring
    A, _ = _dense_AB(S, p.C, p.eps, p.nocc, 2.0, 0.25)
    w, X = O.tda_eigen(S, p.C, p.eps, p.nocc, 4)
    U = X.reshape(4, -1)
    assert np.all(np.diff(w) >= 0)
    assert np.abs(U @ U.T - np.eye(4)).max() < 1e-12
    for k in range(4):
        assert np.abs(A @ U[k] - w[k] * U[k]).max() < 1e-11 * np.abs(A).max()
    wall = np.linalg.eigvalsh(A)
    assert np.abs(w - wall[:4]).max() < 1e-11 * np.abs(wall).max()


def test_zrhs_ris_terms(ring):
    """ris terms of the Z-vector right-hand side: g^ris[D] is symmetric for
    the symmetric R^S and antisymmetric for L^A, sum D1 . g[D2] over the MO
    indices reproduces the bilinear functional E_IJ (computed independently
    from three-centre contractions), so tr G_II = 4 E_II and tr Q_IJ = 4 E_IJ."""
    p, rad, S = ring
    rng = np.random.default_rng(8)
    X, Y = molgen.make_amplitudes(p.eps, p.nocc, 2, False, rng)
    nmo = p.C.shape[1]
    RS, LA = O.mo_densities(X, Y, p.nocc, nmo)
    RSa, LAa = O.ao_densities(p.C, p.nocc, X, Y)
    assert np.abs(p.C @ RS[0] @ p.C.T - RSa[0]).max() < 1e-13
    assert np.abs(p.C @ LA[1] @ p.C.T - LAa[1]).max() < 1e-13
    gR = p.C.T @ O.g_ris_ao(S, RSa[0]) @ p.C
    gL = p.C.T @ O.g_ris_ao(S, LAa[0]) @ p.C
    assert np.abs(gR - gR.T).max() < 1e-12 * np.abs(gR).max()
    assert np.abs(gL + gL.T).max() < 1e-12 * np.abs(gL).max()
    G = O.zrhs_ris_terms(S, p.C, p.nocc, X, Y, [(0, 0), (0, 1)])
    E00 = O.energy_functional(S, RSa[0], RSa[0], LAa[0], LAa[0])
    E01 = O.energy_functional(S, RSa[0], RSa[1], LAa[0], LAa[1])
    assert abs(np.trace(G[0]) - 4.0 * E00) < 1e-11 * max(1.0, abs(E00))
    assert abs(np.trace(G[1]) - 4.0 * E01) < 1e-11 * max(1.0, abs(E01))
    # a flipped sign on the L^A terms is caught (their share of the trace is not zero)
    Gbad = 4.0 * RS[0] @ gR + 4.0 * LA[0] @ gL
    assert abs(np.trace(Gbad) - 4.0 * E00) > 1e-6 * abs(E00)
    # orbital-rotation derivative: rotating MOs p, q by theta (amplitudes fixed in
    # the MO basis) changes E_II at the rate -(G_pq - G_qp): 5-point differences
    o = p.nocc
    h = 1e-3
    for (pp, qq) in ((o + 3, 2), (o + 10, o - 1), (1, 5), (o + 2, o + 7)):
        def E_rot(th):
            c, s_ = np.cos(th), np.sin(th)
            C2 = p.C.copy()
            C2[:, pp], C2[:, qq] = c * p.C[:, pp] - s_ * p.C[:, qq], s_ * p.C[:, pp] + c * p.C[:, qq]
            R2, L2 = O.ao_densities(C2, o, X[:1], Y[:1])
            return O.energy_functional(S, R2[0], R2[0], L2[0], L2[0])
        fd = (E_rot(-2 * h) - 8 * E_rot(-h) + 8 * E_rot(h) - E_rot(2 * h)) / (12 * h)
        an = -(G[0][pp, qq] - G[0][qq, pp])
        assert abs(fd - an) < 1e-8 * max(1.0, abs(an)), (pp, qq, fd, an)


def test_energy_consistency(ring):
    """E_II from AO traces equals 1/2 R.(A+B-D)R + 1/2 L.(A-B-D)L (TDDFT Y != 0)."""
    p0, rad, S = ring
    rng = np.random.default_rng(7)
    X, Y = molgen.make_amplitudes(p0.eps, p0.nocc, 2, False, rng)
    RS, LA = O.ao_densities(p0.C, p0.nocc, X, Y)
    de = p0.eps[p0.nocc:][:, None] - p0.eps[:p0.nocc][None, :]
    for I in range(2):
        e_ao = O.energy_functional(S, RS[I], RS[I], LA[I], LA[I])
        R = X[I] + Y[I]
        L = X[I] - Y[I]
        apb = O.response_matvec(S, p0.C, p0.eps, p0.nocc, R[None], "A+B")[0] - de * R
        amb = O.response_matvec(S, p0.C, p0.eps, p0.nocc, L[None], "A-B")[0] - de * L
        e_mo = 0.5 * np.sum(R * apb) + 0.5 * np.sum(L * amb)
        assert abs(e_ao - e_mo) < 1e-11 * abs(e_mo), (e_ao, e_mo)
    # off-diagonal: E_IJ bilinear form and its symmetry
    e01 = O.energy_functional(S, RS[0], RS[1], LA[0], LA[1])
    e10 = O.energy_functional(S, RS[1], RS[0], LA[1], LA[0])
    assert abs(e01 - e10) < 1e-11 * abs(e01)


def _fd5(fun, xyz, A, d, h=2e-3):
    vals = {}
    for k in (-2, -1, 1, 2):
        x = xyz.copy()
        x[A, d] += k * h
        vals[k] = fun(x)
    return (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * h)


def _check_fd(prob, rad, jp, outputs, coords, tol):
    S = O.setup(prob.mol, rad, j_p_on_heavy=jp)
    RS, LA = O.ao_densities(prob.C, prob.nocc, prob.X, prob.Y)
    g = O.grad_nac(prob, rad, outputs, j_p_on_heavy=jp, S=S)
    for k, (I, J) in enumerate(outputs):
        fun = lambda x: O.energy_at(prob.mol, x, rad, RS[I], RS[J], LA[I], LA[J], j_p_on_heavy=jp)
        for (A, d) in coords:
            fd = _fd5(fun, prob.mol.xyz, A, d)
            assert abs(fd - g[k, A, d]) < tol, (I, J, A, d, fd, g[k, A, d])
    return g


def test_gradient_and_nac_vs_finite_differences_ring(ring):
    p, rad, _ = ring
    _check_fd(p, rad, False, [(0, 0), (1, 2)], [(0, 0), (2, 1), (7, 2), (11, 0)], 1e-9)


def test_gradient_vs_finite_differences_mixed_l_tddft(radii):
    # d on heavy atoms, p aux on heavy atoms, full TDDFT amplitudes (Y != 0)
    p = molgen.make_tiny_problem(11, natm=3, lmax=2, nstate=2, tda=False)
    _check_fd(p, radii, True, [(0, 0), (0, 1)], [(0, 0), (1, 1), (2, 2)], 1e-9)


def test_translational_invariance(ring, radii):
    p, rad, S = ring
    g = O.grad_nac(p, rad, [(0, 0), (0, 2)], j_p_on_heavy=False, S=S)
    assert np.abs(g.sum(1)).max() < 1e-10
    q = molgen.make_tiny_problem(12, natm=4, lmax=2, nstate=2, tda=False)
    g = O.grad_nac(q, radii, [(0, 1)])
    assert np.abs(g.sum(1)).max() < 1e-10


def test_rotational_invariance_s_only():
    p = molgen.make_tiny_problem(13, natm=4, lmax=0, nstate=1, tda=False)
    rad = molgen.radii_bohr_table()
    g = O.grad_nac(p, rad, [(0, 0)], j_p_on_heavy=False)[0]
    torque = np.cross(p.mol.xyz, g).sum(0)
    assert np.abs(torque).max() < 1e-10


def test_nac_structure(ring):
    p, rad, S = ring
    g = O.grad_nac(p, rad, [(0, 0), (0, 1), (1, 0)], j_p_on_heavy=False, S=S)
    grad0 = g[0]
    assert np.abs(g[1] - g[2]).max() < 1e-13
    # bilinear in the second state's amplitudes: scaling X_J scales the numerator
    p2 = molgen.Problem(p.mol, p.C, p.eps, p.nocc, p.X.copy(), None)
    p2.X[1] *= 3.0
    g2 = O.grad_nac(p2, rad, [(0, 1), (0, 0)], j_p_on_heavy=False, S=S)
    assert np.abs(g2[0] - 3.0 * g[1]).max() < 1e-13
    assert np.abs(g2[1] - grad0).max() < 1e-14


def test_tda_none_equals_zero_y(ring):
    p, rad, S = ring
    g1 = O.grad_nac(p, rad, [(0, 1)], j_p_on_heavy=False, S=S)
    p0 = molgen.Problem(p.mol, p.C, p.eps, p.nocc, p.X, np.zeros_like(p.X))
    g2 = O.grad_nac(p0, rad, [(0, 1)], j_p_on_heavy=False, S=S)
    # thread-order summation in the oracle makes this equal to rounding only
    assert np.abs(g1 - g2).max() < 1e-15


def test_planted_mistakes_are_caught(ring, monkeypatch):
    """A dropped metric-derivative term or a flipped exchange sign must fail
    the finite-difference pin."""
    p, rad, S = ring
    RS, LA = O.ao_densities(p.C, p.nocc, p.X, p.Y)
    fun = lambda x: O.energy_at(p.mol, x, rad, RS[0], RS[0], LA[0], LA[0], j_p_on_heavy=False)
    fd = _fd5(fun, p.mol.xyz, 0, 0)
    orig = O.pair_weights

    def no_metric(*a, **k):
        w3j, w2j, w3k, w2k = orig(*a, **k)
        return w3j, w2j, w3k, 0 * w2k

    monkeypatch.setattr(O, "pair_weights", no_metric)
    g = O.grad_nac(p, rad, [(0, 0)], j_p_on_heavy=False, S=S)[0]
    assert abs(g[0, 0] - fd) > 1e-7

    def flip(*a, **k):
        w3j, w2j, w3k, w2k = orig(*a, **k)
        return w3j, w2j, -w3k, -w2k

    monkeypatch.setattr(O, "pair_weights", flip)
    g = O.grad_nac(p, rad, [(0, 0)], j_p_on_heavy=False, S=S)[0]
    assert abs(g[0, 0] - fd) > 1e-7


# ------------------------------------------------- auxiliary basis values --
def test_aux_exponent_values():
    """alpha_A = theta / R_A^2 with theta = 0.2 and R_A in Bohr: H (0.37 A)
    0.409099, C (0.77 A) 0.094461, N (0.75 A) 0.099566, O (0.73 A) 0.105096
    Bohr^-2 (values worked out by hand from the radii, 1 Bohr = 0.529177210903 A)."""
    p = molgen.make_problem("ring12")
    rad = molgen.radii_bohr_table()
    aux = O.aux_build(p.mol, rad, 0.2, True)
    exp_by_z = {int(z): float(e) for z, e in zip(p.mol.Z[aux.J.atom], aux.J.exp)}
    assert abs(exp_by_z[1] - 0.409099) < 5e-7
    assert abs(exp_by_z[6] - 0.094461) < 5e-7
    assert abs(0.2 / rad[7] ** 2 - 0.099566) < 5e-7
    assert abs(0.2 / rad[8] ** 2 - 0.105096) < 5e-7
    # J = s on every atom then p on heavy atoms, one exponent per atom; K = the s set
    assert list(aux.J.l) == [0] * 12 + [1] * 6
    assert np.array_equal(aux.J.exp[12:], aux.J.exp[:6])
    assert np.array_equal(aux.K.exp, aux.J.exp[:12])


# --------------------------------------------- aux normalisation (P7) --
def test_aux_normalisation_invariance(radii):
    """Multiplying each auxiliary function by a constant changes (mn|P) and
    (P|Q) but no RI result.  With powers of two as the constants every scaled
    quantity is exact in floating point, so energies, matvecs and gradients
    must agree to 1e-14 relative (gradients: 1e-14 Ha/Bohr absolute, the
    noise of the oracle's threaded sums; mixed-l AOs, p auxiliary functions,
    TDDFT amplitudes).  With general constants (0.3..3) the results differ by the
    rounding of the metric solves, about cond(M_J) u = 3e-12 of their largest
    terms: bar 1e-10.  A result that dropped or doubled a metric factor moves
    by O(1) (planted below)."""
    p = molgen.make_tiny_problem(31, natm=3, lmax=2, nstate=2, tda=False)
    S0 = O.setup(p.mol, radii, j_p_on_heavy=True)
    nJ = S0.MJ.shape[0]
    rng = np.random.default_rng(5)
    RS, LA = O.ao_densities(p.C, p.nocc, p.X, p.Y)
    V = np.random.default_rng(6).standard_normal((2,) + p.X.shape[1:])
    g0 = O.grad_nac(p, radii, [(0, 0), (0, 1)], S=S0)
    for scale, bar, gbar in ((2.0 ** rng.integers(-3, 4, nJ), 1e-14, 1e-14),
                             (rng.uniform(0.3, 3.0, nJ), 1e-10, 1e-10 * np.abs(g0).max())):
        S1 = O.setup(p.mol, radii, j_p_on_heavy=True, aux_scale=scale)
        assert np.abs(S1.MJ - S0.MJ).max() > 1e-3          # the integrals did change
        for aJ, cx in ((2.0, 0.0), (0.0, 0.25)):            # Coulomb and exchange parts
            e0 = O.energy_functional(S0, RS[0], RS[1], LA[0], LA[1], alpha_J=aJ, c_x=cx)
            e1 = O.energy_functional(S1, RS[0], RS[1], LA[0], LA[1], alpha_J=aJ, c_x=cx)
            assert abs(e1 - e0) <= bar * abs(e0), (aJ, cx, e0, e1)
        for op in ("A", "B"):
            m0 = O.response_matvec(S0, p.C, p.eps, p.nocc, V, op)
            m1 = O.response_matvec(S1, p.C, p.eps, p.nocc, V, op)
            assert np.abs(m1 - m0).max() <= bar * np.abs(m0).max()
        g1 = O.grad_nac(p, radii, [(0, 0), (0, 1)], S=S1)
        assert np.abs(g1 - g0).max() <= gbar
    # planted mistake: the scaled integrals without the scale in the derivative weights
    S_bad = O.Setup(S1.ao, S1.aux, S1.int3J, S1.int3K, S1.MJ, S1.MK, None)
    g_bad = O.grad_nac(p, radii, [(0, 0)], S=S_bad)
    assert np.abs(g_bad[0] - g0[0]).max() > 1e-3 * np.abs(g0[0]).max()


# ------------------------------- densities of Appendix A.1-A.2, extra pairs --
def test_difference_density_forms(radii):
    """T_IJ of eq. T (from X, Y) against the R, L form the ris right-hand side
    uses for I = J (Appendix A.3: T_II = [[-(R^T R + L^T L)/2, 0], [0, (R R^T +
    L L^T)/2]]); T_II conserves the electron count (tr S T = 0); T_IJ is
    symmetric and T_IJ = T_JI."""
    p = molgen.make_tiny_problem(32, natm=3, lmax=2, nstate=2, tda=False)
    C, o = p.C, p.nocc
    Smat = molgen.overlap_matrix(p.mol)
    R, L = p.X + p.Y, p.X - p.Y
    for I in range(2):
        T = O.difference_density(C, o, p.X, p.Y, I, I)
        nmo = C.shape[1]
        Tm = np.zeros((nmo, nmo))
        Tm[:o, :o] = -0.5 * (R[I].T @ R[I] + L[I].T @ L[I])
        Tm[o:, o:] = 0.5 * (R[I] @ R[I].T + L[I] @ L[I].T)
        assert np.abs(T - C @ Tm @ C.T).max() < 1e-13 * np.abs(T).max()
        assert abs(np.sum(Smat * T)) < 1e-12
    T01 = O.difference_density(C, o, p.X, p.Y, 0, 1)
    assert np.abs(T01 - T01.T).max() < 1e-14 * np.abs(T01).max()
    assert np.abs(T01 - O.difference_density(C, o, p.X, p.Y, 1, 0)).max() < 1e-14 * np.abs(T01).max()
    # the ground density is the occupied projector: D S D = D, tr S D = nocc
    D = O.ground_density(C, o)
    assert np.abs(D @ Smat @ D - D).max() < 1e-12 * np.abs(D).max()
    assert abs(np.sum(Smat * D) - o) < 1e-11


def _extra_case(seed, natm, lmax, radii, jp):
    p = molgen.make_tiny_problem(seed, natm=natm, lmax=lmax, nstate=2, tda=False)
    Z = np.random.default_rng(seed + 100).standard_normal(p.X.shape[1:])
    Z *= 0.1 / np.linalg.norm(Z)
    D = O.ground_density(p.C, p.nocc)
    P = O.relaxed_density(p.C, p.nocc, p.X, p.Y, 1, Z)
    return p, D, P


@pytest.mark.parametrize("seed,natm,lmax,jp", [(41, 3, 2, True), (42, 4, 1, False)])
def test_extra_pair_vs_finite_differences(radii, seed, natm, lmax, jp):
    """The extra-pair branch: the derivative it adds to an output equals the
    5-point finite difference of cJ sum (mn|ls)_J D1 D2 - cK sum (ml|ns)_K D1 D2
    at fixed D1 = D (ground density), D2 = P_1 = T_11 + Z^S (seeded Z,
    |Z| = 0.1), within 1e-9 Ha/Bohr; cJ and cK enter as given (0.7, 0.3 are
    chosen unlike a_J and c_x so a mixed-up coefficient shows)."""
    p, D, P = _extra_case(seed, natm, lmax, radii, jp)
    S = O.setup(p.mol, radii, j_p_on_heavy=jp)
    cJ, cK = 0.7, 0.3
    base = O.grad_nac(p, radii, [(1, 1), (0, 1)], j_p_on_heavy=jp, S=S)
    g = O.grad_nac(p, radii, [(1, 1), (0, 1)], j_p_on_heavy=jp, S=S, extra=[(1, D, P, cJ, cK)])
    assert np.abs(g[0] - base[0]).max() < 1e-14       # only output 1 gets the pair
    add = g[1] - base[1]
    zero = np.zeros_like(D)
    fun = lambda x: O.energy_at(p.mol, x, radii, D, P, zero, zero, alpha_J=cJ, c_x=cK, j_p_on_heavy=jp)
    for A in range(natm):
        for d in range(3):
            fd = _fd5(fun, p.mol.xyz, A, d)
            assert abs(fd - add[A, d]) < 1e-9, (A, d, fd, add[A, d])
    assert np.abs(add.sum(0)).max() < 1e-10


def test_extra_pair_planted_mistakes(radii, monkeypatch):
    """cJ and cK swapped, or the exchange part's sign flipped, in the
    extra-pair branch must fail the finite-difference pin."""
    p, D, P = _extra_case(41, 3, 2, radii, True)
    S = O.setup(p.mol, radii, j_p_on_heavy=True)
    zero = np.zeros_like(D)
    fd = _fd5(lambda x: O.energy_at(p.mol, x, radii, D, P, zero, zero, alpha_J=0.7, c_x=0.3), p.mol.xyz, 0, 0)
    base = O.grad_nac(p, radii, [(1, 1)], S=S)[0]
    for bad in ((D, P, 0.3, 0.7), (D, P, 0.7, -0.3)):
        g = O.grad_nac(p, radii, [(1, 1)], S=S, extra=[(0,) + bad])[0]
        assert abs((g - base)[0, 0] - fd) > 1e-7


# ------------------------------------------- stored 60-atom oracle outputs --
def test_chain60_golden_matches_oracle(radii):
    """The stored 60-atom outputs (tests/golden/chain60_grad_nac.txt, written by
    make_chain60_ref.py from the oracle alone) are the current oracle's: the
    gradient of state 0 recomputed here agrees to 1e-13 Ha/Bohr (threaded BLAS
    sums), and the stored set is translationally invariant."""
    import os
    p = molgen.make_problem("chain60")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "chain60_grad_nac.txt")
    ref = np.loadtxt(path).reshape(2 * p.nstate - 1, p.mol.natm, 3)
    S = O.setup(p.mol, radii, j_p_on_heavy=True)
    g0 = O.grad_nac(p, radii, [(0, 0)], S=S)[0]
    assert np.abs(g0 - ref[0]).max() <= 1e-13
    assert np.abs(ref.sum(axis=1)).max() <= 1e-10
