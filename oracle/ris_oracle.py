"""CPU ORACLE -- test infrastructure only.

Plain FP64 reference for the TDDFT-ris response hot path (arXiv 2511.18233).
Only ``tests/``, the smoke check and the bench's CPU-baseline leg may import
this module; the product path never does.  It shares no code with the HIP
library: integrals come from ``ris_ints.c`` (textbook McMurchie-Davidson),
linear algebra from NumPy/SciPy.

What it computes, and where the paper defines it:

* ris kernel: g^ris_{pq,sr} = sum_AB (pq|A)(M^-1)_AB (B|sr)
  - c_x sum_AB (pr|A)(M^-1)_AB (B|sq), M_AB = (A|B), with J-fit and K-fit
  auxiliary sets allowed to differ (Sec. 2.2, eqs. ris / g_modified).
* minimal auxiliary basis: one Gaussian per angular-momentum component per
  atom; Coulomb fit s (+p), exchange fit s only (Sec. 2.2; Sec. 4 opening).
  Exponent per atom alpha_A = theta / R_A^2 (R_A covalent radius in Bohr).
* response matrices A_{ai,bj} = (e_a - e_i) d d + K_{ai,bj},
  B_{ai,bj} = K_{ai,jb}, K_{pq,rs} = g_{pq,sr} (Sec. 2.1, eqs. A_matrix,
  B_matrix, K_matrix); f_xc is dropped under ris.
* transition densities R_I = X_I + Y_I, L_I = X_I - Y_I, AO forms
  R^S = (C_V R C_O^T + transpose)/2, L^A = (C_V L C_O^T - transpose)/2 and
  Gamma_IJ = {R^S_I, R^S_J} + {L^A_I, L^A_J} (Appendix A.1).
* the ris two-electron part of the gradient / NAC numerator,
  <g^{ris,(xi)}; Gamma_IJ> (Sec. 2.2, eqs. gI_xi_ris / gIJ_xi_ris), as the
  explicit nuclear derivative of the bilinear functional
      E_IJ = a_J sum (mn|ls)_J R^S_I,mn R^S_J,ls
             - c_x sum (ml|ns)_K [R^S_I,mn R^S_J,ls + L^A_I,mn L^A_J,ls]
  at fixed AO densities, differentiated with the three-term RI derivative
  (Sec. 2.2, last equation): (pq|A)^x M^-1 (B|sr) + (pq|A) M^-1 (B|sr)^x
  - (pq|A) M^-1 M^x M^-1 (B|sr).

* TDA-ris excitation energies: the lowest eigenpairs of the symmetric A^ris
  (Sec. 2.1 eq. casida with B = 0, the TDA; the ris kernel in A), here the
  dense A^ris assembled column by column from the matvec and a full
  symmetric eigendecomposition.
* ris terms of the Z-vector right-hand side (Appendix A.3, eqs.
  g_I_pp_ris and g_IJ_pp_ris): in the MO basis, for a gradient
  4 [R^S_I g^ris[R^S_I]] - 4 [L^A_I g^ris[L^A_I]], for a NAC pair
  2 [R^S_I g[R^S_J]] - 2 [L^A_I g[L^A_J]] + 2 [R^S_J g[R^S_I]] - 2 [L^A_J g[L^A_I]],
  with R^S = [[0, R^T/2], [R/2, 0]], L^A = [[0, -L^T/2], [L/2, 0]] (occupied
  first) and g^ris[D]_mn = a_J sum (mn|ls)_J D_ls - c_x sum (ml|ns)_K D_ls,
  the convention under which sum_mn D1_mn g[D2]_mn is the bilinear ris
  functional E (reading A2); built here from explicit four-index tensors.
* ris-approximated Z-vector solve: (A+B)^ris Z = rhs with the ris kernel
  in the (A+B) matrix of the Z-vector equation (Sec. 4.2; the equation is
  eq. Z_vector of Sec. 2.1, restated in Appendix A.2), solved here by its
  definition: the dense (A+B)^ris assembled column by column from the matvec
  and a direct solve.

* extra density pairs: the <g^(xi); {D, P}> terms of the gradient and NAC
  (Sec. 2.2, eqs. gI_xi_ris / gIJ_xi_ris) with the ground density D, the
  difference density T_IJ (Appendix A.1 eq. T) and the relaxed density
  P = T + Z^S (Appendix A.2), each pair (D1, D2, cJ, cK) contributing the
  derivative of cJ sum (mn|ls)_J D1 D2 - cK sum (ml|ns)_K D1 D2 over the same
  ris auxiliary sets (the paper's full density-fitting basis is not part of
  the path).  Pinned by 5-point finite differences of that functional.

Readings where the paper is silent or ambiguous (each one a parameter here):
a_J (closed-shell Coulomb factor, default 2), c_x (default 0.25, PBE0),
the exchange index order for antisymmetric L^A (chosen so that E_II equals
1/2 R.(A+B-D)R + 1/2 L.(A-B-D)L), the J/K auxiliary split and the p exponent
(same as the atom's s exponent).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ris_ints.c")
_SO = os.path.join(_HERE, "libris_oracle.so")
_lib = None

NCART = (1, 3, 6)
DEFAULT_THETA = 0.2
DEFAULT_CX = 0.25
DEFAULT_ALPHA_J = 2.0


def build_lib(force: bool = False) -> str:
    """Compile ris_ints.c with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build_lib())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        up = ctypes.POINTER(ctypes.c_ubyte)
        _lib.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        _lib.oracle_int3c.argtypes = [ctypes.c_int, dp, ip, dp, ctypes.c_int, dp, ip, dp, dp]
        _lib.oracle_int2c.argtypes = [ctypes.c_int, dp, ip, dp, dp]
        _lib.oracle_int3c_grad.argtypes = [ctypes.c_int, dp, ip, dp, ip, ctypes.c_int, dp, ip, dp, ip,
                                           ctypes.c_int, ctypes.c_int, dp, up, dp]
        _lib.oracle_int2c_grad.argtypes = [ctypes.c_int, dp, ip, dp, ip, ctypes.c_int, ctypes.c_int, dp, dp]
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def boys(mmax: int, T: float) -> np.ndarray:
    out = np.zeros(mmax + 1)
    lib().oracle_boys(mmax, float(T), _d(out))
    return out


# ---------------------------------------------------------------- shells --
@dataclass
class Shells:
    xyz: np.ndarray      # [n, 3]
    l: np.ndarray        # [n] int32
    exp: np.ndarray      # [n]
    atom: np.ndarray     # [n] int32

    @property
    def n(self) -> int:
        return int(self.l.shape[0])

    @property
    def nfunc(self) -> int:
        return int(sum(NCART[x] for x in self.l))

    def at(self, xyz_atoms: np.ndarray) -> "Shells":
        return Shells(np.ascontiguousarray(xyz_atoms[self.atom]), self.l, self.exp, self.atom)

    def scaled(self, atom_xyz):
        return self.at(atom_xyz)


def ao_shells(mol) -> Shells:
    return Shells(np.ascontiguousarray(mol.xyz[mol.shell_atom], dtype=np.float64),
                  np.ascontiguousarray(mol.shell_l, dtype=np.int32),
                  np.ascontiguousarray(mol.shell_exp, dtype=np.float64),
                  np.ascontiguousarray(mol.shell_atom, dtype=np.int32))


@dataclass
class AuxSets:
    J: Shells
    K: Shells


def aux_build(mol, radius_bohr: np.ndarray, theta: float = DEFAULT_THETA,
              j_p_on_heavy: bool = True) -> AuxSets:
    """Minimal ris auxiliary sets: one s per atom (J and K), plus one p shell
    per heavy atom (Z > 1) in the J set; exponent theta / R_A^2 for both.
    J order: s on every atom in atom order, then p on heavy atoms in atom order."""
    Z = np.asarray(mol.Z)
    alpha = theta / radius_bohr[Z] ** 2
    natm = Z.shape[0]
    s_atoms = np.arange(natm, dtype=np.int32)
    p_atoms = np.nonzero(Z > 1)[0].astype(np.int32) if j_p_on_heavy else np.zeros(0, np.int32)
    atomsJ = np.concatenate([s_atoms, p_atoms]).astype(np.int32)
    lJ = np.concatenate([np.zeros(natm, np.int32), np.ones(p_atoms.size, np.int32)])
    J = Shells(np.ascontiguousarray(mol.xyz[atomsJ]), lJ, np.ascontiguousarray(alpha[atomsJ]), atomsJ)
    K = Shells(np.ascontiguousarray(mol.xyz[s_atoms]), np.zeros(natm, np.int32),
               np.ascontiguousarray(alpha[s_atoms]), s_atoms)
    return AuxSets(J, K)


# ------------------------------------------------------------- integrals --
def int3c(ao: Shells, aux: Shells) -> np.ndarray:
    """(mu nu|P) as [naux][nao][nao]."""
    out = np.zeros((aux.nfunc, ao.nfunc, ao.nfunc))
    lib().oracle_int3c(ao.n, _d(ao.xyz), _i(ao.l), _d(ao.exp), aux.n, _d(aux.xyz), _i(aux.l),
                       _d(aux.exp), _d(out))
    return out


def int2c(aux: Shells) -> np.ndarray:
    out = np.zeros((aux.nfunc, aux.nfunc))
    lib().oracle_int2c(aux.n, _d(aux.xyz), _i(aux.l), _d(aux.exp), _d(out))
    return out


def int3c_grad(ao: Shells, aux: Shells, natm: int, W: np.ndarray, atom_mask=None) -> np.ndarray:
    """sum_{P mu nu} W[o,P,mu,nu] d(mu nu|P)/dR -> [nout][natm][3]."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    nout = W.shape[0]
    g = np.zeros((nout, natm, 3))
    mask = None
    if atom_mask is not None:
        mask = np.ascontiguousarray(atom_mask, dtype=np.uint8)
    lib().oracle_int3c_grad(ao.n, _d(ao.xyz), _i(ao.l), _d(ao.exp), _i(ao.atom), aux.n, _d(aux.xyz),
                            _i(aux.l), _d(aux.exp), _i(aux.atom), natm, nout, _d(W),
                            None if mask is None else mask.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                            _d(g))
    return g


def int2c_grad(aux: Shells, natm: int, W: np.ndarray) -> np.ndarray:
    W = np.ascontiguousarray(W, dtype=np.float64)
    nout = W.shape[0]
    g = np.zeros((nout, natm, 3))
    lib().oracle_int2c_grad(aux.n, _d(aux.xyz), _i(aux.l), _d(aux.exp), _i(aux.atom), natm, nout,
                            _d(W), _d(g))
    return g


# ----------------------------------------------------------- the problem --
@dataclass
class Setup:
    """Everything geometry-dependent for one problem (the plain route)."""
    ao: Shells
    aux: AuxSets
    int3J: np.ndarray   # [nJ][nao][nao]
    int3K: np.ndarray   # [nK][nao][nao]
    MJ: np.ndarray
    MK: np.ndarray
    scale: np.ndarray | None = None   # [nJ] factors multiplying the auxiliary functions (None: 1)


def setup(mol, radius_bohr, theta=DEFAULT_THETA, j_p_on_heavy=True, aux_scale=None) -> Setup:
    """Integrals of the problem.  aux_scale (optional, [nJ]) multiplies each J
    auxiliary function (and the K functions, the leading s functions of the J
    set, by the same factors): an RI result must not depend on it."""
    ao = ao_shells(mol)
    aux = aux_build(mol, radius_bohr, theta, j_p_on_heavy)
    S = Setup(ao, aux, int3c(ao, aux.J), int3c(ao, aux.K), int2c(aux.J), int2c(aux.K))
    if aux_scale is not None:
        sJ = np.asarray(aux_scale, dtype=np.float64)
        sK = sJ[:S.MK.shape[0]]
        S = Setup(ao, aux, S.int3J * sJ[:, None, None], S.int3K * sK[:, None, None], S.MJ * np.outer(sJ, sJ),
                  S.MK * np.outer(sK, sK), sJ)
    return S


def metric_solve(M: np.ndarray, t: np.ndarray) -> np.ndarray:
    """M^-1 t by Cholesky (M symmetric positive definite)."""
    cf = sla.cho_factor(M, lower=True)
    return sla.cho_solve(cf, t)


def mo_int3c(S: Setup, C: np.ndarray, which: str) -> np.ndarray:
    """(pq|P) in the MO basis for all p, q: [naux][nmo][nmo]."""
    t = S.int3J if which == "J" else S.int3K
    return np.einsum("mp,Pmn,nq->Ppq", C, t, C, optimize=True)


def response_matvec(S: Setup, C, eps, nocc, V: np.ndarray, op: str,
                    alpha_J=DEFAULT_ALPHA_J, c_x=DEFAULT_CX) -> np.ndarray:
    """A.V, B.V, (A+B).V or (A-B).V for V[nvec][nvir][nocc] (Sec. 2.1 A/B with
    the ris kernel).  (A V)_ai = (e_a-e_i) V_ai + a_J sum_bj (ai|bj)_J V_bj
    - c_x sum_bj (ab|ij)_K V_bj ;  (B V)_ai = a_J sum_bj (ai|bj)_J V_bj
    - c_x sum_bj (aj|bi)_K V_bj ; (pq|rs)_X = sum_PQ (pq|P)(M_X^-1)_PQ (Q|rs)."""
    V = np.asarray(V, dtype=np.float64)
    o = nocc
    moJ = mo_int3c(S, C, "J")
    moK = mo_int3c(S, C, "K")
    aiJ = moJ[:, o:, :o]             # (ai|P)
    ab = moK[:, o:, o:]
    ij = moK[:, :o, :o]
    aiK = moK[:, o:, :o]
    de = eps[o:][:, None] - eps[:o][None, :]
    out = np.empty_like(V)
    for k in range(V.shape[0]):
        v = V[k]
        t = np.einsum("Pbj,bj->P", aiJ, v)
        cJ = metric_solve(S.MJ, t)
        jterm = alpha_J * np.einsum("Pai,P->ai", aiJ, cJ)
        # exchange parts with M_K^-1 applied on the second index
        ijw = np.einsum("PQ,Qij->Pij", np.linalg.inv(S.MK), ij)
        aiw = np.einsum("PQ,Qai->Pai", np.linalg.inv(S.MK), aiK)
        kA = np.einsum("Pab,Pij,bj->ai", ab, ijw, v, optimize=True)        # (ab|ij) V_bj
        kB = np.einsum("Paj,Pbi,bj->ai", aiK, aiw, v, optimize=True)       # (aj|bi) V_bj
        Av = de * v + jterm - c_x * kA
        Bv = jterm - c_x * kB
        out[k] = {"A": Av, "B": Bv, "A+B": Av + Bv, "A-B": Av - Bv}[op]
    return out


def dense_apb(S: Setup, C, eps, nocc, alpha_J=DEFAULT_ALPHA_J, c_x=DEFAULT_CX) -> np.ndarray:
    """(A+B)^ris as a dense (vo x vo) matrix, columns = matvecs of unit vectors."""
    o = nocc
    v = C.shape[1] - o
    E = np.eye(v * o).reshape(v * o, v, o)
    cols = response_matvec(S, C, eps, nocc, E, "A+B", alpha_J, c_x)
    return cols.reshape(v * o, v * o).T


def g_ris_ao(S: Setup, D: np.ndarray, alpha_J=DEFAULT_ALPHA_J, c_x=DEFAULT_CX) -> np.ndarray:
    """g^ris[D] in the AO basis from the explicit four-index RI tensors (small
    molecules only): a_J sum (mn|ls)_J D_ls - c_x sum (ml|ns)_K D_ls."""
    eriJ = np.einsum("Pmn,PQ,Qls->mnls", S.int3J, np.linalg.inv(S.MJ), S.int3J, optimize=True)
    eriK = np.einsum("Pmn,PQ,Qls->mnls", S.int3K, np.linalg.inv(S.MK), S.int3K, optimize=True)
    return alpha_J * np.einsum("mnls,ls->mn", eriJ, D) - c_x * np.einsum("mlns,ls->mn", eriK, D)


def mo_densities(X, Y, nocc, nmo):
    """R^S_I and L^A_I in the MO basis (occupied first), Appendix A.2."""
    R = X if Y is None else X + Y
    L = X if Y is None else X - Y
    o = nocc
    RS = np.zeros((X.shape[0], nmo, nmo))
    LA = np.zeros((X.shape[0], nmo, nmo))
    for I in range(X.shape[0]):
        RS[I, o:, :o] = 0.5 * R[I]
        RS[I, :o, o:] = 0.5 * R[I].T
        LA[I, o:, :o] = 0.5 * L[I]
        LA[I, :o, o:] = -0.5 * L[I].T
    return RS, LA


def zrhs_ris_terms(S: Setup, C, nocc, X, Y, pairs, alpha_J=DEFAULT_ALPHA_J, c_x=DEFAULT_CX) -> np.ndarray:
    """The ris terms of g^(pp') (Appendix A.3) per output pair (I, J), as
    [npair][nmo][nmo] MO matrices: I == J the gradient form, I != J the four
    ris terms of Q_IJ."""
    nmo = C.shape[1]
    RS, LA = mo_densities(X, Y, nocc, nmo)
    cache = {}

    def g_mo(kind, I):
        if (kind, I) not in cache:
            D = RS[I] if kind == "R" else LA[I]
            cache[(kind, I)] = C.T @ g_ris_ao(S, C @ D @ C.T, alpha_J, c_x) @ C
        return cache[(kind, I)]

    out = np.zeros((len(pairs), nmo, nmo))
    for k, (I, J) in enumerate(pairs):
        if I == J:
            out[k] = 4.0 * RS[I] @ g_mo("R", I) - 4.0 * LA[I] @ g_mo("L", I)
        else:
            out[k] = (2.0 * RS[I] @ g_mo("R", J) - 2.0 * LA[I] @ g_mo("L", J)
                      + 2.0 * RS[J] @ g_mo("R", I) - 2.0 * LA[J] @ g_mo("L", I))
    return out


def dense_a(S: Setup, C, eps, nocc, alpha_J=DEFAULT_ALPHA_J, c_x=DEFAULT_CX) -> np.ndarray:
    """A^ris as a dense (vo x vo) matrix, columns = matvecs of unit vectors."""
    o = nocc
    v = C.shape[1] - o
    E = np.eye(v * o).reshape(v * o, v, o)
    cols = response_matvec(S, C, eps, nocc, E, "A", alpha_J, c_x)
    return cols.reshape(v * o, v * o).T


def tda_eigen(S: Setup, C, eps, nocc, nroots: int, alpha_J=DEFAULT_ALPHA_J, c_x=DEFAULT_CX):
    """Lowest nroots eigenpairs of A^ris (TDA): omega[nroots] ascending and
    X[nroots][nvir][nocc] with unit norm (signs as numpy returns them)."""
    A = dense_a(S, C, eps, nocc, alpha_J, c_x)
    w, U = np.linalg.eigh(0.5 * (A + A.T))
    o = nocc
    v = C.shape[1] - o
    return w[:nroots], U[:, :nroots].T.reshape(nroots, v, o)


def zvector_solve(S: Setup, C, eps, nocc, rhs: np.ndarray, alpha_J=DEFAULT_ALPHA_J,
                  c_x=DEFAULT_CX) -> np.ndarray:
    """Z[k] = ((A+B)^ris)^-1 rhs[k] for rhs[nrhs][nvir][nocc] (Sec. 4.2 with
    eq. Z_vector of Sec. 2.1), by a direct dense solve."""
    M = dense_apb(S, C, eps, nocc, alpha_J, c_x)
    rhs = np.asarray(rhs, dtype=np.float64)
    Z = np.linalg.solve(M, rhs.reshape(rhs.shape[0], -1).T).T
    return Z.reshape(rhs.shape)


def ao_densities(C, nocc, X, Y):
    """R^S_I and L^A_I in the AO basis (Appendix A.1)."""
    CO = C[:, :nocc]
    CV = C[:, nocc:]
    R = X if Y is None else X + Y
    L = X if Y is None else X - Y
    RS, LA = [], []
    for I in range(X.shape[0]):
        Rm = CV @ R[I] @ CO.T
        Lm = CV @ L[I] @ CO.T
        RS.append(0.5 * (Rm + Rm.T))
        LA.append(0.5 * (Lm - Lm.T))
    return np.array(RS), np.array(LA)


def energy_functional(S: Setup, RS1, RS2, LA1, LA2, alpha_J=DEFAULT_ALPHA_J, c_x=DEFAULT_CX) -> float:
    """E_IJ at fixed AO densities (the bilinear ris functional)."""
    t1 = np.einsum("Pmn,mn->P", S.int3J, RS1)
    t2 = np.einsum("Pmn,mn->P", S.int3J, RS2)
    eJ = alpha_J * t1 @ metric_solve(S.MJ, t2)
    MKinv = np.linalg.inv(S.MK)
    eK = 0.0
    for D1, D2 in ((RS1, RS2), (LA1, LA2)):
        # S_PQ = sum (ml|P)(Q|ns) D1_mn D2_ls = tr(X_P^T D1 X_Q D2^T)
        Y = np.einsum("mn,Qns,ls->Qml", D1, S.int3K, D2, optimize=True)
        Spq = np.einsum("Pml,Qml->PQ", S.int3K, Y, optimize=True)
        eK += np.sum(MKinv * Spq)
    return float(eJ - c_x * eK)


def energy_at(mol, xyz, radius_bohr, RS1, RS2, LA1, LA2, alpha_J=DEFAULT_ALPHA_J, c_x=DEFAULT_CX,
              theta=DEFAULT_THETA, j_p_on_heavy=True) -> float:
    m2 = mol.with_xyz(xyz)
    S2 = setup(m2, radius_bohr, theta, j_p_on_heavy)
    return energy_functional(S2, RS1, RS2, LA1, LA2, alpha_J, c_x)


def pair_weights(S: Setup, D1, D2, alpha_J, c_x):
    """Weights of the derivative integrals for one density pair (D1, D2) of the
    bilinear functional a_J sum (mn|ls)_J D1_mn D2_ls - c_x sum (ml|ns)_K D1_mn D2_ls:
    W3J[P] = a_J (D1 c2_P + D2 c1_P), W2J = -a_J c1 c2^T           (Coulomb)
    W3K[P] = -c_x (D1 C^P D2^T + D1^T C^P D2), W2K[P,Q] = c_x V_PQ  (exchange)
    with c = M_J^-1 t, t_P = sum (mn|P) D_mn, C^P = sum_Q (M_K^-1)_PQ (Q|..),
    V_PQ = sum C^P_ml (D1 C^Q D2^T)_ml.  a_J = 0 skips the Coulomb part."""
    nJ = S.MJ.shape[0]
    nK = S.MK.shape[0]
    if alpha_J != 0.0:
        t1 = np.einsum("Pmn,mn->P", S.int3J, D1)
        t2 = np.einsum("Pmn,mn->P", S.int3J, D2)
        c1 = metric_solve(S.MJ, t1)
        c2 = metric_solve(S.MJ, t2)
        W3J = alpha_J * (D1[None] * c2[:, None, None] + D2[None] * c1[:, None, None])
        W2J = -alpha_J * np.outer(c1, c2)
    else:
        W3J = np.zeros((nJ,) + D1.shape)
        W2J = np.zeros((nJ, nJ))
    MKinv = np.linalg.inv(S.MK)
    Cp = np.einsum("PQ,Qmn->Pmn", MKinv, S.int3K, optimize=True)
    G = np.einsum("mn,Pns,ls->Pml", D1, Cp, D2, optimize=True)        # D1 C^P D2^T
    Gt = np.einsum("nm,Pns,sl->Pml", D1, Cp, D2, optimize=True)       # D1^T C^P D2
    W3K = -c_x * (G + Gt)
    V = np.einsum("Pml,Qml->PQ", Cp, G, optimize=True)
    W2K = c_x * V
    return W3J, W2J, W3K, W2K


def ris_derivative(S: Setup, natm: int, pairs, atom_mask=None) -> np.ndarray:
    """Nuclear derivative of a sum of bilinear ris functionals for a list of
    outputs.  Each output is a list of (D1, D2, a_J, c_x) terms, each the
    functional a_J sum (mn|ls)_J D1_mn D2_ls - c_x sum (ml|ns)_K D1_mn D2_ls;
    returns [nout][natm][3] (Ha/Bohr)."""
    nout = len(pairs)
    nJ = S.MJ.shape[0]
    nK = S.MK.shape[0]
    nao = S.int3J.shape[1]
    g = np.zeros((nout, natm, 3))
    # batch outputs to bound memory (~2 GB of weights per batch)
    per = (nJ + nK) * nao * nao * 8
    bs = max(1, min(nout, int(2e9 // max(per, 1))))
    for o0 in range(0, nout, bs):
        ob = range(o0, min(nout, o0 + bs))
        W3J = np.zeros((len(ob), nJ, nao, nao))
        W3K = np.zeros((len(ob), nK, nao, nao))
        W2J = np.zeros((len(ob), nJ, nJ))
        W2K = np.zeros((len(ob), nK, nK))
        for k, o in enumerate(ob):
            for (D1, D2, aJ, cx) in pairs[o]:
                a, b, c, d = pair_weights(S, D1, D2, aJ, cx)
                if S.scale is not None:   # scaled auxiliary functions (P7): (mn|P)^x scales with P
                    sJ, sK = S.scale, S.scale[:nK]
                    a, b = a * sJ[:, None, None], b * np.outer(sJ, sJ)
                    c, d = c * sK[:, None, None], d * np.outer(sK, sK)
                W3J[k] += a
                W2J[k] += b
                W3K[k] += c
                W2K[k] += d
        g[o0:o0 + len(ob)] += int3c_grad(S.ao, S.aux.J, natm, W3J, atom_mask)
        g[o0:o0 + len(ob)] += int3c_grad(S.ao, S.aux.K, natm, W3K, atom_mask)
        g[o0:o0 + len(ob)] += int2c_grad(S.aux.J, natm, W2J)
        g[o0:o0 + len(ob)] += int2c_grad(S.aux.K, natm, W2K)
    return g


def output_pairs(RS, LA, I: int, J: int, alpha_J=DEFAULT_ALPHA_J, c_x=DEFAULT_CX):
    """Density pairs of E_IJ: the Coulomb + exchange pair {R^S_I, R^S_J} and the
    exchange-only pair {L^A_I, L^A_J} (the Coulomb contraction of an
    antisymmetric density vanishes)."""
    return [(RS[I], RS[J], alpha_J, c_x), (LA[I], LA[J], 0.0, c_x)]


def grad_nac(prob, radius_bohr, outputs, alpha_J=DEFAULT_ALPHA_J, c_x=DEFAULT_CX,
             theta=DEFAULT_THETA, j_p_on_heavy=True, extra=None, S: Setup | None = None):
    """ris gradient (I == J) / NAC numerator (I != J) for each (I, J) in outputs,
    [nout][natm][3] in Ha/Bohr.

    `extra` optionally adds density pairs to single outputs: a list of
    (k, D1, D2, cJ, cK), each adding to output k the nuclear derivative of
    cJ sum (mn|ls)_J D1_mn D2_ls - cK sum (ml|ns)_K D1_mn D2_ls at fixed AO
    matrices D1, D2 over the same ris auxiliary sets.  This is how the
    ground-state density D and the relaxed density P_I = T_II + Z^S (or the
    difference density T_IJ) enter the <g^(xi); {D, P}> terms of the
    gradient and NAC expressions (Sec. 2.2, eqs. gI_xi_ris and gIJ_xi_ris;
    Appendix A.1 eq. T and A.2), taken here over the ris auxiliary basis
    because the full density-fitting basis is not part of the path."""
    mol = prob.mol
    if S is None:
        S = setup(mol, radius_bohr, theta, j_p_on_heavy)
    RS, LA = ao_densities(prob.C, prob.nocc, prob.X, prob.Y)
    pairs = [output_pairs(RS, LA, I, J, alpha_J, c_x) for (I, J) in outputs]
    for (k, D1, D2, cJ, cK) in (extra or ()):
        pairs[k].append((D1, D2, cJ, cK))
    return ris_derivative(S, mol.natm, pairs)


# ------------------------------------------- densities of Appendix A.1-A.2 --
def ground_density(C, nocc):
    """D = C [[1, 0], [0, 0]] C^T: the occupied projector in the AO basis
    (the matrix D of Appendix A.3 carried to the AO basis)."""
    CO = C[:, :nocc]
    return CO @ CO.T


def difference_density(C, nocc, X, Y, I: int, J: int):
    """T_IJ = (gamma + gamma^T) / 2 in the AO basis with the MO matrix
    gamma^IJ = [[-(X_J^T X_I + Y_I^T Y_J)_ij, 0], [0, (X_I X_J^T + Y_J Y_I^T)_ab]]
    (Appendix A.1, eq. T); amplitudes X[a][i] (Y = None: TDA)."""
    o = nocc
    nmo = C.shape[1]
    XI, XJ = X[I], X[J]
    YI = np.zeros_like(XI) if Y is None else Y[I]
    YJ = np.zeros_like(XJ) if Y is None else Y[J]
    g = np.zeros((nmo, nmo))
    g[:o, :o] = -(XJ.T @ XI + YI.T @ YJ)
    g[o:, o:] = XI @ XJ.T + YJ @ YI.T
    Tm = 0.5 * (g + g.T)
    return C @ Tm @ C.T


def z_symmetric(C, nocc, Z):
    """Z^S = (Z + Z^T) / 2 with Z = C_V Z C_O^T (Appendix A.2); Z[a][i]."""
    Zm = C[:, nocc:] @ Z @ C[:, :nocc].T
    return 0.5 * (Zm + Zm.T)


def relaxed_density(C, nocc, X, Y, I: int, Z, J: int | None = None):
    """P_I = T_II + Z^S (gradient), or P_IJ = T_IJ + Z~^S when J is given and Z
    is the scaled multiplier of the coupling (Appendix A.2)."""
    J = I if J is None else J
    return difference_density(C, nocc, X, Y, I, J) + z_symmetric(C, nocc, Z)
