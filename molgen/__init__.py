"""Seeded synthetic molecules, basis sets, orbitals and amplitudes.

This module only builds inputs: geometry, an uncontracted Cartesian AO basis,
orthonormal molecular orbitals C = S^{-1/2} Q, orbital energies and response
amplitudes X (and Y).  It holds none of the TDDFT-ris arithmetic: no Coulomb
integrals, no auxiliary basis, no metric, no response or gradient terms.  Both
the CPU oracle and the GPU path consume what it returns.

Workloads (all lengths in Bohr internally):

* ``ring``  -- 6 C on a ring (bond 1.40 A +-0.03 jitter, z jitter +-0.03 A)
  plus 6 H at 1.09 A radially outward.  Basis C s{0.15,0.6,2.4} p{0.3,1.2},
  H s{0.2,1.0}.
* ``chain`` -- seeded self-avoiding chain of C/N/O (6:1:1), bonds U(1.35,1.50) A,
  bond angle 120+-10 deg, random dihedral, non-bonded heavy-heavy >= 2.5 A,
  H-capped at 1.09 A.  Basis as ``ring`` plus d{0.8} on heavy atoms and
  p{1.0} on H.

Orbitals: Loewdin S^{-1/2} times a Haar-random orthogonal Q (QR of a seeded
Gaussian with diag(R) > 0), nmo = nao, orbital energies sorted U(-1, 0.5) Ha,
nocc = n_electrons / 2.  Amplitudes X_ai = u_ai / (e_a - e_i) normalised;
for full TDDFT Y_ai = 0.1 w_ai / (e_a - e_i), then (X, Y) scaled so that
X.X - Y.Y = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ANGSTROM_TO_BOHR = 1.0 / 0.529177210903
ZNUC = {"H": 1, "C": 6, "N": 7, "O": 8}
SYMBOL = {1: "H", 6: "C", 7: "N", 8: "O"}
# classical covalent radii (Angstrom) used for the ris exponent rule; C and H
# are fixed by the workload definition, N and O are the matching table values
COVALENT_RADIUS_ANG = {1: 0.37, 6: 0.77, 7: 0.75, 8: 0.73}

# (l, exponent) per element; heavy atoms N, O share the C basis
BASIS_SMALL = {
    "C": [(0, 0.15), (0, 0.6), (0, 2.4), (1, 0.3), (1, 1.2)],
    "H": [(0, 0.2), (0, 1.0)],
}
BASIS_SMALL["N"] = BASIS_SMALL["C"]
BASIS_SMALL["O"] = BASIS_SMALL["C"]
BASIS_LARGE = {
    "C": BASIS_SMALL["C"] + [(2, 0.8)],
    "H": BASIS_SMALL["H"] + [(1, 1.0)],
}
BASIS_LARGE["N"] = BASIS_LARGE["C"]
BASIS_LARGE["O"] = BASIS_LARGE["C"]

NCART = (1, 3, 6)
# Cartesian component order inside a shell: x,y,z and xx,xy,xz,yy,yz,zz
CART = {
    0: [(0, 0, 0)],
    1: [(1, 0, 0), (0, 1, 0), (0, 0, 1)],
    2: [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)],
}


@dataclass
class Molecule:
    Z: np.ndarray            # [natm] int32 nuclear charges
    xyz: np.ndarray          # [natm, 3] float64, Bohr
    shell_atom: np.ndarray   # [nshell] int32
    shell_l: np.ndarray      # [nshell] int32
    shell_exp: np.ndarray    # [nshell] float64

    @property
    def natm(self) -> int:
        return int(self.Z.shape[0])

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nao(self) -> int:
        return int(sum(NCART[l] for l in self.shell_l))

    @property
    def nelec(self) -> int:
        return int(self.Z.sum())

    def with_xyz(self, xyz: np.ndarray) -> "Molecule":
        return Molecule(self.Z.copy(), np.ascontiguousarray(xyz, dtype=np.float64),
                        self.shell_atom.copy(), self.shell_l.copy(), self.shell_exp.copy())


@dataclass
class Problem:
    """One gradient/NAC request: molecule, orbitals and amplitudes."""
    mol: Molecule
    C: np.ndarray            # [nao, nmo]
    eps: np.ndarray          # [nmo]
    nocc: int
    X: np.ndarray            # [nstate, nvir, nocc]
    Y: np.ndarray | None     # [nstate, nvir, nocc] or None (TDA)
    meta: dict = field(default_factory=dict)

    @property
    def nstate(self) -> int:
        return int(self.X.shape[0])


def radii_bohr_table() -> np.ndarray:
    """[119] covalent radius (Bohr) by Z, 0 where undefined."""
    t = np.zeros(119)
    for z, r in COVALENT_RADIUS_ANG.items():
        t[z] = r * ANGSTROM_TO_BOHR
    return t


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def ring_geometry(rng: np.random.Generator) -> tuple[list[int], np.ndarray]:
    Z, pos = [], []
    for k in range(6):
        ang = math.radians(60.0 * k)
        r = 1.40 + rng.uniform(-0.03, 0.03)
        z = rng.uniform(-0.03, 0.03)
        Z.append(6)
        pos.append([r * math.cos(ang), r * math.sin(ang), z])
    for k in range(6):
        ang = math.radians(60.0 * k)
        c = np.array(pos[k])
        u = np.array([math.cos(ang), math.sin(ang), 0.0])
        Z.append(1)
        pos.append(list(c + 1.09 * u))
    return Z, np.array(pos) * ANGSTROM_TO_BOHR


def _perp(u: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal(3)
    v -= v.dot(u) * u
    return v / np.linalg.norm(v)


def chain_geometry(natm_target: int, rng: np.random.Generator) -> tuple[list[int], np.ndarray]:
    """Self-avoiding heavy-atom chain with H caps; returns (Z, xyz Bohr)."""
    valence = {6: 3, 7: 2, 8: 2}

    def n_h(elems: list[int]) -> int:
        n = len(elems)
        tot = 0
        for k, e in enumerate(elems):
            nb = (1 if k > 0 else 0) + (1 if k < n - 1 else 0)
            tot += max(0, valence[e] - nb)
        return tot

    def pick() -> int:
        r = rng.integers(0, 8)
        return 6 if r < 6 else (7 if r == 6 else 8)

    heavy_Z: list[int] = [pick()]
    heavy: list[np.ndarray] = [np.zeros(3)]
    while len(heavy) + n_h(heavy_Z) < natm_target:
        for _attempt in range(200):
            bond = rng.uniform(1.35, 1.50)
            if len(heavy) == 1:
                d = rng.standard_normal(3)
                d /= np.linalg.norm(d)
            else:
                u = heavy[-1] - heavy[-2]
                u /= np.linalg.norm(u)
                theta = math.radians(120.0 + rng.uniform(-10.0, 10.0))
                if len(heavy) >= 3:
                    w = heavy[-2] - heavy[-3]
                    w -= w.dot(u) * u
                    nw = np.linalg.norm(w)
                    w = w / nw if nw > 1e-8 else _perp(u, rng)
                else:
                    w = _perp(u, rng)
                w2 = np.cross(u, w)
                phi = rng.uniform(0.0, 2.0 * math.pi)
                # the new bond leaves at angle theta to the previous bond
                d = -math.cos(theta) * u + math.sin(theta) * (math.cos(phi) * w + math.sin(phi) * w2)
                d = d / np.linalg.norm(d)
            cand = heavy[-1] + bond * d
            ok = all(np.linalg.norm(cand - heavy[k]) >= 2.5 for k in range(len(heavy) - 1))
            if ok:
                heavy.append(cand)
                heavy_Z.append(pick())
                break
        else:
            raise RuntimeError("chain generator could not place an atom")

    nheavy = len(heavy)
    Z = list(heavy_Z)
    pos = [p.copy() for p in heavy]
    h_parent: list[int] = []
    for k in range(nheavy):
        nbrs = [j for j in (k - 1, k + 1) if 0 <= j < nheavy]
        nh = max(0, valence[heavy_Z[k]] - len(nbrs))
        if nh == 0:
            continue
        us = [(heavy[j] - heavy[k]) / np.linalg.norm(heavy[j] - heavy[k]) for j in nbrs]
        if len(us) == 2:
            b = -(us[0] + us[1])
            nb = np.linalg.norm(b)
            dirs = [b / nb if nb > 1e-8 else _perp(us[0], rng)]
        else:
            u = us[0] if us else np.array([0.0, 0.0, 1.0])
            w = _perp(u, rng)
            w2 = np.cross(u, w)
            phi0 = rng.uniform(0.0, 2.0 * math.pi)
            theta = math.radians(120.0)
            dirs = []
            for m in range(nh):
                phi = phi0 + 2.0 * math.pi * m / nh
                dirs.append(math.cos(theta) * u + math.sin(theta) * (math.cos(phi) * w + math.sin(phi) * w2))
        for m in range(nh):
            Z.append(1)
            pos.append(heavy[k] + 1.09 * dirs[m % len(dirs)])
            h_parent.append(k)
    # trim H (from the end) down to the target count, then fix electron parity
    while len(Z) > natm_target and Z[-1] == 1:
        Z.pop()
        pos.pop()
    if sum(Z) % 2 == 1:
        idx = max(i for i, z in enumerate(Z) if z == 1)
        Z.pop(idx)
        pos.pop(idx)
    return Z, np.array(pos) * ANGSTROM_TO_BOHR


def build_shells(Z: list[int], basis: dict) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    sa, sl, se = [], [], []
    for a, z in enumerate(Z):
        for (l, e) in basis[SYMBOL[z]]:
            sa.append(a)
            sl.append(l)
            se.append(e)
    return (np.array(sa, dtype=np.int32), np.array(sl, dtype=np.int32),
            np.array(se, dtype=np.float64))


# --------------------------------------------------------------------------
# overlap (only to build orthonormal orbitals)
# --------------------------------------------------------------------------
def _dfact(n: int) -> float:
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


def cart_norm(alpha: float, lx: int, ly: int, lz: int) -> float:
    l = lx + ly + lz
    return ((2.0 * alpha / math.pi) ** 0.75 * (4.0 * alpha) ** (l / 2.0)
            / math.sqrt(_dfact(2 * lx - 1) * _dfact(2 * ly - 1) * _dfact(2 * lz - 1)))


def ao_offsets(mol: Molecule) -> np.ndarray:
    off = np.zeros(mol.nshell + 1, dtype=np.int64)
    for s in range(mol.nshell):
        off[s + 1] = off[s] + NCART[mol.shell_l[s]]
    return off


def overlap_matrix(mol: Molecule) -> np.ndarray:
    """AO overlap by the 1D Obara-Saika recursion, vectorised over shell pairs."""
    off = ao_offsets(mol)
    nao = int(off[-1])
    S = np.zeros((nao, nao))
    A_all = mol.xyz[mol.shell_atom]
    # component normalisations per shell (the same scalar formula, once per shell)
    cnorm = [np.array([[cart_norm(float(e), *c) for c in CART[l]] for e in mol.shell_exp]) for l in range(3)]
    for la in range(3):
        for lb in range(3):
            ia = np.nonzero(mol.shell_l == la)[0]
            ib = np.nonzero(mol.shell_l == lb)[0]
            if ia.size == 0 or ib.size == 0:
                continue
            I, J = np.meshgrid(ia, ib, indexing="ij")
            I = I.ravel()
            J = J.ravel()
            a = mol.shell_exp[I]
            b = mol.shell_exp[J]
            p = a + b
            A = A_all[I]
            B = A_all[J]
            P = (a[:, None] * A + b[:, None] * B) / p[:, None]
            PA = P - A
            PB = P - B
            AB2 = ((A - B) ** 2).sum(1)
            s00 = (math.pi / p) ** 1.5 * np.exp(-a * b / p * AB2)
            # 1D tables s[d][i][j] (unit prefactor), i<=la, j<=lb
            oneD = []
            for d in range(3):
                t = np.zeros((la + 1, lb + 1, I.size))
                t[0, 0] = 1.0
                for i in range(la + 1):
                    for j in range(lb + 1):
                        if i == 0 and j == 0:
                            continue
                        if i > 0:
                            v = PA[:, d] * t[i - 1, j]
                            if i > 1:
                                v = v + (i - 1) / (2 * p) * t[i - 2, j]
                            if j > 0:
                                v = v + j / (2 * p) * t[i - 1, j - 1]
                        else:
                            v = PB[:, d] * t[i, j - 1]
                            if j > 1:
                                v = v + (j - 1) / (2 * p) * t[i, j - 2]
                        t[i, j] = v
                oneD.append(t)
            for ca, (ax, ay, az) in enumerate(CART[la]):
                na = cnorm[la][I, ca]
                for cb, (bx, by, bz) in enumerate(CART[lb]):
                    nb = cnorm[lb][J, cb]
                    val = s00 * na * nb * oneD[0][ax, bx] * oneD[1][ay, by] * oneD[2][az, bz]
                    S[off[I] + ca, off[J] + cb] = val
    return S


# --------------------------------------------------------------------------
# orbitals and amplitudes
# --------------------------------------------------------------------------
def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))[None, :]


def make_orbitals(mol: Molecule, rng: np.random.Generator):
    S = overlap_matrix(mol)
    w, V = np.linalg.eigh(S)
    if w.min() <= 1e-10:
        raise RuntimeError(f"AO overlap nearly singular (min eig {w.min():.3e})")
    Sm12 = (V * (1.0 / np.sqrt(w))[None, :]) @ V.T
    nmo = mol.nao
    Q = haar_orthogonal(nmo, rng)
    C = Sm12 @ Q
    eps = np.sort(rng.uniform(-1.0, 0.5, nmo))
    nocc = mol.nelec // 2
    return np.ascontiguousarray(C), eps, nocc


def make_amplitudes(eps: np.ndarray, nocc: int, nstate: int, tda: bool,
                    rng: np.random.Generator):
    e_o = eps[:nocc]
    e_v = eps[nocc:]
    de = e_v[:, None] - e_o[None, :]           # [nvir, nocc], may be <= 0 rarely
    de = np.where(np.abs(de) < 1e-3, np.copysign(1e-3, de + 1e-300), de)
    nvir = e_v.size
    X = np.empty((nstate, nvir, nocc))
    Y = None if tda else np.empty((nstate, nvir, nocc))
    for s in range(nstate):
        x = rng.standard_normal((nvir, nocc)) / de
        if tda:
            X[s] = x / np.linalg.norm(x)
        else:
            y = 0.1 * rng.standard_normal((nvir, nocc)) / de
            nrm2 = (x * x).sum() - (y * y).sum()
            if nrm2 <= 0:
                y *= 0.0
                nrm2 = (x * x).sum()
            sc = 1.0 / math.sqrt(nrm2)
            X[s] = x * sc
            Y[s] = y * sc
    return X, Y


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
WORKLOADS = {
    # name: (geometry kind, natm target, basis, nstate, tda)
    "ring12": ("ring", 12, BASIS_SMALL, 3, True),
    "chain60": ("chain", 60, BASIS_LARGE, 10, False),
    "chain200": ("chain", 200, BASIS_LARGE, 10, False),
    "chain500": ("chain", 500, BASIS_LARGE, 20, False),
}
WORKLOAD_SEED = {"ring12": 0, "chain60": 1, "chain200": 2, "chain500": 4}


def make_molecule(kind: str, natm: int, basis: dict, rng: np.random.Generator) -> Molecule:
    if kind == "ring":
        Z, xyz = ring_geometry(rng)
    else:
        Z, xyz = chain_geometry(natm, rng)
    sa, sl, se = build_shells(Z, basis)
    return Molecule(np.array(Z, dtype=np.int32), np.ascontiguousarray(xyz), sa, sl, se)


def make_problem(name: str, seed: int | None = None, nstate: int | None = None,
                 tda: bool | None = None) -> Problem:
    """Build one of the named workloads (seeded)."""
    kind, natm, basis, ns, td = WORKLOADS[name]
    if seed is None:
        seed = WORKLOAD_SEED[name]
    ns = ns if nstate is None else nstate
    td = td if tda is None else tda
    rng = np.random.default_rng(seed)
    mol = make_molecule(kind, natm, basis, rng)
    C, eps, nocc = make_orbitals(mol, rng)
    X, Y = make_amplitudes(eps, nocc, ns, td, rng)
    return Problem(mol, C, eps, nocc, X, Y, dict(name=name, seed=seed))


def make_chain_problem(natm: int, seed: int, nstate: int, tda: bool = False,
                       small_basis: bool = False) -> Problem:
    """Chain molecule of any size (serving requests, parity sweeps)."""
    rng = np.random.default_rng(seed)
    mol = make_molecule("chain", natm, BASIS_SMALL if small_basis else BASIS_LARGE, rng)
    C, eps, nocc = make_orbitals(mol, rng)
    X, Y = make_amplitudes(eps, nocc, nstate, tda, rng)
    return Problem(mol, C, eps, nocc, X, Y, dict(name=f"chain{natm}", seed=seed))


def make_tiny_problem(seed: int, natm: int = 3, lmax: int = 2, nstate: int = 2,
                      tda: bool = False, elements=(6, 1, 8), spread: float = 2.2) -> Problem:
    """A few atoms at random positions with a small mixed-l basis (test sizes)."""
    rng = np.random.default_rng(seed)
    Z = [int(elements[k % len(elements)]) for k in range(natm)]
    pos = []
    while len(pos) < natm:
        c = rng.uniform(-spread, spread, 3)
        if all(np.linalg.norm(c - q) > 1.6 for q in pos):
            pos.append(c)
    basis = {}
    for z in set(Z):
        sym = SYMBOL[z]
        sh = [(0, 0.3 + 0.2 * (z % 3)), (0, 1.3)]
        if lmax >= 1:
            sh.append((1, 0.7))
        if lmax >= 2 and z != 1:
            sh.append((2, 0.9))
        basis[sym] = sh
    sa, sl, se = build_shells(Z, basis)
    mol = Molecule(np.array(Z, dtype=np.int32), np.array(pos), sa, sl, se)
    nelec = mol.nelec
    C, eps, _ = make_orbitals(mol, rng)
    nocc = max(1, min(nelec // 2, mol.nao - 1))
    X, Y = make_amplitudes(eps, nocc, nstate, tda, rng)
    return Problem(mol, C, eps, nocc, X, Y, dict(name=f"tiny{natm}", seed=seed))
