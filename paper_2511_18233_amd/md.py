"""Consumers of the gradients and NACs in a surface-hopping-shaped loop.

Small host-side algebra on per-atom vectors ([natm][3] arrays), applied to
what the library returns:

* ``time_derivative_coupling``: T_IJ = g_IJ . v, the quantity that sets the
  fewest-switches hopping probability (Sec. 5.4).
* ``mecp_effective_gradient``: the effective gradient of a minimum-energy
  crossing point search (Sec. 5.3): g_eff = f + P g_J with x1 = g_J - g_I,
  f = (E_J - E_I) x1 / |x1| and P the projector onto the orthogonal
  complement of the branching plane spanned by x1 and g_IJ.
* ``phase_signs``: the phase of each excited state fixed against the previous
  step by the overlap over the five most dominant single excitations
  (Sec. 3, last paragraph), including the sign each MO keeps between steps.
"""
from __future__ import annotations

import numpy as np


def time_derivative_coupling(nac: np.ndarray, velocity: np.ndarray) -> float:
    """T_IJ = sum_A g_IJ[A] . v[A] for one NAC vector and nuclear velocities."""
    nac = np.asarray(nac, dtype=np.float64)
    velocity = np.asarray(velocity, dtype=np.float64)
    if nac.shape != velocity.shape:
        raise ValueError(f"shape mismatch {nac.shape} vs {velocity.shape}")
    return float(np.sum(nac * velocity))


def branching_plane(x1: np.ndarray, x2: np.ndarray, tiny: float = 1e-14) -> np.ndarray:
    """Orthonormal basis (rows) of span{x1, x2} by Gram-Schmidt on the flattened
    vectors; a vector that is (numerically) dependent on the previous ones is
    dropped."""
    basis = []
    for x in (np.ravel(x1), np.ravel(x2)):
        y = np.array(x, dtype=np.float64)
        for b in basis:
            y = y - (b @ y) * b
        n = np.linalg.norm(y)
        if n > tiny * max(1.0, np.linalg.norm(x)):
            basis.append(y / n)
    return np.array(basis).reshape(len(basis), -1)


def mecp_effective_gradient(g_i: np.ndarray, g_j: np.ndarray, nac_ij: np.ndarray, e_i: float,
                            e_j: float) -> np.ndarray:
    """g_eff = (E_J - E_I) x1 / |x1| + P g_J, x1 = g_J - g_I, P = 1 - sum_b b b^T
    over an orthonormal basis b of span{x1, g_IJ}; same shape as g_j."""
    g_i = np.asarray(g_i, dtype=np.float64)
    g_j = np.asarray(g_j, dtype=np.float64)
    x1 = g_j - g_i
    n1 = np.linalg.norm(x1)
    f = (e_j - e_i) * x1 / n1 if n1 > 0.0 else np.zeros_like(x1)
    B = branching_plane(x1, nac_ij)
    gj = g_j.ravel()
    pg = gj - B.T @ (B @ gj) if B.size else gj.copy()
    return f + pg.reshape(g_j.shape)


def phase_signs(X_prev: np.ndarray, X_cur: np.ndarray, C_prev: np.ndarray, C_cur: np.ndarray, S_cur: np.ndarray,
                nocc: int, ndet: int = 5) -> np.ndarray:
    """+1 / -1 per state: the sign that makes state I at the current step
    continue state I of the previous step.

    X_prev, X_cur: [nstate][nvir][nocc] amplitudes; C_prev, C_cur: [nao][nmo]
    MO coefficients of the two steps; S_cur: AO overlap at the current
    geometry (for small steps it stands in for the mixed-geometry overlap).
    MO p keeps the sign d_p = sign(C_prev[:, p] . S_cur C_cur[:, p]); the
    overlap of state I is taken over its ndet largest |X_prev| excitations
    (a, i): s_I = sum X_prev[a, i] X_cur[a, i] d_a d_i, and the sign is that
    of s_I (+1 when s_I is 0)."""
    X_prev = np.asarray(X_prev, dtype=np.float64)
    X_cur = np.asarray(X_cur, dtype=np.float64)
    d = np.sign(np.einsum("mp,mp->p", C_prev, S_cur @ C_cur))   # diag(C_prev^T S C_cur)
    d[d == 0] = 1.0
    dv, do = d[nocc:], d[:nocc]
    out = np.ones(X_prev.shape[0])
    for I in range(X_prev.shape[0]):
        flat = np.abs(X_prev[I]).ravel()
        k = min(ndet, flat.size)
        top = np.argpartition(-flat, k - 1)[:k]
        a, i = np.unravel_index(top, X_prev[I].shape)
        s = float(np.sum(X_prev[I][a, i] * X_cur[I][a, i] * dv[a] * do[i]))
        out[I] = -1.0 if s < 0.0 else 1.0
    return out
