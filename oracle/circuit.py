"""Circuit simulation by BP-gauged simple update (FP64 oracle).  TEST
INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper:

* Methods, "Quantum Circuit Simulation": a two-qubit gate is applied exactly to
  the pair of site tensors it acts on and the bond between them is truncated
  back to its dimension by an SVD, with the environment of the pair replaced by
  the BP messages of the norm network; the messages are refreshed between
  layers of gates that share no qubit.  The gate error is the discarded weight
  of the normalised singular values, eps_i (Eq. error_per_gate), and the
  fidelity estimate f = prod_i (1 - eps_i) (Eq. total_fidelity);
* Appendix, "Applying Gates to a Tensor Network State": the pair is gauged with
  the square roots of its incoming messages, the gate applied, the SVD taken,
  and the gauge undone with the inverse square roots.

The circuit (gate list, gate matrix, colour groups, initial state) is an input:
``peps_inputs.circuits``.  Site tensors are [p][u][l][d][r]; messages are the
BP oracle's (``oracle.bp``: into site (r, c) through a leg, m[k][k'] with k the
ket index).

Readings where the paper is silent:

* the square root of a message (Hermitian and positive in exact arithmetic) is
  U diag(sqrt(lambda)) U^H over its eigenvalues lambda > 1e-12 lambda_max, the
  others (rounding of a rank-deficient message, e.g. a product state's) taken
  as 0; the inverse square root keeps 1 / sqrt(lambda) over the same
  eigenvalues (a pseudo-inverse: the gauge round trip projects each leg on the
  support of its message, which leaves the pair's contraction with its
  neighbour unchanged);
* the bond keeps the lattice dimension D: the SVD keeps min(D, rank) values,
  rank = the count of singular values above 1e-12 of the largest; the kept
  factors are U sqrt(S) on the first qubit's side and sqrt(S) V^H on the
  second's, zero-padded to D;
* eps is the discarded weight over all singular values, sum_{j >= k} s_j^2 /
  sum_j s_j^2 (the rank cut's part is below 1e-24);
* gates in one group act on disjoint qubits and use the messages computed at
  the start of the group, in the order of the gate list; each group's BP starts
  from the converged messages of the group before (the first from identity /
  sqrt(D)), run to the same tolerance.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from . import bp as obp

UP, LEFT, DOWN, RIGHT = obp.UP, obp.LEFT, obp.DOWN, obp.RIGHT
RANK_RTOL = 1e-12
LEGS = (UP, LEFT, DOWN, RIGHT)


def message_roots(m: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """(sqrt(m), pseudo-inverse of sqrt(m)) of a Hermitian positive message."""
    lam, U = np.linalg.eigh(0.5 * (m + m.conj().T))
    keep = lam > RANK_RTOL * max(float(lam.max()), 0.0)
    s = np.where(keep, np.sqrt(np.where(keep, lam, 1.0)), 0.0)
    si = np.where(keep, 1.0 / np.where(keep, s, 1.0), 0.0)
    return (U * s) @ U.conj().T, (U * si) @ U.conj().T


def _leg_times(A: np.ndarray, leg: int, X: np.ndarray) -> np.ndarray:
    """A'[.., j, ..] = sum_k A[.., k, ..] X[k, j] on axis ``leg``."""
    return np.moveaxis(np.tensordot(A, X, axes=(leg, 0)), -1, leg)


def bond_legs(r, c, r2, c2):
    if (r2, c2) == (r, c + 1):
        return RIGHT, LEFT
    if (r2, c2) == (r + 1, c):
        return DOWN, UP
    raise ValueError("a gate acts on grid neighbours (r, c), (r, c + 1) or (r + 1, c)")


def apply_gate(T, M, r, c, r2, c2, G) -> float:
    """Replaces T[r][c] and T[r2][c2] (in place) by the gauged, gate-applied,
    truncated pair; returns the gate error eps."""
    lv, lw = bond_legs(r, c, r2, c2)
    A, B = T[r][c], T[r2][c2]
    De = A.shape[lv]
    ext_v = [x for x in LEGS if x != lv]
    ext_w = [x for x in LEGS if x != lw]
    Rv = {x: message_roots(M[(r, c, x)]) for x in ext_v}
    Rw = {x: message_roots(M[(r2, c2, x)]) for x in ext_w}
    for x in ext_v:
        A = _leg_times(A, x, Rv[x][0])
    for x in ext_w:
        B = _leg_times(B, x, Rw[x][0])
    Av = np.moveaxis(A, lv, -1)                 # [s, e1, e2, e3, bond]
    Bw = np.moveaxis(B, lw, 0)                  # [bond, t, f1, f2, f3]
    theta = np.tensordot(Av, Bw, axes=(-1, 0))  # [s, e1, e2, e3, t, f1, f2, f3]
    theta = np.moveaxis(theta, 4, 1)            # [s, t, e.., f..]
    theta = np.tensordot(G.reshape(2, 2, 2, 2), theta, axes=([2, 3], [0, 1]))
    theta = np.moveaxis(theta, 1, 4)            # [s, e.., t, f..]
    sv, sw = Av.shape[:-1], Bw.shape[1:]
    mat = theta.reshape(int(np.prod(sv)), int(np.prod(sw)))
    mat = mat / np.linalg.norm(mat)
    U, S, Vh = np.linalg.svd(mat, full_matrices=False)
    rank = int(np.count_nonzero(S > RANK_RTOL * S[0]))
    k = min(De, rank)
    eps = float(np.sum(S[k:] ** 2) / np.sum(S ** 2))
    ua = np.zeros((mat.shape[0], De), dtype=np.complex128)
    vb = np.zeros((De, mat.shape[1]), dtype=np.complex128)
    ua[:, :k] = U[:, :k] * np.sqrt(S[:k])
    vb[:k] = np.sqrt(S[:k])[:, None] * Vh[:k]
    An = np.moveaxis(ua.reshape(sv + (De,)), -1, lv)
    Bn = np.moveaxis(vb.reshape((De,) + sw), 0, lw)
    for x in ext_v:
        An = _leg_times(An, x, Rv[x][1])
    for x in ext_w:
        Bn = _leg_times(Bn, x, Rw[x][1])
    T[r][c], T[r2][c2] = An, Bn
    return eps


def simple_update(T, gates, G, bp_sweeps: int = 1000, bp_tol: float = 1e-13):
    """Applies the gate list (``peps_inputs.circuits``: (group, r, c, r2, c2))
    with gate matrix G (4 x 4, or one per gate) to a copy of T, refreshing the
    BP messages whenever the group changes.  Returns (tensors, eps list,
    f = prod (1 - eps))."""
    T = [[t.copy() for t in row] for row in T]
    Gs = G if (isinstance(G, np.ndarray) and G.ndim == 3) or isinstance(G, list) else None
    eps: List[float] = []
    cur = None
    M = None
    for i, (grp, r, c, r2, c2) in enumerate(gates):
        if grp != cur:
            M, _, _ = obp.bp_messages(T, max_iter=bp_sweeps, tol=bp_tol, init=M)
            cur = grp
        eps.append(apply_gate(T, M, r, c, r2, c2, Gs[i] if Gs is not None else G))
    f = float(np.prod([1.0 - e for e in eps]))
    return T, eps, f
