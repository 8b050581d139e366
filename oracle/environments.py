"""Local expectation values from the stored boundary MPSs (FP64 oracle).

The paper computes local observables directly by boundary-MPS contraction of
<psi|Z_i|psi> and <psi|psi> (Results, "Discrete-time dynamics of the
Heisenberg model", Fig. 4). Here:

* boundaries from below come from ``boundary_set`` (bottom-up) and boundaries
  from above from the same routine on the vertically mirrored lattice;
* within row r, double-layer row environments between the boundary above and
  the boundary below give the one-site reduced density matrix rho_i (site open,
  other sites of the row traced), and the diagonal of the two-site marginal of
  horizontally adjacent qubits;
* vertically adjacent qubits (r, c), (r+1, c) use a two-row environment between
  the boundary above row r and the boundary below row r+1.

<Z_i> = Re(rho_00 - rho_11) / Re(rho_00 + rho_11); <Z_i Z_j> = sum_{s,t}
(-1)^{s+t} Re P2[s,t] / sum Re P2. Entries touching a dummy site are NaN.
Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from .boundary import boundary_set, flip_vertical
from .philox import TAG_INIT_DOWN, TAG_INIT_UP

ein = lambda expr, *ops: np.einsum(expr, *ops, optimize=True)  # noqa: E731


def _unit(x):
    return x / np.linalg.norm(x)


def row_env_left(Le, U, A, B, s=None, t=None):
    """[p,h,k,g] -> [P,H,K,G]; s/t project ket/bra physical index (None: traced)."""
    x1 = ein("phkg,puvP->hkguvP", Le, U)
    if s is None:
        x2 = ein("hkguvP,suhdH->kgvPsdH", x1, A)
        x3 = ein("kgvPsdH,svkeK->gPdHeK", x2, A.conj())
    else:
        x2 = ein("hkguvP,uhdH->kgvPdH", x1, A[s])
        x3 = ein("kgvPdH,vkeK->gPdHeK", x2, A[t].conj())
    return ein("gPdHeK,gdeG->PHKG", x3, B)


def row_env_right(Re, U, A, B):
    """[P,H,K,G] -> [p,h,k,g] (physical index traced)."""
    x1 = ein("puvP,PHKG->puvHKG", U, Re)
    x2 = ein("puvHKG,suhdH->pvKGshd", x1, A)
    x3 = ein("pvKGshd,svkeK->pGhdke", x2, A.conj())
    return ein("pGhdke,gdeG->phkg", x3, B)


def two_row_left(Le, U, A1, A2, B, s=None, t=None):
    """Two-row environment [p,h1,k1,h2,k2,g] -> [P,H1,K1,H2,K2,G]; s and t
    project (diagonally) the upper and lower site of the column."""
    x1 = ein("pabcdg,puvP->abcdguvP", Le, U)  # a=h1 b=k1 c=h2 d=k2
    if s is None:
        x2 = ein("abcdguvP,suamH->bcdgvPsmH", x1, A1)
        x3 = ein("bcdgvPsmH,svbnK->cdgPmHnK", x2, A1.conj())
    else:
        x2 = ein("abcdguvP,uamH->bcdgvPmH", x1, A1[s])
        x3 = ein("bcdgvPmH,vbnK->cdgPmHnK", x2, A1[s].conj())
    if t is None:
        x4 = ein("cdgPmHnK,tmcxJ->dgPHnKtxJ", x3, A2)
        x5 = ein("dgPHnKtxJ,tndeL->gPHKxJeL", x4, A2.conj())
    else:
        x4 = ein("cdgPmHnK,mcxJ->dgPHnKxJ", x3, A2[t])
        x5 = ein("dgPHnKxJ,ndeL->gPHKxJeL", x4, A2[t].conj())
    return ein("gPHKxJeL,gxeG->PHKJLG", x5, B)


def two_row_right(Re, U, A1, A2, B):
    """[P,H1,K1,H2,K2,G] -> [p,h1,k1,h2,k2,g] (both physical indices traced)."""
    x1 = ein("puvP,PHKJLG->puvHKJLG", U, Re)
    x2 = ein("puvHKJLG,suamH->pvKJLGsam", x1, A1)
    x3 = ein("pvKJLGsam,svbnK->pJLGambn", x2, A1.conj())
    x4 = ein("pJLGambn,tmcxJ->pLGabntcx", x3, A2)
    x5 = ein("pLGabntcx,tndeL->pGabcxde", x4, A2.conj())
    return ein("pGabcxde,gxeG->pabcdg", x5, B)


def environments(tensors, chi: int, sweeps: int = 2, seed: int = 0, force_fit: bool = False,
                 vertical: bool = True):
    """Returns dict with rho1 [rows][cols][2][2] (normalised, NaN for dummies),
    zz_h [rows][cols-1], zz_v [rows-1][cols], p2_h [rows][cols-1][4],
    p2_v [rows-1][cols][4] (diagonal of the two-site marginal, order
    (s,t) = 00, 01, 10, 11) and the row-wise norm estimates.  vertical=False
    skips the two-row environments (zz_v and p2_v stay NaN), by far the
    costliest part at large bond."""
    rows, cols = len(tensors), len(tensors[0])
    below, _, _ = boundary_set(tensors, chi, sweeps, seed, TAG_INIT_DOWN, force_fit)
    fb, _, _ = boundary_set(flip_vertical(tensors), chi, sweeps, seed, TAG_INIT_UP, force_fit)
    above = [fb[rows - 1 - r] for r in range(rows)]
    rho1 = np.full((rows, cols, 2, 2), np.nan, dtype=np.complex128)
    zz_h = np.full((rows, max(cols - 1, 0)), np.nan)
    zz_v = np.full((max(rows - 1, 0), cols), np.nan)
    p2_h = np.full((rows, max(cols - 1, 0), 4), np.nan)
    p2_v = np.full((max(rows - 1, 0), cols, 4), np.nan)
    one4 = np.ones((1, 1, 1, 1), dtype=np.complex128)
    for r in range(rows):
        U, B, row = above[r], below[r], tensors[r]
        Le = [None] * (cols + 1)
        Ri = [None] * (cols + 1)
        Le[0] = one4
        for c in range(cols):
            Le[c + 1] = _unit(row_env_left(Le[c], U[c], row[c], B[c]))
        Ri[cols] = one4
        for c in range(cols - 1, -1, -1):
            Ri[c] = _unit(row_env_right(Ri[c + 1], U[c], row[c], B[c]))
        for c in range(cols):
            if row[c].shape[0] != 2:
                continue
            rho = np.zeros((2, 2), dtype=np.complex128)
            for s in range(2):
                for t in range(2):
                    rho[s, t] = np.sum(row_env_left(Le[c], U[c], row[c], B[c], s, t) * Ri[c + 1])
            rho1[r, c] = rho / np.trace(rho)
        for c in range(cols - 1):
            if row[c].shape[0] != 2 or row[c + 1].shape[0] != 2:
                continue
            P = np.zeros(4)
            for s in range(2):
                x = row_env_left(Le[c], U[c], row[c], B[c], s, s)
                for t in range(2):
                    y = row_env_left(x, U[c + 1], row[c + 1], B[c + 1], t, t)
                    P[2 * s + t] = np.sum(y * Ri[c + 2]).real
            p2_h[r, c] = P / P.sum()
            zz_h[r, c] = (P[0] - P[1] - P[2] + P[3]) / P.sum()
    one6 = np.ones((1,) * 6, dtype=np.complex128)
    for r in range(rows - 1 if vertical else 0):
        U, B, r1, r2 = above[r], below[r + 1], tensors[r], tensors[r + 1]
        Le = [None] * (cols + 1)
        Ri = [None] * (cols + 1)
        Le[0] = one6
        for c in range(cols):
            Le[c + 1] = _unit(two_row_left(Le[c], U[c], r1[c], r2[c], B[c]))
        Ri[cols] = one6
        for c in range(cols - 1, -1, -1):
            Ri[c] = _unit(two_row_right(Ri[c + 1], U[c], r1[c], r2[c], B[c]))
        for c in range(cols):
            if r1[c].shape[0] != 2 or r2[c].shape[0] != 2:
                continue
            P = np.zeros(4)
            for s in range(2):
                for t in range(2):
                    P[2 * s + t] = np.sum(two_row_left(Le[c], U[c], r1[c], r2[c], B[c], s, t) * Ri[c + 1]).real
            p2_v[r, c] = P / P.sum()
            zz_v[r, c] = (P[0] - P[1] - P[2] + P[3]) / P.sum()
    return dict(rho1=rho1, zz_h=zz_h, zz_v=zz_v, p2_h=p2_h, p2_v=p2_v, above=above, below=below)


def z_expectation(rho1):
    return (rho1[..., 0, 0] - rho1[..., 1, 1]).real
