"""Boundary-MPS contraction of the norm network <psi|psi> (FP64 oracle).

Follows the paper's Methods ("The Boundary Matrix Product State Method for
Planar Tensor Networks") and Appendix ("Sampling from a Tensor Network
State"):

* the network is partitioned into rows; row b of the norm network is the MPO
  T_b = psi_b^dagger psi_b, whose ket and bra tensors stay separate (the
  grouping is book-keeping only);
* boundary MPSs are passed through the rows in reverse order, last row first,
  and every intermediate boundary is stored (the set M_{b+1 -> b});
* each MPS-MPO product is approximated by an MPS of maximum bond chi with the
  one-site variational fit: sweep through the output MPS and replace each site
  tensor by the derivative of the overlap <Y | M T_b> with respect to it.

Readings where the paper is silent (listed in the design notes):

* initial guess: if chi reaches the exact bond bound at every cut, the product
  is applied exactly and brought to canonical form by QR sweeps (no
  truncation); otherwise the guess is a Philox-uniform random MPS with the
  target bonds, right-canonicalised by LQ;
* a sweep is left-to-right (QR) then right-to-left (LQ); the number of sweeps is
  a parameter (default 2); the orthogonality centre ends on site 0, which is
  then normalised, the norm going into a log-scale;
* the norm is the closing contraction of row 0 with the stored boundary below
  it, times the exponentiated log-scales.

Index conventions: site tensor A[s, u, l, d, r]; double-layer boundary site
Y[y, u, v, y2] (ket phys u, bra phys v); environments [y, g, h, k] = (output
bond, input bond, ket MPO bond, bra MPO bond).

Plain NumPy, complex128, pairwise einsum contractions. Test infrastructure only.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from .philox import init_tensor_vec, TAG_INIT_DOWN, TAG_INIT_UP

ein = lambda expr, *ops: np.einsum(expr, *ops, optimize=True)  # noqa: E731


# ---------------------------------------------------------------------------
# factorisations

def qr_reduced(M: np.ndarray):
    Q, R = np.linalg.qr(M, mode="reduced")
    return Q, R


def lq_reduced(M: np.ndarray):
    """M = L Q with Q having orthonormal rows."""
    Q, R = np.linalg.qr(M.conj().T, mode="reduced")
    return R.conj().T, Q.conj().T


# ---------------------------------------------------------------------------
# bond planning (shared reading for every fit)

def plan_bonds(phys: List[int], bond_in: List[int], chi: int):
    """Exact bond bound per cut and the (consistent) target bonds.

    phys[c]    : product of the output physical dims at site c;
    bond_in[c] : bond of the exactly applied MPS-MPO product at cut c|c+1.
    Returns (exact_ok, targets): exact_ok is True when chi reaches the exact
    bound at every cut and the exact product itself is small (bond_in[c] <=
    max(chi, 64) everywhere; rows with few sites can have a small bound but a
    huge product bond, which is then fitted with the bound as target instead);
    targets are min(chi, bound) made consistent so that a reduced QR/LQ never
    shrinks them (t[c] <= t[c-1] phys[c], t[c] <= phys[c+1] t[c+1])."""
    L = len(phys)
    ex = []
    for c in range(L - 1):
        pl = math.prod(phys[: c + 1])
        pr = math.prod(phys[c + 1:])
        ex.append(min(pl, pr, bond_in[c]))
    exact_ok = all(chi >= e for e in ex) and all(b <= max(chi, 64) for b in bond_in)
    t = [min(chi, e) for e in ex]
    for c in range(L - 1):
        left = t[c - 1] if c > 0 else 1
        t[c] = min(t[c], left * phys[c])
    for c in range(L - 2, -1, -1):
        right = t[c + 1] if c < L - 2 else 1
        t[c] = min(t[c], phys[c + 1] * right)
    return exact_ok, t


def canonicalise_exact(Y: List[np.ndarray]) -> Tuple[List[np.ndarray], float]:
    """Left QR sweep then right-to-left LQ sweep (bonds shrink to the reduced
    factor sizes, nothing is truncated); normalise the centre at site 0."""
    Y = [y.copy() for y in Y]
    L = len(Y)
    for c in range(L - 1):
        sh = Y[c].shape
        Q, R = qr_reduced(Y[c].reshape(-1, sh[-1]))
        Y[c] = Q.reshape(sh[:-1] + (Q.shape[1],))
        Y[c + 1] = np.tensordot(R, Y[c + 1], axes=(1, 0))
    for c in range(L - 1, 0, -1):
        sh = Y[c].shape
        Lm, Q = lq_reduced(Y[c].reshape(sh[0], -1))
        Y[c] = Q.reshape((Q.shape[0],) + sh[1:])
        Y[c - 1] = np.tensordot(Y[c - 1], Lm, axes=(Y[c - 1].ndim - 1, 0))
    nrm = np.linalg.norm(Y[0])
    Y[0] = Y[0] / nrm
    return Y, math.log(nrm)


def right_canonicalise(Y: List[np.ndarray]) -> List[np.ndarray]:
    Y = [y.copy() for y in Y]
    for c in range(len(Y) - 1, 0, -1):
        sh = Y[c].shape
        Lm, Q = lq_reduced(Y[c].reshape(sh[0], -1))
        assert Q.shape[0] == sh[0], "target bonds must survive a reduced LQ"
        Y[c] = Q.reshape(sh)
        Y[c - 1] = np.tensordot(Y[c - 1], Lm, axes=(Y[c - 1].ndim - 1, 0))
    return Y


# ---------------------------------------------------------------------------
# double-layer (norm network) pieces

def apply_row_exact(Bin, row):
    """E_c[(g,h,k), u, v, (G,H,K)] = sum_{s,d,e} B[g,d,e,G] A[s,u,h,d,H] conj(A)[s,v,k,e,K]."""
    out = []
    for B, A in zip(Bin, row):
        g, _, _, G = B.shape
        _, u, h, _, H = A.shape
        E = ein("gdeG,suhdH,svkeK->ghkuvGHK", B, A, A.conj())
        out.append(E.reshape(g * h * h, u, u, G * H * H))
    return out


def left_partial(Lenv, B, A):
    """t[y,G,u,H,v,K] = sum L[y,g,h,k] B[g,d,e,G] A[s,u,h,d,H] conj(A)[s,v,k,e,K]."""
    t1 = ein("yghk,gdeG->yhkdeG", Lenv, B)
    t2 = ein("yhkdeG,suhdH->ykeGsuH", t1, A)
    return ein("ykeGsuH,svkeK->yGuHvK", t2, A.conj())


def right_partial(Renv, B, A):
    """t[g,h,k,u,v,Y] = sum B[g,d,e,G] A[s,u,h,d,H] conj(A)[s,v,k,e,K] R[Y,G,H,K]."""
    t1 = ein("gdeG,YGHK->gdeYHK", B, Renv)
    t2 = ein("gdeYHK,suhdH->geYKsuh", t1, A)
    return ein("geYKsuh,svkeK->ghkuvY", t2, A.conj())


def fit_double(Bin, row, chi: int, sweeps: int, seed: int, tag: int, row_id: int,
               force_fit: bool = False):
    """Approximate the MPS-MPO product Bin . T_row by an MPS of bond <= chi.
    Returns (Y, log_scale, info)."""
    L = len(row)
    phys = [A.shape[1] ** 2 for A in row]
    bond_in = [Bin[c].shape[3] * row[c].shape[4] ** 2 for c in range(L - 1)]
    exact_ok, t = plan_bonds(phys, bond_in, chi)
    if exact_ok and not force_fit:
        Y, lg = canonicalise_exact(apply_row_exact(Bin, row))
        return Y, lg, dict(mode="exact", bonds=[y.shape[3] for y in Y[:-1]])
    # random initial guess with the target bonds
    Y = []
    for c in range(L):
        u = row[c].shape[1]
        tl = t[c - 1] if c > 0 else 1
        tr = t[c] if c < L - 1 else 1
        Y.append(init_tensor_vec(seed, tag, row_id, c, 0, (tl, u, u, tr)))
    Y = right_canonicalise(Y)
    one = np.ones((1, 1, 1, 1), dtype=np.complex128)
    R = [None] * (L + 1)
    R[L] = one
    for c in range(L - 1, 0, -1):
        tR = right_partial(R[c + 1], Bin[c], row[c])
        R[c] = ein("yuvY,ghkuvY->yghk", Y[c].conj(), tR)
    Lenv = [None] * (L + 1)
    Lenv[0] = one
    for _ in range(sweeps):
        for c in range(L - 1):
            t3 = left_partial(Lenv[c], Bin[c], row[c])
            N = ein("yGuHvK,YGHK->yuvY", t3, R[c + 1])
            Q, _ = qr_reduced(N.reshape(-1, N.shape[3]))
            Y[c] = Q.reshape(N.shape)
            Lenv[c + 1] = ein("yuvY,yGuHvK->YGHK", Y[c].conj(), t3)
        for c in range(L - 1, 0, -1):
            tR = right_partial(R[c + 1], Bin[c], row[c])
            N = ein("yghk,ghkuvY->yuvY", Lenv[c], tR)
            _, Q = lq_reduced(N.reshape(N.shape[0], -1))
            Y[c] = Q.reshape(N.shape)
            R[c] = ein("yuvY,ghkuvY->yghk", Y[c].conj(), tR)
    tR = right_partial(R[1], Bin[0], row[0])
    Y[0] = ein("yghk,ghkuvY->yuvY", Lenv[0], tR)
    nrm = np.linalg.norm(Y[0])
    Y[0] = Y[0] / nrm
    return Y, math.log(nrm), dict(mode="fit", bonds=t)


def trivial_boundary(row):
    """Boundary below the last row: bond 1, phys (d, e) of the row (all dim 1)."""
    return [np.ones((1, A.shape[3], A.shape[3], 1), dtype=np.complex128) for A in row]


def flip_vertical(tensors):
    """Lattice mirrored top-bottom: rows reversed, up and down legs exchanged."""
    return [[A.transpose(0, 3, 2, 1, 4).copy() for A in row] for row in reversed(tensors)]


def transpose_lattice(tensors):
    """Rows and columns exchanged: A[s,u,l,d,r] -> A'[s,l,u,r,d]."""
    rows, cols = len(tensors), len(tensors[0])
    return [[tensors[r][c].transpose(0, 2, 1, 4, 3).copy() for r in range(rows)] for c in range(cols)]


def boundary_set(tensors, chi: int, sweeps: int = 2, seed: int = 0, tag: int = TAG_INIT_DOWN,
                 force_fit: bool = False):
    """Norm boundaries in reverse row order (paper: b = N_b, ..., 2).

    below[r] approximates rows r+1..rows-1 and has the down legs of row r as
    physical legs; below[rows-1] is trivial. log_scale[r] is the log of the
    norm divided out of below[r]."""
    rows = len(tensors)
    below = [None] * rows
    logs = [0.0] * rows
    info = [None] * rows
    below[rows - 1] = trivial_boundary(tensors[rows - 1])
    for r in range(rows - 1, 0, -1):
        below[r - 1], logs[r - 1], info[r - 1] = fit_double(below[r], tensors[r], chi, sweeps,
                                                            seed, tag, r, force_fit)
    return below, logs, info


def close_row(row, B):
    """Contraction of a row whose up legs are all dimension 1 with the boundary below it."""
    Lenv = np.ones((1, 1, 1, 1), dtype=np.complex128)
    for A, Bc in zip(row, B):
        t = left_partial(Lenv, Bc, A)  # [y,G,u,H,v,K], y=u=v=1
        Lenv = t.reshape(1, t.shape[1], t.shape[3], t.shape[5])
    return Lenv.reshape(())[()]


def norm(tensors, chi: int, sweeps: int = 2, seed: int = 0, direction: int = 0,
         force_fit: bool = False):
    """(log|Z|, arg Z) of Z = <psi|psi> by boundary MPS.

    direction 0: bottom-up (paper's order), 1: top-down, 2: right-to-left over
    columns, 3: left-to-right over columns (columns by transposing the lattice)."""
    t = tensors
    tag = TAG_INIT_DOWN
    if direction in (2, 3):
        t = transpose_lattice(t)
    if direction in (1, 3):
        t = flip_vertical(t)
        tag = TAG_INIT_UP
    below, logs, _ = boundary_set(t, chi, sweeps, seed, tag, force_fit)
    z = close_row(t[0], below[0])
    return sum(logs) + math.log(abs(z)), float(np.angle(z))
