"""Belief propagation on the norm network <psi|psi> and the loop BP error
(FP64 oracle).  TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper:

* Methods, "Quantum Circuit Simulation": message tensors on the edges of the
  norm network, obtained by the belief propagation (BP) algorithm, exact when
  the virtual indices form no loops;
* Appendix, "Applying Gates to a Tensor Network State": the norm network keeps
  each site as the uncontracted pair (psi_v, conj(psi_v)); a message on an edge
  carries that edge's ket and bra indices; the message sent along v -> v' is the
  product of the pair at v with the messages into v from its other edges; each
  message is normalised to unit norm and the rule iterated to convergence;
* Methods, "The Boundary Matrix Product State Method", Eqs. avBPError and
  loopBPerror, and Appendix, "Computing the BP Error": for every primitive
  loop (smallest loop) of the network, the transfer matrix obtained by
  inserting BP messages on the loop's boundary and cutting one loop edge open;
  with its eigenvalues lambda_1, lambda_2, ... sorted by modulus,
  eps_l = 1 - |lambda_1| / sum_i |lambda_i| and eps = mean_l eps_l.

Site tensors have index order [p][u][l][d][r]; a message into site v through
leg x is a D x D matrix m[k, k'] (k the ket index of that bond at v, k' the
bra index).  Legs of dimension 1 (absent bonds, grid border) carry [[1]].

Readings where the paper is silent:

* messages start as the identity divided by sqrt(D) (Hermitian, positive,
  unit Frobenius norm) and are updated in parallel sweeps (every new message
  from the previous sweep's messages); each is divided by its Frobenius norm;
  sweeps stop when the largest element change is below ``tol``;
* the update maps Hermitian messages to Hermitian messages, but its
  anti-Hermitian directions are unstable: rounding seeds them and the sweeps
  then stop converging.  Each new message is therefore replaced by its
  Hermitian part (m + m^H) / 2 before the normalisation, which changes nothing
  in exact arithmetic;
* the BP estimate of the norm is Z_BP = prod_v Z_v / prod_e Z_e, Z_v the pair
  at v closed with all its incoming messages and Z_e = sum_kk' m_{v->w} m_{w->v}
  (the standard BP free energy; exact on trees);
* the primitive loops of a grid-embedded lattice are the bounded faces of the
  planar embedding: grid cells merged across absent bonds, each face's boundary
  walked as a cycle; the cut edge is the one closing the walk.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

ein = lambda expr, *ops: np.einsum(expr, *ops, optimize=True)  # noqa: E731

UP, LEFT, DOWN, RIGHT = 1, 2, 3, 4          # axes of A[p, u, l, d, r]
OPP = {UP: DOWN, DOWN: UP, LEFT: RIGHT, RIGHT: LEFT}
STEP = {UP: (-1, 0), DOWN: (1, 0), LEFT: (0, -1), RIGHT: (0, 1)}
# einsum letters of the ket and bra legs and of the message on each leg
KET = {UP: "a", LEFT: "b", DOWN: "c", RIGHT: "d"}
BRA = {UP: "e", LEFT: "f", DOWN: "g", RIGHT: "h"}


def _has_bond(T, r, c, leg) -> bool:
    rows, cols = len(T), len(T[0])
    dr, dc = STEP[leg]
    r2, c2 = r + dr, c + dc
    return 0 <= r2 < rows and 0 <= c2 < cols and T[r][c].shape[leg] > 1


def _pair(A, keep, msgs):
    """Sum over s of A conj(A) with the messages on every leg not in `keep`
    contracted; the kept legs stay open as (ket, bra) index pairs, in the order
    of `keep`."""
    ops = [A, A.conj()]
    terms = ["s" + "".join(KET[x] for x in (UP, LEFT, DOWN, RIGHT)),
             "s" + "".join(BRA[x] for x in (UP, LEFT, DOWN, RIGHT))]
    for leg in (UP, LEFT, DOWN, RIGHT):
        if leg in keep:
            continue
        ops.append(msgs[leg])
        terms.append(KET[leg] + BRA[leg])
    out = "".join(KET[x] + BRA[x] for x in keep)
    return ein(",".join(terms) + "->" + out, *ops)


def initial_messages(T) -> Dict[Tuple[int, int, int], np.ndarray]:
    """Incoming message of every (site, leg): identity / sqrt(D) on bonds,
    [[1]] on legs of dimension 1."""
    M = {}
    for r, row in enumerate(T):
        for c, A in enumerate(row):
            for leg in (UP, LEFT, DOWN, RIGHT):
                D = A.shape[leg]
                M[(r, c, leg)] = np.eye(D, dtype=np.complex128) / math.sqrt(D) if _has_bond(T, r, c, leg) \
                    else np.ones((1, 1), dtype=np.complex128)
    return M


def send(T, M, r, c, leg) -> np.ndarray:
    """Message from site (r, c) through `leg` (unnormalised): the pair at
    (r, c) closed with its incoming messages on the other legs."""
    A = T[r][c]
    msgs = {x: M[(r, c, x)] for x in (UP, LEFT, DOWN, RIGHT)}
    return _pair(A, (leg,), msgs)


def bp_messages(T, max_iter: int = 1000, tol: float = 1e-13, init=None):
    """Parallel BP sweeps to convergence.  Returns (messages, sweeps, last
    change); messages[(r, c, leg)] is the message into (r, c) through leg.
    init: messages to start from (those of a previous state on the same
    lattice), else identity / sqrt(D) on every bond."""
    rows, cols = len(T), len(T[0])
    M = initial_messages(T) if init is None else {k: v.copy() for k, v in init.items()}
    delta = math.inf
    it = 0
    for it in range(1, max_iter + 1):
        new = {}
        for r in range(rows):
            for c in range(cols):
                for leg in (UP, LEFT, DOWN, RIGHT):
                    if not _has_bond(T, r, c, leg):
                        continue
                    m = send(T, M, r, c, leg)
                    m = 0.5 * (m + m.conj().T)
                    dr, dc = STEP[leg]
                    new[(r + dr, c + dc, OPP[leg])] = m / np.linalg.norm(m)
        delta = max(float(np.abs(v - M[k]).max()) for k, v in new.items()) if new else 0.0
        M.update(new)
        if delta < tol:
            break
    return M, it, delta


def site_value(T, M, r, c) -> complex:
    """Z_v: the pair at (r, c) closed with all four incoming messages."""
    A = T[r][c]
    return complex(_pair(A, (), {x: M[(r, c, x)] for x in (UP, LEFT, DOWN, RIGHT)}))


def edge_value(M, r, c, leg) -> complex:
    """Z_e of the bond leaving (r, c) through `leg`: sum_kk' m_{v->w} m_{w->v}."""
    dr, dc = STEP[leg]
    return complex(np.sum(M[(r, c, leg)] * M[(r + dr, c + dc, OPP[leg])]))


def bp_log_norm(T, M=None) -> Tuple[float, float]:
    """(log |Z_BP|, arg Z_BP) with Z_BP = prod_v Z_v / prod_e Z_e."""
    if M is None:
        M, _, _ = bp_messages(T)
    rows, cols = len(T), len(T[0])
    lz = 0.0
    ph = 0.0
    for r in range(rows):
        for c in range(cols):
            z = site_value(T, M, r, c)
            lz += math.log(abs(z))
            ph += math.atan2(z.imag, z.real)
            for leg in (RIGHT, DOWN):
                if _has_bond(T, r, c, leg):
                    e = edge_value(M, r, c, leg)
                    lz -= math.log(abs(e))
                    ph -= math.atan2(e.imag, e.real)
    ph = math.remainder(ph, 2.0 * math.pi)
    return lz, ph


# ---------------------------------------------------------------------------
# primitive loops: bounded faces of the planar grid embedding

def primitive_loops(T) -> List[List[Tuple[int, int, int, int]]]:
    """Every bounded face as a cycle of (r, c, in_leg, out_leg): the walk
    enters site (r, c) through in_leg and leaves through out_leg; the edge
    closing the walk (out of the last site, into the first) is the cut edge."""
    rows, cols = len(T), len(T[0])
    hb = lambda r, c: c + 1 < cols and T[r][c].shape[RIGHT] > 1   # noqa: E731  bond (r,c)-(r,c+1)
    vb = lambda r, c: r + 1 < rows and T[r][c].shape[DOWN] > 1    # noqa: E731  bond (r,c)-(r+1,c)
    nr, nc = rows - 1, cols - 1
    if nr <= 0 or nc <= 0:
        return []
    parent = list(range(nr * nc + 1))
    OUT = nr * nc

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    def union(a, b):
        parent[find(a)] = find(b)

    cell = lambda i, j: i * nc + j if 0 <= i < nr and 0 <= j < nc else OUT  # noqa: E731
    for i in range(nr):
        for j in range(nc):
            if not hb(i, j):          # top side
                union(cell(i, j), cell(i - 1, j))
            if not hb(i + 1, j):      # bottom side
                union(cell(i, j), cell(i + 1, j))
            if not vb(i, j):          # left side
                union(cell(i, j), cell(i, j - 1))
            if not vb(i, j + 1):      # right side
                union(cell(i, j), cell(i, j + 1))
    faces: Dict[int, List[Tuple[int, int]]] = {}
    for i in range(nr):
        for j in range(nc):
            root = find(cell(i, j))
            if root != find(OUT):
                faces.setdefault(root, []).append((i, j))
    loops = []
    for cells in faces.values():
        inside = set(cells)
        # boundary bonds: present bonds with a face cell on exactly one side
        edges = []
        for (i, j) in cells:
            for side, bond in (("t", ((i, j), (i, j + 1))), ("b", ((i + 1, j), (i + 1, j + 1))),
                               ("l", ((i, j), (i + 1, j))), ("r", ((i, j + 1), (i + 1, j + 1)))):
                other = {"t": (i - 1, j), "b": (i + 1, j), "l": (i, j - 1), "r": (i, j + 1)}[side]
                if other in inside:
                    continue
                edges.append(bond)
        adj: Dict[Tuple[int, int], List[Tuple[int, int]]] = {}
        for a, b in edges:
            adj.setdefault(a, []).append(b)
            adj.setdefault(b, []).append(a)
        if any(len(v) != 2 for v in adj.values()):
            raise ValueError("face boundary is not a simple cycle")
        start = min(adj)
        cyc = [start]
        prev, cur = None, start
        while True:
            nxt = adj[cur][0] if adj[cur][0] != prev else adj[cur][1]
            if nxt == start:
                break
            cyc.append(nxt)
            prev, cur = cur, nxt

        def leg_to(a, b):
            d = (b[0] - a[0], b[1] - a[1])
            return {v: k for k, v in STEP.items()}[d]

        L = len(cyc)
        loops.append([(cyc[k][0], cyc[k][1], leg_to(cyc[k], cyc[k - 1]), leg_to(cyc[k], cyc[(k + 1) % L]))
                      for k in range(L)])
    loops.sort(key=lambda lp: (lp[0][0], lp[0][1]))
    return loops


def loop_matrix(T, M, loop) -> np.ndarray:
    """Transfer matrix of a loop with BP messages on its boundary and the edge
    from the last site back to the first cut open: the product of the sites'
    pair matrices [(in, in'), (out, out')] in walk order."""
    X = None
    for (r, c, lin, lout) in loop:
        A = T[r][c]
        msgs = {x: M[(r, c, x)] for x in (UP, LEFT, DOWN, RIGHT)}
        E = _pair(A, (lin, lout), msgs)              # [in, in', out, out']
        Din, Dout = A.shape[lin], A.shape[lout]
        E = E.reshape(Din * Din, Dout * Dout)
        X = E if X is None else X @ E
    return X


def loop_bp_error(T, M=None):
    """(eps, [eps_l], [eigenvalues of each loop matrix, by decreasing modulus],
    loops) of Eqs. avBPError and loopBPerror."""
    if M is None:
        M, _, _ = bp_messages(T)
    loops = primitive_loops(T)
    eps, spectra = [], []
    for lp in loops:
        lam = np.linalg.eigvals(loop_matrix(T, M, lp))
        lam = lam[np.argsort(-np.abs(lam), kind="stable")]
        spectra.append(lam)
        eps.append(1.0 - abs(lam[0]) / float(np.sum(np.abs(lam))))
    mean = float(np.mean(eps)) if eps else 0.0
    return mean, eps, spectra, loops
