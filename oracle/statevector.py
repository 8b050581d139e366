"""Exact amplitudes <x|psi> of a small PEPS by full contraction.

The plain definition of the state the tensor network encodes (Methods,
"Quantum Circuit Simulation": one tensor per qubit, virtual indices contracted
along the lattice bonds). Feasible up to ~20 qubits. Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def statevector(tensors, site_index) -> np.ndarray:
    """psi[x_0, ..., x_{N-1}] with x_q the bit of the qubit whose site_index is q.

    Sites are absorbed in row-major grid order. The running tensor has axes
    (bits so far, frontier leg of column 0..cols-1, current horizontal leg)."""
    rows = len(tensors)
    cols = len(tensors[0])
    # frontier legs: the up-leg of the next site in each column (all dim 1 above row 0)
    T = np.ones((1,) + (1,) * cols + (1,), dtype=np.complex128)
    order = []
    for r in range(rows):
        # the horizontal leg entering column 0 is dimension 1
        assert T.shape[-1] == 1
        for c in range(cols):
            A = tensors[r][c]  # [p][u][l][d][rr]
            p, du, dl, dd, dr = A.shape
            nb = T.shape[0]
            # move the frontier leg of column c and the horizontal leg to the end
            shp = T.shape
            axes = [0] + [1 + k for k in range(cols) if k != c] + [1 + c, 1 + cols]
            Tp = np.transpose(T, axes)
            rest = [shp[1 + k] for k in range(cols) if k != c]
            Tp = Tp.reshape(nb, int(np.prod(rest)) if rest else 1, du * dl)
            Am = np.transpose(A, (1, 2, 0, 3, 4)).reshape(du * dl, p * dd * dr)
            N = Tp @ Am  # [nb][rest][p dd dr]
            N = N.reshape(nb, *rest, p, dd, dr) if rest else N.reshape(nb, p, dd, dr)
            # new axes: (nb, p) -> bits; dd -> frontier c; dr -> horizontal
            nrest = len(rest)
            # current order: 0:nb, 1..nrest: rest, nrest+1: p, nrest+2: dd, nrest+3: dr
            new_axes = [0, nrest + 1]
            fr = []
            j = 1
            for k in range(cols):
                if k == c:
                    fr.append(nrest + 2)
                else:
                    fr.append(j)
                    j += 1
            new_axes += fr + [nrest + 3]
            N = np.transpose(N, new_axes)
            newshape = (nb * p,) + tuple(N.shape[2:])
            T = N.reshape(newshape)
            if p == 2:
                order.append(int(site_index[r][c]))
        # the horizontal leg leaving the last column is dimension 1: drop it into the next row
    vec = T.reshape(-1)
    n = len(order)
    psi = vec.reshape((2,) * n) if n else vec.reshape(())
    # axis k of psi is the k-th absorbed qubit; reorder to site_index order
    perm = np.argsort(np.array(order)) if n else []
    return np.transpose(psi, perm) if n else psi


def brute_force_amplitude(tensors, site_index, bits) -> complex:
    """<x|psi> for one bitstring by explicit summation over every assignment of
    every virtual bond (tiny lattices only)."""
    import itertools
    rows = len(tensors)
    cols = len(tensors[0])
    bonds = []  # (kind, r, c, dim)
    for r in range(rows):
        for c in range(cols):
            A = tensors[r][c]
            if c < cols - 1:
                bonds.append(("h", r, c, A.shape[4]))
            if r < rows - 1:
                bonds.append(("v", r, c, A.shape[3]))
    total = 0j
    for assign in itertools.product(*[range(b[3]) for b in bonds]):
        val = dict(((b[0], b[1], b[2]), a) for b, a in zip(bonds, assign))
        prod = 1 + 0j
        for r in range(rows):
            for c in range(cols):
                A = tensors[r][c]
                s = bits[site_index[r][c]] if A.shape[0] == 2 else 0
                u = val[("v", r - 1, c)] if r > 0 else 0
                l = val[("h", r, c - 1)] if c > 0 else 0
                d = val[("v", r, c)] if r < rows - 1 else 0
                rr = val[("h", r, c)] if c < cols - 1 else 0
                prod *= A[s, u, l, d, rr]
        total += prod
    return total
