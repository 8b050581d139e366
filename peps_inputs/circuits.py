"""Quantum circuits applied to the lattices of this package (inputs of the
simple-update simulation; no arithmetic of the method itself).

Results, discrete-time Heisenberg dynamics (Eqs. Heisenberg and
HeisenbergProp): H_ij = J (X_i X_j + Y_i Y_j + Z_i Z_j) on every bond, first-
order Trotter layers U = prod_k prod_{<ij> in E_k} exp(-i H_ij dt) over an edge
colouring E_1..E_K of the lattice, from a domain-wall product state.

Readings (the paper names the colouring and the initial state, not their
layout on a lattice):

* the colour groups of a grid-embedded lattice, in this order: horizontal
  bonds whose left qubit is in an even grid column, then odd; vertical bonds
  whose upper qubit is in an even grid row, then odd; the two vertical groups
  are merged when no qubit carries two vertical bonds; empty groups dropped.
  Bonds within a group are listed row by row, column by column; they share no
  qubit;
* the domain wall: qubits in grid columns c < cols // 2 in |0>, the others in
  |1>; every bond keeps its lattice dimension, the product state sitting on
  virtual index 0.

A gate is (group, r, c, r2, c2) with (r2, c2) = (r, c + 1) or (r + 1, c), both
qubits, and a 4 x 4 unitary G in the basis 2 a + b (a the qubit at (r, c)).
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from . import Lattice, site_dims

__all__ = ["heisenberg_gate", "edge_groups", "heisenberg_circuit", "domain_wall_peps", "domain_wall_ones", "Gate"]

Gate = Tuple[int, int, int, int, int]


def heisenberg_gate(dt: float, J: float = 1.0) -> np.ndarray:
    """exp(-i dt J (XX + YY + ZZ)) on two qubits, basis 2 a + b.  With
    XX + YY + ZZ = 2 SWAP - I and SWAP^2 = I this is
    e^{i J dt} (cos(2 J dt) I - i sin(2 J dt) SWAP)."""
    th = J * dt
    swap = np.zeros((4, 4), dtype=np.complex128)
    for a in range(2):
        for b in range(2):
            swap[2 * b + a, 2 * a + b] = 1.0
    return np.exp(1j * th) * (math.cos(2 * th) * np.eye(4) - 1j * math.sin(2 * th) * swap)


def edge_groups(lat: Lattice) -> List[List[Tuple[int, int, int, int]]]:
    """The colour groups of the lattice's qubit-qubit bonds, (r, c, r2, c2) each."""
    h: List[list] = [[], []]
    v: List[list] = [[], []]
    for r in range(lat.rows):
        for c in range(lat.cols):
            if lat.phys[r, c] != 2:
                continue
            if c + 1 < lat.cols and lat.dim_h[r, c] > 1 and lat.phys[r, c + 1] == 2:
                h[c % 2].append((r, c, r, c + 1))
            if r + 1 < lat.rows and lat.dim_v[r, c] > 1 and lat.phys[r + 1, c] == 2:
                v[r % 2].append((r, c, r + 1, c))
    count = {}
    for (r, c, r2, c2) in v[0] + v[1]:
        for q in ((r, c), (r2, c2)):
            count[q] = count.get(q, 0) + 1
    groups = [h[0], h[1]]
    if count and max(count.values()) == 1:
        groups.append(sorted(v[0] + v[1]))
    else:
        groups += [v[0], v[1]]
    return [g for g in groups if g]


def heisenberg_circuit(lat: Lattice, layers: int, dt: float, J: float = 1.0):
    """(gates, G): ``layers`` first-order Trotter layers, one gate per bond per
    colour group; the group index runs over all layers (layer l, group k ->
    l * K + k), so a new index marks every point where the messages are
    refreshed.  Every gate is the same matrix G."""
    groups = edge_groups(lat)
    gates: List[Gate] = []
    for l in range(layers):
        for k, grp in enumerate(groups):
            for (r, c, r2, c2) in grp:
                gates.append((l * len(groups) + k, r, c, r2, c2))
    return gates, heisenberg_gate(dt, J)


def domain_wall_peps(lat: Lattice) -> List[List[np.ndarray]]:
    """The domain-wall product state on the lattice's bond dimensions."""
    out = []
    for r in range(lat.rows):
        row = []
        for c in range(lat.cols):
            dims = site_dims(lat, r, c)
            t = np.zeros(dims, dtype=np.complex128)
            if dims[0] == 1:
                assert t.size == 1, "the circuits act on lattices whose non-qubit sites are dummies"
                t[(0,) * 5] = 1.0
            else:
                t[(0 if c < lat.cols // 2 else 1, 0, 0, 0, 0)] = 1.0
            row.append(t)
        out.append(row)
    return out


def domain_wall_ones(lat: Lattice) -> int:
    """Qubits in |1> in the domain-wall state: the total magnetisation every
    Heisenberg layer conserves (each gate commutes with sum_i Z_i)."""
    return int(sum(1 for r in range(lat.rows) for c in range(lat.cols)
                   if lat.phys[r, c] == 2 and c >= lat.cols // 2))
