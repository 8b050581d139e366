"""Seeded synthetic PEPS inputs: lattices embedded in a grid and random site tensors.

This module is shared by the oracle, the tests and the benchmark. It holds no
arithmetic of the contraction or sampling method: it only builds lattice
geometry, draws seeded random tensors and random uniforms, and packs them.

Geometry (the paper's planar tensor-network states, Methods "Quantum Circuit
Simulation" and Fig. 1; partitions into a line of rows, Methods "The Boundary
Matrix Product State Method"):

* every lattice is embedded in a ``rows x cols`` grid; the rows are the
  partitions of the boundary-MPS method;
* a site tensor has index order ``[p][u][l][d][r]`` (physical, up, left, down,
  right), complex, row-major;
* a bond that is absent from the lattice, or that leaves the grid, has
  dimension 1; a grid position with no qubit is a *dummy* site with physical
  dimension 1 (its tensor is the scalar 1).

Lattices:

* ``square``: open-boundary square lattice, every grid bond present (z = 4);
* ``brick``: heavy-hex-shaped brick layout (z = 3): all horizontal bonds, and
  the vertical bond (r, c)-(r+1, c) only when r + c is even, i.e. the degree-2
  bridge qubits of a heavy-hex lattice merged into their neighbours;
* ``rotated_square``: 105-qubit 45-degree-rotated square lattice shaped like
  the Willow chip (10 staggered rows of 11/10 qubits), mapped into a 15 x 15
  grid by (r, x) -> (u, v) = ((r + x) / 2, (x - r) / 2 + 4): the partitions
  are the chip's diagonal cuts;
* ``heavy_hex``: heavy-hex lattice with its degree-2 bridge qubits as sites of
  their own: chains of qubits on the even grid rows, one bridge qubit every
  ``period`` columns on the odd rows between them (columns offset by half a
  period on alternate bridge rows), bonded to the chain qubits above and below;
  the other positions of the bridge rows are dummies.  Its hexagons have 12
  qubits (2 bridges and 5 qubits of each chain);
* ``staggered``: a rotated square lattice (chip rows r with x = r mod 2,
  r mod 2 + 2, ..; neighbours (r +- 1, x +- 1)) partitioned into its staggered
  rows, the chip row r being grid row r and x the grid column.  A qubit's two
  down-diagonal bonds are fused into one down leg (index a * D_b + b, a the
  bond to (r + 1, x - 1), b the one to (r + 1, x + 1)); the grid position
  below it, (r + 1, x), holds a *junction*: a fixed tensor without a qubit that
  splits that leg into its left (a) and right (b) legs, J[0][a * D_b + b][a][0][b]
  = 1.  The qubit (r + 1, x - 1) then reaches (r, x) through its right leg, and
  (r + 1, x + 1) through its left leg.  A row's MPO therefore alternates
  qubits and junctions (a staircase of diagonal bonds in grid form).

Tensor recipes (synthetic stand-ins for circuit-evolved states, which the paper
does not publish):

* ``product0``: |0> component on virtual index 0 plus ``eps`` times iid
  standard complex Gaussians (Re, Im ~ N(0, 1/2));
* ``haar``: U|0> component on virtual index 0, with U a Haar-random 2x2
  unitary per site (QR of a complex Gaussian matrix with the phase of R's
  diagonal divided out), plus ``eps`` times iid complex Gaussians.

Each tensor is then divided by its Frobenius norm ("network normalised" is
read as per-tensor normalisation), and optionally rounded once to complex64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Lattice", "square_lattice", "brick_lattice", "rotated_square_lattice", "heavy_hex_lattice",
    "staggered_lattice", "staggered_sites", "junction_tensor",
    "site_dims", "random_peps", "make_config", "CONFIGS", "sample_uniforms",
    "flatten_peps",
]


@dataclass
class Lattice:
    """A planar lattice embedded in a rows x cols grid.

    phys[r][c]       : 2 for a qubit, 1 for a grid position without one.
    dim_h[r][c]      : bond dimension between (r, c) and (r, c+1); 1 = absent.
    dim_v[r][c]      : bond dimension between (r, c) and (r+1, c); 1 = absent.
    site_index[r][c] : position of the qubit in a bitstring, -1 for non-qubits.
    junction[r][c]   : True where a non-qubit position holds a junction tensor
                       (``staggered`` lattices); other non-qubits are dummies.
    """
    name: str
    rows: int
    cols: int
    phys: np.ndarray
    dim_h: np.ndarray
    dim_v: np.ndarray
    site_index: np.ndarray
    junction: Optional[np.ndarray] = None
    n_qubits: int = field(init=False)

    def __post_init__(self):
        self.n_qubits = int((self.site_index >= 0).sum())
        if self.junction is None:
            self.junction = np.zeros((self.rows, self.cols), dtype=bool)

    def transposed(self) -> "Lattice":
        """The same lattice with rows and columns exchanged."""
        if self.junction.any():
            raise ValueError("a lattice with junctions has a fixed leg layout and is not transposed")
        return Lattice(self.name + "^T", self.cols, self.rows, self.phys.T.copy(),
                       self.dim_v.T.copy(), self.dim_h.T.copy(), self.site_index.T.copy())


def _index_sites(phys: np.ndarray) -> np.ndarray:
    idx = -np.ones(phys.shape, dtype=np.int32)
    k = 0
    for r in range(phys.shape[0]):
        for c in range(phys.shape[1]):
            if phys[r, c] == 2:
                idx[r, c] = k
                k += 1
    return idx


def square_lattice(rows: int, cols: int, D: int) -> Lattice:
    phys = np.full((rows, cols), 2, dtype=np.int32)
    dim_h = np.full((rows, max(cols - 1, 0)), D, dtype=np.int32)
    dim_v = np.full((max(rows - 1, 0), cols), D, dtype=np.int32)
    return Lattice(f"square{rows}x{cols}_D{D}", rows, cols, phys, dim_h, dim_v, _index_sites(phys))


def brick_lattice(rows: int, cols: int, D: int) -> Lattice:
    phys = np.full((rows, cols), 2, dtype=np.int32)
    dim_h = np.full((rows, max(cols - 1, 0)), D, dtype=np.int32)
    dim_v = np.ones((max(rows - 1, 0), cols), dtype=np.int32)
    for r in range(rows - 1):
        for c in range(cols):
            if (r + c) % 2 == 0:
                dim_v[r, c] = D
    return Lattice(f"brick{rows}x{cols}_D{D}", rows, cols, phys, dim_h, dim_v, _index_sites(phys))


def rotated_square_lattice(D: int, chip_rows: int = 10, xmax: int = 20) -> Lattice:
    """Rotated square lattice: chip rows r = 0..chip_rows-1 with x = 0,2,..,xmax
    (r even) or 1,3,..,xmax-1 (r odd); neighbours (r +- 1, x +- 1).  Grid
    position (u, v) = ((r + x)/2, (x - r)/2 + offset), offset making v >= 0.
    The defaults give the 105-qubit chip in a 15x15 embedding."""
    sites = []
    for r in range(chip_rows):
        xs = range(0, xmax + 1, 2) if r % 2 == 0 else range(1, xmax, 2)
        for x in xs:
            sites.append((r, x))
    off = -min((x - r) // 2 for r, x in sites)
    occ = set(((r + x) // 2, (x - r) // 2 + off) for r, x in sites)
    rows = 1 + max(u for u, _ in occ)
    cols = 1 + max(v for _, v in occ)
    phys = np.ones((rows, cols), dtype=np.int32)
    for u, v in occ:
        phys[u, v] = 2
    dim_h = np.ones((rows, cols - 1), dtype=np.int32)
    dim_v = np.ones((rows - 1, cols), dtype=np.int32)
    for u, v in occ:
        if (u, v + 1) in occ:
            dim_h[u, v] = D
        if (u + 1, v) in occ:
            dim_v[u, v] = D
    lat = Lattice(f"rotsq{len(occ)}_D{D}", rows, cols, phys, dim_h, dim_v, _index_sites(phys))
    if (chip_rows, xmax) == (10, 20):
        assert lat.n_qubits == 105
    return lat


def heavy_hex_lattice(chains: int, length: int, D: int, period: int = 4) -> Lattice:
    """Heavy-hex lattice with degree-2 bridge sites: ``chains`` chains of
    ``length`` qubits on grid rows 0, 2, .., 2 (chains - 1); on grid row
    2 i + 1 a bridge qubit at every column c with c % period == offset_i
    (offset_i = 0 for even i, period // 2 for odd i), bonded to (2 i, c) and
    (2 i + 2, c).  Chain qubits have degree <= 3, bridges degree 2."""
    rows, cols = 2 * chains - 1, length
    phys = np.ones((rows, cols), dtype=np.int32)
    dim_h = np.ones((rows, max(cols - 1, 0)), dtype=np.int32)
    dim_v = np.ones((max(rows - 1, 0), cols), dtype=np.int32)
    for i in range(chains):
        phys[2 * i, :] = 2
        dim_h[2 * i, :] = D
    for i in range(chains - 1):
        off = 0 if i % 2 == 0 else period // 2
        for c in range(cols):
            if c % period == off:
                phys[2 * i + 1, c] = 2
                dim_v[2 * i, c] = D
                dim_v[2 * i + 1, c] = D
    return Lattice(f"heavyhex{chains}x{length}_D{D}", rows, cols, phys, dim_h, dim_v, _index_sites(phys))


def staggered_sites(chip_rows: int, xmax: int):
    """Qubit positions (r, x) of a rotated square lattice: x = r % 2,
    r % 2 + 2, .. <= xmax in chip row r."""
    return [(r, x) for r in range(chip_rows) for x in range(r % 2, xmax + 1, 2)]


def staggered_lattice(D: int, chip_rows: int = 10, xmax: int = 20) -> Lattice:
    """The rotated square lattice of ``staggered_sites`` partitioned into its
    chip rows, with junctions below the qubits (see the module docstring).  The
    defaults give the 105-qubit chip in a 10 x 21 grid."""
    occ = set(staggered_sites(chip_rows, xmax))
    rows, cols = chip_rows, xmax + 1

    def diag(r, x, dx):  # dimension of the bond from (r, x) to (r + 1, x + dx)
        return D if (r, x) in occ and (r + 1, x + dx) in occ else 1

    phys = np.ones((rows, cols), dtype=np.int32)
    junction = np.zeros((rows, cols), dtype=bool)
    dim_h = np.ones((rows, max(cols - 1, 0)), dtype=np.int32)
    dim_v = np.ones((max(rows - 1, 0), cols), dtype=np.int32)
    for (r, x) in occ:
        phys[r, x] = 2
        a, b = diag(r, x, -1), diag(r, x, +1)
        if r + 1 < rows and a * b > 1:
            dim_v[r, x] = a * b
            junction[r + 1, x] = True
            if x - 1 >= 0:
                dim_h[r + 1, x - 1] = a   # (r + 1, x - 1) -- junction (r + 1, x)
            if x + 1 < cols:
                dim_h[r + 1, x] = b       # junction (r + 1, x) -- (r + 1, x + 1)
    lat = Lattice(f"stag{len(occ)}_D{D}", rows, cols, phys, dim_h, dim_v, _index_sites(phys), junction)
    if (chip_rows, xmax) == (10, 20):
        assert lat.n_qubits == 105
    return lat


def junction_tensor(lat: Lattice, r: int, c: int) -> np.ndarray:
    """J[0][a * D_b + b][a][0][b] = 1: the junction at (r, c) splitting its up
    leg into its left and right legs."""
    p, du, dl, dd, dr = site_dims(lat, r, c)
    assert p == 1 and dd == 1 and du == dl * dr
    t = np.zeros((1, du, dl, 1, dr), dtype=np.complex128)
    for a in range(dl):
        for b in range(dr):
            t[0, a * dr + b, a, 0, b] = 1.0
    return t


def site_dims(lat: Lattice, r: int, c: int):
    """(p, Du, Dl, Dd, Dr) of grid position (r, c)."""
    p = int(lat.phys[r, c])
    du = int(lat.dim_v[r - 1, c]) if r > 0 else 1
    dd = int(lat.dim_v[r, c]) if r < lat.rows - 1 else 1
    dl = int(lat.dim_h[r, c - 1]) if c > 0 else 1
    dr = int(lat.dim_h[r, c]) if c < lat.cols - 1 else 1
    return p, du, dl, dd, dr


def _haar_2x2(rng: np.random.Generator) -> np.ndarray:
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))


def random_peps(lat: Lattice, recipe: str, eps: float, seed: int,
                dtype=np.complex128) -> List[List[np.ndarray]]:
    """Seeded random site tensors, index order [p][u][l][d][r]."""
    rng = np.random.default_rng(seed)
    out: List[List[np.ndarray]] = []
    for r in range(lat.rows):
        row = []
        for c in range(lat.cols):
            p, du, dl, dd, dr = site_dims(lat, r, c)
            if lat.junction[r, c]:
                row.append(junction_tensor(lat, r, c).astype(dtype))
                continue
            if p == 1:
                # dummy: every leg is dimension 1 because every bond touching it is absent
                t = np.ones((1, du, dl, dd, dr), dtype=np.complex128)
                assert t.size == 1, "a dummy site must have only dimension-1 bonds"
                row.append(t.astype(dtype))
                continue
            shape = (p, du, dl, dd, dr)
            if recipe == "product0":
                prod = np.array([1.0, 0.0], dtype=np.complex128)
            elif recipe == "haar":
                prod = _haar_2x2(rng)[:, 0]
            else:
                raise ValueError(recipe)
            noise = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
            t = eps * noise
            t[:, 0, 0, 0, 0] += prod
            t = t / np.linalg.norm(t)
            row.append(t.astype(dtype))
        out.append(row)
    return out


def sample_uniforms(seed: int, n: int, n_qubits: int) -> np.ndarray:
    """Seeded uniforms in [0, 1), shape [n][n_qubits], for sampling with
    caller-supplied random numbers."""
    rng = np.random.default_rng(seed)
    return rng.random((n, n_qubits))


def flatten_peps(tensors) -> List[np.ndarray]:
    """Row-major list of the site tensors (grid order)."""
    return [t for row in tensors for t in row]


# Named workloads. Sizes follow the paper's square, heavy-hex and rotated-square
# (Willow) geometries at the bond dimensions of the scaled-down study.
CONFIGS = {
    # 4x4 square, D=2, exact boundary chi=16, 1000 samples, checked against the 2^16 statevector
    "c1": dict(lattice=("square", 4, 4, 2), recipe="product0", eps=0.3, seed=1001,
               dtype="c128", chi=16, chi_x=16, n_samples=1000),
    # 8x8 square, D=4, chi in {32, 64}, 4096 samples
    "c2": dict(lattice=("square", 8, 8, 4), recipe="haar", eps=0.2, seed=1002,
               dtype="c128", chi=32, chi_x=32, n_samples=4096),
    # 12x12 brick (heavy-hex-shaped, 144 sites), D=8, chi=64, complex64
    "c3": dict(lattice=("brick", 12, 12, 8), recipe="haar", eps=0.2, seed=1003,
               dtype="c64", chi=64, chi_x=64, n_samples=64),
    # 105-site rotated square in a 15x15 grid, D=8, complex64
    # amplitude-boundary bond adaptive in [16, 128] by an SVD cutoff of 1e-8
    "c4": dict(lattice=("rotsq", 0, 0, 8), recipe="haar", eps=0.2, seed=1004,
               dtype="c64", chi=128, chi_x=128, n_samples=16384, svd_cutoff=1e-8, chi_x_min=16),
    # 12x12 square, D=16, complex64
    "c5sq": dict(lattice=("square", 12, 12, 16), recipe="haar", eps=0.2, seed=1005,
                 dtype="c64", chi=256, chi_x=16, n_samples=8192),
    "c5hh": dict(lattice=("brick", 12, 12, 16), recipe="haar", eps=0.2, seed=1006,
                 dtype="c64", chi=256, chi_x=16, n_samples=8192),
    # heavy-hex with its bridge qubits as sites: 7 chains of 15 and 24 bridges (129 qubits)
    "hhx": dict(lattice=("heavyhex", 7, 15, 8), recipe="haar", eps=0.2, seed=1007,
                dtype="c64", chi=64, chi_x=64, n_samples=64),
    # the 105-qubit rotated square partitioned into its staggered rows (junctions)
    "stag": dict(lattice=("stag", 0, 0, 4), recipe="haar", eps=0.2, seed=1008,
                 dtype="c64", chi=64, chi_x=32, n_samples=64),
}


def build_lattice(spec) -> Lattice:
    kind, rows, cols, D = spec
    if kind == "square":
        return square_lattice(rows, cols, D)
    if kind == "brick":
        return brick_lattice(rows, cols, D)
    if kind == "rotsq":
        return rotated_square_lattice(D)
    if kind == "heavyhex":
        return heavy_hex_lattice(rows, cols, D)
    if kind == "stag":
        return staggered_lattice(D)
    raise ValueError(kind)


def make_config(name: str, **overrides):
    """(lattice, tensors, params) for a named workload; tensors are complex128
    arrays holding the values of the configured storage type (a complex64
    workload is rounded to complex64 once and widened back)."""
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    lat = build_lattice(cfg["lattice"])
    tens = random_peps(lat, cfg["recipe"], cfg["eps"], cfg["seed"])
    if cfg["dtype"] == "c64":
        tens = [[t.astype(np.complex64).astype(np.complex128) for t in row] for row in tens]
    return lat, tens, cfg
