"""Pins of the BP oracle (oracle/bp.py) against what the mathematics fixes:

* BP is exact on networks without loops: Z_BP equals the statevector norm on a
  comb lattice (a tree of bonds);
* on a network with a single loop, the exact norm is the trace of the loop's
  transfer matrix and BP keeps its dominant eigenvalue, so
  Z / Z_BP = sum_i lambda_i / lambda_1 (2x2 square, one 6-site brick loop);
* rank-one (product) site tensors carry no loop correlations: every loop's
  eps_l vanishes and Z_BP is exact;
* a gauge transformation G, G^-1 on every bond changes neither Z_BP nor any
  eps_l;
* 0 <= eps_l <= 1 - 1/D^2 (Methods, after Eq. loopBPerror);
* the returned messages are a fixed point of the update rule;
* the primitive loops found are the faces of the lattice: (rows-1)(cols-1)
  squares, 6-site brick cells, the square cells of a rotated-square patch."""
import math

import numpy as np
import pytest

from peps_inputs import (Lattice, square_lattice, brick_lattice, rotated_square_lattice, random_peps,
                         _index_sites)
from oracle.statevector import statevector
from oracle import bp


def comb_lattice(rows, cols, D):
    """All horizontal bonds, vertical bonds only in column 0: a tree."""
    phys = np.full((rows, cols), 2, np.int32)
    dh = np.full((rows, cols - 1), D, np.int32)
    dv = np.ones((rows - 1, cols), np.int32)
    dv[:, 0] = D
    return Lattice(f"comb{rows}x{cols}_D{D}", rows, cols, phys, dh, dv, _index_sites(phys))


def exact_log_norm(lat, T):
    psi = statevector(T, lat.site_index)
    return math.log(float(np.sum(np.abs(psi) ** 2)))


@pytest.mark.parametrize("rows,cols,D,seed", [(3, 4, 2, 7), (4, 3, 3, 8), (1, 6, 3, 9)])
def test_bp_exact_on_trees(rows, cols, D, seed):
    lat = comb_lattice(rows, cols, D)
    T = random_peps(lat, "haar", 0.7, seed)
    assert bp.primitive_loops(T) == []
    M, it, delta = bp.bp_messages(T)
    assert delta < 1e-13
    lz, ph = bp.bp_log_norm(T, M)
    assert abs(lz - exact_log_norm(lat, T)) < 1e-11
    assert abs(ph) < 1e-11


@pytest.mark.parametrize("lat,seed", [(square_lattice(2, 2, 2), 5), (square_lattice(2, 2, 3), 6),
                                      (brick_lattice(2, 3, 2), 7), (brick_lattice(2, 3, 3), 8)])
def test_single_loop_norm_ratio_is_spectral(lat, seed):
    T = random_peps(lat, "haar", 0.7, seed)
    M, _, _ = bp.bp_messages(T)
    lz, _ = bp.bp_log_norm(T, M)
    mean, eps, spectra, loops = bp.loop_bp_error(T, M)
    assert len(loops) == 1
    lam = spectra[0]
    ratio = np.sum(lam) / lam[0]
    assert abs(ratio.imag) < 1e-12
    assert abs(math.exp(exact_log_norm(lat, T) - lz) - ratio.real) < 1e-10
    assert abs(mean - eps[0]) < 1e-15
    assert eps[0] > 1e-4  # a random state does have loop correlations


def test_product_tensors_have_no_loop_error():
    lat = square_lattice(3, 3, 2)
    rng = np.random.default_rng(3)
    cn = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)  # noqa: E731
    T = []
    for r in range(3):
        row = []
        for c in range(3):
            dims = [2] + [2 if (r > 0) else 1, 2 if c > 0 else 1, 2 if r < 2 else 1, 2 if c < 2 else 1]
            t = cn(dims[0])
            for d in dims[1:]:
                t = np.multiply.outer(t, cn(d))
            row.append(t)
        T.append(row)
    M, _, _ = bp.bp_messages(T)
    lz, _ = bp.bp_log_norm(T, M)
    assert abs(lz - exact_log_norm(lat, T)) < 1e-11
    mean, eps, spectra, loops = bp.loop_bp_error(T, M)
    assert len(loops) == 4
    assert max(eps) < 1e-12


def test_gauge_invariance():
    lat = square_lattice(3, 3, 2)
    T = random_peps(lat, "haar", 0.6, 11)
    rng = np.random.default_rng(12)
    G = [[None] * 3 for _ in range(3)]
    T2 = [[t.copy() for t in row] for row in T]
    for r in range(3):
        for c in range(3):
            for leg, (dr, dc) in ((bp.RIGHT, (0, 1)), (bp.DOWN, (1, 0))):
                r2, c2 = r + dr, c + dc
                if r2 >= 3 or c2 >= 3:
                    continue
                g = np.eye(2) + 0.4 * (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)))
                gi = np.linalg.inv(g)
                # A[..leg..] G on this side, G^-1 A on the other
                T2[r][c] = np.moveaxis(np.tensordot(T2[r][c], g, axes=(leg, 0)), -1, leg)
                T2[r2][c2] = np.moveaxis(np.tensordot(gi, T2[r2][c2], axes=(1, bp.OPP[leg])), 0, bp.OPP[leg])
    assert abs(exact_log_norm(lat, T2) - exact_log_norm(lat, T)) < 1e-10
    lz1, _ = bp.bp_log_norm(T)
    lz2, _ = bp.bp_log_norm(T2)
    assert abs(lz1 - lz2) < 1e-9
    e1 = bp.loop_bp_error(T)[1]
    e2 = bp.loop_bp_error(T2)[1]
    assert np.abs(np.array(e1) - np.array(e2)).max() < 1e-9


@pytest.mark.parametrize("D", [2, 3])
def test_loop_error_bounds_and_fixed_point(D):
    lat = square_lattice(4, 4, D)
    T = random_peps(lat, "haar", 0.8, 20 + D)
    M, _, _ = bp.bp_messages(T)
    mean, eps, spectra, loops = bp.loop_bp_error(T, M)
    assert len(eps) == 9
    assert all(0.0 <= e <= 1.0 - 1.0 / D ** 2 + 1e-14 for e in eps)
    assert abs(mean - np.mean(eps)) < 1e-15
    for (r, c, leg), m in M.items():
        if not bp._has_bond(T, r, c, leg):
            continue
        dr, dc = bp.STEP[leg]
        s = bp.send(T, M, r + dr, c + dc, bp.OPP[leg])
        assert np.abs(s / np.linalg.norm(s) - m).max() < 1e-12


@pytest.mark.parametrize("lat,count,length", [(square_lattice(4, 5, 2), 12, 4), (brick_lattice(4, 4, 2), 3, 6),
                                              (brick_lattice(12, 12, 2), 55, 6),
                                              (rotated_square_lattice(2, 4, 4), 3, 4)])
def test_primitive_loops_are_the_faces(lat, count, length):
    T = random_peps(lat, "haar", 0.5, 1)
    loops = bp.primitive_loops(T)
    assert len(loops) == count
    assert all(len(lp) == length for lp in loops)
    for lp in loops:
        # consecutive sites are neighbours through the recorded legs, and the walk closes
        for k, (r, c, lin, lout) in enumerate(lp):
            r2, c2, lin2, _ = lp[(k + 1) % len(lp)]
            dr, dc = bp.STEP[lout]
            assert (r + dr, c + dc) == (r2, c2) and lin2 == bp.OPP[lout]
            assert T[r][c].shape[lout] > 1
