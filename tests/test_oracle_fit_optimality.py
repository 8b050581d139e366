"""Pins of the oracle's one-site variational fit (Methods, boundary MPS: the
MPS-MPO product compressed by fitting one site at a time) against what the
variational principle fixes, at a bond below the exact one:

* the returned MPS Y is the orthogonal projection of the exact product X onto
  the span of its final gauge (the centre site is the projection), so
  <Y, X> = ||Y||^2 and ||X - Y||^2 = ||X||^2 - ||Y||^2;
* every site update minimises ||X - Y|| over that site with the others fixed,
  so the distance cannot grow from one sweep to the next;
* no MPS with bond t at a cut does better than the best rank-t approximation
  of X across that cut (Eckart-Young).

A dropped conjugate, a transposed leg or a wrong environment in the partial
products breaks the first two.
"""
import numpy as np
import pytest

from peps_inputs import square_lattice, random_peps
from oracle.boundary import apply_row_exact, fit_double, trivial_boundary, plan_bonds


def _dense(m):
    v = m[0]
    for mc in m[1:]:
        v = np.tensordot(v, mc, axes=(v.ndim - 1, 0))
    return v.reshape(-1)


def _case(D, chi, seed):
    lat = square_lattice(3, 4, D)
    T = random_peps(lat, "haar", 0.5, seed)
    # exact boundary below row 1 (the last row applied to the trivial boundary)
    B = apply_row_exact(trivial_boundary(T[2]), T[2])
    row = T[1]
    X = _dense(apply_row_exact(B, row))
    return B, row, X


def _fit(B, row, chi, sweeps):
    Y, lg, info = fit_double(B, row, chi, sweeps, seed=3, tag=0, row_id=1, force_fit=True)
    assert info["mode"] == "fit"
    Y = [y.copy() for y in Y]
    Y[0] = Y[0] * np.exp(lg)
    return _dense(Y), info["bonds"]


@pytest.mark.parametrize("D,chi", [(2, 3), (2, 5), (3, 4)])
def test_fit_is_a_projection(D, chi):
    B, row, X = _case(D, chi, 60 + D)
    Y, bonds = _fit(B, row, chi, 2)
    nx, ny = np.vdot(X, X).real, np.vdot(Y, Y).real
    ov = np.vdot(Y, X)
    assert abs(ov - ny) <= 1e-10 * nx
    assert abs(np.vdot(X - Y, X - Y).real - (nx - ny)) <= 1e-10 * nx
    assert ny < nx * (1 - 1e-6)  # the bond is really truncating


@pytest.mark.parametrize("D,chi", [(2, 3), (3, 4)])
def test_fit_distance_never_grows_with_sweeps(D, chi):
    B, row, X = _case(D, chi, 70 + D)
    nx = np.vdot(X, X).real
    dist = []
    for sweeps in (1, 2, 3, 5):
        Y, _ = _fit(B, row, chi, sweeps)
        dist.append(np.vdot(X - Y, X - Y).real / nx)
    for a, b in zip(dist, dist[1:]):
        assert b <= a * (1 + 1e-9) + 1e-14


@pytest.mark.parametrize("D,chi", [(2, 3), (2, 5), (3, 4)])
def test_fit_respects_eckart_young(D, chi):
    B, row, X = _case(D, chi, 80 + D)
    Y, bonds = _fit(B, row, chi, 3)
    err = np.vdot(X - Y, X - Y).real
    phys = [A.shape[1] ** 2 for A in row]
    for c, t in enumerate(bonds):
        left = int(np.prod(phys[:c + 1]))
        s = np.linalg.svd(X.reshape(left, -1), compute_uv=False)
        assert err >= np.sum(s[t:] ** 2) * (1 - 1e-9) - 1e-14 * np.sum(s ** 2)
    _, t = plan_bonds(phys, [B[c].shape[3] * row[c].shape[4] ** 2 for c in range(len(row) - 1)], chi)
    assert list(bonds) == list(t)
