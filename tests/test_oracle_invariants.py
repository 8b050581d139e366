"""Invariants of the method that pin the oracle at truncated bond dimension,
where no exact reference exists:

* q(x) is a product of normalised conditionals, so sum_x q(x) = 1 for any
  chi and chi_x (enumerated over every bitstring);
* within a row, the first site's sampling marginal equals the one-site density
  matrix of the environment computation (same boundary below, trivial above);
* gauge freedom on every bond leaves every output unchanged (exact bond);
* the spread of the norm over the four contraction directions shrinks as chi
  grows and vanishes at the exact bound;
* sample histograms agree with exact marginals within the shot-noise bound.
"""
import itertools
import math

import numpy as np
import pytest

from peps_inputs import square_lattice, brick_lattice, random_peps, make_config
from oracle.statevector import statevector
from oracle.boundary import norm, boundary_set
from oracle.sampler import sample, sample_one
from oracle.environments import environments


@pytest.mark.parametrize("chi,chi_x", [(1, 1), (2, 1), (2, 2), (3, 2)])
def test_sum_q_is_one_truncated(chi, chi_x):
    lat = square_lattice(3, 3, 2)
    T = random_peps(lat, "haar", 0.6, 41)
    below, _, info = boundary_set(T, chi)
    if chi < 4:
        assert any(i["mode"] == "fit" for i in info[:-1])
    tot = 0.0
    for x in itertools.product([0, 1], repeat=lat.n_qubits):
        _, lq, _ = sample_one(T, lat.site_index, below, chi_x, 2, 0, 5, forced_bits=x)
        tot += math.exp(lq)
    assert abs(tot - 1.0) < 1e-12


def test_first_site_marginal_matches_environment():
    # the sampler's first conditional (trivial amplitude boundary, stored norm
    # boundary below row 0) and the environment code's rho at site (0, 0) are two
    # contractions of the same network: their diagonal ratios agree at any chi
    lat = square_lattice(4, 4, 2)
    T = random_peps(lat, "haar", 0.5, 43)
    for chi in (2, 3, 16):
        env = environments(T, chi)
        below, _, _ = boundary_set(T, chi)
        rho = env["rho1"][0, 0]
        pt = _first_conditional(T, below)
        assert abs(pt[0] / pt[1] - rho[0, 0] / rho[1, 1]) < 1e-12 * abs(pt[0] / pt[1])


def _first_conditional(T, below):
    from oracle import sampler as smp
    row = T[0]
    B = below[0]
    cols = len(row)
    m = [np.ones((1, 1, 1), dtype=np.complex128) for _ in range(cols)]
    R = np.ones((1, 1, 1, 1, 1), dtype=np.complex128)
    for c in range(cols - 1, 0, -1):
        R = smp.env_right(R, m[c], row[c], B[c])
    L0 = np.ones((1, 1, 1, 1, 1), dtype=np.complex128)
    return [np.sum(smp.env_left(L0, m[0], row[0], B[0], s) * R) for s in (0, 1)]


def _gauge(T, seed):
    rng = np.random.default_rng(seed)
    rows, cols = len(T), len(T[0])
    T = [[t.copy() for t in row] for row in T]
    for r in range(rows):
        for c in range(cols):
            if c + 1 < cols:
                D = T[r][c].shape[4]
                G = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D)) + 3 * np.eye(D)
                T[r][c] = np.einsum("suldr,rR->suldR", T[r][c], G)
                T[r][c + 1] = np.einsum("Ll,suldr->suLdr", np.linalg.inv(G), T[r][c + 1])
            if r + 1 < rows:
                D = T[r][c].shape[3]
                G = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D)) + 3 * np.eye(D)
                T[r][c] = np.einsum("suldr,dD->sulDr", T[r][c], G)
                T[r + 1][c] = np.einsum("Uu,suldr->sUldr", np.linalg.inv(G), T[r + 1][c])
    return T


def test_gauge_invariance_exact():
    lat = square_lattice(3, 3, 2)
    T = random_peps(lat, "haar", 0.4, 45)
    Tg = _gauge(T, 1)
    lz, _ = norm(T, 64)
    lzg, _ = norm(Tg, 64)
    assert abs(lz - lzg) < 1e-10
    e1 = environments(T, 64)
    e2 = environments(Tg, 64)
    assert np.nanmax(np.abs(e1["rho1"] - e2["rho1"])) < 1e-10
    assert np.nanmax(np.abs(e1["zz_v"] - e2["zz_v"])) < 1e-10
    b1, q1, p1 = sample(T, lat.site_index, 64, 64, 6, seed=9)
    b2, q2, p2 = sample(Tg, lat.site_index, 64, 64, 6, seed=9)
    assert np.array_equal(b1, b2) and np.abs(q1 - q2).max() < 1e-10


def test_gauge_changes_truncated_norm():
    # sanity for the previous test: a truncated boundary does see the gauge
    lat = square_lattice(4, 4, 3)
    T = random_peps(lat, "haar", 0.8, 47)
    Tg = _gauge(T, 2)
    assert abs(norm(T, 2)[0] - norm(Tg, 2)[0]) > 1e-8


def test_direction_spread_shrinks_with_chi():
    lat = square_lattice(4, 4, 3)
    T = random_peps(lat, "haar", 0.8, 49)
    psi = statevector(T, lat.site_index)
    lz = math.log(np.sum(np.abs(psi) ** 2))
    errs = []
    for chi in (2, 9, 81):
        vals = [norm(T, chi, direction=d)[0] for d in range(4)]
        errs.append(max(abs(v - lz) for v in vals))
    assert errs[2] < 1e-11
    assert errs[1] < errs[0]


def test_sample_histograms_within_shot_noise():
    lat, T, cfg = make_config("c1")
    n = 300
    psi = statevector(T, lat.site_index)
    P = np.abs(psi) ** 2
    P /= P.sum()
    bits, _, _ = sample(T, lat.site_index, 16, 16, n, seed=2024)
    delta = 1e-3 / lat.n_qubits
    tau = 0.5 * math.sqrt(1.0 / n) + math.sqrt(math.log(1 / delta) / (2 * n))
    for q in range(lat.n_qubits):
        p1 = np.moveaxis(P, q, 0).reshape(2, -1).sum(axis=1)[1]
        f1 = bits[:, q].mean()
        assert abs(f1 - p1) <= tau, (q, f1, p1, tau)
