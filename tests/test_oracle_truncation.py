"""Pins of the oracle's adaptive-bond truncation (SVD cutoff on the amplitude
boundary) against textbook linear algebra and the method's invariants:

* the keep rule on spectra worked by hand (discarded weight, clamp, rank);
* two sites: the truncated state is the best rank-k approximation of the
  dense matrix (Eckart-Young), with k from the dense matrix's own spectrum;
* several sites: the Schmidt rank at every cut is at most the reported k, the
  error obeys ||psi - psi_t||^2 <= sum over cuts of cutoff ||psi||^2, and a
  cutoff that drops nothing leaves the state unchanged;
* the sampler with the cutoff still gives sum_x q(x) = 1, and a cutoff that
  drops nothing reproduces the fixed-bond sampler.
"""
import itertools
import math

import numpy as np
import pytest

from peps_inputs import square_lattice, random_peps
from oracle.boundary import boundary_set, canonicalise_exact
from oracle.sampler import keep_count, truncate_cutoff, sample, sample_one


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


def _dense(m):
    v = m[0]
    for mc in m[1:]:
        v = np.tensordot(v, mc, axes=(v.ndim - 1, 0))
    return v.reshape(-1)


def _random_mps(rng, L, d, chi, decay=0.0):
    """Random MPS with bonds <= chi; decay > 0 gives each bond a geometric
    spectrum so that a cutoff truncates."""
    m = []
    for c in range(L):
        a = 1 if c == 0 else min(chi, d ** c, d ** (L - c))
        b = 1 if c == L - 1 else min(chi, d ** (c + 1), d ** (L - c - 1))
        t = _cn(rng, (a, d, b))
        if decay > 0 and b > 1:
            t = t * np.exp(-decay * np.arange(b))[None, None, :]
        m.append(t)
    Y, _ = canonicalise_exact(m)  # right-canonical, unit centre at site 0
    return Y


def test_keep_count_worked_spectra():
    s = [1.0, 0.1, 0.01, 0.001]  # weights 1, 1e-2, 1e-4, 1e-6; total 1.010101
    assert keep_count(s, 1e-5, 1) == 3     # 1e-6 fits under 1.0101e-5, 1e-4 more does not
    assert keep_count(s, 1e-3, 1) == 2     # 1.01e-4 <= 1.0101e-3 < 1.0101e-2
    assert keep_count(s, 2e-2, 1) == 1     # everything but the largest
    assert keep_count(s, 1e-3, 3) == 3     # clamp from below
    assert keep_count(s, 1e-3, 9) == 4     # ... never above the rank
    assert keep_count(s[::-1], 1e-3, 1) == 2  # order of the input does not matter
    assert keep_count([1.0, 1e-13], 0.0, 1) == 1  # numerical rank
    assert keep_count([1.0, 0.5], 0.0, 1) == 2
    assert keep_count([0.0, 0.0], 0.1, 4) == 0
    assert keep_count([2.0], 1.0, 1) == 1


@pytest.mark.parametrize("cutoff", [1e-1, 1e-2, 1e-4])
def test_two_sites_best_rank_k(cutoff):
    rng = np.random.default_rng(7)
    d = 6
    M = _cn(rng, (d, d)) @ np.diag(np.exp(-0.7 * np.arange(d))) @ _cn(rng, (d, d))
    # M as a two-site MPS in the fit's gauge (site 1 right-canonical)
    Q, R = np.linalg.qr(M.T)
    m = [(R.T).reshape(1, d, d), (Q.T).reshape(d, d, 1)]
    mt, ks = truncate_cutoff(m, cutoff, 1)
    U, S, Vh = np.linalg.svd(M)
    k = keep_count(S, cutoff, 1)
    assert ks == [k]
    best = (U[:, :k] * S[:k]) @ Vh[:k]
    got = _dense(mt).reshape(d, d)
    assert np.linalg.norm(got - best) <= 1e-12 * np.linalg.norm(M)
    # the discarded weight is the Eckart-Young error
    err = np.linalg.norm(M - got) ** 2
    assert abs(err - np.sum(S[k:] ** 2)) <= 1e-12 * np.sum(S ** 2)


@pytest.mark.parametrize("cutoff,chi_min", [(1e-2, 1), (1e-3, 2), (5e-2, 3)])
def test_multisite_rank_and_error_bound(cutoff, chi_min):
    rng = np.random.default_rng(11)
    L, d, chi = 6, 2, 8
    m = _random_mps(rng, L, d, chi, decay=0.6)
    psi = _dense(m)
    mt, ks = truncate_cutoff(m, cutoff, chi_min)
    assert [x.shape for x in mt] == [x.shape for x in m]  # zero padding keeps shapes
    psit = _dense(mt)
    for c in range(L - 1):
        sv = np.linalg.svd(psit.reshape(d ** (c + 1), -1), compute_uv=False)
        rank = int(np.count_nonzero(sv > 1e-10 * sv[0]))
        assert rank <= ks[c]
        full = np.linalg.svd(psi.reshape(d ** (c + 1), -1), compute_uv=False)
        assert ks[c] >= min(chi_min, int(np.count_nonzero(full > 1e-12 * full[0])))
    err = np.linalg.norm(psi - psit) ** 2
    assert err <= (L - 1) * cutoff * np.linalg.norm(psi) ** 2 * (1 + 1e-9)
    assert any(k < x.shape[2] for k, x in zip(ks, m[:-1]))  # something was truncated


def test_cutoff_that_drops_nothing_is_identity():
    rng = np.random.default_rng(12)
    m = _random_mps(rng, 5, 2, 4)
    mt, ks = truncate_cutoff(m, 1e-300, 64)
    assert ks == [x.shape[2] for x in m[:-1]]
    assert np.linalg.norm(_dense(mt) - _dense(m)) <= 1e-13


@pytest.mark.parametrize("cutoff,chi_min", [(1e-2, 1), (1e-1, 1), (3e-2, 2)])
def test_sum_q_is_one_with_cutoff(cutoff, chi_min):
    lat = square_lattice(3, 3, 2)
    T = random_peps(lat, "haar", 0.6, 41)
    below, _, _ = boundary_set(T, 4)
    tot = 0.0
    truncated = False
    for x in itertools.product([0, 1], repeat=lat.n_qubits):
        used = np.zeros(3, dtype=np.int64)
        _, lq, _ = sample_one(T, lat.site_index, below, 4, 2, 0, 5, forced_bits=x,
                              svd_cutoff=cutoff, chi_x_min=chi_min, chi_used=used)
        truncated |= bool(used[1] < 4 or used[2] < 4)
        tot += math.exp(lq)
    assert abs(tot - 1.0) < 1e-12
    assert truncated


def test_cutoff_that_drops_nothing_matches_fixed_bond():
    lat = square_lattice(3, 4, 2)
    T = random_peps(lat, "haar", 0.4, 42)
    a = sample(T, lat.site_index, 6, 3, 6, seed=9)
    used = np.zeros((6, 3), dtype=np.int64)
    b = sample(T, lat.site_index, 6, 3, 6, seed=9, svd_cutoff=1e-300, chi_x_min=64, chi_used=used)
    assert np.array_equal(a[0], b[0])
    assert np.allclose(a[1], b[1], rtol=0, atol=1e-11)
    assert np.allclose(a[2], b[2], rtol=0, atol=1e-10)
    # row 0 is conditioned on nothing; after row 0 the exact product has bond
    # D = 2; after row 1 the fit keeps chi_x = 3
    assert np.all(used[:, 0] == 1) and np.all(used[:, 1] == 2) and np.all(used[:, 2] == 3)
