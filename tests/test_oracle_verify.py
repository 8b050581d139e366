"""Pins of the oracle's independent p(x) check and sample-quality metrics.

* <x|psi> at a bond that reaches the exact bound equals the statevector
  amplitude (modulus and phase), for the direct path and the forced fit;
* a truncated bond gives a different (approximate) p that converges as the bond
  grows;
* the metrics reduce to closed forms: q = p/Z gives KLD = 0, N = Z and an
  effective sample size of n; small hand-computed two- and three-sample cases;
* unbiasedness of N: sum_x q(x) p(x)/q(x) = Z, with q from exhaustive
  enumeration of the sampler at a truncated bond and p from the statevector.
"""
import itertools
import math

import numpy as np
import pytest

from peps_inputs import square_lattice, brick_lattice, random_peps, make_config
from oracle.statevector import statevector
from oracle.sampler import sample, sample_one
from oracle.boundary import boundary_set
from oracle.philox import TAG_INIT_DOWN
from oracle.verify import amplitude, amplitudes, sample_stats


def _cases():
    yield "square3x3D2", square_lattice(3, 3, 2), random_peps(square_lattice(3, 3, 2), "product0", 0.3, 21), 8
    yield "brick4x4D2", brick_lattice(4, 4, 2), random_peps(brick_lattice(4, 4, 2), "haar", 0.4, 23), 8
    lat, T, cfg = make_config("c1")
    yield "c1", lat, T, 16


@pytest.mark.parametrize("case", list(_cases()), ids=lambda c: c[0])
@pytest.mark.parametrize("force_fit", [False, True])
def test_amplitude_exact_equals_statevector(case, force_fit):
    name, lat, T, chi_v = case
    psi = statevector(T, lat.site_index)
    rng = np.random.default_rng(5)
    for i in range(5):
        x = rng.integers(0, 2, lat.n_qubits).astype(np.uint8)
        lp, arg = amplitude(T, lat.site_index, x, chi_v, sample=i, force_fit=force_fit)
        a = psi[tuple(int(b) for b in x)]
        assert abs(lp - math.log(abs(a) ** 2)) < 1e-10, (name, i)
        d = (arg - math.atan2(a.imag, a.real) + math.pi) % (2 * math.pi) - math.pi
        assert abs(d) < 1e-9


def test_amplitude_truncated_converges():
    lat = square_lattice(4, 4, 3)
    T = random_peps(lat, "haar", 0.6, 41)
    psi = statevector(T, lat.site_index)
    rng = np.random.default_rng(9)
    X = rng.integers(0, 2, (6, lat.n_qubits)).astype(np.uint8)
    ref = np.array([math.log(abs(psi[tuple(int(b) for b in x)]) ** 2) for x in X])
    errs = []
    for chi_v in (1, 3, 81):
        lp, _ = amplitudes(T, lat.site_index, X, chi_v)
        errs.append(np.max(np.abs(lp - ref)))
    assert errs[0] > 1e-6          # the bond-1 contraction is really an approximation
    assert errs[2] < 1e-10         # 81 = 3^4 is the exact bound of a 4-column row
    assert errs[1] < errs[0]


def test_stats_exact_sampling_closed_form():
    rng = np.random.default_rng(3)
    log_Z = 2.7
    log_p = rng.normal(size=50) - 30.0
    log_q = log_p - log_Z
    s = sample_stats(log_q, log_p, log_Z)
    assert abs(s["kld"]) < 1e-13
    assert abs(s["log_norm_est"] - log_Z) < 1e-13
    assert abs(s["ess"] - 50) < 1e-9


def test_stats_hand_computed():
    # two samples, q = 1/2 each, p = 0.3 and 0.1 (Z = 0.5)
    lq = np.log([0.5, 0.5])
    lp = np.log([0.3, 0.1])
    s = sample_stats(lq, lp, math.log(0.5), bits=np.array([[0, 1], [1, 1]], dtype=np.uint8))
    assert abs(math.exp(s["log_norm_est"]) - (0.6 + 0.2) / 2) < 1e-15
    kld = 0.5 * (math.log(0.5 / 0.6) + math.log(0.5 / 0.2))
    assert abs(s["kld"] - kld) < 1e-15
    assert abs(s["ess"] - 0.8 ** 2 / (0.36 + 0.04)) < 1e-12
    # weights 0.6 : 0.2 = 3 : 1; qubit 0 is 0 then 1, qubit 1 is 1 twice
    assert np.allclose(s["z_is"], [(3 - 1) / 4, -1.0], atol=1e-15)
    # ratios far out of exp's range
    s2 = sample_stats(np.array([-800.0, -801.0, -802.0]), np.array([-1600.0, -1600.0, -1600.0]), -700.0)
    w = np.exp([-800.0 + 800, -799.0 + 800, -798.0 + 800])
    assert abs(s2["log_norm_est"] - (-800.0 + math.log(w.sum() / 3))) < 1e-12


def test_norm_estimate_unbiased_by_enumeration():
    # sum_x q(x) [p(x)/q(x)] = Z with q from the truncated sampler over all 2^9 x
    lat = square_lattice(3, 3, 2)
    T = random_peps(lat, "haar", 0.7, 44)
    psi = statevector(T, lat.site_index)
    p = np.abs(psi) ** 2
    below, _, _ = boundary_set(T, 2, 2, 0, TAG_INIT_DOWN)
    n = lat.n_qubits
    tot_q = 0.0
    est = 0.0
    for x in itertools.product((0, 1), repeat=n):
        _, lq, _ = sample_one(T, lat.site_index, below, 1, 2, 0, 0, forced_bits=np.array(x, dtype=np.uint8))
        q = math.exp(lq)
        tot_q += q
        if q > 0:
            est += q * (p[x] / q)
    assert abs(tot_q - 1.0) < 1e-12
    assert abs(est - p.sum()) < 1e-12 * p.sum()
    # the same truncated sampler draws samples whose KLD is positive (q != p/Z)
    bits, lq, _ = sample(T, lat.site_index, 2, 1, 64, seed=8)
    lp = np.array([math.log(p[tuple(int(v) for v in b)]) for b in bits])
    assert sample_stats(lq, lp, math.log(p.sum()))["kld"] > 1e-6
