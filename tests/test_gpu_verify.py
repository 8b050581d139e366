"""Parity of the independent p(x) check (tn_amplitude) and of the sample-quality
metrics (tn_sample_stats) with the FP64 oracle, on the same seeded inputs and
bitstrings; exact bonds are also checked against the statevector."""
import math

import numpy as np
import pytest

from peps_inputs import square_lattice, brick_lattice, random_peps, make_config
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    import paper_2507_11424_amd as tnb
    h = tnb.Handle(0)
    yield h
    h.close()


def dev_peps(lat, T, dtype="c128"):
    import paper_2507_11424_amd as tnb
    return tnb.Peps.from_numpy(lat, T, dtype=dtype)


def opts(**kw):
    import paper_2507_11424_amd as tnb
    return tnb.make_opts(**kw)


STATES = {
    "c1": lambda: make_config("c1")[:2],
    "sq4x4D3": lambda: (lambda l: (l, random_peps(l, "haar", 0.6, 51)))(square_lattice(4, 4, 3)),
    "brick5x4D2": lambda: (lambda l: (l, random_peps(l, "haar", 0.5, 52)))(brick_lattice(5, 4, 2)),
}


def _bits(lat, n, seed):
    return np.random.default_rng(seed).integers(0, 2, (n, lat.n_qubits)).astype(np.uint8)


@pytest.mark.parametrize("name,chi_v,force", [("c1", 16, False), ("c1", 16, True), ("sq4x4D3", 81, False),
                                              ("sq4x4D3", 3, False), ("sq4x4D3", 5, True), ("brick5x4D2", 2, False)])
def test_amplitude_fp64(handle, name, chi_v, force):
    import torch
    lat, T = STATES[name]()
    X = _bits(lat, 37, 4)   # 37: more than one tile of samples and a ragged tail
    ref_lp, ref_arg = oracle.amplitudes(T, lat.site_index, X, chi_v, first=5, force_fit=force)
    lp, arg = handle.amplitude(dev_peps(lat, T), opts(chi_x=chi_v, force_fit=force), torch.from_numpy(X).cuda(),
                               first=5, want_arg=True)
    lp = lp.cpu().numpy()
    arg = arg.cpu().numpy()
    assert np.max(np.abs(lp - ref_lp)) < 1e-9
    d = (arg - ref_arg + math.pi) % (2 * math.pi) - math.pi
    assert np.max(np.abs(d)) < 1e-8
    if chi_v >= 16:  # exact bond: the statevector itself
        psi = oracle.statevector(T, lat.site_index)
        ex = np.array([math.log(abs(psi[tuple(int(b) for b in x)]) ** 2) for x in X])
        assert np.max(np.abs(lp - ex)) < 1e-10


# bf16x3 keeps ~16 significand bits per operand (hi + lo bf16 parts, the lo*lo
# product dropped): a relative error of ~2^-16 per GEMM compounds over the
# fits of 3 rows; measured 1.3e-4 on log p here, hence its looser bound.
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x6", 1e-5), ("bf16x3", 5e-4)])
def test_amplitude_reduced_precision(handle, prec, tol):
    import torch
    lat, T = STATES["sq4x4D3"]()
    T64 = [[t.astype(np.complex64).astype(np.complex128) for t in row] for row in T]
    X = _bits(lat, 20, 6)
    ref, _ = oracle.amplitudes(T64, lat.site_index, X, 4)
    lp = handle.amplitude(dev_peps(lat, T64, "c64"), opts(chi_x=4, prec=prec), torch.from_numpy(X).cuda())
    assert np.max(np.abs(lp.cpu().numpy() - ref)) < tol


def test_amplitude_agrees_with_exact_sampler(handle):
    # at exact bonds the sampler's p(x) and the separate check coincide
    lat, T = STATES["c1"]()
    P = dev_peps(lat, T)
    bits, lq, lp = handle.sample(P, opts(chi=16, chi_x=16), 16, seed=3)
    lp2 = handle.amplitude(P, opts(chi_x=16), bits)
    assert np.max(np.abs(lp.cpu().numpy() - lp2.cpu().numpy())) < 1e-10


@pytest.mark.parametrize("n", [1, 7, 300, 1000])
def test_sample_stats_matches_oracle(handle, n):
    import torch
    rng = np.random.default_rng(n)
    lq = rng.normal(size=n) - 20.0
    lp = lq + rng.normal(size=n) * 0.7 - 400.0
    bits = rng.integers(0, 2, (n, 13)).astype(np.uint8)
    ref = oracle.sample_stats(lq, lp, -399.0, bits)
    got = handle.sample_stats(torch.from_numpy(lq).cuda(), torch.from_numpy(lp).cuda(), -399.0,
                              bits=torch.from_numpy(bits).cuda())
    for k in ("log_norm_est", "kld", "ess"):
        assert abs(got[k] - ref[k]) < 1e-12 * max(1.0, abs(ref[k])), k
    assert np.max(np.abs(got["z_is"].cpu().numpy() - ref["z_is"])) < 1e-12


def test_truncated_sampling_metrics_end_to_end(handle):
    # truncated sampler (chi_x = 1) checked by a separate exact contraction: the
    # metrics from the GPU outputs equal the oracle's metrics of the same numbers,
    # and the KLD is positive (the samples are not exact)
    import torch
    lat, T = STATES["sq4x4D3"]()
    P = dev_peps(lat, T)
    lz, _ = handle.boundary_contract(P, opts(chi=81))
    bits, lq, _ = handle.sample(P, opts(chi=81, chi_x=1), 64, seed=12)
    lp = handle.amplitude(P, opts(chi_x=81), bits)
    got = handle.sample_stats(lq, lp, lz, bits=bits)
    ref = oracle.sample_stats(lq.cpu().numpy(), lp.cpu().numpy(), lz, bits.cpu().numpy())
    assert abs(got["kld"] - ref["kld"]) < 1e-12 and got["kld"] > 1e-6
    assert abs(got["log_norm_est"] - ref["log_norm_est"]) < 1e-12
    psi = oracle.statevector(T, lat.site_index)
    ex = np.array([math.log(abs(psi[tuple(int(b) for b in x)]) ** 2) for x in bits.cpu().numpy()])
    assert np.max(np.abs(lp.cpu().numpy() - ex)) < 1e-10
