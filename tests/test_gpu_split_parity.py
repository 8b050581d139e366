"""Parity of the reduced-precision GEMM modes (FP32, split-BF16 with six and
with three products) with the FP64 oracle, element by element on the same
complex64-rounded inputs: one-site density matrices, <ZZ> and two-site
marginals (tn_environments), and samples (bits, log q, log p and every drawn
qubit's conditional, tn_sample), in truncated regimes.

Tolerances (absolute; an absolute error of a log is the relative error of the
quantity):
* FP32 and bf16x6 are held to 1e-5.  Their GEMM operands carry 24 significand
  bits (FP32 rounding, or three BF16 parts of 8 bits each).
* bf16x3 keeps two BF16 parts (16 significand bits) and drops the lo*lo
  product, so every product carries a relative error of about 2^-16 = 1.5e-5
  before any accumulation: it cannot meet 1e-5 on quantities built from chains
  of contractions.  It is held to BF16X3_TOL, with the measured errors printed.
* FP64 (the reference mode of the kernels) is held to 1e-9 in the rare-bit test.
"""
import math

import numpy as np
import pytest

from peps_inputs import square_lattice, brick_lattice, rotated_square_lattice, random_peps, sample_uniforms
import oracle

pytestmark = pytest.mark.gpu

BF16X3_TOL = 3e-4
TOL = {"fp64": 1e-9, "fp32": 1e-5, "bf16x6": 1e-5, "bf16x3": BF16X3_TOL}


@pytest.fixture(scope="module")
def handle():
    import paper_2507_11424_amd as tnb
    h = tnb.Handle(0)
    yield h
    h.test_sample_config(0, 0, None)
    h.close()


def c64(T):
    return [[t.astype(np.complex64).astype(np.complex128) for t in row] for row in T]


STATES = {
    "sq4x4D3": lambda: (lambda l: (l, c64(random_peps(l, "haar", 0.6, 51))))(square_lattice(4, 4, 3)),
    "brick5x4D2": lambda: (lambda l: (l, c64(random_peps(l, "haar", 0.5, 52))))(brick_lattice(5, 4, 2)),
    "rotsq18D3": lambda: (lambda l: (l, c64(random_peps(l, "haar", 0.4, 55))))(rotated_square_lattice(3, 4, 8)),
    "sq3x5D4": lambda: (lambda l: (l, c64(random_peps(l, "haar", 0.3, 56))))(square_lattice(3, 5, 4)),
}
PRECS = ["fp32", "bf16x6", "bf16x3"]


def dev_peps(lat, T, dtype="c64"):
    import paper_2507_11424_amd as tnb
    return tnb.Peps.from_numpy(lat, T, dtype=dtype)


def opts(**kw):
    import paper_2507_11424_amd as tnb
    return tnb.make_opts(**kw)


@pytest.mark.parametrize("name,chi", [("sq4x4D3", 4), ("brick5x4D2", 3), ("rotsq18D3", 5), ("sq3x5D4", 6)])
@pytest.mark.parametrize("prec", PRECS)
def test_environments_split(handle, name, chi, prec):
    lat, T = STATES[name]()
    ref = oracle.environments(T, chi)
    got = handle.environments(dev_peps(lat, T), opts(chi=chi, prec=prec))
    errs = {}
    rho = got["rho1"].cpu().numpy()
    errs["rho1"] = float(np.nanmax(np.abs(rho - ref["rho1"])))
    for k in ("zz_h", "zz_v", "p2_h", "p2_v"):
        errs[k] = float(np.nanmax(np.abs(got[k].cpu().numpy() - ref[k])))
    print(f"{name} chi={chi} {prec}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v < TOL[prec], (k, v)


@pytest.mark.parametrize("name,chi,chi_x", [("sq4x4D3", 4, 3), ("brick5x4D2", 3, 2), ("rotsq18D3", 5, 3),
                                            ("sq3x5D4", 6, 5)])
@pytest.mark.parametrize("prec", PRECS)
def test_sample_split(handle, name, chi, chi_x, prec):
    """Bits identical to the oracle's on stored uniforms; log q, log p and every
    drawn qubit's conditional log P(x_q | earlier) within the mode's bound."""
    import torch
    lat, T = STATES[name]()
    n = 24
    nq = lat.n_qubits
    u = sample_uniforms(19, n, nq)
    lc_ref = np.full((n, nq), np.nan)
    rb, rq, rp = oracle.sample(T, lat.site_index, chi, chi_x, n, seed=5, first=2, uniforms=u, log_cond=lc_ref)
    lc = torch.full((n, nq), float("nan"), dtype=torch.float64, device="cuda")
    handle.test_sample_config(0, 0, lc)
    try:
        bits, lq, lp = handle.sample(dev_peps(lat, T), opts(chi=chi, chi_x=chi_x, prec=prec), n, seed=5, first=2,
                                     uniforms=torch.from_numpy(u))
    finally:
        handle.test_sample_config(0, 0, None)
    bits, lq, lp, lc = bits.cpu().numpy(), lq.cpu().numpy(), lp.cpu().numpy(), lc.cpu().numpy()
    e = dict(log_q=np.abs(lq - rq).max(), log_p=np.abs(lp - rp).max(), log_cond=np.abs(lc - lc_ref).max())
    print(f"{name} chi={chi} chi_x={chi_x} {prec}: " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert np.array_equal(bits, rb)
    for k, v in e.items():
        assert v < TOL[prec], (k, v)


def rare_bit_state():
    """A 3x4 square D=2 state whose qubit at (1, 2) has P(1) of order 1e-6:
    that site's s = 1 slice is scaled by 1e-3 (amplitudes, so 1e-6 in
    probability).  The qubit is not first in its row, so the sampler's
    difference route applies to it."""
    lat = square_lattice(3, 4, 2)
    T = random_peps(lat, "haar", 0.5, 71)
    T[1][2] = T[1][2].copy()
    T[1][2][1] *= 1e-3
    return lat, c64(T), int(lat.site_index[1, 2])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3"])
@pytest.mark.parametrize("chi,chi_x", [(4, 4), (3, 2)])
def test_rare_bit_conditional(handle, prec, chi, chi_x):
    """Samples forced (by their uniforms) to draw the improbable bit: identical
    bits, and its conditional -- never clamped to zero, never taken from a
    difference of two near-equal numbers -- within the mode's bound of the
    oracle's."""
    import torch
    lat, T, q = rare_bit_state()
    n = 8
    nq = lat.n_qubits
    u = sample_uniforms(23, n, nq)
    u[:, q] = 1.0 - 1e-12  # draws x_q = 1 whenever P(0) < 1 - 1e-12
    lc_ref = np.full((n, nq), np.nan)
    rb, rq, rp = oracle.sample(T, lat.site_index, chi, chi_x, n, seed=1, uniforms=u, log_cond=lc_ref)
    assert np.all(rb[:, q] == 1)
    assert np.all(lc_ref[:, q] < math.log(1e-4)), lc_ref[:, q]
    lc = torch.full((n, nq), float("nan"), dtype=torch.float64, device="cuda")
    handle.test_sample_config(0, 0, lc)
    try:
        bits, lq, lp = handle.sample(dev_peps(lat, T, "c128" if prec == "fp64" else "c64"),
                                     opts(chi=chi, chi_x=chi_x, prec=prec), n, seed=1, uniforms=torch.from_numpy(u))
    finally:
        handle.test_sample_config(0, 0, None)
    bits, lq, lc = bits.cpu().numpy(), lq.cpu().numpy(), lc.cpu().numpy()
    print(f"{prec} chi={chi}: rare log P {lc[:, q]} vs {lc_ref[:, q]}; max |d log q| {np.abs(lq - rq).max():.2e}")
    assert np.array_equal(bits, rb)
    assert np.abs(lc[:, q] - lc_ref[:, q]).max() < TOL[prec]
    assert np.abs(lq - rq).max() < TOL[prec]
