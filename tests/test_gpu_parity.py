"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same
seeded inputs: norms in all four contraction directions, environments, and
samples (bits, log q, log p), in exact and truncated regimes, FP64 and the
reduced-precision GEMM modes."""
import math

import numpy as np
import pytest

from peps_inputs import (square_lattice, brick_lattice, rotated_square_lattice, random_peps, make_config,
                         sample_uniforms)
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
    "sq3x5D2": lambda: (lambda l: (l, random_peps(l, "product0", 0.4, 53)))(square_lattice(3, 5, 2)),
    # rotated-square patches: dummy grid positions and staggered rows, as in the 105-qubit chip
    "rotsq10D2": lambda: (lambda l: (l, random_peps(l, "haar", 0.5, 54)))(rotated_square_lattice(2, 4, 4)),
    "rotsq18D3": lambda: (lambda l: (l, random_peps(l, "haar", 0.4, 55)))(rotated_square_lattice(3, 4, 8)),
}


@pytest.mark.parametrize("name,chi", [("c1", 16), ("sq4x4D3", 4), ("sq4x4D3", 9), ("brick5x4D2", 3),
                                      ("sq3x5D2", 2), ("sq4x4D3", 81), ("rotsq10D2", 64), ("rotsq18D3", 5)])
@pytest.mark.parametrize("direction", [0, 1, 2, 3])
@pytest.mark.parametrize("force_fit", [False, True])
def test_norm_fp64(handle, name, chi, direction, force_fit):
    lat, T = STATES[name]()
    ref = oracle.norm(T, chi, sweeps=2, seed=0, direction=direction, force_fit=force_fit)
    got = handle.boundary_contract(dev_peps(lat, T), opts(chi=chi, direction=direction, force_fit=force_fit))
    assert abs(got[0] - ref[0]) < 1e-10, (got, ref)
    assert abs(got[1] - ref[1]) < 1e-9


@pytest.mark.parametrize("sweeps", [1, 3])
def test_norm_sweeps_and_seed(handle, sweeps):
    lat, T = STATES["sq4x4D3"]()
    ref = oracle.norm(T, 5, sweeps=sweeps, seed=77)
    got = handle.boundary_contract(dev_peps(lat, T), opts(chi=5, sweeps=sweeps, init_seed=77))
    assert abs(got[0] - ref[0]) < 1e-10


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 1e-4), ("bf16x6", 1e-5)])
def test_norm_reduced_precision(handle, prec, tol):
    lat, T = STATES["sq4x4D3"]()
    T64 = [[t.astype(np.complex64).astype(np.complex128) for t in row] for row in T]
    ref = oracle.norm(T64, 9)
    got = handle.boundary_contract(dev_peps(lat, T64, "c64"), opts(chi=9, prec=prec))
    assert abs(got[0] - ref[0]) < tol, (got, ref)


def test_norm_c2_chi32(handle):
    lat, T, cfg = make_config("c2")
    ref = oracle.norm(T, 32)
    got = handle.boundary_contract(dev_peps(lat, T), opts(chi=32))
    assert abs(got[0] - ref[0]) < 1e-10, (got, ref)


@pytest.mark.parametrize("name,chi", [("c1", 16), ("sq4x4D3", 4), ("brick5x4D2", 3), ("rotsq10D2", 64),
                                      ("rotsq18D3", 5)])
def test_environments_fp64(handle, name, chi):
    lat, T = STATES[name]()
    ref = oracle.environments(T, chi)
    got = handle.environments(dev_peps(lat, T), opts(chi=chi))
    rho = got["rho1"].cpu().numpy()
    assert np.nanmax(np.abs(rho - ref["rho1"])) < 1e-10
    assert np.array_equal(np.isnan(rho.real), np.isnan(ref["rho1"].real))
    for k in ("zz_h", "zz_v", "p2_h", "p2_v"):
        g = got[k].cpu().numpy()
        assert np.nanmax(np.abs(g - ref[k])) < 1e-10, k


@pytest.mark.parametrize("name,chi,chi_x,force", [("c1", 16, 16, False), ("c1", 16, 16, True),
                                                   ("sq4x4D3", 4, 3, False), ("brick5x4D2", 3, 2, False),
                                                   ("sq3x5D2", 2, 2, True), ("rotsq10D2", 64, 64, False),
                                                   ("rotsq18D3", 5, 3, False)])
@pytest.mark.parametrize("given_uniforms", [True, False])
def test_sample_fp64(handle, name, chi, chi_x, force, given_uniforms):
    import torch
    lat, T = STATES[name]()
    n = 24
    u = sample_uniforms(9, n, lat.n_qubits) if given_uniforms else None
    rb, rq, rp = oracle.sample(T, lat.site_index, chi, chi_x, n, seed=123, first=5, force_fit=force,
                               uniforms=u)
    P = dev_peps(lat, T)
    o = opts(chi=chi, chi_x=chi_x, force_fit=force)
    bits, lq, lp = handle.sample(P, o, n, seed=123, first=5,
                                 uniforms=torch.from_numpy(u) if u is not None else None)
    bits, lq, lp = bits.cpu().numpy(), lq.cpu().numpy(), lp.cpu().numpy()
    assert np.array_equal(bits, rb)
    assert np.abs(lq - rq).max() < 1e-9
    assert np.abs(lp - rp).max() < 1e-9


def test_sample_split_runs_reproduce_one_run(handle):
    lat, T = STATES["sq4x4D3"]()
    P = dev_peps(lat, T)
    o = opts(chi=4, chi_x=3)
    b_all, q_all, _ = handle.sample(P, o, 20, seed=5, first=0)
    b1, q1, _ = handle.sample(P, o, 7, seed=5, first=0)
    b2, q2, _ = handle.sample(P, o, 13, seed=5, first=7)
    import torch
    assert torch.equal(torch.cat([b1, b2]), b_all)
    assert torch.equal(torch.cat([q1, q2]), q_all)


def test_sample_exact_matches_statevector(handle):
    lat, T, cfg = make_config("c1")
    psi = oracle.statevector(T, lat.site_index)
    p = np.abs(psi) ** 2
    Z = p.sum()
    bits, lq, lp = handle.sample(dev_peps(lat, T), opts(chi=16, chi_x=16), 200, seed=11)
    bits, lq, lp = bits.cpu().numpy(), lq.cpu().numpy(), lp.cpu().numpy()
    for b, q, pp in zip(bits, lq, lp):
        x = tuple(int(v) for v in b)
        assert abs(q - math.log(p[x] / Z)) < 1e-10
        assert abs(pp - math.log(p[x])) < 1e-10


@pytest.mark.parametrize("name,chi,chi_x,cutoff,chi_min", [("sq4x4D3", 9, 9, 1e-2, 1), ("sq4x4D3", 9, 9, 1e-4, 2),
                                                           ("brick5x4D2", 3, 4, 1e-3, 2),
                                                           ("rotsq18D3", 5, 6, 5e-3, 1), ("c1", 16, 16, 1e-2, 1)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sample_svd_cutoff(handle, name, chi, chi_x, cutoff, chi_min, prec):
    """Adaptive amplitude-boundary bond: bits, log q, log p and the per-row
    kept bonds against the oracle's SVD sweep."""
    lat, T = STATES[name]()
    n = 16
    rows = len(T)
    used = np.zeros((n, rows), dtype=np.int64)
    rb, rq, rp = oracle.sample(T, lat.site_index, chi, chi_x, n, seed=77, first=3, svd_cutoff=cutoff,
                               chi_x_min=chi_min, chi_used=used)
    dtype = "c128" if prec == "fp64" else "c64"
    if dtype == "c64":
        T = [[t.astype(np.complex64).astype(np.complex128) for t in row] for row in T]
        rb, rq, rp = oracle.sample(T, lat.site_index, chi, chi_x, n, seed=77, first=3, svd_cutoff=cutoff,
                                   chi_x_min=chi_min, chi_used=used)
    o = opts(chi=chi, chi_x=chi_x, svd_cutoff=cutoff, chi_x_min=chi_min, prec=prec)
    bits, lq, lp, cu = handle.sample(dev_peps(lat, T, dtype), o, n, seed=77, first=3, want_chi=True)
    bits, lq, lp, cu = bits.cpu().numpy(), lq.cpu().numpy(), lp.cpu().numpy(), cu.cpu().numpy()
    tol = 1e-9 if prec == "fp64" else 1e-5
    assert np.array_equal(bits, rb)
    assert np.array_equal(cu, used)
    assert np.abs(lq - rq).max() < tol
    assert np.abs(lp - rp).max() < tol


def test_sample_svd_cutoff_truncates_and_reports(handle):
    """With the cutoff the kept bonds vary per sample and stay within
    [chi_x_min, chi_x]; without it they equal the fixed widths."""
    lat, T = STATES["sq4x4D3"]()
    P = dev_peps(lat, T)
    _, _, _, cu0 = handle.sample(P, opts(chi=9, chi_x=9), 32, seed=4, want_chi=True)
    _, _, _, cu1 = handle.sample(P, opts(chi=9, chi_x=9, svd_cutoff=3e-2, chi_x_min=2), 32, seed=4, want_chi=True)
    cu0, cu1 = cu0.cpu().numpy(), cu1.cpu().numpy()
    assert np.all(cu0[:, 0] == 1) and np.all(cu1[:, 0] == 1)
    assert np.all(cu0 == cu0[0])
    assert np.all(cu1 <= cu0) and np.all(cu1[:, 1:] >= 2)
    assert (cu1 < cu0).any()
    assert len({tuple(r) for r in cu1}) > 1


@pytest.mark.parametrize("call", ["sample", "environments"])
def test_cache_follows_contents_not_addresses(handle, call):
    """A state overwritten in place (same device pointers, same lattice and
    options) must not be served the boundary set cached for the old contents:
    sample / environments of state A, copy state B into A's buffers, call again,
    compare with the oracle on B."""
    import torch
    lat = square_lattice(4, 4, 3)
    TA = random_peps(lat, "haar", 0.6, 61)
    TB = random_peps(lat, "haar", 0.6, 62)
    P = dev_peps(lat, TA)
    o = opts(chi=4, chi_x=3)
    if call == "sample":
        handle.sample(P, o, 8, seed=3)
    else:
        handle.environments(P, o)
    flat = [t for row in TB for t in row]
    for dst, src in zip(P.tensors, flat):
        dst.copy_(torch.from_numpy(np.ascontiguousarray(src)).to(dst.device))
    if call == "sample":
        rb, rq, rp = oracle.sample(TB, lat.site_index, 4, 3, 8, seed=3)
        bits, lq, lp = handle.sample(P, o, 8, seed=3)
        assert np.array_equal(bits.cpu().numpy(), rb)
        assert np.abs(lq.cpu().numpy() - rq).max() < 1e-9
        assert np.abs(lp.cpu().numpy() - rp).max() < 1e-9
    else:
        ref = oracle.environments(TB, 4)
        got = handle.environments(P, o)
        assert np.nanmax(np.abs(got["rho1"].cpu().numpy() - ref["rho1"])) < 1e-10
        assert np.nanmax(np.abs(got["zz_h"].cpu().numpy() - ref["zz_h"])) < 1e-10
