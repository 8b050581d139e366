"""Parity of the HIP path with the FP64 oracle on the other planar partitions:
the heavy-hex lattice with its degree-2 bridge qubits as sites of their own
(bridge rows of the grid, mostly dummies), and the staggered-row partition of
the rotated square lattice (rows alternating qubits with fused down-diagonal
legs and junction tensors).  Norms in the four contraction directions, one-site
density matrices and <ZZ>, and samples (bits, log q, log p), exact and
truncated.  The oracle is pinned on these lattices to statevectors and, for
the staggered rows, to the native diagonal network (test_oracle_pins.py)."""
import numpy as np
import pytest

from peps_inputs import heavy_hex_lattice, staggered_lattice, random_peps, sample_uniforms
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
    "heavyhex3x5D2": lambda: (lambda l: (l, random_peps(l, "haar", 0.5, 61)))(heavy_hex_lattice(3, 5, 2)),
    "heavyhex3x9D3": lambda: (lambda l: (l, random_peps(l, "haar", 0.4, 62)))(heavy_hex_lattice(3, 9, 3)),
    "stag10D2": lambda: (lambda l: (l, random_peps(l, "haar", 0.5, 63)))(staggered_lattice(2, 4, 4)),
    "stag18D2": lambda: (lambda l: (l, random_peps(l, "haar", 0.5, 64)))(staggered_lattice(2, 4, 8)),
}


@pytest.mark.parametrize("name,chi", [("heavyhex3x5D2", 64), ("heavyhex3x5D2", 3), ("heavyhex3x9D3", 6),
                                      ("stag10D2", 256), ("stag10D2", 5), ("stag18D2", 7)])
@pytest.mark.parametrize("direction", [0, 1, 2, 3])
@pytest.mark.parametrize("force_fit", [False, True])
def test_norm_partitions(handle, name, chi, direction, force_fit):
    lat, T = STATES[name]()
    ref = oracle.norm(T, chi, sweeps=2, seed=0, direction=direction, force_fit=force_fit)
    got = handle.boundary_contract(dev_peps(lat, T), opts(chi=chi, direction=direction, force_fit=force_fit))
    assert abs(got[0] - ref[0]) < 1e-10, (got, ref)
    assert abs(got[1] - ref[1]) < 1e-9


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x6", 1e-5)])
@pytest.mark.parametrize("name,chi", [("heavyhex3x9D3", 6), ("stag18D2", 7)])
def test_norm_partitions_reduced_precision(handle, name, chi, prec, tol):
    lat, T = STATES[name]()
    T64 = [[t.astype(np.complex64).astype(np.complex128) for t in row] for row in T]
    ref = oracle.norm(T64, chi)
    got = handle.boundary_contract(dev_peps(lat, T64, "c64"), opts(chi=chi, prec=prec))
    assert abs(got[0] - ref[0]) < tol, (got, ref)


@pytest.mark.parametrize("name,chi", [("heavyhex3x5D2", 64), ("heavyhex3x9D3", 6), ("stag10D2", 256),
                                      ("stag18D2", 7)])
def test_environments_partitions(handle, name, chi):
    lat, T = STATES[name]()
    ref = oracle.environments(T, chi)
    got = handle.environments(dev_peps(lat, T), opts(chi=chi))
    rho = got["rho1"].cpu().numpy()
    assert np.nanmax(np.abs(rho - ref["rho1"])) < 1e-10
    assert np.array_equal(np.isnan(rho.real), np.isnan(ref["rho1"].real))
    for k in ("zz_h", "zz_v", "p2_h", "p2_v"):
        g = got[k].cpu().numpy()
        assert np.array_equal(np.isnan(g), np.isnan(ref[k])), k
        if not np.all(np.isnan(g)):  # staggered rows: no two qubits are grid neighbours in a row
            assert np.nanmax(np.abs(g - ref[k])) < 1e-10, k


@pytest.mark.parametrize("name,chi,chi_x", [("heavyhex3x5D2", 64, 64), ("heavyhex3x9D3", 6, 4),
                                            ("stag10D2", 256, 256), ("stag18D2", 7, 5)])
@pytest.mark.parametrize("given_uniforms", [True, False])
def test_sample_partitions(handle, name, chi, chi_x, given_uniforms):
    import torch
    lat, T = STATES[name]()
    n = 24
    u = sample_uniforms(19, n, lat.n_qubits) if given_uniforms else None
    rb, rq, rp = oracle.sample(T, lat.site_index, chi, chi_x, n, seed=321, first=3, uniforms=u)
    bits, lq, lp = handle.sample(dev_peps(lat, T), opts(chi=chi, chi_x=chi_x), n, seed=321, first=3,
                                 uniforms=torch.from_numpy(u) if u is not None else None)
    bits, lq, lp = bits.cpu().numpy(), lq.cpu().numpy(), lp.cpu().numpy()
    assert np.array_equal(bits, rb)
    assert np.abs(lq - rq).max() < 1e-9
    assert np.abs(lp - rp).max() < 1e-9
