"""End to end: the Heisenberg quench by simple update (tn_simple_update), then
the boundary-MPS norm and sampler (tn_boundary_contract, tn_sample,
tn_sample_stats) on the evolved state, as in the paper's sampling experiments
on its Heisenberg states.

Properties that fix the answer without an oracle run at this size: every
Heisenberg gate commutes with the total magnetisation sum_i Z_i, so with no
truncation (every gate error 0) the evolved state has exactly the domain
wall's number of 1s and every sample must carry it; with boundaries at the
exact bond, q(x) = p(x) / Z, so log q + log Z - log p vanishes per sample (to
the 1e-9 of the FP64 sampler) and so does the sample KLD."""
import numpy as np
import pytest

from peps_inputs import heavy_hex_lattice, square_lattice
from peps_inputs.circuits import heisenberg_circuit, domain_wall_peps, domain_wall_ones

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    import paper_2507_11424_amd as tnb
    h = tnb.Handle(0)
    yield h
    h.close()


@pytest.mark.parametrize("name,lat_fn,layers", [
    ("heavyhex3x5D8", lambda: heavy_hex_lattice(3, 5, 8), 1),
    ("heavyhex3x5D16", lambda: heavy_hex_lattice(3, 5, 16), 2),
    ("sq3x3D4", lambda: square_lattice(3, 3, 4), 1),
])
def test_quench_samples_keep_magnetisation(handle, name, lat_fn, layers):
    import torch
    import paper_2507_11424_amd as tnb
    lat = lat_fn()
    gates, G = heisenberg_circuit(lat, layers, 0.3)
    P = tnb.Peps.from_numpy(lat, domain_wall_peps(lat))
    _, eps, f = handle.simple_update(P, gates, G, in_place=True)
    assert eps.max() < 1e-14, eps.max()  # no truncation: the state is the exact Trotter state
    o = tnb.make_opts(chi=64, chi_x=64)  # above every boundary's rank after these layers
    lz, _ = handle.boundary_contract(P, o)
    n = 512
    bits, lq, lp = handle.sample(P, o, n, seed=21)[:3]
    ones = bits.to(torch.int64).sum(dim=1).cpu().numpy()
    want = domain_wall_ones(lat)
    d = (lq + lz - lp).abs().max().item()
    st = handle.sample_stats(lq, lp, lz)
    print(f"{name}: {lat.n_qubits} qubits, {len(gates)} gates, f {f:.15f}; ones {np.unique(ones)} (want {want}); "
          f"max |log q + log Z - log p| {d:.2e}; KLD {st['kld']:.2e}")
    assert np.all(ones == want)
    assert d < 1e-9
    # the separate amplitude contraction agrees at bonds well above the state's ranks
    for cx in (16, 64):
        lpc = handle.amplitude(P, tnb.make_opts(chi=cx, chi_x=cx), bits)
        assert (lpc - lp).abs().max().item() < 1e-9, cx
    assert abs(st["kld"]) < 1e-9
    # the samples are not all alike: the quench spread the domain wall
    assert len({tuple(b) for b in bits.cpu().numpy().tolist()}) > 8


def test_truncated_quench_norm_and_sampler_exact(handle):
    """A quench that truncates (gate errors up to ~1e-2 on the 4x4 square at
    D = 3): the state is no longer an exact Trotter state, but its norm and
    amplitudes are what they are -- the boundary contraction at the exact bond
    gives the statevector's norm, and the sampler's q(x) = p(x) / Z with p from
    the statevector."""
    import torch
    import paper_2507_11424_amd as tnb
    from oracle.statevector import statevector
    lat = square_lattice(4, 4, 3)
    gates, G = heisenberg_circuit(lat, 3, 0.3)
    P = tnb.Peps.from_numpy(lat, domain_wall_peps(lat))
    _, eps, f = handle.simple_update(P, gates, G, in_place=True)
    assert eps.max() > 1e-6  # truncation happened
    T = [[P.tensors[r * lat.cols + c].cpu().numpy() for c in range(lat.cols)] for r in range(lat.rows)]
    psi = statevector(T, lat.site_index)
    Z = float(np.sum(np.abs(psi) ** 2))
    o = tnb.make_opts(chi=128, chi_x=128)
    lz, _ = handle.boundary_contract(P, o)
    bits, lq, lp = handle.sample(P, o, 256, seed=5)[:3]
    b = bits.cpu().numpy()
    exact = np.array([2 * np.log(abs(psi[tuple(x)])) for x in b])
    print(f"max eps {eps.max():.2e}, f {f:.6f}; log Z {lz:.12f} vs {np.log(Z):.12f}; "
          f"max |log p - exact| {np.abs(lp.cpu().numpy() - exact).max():.2e}")
    assert abs(lz - np.log(Z)) < 1e-10
    assert np.abs(lp.cpu().numpy() - exact).max() < 1e-9
    assert (lq + lz - lp).abs().max().item() < 1e-9


def test_padded_bonds_exact(handle):
    """A state whose bonds are zero-padded beyond their rank (as simple update
    leaves them) gives the unpadded state's norm, amplitudes and samples: its
    fits meet exactly dependent columns, where CholeskyQR flags the items and
    Householder refactors them on the device."""
    import torch
    import paper_2507_11424_amd as tnb
    from peps_inputs import random_peps
    lat3, lat5 = square_lattice(4, 3, 3), square_lattice(4, 3, 5)
    small = random_peps(lat3, "haar", 0.5, seed=5)
    padded = []
    for row in small:
        prow = []
        for t in row:
            shape = (t.shape[0],) + tuple(5 if d == 3 else d for d in t.shape[1:])
            z = np.zeros(shape, dtype=t.dtype)
            z[tuple(slice(0, d) for d in t.shape)] = t
            prow.append(z)
        padded.append(prow)
    # every boundary of a 3-column lattice at D = 3 has rank <= 9: exact at chi 16,
    # where the factorised matrices are at most 16 wide (no blocked scheme)
    o = tnb.make_opts(chi=16, chi_x=16)
    res = {}
    for name, lat, T in (("plain", lat3, small), ("padded", lat5, padded)):
        P = tnb.Peps.from_numpy(lat, T)
        lz, arg = handle.boundary_contract(P, o)
        bits, lq, lp = handle.sample(P, o, 256, seed=9)[:3]
        res[name] = (lz, arg, bits.cpu().numpy(), lp.cpu().numpy())
        print(f"{name}: log|Z| {lz:.15f} arg {arg:.3e}")
    from oracle.statevector import statevector
    psi = statevector(small, lat3.site_index)
    exact = np.array([2 * np.log(abs(psi[tuple(x)])) for x in res["plain"][2]])
    assert abs(res["plain"][0] - np.log(np.sum(np.abs(psi) ** 2))) < 1e-10
    assert abs(res["plain"][0] - res["padded"][0]) < 1e-10
    assert np.array_equal(res["plain"][2], res["padded"][2])
    assert np.abs(res["plain"][3] - exact).max() < 1e-9
    assert np.abs(res["padded"][3] - exact).max() < 1e-9
