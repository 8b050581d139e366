"""Simple-update circuit simulation through the C ABI (tn_simple_update)
against the FP64 oracle (oracle/circuit.py): the gate errors eps_i, the
fidelity estimate, and the evolved state itself (its statevector: the gauge of
the new bonds, SVD phases included, cancels in the contracted state).

Tolerances: eps 1e-9 absolute (the GPU's BP stops up to three sweeps after the
oracle's, each changing messages by < 1e-13, and the reduced QR route rounds
differently from the oracle's full SVD); statevector 1e-9 relative to its
largest amplitude."""
import numpy as np
import pytest
import scipy.linalg

from peps_inputs import square_lattice, brick_lattice, heavy_hex_lattice, random_peps
from peps_inputs.circuits import heisenberg_circuit, domain_wall_peps
from oracle.circuit import simple_update
from oracle.statevector import statevector

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    import paper_2507_11424_amd as tnb
    h = tnb.Handle(0)
    yield h
    h.close()


def _random_gates(lat, layers, seed):
    """Heisenberg-coloured gate list with a different random unitary per gate."""
    gates, _ = heisenberg_circuit(lat, layers, 0.1)
    rng = np.random.default_rng(seed)
    Gs = []
    for _ in gates:
        z = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        q, r = np.linalg.qr(z)
        Gs.append(q * (np.diagonal(r) / np.abs(np.diagonal(r))))
    return gates, np.array(Gs)


# (lattice, initial state, circuit, comparison): "full" compares every gate
# error and the final state; "first" stops after the first group with a
# truncation.  The Heisenberg gate on the domain wall keeps the magnetisation,
# and the resulting degenerate pairs of singular values can straddle the cut,
# where the kept vectors are not unique (the oracle and the GPU may keep
# different ones; the gate errors up to there are fixed).
CASES = {
    "sq3x3D2-heis": lambda: (square_lattice(3, 3, 2), "dw", lambda l: heisenberg_circuit(l, 2, 0.2), "first"),
    "brick4x4D2-heis": lambda: (brick_lattice(4, 4, 2), "dw", lambda l: heisenberg_circuit(l, 2, 0.3), "first"),
    "heavyhex3x5D2-heis": lambda: (heavy_hex_lattice(3, 5, 2), "dw", lambda l: heisenberg_circuit(l, 2, 0.25),
                                   "first"),
    "sq3x3D2-product-random": lambda: (square_lattice(3, 3, 2), "product", lambda l: _random_gates(l, 2, 6),
                                       "full"),
    "heavyhex3x5D2-product-random": lambda: (heavy_hex_lattice(3, 5, 2), "product",
                                             lambda l: _random_gates(l, 2, 10), "full"),
    "sq3x3D3-random": lambda: (square_lattice(3, 3, 3), "haar", lambda l: _random_gates(l, 1, 7), "full"),
    "brick3x4D4-random": lambda: (brick_lattice(3, 4, 4), "haar", lambda l: _random_gates(l, 2, 8), "full"),
    "sq1x6D2-random": lambda: (square_lattice(1, 6, 2), "haar", lambda l: _random_gates(l, 2, 9), "full"),
    # bonds above 32: the middle column's vertical gate reduces to a 136 x 136
    # pair matrix (the SVD's global-memory path)
    "sq2x3D34-random": lambda: (square_lattice(2, 3, 34), "haar", lambda l: _random_gates(l, 1, 12), "full"),
}


def _initial(lat, init):
    if init == "dw":
        return domain_wall_peps(lat)
    if init == "product":  # random single-qubit states, rank-one messages
        return random_peps(lat, "haar", 0.0, 70)
    return random_peps(lat, "haar", 0.6, 71)


@pytest.mark.parametrize("name", list(CASES))
def test_simple_update_matches_oracle(handle, name):
    import paper_2507_11424_amd as tnb
    lat, init, circ, mode = CASES[name]()
    T0 = _initial(lat, init)
    gates, G = circ(lat)
    if mode == "first":
        groups = [g[0] for g in gates]
        T, eps, _ = simple_update(T0, gates, G)
        first = next(i for i, e in enumerate(eps) if e > 1e-12)
        last = max(i for i, g in enumerate(groups) if g == groups[first])
        gates = gates[:last + 1]
    T, eps, f = simple_update(T0, gates, G)
    out, geps, gf = handle.simple_update(tnb.Peps.from_numpy(lat, T0), gates, G)
    print(f"{name}: {len(gates)} gates, max eps {max(eps):.3e}, f {f:.12f} vs {gf:.12f}, "
          f"max |d eps| {np.abs(geps - np.array(eps)).max():.2e}")
    assert max(eps) > 1e-4  # truncation happened
    assert np.abs(geps - np.array(eps)).max() < 1e-9
    assert abs(gf - f) < 1e-9
    if mode == "full":
        ref = statevector(T, lat.site_index)
        got = statevector([[t.cpu().numpy() for t in out.tensors[r * lat.cols:(r + 1) * lat.cols]]
                           for r in range(lat.rows)], lat.site_index)
        assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max()


def test_simple_update_in_place_and_complex64(handle):
    """The result written over the input (complex64 storage, FP64 arithmetic)
    equals the complex128 run rounded once."""
    import paper_2507_11424_amd as tnb
    lat = brick_lattice(4, 4, 2)
    T0 = [[t.astype(np.complex64).astype(np.complex128) for t in row] for row in random_peps(lat, "haar", 0.5, 72)]
    gates, G = _random_gates(lat, 1, 11)
    ref, reps, _ = handle.simple_update(tnb.Peps.from_numpy(lat, T0), gates, G)
    P = tnb.Peps.from_numpy(lat, T0, dtype="c64")
    out, eps, _ = handle.simple_update(P, gates, G, in_place=True)
    assert out is P
    assert np.abs(eps - reps).max() < 1e-12
    for a, b in zip(P.tensors, ref.tensors):
        assert np.abs(a.cpu().numpy() - b.cpu().numpy().astype(np.complex64)).max() == 0.0


def test_simple_update_continues_from_messages(handle):
    """A circuit split over two calls, the second starting its BP from the
    first call's final messages, gives the same gate errors and state as one
    call over the whole circuit (and the oracle's)."""
    import paper_2507_11424_amd as tnb
    lat = brick_lattice(3, 4, 3)
    T0 = random_peps(lat, "haar", 0.5, 74)
    gates, G = _random_gates(lat, 2, 13)
    cut = next(i for i, g in enumerate(gates) if g[0] != gates[0][0])  # after the first group
    ref, reps, _ = handle.simple_update(tnb.Peps.from_numpy(lat, T0), gates, G)
    P = tnb.Peps.from_numpy(lat, T0)
    m = handle.message_buffer(P)
    _, e1, _ = handle.simple_update(P, gates[:cut], G[:cut], in_place=True, messages_out=m)
    _, e2, _ = handle.simple_update(P, gates[cut:], G[cut:], in_place=True, messages_in=m, messages_out=m)
    eps = np.concatenate([e1, e2])
    assert np.abs(eps - reps).max() < 1e-12
    for a, b in zip(P.tensors, ref.tensors):
        assert (a - b).abs().max().item() < 1e-12
    _, oeps, _ = simple_update(T0, gates, G)
    assert np.abs(eps - np.array(oeps)).max() < 1e-9


def test_simple_update_rejects_bad_gates(handle):
    import paper_2507_11424_amd as tnb
    lat = square_lattice(2, 2, 2)
    P = tnb.Peps.from_numpy(lat, random_peps(lat, "haar", 0.5, 73))
    with pytest.raises(tnb.TnError):
        handle.simple_update(P, [(0, 0, 0, 1, 1)], np.eye(4))  # diagonal pair
    with pytest.raises(tnb.TnError):
        handle.simple_update(P, [(0, 1, 1, 1, 2)], np.eye(4))  # outside the grid
    with pytest.raises(tnb.TnError):  # two gates of one group on qubit (0, 0)
        handle.simple_update(P, [(0, 0, 0, 0, 1), (0, 0, 0, 1, 0)], np.eye(4))
    # the same pair in consecutive groups is fine
    handle.simple_update(P, [(0, 0, 0, 0, 1), (1, 0, 0, 1, 0)], np.eye(4))
    # bonds above 64 (pair matrices above 256) are refused before any work
    big = square_lattice(1, 2, 65)
    Pb = tnb.Peps.from_numpy(big, random_peps(big, "haar", 0.5, 75))
    with pytest.raises(tnb.TnError, match="UNSUPPORTED"):
        handle.simple_update(Pb, [(0, 0, 0, 0, 1)], np.eye(4))
