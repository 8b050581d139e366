"""Pins of the simple-update oracle (oracle/circuit.py) and of the circuit
inputs (peps_inputs/circuits.py) against things other than themselves:

* the Heisenberg gate against SciPy's matrix exponential of -i dt H;
* the colour groups are matchings that cover every bond once;
* where no singular value is discarded (eps = 0) the evolved PEPS is the
  statevector evolved gate by gate (dense linear algebra, global phase and norm
  aside);
* on a tree (no loops) the BP messages are exact environments, so a single
  truncated gate keeps exactly the fraction 1 - eps of the norm: 1 - eps
  equals the fidelity |<psi_exact|psi>|^2 / (|psi_exact|^2 |psi|^2);
* the gate errors do not depend on the gauge of the input state (random
  invertible matrices on every bond), on a lattice with loops too.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from peps_inputs import square_lattice, brick_lattice, heavy_hex_lattice, Lattice, random_peps, _index_sites
from peps_inputs.circuits import heisenberg_gate, edge_groups, heisenberg_circuit, domain_wall_peps
from oracle.circuit import simple_update, message_roots, bond_legs
from oracle.statevector import statevector
from oracle import bp as obp

X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.diag([1.0, -1.0]).astype(np.complex128)


@pytest.mark.parametrize("dt,J", [(0.1, 1.0), (0.37, -0.6), (1.3, 2.0)])
def test_heisenberg_gate_is_the_exponential(dt, J):
    H = J * (np.kron(X, X) + np.kron(Y, Y) + np.kron(Z, Z))
    G = heisenberg_gate(dt, J)
    assert np.abs(G - scipy.linalg.expm(-1j * dt * H)).max() < 1e-14
    assert np.abs(G @ G.conj().T - np.eye(4)).max() < 1e-14


@pytest.mark.parametrize("lat,K", [(square_lattice(4, 5, 2), 4), (brick_lattice(5, 6, 2), 3),
                                   (heavy_hex_lattice(3, 9, 2), 4)])
def test_edge_groups_are_matchings(lat, K):
    groups = edge_groups(lat)
    assert len(groups) == K
    seen = set()
    for g in groups:
        qubits = [q for (r, c, r2, c2) in g for q in ((r, c), (r2, c2))]
        assert len(qubits) == len(set(qubits))
        for e in g:
            assert e not in seen
            seen.add(e)
    bonds = {(r, c, r, c + 1) for r in range(lat.rows) for c in range(lat.cols - 1) if lat.dim_h[r, c] > 1}
    bonds |= {(r, c, r + 1, c) for r in range(lat.rows - 1) for c in range(lat.cols) if lat.dim_v[r, c] > 1}
    assert seen == bonds


def test_domain_wall_state():
    lat = square_lattice(2, 4, 3)
    psi = statevector(domain_wall_peps(lat), lat.site_index)
    bits = tuple(0 if c < 2 else 1 for r in range(2) for c in range(4))
    assert abs(psi[bits] - 1.0) < 1e-15 and abs(np.sum(np.abs(psi) ** 2) - 1.0) < 1e-15


def _dense_evolve(psi, lat, gates, G):
    """Gates applied to the statevector (axis = the qubit's bit position)."""
    psi = psi.copy()
    for (_, r, c, r2, c2) in gates:
        a, b = int(lat.site_index[r, c]), int(lat.site_index[r2, c2])
        psi = np.moveaxis(psi, (a, b), (0, 1))
        sh = psi.shape
        psi = (G @ psi.reshape(4, -1)).reshape(sh)
        psi = np.moveaxis(psi, (0, 1), (a, b))
    return psi


def _fidelity(a, b):
    return abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


@pytest.mark.parametrize("lat,layers", [(square_lattice(1, 5, 4), 3), (square_lattice(2, 2, 4), 1),
                                        (square_lattice(2, 2, 16), 2), (brick_lattice(3, 3, 4), 1),
                                        (square_lattice(2, 3, 8), 1)])
def test_exact_regime_is_the_evolved_statevector(lat, layers):
    T0 = domain_wall_peps(lat)
    gates, G = heisenberg_circuit(lat, layers, 0.3)
    T, eps, f = simple_update(T0, gates, G)
    assert max(eps) < 1e-24 and abs(f - 1.0) < 1e-15
    ref = _dense_evolve(statevector(T0, lat.site_index), lat, gates, G)
    got = statevector(T, lat.site_index)
    assert 1.0 - _fidelity(ref, got) < 1e-12
    # an entangled state was reached (not a product state)
    p = np.abs(ref) ** 2
    assert np.count_nonzero(p > 1e-6) > 2


@pytest.mark.parametrize("lat,layers", [(square_lattice(2, 3, 8), 1), (heavy_hex_lattice(3, 5, 8), 1)])
def test_quench_conserves_the_magnetisation(lat, layers):
    """Every Heisenberg gate commutes with sum_i Z_i: the exactly evolved
    domain wall has weight only on bitstrings with the domain wall's number of
    1s (domain_wall_ones), the property the GPU quench-then-sample test and
    bench check on the samples."""
    from peps_inputs.circuits import domain_wall_ones
    T0 = domain_wall_peps(lat)
    gates, G = heisenberg_circuit(lat, layers, 0.3)
    T, eps, _ = simple_update(T0, gates, G)
    assert max(eps) < 1e-24
    psi = statevector(T, lat.site_index)
    ones = np.indices(psi.shape).sum(axis=0)
    want = domain_wall_ones(lat)
    w = np.abs(psi) ** 2
    assert np.sum(w[ones != want]) < 1e-24 * np.sum(w)
    assert np.count_nonzero(w[ones == want] > 1e-8 * w.max()) > 2


def _comb(rows, cols, D):
    phys = np.full((rows, cols), 2, np.int32)
    dh = np.full((rows, cols - 1), D, np.int32)
    dv = np.ones((rows - 1, cols), np.int32)
    dv[:, 0] = D
    return Lattice(f"comb{rows}x{cols}_D{D}", rows, cols, phys, dh, dv, _index_sites(phys))


@pytest.mark.parametrize("lat,gate", [(square_lattice(1, 6, 2), (0, 0, 2, 0, 3)),
                                      (square_lattice(1, 5, 3), (0, 0, 1, 0, 2)),
                                      (_comb(3, 3, 2), (0, 1, 0, 2, 0)),
                                      (_comb(3, 3, 2), (0, 1, 0, 1, 1))])
def test_tree_truncation_keeps_one_minus_eps(lat, gate):
    """A random (entangled) state on a tree, one gate with truncation: BP
    messages are the exact environments, so the fidelity of the truncated
    state with the exactly evolved one is 1 - eps."""
    rng = np.random.default_rng(5)
    T0 = random_peps(lat, "haar", 0.9, 11)
    G = scipy.linalg.expm(-1j * 0.7 * (np.kron(X, X) + 0.3 * np.kron(Y, Z) + np.kron(Z, X)))
    gates = [gate]
    T, eps, f = simple_update(T0, gates, G)
    assert eps[0] > 1e-6  # something was discarded
    ref = _dense_evolve(statevector(T0, lat.site_index), lat, gates, G)
    got = statevector(T, lat.site_index)
    assert abs(_fidelity(ref, got) - (1.0 - eps[0])) < 1e-10
    assert abs(f - (1.0 - eps[0])) < 1e-15


def _gauge(lat, T, seed):
    """The same state with a random invertible matrix on every bond."""
    rng = np.random.default_rng(seed)
    T = [[t.copy() for t in row] for row in T]
    for r in range(lat.rows):
        for c in range(lat.cols):
            for (r2, c2) in ((r, c + 1), (r + 1, c)):
                if r2 >= lat.rows or c2 >= lat.cols:
                    continue
                lv, lw = bond_legs(r, c, r2, c2)
                D = T[r][c].shape[lv]
                if D == 1:
                    continue
                Xg = np.eye(D) + 0.4 * (rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D)))
                T[r][c] = np.moveaxis(np.tensordot(T[r][c], Xg, axes=(lv, 0)), -1, lv)
                T[r2][c2] = np.moveaxis(np.tensordot(T[r2][c2], np.linalg.inv(Xg).T, axes=(lw, 0)), -1, lw)
    return T


@pytest.mark.parametrize("lat", [square_lattice(3, 3, 2), brick_lattice(4, 4, 2), _comb(3, 3, 2)],
                         ids=lambda l: l.name)
def test_gate_errors_are_gauge_invariant(lat):
    T0 = random_peps(lat, "haar", 0.6, 12)
    T1 = _gauge(lat, T0, 3)
    assert 1.0 - _fidelity(statevector(T0, lat.site_index), statevector(T1, lat.site_index)) < 1e-12
    gates, G = heisenberg_circuit(lat, 1, 0.4)
    _, e0, f0 = simple_update(T0, gates, G)
    _, e1, f1 = simple_update(T1, gates, G)
    assert max(e0) > 1e-8
    assert np.abs(np.array(e0) - np.array(e1)).max() < 1e-9
    assert abs(f0 - f1) < 1e-9


def test_message_roots():
    """Root and pseudo-inverse root of a rank-deficient message: s^2 = m, s
    Hermitian, s si the projector on the range of m."""
    rng = np.random.default_rng(2)
    A = rng.standard_normal((5, 3)) + 1j * rng.standard_normal((5, 3))
    m = A @ A.conj().T  # rank 3 of 5
    s, si = message_roots(m)
    assert np.abs(s @ s - m).max() < 1e-12 * np.abs(m).max()
    assert np.abs(s - s.conj().T).max() < 1e-14
    P = s @ si
    assert np.abs(P @ P - P).max() < 1e-12 and abs(np.trace(P).real - 3) < 1e-12
    assert np.abs(P @ m - m).max() < 1e-12 * np.abs(m).max()


def _random_unitaries(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        q, r = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
        out.append(q * (np.diagonal(r) / np.abs(np.diagonal(r))))
    return np.array(out)


def test_gauge_covariance_within_a_group():
    """From a random product state (rank-one messages) through random gates
    (generic, non-degenerate singular values), a unitary gauge on every bond
    leaves every later gate error and the evolved state unchanged, also where
    both ends of a bond are updated within one group on the messages of the
    group's start.  (Symmetric inputs, such as the domain wall under the
    Heisenberg gate, can put a degenerate pair of singular values across the
    cut, where the kept vectors are not unique.)"""
    lat = square_lattice(3, 3, 2)
    gates, _ = heisenberg_circuit(lat, 2, 0.2)
    Gs = _random_unitaries(len(gates), 4)
    T, _, _ = simple_update(random_peps(lat, "haar", 0.0, 13), gates[:6], Gs[:6])
    for seed in range(4):
        rng = np.random.default_rng(seed)
        Tg = [[t.copy() for t in row] for row in T]
        for r in range(lat.rows):
            for c in range(lat.cols):
                for (r2, c2) in ((r, c + 1), (r + 1, c)):
                    if r2 >= lat.rows or c2 >= lat.cols:
                        continue
                    lv, lw = bond_legs(r, c, r2, c2)
                    D = Tg[r][c].shape[lv]
                    Xg, _ = np.linalg.qr(rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D)))
                    Tg[r][c] = np.moveaxis(np.tensordot(Tg[r][c], Xg, axes=(lv, 0)), -1, lv)
                    Tg[r2][c2] = np.moveaxis(np.tensordot(Tg[r2][c2], Xg.conj(), axes=(lw, 0)), -1, lw)
        Ta, ea, _ = simple_update(T, gates[6:12], Gs[6:12])
        Tb, eb, _ = simple_update(Tg, gates[6:12], Gs[6:12])
        assert max(ea) > 1e-4
        assert np.abs(np.array(ea) - np.array(eb)).max() < 1e-9
        sa, sb = statevector(Ta, lat.site_index), statevector(Tb, lat.site_index)
        assert 1.0 - _fidelity(sa, sb) < 1e-12
