"""Pins of the FP64 oracle against things other than itself.

* NumPy's Philox bit generator (a library implementation of the same published
  generator);
* brute-force summation over every bond assignment;
* exact statevectors (the definition of the state) for the norm, one-site
  density matrices, <ZZ>, and per-sample q(x) = |psi(x)|^2 / Z at exact bond;
* the product-state closed form (D = 1) and the single-row case (an MPS,
  perfect sampling);
* for the staggered-row partition of the rotated square lattice (qubits with
  fused down-diagonal legs and junction tensors in the grid), the state of the
  native diagonal network, contracted directly with one tensor per qubit and
  one index per diagonal bond.
"""
import itertools
import math

import numpy as np
import pytest

from peps_inputs import (square_lattice, brick_lattice, random_peps, Lattice, site_dims,
                         rotated_square_lattice, make_config, heavy_hex_lattice, staggered_lattice,
                         staggered_sites)
from oracle import philox
from oracle.statevector import statevector, brute_force_amplitude
from oracle.boundary import norm, boundary_set, plan_bonds
from oracle.sampler import sample, sample_one
from oracle.environments import environments


# --------------------------------------------------------------------------- Philox

@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2**64 - 1, 2**63 + 11)])
@pytest.mark.parametrize("start", [(0, 0, 0, 0), (41, 3, 9, 2), (2**64 - 2, 7, 0, 5)])
def test_philox_matches_numpy(key, start):
    # NumPy increments the 256-bit counter (word 0 least significant) before each block
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(start, dtype=np.uint64))
    raw = bg.random_raw(12)
    ctr = list(start)
    for blk in range(3):
        # 256-bit increment with carry
        for i in range(4):
            ctr[i] = (ctr[i] + 1) % 2**64
            if ctr[i] != 0:
                break
        mine = philox.philox4x64_10(tuple(ctr), key)
        assert tuple(int(x) for x in raw[4 * blk: 4 * blk + 4]) == mine
        vec = philox.philox4x64_10_vec(np.array([ctr[0]], dtype=np.uint64), ctr[1], ctr[2], ctr[3],
                                       *key)
        assert tuple(int(v[0]) for v in vec) == mine


def test_philox_uniform_and_init_maps():
    w = philox.philox4x64_10((3, 1, 4, 1), (5, 2))
    u = philox.word_to_uniform(w[0])
    assert 0.0 <= u < 1.0 and u == (w[0] >> 11) / 2.0**53
    t1 = philox.init_tensor(9, 2, 4, 3, 17, (2, 3, 2))
    t2 = philox.init_tensor_vec(9, 2, 4, 3, 17, (2, 3, 2))
    assert np.array_equal(t1, t2)
    assert np.all(np.abs(t2.real) <= 1) and np.all(np.abs(t2.imag) <= 1)
    d = philox.draw_uniforms_vec(123, 5, 7, 3)
    assert d[2, 4] == philox.draw_uniform(123, 4, 9)


# --------------------------------------------------------------------------- statevector

def _small_lattices():
    yield square_lattice(2, 2, 2)
    yield square_lattice(2, 3, 3)
    yield brick_lattice(3, 3, 2)
    # a lattice with a dummy grid position in the middle of the top row
    lat = square_lattice(2, 3, 2)
    lat.phys[0, 1] = 1
    lat.dim_h[0, 0] = lat.dim_h[0, 1] = 1
    lat.dim_v[0, 1] = 1
    yield Lattice("dummy2x3", 2, 3, lat.phys, lat.dim_h, lat.dim_v,
                  np.array([[0, -1, 1], [2, 3, 4]], dtype=np.int32))


@pytest.mark.parametrize("lat", list(_small_lattices()), ids=lambda l: l.name)
def test_statevector_vs_brute_force(lat):
    T = random_peps(lat, "haar", 0.4, 3)
    psi = statevector(T, lat.site_index)
    assert psi.shape == (2,) * lat.n_qubits
    rng = np.random.default_rng(0)
    for _ in range(6):
        x = tuple(int(b) for b in rng.integers(0, 2, lat.n_qubits))
        a = brute_force_amplitude(T, lat.site_index, x)
        assert abs(psi[x] - a) <= 1e-13 * max(1.0, abs(a))


def test_product_state_closed_form():
    # D = 1: psi is a product state; Z = prod ||a_i||^2 and the qubits are independent
    lat = square_lattice(3, 3, 1)
    rng = np.random.default_rng(4)
    T = [[(rng.standard_normal((2, 1, 1, 1, 1)) + 1j * rng.standard_normal((2, 1, 1, 1, 1)))
          for _ in range(3)] for _ in range(3)]
    Z = np.prod([np.linalg.norm(t) ** 2 for row in T for t in row])
    lz, ph = norm(T, 4)
    assert abs(lz - math.log(Z)) < 1e-12 and abs(ph) < 1e-12
    env = environments(T, 4)
    for r in range(3):
        for c in range(3):
            a = T[r][c].reshape(2)
            p0 = abs(a[0]) ** 2 / np.sum(np.abs(a) ** 2)
            assert abs(env["rho1"][r, c, 0, 0].real - p0) < 1e-13
            assert abs(env["rho1"][r, c, 0, 1] - a[0] * np.conj(a[1]) / np.sum(np.abs(a) ** 2)) < 1e-13
    # q(x) = prod_i p_i(x_i)
    bits, lq, lp = sample(T, square_lattice(3, 3, 1).site_index, 4, 4, 5, seed=1)
    for b, q in zip(bits, lq):
        ref = 0.0
        for r in range(3):
            for c in range(3):
                a = T[r][c].reshape(2)
                ref += math.log(abs(a[b[3 * r + c]]) ** 2 / np.sum(np.abs(a) ** 2))
        assert abs(q - ref) < 1e-12


# --------------------------------------------------------------------------- exact bond

EXACT_CASES = [
    ("square3x3D2", lambda: square_lattice(3, 3, 2), "product0", 0.3, 21, 64),
    ("square3x4D3", lambda: square_lattice(3, 4, 3), "haar", 0.5, 22, 4096),
    ("brick4x4D2", lambda: brick_lattice(4, 4, 2), "haar", 0.4, 23, 64),
    ("c1", None, None, None, None, 16),
    # rotated square patch: 10 qubits in a 4x4 embedding with dummy sites
    ("rotsq10D2", lambda: rotated_square_lattice(2, 4, 4), "haar", 0.5, 24, 64),
    # heavy-hex with bridge sites: 3 chains of 5 and 3 bridges (18 qubits)
    ("heavyhex3x5D2", lambda: heavy_hex_lattice(3, 5, 2), "haar", 0.5, 25, 64),
    # the same 10-qubit rotated square in staggered rows (junctions, fused legs)
    ("stag10D2", lambda: staggered_lattice(2, 4, 4), "haar", 0.5, 26, 256),
]


def _case(name):
    for nm, mk, rec, eps, seed, chi in EXACT_CASES:
        if nm == name:
            if mk is None:
                lat, T, cfg = make_config("c1")
                return lat, T, chi
            lat = mk()
            return lat, random_peps(lat, rec, eps, seed), chi
    raise KeyError(name)


@pytest.mark.parametrize("name", [c[0] for c in EXACT_CASES])
@pytest.mark.parametrize("force_fit", [False, True])
def test_norm_exact_all_directions(name, force_fit):
    lat, T, chi = _case(name)
    psi = statevector(T, lat.site_index)
    lz = math.log(np.sum(np.abs(psi) ** 2))
    for d in range(4):
        l, ph = norm(T, chi, direction=d, force_fit=force_fit)
        assert abs(l - lz) < 1e-11, (d, l, lz)
        assert abs(ph) < 1e-10


def test_c1_bond_16_is_exact():
    # 4x4 square, D=2: the exact bound of every boundary is <= 16 (phys 4 per site, 4 columns)
    lat, T, cfg = make_config("c1")
    below, logs, info = boundary_set(T, 16)
    assert all(i["mode"] == "exact" for i in info[:-1])
    _, _, info8 = boundary_set(T, 8)
    assert any(i["mode"] == "fit" for i in info8[:-1])


@pytest.mark.parametrize("name", ["square3x3D2", "brick4x4D2", "rotsq10D2", "heavyhex3x5D2", "stag10D2"])
def test_environments_exact(name):
    lat, T, chi = _case(name)
    psi = statevector(T, lat.site_index)
    Z = np.sum(np.abs(psi) ** 2)
    env = environments(T, chi)
    n = lat.n_qubits
    P = np.abs(psi) ** 2 / Z
    idx = np.indices((2,) * n)
    for r in range(lat.rows):
        for c in range(lat.cols):
            q = lat.site_index[r, c]
            if q < 0:  # dummy grid position: no qubit, NaN by definition
                assert np.all(np.isnan(env["rho1"][r, c]))
                continue
            ps = np.moveaxis(psi, q, 0).reshape(2, -1)
            rho = ps @ ps.conj().T / Z
            assert np.abs(rho - env["rho1"][r, c]).max() < 1e-12
            if c + 1 < lat.cols and lat.site_index[r, c + 1] >= 0:
                q2 = lat.site_index[r, c + 1]
                zz = np.sum(P * (1 - 2 * idx[q]) * (1 - 2 * idx[q2]))
                assert abs(zz - env["zz_h"][r, c]) < 1e-12
                p2 = [np.sum(P * (idx[q] == s) * (idx[q2] == t)) for s in (0, 1) for t in (0, 1)]
                assert np.abs(np.array(p2) - env["p2_h"][r, c]).max() < 1e-12
            if r + 1 < lat.rows and lat.site_index[r + 1, c] >= 0:
                q2 = lat.site_index[r + 1, c]
                zz = np.sum(P * (1 - 2 * idx[q]) * (1 - 2 * idx[q2]))
                assert abs(zz - env["zz_v"][r, c]) < 1e-12
                # (s, t) = (upper, lower) qubit: a swapped order leaves zz unchanged but not p2
                p2 = [np.sum(P * (idx[q] == s) * (idx[q2] == t)) for s in (0, 1) for t in (0, 1)]
                assert np.abs(np.array(p2) - env["p2_v"][r, c]).max() < 1e-12
    # without the two-row environments: the same one-site and horizontal values
    env_h = environments(T, chi, vertical=False)
    for k in ("rho1", "zz_h", "p2_h"):
        assert np.array_equal(env_h[k], env[k], equal_nan=True)
    assert np.all(np.isnan(env_h["zz_v"])) and np.all(np.isnan(env_h["p2_v"]))


@pytest.mark.parametrize("name", ["square3x3D2", "brick4x4D2", "c1", "rotsq10D2", "heavyhex3x5D2", "stag10D2"])
@pytest.mark.parametrize("force_fit", [False, True])
def test_sampler_exact_q_equals_p_over_Z(name, force_fit):
    lat, T, chi = _case(name)
    psi = statevector(T, lat.site_index)
    p = np.abs(psi) ** 2
    Z = p.sum()
    bits, lq, lp = sample(T, lat.site_index, chi, chi, 12, seed=77, force_fit=force_fit)
    for b, q, pp in zip(bits, lq, lp):
        x = tuple(int(v) for v in b)
        assert abs(q - math.log(p[x] / Z)) < 1e-10
        assert abs(pp - math.log(p[x])) < 1e-10


def test_single_row_is_mps_perfect_sampling():
    # one row: the PEPS is an MPS and boundary-MPS sampling is exact at any chi
    lat = square_lattice(1, 6, 3)
    T = random_peps(lat, "haar", 0.7, 31)
    psi = statevector(T, lat.site_index)
    p = np.abs(psi) ** 2
    bits, lq, lp = sample(T, lat.site_index, 1, 1, 10, seed=3)
    for b, q in zip(bits, lq):
        assert abs(q - math.log(p[tuple(b)] / p.sum())) < 1e-11
    lz, _ = norm(T, 1)
    assert abs(lz - math.log(p.sum())) < 1e-12


def test_rotated_square_geometry():
    lat = rotated_square_lattice(2)
    assert (lat.rows, lat.cols) == (15, 15)
    occ = (lat.phys == 2).sum(axis=1)
    assert occ.sum() == 105
    deg = np.zeros((lat.rows, lat.cols), int)
    deg[:, :-1] += lat.dim_h > 1
    deg[:, 1:] += lat.dim_h > 1
    deg[:-1, :] += lat.dim_v > 1
    deg[1:, :] += lat.dim_v > 1
    assert deg.max() == 4 and deg[lat.phys == 1].max() == 0
    # chip bonds (r, x)-(r+1, x+-1): 20 between each of the 9 pairs of adjacent chip rows
    assert (lat.dim_h > 1).sum() + (lat.dim_v > 1).sum() == 180


def test_brick_is_degree_three():
    lat = brick_lattice(6, 6, 2)
    for r in range(1, 5):
        for c in range(1, 5):
            p, du, dl, dd, dr = site_dims(lat, r, c)
            assert (du > 1) + (dd > 1) + (dl > 1) + (dr > 1) == 3


def test_plan_bonds_consistency():
    ok, t = plan_bonds([4, 4, 4, 4], [16, 16, 16], 16)
    assert ok and t == [4, 16, 4]
    # every cut has a side with a physical space of at most 64, but the exact
    # product's bond (4096) is far above max(chi, 64): fitted to the bound instead
    ok, t = plan_bonds([64, 1, 64, 1], [4096, 4096, 4096], 64)
    assert not ok and t == [64, 64, 1]
    ok, t = plan_bonds([64, 1, 64, 1], [64, 64, 64], 64)
    assert ok and t == [64, 64, 1]
    phys = [64, 64, 1, 64, 64, 1]
    ok, t = plan_bonds(phys, [4096, 512, 4096, 4096, 512], 64)
    assert not ok and t == [64, 64, 64, 64, 1]
    ok, t = plan_bonds([2, 2, 2, 2], [100, 3, 100], 8)
    assert t == [2, 3, 2]


@pytest.mark.parametrize("name", ["square3x3D2", "brick4x4D2", "rotsq10D2", "heavyhex3x5D2", "stag10D2"])
@pytest.mark.parametrize("rows_limit", [1, 2])
def test_sampler_partial_rows_and_conditionals_exact(name, rows_limit):
    """At exact bond, the per-qubit conditionals are ratios of statevector
    marginals of the prefixes in sampling order (rows top-down, columns
    left-to-right), and a run stopped after k rows has log q = log of the
    marginal probability of the drawn bits of those rows."""
    lat, T, chi = _case(name)
    psi = statevector(T, lat.site_index)
    P = np.abs(psi) ** 2
    P = P / P.sum()
    n_q = lat.n_qubits
    order = [int(lat.site_index[r, c]) for r in range(lat.rows) for c in range(lat.cols)
             if lat.site_index[r, c] >= 0]
    n = 6
    lc = np.full((n, n_q), np.nan)
    bits, lq, lp = sample(T, lat.site_index, chi, chi, n, seed=91, rows_limit=rows_limit, log_cond=lc)
    done = [int(lat.site_index[r, c]) for r in range(rows_limit) for c in range(lat.cols)
            if lat.site_index[r, c] >= 0]
    for i in range(n):
        prev = 0.0
        for k in range(1, len(done) + 1):
            sel = order[:k]
            marg = np.moveaxis(P, sel, list(range(k))).reshape((2,) * k + (-1,)).sum(axis=-1)
            lm = math.log(marg[tuple(int(bits[i, q]) for q in sel)])
            assert abs((lm - prev) - lc[i, sel[-1]]) < 1e-10
            prev = lm
        assert abs(prev - lq[i]) < 1e-10
        assert np.all(np.isnan(lc[i, [q for q in range(n_q) if q not in done]]))
        assert not np.any(bits[i, [q for q in range(n_q) if q not in done]])
        assert math.isnan(lp[i])


# --------------------------------------------------------------------------- new partitions

def test_heavy_hex_geometry():
    """Chain qubits have degree <= 3, bridges degree 2; every hexagon of the
    3 x 9 patch has 12 qubits: 2 bridges and 5 qubits of each chain."""
    lat = heavy_hex_lattice(3, 9, 2)
    deg = np.zeros((lat.rows, lat.cols), int)
    deg[:, :-1] += lat.dim_h > 1
    deg[:, 1:] += lat.dim_h > 1
    deg[:-1, :] += lat.dim_v > 1
    deg[1:, :] += lat.dim_v > 1
    chain = lat.phys.copy() == 2
    chain[1::2, :] = False
    bridge = (lat.phys == 2) & ~chain
    assert deg[chain].max() == 3 and set(deg[bridge].tolist()) == {2}
    assert deg[lat.phys == 1].max() == 0
    assert bridge.sum() == 3 + 2 and lat.n_qubits == 27 + 5
    # bonds: 8 per chain, 2 per bridge; a planar graph with V - E + F = 2 has
    # E - V + 1 bounded faces: here 4 hexagons of 12 edges (+ the outer face)
    V, E = lat.n_qubits, 3 * 8 + 2 * 5
    assert E - V + 1 == 3


def _native_state(lat, T, D):
    """The state of the staggered lattice contracted as its native network:
    qubit (r, x) with legs (p, ul, ur, dl, dr), one index per diagonal bond,
    read off the grid tensors (left leg = up-left bond, right leg = up-right
    bond, down leg = the fused pair of down bonds) without the junctions."""
    occ = {(r, x) for r in range(lat.rows) for x in range(lat.cols) if lat.phys[r, x] == 2}
    letters = iter("abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ")
    bond = {}

    def lab(u, v):
        key = (min(u, v), max(u, v))
        if key not in bond:
            bond[key] = next(letters)
        return bond[key]

    ops, terms, out = [], [], []
    for (r, x) in sorted(occ, key=lambda q: lat.site_index[q]):
        t = T[r][x]
        p, du, dl, dd, dr = t.shape
        assert du == 1
        ul, ur = (r - 1, x - 1), (r - 1, x + 1)
        dlq, drq = (r + 1, x - 1), (r + 1, x + 1)
        a = D if dlq in occ else 1
        b = D if drq in occ else 1
        nat = t.reshape(p, dl, a, b, dr)          # (p, ul, dl, dr, ur) after unfusing
        legs, sub = [], ["P%d" % lat.site_index[r, x]]
        names = []
        for nb, ext in ((ul, dl), (dlq, a), (drq, b), (ur, dr)):
            if nb in occ:
                names.append(lab((r, x), nb))
            else:
                assert ext == 1
                names.append(None)
        keep = [i + 1 for i, nm in enumerate(names) if nm is not None]
        sl = tuple(slice(None) if (i == 0 or i in keep) else 0 for i in range(5))
        ops.append(nat[sl])
        terms.append([nm for nm in names if nm is not None])
    phys_letters = [next(letters) for _ in ops]
    expr = ",".join(pl + "".join(tm) for pl, tm in zip(phys_letters, terms)) + "->" + "".join(phys_letters)
    return np.einsum(expr, *ops, optimize=True)


@pytest.mark.parametrize("shape", [(3, 4), (4, 4), (4, 6)])
def test_staggered_embedding_matches_native_network(shape):
    """The grid embedding (fused legs + junction tensors) holds the same state
    as the native diagonal network; the staggered 10-qubit patch and the
    45-degree embedding of the same lattice hold the same norm at exact bond."""
    rows, xmax = shape
    lat = staggered_lattice(2, rows, xmax)
    assert lat.n_qubits == len(staggered_sites(rows, xmax))
    T = random_peps(lat, "haar", 0.6, 40 + rows + xmax)
    psi_grid = statevector(T, lat.site_index)
    psi_nat = _native_state(lat, T, 2)
    assert np.abs(psi_grid - psi_nat).max() < 1e-13 * max(1.0, np.abs(psi_nat).max())
    lz, _ = norm(T, 256)
    assert abs(lz - math.log(np.sum(np.abs(psi_nat) ** 2))) < 1e-11


def test_staggered_geometry_105():
    lat = staggered_lattice(8)
    assert (lat.rows, lat.cols, lat.n_qubits) == (10, 21, 105)
    # 180 diagonal bonds: each appears once as a fused down leg and once as a
    # junction leg (left or right)
    fused = lat.dim_v[lat.dim_v > 1]
    assert sum(int(round(math.log(int(v), 8))) for v in fused) == 180
    assert (lat.dim_h > 1).sum() == 180
    # one junction below every qubit of chip rows 0..8 (5 rows of 11, 4 of 10)
    assert lat.junction.sum() == 5 * 11 + 4 * 10
