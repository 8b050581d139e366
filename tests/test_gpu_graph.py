"""Graph replay of sampler waves: the second full wave's launches are captured
into a HIP graph and replayed for the later full waves.  The same samples drawn
with replay and with every wave run directly must agree exactly (same kernels,
arguments, memory and order), every replayed wave is checked (eager work --
the wave's input and output copies and the host's flag check -- and a stream
synchronisation sit between replays), and both agree with the FP64 oracle."""
import numpy as np
import pytest

from peps_inputs import square_lattice, brick_lattice, random_peps, sample_uniforms
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    import paper_2507_11424_amd as tnb
    h = tnb.Handle(0)
    yield h
    h.test_sample_config(0, 0, None)
    h.close()


def c64(T):
    return [[t.astype(np.complex64).astype(np.complex128) for t in row] for row in T]


CASES = {
    # name: (lattice, recipe, eps, seed, chi, chi_x, svd_cutoff)
    "sq4x4D3": (lambda: square_lattice(4, 4, 3), "haar", 0.6, 51, 4, 3, 0.0),
    "brick5x4D2": (lambda: brick_lattice(5, 4, 2), "haar", 0.5, 52, 3, 2, 0.0),
    "sq4x4D3_cutoff": (lambda: square_lattice(4, 4, 3), "haar", 0.6, 51, 9, 9, 1e-3),
}


def _run(h, P, o, n, wave, graphs, uniforms, timing=False):
    import torch
    nq = P.n_qubits
    lc = torch.full((n, nq), float("nan"), dtype=torch.float64, device="cuda")
    h.test_sample_config(wave, 0, lc, graphs)
    h.set_timing(timing)
    try:
        bits, lq, lp, cu = h.sample(P, o, n, seed=9, first=3, uniforms=uniforms, want_chi=True)
        ctr = h.counters()
    finally:
        h.set_timing(False)
        h.test_sample_config(0, 0, None)
    torch.cuda.synchronize()
    return bits.cpu().numpy(), lq.cpu().numpy(), lp.cpu().numpy(), cu.cpu().numpy(), lc.cpu().numpy(), ctr


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "bf16x6"])
@pytest.mark.parametrize("given_uniforms", [False, True])
def test_replayed_waves_equal_direct_waves(handle, name, prec, given_uniforms):
    import torch
    import paper_2507_11424_amd as tnb
    mk, rec, eps, seed, chi, chi_x, cutoff = CASES[name]
    lat = mk()
    T = random_peps(lat, rec, eps, seed)
    if prec != "fp64":
        T = c64(T)
    P = tnb.Peps.from_numpy(lat, T, dtype="c128" if prec == "fp64" else "c64")
    o = tnb.make_opts(chi=chi, chi_x=chi_x, prec=prec, svd_cutoff=cutoff, chi_x_min=2)
    n, wave = 26, 4  # 6 full waves (1 direct, 1 captured, 4 replayed) and a ragged wave of 2
    u = torch.from_numpy(sample_uniforms(5, n, lat.n_qubits)) if given_uniforms else None
    handle.sample(P, o, 2, seed=1)  # computes and caches the norm boundary set before the counted calls
    g = _run(handle, P, o, n, wave, True, u)
    d = _run(handle, P, o, n, wave, False, u)
    names = ("bits", "log_q", "log_p", "chi_x_used", "log_cond")
    for k, (a, b) in enumerate(zip(g[:5], d[:5])):
        assert np.array_equal(a, b, equal_nan=(a.dtype.kind == "f")), names[k]
    # waves 3-6 replayed the graph captured (and launched) for wave 2
    assert g[5]["graph_launches"] == 5 and d[5]["graph_launches"] == 0
    # the replays' work enters the counters like the direct waves' work
    assert g[5]["gemm_launches"] == d[5]["gemm_launches"]
    assert g[5]["gemm_flops"] == d[5]["gemm_flops"]
    # and against the oracle (FP64 on the same, possibly complex64-rounded, values)
    used = np.zeros((n, lat.rows), dtype=np.int64)
    rb, rq, rp = oracle.sample(T, lat.site_index, chi, chi_x, n, seed=9, first=3,
                               uniforms=None if u is None else u.numpy(), svd_cutoff=cutoff, chi_x_min=2,
                               chi_used=used)
    # FP64 1e-9; bf16x6 1e-5 per conditional, so 1e-5 sqrt(N) on sums of N of them
    tol = 1e-9 if prec == "fp64" else 1e-5 * np.sqrt(lat.n_qubits)
    assert np.array_equal(g[0], rb)
    assert np.array_equal(g[3], used)
    assert np.abs(g[1] - rq).max() < tol
    assert np.abs(g[2] - rp).max() < tol


def test_timed_calls_run_waves_directly(handle):
    """Per-launch timing needs host-issued launches: with timing on, no wave is
    replayed, and the results equal the replayed run's."""
    import paper_2507_11424_amd as tnb
    lat = square_lattice(4, 4, 3)
    T = random_peps(lat, "haar", 0.6, 51)
    P = tnb.Peps.from_numpy(lat, T)
    o = tnb.make_opts(chi=4, chi_x=3)
    handle.sample(P, o, 2, seed=1)  # caches the norm boundary set
    g = _run(handle, P, o, 20, 4, True, None, timing=False)
    t = _run(handle, P, o, 20, 4, True, None, timing=True)
    assert g[5]["graph_launches"] == 4 and t[5]["graph_launches"] == 0
    assert np.array_equal(g[0], t[0]) and np.array_equal(g[1], t[1])
    assert t[5]["gemm_launches"] == g[5]["gemm_launches"] > 0 and t[5]["gemm_ms"] > 0
