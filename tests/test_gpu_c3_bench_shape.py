"""Parity at the benchmark's own shapes (144-qubit heavy-hex-shaped brick
lattice, D = 8, chi = 64, sampling bond chi_x = 64) against FP64 oracle values
stored by tests/golden/make_golden.py (the oracle needs about an hour for them):

* the one-site density matrices of all 144 qubits and the <ZZ> and two-site
  diagonals of horizontal neighbours (the per-marginal error of every precision
  mode; the oracle's vertical two-row environments at this size are not stored);
* the first four sampled rows of two samples on stored uniforms: bits, the
  partial log q and every drawn qubit's log P(x_q | earlier qubits).  Rows 0-1
  sample under exact amplitude boundaries (bond 1 and 8), the fit after row 1
  is exact (bond 64) and the fit after row 2 truncates 512 -> 64, so row 3
  samples under a fitted boundary of the benchmark's shape.  The run draws 18
  samples in the benchmark's launch configuration (autotuned tiles, waves sized
  from free memory: 9 + 9 in FP64, 16 + 2 in the complex64 modes, so the
  transfer-matrix route, the masked steps and a ragged last wave all run) and
  compares samples 0 and 17.

Tolerances: FP64 1e-10 on marginals and 1e-9 on log-conditionals; FP32 and
bf16x6 1e-5 on every marginal and conditional, 1e-5 sqrt(N) on a log q summing
N conditionals; bf16x3 (two bf16 parts, about 2^-16 relative per product) 3e-4
on each marginal and conditional, 3e-4 sqrt(N) on log q.
"""
import json
import math
import os

import numpy as np
import pytest

from peps_inputs import make_config, sample_uniforms

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROWS = json.load(open(os.path.join(HERE, "golden", "c3_rows_chix64.json")))
ENV = json.load(open(os.path.join(HERE, "golden", "c3_env_chi64.json")))
MARG_TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x6": 1e-5, "bf16x3": 3e-4}
COND_TOL = {"fp64": 1e-9, "fp32": 1e-5, "bf16x6": 1e-5, "bf16x3": 3e-4}


@pytest.fixture(scope="module")
def state():
    import paper_2507_11424_amd as tnb
    lat, T, cfg = make_config("c3")
    h = tnb.Handle(0)
    h.set_autotune(True)
    yield h, lat, T
    h.test_sample_config(0, 0, None)
    h.close()


def _env_ref():
    rho = np.array([complex(a, b) for a, b in ENV["rho1"]]).reshape(ENV["rho1_shape"])
    f = lambda v: np.nan if v is None else v  # noqa: E731
    zzh = np.array([f(v) for v in ENV["zz_h"]]).reshape(ENV["zz_h_shape"])
    p2h = np.array([f(v) for v in ENV["p2_h"]]).reshape(ENV["p2_h_shape"])
    return rho, zzh, p2h


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3"])
def test_c3_marginals_per_qubit(state, prec):
    import paper_2507_11424_amd as tnb
    h, lat, T = state
    P = tnb.Peps.from_numpy(lat, T, dtype="c128" if prec == "fp64" else "c64")
    o = tnb.make_opts(chi=ENV["chi"], sweeps=ENV["sweeps"], init_seed=ENV["init_seed"], prec=prec)
    got = h.environments(P, o, want_p2=True)
    rho, zzh, p2h = _env_ref()
    g = got["rho1"].cpu().numpy().reshape(rho.shape)
    qubit = ~np.isnan(rho[..., 0, 0].real)
    assert int(qubit.sum()) == lat.n_qubits
    e_rho = np.abs(g - rho)[qubit].reshape(-1, 4).max(axis=1)
    z = (g[..., 0, 0] - g[..., 1, 1]).real[qubit]
    zr = (rho[..., 0, 0] - rho[..., 1, 1]).real[qubit]
    gz = got["zz_h"].cpu().numpy().reshape(zzh.shape)
    gp = got["p2_h"].cpu().numpy().reshape(p2h.shape)
    pair = ~np.isnan(zzh)
    e_h = np.abs(gz - zzh)[pair].max()
    e_p = np.abs(gp - p2h)[pair].max()
    print(f"{prec}: per-qubit rho error max {e_rho.max():.2e} median {np.median(e_rho):.2e}; "
          f"<Z> max {np.abs(z - zr).max():.2e}; zz_h {e_h:.2e}, p2_h {e_p:.2e} ({int(pair.sum())} pairs)")
    assert e_rho.max() < MARG_TOL[prec]
    assert e_h < MARG_TOL[prec] and e_p < MARG_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3"])
def test_c3_first_rows_at_chi_x_64(state, prec):
    import torch
    import paper_2507_11424_amd as tnb
    h, lat, T = state
    nq = lat.n_qubits
    n = 18
    u = sample_uniforms(43, n, nq)
    ug = sample_uniforms(ROWS["uniforms_seed"], len(ROWS["samples"]), nq)
    for k, s in enumerate(ROWS["samples"]):
        u[s["index"]] = ug[k]
    P = tnb.Peps.from_numpy(lat, T, dtype="c128" if prec == "fp64" else "c64")
    o = tnb.make_opts(chi=ROWS["chi"], chi_x=ROWS["chi_x"], sweeps=ROWS["sweeps"], init_seed=ROWS["init_seed"],
                      prec=prec)
    lc = torch.full((n, nq), float("nan"), dtype=torch.float64, device="cuda")
    h.test_sample_config(0, ROWS["rows_limit"], lc)
    try:
        bits, lq, lp = h.sample(P, o, n, seed=0, first=0, uniforms=torch.from_numpy(u))
    finally:
        h.test_sample_config(0, 0, None)
    bits, lq, lc = bits.cpu().numpy(), lq.cpu().numpy(), lc.cpu().numpy()
    for s in ROWS["samples"]:
        i = s["index"]
        ref_lc = np.array([np.nan if v is None else v for v in s["log_cond"]])
        drawn = ~np.isnan(ref_lc)
        n_cond = int(drawn.sum())
        e_c = np.abs(lc[i, drawn] - ref_lc[drawn])
        e_q = abs(lq[i] - s["log_q"])
        print(f"{prec} sample {i}: {n_cond} conditionals, max error {e_c.max():.2e}, log q error {e_q:.2e}")
        assert np.array_equal(bits[i], np.array(s["bits"], dtype=np.uint8))
        assert np.all(np.isnan(lc[i, ~drawn]))
        assert e_c.max() < COND_TOL[prec]
        assert e_q < COND_TOL[prec] * (1.0 if prec == "fp64" else math.sqrt(n_cond))
