"""Parity at the benchmark's own shapes (144-qubit heavy-hex-shaped brick
lattice, D = 8, chi = 64, sampling bond chi_x = 64) against FP64 oracle values
stored by tests/golden/make_golden.py (the oracle needs about an hour for them):

* the first four sampled rows of two samples on stored uniforms: bits, the
  partial log q and every drawn qubit's log P(x_q | earlier qubits).  Rows 0-1
  sample under exact amplitude boundaries (bond 1 and 8), the fit after row 1
  is exact (bond 64) and the fit after row 2 truncates 512 -> 64, so row 3
  samples under a fitted boundary of the benchmark's shape.  The run draws 18
  samples in the benchmark's launch configuration (autotuned tiles, waves sized
  from free memory: 9 + 9 in FP64, 16 + 2 in the complex64 modes, so the
  transfer-matrix route, the masked steps and a ragged last wave all run) and
  compares samples 0 and 17.

Tolerances: FP64 1e-9 on log-conditionals; FP32 and bf16x6 1e-5 on every
conditional, 1e-5 sqrt(N) on a log q summing N conditionals; bf16x3 (two bf16
parts, about 2^-16 relative per product) 3e-4 on each conditional, 3e-4 sqrt(N)
on log q.
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
