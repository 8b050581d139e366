"""Writes the stored expected values of the full-size parity tests.

Calls only the FP64 oracle (``oracle/``) on the seeded inputs of
``peps_inputs``; nothing here touches the GPU library.  Run from the repo root:

    python tests/golden/make_golden.py c3_norm       # ~10 min on 8 cores
    python tests/golden/make_golden.py c3_samples    # a few samples at chi_x = 8
    python tests/golden/make_golden.py c2_env        # 8x8 D=4 environments at chi = 32
    python tests/golden/make_golden.py c2_env64      # the same at chi = 64 (~10 min)
    python tests/golden/make_golden.py c2_samples64  # 3 samples of c2 at chi = chi_x = 64
    python tests/golden/make_golden.py c4_small      # c4's lattice at chi = 16: norm, 2 samples with the SVD cutoff
    python tests/golden/make_golden.py c3_rows       # first 4 sampled rows at chi_x = 64 (~1 h)
    python tests/golden/make_golden.py c3_env        # c3 one-site and horizontal marginals at chi = 64
    python tests/golden/make_golden.py c3_bp         # c3 belief propagation and loop errors (~1 min)
"""
import json
import math

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from peps_inputs import make_config, sample_uniforms  # noqa: E402
import oracle  # noqa: E402
from oracle import boundary as ob  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def c3_norm():
    lat, T, cfg = make_config("c3")
    t0 = time.time()
    below, logs, info = ob.boundary_set(T, 64, 2, 0, 0)
    z = ob.close_row(T[0], below[0])
    out = dict(config="c3", chi=64, sweeps=2, init_seed=0, direction=0,
               log_abs_Z=sum(logs) + math.log(abs(z)), arg_Z=math.atan2(z.imag, z.real),
               row_logs=logs, modes=[i["mode"] if i else None for i in info],
               oracle_seconds=time.time() - t0,
               command="python tests/golden/make_golden.py c3_norm")
    json.dump(out, open(os.path.join(HERE, "c3_norm.json"), "w"), indent=1)
    print(out)


def c3_samples(n=2, chi_x=8):
    lat, T, cfg = make_config("c3")
    t0 = time.time()
    below, logs, info = ob.boundary_set(T, 64, 2, 0, 0)
    u = sample_uniforms(31, n, lat.n_qubits)
    bits, lq, lp = oracle.sample(T, lat.site_index, 64, chi_x, n, seed=0, first=0, uniforms=u, below=below)
    out = dict(config="c3", chi=64, chi_x=chi_x, sweeps=2, init_seed=0, uniforms_seed=31, n=n,
               bits=bits.tolist(), log_q=lq.tolist(), log_p=lp.tolist(), oracle_seconds=time.time() - t0,
               command=f"python tests/golden/make_golden.py c3_samples")
    json.dump(out, open(os.path.join(HERE, "c3_samples_chix8.json"), "w"), indent=1)
    print({k: v for k, v in out.items() if k != "bits"})


def c2_env(chi=32):
    lat, T, cfg = make_config("c2")
    t0 = time.time()
    e = oracle.environments(T, chi)
    enc = lambda a: [[float(v.real), float(v.imag)] for v in a.reshape(-1)]  # noqa: E731
    out = dict(config="c2", chi=chi, sweeps=2, init_seed=0,
               rho1=enc(e["rho1"]), rho1_shape=list(e["rho1"].shape),
               zz_h=[float(v) for v in e["zz_h"].reshape(-1)], zz_h_shape=list(e["zz_h"].shape),
               zz_v=[float(v) for v in e["zz_v"].reshape(-1)], zz_v_shape=list(e["zz_v"].shape),
               oracle_seconds=time.time() - t0,
               command="python tests/golden/make_golden.py " + ("c2_env" if chi == 32 else f"c2_env{chi}"))
    json.dump(out, open(os.path.join(HERE, f"c2_env_chi{chi}.json"), "w"))
    print({k: v for k, v in out.items() if k in ("config", "chi", "oracle_seconds")})


def c2_samples(n=3, chi=64):
    """Samples of the 8x8 D=4 lattice at chi = chi_x = 64 on stored uniforms."""
    lat, T, cfg = make_config("c2")
    t0 = time.time()
    u = sample_uniforms(53, n, lat.n_qubits)
    bits, lq, lp = oracle.sample(T, lat.site_index, chi, chi, n, seed=0, first=0, uniforms=u)
    out = dict(config="c2", chi=chi, chi_x=chi, sweeps=2, init_seed=0, uniforms_seed=53, n=n,
               bits=bits.tolist(), log_q=lq.tolist(), log_p=lp.tolist(), oracle_seconds=time.time() - t0,
               command="python tests/golden/make_golden.py c2_samples64")
    json.dump(out, open(os.path.join(HERE, f"c2_samples_chi{chi}.json"), "w"))
    print({k: v for k, v in out.items() if k != "bits"})


def c4_small(chi=16, chi_x=16, cutoff=1e-8, chi_x_min=4, n=2):
    """The batching workload's lattice (105-qubit rotated square in a 15 x 15
    grid with dummy sites, D = 8) at a reduced boundary bond: the norm and two
    samples with the adaptive amplitude bond (SVD cutoff, clamped to
    [chi_x_min, chi_x]) on stored uniforms, with the kept bond of every row."""
    lat, T, cfg = make_config("c4")
    t0 = time.time()
    below, logs, info = ob.boundary_set(T, chi, 2, 0, 0)
    z = ob.close_row(T[0], below[0])
    t1 = time.time()
    u = sample_uniforms(67, n, lat.n_qubits)
    used = np.zeros((n, lat.rows), dtype=np.int64)
    bits, lq, lp = oracle.sample(T, lat.site_index, chi, chi_x, n, seed=0, first=0, uniforms=u, below=below,
                                 svd_cutoff=cutoff, chi_x_min=chi_x_min, chi_used=used)
    out = dict(config="c4", chi=chi, chi_x=chi_x, svd_cutoff=cutoff, chi_x_min=chi_x_min, sweeps=2, init_seed=0,
               log_abs_Z=sum(logs) + math.log(abs(z)), arg_Z=math.atan2(z.imag, z.real), uniforms_seed=67, n=n,
               bits=bits.tolist(), log_q=lq.tolist(), log_p=lp.tolist(), chi_used=used.tolist(),
               boundary_seconds=t1 - t0, sample_seconds=time.time() - t1,
               command="python tests/golden/make_golden.py c4_small")
    json.dump(out, open(os.path.join(HERE, f"c4_chi{chi}_cutoff.json"), "w"))
    print({k: v for k, v in out.items() if k not in ("bits",)})


def c3_rows(chi_x=64, rows_limit=4, indices=(0, 17)):
    """The first rows of samples at the benchmark's sampling bond chi_x = 64:
    rows 0-1 sample under an exact amplitude boundary (bond 1, then 8), the fit
    after row 1 is exact (bond 64), the fit after row 2 truncates 512 -> 64, so
    row 3 samples under a fitted boundary of the benchmark's shape.  Stored:
    bits of those rows, the partial log q and every drawn qubit's
    log P(x_q | earlier qubits), for the given sample indices (each with its
    own row of stored uniforms)."""
    lat, T, cfg = make_config("c3")
    t0 = time.time()
    below, logs, info = ob.boundary_set(T, 64, 2, 0, 0)
    t1 = time.time()
    u = sample_uniforms(41, len(indices), lat.n_qubits)
    res = []
    for i, idx in enumerate(indices):
        lcv = np.full((1, lat.n_qubits), float("nan"))
        bits, lq, lp = oracle.sample(T, lat.site_index, 64, chi_x, 1, seed=0, first=idx, uniforms=u[i:i + 1],
                                     below=below, rows_limit=rows_limit, log_cond=lcv)
        lc = [None if v != v else float(v) for v in lcv[0]]
        res.append(dict(index=idx, bits=bits[0].tolist(), log_q=float(lq[0]), log_cond=lc))
        print(f"sample {idx}: log q = {lq[0]!r} ({time.time() - t1:.0f} s)", flush=True)
    out = dict(config="c3", chi=64, chi_x=chi_x, sweeps=2, init_seed=0, uniforms_seed=41,
               rows_limit=rows_limit, samples=res, boundary_seconds=t1 - t0,
               sample_seconds=time.time() - t1,
               command="python tests/golden/make_golden.py c3_rows")
    json.dump(out, open(os.path.join(HERE, "c3_rows_chix64.json"), "w"))


def c3_env(chi=64):
    """One-site density matrices and horizontal nearest-neighbour <ZZ> and
    two-site diagonals of the benchmark lattice at chi = 64 (the per-marginal
    error reference).  The vertical pairs' two-row environments are left out:
    at this size they take the oracle hours and more than 40 GB."""
    lat, T, cfg = make_config("c3")
    t0 = time.time()
    e = oracle.environments(T, chi, vertical=False)
    enc = lambda a: [[float(v.real), float(v.imag)] for v in a.reshape(-1)]  # noqa: E731
    fl = lambda a: [None if v != v else float(v) for v in a.reshape(-1)]  # noqa: E731
    out = dict(config="c3", chi=chi, sweeps=2, init_seed=0,
               rho1=enc(e["rho1"]), rho1_shape=list(e["rho1"].shape),
               zz_h=fl(e["zz_h"]), zz_h_shape=list(e["zz_h"].shape),
               p2_h=fl(e["p2_h"]), p2_h_shape=list(e["p2_h"].shape),
               oracle_seconds=time.time() - t0, command="python tests/golden/make_golden.py c3_env")
    json.dump(out, open(os.path.join(HERE, "c3_env_chi64.json"), "w"))
    print({k: v for k, v in out.items() if k in ("config", "chi", "oracle_seconds")})


def c3_bp():
    """Belief propagation on the benchmark lattice's norm network: log Z_BP and
    the loop BP error of each of its 55 six-site loops."""
    from oracle import bp as obp
    lat, T, cfg = make_config("c3")
    t0 = time.time()
    M, sweeps, delta = obp.bp_messages(T)
    lz, ph = obp.bp_log_norm(T, M)
    mean, eps, spectra, loops = obp.loop_bp_error(T, M)
    out = dict(config="c3", sweeps=sweeps, last_change=delta, log_abs_Z_bp=lz, arg_Z_bp=ph, eps=mean,
               eps_loops=[float(e) for e in eps], loop_first_sites=[[lp[0][0], lp[0][1]] for lp in loops],
               oracle_seconds=time.time() - t0, command="python tests/golden/make_golden.py c3_bp")
    json.dump(out, open(os.path.join(HERE, "c3_bp.json"), "w"), indent=1)
    print({k: v for k, v in out.items() if k not in ("eps_loops", "loop_first_sites")})


if __name__ == "__main__":
    {"c3_norm": c3_norm, "c3_samples": c3_samples, "c2_env": c2_env, "c2_env64": lambda: c2_env(64),
     "c2_samples64": c2_samples, "c4_small": c4_small, "c3_rows": c3_rows, "c3_env": c3_env, "c3_bp": c3_bp}[sys.argv[1]]()
