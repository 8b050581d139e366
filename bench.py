#!/usr/bin/env python3
"""Benchmark: boundary-MPS contraction + sequential sampling on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
the norm <psi|psi> by boundary MPS (the stored norm boundary set), the
one-site density matrices by direct contraction, and `--samples` sequential
samples drawn from the stored set.  Inputs are resident in HBM before the
timed region.  Prints ONE JSON line.

Default workload: 12x12 heavy-hex-shaped brick lattice (144 qubits, z = 3),
bond D = 8, boundary bond chi = chi_x = 64, complex64 input tensors.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "samples/sec + boundary-contraction TFLOP/s, D=8 χ=64, FP64 vs split-BF16"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3 (fp32 accumulate)", "bf16x6": "bf16x6 (fp32 accumulate)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--prec", default="fp64", choices=list(PEAK_TFLOPS))
    ap.add_argument("--samples", type=int, default=16, help="samples per step")
    ap.add_argument("--chi", type=int, default=None)
    ap.add_argument("--chi-x", type=int, default=None)
    ap.add_argument("--svd-cutoff", type=float, default=None,
                    help="adaptive amplitude-boundary bond: discarded-weight cutoff (0 = fixed chi_x)")
    ap.add_argument("--chi-x-min", type=int, default=None)
    ap.add_argument("--no-env", action="store_true", help="leave the density matrices out of the step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the planner's heuristic tile choice instead of timing the candidates")
    ap.add_argument("--tune-cache", default="",
                    help="text file of tile choices: loaded if present, new choices appended")
    ap.add_argument("--plan-report", default="", help="write the per-shape contraction timing table here")
    ap.add_argument("--no-timing", action="store_true",
                    help="no HIP events around the launches (for counter runs; roofline.achieved is then null)")
    ap.add_argument("--compare", default="bf16x6,bf16x3",
                    help="with --prec fp64: comma-separated modes also timed on the same workload and samples "
                         "('none' for none); each reports its rate, its contraction roofline and its agreement "
                         "with fp64 and with the oracle under 'compare'")
    ap.add_argument("--replay-step", action="store_true",
                    help="after the timed steps, one more step without per-launch timing, in which the sampler "
                         "replays its captured wave graph for every full wave after the second; reported under "
                         "'graph_replay_step'")
    ap.add_argument("--cpu-full", action="store_true",
                    help="cpu_baseline also runs the oracle on the 8x8 D=4 lattice at chi=32 (norm, "
                         "environments, a few samples), all threads and one thread: several minutes")
    ap.add_argument("--simple-update", default="", choices=["", "hhx", "rotsq"],
                    help="instead of the sampling step: Heisenberg Trotter layers by simple update (tn_simple_update) "
                         "from the domain wall on this lattice (hhx: 129-qubit heavy-hex with bridge sites; rotsq: "
                         "the 105-qubit rotated square), one JSON line of its own")
    ap.add_argument("--su-D", type=int, default=16, help="bond dimension of the simple-update state")
    ap.add_argument("--su-layers", type=int, default=4, help="timed Trotter layers (one more untimed first)")
    ap.add_argument("--su-dt", type=float, default=0.1)
    ap.add_argument("--quench-R", default="",
                    help="with --quench-sample: comma-separated boundary dimensions R, each sampled in turn from "
                         "the same evolved state (default: --chi, else 8)")
    ap.add_argument("--quench-Rref", type=int, default=0,
                    help="with --quench-sample: boundary dimension of the reference norm Z in the KLD "
                         "(default: the largest R)")
    ap.add_argument("--quench-bp", default="", choices=["", "hhx", "rotsq"],
                    help="the paper's loop-correlation experiment: after each Trotter layer of the quench (simple "
                         "update at --su-D <= 16, 1 + --su-layers layers) the loop BP error of every primitive loop "
                         "(tn_bp); one JSON line of its own")
    ap.add_argument("--quench-sample", default="", choices=["", "hhx", "rotsq"],
                    help="the paper's end-to-end experiment: the Heisenberg quench by simple update (--su-D, "
                         "1 + --su-layers layers), then the norm and --samples samples from the evolved state at "
                         "R = --chi (boundary and amplitude bonds), the sample KLD and the share of samples with "
                         "the conserved magnetisation; one JSON line of its own")
    ap.add_argument("--copy-ref", type=int, default=0,
                    help="only run a plain device copy of this many bytes (HBM counter calibration)")
    return ap.parse_args()


def copy_reference(nbytes: int):
    """A plain elementwise kernel of known traffic: reads nbytes and writes
    nbytes once per launch (a shader kernel, so the HBM counters see it)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}))


COUNTER_FILE = os.path.join(ROOT, "profiles", "gett_brick12x12_D8_chi64_counters.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2507_11424_amd", "csrc", f) for f in ("gett.hip", "kernels.hpp")]


def kernel_hash() -> str:
    """sha256 of the contraction kernel's source: gett.hip and the part of
    kernels.hpp that declares its arguments, tiles and launches (from
    `struct GettArgs` to the linear-algebra section), so that edits to other
    kernels' declarations keep the counter record valid."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            text = fh.read()
        if f.endswith("kernels.hpp"):
            i = text.find(b"struct GettArgs")
            j = text.find(b"// ---------------------------------------------------------------- linear algebra")
            if i >= 0 and j > i:
                text = text[i:j]
        h.update(text)
    return h.hexdigest()


def stored_counters(workload: str) -> dict:
    """The committed rocprofv3 counter record of the contraction launches for
    this workload (HBM bytes per launch from FETCH_SIZE / WRITE_SIZE scaled by
    the copy-kernel calibration, HBM GB/s, MFMA busy fraction), if it was taken
    with the current kernel sources; else {}."""
    try:
        with open(COUNTER_FILE) as f:
            text = f.read()
    except OSError:
        return {}
    h = kernel_hash()
    for block in text.split("\n\n"):
        kv = {}
        for line in block.splitlines():
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("workload") == workload and kv.get("kernel_sources_sha256") == h:
            return kv
    return {}


GOLDEN = os.path.join(ROOT, "tests", "golden")


def oracle_reference(config: str, chi: int):
    """Stored oracle values for this workload, if any (written by
    tests/golden/make_golden.py, which calls only the FP64 oracle): log|Z| and
    the one-site density matrices of every qubit."""
    ref = {}
    try:
        with open(os.path.join(GOLDEN, f"{config}_norm.json")) as f:
            g = json.load(f)
        if g.get("chi") == chi:
            ref["log_abs_Z"] = g["log_abs_Z"]
    except (OSError, ValueError):
        pass
    try:
        import numpy as np
        with open(os.path.join(GOLDEN, f"{config}_env_chi{chi}.json")) as f:
            g = json.load(f)
        rho = np.array(g["rho1"], dtype=np.float64)
        ref["rho1"] = (rho[:, 0] + 1j * rho[:, 1]).reshape(g["rho1_shape"])
    except (OSError, ValueError, KeyError):
        pass
    return ref


def marginal_errors(env, ref, lz):
    """Largest distance of the GPU's one-site density matrices (and <Z_i>) and
    log|Z| from the stored oracle values."""
    import numpy as np
    out = {}
    if "log_abs_Z" in ref:
        out["log_abs_Z_error"] = abs(lz - ref["log_abs_Z"])
    if env is not None and "rho1" in ref:
        rho = env["rho1"].cpu().numpy().reshape(ref["rho1"].shape)
        d = np.abs(rho - ref["rho1"])
        z = (rho[..., 0, 0] - rho[..., 1, 1]).real
        zr = (ref["rho1"][..., 0, 0] - ref["rho1"][..., 1, 1]).real
        out["max_abs_rho1_error"] = float(np.nanmax(d))
        out["max_abs_z_error"] = float(np.nanmax(np.abs(z - zr)))
        out["marginals"] = int(np.count_nonzero(~np.isnan(z)))
    if out:
        out["reference"] = "FP64 oracle values stored in tests/golden"
    return out


def sample_quality(h, P, o, lat, bits):
    """Total-variation distance between the step's samples and the contracted
    marginals (after the timed steps, untimed): per qubit |f(0) - P(0)|, per
    neighbouring pair 1/2 sum_st |f(s,t) - P(s,t)| against the two-site
    diagonals of tn_environments, with the bound that shot noise alone stays
    under with probability 1 - 1e-3 over all tested marginals (k outcomes, n
    samples: 1/2 sqrt((k-1)/n) + sqrt(ln(m/delta)/(2n)), m marginals)."""
    import math
    import numpy as np
    env = h.environments(P, o, want_zz=False, want_p2=True)
    b = bits.cpu().numpy().astype(np.int64)
    n = b.shape[0]
    idx = lat.site_index
    rho = env["rho1"].cpu().numpy().reshape(lat.rows, lat.cols, 2, 2)
    one = []
    for r in range(lat.rows):
        for c in range(lat.cols):
            if idx[r, c] >= 0:
                one.append(abs(np.mean(b[:, idx[r, c]] == 0) - rho[r, c, 0, 0].real))
    two = []
    for key, dr, dc in (("p2_h", 0, 1), ("p2_v", 1, 0)):
        p2 = env[key].cpu().numpy()
        for r in range(p2.shape[0]):
            for c in range(p2.shape[1]):
                q1, q2 = idx[r, c], idx[r + dr, c + dc]
                if q1 < 0 or q2 < 0 or not np.all(np.isfinite(p2[r, c])):
                    continue
                f = np.bincount(2 * b[:, q1] + b[:, q2], minlength=4) / n
                two.append(0.5 * np.abs(f - p2[r, c]).sum())
    m = len(one) + len(two)
    bound = lambda k: 0.5 * math.sqrt((k - 1) / n) + math.sqrt(math.log(m / 1e-3) / (2 * n))  # noqa: E731
    return {"samples": n, "qubits": len(one), "pairs": len(two),
            "max_1site_tvd": float(max(one)), "mean_1site_tvd": float(np.mean(one)), "bound_1site": bound(2),
            "max_2site_tvd": float(max(two)) if two else None, "mean_2site_tvd": float(np.mean(two)) if two else None,
            "bound_2site": bound(4)}


def host_info():
    """CPU model, usable cores and the BLAS thread pool the oracle's NumPy runs on."""
    import numpy as np
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    np.dot(np.ones((4, 4)), np.ones((4, 4)))  # loads the BLAS library
    blas = []
    try:
        import threadpoolctl
        blas = [dict(api=i.get("internal_api"), threads=i.get("num_threads"), version=i.get("version"))
                for i in threadpoolctl.threadpool_info() if i.get("user_api") == "blas"]
    except Exception:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(cpu_model=model, cores_available=cores, blas=blas,
                blas_threads=blas[0]["threads"] if blas else None)


def _threads(n):
    """Context limiting the BLAS pool to n threads (None = unchanged)."""
    import contextlib
    if n is None:
        return contextlib.nullcontext()
    import threadpoolctl
    return threadpoolctl.threadpool_limits(limits=n, user_api="blas")


def oracle_run(config, chi, samples, threads):
    """The oracle on a whole workload: the norm boundary set and norm, all
    environments, and `samples` samples (Philox draws); wall times in seconds."""
    from peps_inputs import make_config
    from oracle import boundary as ob
    import oracle
    lat, T, cfg = make_config(config)
    with _threads(threads):
        t0 = time.perf_counter()
        below, logs, info = ob.boundary_set(T, chi, 2, 0, 0)
        ob.close_row(T[0], below[0])
        t1 = time.perf_counter()
        oracle.environments(T, chi)
        t2 = time.perf_counter()
        oracle.sample(T, lat.site_index, chi, chi, samples, seed=17, below=below)
        t3 = time.perf_counter()
    return dict(norm_s=t1 - t0, environments_s=t2 - t1, samples=samples, sample_s=t3 - t2,
                samples_per_s=samples / (t3 - t2), threads=threads or "all")


def cpu_baseline(lat, T, chi, chi_x, contraction_flops, full=False):
    """The FP64 oracle, as it stands, on the host cores, on a bounded sample of
    the workload: one sampler environment step (the oracle's env_right) for the
    costliest kind of site of a row, at the steady-state shapes of the workload
    (bond chi_x amplitude boundary, bond chi norm boundary; seeded stand-in
    values), and one fit site update (left partial, derivative, QR, environment
    update) for each kind of site.  Every site of a sample costs one right step
    and two projected left steps (about one full step), so a sample is
    extrapolated as 2 x (sum of the right steps over all sites); the norm as
    sweeps x 2 site updates per site per row.  Also timed: the whole 4x4 D=2
    workload (norm, environments, 200 samples) with all threads and with one;
    with full=True the 8x8 D=4 workload at chi=32 (norm, environments, 2
    samples) likewise, and the bounded sample above on one thread."""
    import numpy as np
    from oracle import boundary as ob
    from oracle import sampler as osm
    info = host_info()
    threads = info["blas_threads"] or int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
    rng = np.random.default_rng(0)
    cn = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)  # noqa: E731
    rows, cols = len(T), len(T[0])
    kinds = {}
    for r in range(1, rows - 1):
        for c in range(1, cols - 1):
            A = T[r][c]
            kinds.setdefault((A.shape[1], A.shape[3]), (r, c))
    # the sampler step is timed for the kind with the largest down bond (the costliest
    # on the GPU) and used for every kind, which understates the oracle's time
    env_kind = max(kinds, key=lambda k: (k[1], k[0]))

    def bounded(nthreads):
        t_env, t_fit = {}, {}
        with _threads(nthreads):
            for (du, dd), (r, c) in kinds.items():
                A = T[r][c]
                h, H = A.shape[2], A.shape[4]
                m = cn(chi_x, du, chi_x)
                B = cn(chi, dd, dd, chi)
                R = cn(chi_x, chi_x, chi, H, H)
                if (du, dd) == env_kind:
                    t0 = time.perf_counter()
                    osm.env_right(R, m, A, B)
                    t_env[(du, dd)] = time.perf_counter() - t0
                    print(f"cpu baseline ({nthreads or 'all'} threads): sampler env step (u={du}, d={dd}) "
                          f"{t_env[(du, dd)]:.2f} s", file=sys.stderr, flush=True)
                Le = cn(chi, chi, h, h)
                Re = cn(chi, chi, H, H)
                t0 = time.perf_counter()
                t3 = ob.left_partial(Le, B, A)
                N = np.einsum("yGuHvK,YGHK->yuvY", t3, Re, optimize=True)
                Q, _ = ob.qr_reduced(N.reshape(-1, N.shape[3]))
                np.einsum("yuvY,yGuHvK->YGHK", Q.reshape(N.shape).conj(), t3, optimize=True)
                t_fit[(du, dd)] = time.perf_counter() - t0
                print(f"cpu baseline ({nthreads or 'all'} threads): fit site update (u={du}, d={dd}) "
                      f"{t_fit[(du, dd)]:.2f} s", file=sys.stderr, flush=True)
        per_sample = 0.0
        per_norm = 0.0
        for r in range(rows):
            for c in range(cols):
                A = T[r][c]
                k = (A.shape[1], A.shape[3])
                per_sample += 2.0 * t_env[env_kind]
                per_norm += 4.0 * t_fit.get(k, 0.0) if r > 0 else 0.0
        return per_sample, per_norm, sum(t_env.values()) + sum(t_fit.values())

    per_sample, per_norm, spent = bounded(None)
    out = dict(value=1.0 / per_sample, unit="samples/s", cores=threads, kind="oracle",
               sample=(f"one sampler environment step (site kind u,d = {env_kind}, used for every site) "
                       f"and one fit site update per kind of site {sorted(kinds)} at chi={chi}, "
                       f"chi_x={chi_x}, seeded stand-in values, timed once each ({spent:.1f} s) and "
                       f"extrapolated over {rows}x{cols} sites: {per_sample:.0f} s per sample, "
                       f"{per_norm:.0f} s per norm (extrapolated)"),
               contraction_tflops=contraction_flops / per_norm / 1e12 if per_norm > 0 else None,
               host=info, full_runs={})
    for nthr in (None, 1):
        r = oracle_run("c1", 16, 200, nthr)
        out["full_runs"][f"c1 4x4 D=2 chi=16, {nthr or threads} threads"] = r
        print(f"cpu baseline: c1 oracle ({nthr or 'all'} threads) {r}", file=sys.stderr, flush=True)
    if full:
        for nthr in (None, 1):
            r = oracle_run("c2", 32, 2, nthr)
            out["full_runs"][f"c2 8x8 D=4 chi=32, {nthr or threads} threads"] = r
            print(f"cpu baseline: c2 oracle ({nthr or 'all'} threads) {r}", file=sys.stderr, flush=True)
        ps1, pn1, _ = bounded(1)
        out["single_thread"] = dict(value=1.0 / ps1, unit="samples/s", cores=1,
                                    per_sample_s=ps1, per_norm_s=pn1, note="same bounded sample, one thread")
    return out


# bf16 MFMA products issued per complex multiply-add (4 real products, each
# split into 3 or 6 bf16 products): the algorithmic ceiling is the bf16 peak
# times 8 / (2 x that count)
BF16_PRODUCTS = {"bf16x3": 12, "bf16x6": 24}


def compare_mode(a, prec, h, lat, T, chi, chi_x, cutoff, chi_x_min, step, ref_res, lz_ref, last, oref,
                 fp64_rate):
    """The same step in another precision mode (one warmup step, one timed step)
    on the same samples (same seed and indices): its rate, its boundary
    contraction rate, the roofline of its contraction launches, how far its
    log|Z|, log q and log p lie from the FP64 run's on the samples that drew the
    same bits, and how far its log|Z| and one-site marginals lie from the stored
    oracle values."""
    import torch
    import paper_2507_11424_amd as tnb

    ref_bits, ref_lq, ref_lp = ref_res
    P2 = tnb.Peps.from_numpy(lat, T, dtype="c128" if prec == "fp64" else "c64", device="cuda:0")
    o2 = tnb.make_opts(chi=chi, chi_x=chi_x, prec=prec, svd_cutoff=cutoff, chi_x_min=chi_x_min)
    tw = time.perf_counter()
    step(P=P2, o=o2)
    print(f"{prec} warmup step done in {time.perf_counter() - tw:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lz, rec = step(timing=not a.no_timing, P=P2, o=o2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"{prec} timed step done ({dt:.1f} s)", file=sys.stderr, flush=True)
    con_t, con_c = rec["contract"]
    con_f = con_c["gemm_flops"] - con_c["qr_gemm_flops"]
    g_ms = sum(c["gemm_ms"] for _, c in rec.values())
    g_fl = sum(c["gemm_flops"] for _, c in rec.values())
    g_n = sum(c["gemm_launches"] for _, c in rec.values())
    g_by = sum(c["gemm_bytes"] for _, c in rec.values())
    achieved = g_fl / (g_ms * 1e-3) / 1e12 if g_ms > 0 else None
    peak = PEAK_TFLOPS[prec]
    ceiling = peak * 8 / (2 * BF16_PRODUCTS[prec]) if prec in BF16_PRODUCTS else peak
    workload = (f"{a.config} {prec} samples={a.samples} chi={chi} chi_x={chi_x} cutoff={cutoff:g} "
                f"env={'no' if a.no_env else 'yes'}")
    ctr = stored_counters(workload)
    h.set_timing(False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h.boundary_contract(P2, o2)
    torch.cuda.synchronize()
    dt_c = time.perf_counter() - t1
    bits, lq, lp = last["res"][:3]
    same = (bits == ref_bits).all(dim=1)
    n_same = int(same.sum())
    dq = (lq - ref_lq)[same].abs()
    dp = (lp - ref_lp)[same].abs()
    out = {"prec": prec, "dtype": DTYPE[prec], "value": a.samples / dt, "unit": "samples/s",
           "ms_per_step": 1e3 * dt, "contraction_tflops": con_f / con_t / 1e12 if con_t > 0 else None,
           "contraction_untimed_tflops": con_f / dt_c / 1e12 if dt_c > 0 else None,
           "speedup_vs_fp64": a.samples / dt / fp64_rate if fp64_rate else None,
           "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                        "frac": achieved / peak if achieved else None,
                        "algorithmic_ceiling": ceiling,
                        "frac_of_ceiling": achieved / ceiling if achieved else None,
                        "ceiling_note": (f"{BF16_PRODUCTS[prec]} bf16 MFMA products per complex multiply-add "
                                         f"(4M, {BF16_PRODUCTS[prec] // 4} per real product)")
                        if prec in BF16_PRODUCTS else "the mode's own MFMA peak",
                        "kernel": "gett (all tile variants; the autotuner may run a contraction on the FP32 "
                                  "kernel in split-BF16 modes)",
                        "traffic": float(ctr["traffic_bytes_per_launch"]) if ctr else None,
                        "traffic_unit": "HBM bytes per launch (all contraction launches, masked included)",
                        "hbm_gbs_rocprof": float(ctr["hbm_gbs"]) if ctr else None,
                        "mfma_util_rocprof": float(ctr["mfma_util"]) if ctr else None,
                        "counter_workload": workload,
                        "launches_per_step": g_n,
                        "kernel_avg_us": 1e3 * g_ms / g_n if g_n and g_ms > 0 else None,
                        "algorithmic_bytes_per_launch": g_by / g_n if g_n else None,
                        "kernel_ms_per_step": g_ms},
           "log_abs_Z_minus_fp64": lz - lz_ref,
           "same_bitstrings": n_same, "samples": int(bits.shape[0]),
           "max_abs_dlog_q_vs_fp64": float(dq.max()) if n_same else None,
           "max_abs_dlog_p_vs_fp64": float(dp.max()) if n_same else None,
           "vs_oracle": marginal_errors(last.get("env"), oref, lz),
           "note": "one warmup and one timed step after the fp64 steps, same seed and sample indices; "
                   "log q and log p differences over the samples that drew the same bits"}
    return out


def simple_update_bench(a):
    """Heisenberg quench (dt, J = 1, colour-group Trotter layers, domain wall)
    by BP-gauged simple update: layers per second on the GPU, the gate errors
    and fidelity estimate, and the oracle's time per gate on the host."""
    import numpy as np
    import torch
    import paper_2507_11424_amd as tnb
    from peps_inputs import heavy_hex_lattice, rotated_square_lattice
    from peps_inputs.circuits import heisenberg_circuit, domain_wall_peps
    D = a.su_D
    lat = heavy_hex_lattice(7, 15, D) if a.simple_update == "hhx" else rotated_square_lattice(D)
    T0 = domain_wall_peps(lat)
    gates1, G = heisenberg_circuit(lat, 1, a.su_dt)
    h = tnb.Handle(0, torch.cuda.current_stream(0))
    h.set_autotune(True, None)
    P = tnb.Peps.from_numpy(lat, T0, dtype="c128", device="cuda:0")
    ngroups = len({g[0] for g in gates1})
    msgs = h.message_buffer(P)  # each layer's BP continues from the previous layer's messages

    def layer(l):
        gl = [(l * ngroups + g[0],) + tuple(g[1:]) for g in gates1]
        return h.simple_update(P, gl, G, in_place=True, messages_in=msgs if l > 0 else None, messages_out=msgs)

    t0 = time.perf_counter()
    _, eps0, _ = layer(0)
    torch.cuda.synchronize()
    warm = time.perf_counter() - t0
    print(f"warmup layer {warm:.1f} s", file=sys.stderr, flush=True)
    eps_all, ms = [], []
    t0 = time.perf_counter()
    for l in range(1, a.su_layers + 1):
        tl = time.perf_counter()
        _, eps, _ = layer(l)
        torch.cuda.synchronize()
        ms.append(1e3 * (time.perf_counter() - tl))
        eps_all.extend(eps.tolist())
        print(f"layer {l}: {ms[-1]:.0f} ms, max eps {max(eps):.2e}", file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    c = h.counters()
    out = {"metric": "simple-update Trotter layers/sec (Heisenberg quench, BP-gauged)",
           "value": a.su_layers / dt, "unit": "layers/s", "n_gpus": 1, "steps": a.su_layers, "warmup": 1,
           "ms_per_step": 1e3 * dt / a.su_layers, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{lat.name}: {lat.n_qubits} qubits, D={D}, dt={a.su_dt}, J=1, "
                                  f"{len(gates1)} gates in {ngroups} colour groups per layer, domain wall",
                      "gates_per_layer": len(gates1)},
           "gates_per_s": len(gates1) * a.su_layers / dt,
           "layer_ms": ms,
           "eps_max": max(eps_all), "eps_mean": float(np.mean(eps_all)),
           "fidelity_estimate_timed_layers": float(np.prod([1 - e for e in eps_all])),
           "layers_total": a.su_layers + 1,
           "fidelity_estimate_all_layers": float(np.prod([1 - e for e in list(eps0) + eps_all])),
           "last_layer_launches": {"contraction": c["gemm_launches"], "orthonormalisation": c["qr_launches"]},
           "roofline": {"bound": "latency", "note": "per colour group a BP solve, then per class of gates "
                                                    "(same orientation and site shapes) a few tens of batched "
                                                    "launches on D-sized tensors (gauge, QR, Jacobi SVD of at most "
                                                    "4D x 4D per gate, ungauge); no kernel here is near an MFMA "
                                                    "or HBM bound"}}
    if not a.no_cpu_baseline and (D <= 16 or a.cpu_full):
        from oracle.circuit import simple_update as o_su
        n = 4
        print(f"cpu baseline: the oracle on the first {n} gates (one BP solve at D={D})", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        o_su(T0, gates1[:n], G)
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n / tc, "unit": "gates/s (first gates of layer 1, incl. one BP solve)",
                               "cores": os.cpu_count(), "kind": "oracle",
                               "sample": f"the oracle's simple update on the first {n} gates of the first layer"}
    elif not a.no_cpu_baseline:
        out["cpu_baseline"] = None
        out["cpu_baseline_note"] = (f"at D={D} one BP solve of the oracle takes minutes on the host; --cpu-full "
                                    "runs it")
    print(json.dumps(out))
    h.close()


def quench_bp_bench(a):
    """Loop correlations of the evolving quench state (the paper's loop BP
    error per Trotter layer, Eqs. avBPError and loopBPerror): after every layer
    of the simple update, BP on the norm network and the error of every
    primitive loop; the mean, the largest and the BP solve's time per layer."""
    import numpy as np
    import torch
    import paper_2507_11424_amd as tnb
    from peps_inputs import heavy_hex_lattice, rotated_square_lattice
    from peps_inputs.circuits import heisenberg_circuit, domain_wall_peps
    D = a.su_D
    lat = heavy_hex_lattice(7, 15, D) if a.quench_bp == "hhx" else rotated_square_lattice(D)
    gates1, G = heisenberg_circuit(lat, 1, a.su_dt)
    ngroups = len({g[0] for g in gates1})
    layers = a.su_layers + 1
    h = tnb.Handle(0, torch.cuda.current_stream(0))
    P = tnb.Peps.from_numpy(lat, domain_wall_peps(lat), dtype="c128", device="cuda:0")
    msgs = h.message_buffer(P)
    rows, eps_all = [], []
    t_su = t_bp = 0.0
    for l in range(layers):
        gl = [(l * ngroups + g[0],) + tuple(g[1:]) for g in gates1]
        t0 = time.perf_counter()
        _, eps, _ = h.simple_update(P, gl, G, in_place=True, messages_in=msgs if l > 0 else None, messages_out=msgs)
        torch.cuda.synchronize()
        t_su += time.perf_counter() - t0
        eps_all.extend(eps.tolist())
        t0 = time.perf_counter()
        b = h.bp(P, loops=True)
        t_bp += time.perf_counter() - t0
        el = b["eps_loops"]
        rows.append({"layer": l + 1, "eps_mean": b["eps"], "eps_max": float(np.max(el)), "loops": int(el.size),
                     "bp_sweeps": b["sweeps"], "fidelity_estimate": float(np.prod([1 - e for e in eps_all]))})
        print(f"layer {l + 1}: loop BP error mean {b['eps']:.3e} max {np.max(el):.3e} over {el.size} loops "
              f"({b['sweeps']} sweeps)", file=sys.stderr, flush=True)
    out = {"metric": "loop BP error per Trotter layer (evolved Heisenberg quench state)",
           "value": layers / (t_su + t_bp), "unit": "layers/s (simple update + BP with loop errors)",
           "n_gpus": 1, "steps": layers, "warmup": 0, "ms_per_step": 1e3 * (t_su + t_bp) / layers,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{lat.name}: {lat.n_qubits} qubits, Heisenberg quench dt={a.su_dt} J=1 from the "
                                  f"domain wall, {layers} layers by simple update at D={D}, loop BP error after each"},
           "simple_update_s": t_su, "bp_s": t_bp, "layers": rows}
    print(json.dumps(out))
    h.close()


def quench_sample_bench(a):
    """Evolve the domain wall by simple update, then contract and sample the
    evolved state with boundary MPSs of dimension R (the paper's heavy-hex and
    Willow sampling experiments): samples/s, KLD against p / Z, and the share
    of samples whose number of 1s equals the domain wall's (the Heisenberg
    layers conserve it)."""
    import numpy as np
    import torch
    import paper_2507_11424_amd as tnb
    from peps_inputs import heavy_hex_lattice, rotated_square_lattice
    from peps_inputs.circuits import heisenberg_circuit, domain_wall_peps, domain_wall_ones
    D, R = a.su_D, a.chi or 8
    n = a.samples
    lat = heavy_hex_lattice(7, 15, D) if a.quench_sample == "hhx" else rotated_square_lattice(D)
    gates1, G = heisenberg_circuit(lat, 1, a.su_dt)
    ngroups = len({g[0] for g in gates1})
    layers = a.su_layers + 1
    h = tnb.Handle(0, torch.cuda.current_stream(0))
    h.set_autotune(not a.no_autotune, a.tune_cache or None)
    P = tnb.Peps.from_numpy(lat, domain_wall_peps(lat), dtype="c128", device="cuda:0")
    msgs = h.message_buffer(P)
    eps_all = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for l in range(layers):
        gl = [(l * ngroups + g[0],) + tuple(g[1:]) for g in gates1]
        _, eps, _ = h.simple_update(P, gl, G, in_place=True, messages_in=msgs if l > 0 else None, messages_out=msgs)
        eps_all.extend(eps.tolist())
        print(f"layer {l}: max eps {max(eps):.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_su = time.perf_counter() - t0
    Ps = P if a.prec == "fp64" else tnb.Peps(lat, [t.to(torch.complex64) for t in P.tensors])
    want = domain_wall_ones(lat)
    Rs = [int(x) for x in a.quench_R.split(",")] if a.quench_R else [R]
    # references: Z from the boundary contraction at the largest R, p(x) certified by the separate
    # amplitude contraction at bond 2D (the paper's check)
    R_ref = a.quench_Rref or max(Rs)
    t0 = time.perf_counter()
    lz_ref, _ = h.boundary_contract(P, tnb.make_opts(chi=R_ref, chi_x=R_ref))
    t_ref = time.perf_counter() - t0
    o_amp = tnb.make_opts(chi=2 * D, chi_x=2 * D)
    bp_z = h.bp(P, loops=False)["log_abs_Z"]
    print(f"reference log|Z| at R={R_ref}: {lz_ref:.8f} ({t_ref:.1f} s); BP log|Z_BP| {bp_z:.8f}",
          file=sys.stderr, flush=True)
    runs = []
    for R in Rs:
        o = tnb.make_opts(chi=R, chi_x=R, prec=a.prec)
        t0 = time.perf_counter()
        lz, _ = h.boundary_contract(Ps, o)
        torch.cuda.synchronize()
        t_norm = time.perf_counter() - t0
        h.sample(Ps, o, min(n, 2), seed=11)  # warm-up: tile choices and plans
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bits, lq, lp = h.sample(Ps, o, n, seed=11)[:3]
        torch.cuda.synchronize()
        t_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        lp_c = h.amplitude(P, o_amp, bits)
        torch.cuda.synchronize()
        t_amp = time.perf_counter() - t0
        st = h.sample_stats(lq, lp_c, lz_ref)
        ones = bits.to(torch.int64).sum(dim=1).cpu().numpy()
        r = (lp_c - lq - lz_ref).cpu().numpy()  # log (p(x) / Z q(x))
        runs.append({"R": R, "norm_s": t_norm, "log_abs_Z": lz, "samples_per_s": n / t_s, "kld": st["kld"],
                     "ess": st["ess"], "log_norm_estimate": st["log_norm_est"],
                     "share_correct_magnetisation": float(np.mean(ones == want)),
                     "log10_p_over_Zq_range": [float(r.min() / np.log(10)), float(r.max() / np.log(10))],
                     "max_abs_sampler_log_p_vs_certified": float((lp - lp_c).abs().max()),
                     "certify_s": t_amp})
        print(f"R={R}: norm {t_norm:.1f} s, {n} samples {t_s:.1f} s, KLD {st['kld']:.3e}, "
              f"correct magnetisation {runs[-1]['share_correct_magnetisation']:.3f}", file=sys.stderr, flush=True)
    last = runs[-1]
    out = {"metric": "samples/sec (evolved Heisenberg quench state, boundary-MPS sampler)",
           "value": last["samples_per_s"], "unit": "samples/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": 1e3 * n / last["samples_per_s"], "higher_is_better": True, "dtype": DTYPE[a.prec],
           "data": "synthetic",
           "config": {"workload": f"{lat.name}: {lat.n_qubits} qubits, Heisenberg quench dt={a.su_dt} J=1 from the "
                                  f"domain wall, {layers} layers by simple update at D={D}, then norm and {n} "
                                  f"samples per R in {Rs} (value: R={last['R']})"},
           "simple_update_s": t_su, "fidelity_estimate": float(np.prod([1 - e for e in eps_all])),
           "magnetisation_ones": want, "reference_log_abs_Z": lz_ref, "reference_R": R_ref,
           "bp_log_abs_Z": bp_z, "certified_p_bond": 2 * D,
           "note": "kld = mean(log q - log p + log Z) with p from tn_amplitude at bond 2D and Z from the "
                   "boundary contraction at the largest R",
           "runs": runs}
    print(json.dumps(out))
    h.close()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if a.copy_ref:
        copy_reference(a.copy_ref)
        return
    if a.simple_update:
        simple_update_bench(a)
        return
    if a.quench_sample:
        quench_sample_bench(a)
        return
    if a.quench_bp:
        quench_bp_bench(a)
        return
    import numpy as np
    import torch
    import paper_2507_11424_amd as tnb
    from peps_inputs import make_config

    lat, T, cfg = make_config(a.config)
    chi = a.chi or cfg["chi"]
    chi_x = a.chi_x or cfg["chi_x"]
    dtype = "c64" if cfg["dtype"] == "c64" else "c128"
    dev_dtype = "c128" if a.prec == "fp64" else "c64"
    stream = torch.cuda.current_stream(0)
    h = tnb.Handle(0, stream)
    # tile configurations are timed on each new contraction shape during warmup
    h.set_autotune(not a.no_autotune, a.tune_cache or None)
    # inputs resident in HBM before timing (stored as the configured type, computed in the mode's type)
    P = tnb.Peps.from_numpy(lat, T, dtype=dev_dtype, device="cuda:0")
    cutoff = a.svd_cutoff if a.svd_cutoff is not None else cfg.get("svd_cutoff", 0.0)
    chi_x_min = a.chi_x_min or cfg.get("chi_x_min", 1)
    o = tnb.make_opts(chi=chi, chi_x=chi_x, prec=a.prec, svd_cutoff=cutoff, chi_x_min=chi_x_min)
    used = []

    phases = ("contract", "environments", "sample")

    last = {}

    def step(timing=False, P=P, o=o):
        """One pass of the hot path; returns log|Z| and per-phase (seconds, counters)."""
        h.set_timing(timing)
        rec = {}
        t0 = time.perf_counter()
        lz, _ = h.boundary_contract(P, o)
        rec["contract"] = (time.perf_counter() - t0, h.counters())
        print(f"  contract done ({rec['contract'][0]:.1f} s)", file=sys.stderr, flush=True)
        if not a.no_env:
            # one-site marginals of every qubit (pairs are left out at this size)
            t0 = time.perf_counter()
            last["env"] = h.environments(P, o, want_zz=False, want_p2=False)
            torch.cuda.synchronize()
            rec["environments"] = (time.perf_counter() - t0, h.counters())
            print(f"  environments done ({rec['environments'][0]:.1f} s)", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        res = h.sample(P, o, a.samples, seed=17, want_chi=cutoff > 0)
        torch.cuda.synchronize()
        if cutoff > 0:
            used.append(res[3][:, 1:].float())
        rec["sample"] = (time.perf_counter() - t0, h.counters())
        last["res"] = res
        return lz, rec

    for i in range(a.warmup):
        tw = time.perf_counter()
        step()
        print(f"warmup step {i} done in {time.perf_counter() - tw:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    # the contraction kernel's device time comes from HIP events recorded on the
    # handle's stream around every launch inside the timed steps (no host waits
    # between launches; the events are read when each call returns)
    t0 = time.perf_counter()
    acc = {k: [0.0, 0.0] for k in phases}
    gemm_ms = gemm_flops = qr_ms = qr_gemm_flops = masked_ms = gemm_bytes = 0.0
    launches = masked = graphs = 0
    for i in range(a.steps):
        lz, rec = step(timing=not a.no_timing)
        for k, (sec, c) in rec.items():
            acc[k][0] += sec
            acc[k][1] += c["gemm_flops"] - c["qr_gemm_flops"]
            gemm_ms += c["gemm_ms"]
            gemm_flops += c["gemm_flops"]
            qr_ms += c["qr_ms"]
            qr_gemm_flops += c["qr_gemm_flops"]
            launches += c["gemm_launches"]
            masked += c["masked_launches"]
            masked_ms += c["masked_ms"]
            gemm_bytes += c["gemm_bytes"]
            graphs += c["graph_launches"]
        print(f"timed step {i} done ({time.perf_counter() - t0:.1f} s so far)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h.set_timing(False)
    if a.plan_report:
        with open(a.plan_report, "w") as f:
            f.write(h.plan_report(40))
    gemm_ms /= a.steps
    gemm_flops /= a.steps
    qr_ms /= a.steps
    qr_gemm_flops /= a.steps
    launches //= a.steps
    masked //= a.steps
    masked_ms /= a.steps
    gemm_bytes /= a.steps
    achieved = gemm_flops / (gemm_ms * 1e-3) / 1e12 if gemm_ms > 0 else None
    samples = a.samples * a.steps
    con_t, con_f = acc["contract"]
    workload = (f"{a.config} {a.prec} samples={a.samples} chi={chi} chi_x={chi_x} cutoff={cutoff:g} "
                f"env={'no' if a.no_env else 'yes'}")
    ctr = stored_counters(workload)
    out = {
        "metric": METRIC,
        "value": samples / dt,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.prec],
        "data": "synthetic",
        "config": {"workload": f"{a.config}: {lat.name}, {lat.n_qubits} qubits, chi={chi}, "
                               f"chi_x={chi_x}{' (max, SVD cutoff %g)' % cutoff if cutoff > 0 else ''}, "
                               f"{cfg['dtype']} input, {a.samples} samples per step",
                   "samples_per_step": a.samples, "prec": a.prec, "autotune": not a.no_autotune},
        "contraction_tflops": con_f / con_t / 1e12 if con_t > 0 else None,
        "phases": {k: {"ms_per_step": 1e3 * v[0] / a.steps, "tflop_per_step": v[1] / a.steps / 1e12,
                       "tflops": v[1] / v[0] / 1e12 if v[0] > 0 else None} for k, v in acc.items()},
        "log_abs_Z": lz,
        "sampler_waves_replayed_per_step": graphs / a.steps,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[a.prec], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS[a.prec] if achieved else None,
                     "traffic": float(ctr["traffic_bytes_per_launch"]) if ctr else None,
                     "traffic_unit": "HBM bytes per launch (all contraction launches, masked included)",
                     "hbm_gbs_rocprof": float(ctr["hbm_gbs"]) if ctr else None,
                     "mfma_util_rocprof": float(ctr["mfma_util"]) if ctr else None,
                     "algorithmic_bytes_per_launch": gemm_bytes / launches if launches else None,
                     "kernel": "gett (complex contraction engine, all tile variants, with its split-K "
                               "reduction)",
                     "launches_per_step": launches,
                     "kernel_avg_us": 1e3 * gemm_ms / launches if launches and gemm_ms > 0 else None,
                     "algorithmic_flops_per_step": gemm_flops,
                     "algorithmic_bytes_per_step": gemm_bytes,
                     "counter_workload": workload,
                     "of_which_orthonormalisation_flops": qr_gemm_flops,
                     "kernel_ms_per_step": gemm_ms,
                     "qr_ms_per_step": qr_ms,
                     "masked_launches_per_step": masked,
                     "masked_ms_per_step": masked_ms,
                     "masked_note": "launches that extend a qubit's environment by its less likely bit only for "
                                    "the samples that drew that bit (other tiles skipped); excluded from "
                                    "achieved, flops and launches"},
    }
    if cutoff > 0:
        cu = torch.cat(used)
        out["config"]["svd_cutoff"] = cutoff
        out["config"]["chi_x_min"] = chi_x_min
        vals, counts = torch.unique(cu.to(torch.int64).flatten(), return_counts=True)
        out["chi_x_used"] = {"mean": float(cu.mean()), "min": int(cu.min()), "max": int(cu.max()),
                             "histogram": {str(int(v)): int(c) for v, c in zip(vals.cpu(), counts.cpu())},
                             "note": "largest kept bond per row (rows 1..) of each sample's amplitude boundary"}
    n_cfg = int(cfg.get("n_samples", 0))
    if n_cfg > a.samples:
        out["configured_samples"] = n_cfg
        out["projected_total_s"] = n_cfg / out["value"]
        out["projected_note"] = (f"time-boxed prefix: {a.samples} samples per step timed; the configured "
                                 f"{n_cfg} samples would take n / value at this rate")
    # the contraction once more without per-launch events (the timed steps
    # record an event pair around every launch, which drains the queue between
    # the short launches of the fit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.boundary_contract(P, o)
    torch.cuda.synchronize()
    dt_c = time.perf_counter() - t0
    out["contraction_untimed"] = {"tflops": con_f / a.steps / dt_c / 1e12 if dt_c > 0 else None,
                                  "ms": 1e3 * dt_c,
                                  "note": "one boundary contraction after the timed steps, without per-launch "
                                          "HIP events (contraction_tflops is measured inside the timed steps, "
                                          "with them)"}
    if a.replay_step:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rec = step(timing=False)
        torch.cuda.synchronize()
        dt_r = time.perf_counter() - t0
        out["graph_replay_step"] = {"value": a.samples / dt_r, "unit": "samples/s", "ms": 1e3 * dt_r,
                                    "waves_replayed": rec["sample"][1]["graph_launches"],
                                    "note": "one step without per-launch event timing (timed steps issue every "
                                            "launch from the host so that each is timed)"}
    oref = oracle_reference(a.config, chi) if cutoff == 0 else {}
    out["vs_oracle"] = marginal_errors(last.get("env"), oref, lz)
    if a.samples >= 1000 and not a.no_env:
        out["sample_quality"] = sample_quality(h, P, o, lat, last["res"][0])
    modes = [m for m in a.compare.split(",") if m and m != "none" and m != a.prec]
    if a.prec == "fp64" and modes:
        ref_res = tuple(x.clone() for x in last["res"][:3])
        out["compare"] = [compare_mode(a, m, h, lat, T, chi, chi_x, cutoff, chi_x_min, step, ref_res, lz, last,
                                       oref, out["value"]) for m in modes]
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(lat, T, chi, chi_x, con_f / a.steps, full=a.cpu_full)
    print(json.dumps(out))
    h.close()


if __name__ == "__main__":
    main()
