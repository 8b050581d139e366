"""Independent check of sampled bitstrings and sample-quality metrics (FP64 oracle).

Methods, sampling paragraphs: besides q(x), every sample x gets its own
p(x) = |<x|psi>|^2 from a separate contraction of the single-layer network
<x|psi> row by row, with a boundary MPS whose bond is chosen independently of
the sampling bond (the paper uses twice the PEPS bond dimension).  The ratios
w(x) = p(x)/q(x) then give:

* the norm estimate N = (1/n) sum_i w(x_i), unbiased for <psi|psi> under q
  (Methods, the equation following the p/q paragraph);
* the sample KL divergence E_q[log q(x)/p(x)] (Methods, Eq. kld), read with p
  divided by the norm Z of the boundary contraction so that both sides are
  distributions;
* importance-sampled expectation values of diagonal observables (Appendix,
  importance-sampling formula), read as the self-normalised form
  sum_i w_i O(x_i) / sum_i w_i (the printed formula's sum and prefactor do not
  match; this is the form whose limit is <psi|O|psi>/<psi|psi>).

Test infrastructure only.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import TAG_INIT_VERIFY
from .sampler import fit_single

ein = lambda expr, *ops: np.einsum(expr, *ops, optimize=True)  # noqa: E731


def amplitude(tensors, site_index, bits, chi_v: int, sweeps: int = 2, init_seed: int = 0, sample: int = 0,
              force_fit: bool = False):
    """<x|psi> for one bitstring ``bits`` (indexed by qubit) by boundary MPSs of
    bond <= chi_v from the top row down: m <- fit(m . X_b) with X_b the row
    projected on x_b, and the last row contracted exactly against m.
    Returns (log p(x) = 2 log|<x|psi>|, arg <x|psi>)."""
    rows, cols = len(tensors), len(tensors[0])
    m = [np.ones((1, 1, 1), dtype=np.complex128) for _ in range(cols)]
    mlog = 0.0
    for r in range(rows):
        row = tensors[r]
        X = []
        for c in range(cols):
            A = row[c]
            x = 0 if A.shape[0] == 1 else int(bits[int(site_index[r][c])])
            X.append(A[x])  # [u, l, d, r]
        if r < rows - 1:
            m, lg = fit_single(m, X, chi_v, sweeps, init_seed, r, sample, force_fit, tag=TAG_INIT_VERIFY)
            mlog += lg
        else:
            v = np.ones((1, 1), dtype=np.complex128)
            for mc, Xc in zip(m, X):
                v = ein("ah,auA,uhH->AH", v, mc, Xc[:, :, 0, :])
            amp = complex(v.reshape(()))
            if amp == 0:
                return -math.inf, 0.0
            return 2.0 * (mlog + math.log(abs(amp))), math.atan2(amp.imag, amp.real)
    raise ValueError("empty lattice")


def amplitudes(tensors, site_index, bits, chi_v: int, sweeps: int = 2, init_seed: int = 0, first: int = 0,
               force_fit: bool = False):
    """``amplitude`` for every row of ``bits`` [n][N]; sample index first + i
    selects the Philox counter of the initial guesses.  Returns (log_p [n], arg [n])."""
    n = bits.shape[0]
    lp = np.zeros(n)
    ar = np.zeros(n)
    for i in range(n):
        lp[i], ar[i] = amplitude(tensors, site_index, bits[i], chi_v, sweeps, init_seed, first + i, force_fit)
    return lp, ar


def sample_stats(log_q, log_p, log_Z: float, bits=None):
    """Sample-quality metrics from per-sample log q and log p (natural logs).

    Returns a dict with
      log_norm_est  log of N = (1/n) sum_i p_i/q_i (the ratios are scaled by their
                    largest value before summing so that exp stays in range);
      kld           (1/n) sum_i [log q_i - (log p_i - log Z)];
      ess           (sum w)^2 / sum w^2 for w = p/q, the effective sample size;
      z_is          (if bits [n][N] is given) sum_i w_i (1 - 2 x_iq) / sum_i w_i
                    for every qubit q, the importance-sampled <Z_q>."""
    log_q = np.asarray(log_q, dtype=np.float64)
    log_p = np.asarray(log_p, dtype=np.float64)
    n = log_q.shape[0]
    lw = log_p - log_q
    top = float(np.max(lw))
    w = np.exp(lw - top)
    out = {
        "log_norm_est": top + math.log(float(np.sum(w)) / n),
        "kld": float(np.sum(log_q - (log_p - log_Z))) / n,
        "ess": float(np.sum(w)) ** 2 / float(np.sum(w * w)),
    }
    if bits is not None:
        zs = 1.0 - 2.0 * np.asarray(bits, dtype=np.float64)
        out["z_is"] = (w @ zs) / float(np.sum(w))
    return out
