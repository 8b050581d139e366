"""Sequential bitstring sampling from a PEPS with boundary MPSs (FP64 oracle).

Follows the paper's Appendix, "Sampling from a Tensor Network State", and the
sampling paragraphs of Methods:

* the norm boundaries below every row are computed once (``boundary_set``) and
  shared by all samples;
* rows are sampled top to bottom; within a row, qubit by qubit, the one-site
  reduced density matrix is formed conditioned on the incident MPSs (the
  amplitude boundary m from above, its conjugate, and the norm boundary from
  below) and on the qubits already sampled in the row, with the bra and ket
  bonds of the open site split;
* after a row is sampled, the product of m with the projected row
  X_b = x_b . psi_b is fitted to a new m of bond <= chi_x (the same one-site
  fit, single layer);
* q(x) is the product of the drawn conditionals; p(x) is taken from the last
  amplitude boundary contracted with the last projected row.

Optional adaptive bond (the per-sample SVD cutoff of the batched workloads,
not part of the paper's fixed-R_x sampler): after each fit, a left-to-right
SVD sweep over the canonical m keeps at every cut the fewest singular values
whose discarded weight sum_{j>=k} s_j^2 / sum_j s_j^2 is at most the cutoff
(the error measure of the paper's Eq. error_per_gate), clamped to
[chi_x_min, bond width] and to the numerical rank (s_j > 1e-12 s_0).  The
dropped directions stay as zero padding, so tensor shapes (and the next fit's
target bonds) do not depend on the cutoff.

Readings (listed in the design notes): P(s) = max(Re rho_ss, 0) / sum; x = 0
iff u < P(0); environments are divided by their Frobenius norm to stay in
range (probabilities are ratios, so this changes nothing); a non-finite or
non-positive marginal is an error.

Index conventions: amplitude boundary site m[a, u, a2]; sampler environments
[a, b, g, h, k] = (m bond, conj(m) bond, norm-boundary bond, ket bond, bra bond).
Test infrastructure only.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from .boundary import (plan_bonds, qr_reduced, lq_reduced, right_canonicalise, boundary_set)
from .philox import init_tensor_vec, draw_uniforms_vec, TAG_INIT_SAMPLER, TAG_INIT_DOWN

ein = lambda expr, *ops: np.einsum(expr, *ops, optimize=True)  # noqa: E731


class SamplingError(RuntimeError):
    pass


# ---------------------------------------------------------------------------
# single-layer fit: m . X_row -> new m

def apply_xrow_exact(m, X):
    """E_c[(a,h), d, (A,H)] = sum_u m[a,u,A] X[u,h,d,H]."""
    out = []
    for mc, Xc in zip(m, X):
        a, _, A = mc.shape
        _, h, d, H = Xc.shape
        E = ein("auA,uhdH->ahdAH", mc, Xc)
        out.append(E.reshape(a * h, d, A * H))
    return out


def _canonicalise_exact3(Y):
    Y = [y.copy() for y in Y]
    L = len(Y)
    for c in range(L - 1):
        sh = Y[c].shape
        Q, R = qr_reduced(Y[c].reshape(-1, sh[-1]))
        Y[c] = Q.reshape(sh[:-1] + (Q.shape[1],))
        Y[c + 1] = np.tensordot(R, Y[c + 1], axes=(1, 0))
    for c in range(L - 1, 0, -1):
        sh = Y[c].shape
        Lm, Q = lq_reduced(Y[c].reshape(sh[0], -1))
        Y[c] = Q.reshape((Q.shape[0],) + sh[1:])
        Y[c - 1] = np.tensordot(Y[c - 1], Lm, axes=(Y[c - 1].ndim - 1, 0))
    nrm = np.linalg.norm(Y[0])
    Y[0] = Y[0] / nrm
    return Y, math.log(nrm)


def fit_single(m, X, chi_x: int, sweeps: int, seed: int, row_id: int, sample: int,
               force_fit: bool = False, tag: int = TAG_INIT_SAMPLER):
    """Approximate m . X by an MPS of bond <= chi_x (one-site fit).
    Envs: L[y, a, h] (output bond, input bond, MPO bond). ``tag`` names the
    Philox stream of the random initial guess."""
    L = len(X)
    phys = [Xc.shape[2] for Xc in X]
    bond_in = [m[c].shape[2] * X[c].shape[3] for c in range(L - 1)]
    exact_ok, t = plan_bonds(phys, bond_in, chi_x)
    if exact_ok and not force_fit:
        Y, lg = _canonicalise_exact3(apply_xrow_exact(m, X))
        return Y, lg
    Y = []
    for c in range(L):
        tl = t[c - 1] if c > 0 else 1
        tr = t[c] if c < L - 1 else 1
        Y.append(init_tensor_vec(seed, tag, row_id, c, sample, (tl, phys[c], tr)))
    Y = right_canonicalise(Y)
    one = np.ones((1, 1, 1), dtype=np.complex128)

    def lpart(Le, mc, Xc):  # t[y, A, d, H]
        return ein("yah,auA,uhdH->yAdH", Le, mc, Xc)

    def rpart(Re, mc, Xc):  # t[a, h, d, Y]
        return ein("auA,uhdH,YAH->ahdY", mc, Xc, Re)

    R = [None] * (L + 1)
    R[L] = one
    for c in range(L - 1, 0, -1):
        R[c] = ein("ydY,ahdY->yah", Y[c].conj(), rpart(R[c + 1], m[c], X[c]))
    Le = [None] * (L + 1)
    Le[0] = one
    for _ in range(sweeps):
        for c in range(L - 1):
            tl = lpart(Le[c], m[c], X[c])
            N = ein("yAdH,YAH->ydY", tl, R[c + 1])
            Q, _ = qr_reduced(N.reshape(-1, N.shape[2]))
            Y[c] = Q.reshape(N.shape)
            Le[c + 1] = ein("ydY,yAdH->YAH", Y[c].conj(), tl)
        for c in range(L - 1, 0, -1):
            tr = rpart(R[c + 1], m[c], X[c])
            N = ein("yah,ahdY->ydY", Le[c], tr)
            _, Q = lq_reduced(N.reshape(N.shape[0], -1))
            Y[c] = Q.reshape(N.shape)
            R[c] = ein("ydY,ahdY->yah", Y[c].conj(), tr)
    Y[0] = ein("yah,ahdY->ydY", Le[0], rpart(R[1], m[0], X[0]))
    nrm = np.linalg.norm(Y[0])
    Y[0] = Y[0] / nrm
    return Y, math.log(nrm)


# ---------------------------------------------------------------------------
# adaptive bond: SVD truncation by discarded weight

RANK_RTOL = 1e-12


def keep_count(sv, cutoff: float, chi_min: int) -> int:
    """Number of singular values kept from ``sv`` (any order): the smallest k
    with sum of the squares beyond the k largest <= cutoff * total, at most the
    numerical rank (s > RANK_RTOL * s_max), at least min(chi_min, rank)."""
    s = np.sort(np.asarray(sv, dtype=np.float64))[::-1]
    if s.size == 0 or s[0] <= 0.0:
        return 0
    rank = int(np.count_nonzero(s > RANK_RTOL * s[0]))
    w = s * s
    total = float(np.sum(w))
    k = rank
    tail = 0.0
    # grow the discarded tail from the smallest kept value while it stays
    # within the cutoff
    for j in range(rank - 1, 0, -1):
        if tail + w[j] > cutoff * total:
            break
        tail += w[j]
        k = j
    return max(k, min(chi_min, rank))


def truncate_cutoff(m, cutoff: float, chi_min: int):
    """Left-to-right SVD truncation of an MPS m[c][a, u, A] whose sites 1..L-1
    are right-canonical (the gauge the fit and the exact product leave).  At
    cut c the site matrix (a u) x A is factorised M = U S V^H; U's first k
    columns replace site c and S V^H (first k rows) moves into site c+1; the
    other columns and rows become zeros.  Returns (m', k per cut)."""
    m = [x.copy() for x in m]
    ks = []
    for c in range(len(m) - 1):
        a, u, A = m[c].shape
        U, S, Vh = np.linalg.svd(m[c].reshape(a * u, A), full_matrices=False)
        k = keep_count(S, cutoff, chi_min)
        ks.append(k)
        Up = np.zeros((a * u, A), dtype=np.complex128)
        Up[:, :k] = U[:, :k]
        SV = np.zeros((A, A), dtype=np.complex128)
        SV[:k, :] = S[:k, None] * Vh[:k, :]
        m[c] = Up.reshape(a, u, A)
        m[c + 1] = np.tensordot(SV, m[c + 1], axes=(1, 0))
    return m, ks


# ---------------------------------------------------------------------------
# sampler environments (ket boundary m, its conjugate, norm boundary below)

def env_left(Lenv, mc, A, Bc, s: Optional[int]):
    """Absorb one column into a left environment [a,b,g,h,k]; s=None sums the
    physical index (bra = ket), an integer projects ket and bra on s."""
    t1 = ein("abghk,auA->bghkuA", Lenv, mc)
    if s is None:
        t2 = ein("bghkuA,suhdH->bgkAsdH", t1, A)
        t3 = ein("bgkAsdH,gdeG->bkAsHeG", t2, Bc)
        W = ein("bvB,svkeK->bBskeK", mc.conj(), A.conj())
        return ein("bkAsHeG,bBskeK->ABGHK", t3, W)
    t2 = ein("bghkuA,uhdH->bgkAdH", t1, A[s])
    t3 = ein("bgkAdH,gdeG->bkAHeG", t2, Bc)
    W = ein("bvB,vkeK->bBkeK", mc.conj(), A[s].conj())
    return ein("bkAHeG,bBkeK->ABGHK", t3, W)


def env_right(Renv, mc, A, Bc):
    """Absorb one column into a right environment [A,B,G,H,K] -> [a,b,g,h,k]."""
    t1 = ein("auA,ABGHK->auBGHK", mc, Renv)
    t2 = ein("auBGHK,suhdH->aBGKshd", t1, A)
    t3 = ein("aBGKshd,gdeG->aBKshge", t2, Bc)
    W = ein("bvB,svkeK->bBskeK", mc.conj(), A.conj())
    return ein("aBKshge,bBskeK->abghk", t3, W)


def _unit(x):
    n = np.linalg.norm(x)
    if not np.isfinite(n) or n == 0.0:
        raise SamplingError("environment vanished or overflowed")
    return x / n


def sample_one(tensors, site_index, below, chi_x: int, sweeps: int, init_seed: int,
               sample: int, uniforms=None, forced_bits=None, force_fit: bool = False,
               svd_cutoff: float = 0.0, chi_x_min: int = 1, chi_used=None, rows_limit=None,
               log_cond=None):
    """One sample. ``uniforms[q]`` is the uniform for qubit q; ``forced_bits``
    (optional) replaces the draw by a given bitstring (for enumerating q(x)).
    ``svd_cutoff`` > 0 adds the SVD truncation after every fit; ``chi_used``
    (optional, length rows) receives the largest kept bond of the amplitude
    boundary that conditions each row (1 for the first row).  ``rows_limit``
    (optional) stops after that many rows (bits of later rows stay 0, log q is
    the partial sum, log p is NaN); ``log_cond`` (optional, length N) receives
    log P(x_q | earlier qubits) of every drawn qubit q.
    Returns (bits, log_q, log_p_from_final_m)."""
    rows, cols = len(tensors), len(tensors[0])
    if rows_limit is not None:
        rows = min(rows, int(rows_limit))
    n_q = int(np.max(site_index)) + 1
    bits = np.zeros(n_q, dtype=np.uint8)
    logq = 0.0
    m = [np.ones((1, 1, 1), dtype=np.complex128) for _ in range(cols)]
    mlog = 0.0
    logp = float("nan")
    if chi_used is not None:
        chi_used[0] = 1
    for r in range(rows):
        row = tensors[r]
        B = below[r]
        R = [None] * (cols + 1)
        R[cols] = np.ones((1, 1, 1, 1, 1), dtype=np.complex128)
        for c in range(cols - 1, 0, -1):
            R[c] = _unit(env_right(R[c + 1], m[c], row[c], B[c]))
        Lenv = np.ones((1, 1, 1, 1, 1), dtype=np.complex128)
        xs = []
        for c in range(cols):
            A = row[c]
            if A.shape[0] == 1:
                Lenv = _unit(env_left(Lenv, m[c], A, B[c], 0))
                xs.append(0)
                continue
            q = int(site_index[r][c])
            Ls = [env_left(Lenv, m[c], A, B[c], s) for s in (0, 1)]
            Pt = [np.sum(Ls[s] * R[c + 1]) for s in (0, 1)]
            p0 = max(Pt[0].real, 0.0)
            p1 = max(Pt[1].real, 0.0)
            tot = p0 + p1
            if not (np.isfinite(tot) and tot > 0.0):
                raise SamplingError(f"non-positive marginal at sample {sample}, qubit {q}")
            P0 = p0 / tot
            if forced_bits is not None:
                x = int(forced_bits[q])
            else:
                x = 0 if uniforms[q] < P0 else 1
            px = P0 if x == 0 else p1 / tot
            logq += math.log(px) if px > 0 else -math.inf
            if log_cond is not None:
                log_cond[q] = math.log(px) if px > 0 else -math.inf
            bits[q] = x
            xs.append(x)
            Lenv = _unit(Ls[x])
        X = [row[c][xs[c]] for c in range(cols)]  # [u,h,d,H]
        if rows < len(tensors) and r == rows - 1:
            break  # stopped early: no fit for rows that are not sampled
        if r < rows - 1:
            m, lg = fit_single(m, X, chi_x, sweeps, init_seed, r, sample, force_fit)
            mlog += lg
            if svd_cutoff > 0.0:
                m, ks = truncate_cutoff(m, svd_cutoff, chi_x_min)
            else:
                ks = [mc.shape[2] for mc in m[:-1]]
            if chi_used is not None:
                chi_used[r + 1] = max(ks) if ks else 1
        else:
            # the last row has no down legs (dimension 1): m . X_last is the amplitude
            v = np.ones((1, 1), dtype=np.complex128)
            for mc, Xc in zip(m, X):
                v = ein("ah,auA,uhH->AH", v, mc, Xc[:, :, 0, :])
            amp = v.reshape(())[()]
            logp = 2.0 * (mlog + math.log(abs(amp))) if amp != 0 else -math.inf
    return bits, logq, logp


def sample(tensors, site_index, chi: int, chi_x: int, n: int, seed: int, first: int = 0,
           sweeps: int = 2, init_seed: int = 0, uniforms=None, below=None, force_fit=False,
           svd_cutoff: float = 0.0, chi_x_min: int = 1, chi_used=None, rows_limit=None, log_cond=None):
    """n samples (indices first..first+n-1). ``uniforms`` [n][N] overrides the
    Philox draws; ``chi_used`` (optional int array [n][rows]) receives the
    per-row bonds; ``rows_limit`` and ``log_cond`` (optional [n][N]) as in
    sample_one. Returns (bits [n][N] uint8, log_q [n], log_p [n])."""
    if below is None:
        below, _, _ = boundary_set(tensors, chi, sweeps, init_seed, TAG_INIT_DOWN, force_fit)
    n_q = int(np.max(site_index)) + 1
    if uniforms is None:
        uniforms = draw_uniforms_vec(seed, n_q, first, n)
    bits = np.zeros((n, n_q), dtype=np.uint8)
    lq = np.zeros(n)
    lp = np.zeros(n)
    for i in range(n):
        b, q, p = sample_one(tensors, site_index, below, chi_x, sweeps, init_seed, first + i,
                             uniforms[i], force_fit=force_fit, svd_cutoff=svd_cutoff,
                             chi_x_min=chi_x_min,
                             chi_used=None if chi_used is None else chi_used[i], rows_limit=rows_limit,
                             log_cond=None if log_cond is None else log_cond[i])
        bits[i], lq[i], lp[i] = b, q, p
    return bits, lq, lp
