"""Philox4x64-10 counter-based generator, written from its published definition
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11): ten rounds of two 64x64->128-bit multiplies with a Weyl-sequence key
schedule. Pure Python integers; no vectorisation. Test infrastructure only.

Streams used by the method (key = (seed, tag), counter = 4 words):

* tag 0 / 1: random initial guess of a norm-boundary fit (bottom-up / top-down);
  counter = (element, site, row, 0);
* tag 2: random initial guess of a conditioned-boundary fit in the sampler;
  counter = (element, site, row, sample);
* tag 3: the uniform that draws the bit of qubit q of sample i;
  counter = (q, i, 0, 0).

A 64-bit word w maps to the uniform (w >> 11) * 2^-53 in [0, 1); an initial
guess element is the complex number (2 u0 - 1) + i (2 u1 - 1) from the first
two words of one block. Both maps are exact in binary64.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B

TAG_INIT_DOWN = 0
TAG_INIT_UP = 1
TAG_INIT_SAMPLER = 2
TAG_DRAW = 3
TAG_INIT_VERIFY = 4


def philox4x64_10(counter, key):
    """One Philox4x64-10 block: 4 counter words, 2 key words -> 4 words."""
    c0, c1, c2, c3 = (int(x) & MASK64 for x in counter)
    k0, k1 = (int(x) & MASK64 for x in key)
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK64, lo1, (hi0 ^ c3 ^ k1) & MASK64, lo0
        k0 = (k0 + W0) & MASK64
        k1 = (k1 + W1) & MASK64
    return c0, c1, c2, c3


def word_to_uniform(w: int) -> float:
    return float(w >> 11) * (2.0 ** -53)


def draw_uniform(seed: int, qubit: int, sample: int) -> float:
    w = philox4x64_10((qubit, sample, 0, 0), (seed, TAG_DRAW))
    return word_to_uniform(w[0])


def init_tensor(seed: int, tag: int, row: int, site: int, sample: int, shape) -> np.ndarray:
    """Random initial-guess tensor; element e (row-major in ``shape``) comes from
    counter (e, site, row, sample)."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.complex128)
    for e in range(n):
        w = philox4x64_10((e, site, row, sample), (seed, tag))
        out[e] = complex(2.0 * word_to_uniform(w[0]) - 1.0, 2.0 * word_to_uniform(w[1]) - 1.0)
    return out.reshape(shape)


# ---------------------------------------------------------------------------
# Vectorised form of the same definition (NumPy uint64 lanes). The high word of
# a 64x64-bit product is assembled from 32-bit halves.

_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: int):
    b = np.uint64(b)
    a_lo = a & _M32
    a_hi = a >> _S32
    b_lo = b & _M32
    b_hi = b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _M32) + (hl & _M32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64_10_vec(c0, c1, c2, c3, k0: int, k1: int):
    """Philox4x64-10 over arrays of counters (broadcast); returns 4 uint64 arrays."""
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = np.broadcast_arrays(*(np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3)))
        c0, c1, c2, c3 = (x.copy() for x in (c0, c1, c2, c3))
        ka = np.uint64(k0 & MASK64)
        kb = np.uint64(k1 & MASK64)
        for _ in range(10):
            hi0, lo0 = _mulhilo(c0, M0)
            hi1, lo1 = _mulhilo(c2, M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ ka, lo1, hi0 ^ c3 ^ kb, lo0
            ka = ka + np.uint64(W0)
            kb = kb + np.uint64(W1)
    return c0, c1, c2, c3


def words_to_uniform(w: np.ndarray) -> np.ndarray:
    return (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def init_tensor_vec(seed: int, tag: int, row: int, site: int, sample: int, shape) -> np.ndarray:
    """Vectorised ``init_tensor`` (identical values)."""
    n = int(np.prod(shape))
    e = np.arange(n, dtype=np.uint64)
    w0, w1, _, _ = philox4x64_10_vec(e, site, row, sample, seed, tag)
    out = (2.0 * words_to_uniform(w0) - 1.0) + 1j * (2.0 * words_to_uniform(w1) - 1.0)
    return out.reshape(shape)


def draw_uniforms_vec(seed: int, n_qubits: int, first: int, n: int) -> np.ndarray:
    """Uniforms [n][n_qubits] for samples first..first+n-1 (stream tag 3)."""
    q = np.arange(n_qubits, dtype=np.uint64)[None, :]
    i = (np.uint64(first) + np.arange(n, dtype=np.uint64))[:, None]
    w0, _, _, _ = philox4x64_10_vec(q, i, 0, 0, seed, TAG_DRAW)
    return words_to_uniform(w0)
