"""Numerics of the HIP engine primitives through the C ABI test hooks:
the complex contraction kernel in every precision against a float64 NumPy
einsum, and the FP64 Householder QR (orthogonality, reconstruction, triangular R)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 3e-6, "bf16x3": 3e-5, "bf16x6": 3e-6}


@pytest.fixture(scope="module")
def handle():
    import paper_2507_11424_amd as tnb
    h = tnb.Handle(0)
    yield h
    h.close()


def _rand(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


CASES = [
    # (A letters, B letters, C letters, dims) -- shapes span several tiles and ragged tails
    ("ik", "kj", "ij", dict(i=130, k=70, j=97)),
    ("ik", "kj", "ji", dict(i=130, k=70, j=97)),          # output contiguous along M (swap path)
    ("yghk", "gdeG", "yhkdeG", dict(y=9, g=7, h=3, k=3, d=2, e=2, G=11)),
    ("ykeGsuH", "svkeK", "yGuHvK", dict(y=5, k=3, e=2, G=6, s=2, u=3, H=3, v=3, K=3)),
    ("zab", "zbc", "zac", dict(z=5, a=33, b=17, c=65)),   # batched
    ("zbghkuA", "suhdH", "zbgkAsdH", dict(z=3, b=4, g=5, h=2, k=2, u=2, A=6, s=2, d=2, H=3)),
    ("ik", "kj", "ij", dict(i=1, k=300, j=1)),            # dot product
    ("ik", "kj", "ij", dict(i=2000, k=5, j=16)),          # skinny N
    ("ik", "kj", "ij", dict(i=70, k=4100, j=50)),         # split-K with a ragged last slice
    ("zki", "zkj", "zij", dict(z=3, k=1000, i=64, j=64)),  # batched split-K, K-contiguous A and B
    # both matrix sides above 128: split-BF16 packs its operands
    ("ik", "kj", "ij", dict(i=300, k=70, j=200)),
    ("yghk", "gdeG", "yhkdeG", dict(y=20, g=7, h=3, k=3, d=4, e=4, G=11)),
    ("iab", "baj", "ij", dict(i=150, a=40, b=37, j=140)),  # k table longer than one LDS slice
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("conj", [(False, False), (True, False), (False, True)])
def test_contract_matches_einsum(handle, prec, case, conj):
    import torch
    ia, ib, ic, dims = CASES[case]
    rng = np.random.default_rng(100 + case)
    A = _rand(rng, [dims[c] for c in ia])
    B = _rand(rng, [dims[c] for c in ib])
    ref = np.einsum(f"{ia},{ib}->{ic}", A.conj() if conj[0] else A, B.conj() if conj[1] else B)
    td = torch.complex128 if prec == "fp64" else torch.complex64
    if prec != "fp64":
        A = A.astype(np.complex64).astype(np.complex128)
        B = B.astype(np.complex64).astype(np.complex128)
        ref = np.einsum(f"{ia},{ib}->{ic}", A.conj() if conj[0] else A, B.conj() if conj[1] else B)
    dA = torch.from_numpy(A).to("cuda", td)
    dB = torch.from_numpy(B).to("cuda", td)
    dC = torch.zeros([dims[c] for c in ic], dtype=td, device="cuda")
    handle.test_contract(prec, ia, dA, ib, dB, ic, dC, conjA=conj[0], conjB=conj[1])
    torch.cuda.synchronize()
    got = dC.cpu().numpy().astype(np.complex128)
    # error relative to the scale of the products (sum of |a||b| terms)
    scale = np.einsum(f"{ia},{ib}->{ic}", np.abs(A), np.abs(B))
    err = np.max(np.abs(got - ref) / np.maximum(scale, 1e-300))
    assert err < TOL[prec], err


def _packs(ia, ib, dims):
    """Split-BF16 packs its operands when both matrix sides exceed 128."""
    rows = lambda x, y: int(np.prod([dims[c] for c in x if c not in y]))  # noqa: E731
    return rows(ia, ib) > 128 and rows(ib, ia) > 128


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("ksplit", [1, 3])
def test_every_tile_configuration(handle, prec, case, cfg, ksplit):
    """Each kernel variant (tile configuration x K slicing) against einsum, with
    conjugated A; the autotuner may pick any of them."""
    import torch
    ia, ib, ic, dims = CASES[case]
    if cfg == 4 and not (prec.startswith("bf16") and _packs(ia, ib, dims)):
        pytest.skip("the 128x128 tile exists for packed split-BF16 operands only")
    rng = np.random.default_rng(500 + case)
    A = _rand(rng, [dims[c] for c in ia])
    B = _rand(rng, [dims[c] for c in ib])
    td = torch.complex128 if prec == "fp64" else torch.complex64
    if prec != "fp64":
        A = A.astype(np.complex64).astype(np.complex128)
        B = B.astype(np.complex64).astype(np.complex128)
    ref = np.einsum(f"{ia},{ib}->{ic}", A.conj(), B)
    scale = np.einsum(f"{ia},{ib}->{ic}", np.abs(A), np.abs(B))
    dA = torch.from_numpy(A).to("cuda", td)
    dB = torch.from_numpy(B).to("cuda", td)
    dC = torch.full([dims[c] for c in ic], 3.0 + 1j, dtype=td, device="cuda")
    handle.test_contract(prec, ia, dA, ib, dB, ic, dC, conjA=True, cfg=cfg, ksplit=ksplit)
    torch.cuda.synchronize()
    got = dC.cpu().numpy().astype(np.complex128)
    err = np.max(np.abs(got - ref) / np.maximum(scale, 1e-300))
    assert err < TOL[prec], err


@pytest.fixture(scope="module")
def tuned_handle(tmp_path_factory):
    import paper_2507_11424_amd as tnb
    h = tnb.Handle(0)
    path = tmp_path_factory.mktemp("tune") / "choices.txt"
    h.set_autotune(True, str(path))
    yield h, path
    h.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_autotuned_contract_matches_einsum(tuned_handle, prec, case):
    """First call times the candidate tile/split-K configurations (relaunching
    the kernel several times into C), second call runs the winner; both must
    match, and an accumulating call on the tuned plan must add exactly once."""
    import torch
    h, path = tuned_handle
    ia, ib, ic, dims = CASES[case]
    rng = np.random.default_rng(300 + case)
    A = _rand(rng, [dims[c] for c in ia])
    B = _rand(rng, [dims[c] for c in ib])
    td = torch.complex128 if prec == "fp64" else torch.complex64
    if prec != "fp64":
        A = A.astype(np.complex64).astype(np.complex128)
        B = B.astype(np.complex64).astype(np.complex128)
    ref = np.einsum(f"{ia},{ib}->{ic}", A, B)
    scale = np.einsum(f"{ia},{ib}->{ic}", np.abs(A), np.abs(B))
    dA = torch.from_numpy(A).to("cuda", td)
    dB = torch.from_numpy(B).to("cuda", td)
    for call in range(2):
        dC = torch.zeros([dims[c] for c in ic], dtype=td, device="cuda")
        h.test_contract(prec, ia, dA, ib, dB, ic, dC)
        torch.cuda.synchronize()
        got = dC.cpu().numpy().astype(np.complex128)
        err = np.max(np.abs(got - ref) / np.maximum(scale, 1e-300))
        assert err < TOL[prec], (call, err)
    h.test_contract(prec, ia, dA, ib, dB, ic, dC, accumulate=True)
    torch.cuda.synchronize()
    got = dC.cpu().numpy().astype(np.complex128)
    err = np.max(np.abs(got - 2 * ref) / np.maximum(scale, 1e-300))
    assert err < 2 * TOL[prec], err
    assert path.exists() and path.read_text().strip()


@pytest.mark.parametrize("case", [10, 11, 12])
def test_autotune_choices_reload(tuned_handle, case):
    """A fresh handle reading the choices file (tile, K slices, packing, FP32
    kernel) runs the stored choice and still matches einsum."""
    import torch
    import paper_2507_11424_amd as tnb
    h0, path = tuned_handle
    ia, ib, ic, dims = CASES[case]
    rng = np.random.default_rng(400 + case)
    A = _rand(rng, [dims[c] for c in ia]).astype(np.complex64).astype(np.complex128)
    B = _rand(rng, [dims[c] for c in ib]).astype(np.complex64).astype(np.complex128)
    ref = np.einsum(f"{ia},{ib}->{ic}", A, B)
    scale = np.einsum(f"{ia},{ib}->{ic}", np.abs(A), np.abs(B))
    dA = torch.from_numpy(A).to("cuda", torch.complex64)
    dB = torch.from_numpy(B).to("cuda", torch.complex64)
    dC = torch.zeros([dims[c] for c in ic], dtype=torch.complex64, device="cuda")
    h0.test_contract("bf16x3", ia, dA, ib, dB, ic, dC)  # writes the choice if new
    torch.cuda.synchronize()
    lines = path.read_text().split("\n")
    assert all(len(x.split()) == 5 for x in lines if x.strip())  # key, cfg, ksplit, packing, fp32
    h = tnb.Handle(0)
    try:
        h.set_autotune(True, str(path))
        dC.zero_()
        h.test_contract("bf16x3", ia, dA, ib, dB, ic, dC)
        torch.cuda.synchronize()
    finally:
        h.close()
    got = dC.cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - ref) / np.maximum(scale, 1e-300)) < TOL["bf16x3"]


def test_contract_accumulate(handle):
    import torch
    rng = np.random.default_rng(7)
    A, B, C0 = _rand(rng, (70, 40)), _rand(rng, (40, 90)), _rand(rng, (70, 90))
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.from_numpy(C0.copy()).cuda()
    handle.test_contract("fp64", "ik", dA, "kj", dB, "ij", dC, accumulate=True)
    torch.cuda.synchronize()
    assert np.abs(dC.cpu().numpy() - (C0 + A @ B)).max() < 1e-11


@pytest.mark.parametrize("m,n,batch", [(4096, 64, 1), (64, 64, 2), (700, 33, 3), (16, 64, 1), (128, 64, 1),
                                       (300, 100, 1), (1, 1, 1), (5, 3, 4), (20000, 8, 1)])
@pytest.mark.parametrize("esz", [16, 8])
def test_qr(handle, m, n, batch, esz):
    import torch
    rng = np.random.default_rng(m * 7 + n)
    A = _rand(rng, (batch, m, n))
    if esz == 8:
        A = A.astype(np.complex64).astype(np.complex128)
    td = torch.complex128 if esz == 16 else torch.complex64
    k = min(m, n)
    dA = torch.from_numpy(A).to("cuda", td)
    dQ = torch.zeros((batch, m, k), dtype=td, device="cuda")
    dR = torch.zeros((batch, k, n), dtype=td, device="cuda")
    handle.test_qr(dA, dQ, dR)
    torch.cuda.synchronize()
    Q = dQ.cpu().numpy().astype(np.complex128)
    R = dR.cpu().numpy().astype(np.complex128)
    tol = 1e-12 if esz == 16 else 2e-6
    for b in range(batch):
        assert np.abs(Q[b].conj().T @ Q[b] - np.eye(k)).max() < tol * max(m, 16)
        assert np.abs(Q[b] @ R[b] - A[b]).max() < tol * max(m, 16) * np.abs(A[b]).max()
        assert np.abs(np.tril(R[b], -1)).max() == 0.0


@pytest.mark.parametrize("m,n,batch", [(16384, 256, 1), (2000, 130, 2)])
@pytest.mark.parametrize("esz", [16, 8])
def test_qr_wide_rank_deficient(handle, m, n, batch, esz):
    """Householder QR wider than one block (blocks of 64 columns, block
    Gram-Schmidt between them, TSQR within) on matrices of half rank."""
    import torch
    rng = np.random.default_rng(m + n)
    A = _rand(rng, (batch, m, n))
    A[:, :, n // 2:] = A[:, :, : n - n // 2] @ _rand(rng, (n - n // 2, n - n // 2))  # rank n - n // 2
    if esz == 8:
        A = A.astype(np.complex64).astype(np.complex128)
    td = torch.complex128 if esz == 16 else torch.complex64
    dA = torch.from_numpy(A).to("cuda", td)
    dQ = torch.zeros((batch, m, n), dtype=td, device="cuda")
    dR = torch.zeros((batch, n, n), dtype=td, device="cuda")
    handle.test_qr(dA, dQ, dR, "householder")
    torch.cuda.synchronize()
    Q = dQ.cpu().numpy().astype(np.complex128)
    R = dR.cpu().numpy().astype(np.complex128)
    tol = 1e-12 if esz == 16 else 2e-6
    for b in range(batch):
        assert np.abs(Q[b].conj().T @ Q[b] - np.eye(n)).max() < tol * 64
        assert np.abs(Q[b] @ R[b] - A[b]).max() < tol * 64 * np.abs(A[b]).max() * np.sqrt(n)
        assert np.abs(np.tril(R[b], -1)).max() == 0.0


@pytest.mark.parametrize("m,n,batch", [(4096, 64, 1), (64, 64, 3), (700, 33, 2), (512, 8, 5), (8192, 128, 1),
                                       (300, 200, 2), (1024, 65, 1)])
@pytest.mark.parametrize("esz", [16, 8])
@pytest.mark.parametrize("cond", [1.0, 1e6, 1e12])
def test_orthonormalise(handle, m, n, batch, esz, cond):
    # Q only (shifted CholeskyQR3): orthonormal columns spanning the columns of A,
    # also for ill-conditioned A (singular values spread over `cond`)
    import torch
    rng = np.random.default_rng(m + n + int(np.log10(cond)))
    U, _ = np.linalg.qr(_rand(rng, (batch, m, n)))
    V, _ = np.linalg.qr(_rand(rng, (batch, n, n)))
    s = np.logspace(0, -np.log10(cond), n)
    A = (U * s[None, None, :]) @ V
    if esz == 8:
        A = A.astype(np.complex64).astype(np.complex128)
    td = torch.complex128 if esz == 16 else torch.complex64
    dA = torch.from_numpy(A).to("cuda", td)
    dQ = torch.zeros((batch, m, n), dtype=td, device="cuda")
    handle.test_qr(dA, dQ, None)
    torch.cuda.synchronize()
    Q = dQ.cpu().numpy().astype(np.complex128)
    tol = 1e-12 if esz == 16 else 1e-5
    for b in range(batch):
        assert np.abs(Q[b].conj().T @ Q[b] - np.eye(n)).max() < tol * 10
        proj = Q[b] @ (Q[b].conj().T @ A[b])
        assert np.abs(proj - A[b]).max() < tol * 10 * np.abs(A[b]).max()


@pytest.mark.parametrize("m,n", [(200, 50), (4096, 64), (300, 130)])
def test_orthonormalise_zero_columns(handle, m, n):
    """Orthonormalisation of rank-deficient A with exact zero columns, tiny
    ones and singular values spread down to 1e-27 (the fit's matrices when its
    bond exceeds the rank of the state it compresses, e.g. simple-update states
    with zero-padded bonds): the CholeskyQR passes clamp a pivot and the item
    is refactored by Householder, so Q has orthonormal columns whose span
    holds A's."""
    import torch
    rng = np.random.default_rng(m + 7 * n)
    A = _rand(rng, (4, m, 5)) @ _rand(rng, (4, 5, n))  # rank 5
    A[0, :, 7:19] = 0
    A[1, :, ::3] = 0
    A[2, :, 2] = 1e-200 * _rand(rng, (m,))
    U, _ = np.linalg.qr(_rand(rng, (m, n)))
    V, _ = np.linalg.qr(_rand(rng, (n, n)))
    A[3] = (U * (0.15 * 10.0 ** -np.linspace(0, 27, n))) @ V  # numerical rank ~ 20
    dA = torch.from_numpy(A).cuda()
    dQ = torch.zeros((4, m, n), dtype=torch.complex128, device="cuda")
    handle.test_qr(dA, dQ, None, "cholesky")
    torch.cuda.synchronize()
    Q = dQ.cpu().numpy()
    assert np.all(np.isfinite(Q))
    for b in range(4):
        assert np.abs(Q[b].conj().T @ Q[b] - np.eye(n)).max() < 1e-12 * np.sqrt(m)
        assert np.abs(A[b] - Q[b] @ (Q[b].conj().T @ A[b])).max() < 1e-12 * np.abs(A[b]).max()


@pytest.mark.parametrize("m,n,batch", [(4096, 64, 1), (512, 64, 16), (700, 33, 2), (37, 5, 3), (4097, 64, 1)])
@pytest.mark.parametrize("esz", [16, 8])
def test_orthonormalise_lq_layout(handle, m, n, batch, esz):
    """The LQ moves' CholeskyQR3: the input is read and Q written through
    conjugate-transposed strides (rows of the n x m operand), m past several
    row blocks and a ragged last block."""
    import torch
    rng = np.random.default_rng(m * 3 + n)
    B = _rand(rng, (batch, n, m))
    if esz == 8:
        B = B.astype(np.complex64).astype(np.complex128)
    td = torch.complex128 if esz == 16 else torch.complex64
    dB = torch.from_numpy(B).to("cuda", td)
    dQ = torch.zeros((batch, n, m), dtype=td, device="cuda")
    handle.test_qr(dB, dQ, None, method="cholesky_lq")
    torch.cuda.synchronize()
    Q = dQ.cpu().numpy().astype(np.complex128)
    tol = 1e-12 if esz == 16 else 1e-5
    for b in range(batch):
        assert np.abs(Q[b] @ Q[b].conj().T - np.eye(n)).max() < tol * 10
        proj = (B[b] @ Q[b].conj().T) @ Q[b]
        assert np.abs(proj - B[b]).max() < tol * 10 * np.abs(B[b]).max()


@pytest.mark.parametrize("m,n,batch", [(4096, 64, 1), (64, 64, 3), (512, 8, 4), (700, 33, 2), (8192, 128, 1),
                                       (300, 200, 2)])
def test_cholesky_qr_with_r(handle, m, n, batch):
    """CholeskyQR3 with R = R_3 R_2 R_1, as used to right-canonicalise the fits'
    random initial guesses: Q orthonormal, R upper triangular, QR = A."""
    import torch
    rng = np.random.default_rng(m * 7 + n)
    A = (2 * rng.random((batch, m, n)) - 1) + 1j * (2 * rng.random((batch, m, n)) - 1)
    dA = torch.from_numpy(A).cuda()
    dQ = torch.zeros((batch, m, n), dtype=torch.complex128, device="cuda")
    dR = torch.full((batch, n, n), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    handle.test_qr(dA, dQ, dR, method="cholesky")
    torch.cuda.synchronize()
    Q, R = dQ.cpu().numpy(), dR.cpu().numpy()
    for b in range(batch):
        assert np.abs(Q[b].conj().T @ Q[b] - np.eye(n)).max() < 1e-12
        assert np.abs(np.tril(R[b], -1)).max() == 0.0
        assert np.abs(Q[b] @ R[b] - A[b]).max() < 1e-12 * np.abs(A[b]).max() * np.sqrt(m)


def test_qr_rank_deficient(handle):
    import torch
    rng = np.random.default_rng(3)
    A = _rand(rng, (1, 512, 8)) @ _rand(rng, (1, 8, 64))  # rank 8
    A[0, :, 5] = 0
    dA = torch.from_numpy(A).cuda()
    dQ = torch.zeros((1, 512, 64), dtype=torch.complex128, device="cuda")
    dR = torch.zeros((1, 64, 64), dtype=torch.complex128, device="cuda")
    handle.test_qr(dA, dQ, dR)
    torch.cuda.synchronize()
    Q, R = dQ.cpu().numpy()[0], dR.cpu().numpy()[0]
    assert np.all(np.isfinite(Q))
    assert np.abs(Q @ R - A[0]).max() < 1e-10 * np.abs(A).max()


@pytest.mark.parametrize("m,n", [(2500, 100), (3000, 40), (50, 100)])
def test_householder_tiny_columns(handle, m, n):
    """Householder QR of matrices whose column norms span 1 down to the
    subnormal range, with exact zero columns and a tiny multiple of another
    column (the gauged site matrices of the simple update at large bond are
    like this).  Paths: one workgroup in global memory (2500 x 100), a TSQR
    tree (3000 x 40), one LDS block of a wide matrix (50 x 100).  Q must be
    finite and orthonormal and QR must reproduce A: a column norm whose squares
    underflow is taken from scaled values, and the normalised reflectors never
    divide by a squared norm."""
    import torch
    rng = np.random.default_rng(m + 3 * n)
    A = _rand(rng, (2, m, n))
    A *= 10.0 ** -rng.choice([0, 3, 20, 156, 160, 170, 200, 310], size=(2, 1, n))
    A[0, :, 3] = 0
    A[1, :, :5] = 0
    A[1, :, 10] = A[1, :, 11] * 1e-150
    k = min(m, n)
    dA = torch.from_numpy(A).cuda()
    dQ = torch.zeros((2, m, k), dtype=torch.complex128, device="cuda")
    dR = torch.zeros((2, k, n), dtype=torch.complex128, device="cuda")
    handle.test_qr(dA, dQ, dR, "householder")
    torch.cuda.synchronize()
    Q, R = dQ.cpu().numpy(), dR.cpu().numpy()
    assert np.all(np.isfinite(Q)) and np.all(np.isfinite(R))
    for b in range(2):
        assert np.abs(Q[b].conj().T @ Q[b] - np.eye(k)).max() < 1e-12 * np.sqrt(m)
        assert np.abs(np.tril(R[b], -1)).max() == 0.0
        assert np.abs(Q[b] @ R[b] - A[b]).max() < 1e-13 * np.abs(A[b]).max() * np.sqrt(m)


@pytest.mark.parametrize("layout", ["ik,kj->ij", "ki,kj->ij"])
def test_contract_operand_over_2gib(handle, layout):
    """An operand spanning more than 2 GiB is cut into slices on the host (the
    kernel's buffer resources address < 2 GiB); rows sampled across the cuts
    must match float64 NumPy.  With "ki" the cut letter is the summed one, so
    the slices accumulate."""
    import torch
    ia, rest = layout.split(",")
    ib, ic = rest.split("->")
    big = (1 << 23) + 5           # 2^23 + 5 rows x 16 x 16 B = 2.15 GB
    g = torch.Generator(device="cuda").manual_seed(3)
    if ia == "ik":
        A = torch.randn((big, 16), dtype=torch.complex128, device="cuda", generator=g)
        B = torch.randn((16, 8), dtype=torch.complex128, device="cuda", generator=g)
        C = torch.empty((big, 8), dtype=torch.complex128, device="cuda")
    else:  # summed letter is the long one: C[i, j] = sum_k A[k, i] B[k, j]
        A = torch.randn((big, 16), dtype=torch.complex128, device="cuda", generator=g)
        B = torch.randn((big, 8), dtype=torch.complex128, device="cuda", generator=g)
        C = torch.empty((16, 8), dtype=torch.complex128, device="cuda")
    handle.test_contract("fp64", ia, A, ib, B, ic, C)
    torch.cuda.synchronize()
    if ia == "ik":
        rows = np.array([0, 1, 77, (1 << 22) - 1, 1 << 22, (1 << 22) + 1, big - 2, big - 1])
        a = A[torch.from_numpy(rows).cuda()].cpu().numpy()
        ref = a @ B.cpu().numpy()
        got = C[torch.from_numpy(rows).cuda()].cpu().numpy()
        scale = np.abs(a) @ np.abs(B.cpu().numpy())
    else:
        a, b = A.cpu().numpy(), B.cpu().numpy()
        ref = a.T @ b
        got = C.cpu().numpy()
        scale = np.abs(a).T @ np.abs(b)
    del A, B
    torch.cuda.empty_cache()
    assert np.max(np.abs(got - ref) / scale) < 1e-12


def test_timing_mode_with_nested_contractions():
    """Event timing on a fresh handle while a blocked (n > 64) orthonormalisation
    issues nested contractions: the event-pair store grows inside the outer
    pair (this once invalidated the outer pair), and the counters collect."""
    import torch
    import paper_2507_11424_amd as tnb
    h = tnb.Handle(0)
    try:
        h.set_timing(True)
        rng = np.random.default_rng(12)
        for n in (128, 200):
            A = torch.from_numpy(_rand(rng, (2, 1024, n))).cuda()
            Q = torch.zeros_like(A)
            R = torch.zeros((2, n, n), dtype=A.dtype, device="cuda")
            h.test_qr(A, Q, R, method="cholesky")
        c = h.counters()
        torch.cuda.synchronize()
        q = Q.cpu().numpy()
        assert np.abs(q[0].conj().T @ q[0] - np.eye(200)).max() < 1e-11
        assert c["gemm_launches"] > 0 and c["gemm_ms"] > 0 and c["qr_ms"] > 0
    finally:
        h.set_timing(False)
        h.close()


# ---------------------------------------------------------------- SVD truncation

def _svd_cases():
    rng = np.random.default_rng(31)
    out = []
    for n in (1, 2, 7, 16, 33, 64, 65, 128, 200, 256):
        R = _rand(rng, (5, n, n)) * np.exp(-0.35 * np.arange(n))[None, None, :]
        R[1] = np.triu(R[1])                      # QR-shaped
        if n > 2:
            R[2][:, n // 2:] = 0                  # rank-deficient (zero columns)
        if n > 1:
            R[3] = R[3][:, :1] @ _rand(rng, (1, n))  # rank one
        # Householder R of a rank-deficient matrix: zero rows below the rank,
        # small nonzero columns past it (the Jacobi residue of such columns must
        # not be rotated down into underflow)
        r = max(1, n // 2)
        R[4] = np.triu(R[4])
        R[4][r:] = 0
        R[4][:r, r:] *= 1e-4
        out.append(R)
    return out


@pytest.mark.parametrize("case", range(10))
@pytest.mark.parametrize("cutoff,chi_min", [(1e-2, 1), (1e-6, 1), (1e-2, 5), (1e-300, 1)])
@pytest.mark.parametrize("esz", [16, 8])
def test_svd_truncation(handle, case, cutoff, chi_min, esz):
    import torch
    from oracle.sampler import keep_count
    R = _svd_cases()[case]
    n = R.shape[-1]
    U, SV, k = handle.test_svd(torch.from_numpy(R).cuda(), cutoff, chi_min, esz)
    U = U.cpu().numpy().astype(np.complex128)
    SV = SV.cpu().numpy().astype(np.complex128)
    k = k.cpu().numpy()
    tol = 1e-12 if esz == 16 else 2e-6
    for b in range(R.shape[0]):
        u, s, vh = np.linalg.svd(R[b])
        kk = keep_count(s, cutoff, chi_min)
        assert k[b] == kk, (n, b, k[b], kk)
        best = (u[:, :kk] * s[:kk]) @ vh[:kk]
        assert np.linalg.norm(U[b] @ SV[b] - best) <= tol * np.linalg.norm(R[b]) * max(1, n / 16)
        assert np.all(U[b][:, kk:] == 0) and np.all(SV[b][kk:] == 0)
        G = U[b][:, :kk].conj().T @ U[b][:, :kk]
        assert np.abs(G - np.eye(kk)).max() <= (1e-11 if esz == 16 else 1e-5)
        # rows of SV carry the singular values, in descending order
        assert np.allclose(np.linalg.norm(SV[b][:kk], axis=1), s[:kk], rtol=tol * 10, atol=tol * s[0])


# ---------------------------------------------------------------- masked launches

MASK_CASES = [
    # (A, B, C letters, dims, mode): the sample letter z slowest in the kernel's
    # rows (the sampler's environment steps), columns, or the batch index
    ("zab", "bc", "zac", dict(z=5, a=128, b=70, c=96)),
    ("ab", "zbc", "zac", dict(z=5, a=40, b=33, c=64)),
    ("zab", "zbc", "zac", dict(z=5, a=70, b=50, c=66)),
    ("zab", "bc", "zac", dict(z=5, a=256, b=70, c=160)),  # split-BF16 packs these
    ("zab", "bc", "zac", dict(z=5, a=100, b=40, c=30)),  # rows per item not a tile multiple: all computed
]
MASK_ALIGNED = [True, True, True, True, False]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("case", range(len(MASK_CASES)))
@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("ksplit", [1, 3])
def test_masked_contraction(handle, prec, case, cfg, ksplit):
    import torch
    ia, ib, ic, dims = MASK_CASES[case]
    if cfg == 4 and not (prec.startswith("bf16") and _packs(ia, ib, dims)):
        pytest.skip("the 128x128 tile exists for packed split-BF16 operands only")
    rng = np.random.default_rng(100 + case)
    A = _rand(rng, tuple(dims[c] for c in ia))
    B = _rand(rng, tuple(dims[c] for c in ib))
    ref = np.einsum(f"{ia},{ib}->{ic}", A, B)
    td = torch.complex128 if prec == "fp64" else torch.complex64
    if prec != "fp64":
        A = A.astype(np.complex64).astype(np.complex128)
        B = B.astype(np.complex64).astype(np.complex128)
        ref = np.einsum(f"{ia},{ib}->{ic}", A, B)
    sentinel = 7.0 - 3.0j
    C = torch.full(tuple(dims[c] for c in ic), sentinel, dtype=td, device="cuda")
    mask = torch.tensor([1, 0, 1, 1, 0], dtype=torch.int32, device="cuda")
    handle.test_contract(prec, ia, torch.from_numpy(A).to("cuda", td), ib, torch.from_numpy(B).to("cuda", td),
                         ic, C, cfg=cfg, ksplit=ksplit, mask=mask)
    got = C.cpu().numpy().astype(np.complex128)
    tol = TOL[prec] * np.abs(A).max() * np.abs(B).max() * dims[[c for c in ia if c in ib][-1]] * 4
    zc = ic.index("z")
    for z in range(5):
        g = np.take(got, z, axis=zc)
        r = np.take(ref, z, axis=zc)
        if z in (0, 2, 3):
            assert np.abs(g - r).max() <= tol, (z, np.abs(g - r).max())
        elif MASK_ALIGNED[case]:
            assert np.all(g == sentinel), z  # skipped: untouched
        else:
            assert np.abs(g - r).max() <= tol  # misaligned: computed


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_contract_output_over_2g_elements(handle, prec):
    """An output spanning more than 2^31 elements (the outer product that starts
    the fit's right partial at chi = 256, D = 16) is cut into slices whose
    row and column offsets fit int32; sampled entries against the product."""
    import torch
    rng = np.random.default_rng(77)
    n = 216  # 216^4 = 2.18e9 elements
    A = _rand(rng, (n, n))
    B = _rand(rng, (n, n))
    td = torch.complex128 if prec == "fp64" else torch.complex64
    if prec == "fp32":
        A = A.astype(np.complex64).astype(np.complex128)
        B = B.astype(np.complex64).astype(np.complex128)
    C = torch.empty((n, n, n, n), dtype=td, device="cuda")
    handle.test_contract(prec, "ab", torch.from_numpy(A).to("cuda", td), "cd", torch.from_numpy(B).to("cuda", td),
                         "abcd", C)
    torch.cuda.synchronize()
    idx = rng.integers(0, n, size=(20000, 4))
    idx[:4] = [[0, 0, 0, 0], [n - 1, n - 1, n - 1, n - 1], [n - 1, 0, n - 1, 0], [0, n - 1, 0, n - 1]]
    t = torch.from_numpy(idx).cuda()
    got = C[t[:, 0], t[:, 1], t[:, 2], t[:, 3]].cpu().numpy().astype(np.complex128)
    ref = A[idx[:, 0], idx[:, 1]] * B[idx[:, 2], idx[:, 3]]
    tol = 1e-13 if prec == "fp64" else 1e-6
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    del C
    torch.cuda.empty_cache()
