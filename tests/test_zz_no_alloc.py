"""The allocation-free metrics entry point (tn_sample_stats_noalloc) against
tn_sample_stats on the same inputs: same kernels and reduction order, so the
results must agree exactly.  Two calls in a row, the second smaller (the
scratch keeps the first call's partials), and the size limit is an error
raised before any launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _inputs(n, nq, seed):
    import torch
    rng = np.random.default_rng(seed)
    lq = torch.from_numpy(-rng.random(n) * 30.0).cuda()
    lp = torch.from_numpy(-rng.random(n) * 30.0 + rng.standard_normal(n)).cuda()
    bits = torch.from_numpy(rng.integers(0, 2, size=(n, nq), dtype=np.uint8)).cuda()
    return lq, lp, bits


def test_noalloc_matches_sample_stats_twice_second_smaller():
    import torch
    import paper_2507_11424_amd as tnb
    h = tnb.Handle(0)
    try:
        for n, nq, seed in ((70000, 144, 1), (3000, 20, 2)):
            lq, lp, bits = _inputs(n, nq, seed)
            ref = h.sample_stats(lq, lp, -12.5, bits=bits)
            out, zis = h.sample_stats_noalloc(lq, lp, -12.5, bits=bits)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            want = np.array([ref["log_norm_est"], ref["kld"], ref["ess"]])
            assert np.array_equal(got, want), (n, got, want)
            assert torch.equal(zis, ref["z_is"]), n
            # and against a direct float64 evaluation of the definitions
            lw = (lp - lq).cpu().numpy()
            w = np.exp(lw - lw.max())
            assert abs(got[0] - (lw.max() + np.log(w.mean()))) < 1e-10
            assert abs(got[1] - np.mean(lq.cpu().numpy() - lp.cpu().numpy() - 12.5)) < 1e-10
            assert abs(got[2] - w.sum() ** 2 / (w * w).sum()) < 1e-8 * n
            z = (w[:, None] * (1 - 2 * bits.cpu().numpy().astype(np.float64))).sum(0) / w.sum()
            assert np.abs(zis.cpu().numpy() - z).max() < 1e-12
            # without z_is
            out2, z2 = h.sample_stats_noalloc(lq, lp, -12.5)
            torch.cuda.synchronize()
            assert z2 is None and np.array_equal(out2.cpu().numpy(), want)
    finally:
        h.close()


def test_noalloc_rejects_too_many_qubits():
    import torch
    import paper_2507_11424_amd as tnb
    h = tnb.Handle(0)
    try:
        n, nq = 70000, 8189
        lq = torch.zeros(n, dtype=torch.float64, device="cuda")
        lp = torch.zeros(n, dtype=torch.float64, device="cuda")
        bits = torch.zeros((n, nq), dtype=torch.uint8, device="cuda")
        with pytest.raises(tnb.TnError, match="scratch"):
            h.sample_stats_noalloc(lq, lp, 0.0, bits=bits)
        # the limit depends on the qubit count only: the maximum passes
        bits = torch.zeros((n, 8188), dtype=torch.uint8, device="cuda")
        out, zis = h.sample_stats_noalloc(lq, lp, 0.0, bits=bits)
        torch.cuda.synchronize()
        assert np.allclose(out.cpu().numpy(), [0.0, 0.0, n]) and torch.all(zis == 1.0)
    finally:
        h.close()
