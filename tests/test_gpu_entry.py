"""Sampled-entry loss on the GPU: forward/backward parity with the oracle,
the autograd Function against FP64 central differences (h = 1e-3, exact for
a loss quadratic in each scalar) and against the closed-form block gradient
restricted to the sampled entries."""
import numpy as np
import pytest
import torch

import tr_inputs as ti
from oracle import entry, tr
from gpu_util import DEV, rel, rounded, say, to_dev, unfold

pytestmark = pytest.mark.gpu

from paper_2303_16492_amd import api  # noqa: E402
from paper_2303_16492_amd.autograd import tr_entry_loss  # noqa: E402


def _case(seed, N, I, R, B, snr_db=30.0):
    I = [I] * N if np.isscalar(I) else list(I)
    R = [R] * N if np.isscalar(R) else list(R)
    true = ti.gaussian_cores(seed, N, I, R)
    idx = ti.entry_indices(seed + 1, I, B)
    clean = entry.entry_values(true, idx)
    sig = 10 ** (-snr_db / 20) * np.sqrt(np.mean(clean ** 2))
    x = rounded(clean + sig * ti.standard_normal(seed + 2, B), torch.float32)
    cores = [rounded(c, torch.float32) for c in ti.gaussian_cores(seed + 3, N, I, R, scale=0.5)]
    return I, R, cores, idx, x


# the C4 shape; mixed ranks under each rank bound 4, 8, 12 and 16 of the
# backward's padded slices; a gradient slice too large for LDS (700 rows,
# accumulated in global memory); 50000 entries (several index slabs per
# workgroup); B = 1
CASES = [(5, 32, 8, 8192), (3, [7, 9, 5], [2, 3, 4], 100), (4, [6, 5, 7, 4], [3, 1, 2, 5], 1),
         (2, [11, 13], [12, 7], 333), (6, [3, 2, 4, 3, 2, 3], [2, 2, 3, 1, 2, 2], 777),
         (3, [9, 8, 10], [16, 13, 15], 517), (3, [700, 40, 50], [4, 6, 5], 2000),
         (3, [5, 6, 7], [2, 3, 2], 50000)]


@pytest.mark.parametrize("N,I,R,B", CASES)
def test_entry_forward_backward_parity(N, I, R, B):
    I, R, cores, idx, x = _case(1, N, I, R, B)
    desc = api.make_desc(I, R, torch.float32)
    dc = [to_dev(unfold(c), torch.float32) for c in cores]
    didx = to_dev(idx, torch.int32)
    dx = to_dev(x, torch.float32)
    say("entry fwd/bwd", N, I, R, B)
    resid, loss = api.tr_entry_fwd(desc, dc, didx, dx, B)
    lref, rref = entry.entry_loss(cores, idx, x)
    assert rel(resid.cpu().numpy(), rref) < 1e-5
    assert abs(float(loss) - lref) <= 1e-5 * lref
    grads = api.tr_entry_bwd(desc, dc, didx, resid, B)
    gref = entry.entry_grads(cores, idx, x)
    for k in range(N):
        assert rel(grads[k].cpu().numpy(), unfold(gref[k])) < 1e-5


@pytest.mark.parametrize("N,I,R,B", [CASES[0], CASES[1]])
def test_autograd_against_fd_and_closed_form(N, I, R, B):
    I, R, cores, idx, x = _case(2, N, I, R, B)
    desc = api.make_desc(I, R, torch.float32)
    dc = [to_dev(unfold(c), torch.float32).requires_grad_(True) for c in cores]
    say("autograd", N, I, R, B)
    loss = tr_entry_loss(desc, to_dev(idx, torch.int32), to_dev(x, torch.float32), dc)
    (2.0 * loss).backward()
    gref = entry.entry_grads(cores, idx, x)
    rng = np.random.default_rng(0)
    h = 1e-3
    for k in range(N):
        got = dc[k].grad.cpu().numpy()
        want = 2.0 * unfold(gref[k])
        assert rel(got, want) < 1e-5
        scale = np.max(np.abs(want))
        for _ in range(64):
            pos = tuple(int(rng.integers(0, s)) for s in cores[k].shape)
            vals = []
            for sg in (1, -1):
                cc = [c.copy() for c in cores]
                cc[k][pos] += sg * h
                vals.append(entry.entry_loss(cc, idx, x)[0])
            fd = 2.0 * (vals[0] - vals[1]) / (2 * h)
            r_, i_, s_ = pos
            c_ = r_ + cores[k].shape[0] * s_
            assert abs(got[i_, c_] - fd) <= 1e-5 * scale + 1e-7


def test_backward_is_bitwise_reproducible():
    I, R, cores, idx, x = _case(3, 5, 32, 8, 8192)
    desc = api.make_desc(I, R, torch.float32)
    dc = [to_dev(unfold(c), torch.float32) for c in cores]
    didx = to_dev(idx, torch.int32)
    resid, _ = api.tr_entry_fwd(desc, dc, didx, to_dev(x, torch.float32), 8192)
    a = api.tr_entry_bwd(desc, dc, didx, resid, 8192)
    b = api.tr_entry_bwd(desc, dc, didx, resid, 8192)
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_invalid_indices_give_nan_residuals_and_no_gradient():
    """Entries with an index outside the tensor: NaN residual in the forward,
    no contribution in the backward (whose 1/B still counts every entry)."""
    N, I, R, B = 3, [7, 9, 5], [2, 3, 4], 300
    I, R, cores, idx, x = _case(5, N, I, R, B)
    bad = np.array([0, 17, 123, 299])
    idx = idx.copy()
    idx[bad[0], 0] = -1
    idx[bad[1], 1] = I[1]
    idx[bad[2], 2] = I[2] + 5
    idx[bad[3], 0] = -7
    good = np.setdiff1d(np.arange(B), bad)
    desc = api.make_desc(I, R, torch.float32)
    dc = [to_dev(unfold(c), torch.float32) for c in cores]
    say("entry invalid indices")
    resid, _ = api.tr_entry_fwd(desc, dc, to_dev(idx, torch.int32), to_dev(x, torch.float32), B)
    r = resid.cpu().numpy()
    assert np.all(np.isnan(r[bad]))
    _, rref = entry.entry_loss(cores, idx[good], x[good])
    assert rel(r[good], rref) < 1e-5
    grads = api.tr_entry_bwd(desc, dc, to_dev(idx, torch.int32), resid, B)
    gref = entry.entry_grads(cores, idx[good], x[good])   # mean over the valid entries
    for k in range(N):
        g = grads[k].cpu().numpy()
        assert np.all(np.isfinite(g))
        assert rel(g, unfold(gref[k]) * (len(good) / B)) < 1e-5
