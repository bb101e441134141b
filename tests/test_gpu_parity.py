"""Parity of every C-ABI entry point with the CPU oracle on identical inputs.

Bars: sampled index sets and p_F bit-exact; floating results within the
normwise relative tolerance of their arithmetic (1e-12 FP64, 1e-5 FP32)."""
import numpy as np
import pytest
import torch

import tr_inputs as ti
from oracle import brsgd, sampling, tr
from gpu_util import DEV, TOL, flat_paper, fold, problem, rel, rounded, say, to_dev, unfold

pytestmark = pytest.mark.gpu

from paper_2303_16492_amd import _lib as L  # noqa: E402
from paper_2303_16492_amd import api  # noqa: E402

SAMPLE_CASES = [
    (3, [20, 20, 20], [3, 3, 3], 100),
    (4, [7, 64, 3, 11], [2, 5, 3, 4], 513),
    (5, [2, 3, 4, 5, 6], [1, 2, 3, 2, 1], 1),
    (2, [9, 13], [4, 3], 37),
    (3, [400, 400, 400], [10, 10, 10], 4096),
    (8, [2, 3, 2, 3, 2, 3, 2, 2], [2, 1, 2, 3, 1, 2, 2, 1], 257),
]


@pytest.mark.parametrize("N,I,R,m", SAMPLE_CASES)
def test_sample_uniform_bit_exact(N, I, R, m):
    desc = api.make_desc(I, R, torch.float32)
    for n in range(N):
        for step in (0, 7, 123456789):
            say("sample uniform", N, I, R, m, n, step)
            idx, pF = api.tr_sample(desc, 11, step, n, m)
            ridx, rpF = sampling.draw(11, step, n, m, I)
            assert np.array_equal(idx.cpu().numpy(), ridx)
            assert np.array_equal(pF.cpu().numpy(), rpF)


@pytest.mark.parametrize("N,I,R,m", SAMPLE_CASES[:4])
def test_sample_weighted_bit_exact(N, I, R, m):
    desc = api.make_desc(I, R, torch.float32)
    w = [ti.int_weights(20 + k, I[k], 1, 1 << 40) for k in range(N)]
    cdf = [to_dev(np.cumsum(wk).astype(np.int64), torch.int64) for wk in w]
    for n in range(N):
        say("sample weighted", N, I, m, n)
        idx, pF = api.tr_sample(desc, 5, 3, n, m, cdf=cdf)
        ridx, rpF = sampling.draw(5, 3, n, m, I, w)
        assert np.array_equal(idx.cpu().numpy(), ridx)
        assert np.array_equal(pF.cpu().numpy(), rpF)


def test_sample_optimal_direct_draw_bit_exact():
    I, R = [5, 7, 4], [2, 3, 2]
    desc = api.make_desc(I, R, torch.float32)
    for n in range(3):
        Jn = int(np.prod([I[k] for k in range(3) if k != n]))
        wJ = ti.int_weights(40 + n, Jn, 1, 1 << 40)
        say("sample optimal", n)
        idx, pF = api.tr_sample(desc, 9, 4, n, 333, cdf_J=to_dev(np.cumsum(wJ).astype(np.int64), torch.int64))
        ridx, rpF = sampling.draw(9, 4, n, 333, I, w_J=wJ)
        assert np.array_equal(idx.cpu().numpy(), ridx)
        assert np.array_equal(pF.cpu().numpy(), rpF)


def test_sample_zero_samples_is_a_no_op():
    desc = api.make_desc([3, 4, 5], [2, 2, 2], torch.float32)
    idx = torch.full((1, 3), 77, dtype=torch.int32, device=DEV)
    pF = torch.full((1,), 5.0, dtype=torch.float64, device=DEV)
    api.tr_sample(desc, 0, 0, 0, 0, idx=idx, pF=pF)
    assert int(idx[0, 0]) == 77 and float(pF[0]) == 5.0


SUB_CASES = [
    (3, [20, 20, 20], [3, 3, 3], 100),
    (4, [6, 5, 7, 4], [2, 5, 3, 4], 77),
    (5, [3, 4, 3, 5, 2], [8, 8, 8, 8, 8], 300),
    (3, [5, 6, 7], [16, 16, 16], 65),
    (2, [9, 13], [4, 3], 37),
    (3, [4, 3, 5], [1, 1, 1], 10),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("N,I,R,m", SUB_CASES)
def test_subchain_parity(N, I, R, m, dtype):
    I, R, cores, X, dcores, dX = problem(1, N, I, R, dtype)
    desc = api.make_desc(I, R, dtype)
    for n in range(N):
        say("subchain", N, I, R, m, n, dtype)
        idx, pF = api.tr_sample(desc, 3, 0, n, m)
        S = api.tr_subchain(desc, n, dcores, idx, m)
        ref = brsgd.subchain_rows(cores, n, idx.cpu().numpy())
        assert rel(S.cpu().numpy(), ref) < TOL[dtype]


GRAD_CASES = [
    (3, [20, 20, 20], [3, 3, 3], 100),
    (4, [12, 9, 17, 6], [2, 5, 3, 4], 513),
    (3, [70, 33, 65], [4, 5, 3], 200),
    (5, [3, 4, 3, 5, 2], [8, 8, 8, 8, 8], 97),
    (2, [9, 13], [4, 3], 1),
    (3, [70, 33, 130], [10, 12, 9], 300),     # RR in (64, 128]
    (3, [40, 20, 30], [16, 16, 16], 129),     # RR = 256
    (3, [1, 5, 7], [2, 3, 2], 65),            # a mode of size 1
    # R_n R_{n+1} a multiple of 4 in every mode (the FP32 kernel's 16-byte
    # operand form): RR = 100 with a ragged last chunk and odd I_n; RR of
    # 128 and 64 (the widest staged rows); mixed RR in (32, 64]; one sample
    (3, [70, 33, 65], [10, 10, 10], 300),
    (3, [36, 24, 28], [8, 16, 8], 256),
    (4, [9, 12, 10, 8], [2, 6, 10, 4], 129),
    (3, [20, 21, 22], [6, 6, 6], 1),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("N,I,R,m", GRAD_CASES)
def test_grad_loss_gram_parity(N, I, R, m, dtype):
    I, R, cores, X, dcores, dX = problem(2, N, I, R, dtype)
    desc = api.make_desc(I, R, dtype)
    prec = L.TR_PREC_F64 if dtype == torch.float64 else L.TR_PREC_F32
    for n in range(N):
        say("grad", N, I, R, m, n, dtype)
        idx, pF = api.tr_sample(desc, 4, 1, n, m)
        S = api.tr_subchain(desc, n, dcores, idx, m)
        g, loss, gram = api.tr_grad(desc, n, dcores[n], dX, idx, S, pF, m, prec, want_gram=True)
        idn, pFn = idx.cpu().numpy(), pF.cpu().numpy()
        Sref = brsgd.subchain_rows(cores, n, idn)
        XF = brsgd.gather_fibers(X, n, idn)
        Jn = brsgd.J_of(I, n)
        # identical inputs: feed the oracle the S the GPU used (rounded to dtype)
        Sin = S.double().cpu().numpy()
        assert rel(Sin, Sref) < TOL[dtype]
        gref, lref = brsgd.stoch_grad(unfold(cores[n]), Sin, XF, pFn, Jn)
        href = brsgd.stoch_hessian(Sin, pFn, Jn)
        assert rel(g.cpu().numpy(), gref) < TOL[dtype]
        assert abs(float(loss) - lref) <= TOL[dtype] * abs(lref)
        assert rel(gram.cpu().numpy(), href) < 1e-12


def test_grad_from_mode_major_replica():
    """Fibers read from a replica (stride 1 along the mode) equal those from
    the paper-order tensor."""
    dtype = torch.float32
    I, R, cores, X, dcores, dX = problem(3, 3, [30, 20, 25], [3, 4, 2], dtype)
    desc = api.make_desc(I, R, dtype)
    for n in range(3):
        say("replica", n)
        Xn = api.tr_x_replicate(desc, dX, n)
        ref = tr.unfold_cyclic(X, n).reshape(-1, order="F")
        assert np.array_equal(Xn.double().cpu().numpy(), ref)
        order = [(n + q) % 3 for q in range(1, 3)]
        strides = [0, 0, 0]
        strides[n] = 1
        s = I[n]
        for k in order:
            strides[k] = s
            s *= I[k]
        drep = api.make_desc(I, R, dtype, x_strides=strides)
        idx, pF = api.tr_sample(desc, 8, 2, n, 150)
        S = api.tr_subchain(desc, n, dcores, idx, 150)
        g1, l1, _ = api.tr_grad(desc, n, dcores[n], dX, idx, S, pF, 150, L.TR_PREC_F32)
        g2, l2, _ = api.tr_grad(drep, n, dcores[n], Xn, idx, S, pF, 150, L.TR_PREC_F32)
        assert torch.equal(g1, g2) and float(l1) == float(l2)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", ["fixed", "robbins-monro", "adagrad"])
def test_plain_update_parity(dtype, kind):
    I, R, cores, X, dcores, dX = problem(4, 3, [17, 9, 12], [3, 2, 4], dtype)
    desc = api.make_desc(I, R, dtype)
    n = 1
    rule = api.step_rule(kind, alpha=0.05, tau=10.0, eta=0.01)
    cfg = brsgd.Config(m=1, rule=kind, alpha=0.05, tau=10.0, eta=0.01)
    rng = np.random.default_rng(0)
    g = rounded(rng.standard_normal((I[n], R[n] * R[2])), dtype)
    acc0 = rounded(np.abs(rng.standard_normal(g.shape)), dtype)
    acc = to_dev(acc0, dtype) if kind == "adagrad" else None
    core = dcores[n].clone()
    say("plain update", dtype, kind)
    st = api.tr_update(desc, n, core, to_dev(g, dtype), rule=rule, t=7, accum=acc)
    new, A = brsgd.update(unfold(cores[n]), -g, cfg, 7, acc0 if kind == "adagrad" else None)
    assert rel(core.cpu().numpy(), new) < TOL[dtype]
    if kind == "adagrad":
        assert rel(acc.cpu().numpy(), A) < TOL[dtype]
    assert int(st) == 0


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("b,eps", [(0.5, 0.0), (0.0, 0.2), (2.0, 0.25)])
def test_adagrad_update_with_b_and_eps(dtype, b, eps):
    """The AdaGrad rule with b > 0 and/or eps > 0 (the remark after
    Algorithm TR-BRSGD): G += eta p / (b + A)^(1/2 + eps), A += p*p, with
    some accumulator entries zero and some directions zero (b = 0 leaves
    those entries unchanged)."""
    I, R, cores, X, dcores, dX = problem(4, 3, [17, 9, 12], [3, 2, 4], dtype)
    desc = api.make_desc(I, R, dtype)
    n = 1
    rule = api.step_rule("adagrad", eta=0.03, b=b, eps=eps)
    cfg = brsgd.Config(m=1, rule="adagrad", eta=0.03, b=b, eps=eps)
    rng = np.random.default_rng(1)
    g = rounded(rng.standard_normal((I[n], R[n] * R[2])), dtype)
    g[0, :3] = 0.0
    acc0 = rounded(np.abs(rng.standard_normal(g.shape)), dtype)
    acc0[0, :2] = 0.0
    acc = to_dev(acc0, dtype)
    core = dcores[n].clone()
    say("adagrad b eps", dtype, b, eps)
    st = api.tr_update(desc, n, core, to_dev(g, dtype), rule=rule, t=3, accum=acc)
    new, A = brsgd.update(unfold(cores[n]), -g, cfg, 3, acc0)
    assert rel(core.cpu().numpy(), new) < TOL[dtype]
    assert rel(acc.cpu().numpy(), A) < TOL[dtype]
    assert int(st) == 0


@pytest.mark.parametrize("scale", [1e-8, 1e4, 1e8])
@pytest.mark.parametrize("R", [[3, 4, 3], [12, 12, 12]])
def test_scaled_update_scale_invariant(scale, R):
    """p = -g (h + eta I)^{-1} does not change when h, eta and g are all
    multiplied by the same factor: the inverse (sweep route, and the
    Cholesky route at R_n R_{n+1} = 144) keeps its digits whether the
    Hessian's entries are far below or far above 1 (FP64, against the
    oracle's Cholesky on the scaled inputs)."""
    dtype = torch.float64
    I = [40, 30, 35] if R[0] == 3 else [20, 16, 18]
    I, R, cores, X, dcores, dX = problem(5, 3, I, R, dtype)
    desc = api.make_desc(I, R, dtype)
    n, m = 1, 400
    idx, pF = api.tr_sample(desc, 6, 0, n, m)
    S = api.tr_subchain(desc, n, dcores, idx, m)
    g, _, gram = api.tr_grad(desc, n, dcores[n], dX, idx, S, pF, m, L.TR_PREC_F64, want_gram=True)
    eta = 0.2 * float(torch.diagonal(gram).mean())
    core = dcores[n].clone()
    say("scaled update at scale", scale, R)
    st = api.tr_update(desc, n, core, g * scale, gram=gram * scale, damping=eta * scale,
                       rule=api.step_rule("fixed", alpha=1.0), t=0)
    h = gram.cpu().numpy() * scale + eta * scale * np.eye(gram.shape[0])
    p, _ = brsgd.scaled_direction(g.cpu().numpy() * scale, h)
    assert int(st) == 0
    assert rel(core.cpu().numpy() - unfold(cores[n]), p) < 1e-15 * np.linalg.cond(h) + 1e-13


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("damping", [0.0, 0.3])
def test_scaled_update_parity(dtype, damping):
    I, R, cores, X, dcores, dX = problem(5, 3, [40, 30, 35], [3, 4, 3], dtype)
    desc = api.make_desc(I, R, dtype)
    prec = L.TR_PREC_F64 if dtype == torch.float64 else L.TR_PREC_F32
    for n in range(3):
        m = 300
        say("scaled update", dtype, damping, n)
        idx, pF = api.tr_sample(desc, 6, 0, n, m)
        S = api.tr_subchain(desc, n, dcores, idx, m)
        g, loss, gram = api.tr_grad(desc, n, dcores[n], dX, idx, S, pF, m, prec, want_gram=True)
        core = dcores[n].clone()
        st = api.tr_update(desc, n, core, g, gram=gram, damping=damping,
                           rule=api.step_rule("fixed", alpha=0.7), t=0)
        h = gram.cpu().numpy() + damping * np.eye(gram.shape[0])
        p, sref = brsgd.scaled_direction(g.double().cpu().numpy(), h)
        want = unfold(cores[n]) + 0.7 * p
        assert rel(core.cpu().numpy(), want) < TOL[dtype]
        assert int(st) == sref == 0


@pytest.mark.parametrize("R", [[2, 2, 2], [4, 5, 3], [6, 6, 6], [7, 8, 7], [9, 9, 9], [11, 11, 11], [8, 16, 8]])
def test_scaled_update_every_sweep_width(R):
    """The blocked sweep at every tile count it is built for (R_n R_{n+1} from
    4 to 128: one to eight 16 x 16 tile columns, one to sixteen 8-pivot
    blocks, a partial last block), each mode of the ring, FP32 cores."""
    dtype = torch.float32
    I = [2 * max(R) + 5, 2 * max(R) + 4, 2 * max(R) + 3]
    I, R, cores, X, dcores, dX = problem(21, 3, I, R, dtype)
    desc = api.make_desc(I, R, dtype)
    for n in range(3):
        RRn = R[n] * R[(n + 1) % 3]
        m = 6 * RRn + 17
        say("sweep width", R, "mode", n, "RR", RRn)
        idx, pF = api.tr_sample(desc, 8, n, n, m)
        S = api.tr_subchain(desc, n, dcores, idx, m)
        g, loss, gram = api.tr_grad(desc, n, dcores[n], dX, idx, S, pF, m, L.TR_PREC_F32, want_gram=True)
        core = dcores[n].clone()
        st = api.tr_update(desc, n, core, g, gram=gram, rule=api.step_rule("fixed", alpha=0.7), t=0)
        p, sref = brsgd.scaled_direction(g.double().cpu().numpy(), gram.cpu().numpy())
        assert int(st) == sref == 0
        cond = np.linalg.cond(gram.cpu().numpy())
        assert rel(core.cpu().numpy(), unfold(cores[n]) + 0.7 * p) < max(TOL[dtype], 1e-15 * cond), cond


def test_scaled_update_large_gram_global_memory_path():
    """RR = 144: the factorisation and the solves run from global memory."""
    dtype = torch.float32
    I, R, cores, X, dcores, dX = problem(15, 3, [200, 30, 35], [12, 12, 12], dtype)
    desc = api.make_desc(I, R, dtype)
    n, m = 0, 700
    idx, pF = api.tr_sample(desc, 6, 0, n, m)
    S = api.tr_subchain(desc, n, dcores, idx, m)
    g, loss, gram = api.tr_grad(desc, n, dcores[n], dX, idx, S, pF, m, L.TR_PREC_F32, want_gram=True)
    core = dcores[n].clone()
    say("scaled update RR=144")
    st = api.tr_update(desc, n, core, g, gram=gram, rule=api.step_rule("fixed", alpha=0.7), t=0)
    p, sref = brsgd.scaled_direction(g.double().cpu().numpy(), gram.cpu().numpy())
    assert int(st) == sref
    cond = np.linalg.cond(gram.cpu().numpy())
    assert rel(core.cpu().numpy(), unfold(cores[n]) + 0.7 * p) < max(TOL[dtype], 1e-15 * cond)


def test_scaled_update_singular_gram_uses_damping_fallback():
    dtype = torch.float64
    I, R, cores, X, dcores, dX = problem(6, 3, [10, 8, 9], [2, 3, 2], dtype)
    desc = api.make_desc(I, R, dtype)
    n = 0
    m = 3                                   # fewer rows than RR = 6: singular Gram
    idx, pF = api.tr_sample(desc, 1, 0, n, m)
    S = api.tr_subchain(desc, n, dcores, idx, m)
    g, _, gram = api.tr_grad(desc, n, dcores[n], dX, idx, S, pF, m, L.TR_PREC_F64, want_gram=True)
    core = dcores[n].clone()
    say("singular gram")
    st = int(api.tr_update(desc, n, core, g, gram=gram, rule=api.step_rule("fixed", alpha=1.0)))
    p, sref = brsgd.scaled_direction(g.cpu().numpy(), gram.cpu().numpy())
    assert st == sref
    assert np.all(np.isfinite(core.cpu().numpy()))
    if st == brsgd.DEV_DAMPED:
        # the damped matrix is nearly singular: agreement is bounded by its
        # condition number times the unit roundoff
        h = gram.cpu().numpy()
        ok = [k for k in range(7)
              if np.all(np.linalg.eigvalsh(h + 10.0 ** (k - 10) * np.trace(h) / 6 * np.eye(6)) > 0)]
        hd = h + 10.0 ** (ok[0] - 10) * np.trace(h) / 6 * np.eye(6)
        assert rel(core.cpu().numpy(), unfold(cores[n]) + p) < 1e-15 * np.linalg.cond(hd)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("law", ["E", "L"])
def test_product_laws_parity(dtype, law):
    I, R, cores, X, dcores, dX = problem(7, 3, [40, 7, 25], [3, 2, 4], dtype)
    desc = api.make_desc(I, R, dtype)
    code = L.TR_LAW_EUCLID if law == "E" else L.TR_LAW_LEVERAGE
    for k in range(3):
        say("law", law, dtype, k)
        cdf, st = api.tr_dist(desc, k, code, dcores[k])
        w = np.diff(np.concatenate([[0], cdf.cpu().numpy().astype(np.uint64)]))
        p_gpu = w.astype(np.float64) / float(w.sum())
        if law == "E":
            pref, _ = sampling.dist_euclid(cores[k])
        else:
            pref = sampling.dist_leverage(cores[k])
        wref = sampling.quantize(pref)
        assert np.max(np.abs(w.astype(np.int64) - wref.astype(np.int64))) <= 64
        assert rel(p_gpu, wref.astype(np.float64) / float(wref.sum())) < 1e-10
        assert int(st) == 0


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("I,R", [([400, 30, 20], [10, 10, 10]), ([300, 20, 40], [8, 16, 8]),
                                 ([130, 50, 9], [7, 11, 3])])
def test_leverage_law_wide_cores(I, R, dtype):
    """The leverage law where the factor stays in LDS (R_k R_{k+1} up to 128),
    including a core with I_k < R_k R_{k+1} (uniform by the closed form)."""
    I, R, cores, X, dcores, dX = problem(17, 3, I, R, dtype)
    desc = api.make_desc(I, R, dtype)
    for k in range(3):
        say("leverage law", I, R, dtype, k)
        cdf, st = api.tr_dist(desc, k, L.TR_LAW_LEVERAGE, dcores[k])
        w = np.diff(np.concatenate([[0], cdf.cpu().numpy().astype(np.uint64)]))
        wref = sampling.quantize(sampling.dist_leverage(cores[k]))
        assert np.max(np.abs(w.astype(np.int64) - wref.astype(np.int64))) <= 64
        assert int(st) == 0


def test_optimal_law_parity():
    dtype = torch.float64
    I, R, cores, X, dcores, dX = problem(8, 3, [9, 7, 8], [2, 3, 2], dtype)
    desc = api.make_desc(I, R, dtype)
    for n in range(3):
        say("optimal law", n)
        cdf, st = api.tr_dist_optimal(desc, n, dcores, dX)
        w = np.diff(np.concatenate([[0], cdf.cpu().numpy().astype(np.uint64)]))
        q, _ = sampling.dist_optimal(cores, X, n)
        wref = sampling.quantize(q)
        assert np.max(np.abs(w.astype(np.int64) - wref.astype(np.int64))) <= 64
        assert int(st) == 0


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("N,I,R", [(3, [20, 20, 20], [3, 3, 3]), (4, [7, 5, 9, 6], [2, 3, 4, 2]),
                                   (3, [300, 40, 33], [10, 10, 10]), (2, [33, 65], [5, 4])])
def test_relerr_and_reconstruct_parity(N, I, R, dtype):
    I, R, cores, X, dcores, dX = problem(9, N, I, R, dtype)
    desc = api.make_desc(I, R, dtype)
    say("relerr", N, I, R, dtype)
    Xh = api.tr_reconstruct(desc, dcores)
    ref = tr.full_tensor(cores)
    assert rel(Xh.cpu().numpy(), flat_paper(ref)) < TOL[dtype]
    rse = float(api.tr_relerr(desc, dcores, dX))
    want = tr.rse(cores, X)
    assert abs(rse - want) <= TOL[dtype] * want, (rse, want)
    rse2 = float(api.tr_relerr(desc, dcores, dX, x_true_norm2=float(np.sum(X * X))))
    assert abs(rse2 - want) <= TOL[dtype] * want, (rse2, want)


@pytest.mark.parametrize("xdt", [torch.float32, torch.float16])
@pytest.mark.parametrize("N,I,R", [(3, [70, 9, 10], [8, 16, 8]), (3, [40, 30, 21], [6, 7, 5]),
                                   (5, [33, 3, 4, 2, 5], [4, 3, 2, 5, 4]), (3, [1, 130, 1], [3, 4, 2])])
def test_relerr_matrix_core_shapes(N, I, R, xdt):
    """FP32 cores through the matrix-core reconstruction at every operand
    width it has (R_1 R_2 = 128, 42, 16, 6), ragged row tiles (I_1 not a
    multiple of 32), ragged column blocks (J not a multiple of 128), a single
    row, and an FP16 target tensor (compared on its rounded values)."""
    dtype = torch.float32
    I, R, cores, X, dcores, dX = problem(11, N, I, R, dtype)
    X = rounded(X, xdt)
    dX = to_dev(flat_paper(X), xdt)
    desc = api.make_desc(I, R, dtype, xdt)
    say("relerr mfma", N, I, R, xdt)
    rse = float(api.tr_relerr(desc, dcores, dX))
    want = tr.rse(cores, X)
    assert abs(rse - want) <= TOL[dtype] * want, (rse, want)
    Xh = api.tr_reconstruct(desc, dcores)
    ref = rounded(tr.full_tensor(cores), xdt)
    assert rel(Xh.double().cpu().numpy(), flat_paper(ref)) < (TOL[dtype] if xdt == torch.float32 else 1e-3)


def test_relerr_small_residual_matrix_cores():
    """The error sums on the matrix cores (FP16 hi/lo products scaled per
    tile) stay accurate when the residual is small next to the tensor:
    X = TR(G) plus noise of relative size 1e-5 (about where a planted run
    stops), with the rows of G_1 scaled by 1e2, 1 and 1e-2 in its three row
    tiles; the RSE agrees with the FP64 oracle to 1%."""
    I, R = [96, 40, 33], [10, 10, 10]
    cores = ti.gaussian_cores(21, 3, I, R)
    rows = np.repeat([1e2, 1.0, 1e-2], 32)
    cores[0] = cores[0] * rows[None, :, None]
    cores = [rounded(c, torch.float32) for c in cores]
    Xt = tr.full_tensor(cores)
    noise = ti.standard_normal(22, Xt.shape)
    X = rounded(Xt + noise * (1e-5 * np.linalg.norm(Xt) / np.linalg.norm(noise)), torch.float32)
    desc = api.make_desc(I, R, torch.float32)
    say("relerr small residual")
    rse = float(api.tr_relerr(desc, [to_dev(unfold(c), torch.float32) for c in cores],
                              to_dev(flat_paper(X), torch.float32)))
    want = tr.rse(cores, X)
    assert 5e-6 < want < 2e-5
    assert abs(rse - want) <= 1e-2 * want, (rse, want)


@pytest.mark.parametrize("scales", [(1e-20, 1e-5, 1e-5), (1e-11, 1e-11, 1e-11), (1e15, 1e5, 1e5),
                                    (1e-25, 1e12, 1e12)])
def test_relerr_matrix_cores_at_extreme_scales(scales):
    """The RSE is scale-invariant: cores scaled so that X sits near the
    bottom (about 1e-30, 1e-33) or well above (1e25) the usual range, or
    with operand tiles of opposite extremes, give the oracle's RSE on the
    same rounded values at the FP32 bar (the per-tile power-of-two scales
    are undone in FP64)."""
    I, R = [40, 30, 21], [6, 7, 5]
    base = ti.gaussian_cores(41, 3, I, R, scale=0.7)
    cores = [rounded(c * s_, torch.float32) for c, s_ in zip(base, scales)]
    Xt = tr.full_tensor([c * s_ for c, s_ in zip(base, scales)])
    X = rounded(Xt + 0.1 * np.sqrt(np.mean(Xt * Xt)) * ti.standard_normal(42, Xt.shape), torch.float32)
    assert np.all(np.isfinite(X)) and np.min(np.abs(X[X != 0])) > 1.2e-38
    desc = api.make_desc(I, R, torch.float32)
    say("relerr scales", scales)
    rse = float(api.tr_relerr(desc, [to_dev(unfold(c), torch.float32) for c in cores],
                              to_dev(flat_paper(X), torch.float32)))
    want = tr.rse(cores, X)
    assert abs(rse - want) <= TOL[torch.float32] * want, (rse, want)


@pytest.mark.parametrize("N,I,R", [(3, [40, 30, 21], [6, 7, 5]), (3, [70, 9, 10], [8, 16, 8])])
def test_relerr_zero_cores_matrix_cores(N, I, R):
    """All-zero FP32 cores on the matrix-core path (tiles whose largest
    magnitude is zero take scale 2^0): X_hat = 0, so the RSE is exactly 1."""
    rng = np.random.default_rng(5)
    X = rounded(rng.standard_normal(I), torch.float32)
    desc = api.make_desc(I, R, torch.float32)
    zero = [torch.zeros(I[k] * R[k] * R[(k + 1) % N], dtype=torch.float32, device=DEV) for k in range(N)]
    say("relerr zero cores", I, R)
    rse = float(api.tr_relerr(desc, zero, to_dev(flat_paper(X), torch.float32)))
    assert rse == 1.0, rse


def test_relerr_zero_at_truth_fp64():
    cores = [rounded(c, torch.float64) for c in ti.gaussian_cores(3, 3, [12, 10, 11], [3, 2, 4])]
    X = tr.full_tensor(cores)
    desc = api.make_desc([12, 10, 11], [3, 2, 4], torch.float64)
    rse = float(api.tr_relerr(desc, [to_dev(unfold(c), torch.float64) for c in cores],
                              to_dev(flat_paper(X), torch.float64)))
    assert rse < 1e-14


def test_full_size_scaled_step_at_bench_configuration():
    """One TR-ScaledBRSGD step of the 400^3, rank-10, kappa = 1e4 workload with
    |F_n| = 4096, in the launch configuration the benchmark times: indices
    bit-exact, S, g, Gram, the updated core and the RSE against the oracle."""
    dtype = torch.float32
    N, I, R, m = 3, 400, 10, 4096
    true3 = ti.illcond_cores(0, N, I, R, 1e4)
    X = tr.full_tensor(true3)
    X = rounded(X / np.sqrt(np.mean(X * X)), dtype)
    init = [rounded(c, dtype) for c in ti.gaussian_cores(1, N, I, R, scale=(1.0 / R ** N) ** (1 / (2 * N)))]
    desc = api.make_desc([I] * N, [R] * N, dtype)
    dX = to_dev(flat_paper(X), dtype)
    dc = [to_dev(unfold(c), dtype) for c in init]
    Xr = [api.tr_x_replicate(desc, dX, k) for k in range(N)]
    for step in range(3):
        n = api.tr_mode(0, step, N)
        say("full-size step", step, "mode", n)
        idx, pF = api.tr_sample(desc, 0, step, n, m)
        ridx, rpF = sampling.draw(0, step, n, m, [I] * N)
        assert np.array_equal(idx.cpu().numpy(), ridx) and np.array_equal(pF.cpu().numpy(), rpF)
        S = api.tr_subchain(desc, n, dc, idx, m)
        cores_now = [fold(c.double().cpu().numpy(), R, R) for c in dc]
        assert rel(S.cpu().numpy(), brsgd.subchain_rows(cores_now, n, ridx)) < TOL[dtype]
        order = [(n + q) % N for q in range(1, N)]
        strides = [0] * N
        strides[n] = 1
        sz = I
        for k in order:
            strides[k] = sz
            sz *= I
        drep = api.make_desc([I] * N, [R] * N, dtype, x_strides=strides)
        g, loss, gram = api.tr_grad(drep, n, dc[n], Xr[n], idx, S, pF, m, L.TR_PREC_F32, want_gram=True)
        Sin = S.double().cpu().numpy()
        XF = brsgd.gather_fibers(X, n, ridx)
        gref, lref = brsgd.stoch_grad(unfold(cores_now[n]), Sin, XF, rpF, I * I)
        assert rel(g.cpu().numpy(), gref) < TOL[dtype]
        assert abs(float(loss) - lref) <= TOL[dtype] * lref
        href = brsgd.stoch_hessian(Sin, rpF, I * I)
        assert rel(gram.cpu().numpy(), href) < 1e-12
        before = unfold(cores_now[n])
        api.tr_update(desc, n, dc[n], g, gram=gram, rule=api.step_rule("fixed", alpha=1.0), t=step)
        p, st = brsgd.scaled_direction(g.double().cpu().numpy(), gram.cpu().numpy())
        got = dc[n].double().cpu().numpy()
        # the solve amplifies rounding by the condition number of h
        cond = np.linalg.cond(gram.cpu().numpy())
        assert rel(got - before, p) < max(1e-5, 1e-15 * cond), (rel(got - before, p), cond)
    cores_now = [fold(c.double().cpu().numpy(), R, R) for c in dc]
    rse = float(api.tr_relerr(desc, dc, dX))
    assert abs(rse - tr.rse(cores_now, X)) < 1e-5 * tr.rse(cores_now, X)


MIXED_CASES = [
    (3, [20, 20, 20], [3, 3, 3], 100),
    (4, [12, 9, 17, 6], [2, 5, 3, 4], 513),
    (3, [70, 33, 130], [10, 12, 9], 300),
    (3, [40, 20, 30], [16, 16, 16], 129),
    (2, [9, 13], [4, 3], 1),
    # every R_n R_{n+1} a multiple of 4 (the 16-byte-operand form): RR = 100
    # with a ragged chunk and odd I_n, RR of 128 and 64, mixed RR, RR = 36
    # with one sample
    (3, [70, 33, 65], [10, 10, 10], 300),
    (3, [36, 24, 28], [8, 16, 8], 256),
    (4, [9, 12, 10, 8], [2, 6, 10, 4], 129),
    (3, [20, 21, 22], [6, 6, 6], 1),
]


@pytest.mark.parametrize("prec,xdt", [(L.TR_PREC_BF16, torch.float32), (L.TR_PREC_F16, torch.float32),
                                      (L.TR_PREC_F16, torch.float16), (L.TR_PREC_BF16, torch.float16)])
@pytest.mark.parametrize("N,I,R,m", MIXED_CASES)
def test_grad_mixed_precision_parity(N, I, R, m, prec, xdt):
    """16-bit matrix-core gradient (hi/lo split prediction) against the FP64
    oracle on the same inputs: normwise 5e-3 (the 16-bit bar)."""
    I, R, cores, X, dcores, dX = problem(12, N, I, R, torch.float32)
    X = rounded(X, xdt)
    dX = to_dev(flat_paper(X), xdt)
    desc = api.make_desc(I, R, torch.float32, xdt)
    for n in range(N):
        say("mixed grad", prec, xdt, N, I, R, m, n)
        idx, pF = api.tr_sample(desc, 4, 1, n, m)
        S = api.tr_subchain(desc, n, dcores, idx, m)
        g, loss, _ = api.tr_grad(desc, n, dcores[n], dX, idx, S, pF, m, prec)
        idn, pFn = idx.cpu().numpy(), pF.cpu().numpy()
        gref, lref = brsgd.stoch_grad(unfold(cores[n]), S.double().cpu().numpy(),
                                      brsgd.gather_fibers(X, n, idn), pFn, brsgd.J_of(I, n))
        assert rel(g.cpu().numpy(), gref) < TOL[torch.bfloat16]
        assert abs(float(loss) - lref) <= TOL[torch.bfloat16] * lref


def test_mixed_prediction_resolves_small_residuals():
    """Near a fit (residual ~1e-2 of X) the hi/lo prediction (16 mantissa
    bits, error ~1e-5 |X|) keeps the gradient within the 16-bit bar relative
    to the residual; one BF16 product (error ~2^-9 |X|) would be ~20% off."""
    I, R = [60, 50, 40], [4, 3, 5]
    cores = [rounded(c, torch.float32) for c in ti.gaussian_cores(3, 3, I, R)]
    Xc = tr.full_tensor(cores)
    X = rounded(Xc + 1e-2 * np.sqrt(np.mean(Xc * Xc)) * ti.standard_normal(4, I), torch.float32)
    desc = api.make_desc(I, R, torch.float32)
    dc = [to_dev(unfold(c), torch.float32) for c in cores]
    dX = to_dev(flat_paper(X), torch.float32)
    n, m = 1, 512
    idx, pF = api.tr_sample(desc, 2, 0, n, m)
    S = api.tr_subchain(desc, n, dc, idx, m)
    g, _, _ = api.tr_grad(desc, n, dc[n], dX, idx, S, pF, m, L.TR_PREC_BF16)
    gref, _ = brsgd.stoch_grad(unfold(cores[n]), S.double().cpu().numpy(),
                               brsgd.gather_fibers(X, n, idx.cpu().numpy()), pF.cpu().numpy(), 60 * 40)
    assert rel(g.cpu().numpy(), gref) < TOL[torch.bfloat16]


def test_full_size_mixed_gradient_at_bench_configuration():
    dtype = torch.float32
    N, I, R, m = 3, 400, 10, 4096
    true3 = ti.illcond_cores(0, N, I, R, 1e4)
    X = tr.full_tensor(true3)
    X = rounded(X / np.sqrt(np.mean(X * X)), dtype)
    init = [rounded(c, dtype) for c in ti.gaussian_cores(1, N, I, R, scale=(1.0 / R ** N) ** (1 / (2 * N)))]
    desc = api.make_desc([I] * N, [R] * N, dtype)
    dX = to_dev(flat_paper(X), dtype)
    dc = [to_dev(unfold(c), dtype) for c in init]
    for step in range(3):
        n = api.tr_mode(0, step, N)
        say("full-size mixed", step, n)
        idx, pF = api.tr_sample(desc, 0, step, n, m)
        S = api.tr_subchain(desc, n, dc, idx, m)
        g, loss, _ = api.tr_grad(desc, n, dc[n], dX, idx, S, pF, m, L.TR_PREC_BF16)
        gref, lref = brsgd.stoch_grad(unfold(init[n]), S.double().cpu().numpy(),
                                      brsgd.gather_fibers(X, n, idx.cpu().numpy()), pF.cpu().numpy(), I * I)
        assert rel(g.cpu().numpy(), gref) < TOL[torch.bfloat16]
        assert abs(float(loss) - lref) <= TOL[torch.bfloat16] * lref


def _lev_weights(cdf):
    return np.diff(np.concatenate([[0], cdf.cpu().numpy().astype(np.uint64)])).astype(np.int64)


def _uniform_cdf(n):
    w = np.full(n, int(sampling.quantize(np.array([1.0 / n]))[0]), dtype=np.uint64)
    return np.cumsum(w)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_law_degenerate_cores(dtype):
    """Zero cores: the uniform Euclidean CDF with TR_DEV_ZERO_DIST, and the
    uniform leverage CDF (rank 0) with TR_DEV_ZERO_DIST, as the oracle's
    law returns for rank 0.  A core with I_k <= R_k R_{k+1} and full row
    rank: the uniform leverage CDF and no status (every score is 1)."""
    I, R = [60, 7, 30], [3, 4, 2]
    _, _, cores, X, dcores, dX = problem(23, 3, I, R, dtype)
    desc = api.make_desc(I, R, dtype)

    say("euclid zero core")
    cdf, st = api.tr_dist(desc, 0, L.TR_LAW_EUCLID, torch.zeros_like(dcores[0]))
    assert int(st) == L.TR_DEV_ZERO_DIST
    assert np.array_equal(cdf.cpu().numpy().astype(np.uint64), _uniform_cdf(I[0]))

    say("leverage zero core")
    for k in (0, 1):
        cdf, st = api.tr_dist(desc, k, L.TR_LAW_LEVERAGE, torch.zeros_like(dcores[k]))
        assert int(st) == L.TR_DEV_ZERO_DIST
        assert np.array_equal(cdf.cpu().numpy().astype(np.uint64), _uniform_cdf(I[k]))
        assert np.allclose(sampling.dist_leverage(np.zeros_like(cores[k])), 1.0 / I[k])

    say("leverage I_k <= RR")
    cdf, st = api.tr_dist(desc, 1, L.TR_LAW_LEVERAGE, dcores[1])   # 7 x 8
    assert int(st) == 0
    assert np.array_equal(cdf.cpu().numpy().astype(np.uint64), _uniform_cdf(I[1]))


def _rank_deficient_unfoldings(seed, G):
    """Unfoldings of the same shape as G whose rank is below min(shape), with
    the deficiency exact in binary floating point (so an SVD at the usual
    tolerance and the Gram's pivots agree on the rank): a zero column, a
    duplicated column (or row, when rows are fewer than columns), and an
    exact integer product of rank r."""
    Ik, RR = G.shape
    rng = np.random.default_rng(seed)
    out = []
    a = G.copy()
    b = G.copy()
    if Ik > RR:
        a[:, RR // 2] = 0.0
        b[:, RR - 1] = b[:, 1]
        out += [("zero column", a), ("duplicated column", b)]
    else:
        a[Ik // 2, :] = 0.0
        b[Ik - 1, :] = b[0, :]
        out += [("zero row", a), ("duplicated row", b)]
    r = max(1, min(Ik, RR) // 3)
    A = rng.integers(-3, 4, size=(Ik, r)).astype(np.float64)
    B = rng.integers(-3, 4, size=(r, RR)).astype(np.float64)
    out.append((f"integer rank {r}", A @ B))
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("I,R,k", [([60, 7, 30], [3, 4, 2], 0),      # sweep route, I_k > RR
                                   ([60, 7, 30], [3, 4, 2], 1),      # I_k <= RR: G G^T
                                   ([400, 30, 20], [10, 10, 10], 0),  # the benchmark's core shape
                                   ([300, 20, 30], [12, 12, 4], 0)])  # RR = 144: one-block Cholesky route
def test_leverage_law_rank_deficient_cores(dtype, I, R, k):
    """The leverage law p(i) = l_i / rank (Lemma lev_est, Definition
    "Leverage Scores") on unfoldings of lower rank, against the oracle's
    SVD law: same integer weights up to 64 units of the 2^40 scale, no
    status bit (a rank-deficient core has a valid law)."""
    I, R, cores, X, dcores, dX = problem(29, 3, I, R, dtype)
    desc = api.make_desc(I, R, dtype)
    Rk, Rk1 = R[k], R[(k + 1) % 3]
    for name, G in _rank_deficient_unfoldings(31 + k, unfold(cores[k])):
        G = rounded(G, dtype)
        rank = int(np.linalg.matrix_rank(G))
        assert rank < min(G.shape), name
        say("leverage", name, I, R, k, dtype, "rank", rank)
        cdf, st = api.tr_dist(desc, k, L.TR_LAW_LEVERAGE, to_dev(G, dtype))
        wref = sampling.quantize(sampling.dist_leverage(fold(G, Rk, Rk1))).astype(np.int64)
        w = _lev_weights(cdf)
        assert int(st) == 0, name
        assert np.max(np.abs(w - wref)) <= 64, (name, np.max(np.abs(w - wref)))


