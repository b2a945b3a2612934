"""GPU adjoint (implicit differentiation at the fixed point) against the oracle's dense
adjoint and against central finite differences of GPU forward solves (h = 1e-4, FP64)."""
import math

import numpy as np
import pytest
import torch

from oracle import sca_oracle as O
from paper_1701_04900_amd import inputs, sca

pytestmark = pytest.mark.gpu


def _oracle(w):
    return O.Problem(A=w.A_numpy(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)


def _tight(w, **kw):
    return sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed,
                         max_rounds=50000, check_every=20, tol_merit=1e-13, **kw)


def _solve(P, o, n, dtype, x0=None):
    x = torch.zeros(n, dtype=dtype, device="cuda") if x0 is None else x0.clone()
    sca.sca_solve(P.handle, o, x)
    return x


@pytest.mark.parametrize("c_frac,beta", [(0.0, math.inf), (0.15, 3.0)])
def test_adjoint_matches_oracle_and_finite_differences(c_frac, beta):
    w = inputs.dense_problem(120, 300, nnz_frac=0.05, lam_frac=0.1, c_frac=c_frac, beta=beta,
                             block=10, p=1.0, dtype=torch.float64, seed=21)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = _tight(w)
    xs = _solve(P, o, w.n, torch.float64)
    rep = sca.sca_objective(P.handle, o, xs)
    assert rep["MF"] < 1e-11  # solve stops on merit <= 1e-13 (infinity norm)
    rng = np.random.default_rng(0)
    xbar = torch.from_numpy(rng.normal(size=w.n)).cuda()
    bbar = torch.empty(w.m, dtype=torch.float64, device="cuda")
    lb = sca.sca_adjoint(P.handle, o, xs, xbar, bbar)
    # oracle adjoint at the oracle's own fixed point
    prob = _oracle(w)
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=1.0)
    xo, _, _ = O.run_rounds(prob, cfg, np.zeros(w.n), O.residual(prob, np.zeros(w.n)), 0, 20000)
    assert O.stationarity_MF(prob, xo) < 1e-12
    bo, lo = O.adjoint_vjp(prob, xo, xbar.cpu().numpy(), w.tau)
    np.testing.assert_allclose(bbar.cpu().numpy(), bo, rtol=0, atol=1e-8 * max(1, np.abs(bo).max()))
    assert abs(lb - lo) <= 1e-8 * max(1, abs(lo))
    # central differences of GPU forward solves along a seeded direction u (b) and along lam
    u = torch.from_numpy(rng.normal(size=w.m)).cuda()
    h = 1e-4
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, max_rounds=50000,
                      check_every=20, tol_merit=1e-12)  # solve error / h stays below 1e-8
    xp, xm = [], []
    for sgn, out in ((1, xp), (-1, xm)):
        bb = (wd.b + sgn * h * u).contiguous()
        sca.sca_problem_update_rhs(P.handle, bb, w.lam)
        out.append(_solve(P, o, w.n, torch.float64, xs))  # warm start: same solution branch
    fd_b = (xp[0] - xm[0]) / (2 * h)
    assert abs(float(xbar @ fd_b) - float(bbar @ u)) <= 1e-6 * max(1.0, abs(float(bbar @ u)))
    for sgn, out in ((1, xp), (-1, xm)):
        sca.sca_problem_update_rhs(P.handle, wd.b, w.lam + sgn * h)
        out.append(_solve(P, o, w.n, torch.float64, xs))
    fd_l = (xp[1] - xm[1]) / (2 * h)
    assert abs(float(xbar @ fd_l) - lb) <= 1e-6 * max(1.0, abs(lb))


def test_adjoint_fp32_against_fp64():
    w = inputs.dense_problem(400, 1600, nnz_frac=0.03, lam_frac=0.1, block=16, p=1.0,
                             dtype=torch.float32, seed=22)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=1.0, max_rounds=20000,
                      check_every=20, tol_merit=1e-6)
    xs = _solve(P, o, w.n, torch.float32)
    xbar = torch.ones(w.n, dtype=torch.float32, device="cuda")
    bbar = torch.empty(w.m, dtype=torch.float32, device="cuda")
    lb = sca.sca_adjoint(P.handle, o, xs, xbar, bbar)
    prob = _oracle(w)
    xo, _, _ = O.run_rounds(prob, O.RunConfig(tau=w.tau, gamma=w.gamma, p=1.0),
                            np.zeros(w.n), O.residual(prob, np.zeros(w.n)), 0, 8000)
    bo, lo = O.adjoint_vjp(prob, xo, np.ones(w.n), w.tau)
    np.testing.assert_allclose(bbar.double().cpu().numpy(), bo, rtol=0,
                               atol=1e-3 * max(1, np.abs(bo).max()))
    assert abs(lb - lo) <= 1e-3 * max(1, abs(lo))


def test_batch_adjoint_matches_plain_adjoint():
    ws = inputs.batch_lasso(5, m_range=(80, 260), nnz_frac=0.05, lam_range=(3e-2, 1.5e-1),
                            block=8, p=0.5, dtype=torch.float64, seed=23)
    wd = [w.to("cuda") for w in ws]
    B = sca.Batch(wd)
    o = sca.make_opts(gamma=0.9, select_p=0.5, seed=3, max_rounds=100000, check_every=20)
    # forward: per-instance tight solves through the plain path, gathered in the x layout
    xs = torch.zeros(int(B.xoff[-1]), dtype=torch.float64, device="cuda")
    plain = []
    for k, w in enumerate(wd):
        P = sca.Problem.from_workload(w)
        ok = sca.make_opts(gamma=0.9, tau=ws[k].tau, select_p=0.5, seed=3, instance=k,
                           max_rounds=50000, check_every=20, tol_merit=1e-13)
        x = _solve(P, ok, w.n, torch.float64)
        xs[B.xoff[k]:B.xoff[k + 1]] = x
        plain.append((P, ok, x))
    rng = np.random.default_rng(5)
    xbar = torch.from_numpy(rng.normal(size=int(B.xoff[-1]))).cuda()
    bbar = torch.zeros(int(B.roff[-1]), dtype=torch.float64, device="cuda")
    lbs = sca.sca_batch_adjoint(B.handle, o, xs, xbar, bbar, B.K)
    for k, (P, ok, x) in enumerate(plain):
        bb = torch.empty(ws[k].m, dtype=torch.float64, device="cuda")
        lb = sca.sca_adjoint(P.handle, ok, x, xbar[B.xoff[k]:B.xoff[k + 1]].contiguous(), bb)
        got = bbar[B.roff[k]:B.roff[k] + ws[k].m]
        assert float((got - bb).abs().max()) <= 1e-9 * max(1.0, float(bb.abs().max()))
        assert abs(lbs[k] - lb) <= 1e-9 * max(1.0, abs(lb))
        P.close()


def test_autograd_function_gives_the_adjoint():
    w = inputs.dense_problem(150, 400, nnz_frac=0.05, lam_frac=0.1, block=8, p=1.0,
                             dtype=torch.float64, seed=24)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = _tight(w)
    b = wd.b.clone().requires_grad_(True)
    lam = torch.tensor(w.lam, dtype=torch.float64, requires_grad=True)
    x = sca.SolveFn.apply(b, lam, P, o)
    wvec = torch.linspace(-1, 1, w.n, dtype=torch.float64, device="cuda")
    loss = (wvec * x).sum()
    gb, gl = torch.autograd.grad(loss, (b, lam))
    bbar = torch.empty(w.m, dtype=torch.float64, device="cuda")
    lb = sca.sca_adjoint(P.handle, o, x.detach(), wvec, bbar)
    assert torch.allclose(gb, bbar, rtol=0, atol=1e-12)
    assert abs(float(gl) - lb) <= 1e-12 * max(1, abs(lb))


def test_autograd_backward_after_a_second_forward_on_the_same_problem():
    """Two forwards on one Problem (two right-hand sides and weights), then the first
    backward: it must be the adjoint at the first (b, lam), not at the (b, lam) the handle
    held last.  The first b is a temporary, released by the caller after the forward."""
    w = inputs.dense_problem(150, 400, nnz_frac=0.05, lam_frac=0.1, block=8, p=1.0,
                             dtype=torch.float64, seed=24)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = _tight(w)
    rng = np.random.default_rng(8)
    b1 = (wd.b + 0.05 * torch.from_numpy(rng.normal(size=w.m)).cuda()).requires_grad_(True)
    lam1 = torch.tensor(w.lam * 1.3, dtype=torch.float64, requires_grad=True)
    x1 = sca.SolveFn.apply(b1 * 1.0, lam1, P, o)  # b1 * 1.0: a temporary the caller drops
    b2 = wd.b.clone().requires_grad_(True)
    lam2 = torch.tensor(w.lam * 0.7, dtype=torch.float64, requires_grad=True)
    x2 = sca.SolveFn.apply(b2, lam2, P, o)
    assert float((x1 - x2).abs().max()) > 1e-3  # the two solutions differ
    wvec = torch.linspace(-1, 1, w.n, dtype=torch.float64, device="cuda")
    g1b, g1l = torch.autograd.grad((wvec * x1).sum(), (b1, lam1))
    # reference: a problem of its own at the first (b, lam)
    bref = b1.detach().clone()
    Q = sca.Problem.dense(wd.At, w.m, bref, float(lam1), block_ptr=w.block_ptr)
    bbar = torch.empty(w.m, dtype=torch.float64, device="cuda")
    lb = sca.sca_adjoint(Q.handle, o, x1.detach(), wvec, bbar)
    assert torch.allclose(g1b, bbar, rtol=0, atol=1e-12)
    assert abs(float(g1l) - lb) <= 1e-12 * max(1, abs(lb))
    # and the second backward is still the adjoint at the second (b, lam)
    g2b, g2l = torch.autograd.grad((wvec * x2).sum(), (b2, lam2))
    R = sca.Problem.dense(wd.At, w.m, b2.detach().clone(), float(lam2), block_ptr=w.block_ptr)
    lb2 = sca.sca_adjoint(R.handle, o, x2.detach(), wvec, bbar)
    assert torch.allclose(g2b, bbar, rtol=0, atol=1e-12)
    assert abs(float(g2l) - lb2) <= 1e-12 * max(1, abs(lb2))
    Q.close()
    R.close()
    P.close()


def test_batch_autograd_backward_after_a_second_forward():
    ws = inputs.batch_lasso(3, m_range=(80, 200), nnz_frac=0.05, lam_range=(3e-2, 1.5e-1),
                            block=8, p=0.5, dtype=torch.float64, seed=29)
    wd = [w.to("cuda") for w in ws]
    B = sca.Batch(wd)
    o = sca.make_opts(gamma=0.9, select_p=0.5, seed=3, max_rounds=50000, check_every=20,
                      tol_merit=1e-13)
    b_all = torch.zeros(int(B.roff[-1]), dtype=torch.float64, device="cuda")
    for k, w in enumerate(wd):
        b_all[B.roff[k]:B.roff[k] + w.m] = w.b
    lam1 = torch.tensor([w.lam for w in ws], dtype=torch.float64, requires_grad=True)
    b1 = b_all.clone().requires_grad_(True)
    x1 = sca.BatchSolveFn.apply(b1, lam1, B, o)
    lam2 = (lam1.detach() * 0.6).requires_grad_(True)
    b2 = (b_all * 1.1).requires_grad_(True)
    x2 = sca.BatchSolveFn.apply(b2, lam2, B, o)
    assert float((x1 - x2).abs().max()) > 1e-3
    wvec = torch.linspace(-1, 1, int(B.xoff[-1]), dtype=torch.float64, device="cuda")
    g1b, g1l = torch.autograd.grad((wvec * x1).sum(), (b1, lam1))
    # reference: the batch adjoint with the first right-hand sides installed explicitly
    sca.sca_batch_update_rhs(B.handle, b_all, lam1.detach().numpy())
    bbar = torch.zeros(int(B.roff[-1]), dtype=torch.float64, device="cuda")
    lbs = sca.sca_batch_adjoint(B.handle, o, x1.detach(), wvec, bbar, B.K)
    assert torch.allclose(g1b, bbar, rtol=0, atol=1e-12)
    np.testing.assert_allclose(g1l.numpy(), lbs, rtol=1e-12, atol=1e-12)
    B.close()


def test_adjoint_rejects_dc_and_sparse():
    w = inputs.dense_problem(60, 120, nnz_frac=0.05, lam_frac=0.1, block=4, p=1.0,
                             dtype=torch.float64, seed=25).to("cuda")
    P = sca.Problem.from_workload(w)
    sca.sca_problem_set_regularizer(P.handle, sca.SCA_REG_LOG, 20.0)
    x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    bb = torch.empty(w.m, dtype=torch.float64, device="cuda")
    with pytest.raises(sca.SCAError) as e:
        sca.sca_adjoint(P.handle, _tight(w), x, x, bb)
    assert e.value.status == sca.SCA_EINVAL
    s = inputs.sparse_problem(200, 800, per_col=4, nnz_frac=0.02, block=32, p=0.5,
                              dtype=torch.float64, seed=2).to("cuda")
    PS = sca.Problem.from_workload(s)
    xs = torch.zeros(s.n, dtype=torch.float64, device="cuda")
    bs = torch.empty(s.m, dtype=torch.float64, device="cuda")
    with pytest.raises(sca.SCAError) as e:
        sca.sca_adjoint(PS.handle, sca.make_opts(tau=s.tau), xs, xs, bs)
    assert e.value.status == sca.SCA_EINVAL
