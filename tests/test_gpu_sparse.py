"""GPU parity of the sparse (CSR in, CSC inside) path against the FP64 CPU oracle
(scipy.sparse matrices on the oracle side).  Tolerances as for the dense path."""
import math

import numpy as np
import pytest
import torch

from oracle import sca_oracle as O
from paper_1701_04900_amd import inputs, sca

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def _oracle(w, **kw):
    return O.Problem(A=w.scipy_csr().tocsc(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr, **kw)


class Run:
    def __init__(self, w, **optkw):
        print(f"[gpu] sparse workload {w.name} m={w.m} n={w.n} nnz={w.nnz} dtype={w.dtype}",
              flush=True)
        self.w = w.to("cuda")
        self.P = sca.Problem.from_workload(self.w)
        kw = dict(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
        kw.update(optkw)
        self.opts = sca.make_opts(**kw)
        self.x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
        self.r = torch.empty(w.m, dtype=w.dtype, device="cuda")
        sca.sca_residual(self.P.handle, self.x, self.r)
        self.k = 0

    def step(self, n=1):
        sca.sca_step(self.P.handle, self.opts, self.k, n, self.x, self.r)
        self.k += n
        torch.cuda.synchronize()
        return self.x.double().cpu().numpy(), self.r.double().cpu().numpy()


def _oracle_traj(w, prob, rounds, every):
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
    x = np.zeros(w.n)
    r = O.residual(prob, x)
    out = []
    for k in range(0, rounds, every):
        x, r, _ = O.run_rounds(prob, cfg, x, r, k, every)
        out.append((x.copy(), r.copy()))
    return out


@pytest.mark.parametrize("m,n,per_col,p", [(2000, 20000, 20, 0.1), (1531, 7001, 9, 0.3)])
def test_sparse_fp64_parity(m, n, per_col, p):
    w = inputs.sparse_problem(m, n, per_col=per_col, nnz_frac=0.005, lam_frac=0.01, block=256,
                              p=p, dtype=torch.float64, seed=1)
    prob = _oracle(w)
    run = Run(w)
    for xo, ro in _oracle_traj(w, prob, 40, 5):
        xg, rg = run.step(5)
        assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10


def _irregular(m, n, mean_len, long_len, seed, block=64, p=0.3):
    """CSR with uneven columns: lengths 1 + Exp(mean_len), every 37th column long_len
    nonzeros (longer than one pass of the gradient kernel's unrolled loads)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    lens = np.minimum(m, 1 + rng.exponential(mean_len, size=n).astype(np.int64))
    lens[::37] = long_len
    rows = np.concatenate([rng.choice(m, L, replace=False) for L in lens])
    vals = rng.normal(size=rows.size)
    colptr = np.concatenate([[0], np.cumsum(lens)])
    for j in range(n):  # unit columns
        sl = slice(colptr[j], colptr[j + 1])
        vals[sl] /= np.linalg.norm(vals[sl])
    A = sp.csc_matrix((vals, rows, colptr), shape=(m, n)).tocsr()
    A.sort_indices()
    xt = np.zeros(n)
    supp = rng.choice(n, max(1, n // 100), replace=False)
    xt[supp] = rng.uniform(1, 2, supp.size) * rng.choice([-1.0, 1.0], supp.size)
    b = A @ xt + 0.01 * rng.normal(size=m)
    lam = 0.02 * float(np.max(np.abs(A.T @ b)))
    cn = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    tau = inputs.tau_heuristic(float(cn.min()), float(cn.max()), m, n, p)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt)
    return inputs.SparseWorkload(f"irregular_{m}x{n}_mean{mean_len}", m, n,
                                 t(A.indptr, torch.int64), t(A.indices, torch.int32),
                                 t(A.data, torch.float64), t(b, torch.float64), t(xt, torch.float64),
                                 lam, 0.0, math.inf, float(tau), inputs.block_partition(n, block),
                                 p, 0.9, seed, 0)


@pytest.mark.parametrize("mean_len,long_len", [(6, 150), (45, 300), (90, 700)])
def test_sparse_irregular_columns_fp64_parity(mean_len, long_len):
    w = _irregular(2500, 6000, mean_len, long_len, seed=mean_len)
    prob = _oracle(w)
    run = Run(w)
    for xo, ro in _oracle_traj(w, prob, 30, 5):
        xg, rg = run.step(5)
        assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10
    # a fresh residual at the current point equals the running one to rounding
    rf = torch.empty_like(run.r)
    sca.sca_residual(run.P.handle, run.x, rf)
    assert _rel(rf.cpu().numpy(), O.residual(prob, run.x.cpu().numpy())) <= 1e-13


def test_sparse_fp32_objective():
    w = inputs.sparse_lasso_fp32(m=4000, n=40000, per_col=40, seed=2)
    prob = _oracle(w)
    run = Run(w)
    for xo, _ in _oracle_traj(w, prob, 60, 15):
        run.step(15)
        Fo = O.objective(prob, xo)
        Fg = sca.sca_objective(run.P.handle, run.opts, run.x)["F"]
        assert abs(Fg - Fo) <= 1e-4 * abs(Fo)


def test_sparse_report_at_seeded_point_and_determinism():
    w = inputs.sparse_problem(3000, 12000, per_col=30, nnz_frac=0.02, lam_frac=0.05, block=128,
                              p=0.5, dtype=torch.float64, seed=3)
    prob = _oracle(w)
    run = Run(w)
    xs = w.x_true.clone()
    xd = xs.cuda()
    r = torch.empty(w.m, dtype=torch.float64, device="cuda")
    sca.sca_residual(run.P.handle, xd, r)
    rep = sca.sca_objective(run.P.handle, run.opts, xd)
    xo = xs.numpy()
    assert _rel(r.cpu().numpy(), O.residual(prob, xo)) <= 1e-13
    Fo = O.objective(prob, xo)
    assert abs(rep["F"] - Fo) <= 1e-12 * abs(Fo)
    assert abs(rep["merit"] - O.merit(prob, xo, w.tau)) <= 1e-10 * max(1, rep["merit"])
    assert abs(rep["MF"] - O.stationarity_MF(prob, xo)) <= 1e-10 * max(1, rep["MF"])
    assert rep["nnz"] == O.nnz_best_response(prob, xo, w.tau)
    a = Run(w)
    a.step(20)
    b = Run(w)
    b.step(7)
    b.step(13)
    assert torch.equal(a.x, b.x) and torch.equal(a.r, b.r)


def test_sparse_rejects_bad_csr():
    w = inputs.sparse_problem(500, 2000, per_col=5, nnz_frac=0.01, block=64, p=0.5,
                              dtype=torch.float64, seed=4).to("cuda")
    bad = w.colidx.clone()
    bad[7] = w.n  # out of range
    with pytest.raises(sca.SCAError) as e:
        sca.Problem.csr(w.m, w.n, w.rowptr, bad, w.vals, w.b, w.lam, block_ptr=w.block_ptr)
    assert e.value.status == sca.SCA_EINVAL
    dup = w.colidx.clone()
    r0, r1 = int(w.rowptr[0]), int(w.rowptr[1])
    assert r1 - r0 >= 2
    dup[r0 + 1] = dup[r0]  # repeated (row, column)
    with pytest.raises(sca.SCAError) as e:
        sca.Problem.csr(w.m, w.n, w.rowptr, dup, w.vals, w.b, w.lam, block_ptr=w.block_ptr)
    assert e.value.status == sca.SCA_EINVAL
    rp = w.rowptr.clone()
    rp[-1] += 1
    with pytest.raises(sca.SCAError) as e:
        sca.Problem.csr(w.m, w.n, rp, w.colidx, w.vals, w.b, w.lam, block_ptr=w.block_ptr)
    assert e.value.status == sca.SCA_EINVAL


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_sparse_fold_out_of_range_products_become_nan(dtype):
    """The exact fixed-point fold holds products and row sums below 2^55: with b and lam
    scaled by 1e18 (the solution scales with them) the first round's moves give products
    beyond that, and the rows they reach turn into NaN -- never a silently wrong finite
    residual -- while rows no moved column reaches keep r = -b; a solve stops with
    SCA_ENONFINITE."""
    w = inputs.sparse_problem(600, 3000, per_col=6, nnz_frac=0.01, lam_frac=0.01, block=32,
                              p=1.0, dtype=dtype, seed=9)
    w.b = w.b * 1e18
    w.lam = w.lam * 1e18
    prob = _oracle(w)
    run = Run(w)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(run.r).all())  # r = -b: nothing folded yet
    run.step(1)
    r = run.r.double().cpu().numpy()
    # the oracle's first round (FP64 holds these magnitudes): which columns move
    x1, _, _ = O.run_rounds(prob, O.RunConfig(tau=w.tau, gamma=w.gamma, p=1.0, seed=w.seed),
                            np.zeros(w.n), O.residual(prob, np.zeros(w.n)), 0, 1)
    csc = w.scipy_csr().tocsc()
    reach = np.zeros(w.m, dtype=bool)
    for j in np.flatnonzero(x1):
        reach[csc[:, j].indices] = True
    assert np.isnan(r).any()
    assert not np.isnan(r[~reach]).any()
    b = w.b.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(r[~reach], -b[~reach])
    # a solve from x = 0 reports the non-finite objective
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, max_rounds=20,
                      check_every=5)
    x = torch.zeros(w.n, dtype=dtype, device="cuda")
    with pytest.raises(sca.SCAError) as e:
        sca.sca_solve(run.P.handle, o, x)
    assert e.value.status == sca.SCA_ENONFINITE
