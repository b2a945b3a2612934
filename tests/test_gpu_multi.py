"""GPU parity of the many-right-hand-sides path (K problems over one A, one block draw per
round, gradients and residual updates as MFMA products) against the FP64 CPU oracle run
on each problem separately with the same options, and against the single-problem path.
Tolerances as for the dense path: FP64 1e-10, FP32 objectives 1e-4."""
import math

import numpy as np
import pytest
import torch

from oracle import sca_oracle as O
from paper_1701_04900_amd import inputs, sca
from fp32_tolerance import x_tol

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def _oracle(w, k):
    return O.Problem(A=w.At[:, : w.m].cpu().double().numpy().T,
                     b=w.B[k, : w.m].cpu().double().numpy(), lam=float(w.lams[k]), c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)


def _cfg(w, seed=5):
    return O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=seed)


def _opts(w, seed=5, **kw):
    return sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=seed, **kw)


def _setup(w):
    print(f"[gpu] multi workload {w.name} K={w.K}", flush=True)
    At, B = w.At.cuda(), w.B.cuda()
    M = sca.Multi(At, w.m, B, w.lams, w.c, w.beta, w.block_ptr)
    X = M.zeros_x()
    R = M.empty_r()
    sca.sca_multi_residual(M.handle, X, R)
    return M, X, R


@pytest.mark.parametrize("m,n,K,rhs,c_frac,beta,block,p", [
    (150, 600, 5, "sweep", 0.0, math.inf, 10, 0.5),
    (203, 777, 17, "perturbed", 0.0, math.inf, 13, 0.3),
    (97, 333, 64, "sweep", 0.2, 2.0, 7, 0.6),
])
def test_multi_fp64_every_problem_matches_oracle(m, n, K, rhs, c_frac, beta, block, p):
    w = inputs.multi_rhs_problem(m, n, K, rhs=rhs, c_frac=c_frac, beta=beta, block=block, p=p,
                                 dtype=torch.float64, seed=m)
    M, X, R = _setup(w)
    o = _opts(w)
    ks = sorted({0, K // 2, K - 1})
    probs = {k: _oracle(w, k) for k in ks}
    state = {k: (np.zeros(n), O.residual(probs[k], np.zeros(n))) for k in ks}
    for k0 in range(0, 20, 5):
        sca.sca_multi_step(M.handle, o, k0, 5, X, R)
        torch.cuda.synchronize()
        Xh, Rh = X.cpu().numpy(), R.cpu().numpy()
        for k in ks:
            x, r, _ = O.run_rounds(probs[k], _cfg(w), *state[k], k0, 5)
            state[k] = (x, r)
            assert _rel(Xh[k], x) <= 1e-10, (k0, k)
            assert _rel(Rh[k, :m], r) <= 1e-10, (k0, k)
    M.close()


def test_multi_matches_single_problem_path_fp64():
    w = inputs.multi_rhs_problem(300, 1200, 20, rhs="sweep", block=16, p=0.4,
                                 dtype=torch.float64, seed=11)
    M, X, R = _setup(w)
    o = _opts(w)
    sca.sca_multi_step(M.handle, o, 0, 25, X, R)
    At = w.At.cuda()
    for k in (0, 7, 19):
        P = sca.Problem.dense(At, w.m, w.B[k, : w.m].cuda().contiguous(), float(w.lams[k]),
                              w.c, w.beta, w.block_ptr)
        x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
        r = torch.empty(w.m, dtype=torch.float64, device="cuda")
        sca.sca_residual(P.handle, x, r)
        sca.sca_step(P.handle, o, 0, 25, x, r)
        assert _rel(X[k].cpu().numpy(), x.cpu().numpy()) <= 1e-12, k
        assert _rel(R[k, : w.m].cpu().numpy(), r.cpu().numpy()) <= 1e-12, k
        P.close()
    M.close()


def test_multi_fp32_objectives():
    w = inputs.multi_rhs_problem(2000, 8000, 64, rhs="sweep", block=64, p=0.25,
                                 dtype=torch.float32, seed=12)
    M, X, R = _setup(w)
    o = _opts(w)
    sca.sca_multi_step(M.handle, o, 0, 30, X, R)
    rep = sca.sca_multi_objective(M.handle, o, X, w.K)
    for k in (0, 31, 63):
        prob = _oracle(w, k)
        x, r, _ = O.run_rounds(prob, _cfg(w), np.zeros(w.n), O.residual(prob, np.zeros(w.n)), 0,
                               30)
        Fo = O.objective(prob, x, r)
        assert abs(rep["F"][k] - Fo) <= 1e-4 * abs(Fo), k
        print(f"[parity] multi fp32 m={w.m} problem {k}: x err {_rel(X[k].double().cpu().numpy(), x):.2e}", flush=True)
        assert _rel(X[k].double().cpu().numpy(), x) <= x_tol(w.m), k
    M.close()


def test_multi_report_at_seeded_point():
    w = inputs.multi_rhs_problem(180, 700, 9, rhs="perturbed", c_frac=0.1, beta=1.5, block=20,
                                 p=0.5, dtype=torch.float64, seed=13)
    M, X, R = _setup(w)
    o = _opts(w)
    rng = np.random.default_rng(0)
    Xh = np.where(rng.random((w.K, w.n)) < 0.05, rng.normal(size=(w.K, w.n)), 0.0)
    X = torch.from_numpy(Xh).cuda()
    rep = sca.sca_multi_objective(M.handle, o, X, w.K)
    R = M.empty_r()
    sca.sca_multi_residual(M.handle, X, R)
    for k in range(w.K):
        prob = _oracle(w, k)
        assert _rel(R[k, : w.m].cpu().numpy(), O.residual(prob, Xh[k])) <= 1e-13
        Fo = O.objective(prob, Xh[k])
        assert abs(rep["F"][k] - Fo) <= 1e-12 * max(1.0, abs(Fo)), k
        mo = O.merit(prob, Xh[k], w.tau)
        assert abs(rep["merit"][k] - mo) <= 1e-10 * max(1.0, mo), k
        assert rep["nnz"][k] == O.nnz_best_response(prob, Xh[k], w.tau), k
    M.close()


def test_multi_solve_freezes_each_problem_at_its_stop():
    w = inputs.multi_rhs_problem(120, 400, 6, rhs="sweep", lam_range=(0.02, 0.2), block=8,
                                 p=0.5, dtype=torch.float64, seed=14)
    M, X, R = _setup(w)
    cfg = _cfg(w)
    Fs = [O.estimate_F_star(_oracle(w, k), cfg)[0] for k in range(w.K)]
    sca.sca_multi_set_fstar(M.handle, Fs)
    o = _opts(w, max_rounds=20000, check_every=10, tol_rel_obj=1e-8)
    X = M.zeros_x()
    st = sca.sca_multi_solve(M.handle, o, X, w.K)
    At = w.At.cuda()
    for k in range(w.K):
        assert st[k]["status"] == sca.SCA_OK and st[k]["rel_err"] <= 1e-8, (k, st[k])
        # the single-problem solve with the same options stops at the same check
        P = sca.Problem.dense(At, w.m, w.B[k, : w.m].cuda().contiguous(), float(w.lams[k]),
                              w.c, w.beta, w.block_ptr)
        ok = _opts(w, max_rounds=20000, check_every=10, tol_rel_obj=1e-8, F_star=Fs[k])
        x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
        sp = sca.sca_solve(P.handle, ok, x)
        assert sp["rounds"] == st[k]["rounds"], (k, sp["rounds"], st[k]["rounds"])
        assert _rel(X[k].cpu().numpy(), x.cpu().numpy()) <= 1e-12, k
        P.close()
    M.close()


def test_multi_merit_stop_and_determinism():
    w = inputs.multi_rhs_problem(140, 500, 3, rhs="sweep", lam_range=(0.05, 0.1), block=10,
                                 p=0.7, dtype=torch.float64, seed=15)
    M, X, R = _setup(w)
    o = _opts(w, max_rounds=20000, check_every=20, tol_merit=1e-9)
    X1 = M.zeros_x()
    st = sca.sca_multi_solve(M.handle, o, X1, w.K)
    assert all(s["merit"] <= 1e-9 for s in st)
    X2 = M.zeros_x()
    sca.sca_multi_solve(M.handle, o, X2, w.K)
    assert torch.equal(X1, X2)
    M.close()


def test_multi_rejects_bad_arguments():
    w = inputs.multi_rhs_problem(64, 200, 3, dtype=torch.float64, seed=16, block=10)
    At, B = w.At.cuda(), w.B.cuda()
    for bad in (torch.zeros(0, w.lda, dtype=torch.float64, device="cuda"),
                torch.zeros(65, w.lda, dtype=torch.float64, device="cuda")):
        with pytest.raises(sca.SCAError) as e:
            sca.Multi(At, w.m, bad, np.full(bad.shape[0], 0.1), block_ptr=w.block_ptr)
        assert e.value.status == sca.SCA_EINVAL
    with pytest.raises(sca.SCAError) as e:
        sca.Multi(At, w.m, B[:, : w.m - 1].contiguous(), w.lams, block_ptr=w.block_ptr)
    assert e.value.status == sca.SCA_EINVAL
    M = sca.Multi(At, w.m, B, w.lams, block_ptr=w.block_ptr)
    X = M.zeros_x()
    Rbad = torch.zeros(w.K * w.lda + 1, dtype=torch.float64, device="cuda")[1:]
    with pytest.raises(sca.SCAError) as e:
        sca.sca_multi_step(M.handle, _opts(w), 0, 1, X, Rbad)
    assert e.value.status == sca.SCA_EINVAL
    with pytest.raises(sca.SCAError) as e:  # relative-error stop without F*
        sca.sca_multi_solve(M.handle, _opts(w, max_rounds=10, tol_rel_obj=1e-6), X, w.K)
    assert e.value.status == sca.SCA_EINVAL
    M.close()


def test_multi_fp32_ragged_rows_with_nan_padding():
    """m = 1001 (lda 1004) with A's padding rows set to NaN: the fold's whole-row-group loads
    must discard them; objectives against the oracle per problem."""
    w = inputs.multi_rhs_problem(1001, 3000, 9, rhs="perturbed", block=32, p=0.4,
                                 dtype=torch.float32, seed=17)
    assert w.lda > w.m
    probs = {k: _oracle(w, k) for k in (0, 4, 8)}
    w.At[:, w.m:] = float("nan")
    M, X, R = _setup(w)
    o = _opts(w)
    sca.sca_multi_step(M.handle, o, 0, 20, X, R)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(X).all()) and bool(torch.isfinite(R[:, : w.m]).all())
    rep = sca.sca_multi_objective(M.handle, o, X, w.K)
    for k, prob in probs.items():
        x, r, _ = O.run_rounds(prob, _cfg(w), np.zeros(w.n), O.residual(prob, np.zeros(w.n)), 0,
                               20)
        Fo = O.objective(prob, x, r)
        assert abs(rep["F"][k] - Fo) <= 1e-4 * abs(Fo), k
        print(f"[parity] multi fp32 m={w.m} problem {k}: x err {_rel(X[k].double().cpu().numpy(), x):.2e}", flush=True)
        assert _rel(X[k].double().cpu().numpy(), x) <= x_tol(w.m), k
    M.close()


@pytest.mark.parametrize("m,n,K,nan_pad", [(1001, 3000, 64, True), (100, 900, 60, False),
                                           (4100, 6000, 64, False)])
def test_multi_fp32_64_problem_gradient_edges(m, n, K, nan_pad):
    """The FP32 path at 33-64 problems (the direct-to-LDS gradient kernel): ragged m with the
    last row quad straddling m and A's padding rows NaN, splits left empty (m = 100 over 16
    row splits), fewer problems than the 64 padded ones (K = 60: the padding problems' R rows
    must not enter), and partial coordinate tiles; per-problem iterates and objectives against
    the oracle."""
    w = inputs.multi_rhs_problem(m, n, K, rhs="perturbed" if K < 64 else "sweep", block=16,
                                 p=0.37, dtype=torch.float32, seed=31 + m)
    probs = {k: _oracle(w, k) for k in (0, K // 2, K - 1)}
    if nan_pad:
        assert w.lda > w.m
        w.At[:, w.m:] = float("nan")
    M, X, R = _setup(w)
    o = _opts(w)
    sca.sca_multi_step(M.handle, o, 0, 20, X, R)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(X).all()) and bool(torch.isfinite(R[:, : w.m]).all())
    rep = sca.sca_multi_objective(M.handle, o, X, w.K)
    for k, prob in probs.items():
        x, r, _ = O.run_rounds(prob, _cfg(w), np.zeros(w.n), O.residual(prob, np.zeros(w.n)), 0,
                               20)
        Fo = O.objective(prob, x, r)
        ex = _rel(X[k].double().cpu().numpy(), x)
        print(f"[parity] multi fp32 m={w.m} K={K} problem {k}: x err {ex:.2e}", flush=True)
        assert abs(rep["F"][k] - Fo) <= 1e-4 * abs(Fo), k
        assert ex <= x_tol(w.m), k
    M.close()
