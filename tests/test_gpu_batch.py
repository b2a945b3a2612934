"""GPU parity of the batched engine: every instance of a batch against the FP64 oracle
run with the same instance word, against the plain path, and the batched solve."""
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


def _oracle(w):
    return O.Problem(A=w.A_numpy(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)


def _cat_x(ws, xoff, dtype):
    return torch.zeros(int(xoff[-1]), dtype=dtype, device="cuda")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_matches_oracle_per_instance(dtype):
    ws = inputs.batch_lasso(7, m_range=(101, 613), nnz_frac=0.03, lam_range=(1e-2, 1e-1),
                            block=16, p=0.4, dtype=dtype, seed=3)
    print(f"[gpu] batch of {len(ws)}: m = {[w.m for w in ws]}", flush=True)
    wd = [w.to("cuda") for w in ws]
    B = sca.Batch(wd)
    opts = sca.make_opts(gamma=0.9, select_p=0.4, seed=11)
    x = _cat_x(ws, B.xoff, dtype)
    r = torch.zeros(int(B.roff[-1]), dtype=dtype, device="cuda")
    sca.sca_batch_residual(B.handle, x, r)
    sca.sca_batch_step(B.handle, opts, 0, 25, x, r)
    torch.cuda.synchronize()
    xh = x.double().cpu().numpy()
    rh = r.double().cpu().numpy()
    rep = sca.sca_batch_objective(B.handle, opts, x, B.K)
    for k, w in enumerate(ws):
        prob = _oracle(w)
        cfg = O.RunConfig(tau=w.tau, gamma=0.9, p=0.4, seed=11, instance=k)
        xo, ro, _ = O.run_rounds(prob, cfg, np.zeros(w.n), O.residual(prob, np.zeros(w.n)), 0, 25)
        xg = xh[B.xoff[k]:B.xoff[k + 1]]
        rg = rh[B.roff[k]:B.roff[k] + w.m]
        Fo = O.objective(prob, xo)
        if dtype == torch.float64:
            assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10, k
            assert abs(rep["F"][k] - Fo) <= 1e-10 * abs(Fo)
            assert abs(rep["merit"][k] - O.merit(prob, xo, w.tau)) <= 1e-9
            assert rep["nnz"][k] == O.nnz_best_response(prob, xo, w.tau)
        else:
            assert abs(rep["F"][k] - Fo) <= 1e-4 * abs(Fo), k


def test_batch_equals_plain_path():
    ws = inputs.batch_lasso(5, m_range=(64, 700), nnz_frac=0.05, block=32, p=0.3,
                            dtype=torch.float64, seed=5)
    wd = [w.to("cuda") for w in ws]
    B = sca.Batch(wd)
    opts = sca.make_opts(gamma=0.9, select_p=0.3, seed=2)
    x = _cat_x(ws, B.xoff, torch.float64)
    r = torch.zeros(int(B.roff[-1]), dtype=torch.float64, device="cuda")
    sca.sca_batch_residual(B.handle, x, r)
    sca.sca_batch_step(B.handle, opts, 0, 30, x, r)
    for k, w in enumerate(wd):
        P = sca.Problem.from_workload(w)
        o = sca.make_opts(gamma=0.9, tau=w.tau, select_p=0.3, seed=2, instance=k)
        xp = torch.zeros(w.n, dtype=torch.float64, device="cuda")
        rp = torch.empty(w.m, dtype=torch.float64, device="cuda")
        sca.sca_residual(P.handle, xp, rp)
        sca.sca_step(P.handle, o, 0, 30, xp, rp)
        torch.cuda.synchronize()
        xb = x[B.xoff[k]:B.xoff[k + 1]]
        # identical gradient arithmetic; the folds group columns differently (rounding only)
        assert float((xb - xp).abs().max()) <= 1e-12 * max(1.0, float(xp.abs().max()))
        P.close()


def test_batch_solve_reaches_tolerance_per_instance():
    ws = inputs.batch_lasso(6, m_range=(80, 400), nnz_frac=0.05, lam_range=(2e-2, 1e-1),
                            block=8, p=0.5, dtype=torch.float64, seed=7)
    Fs = []
    for k, w in enumerate(ws):
        prob = _oracle(w)
        Fs.append(O.estimate_F_star(prob, O.RunConfig(tau=w.tau, gamma=0.9, p=0.5, seed=4,
                                                      instance=k))[0])
    wd = [w.to("cuda") for w in ws]
    B = sca.Batch(wd, F_star=Fs)
    opts = sca.make_opts(gamma=0.9, select_p=0.5, seed=4, max_rounds=20000, check_every=10,
                         tol_rel_obj=1e-9)
    x = _cat_x(ws, B.xoff, torch.float64)
    st = sca.sca_batch_solve(B.handle, opts, x, B.K)
    for k, s in enumerate(st):
        assert s["status"] == sca.SCA_OK, (k, s)
        assert s["rel_err"] <= 1e-9
        assert s["rounds"] % 10 == 0 and s["rounds"] > 0
        # the plain solve with the same instance word stops at the same check (+- one)
        P = sca.Problem.from_workload(wd[k])
        o = sca.make_opts(gamma=0.9, tau=ws[k].tau, select_p=0.5, seed=4, instance=k,
                          max_rounds=20000, check_every=10, tol_rel_obj=1e-9, F_star=Fs[k])
        xp = torch.zeros(ws[k].n, dtype=torch.float64, device="cuda")
        sp = sca.sca_solve(P.handle, o, xp)
        assert abs(sp["rounds"] - s["rounds"]) <= 10
        P.close()
    # a second solve (graph replayed from the cache) gives the same result bit for bit
    x2 = _cat_x(ws, B.xoff, torch.float64)
    st2 = sca.sca_batch_solve(B.handle, opts, x2, B.K)
    assert [s["rounds"] for s in st] == [s["rounds"] for s in st2]


def test_batch_graph_replays_match_eager_rounds():
    """The solve replays a captured graph (rounds + check from the running residual); with no
    tolerance (no instance is ever a candidate, so the running residual is never restarted)
    it must reproduce the eager rounds of sca_batch_step on every replay."""
    ws = inputs.batch_lasso(4, m_range=(90, 300), nnz_frac=0.05, block=16, p=0.5,
                            dtype=torch.float64, seed=9)
    wd = [w.to("cuda") for w in ws]
    B = sca.Batch(wd)
    for rounds in (10, 30, 20):  # graph cached after the first call, replayed 1, 3, 2 times
        o = sca.make_opts(gamma=0.9, select_p=0.5, seed=1, max_rounds=rounds, check_every=10)
        xs = torch.zeros(int(B.xoff[-1]), dtype=torch.float64, device="cuda")
        sca.sca_batch_solve(B.handle, o, xs, B.K)
        xe = torch.zeros_like(xs)
        re = torch.zeros(int(B.roff[-1]), dtype=torch.float64, device="cuda")
        sca.sca_batch_residual(B.handle, xe, re)
        for k0 in range(0, rounds, 10):
            sca.sca_batch_step(B.handle, o, k0, 10, xe, re)
        torch.cuda.synchronize()
        assert torch.equal(xs, xe), rounds
