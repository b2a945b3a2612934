"""Lock-free rounds (the asynchrony of Algorithm 1 with the delays of Assumption D1 left to
the hardware; sca_opts.async_workgroups).

* One workgroup is a sequential sweep over the drawn coordinates in ascending order: every
  round equals the oracle's delayed round with one coordinate per group and no staleness
  (FP64 1e-10, LASSO and box-nonconvex).
* Many workgroups race (nondeterministic): checked statistically, as the method's theory
  allows -- on a LASSO problem (unique minimiser) the lock-free solve reaches the same
  minimiser as the oracle's synchronous solve, for several workgroup counts and on repeated
  runs; its objective falls over the rounds; FP32 reaches the relative error 1e-5.
* Argument checks: the sparse, batched and multi-right-hand-side paths and bounded-delay
  rounds refuse it, as does a workgroup count above 65536."""
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


def _oracle(w):
    return O.Problem(A=w.A_numpy(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)


@pytest.mark.parametrize("c_frac,beta", [(0.0, math.inf), (0.3, 0.5)])
def test_one_workgroup_is_the_sequential_sweep_fp64(c_frac, beta):
    w = inputs.dense_problem(300, 900, nnz_frac=0.05, lam_frac=0.05, c_frac=c_frac, beta=beta,
                             block=4, p=0.5, dtype=torch.float64, seed=21)
    print(f"[gpu] lock-free W=1 {w.m}x{w.n} c={w.c:.3g} beta={w.beta}", flush=True)
    prob = _oracle(w)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, async_workgroups=1)
    x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    r = torch.empty(w.m, dtype=torch.float64, device="cuda")
    sca.sca_residual(P.handle, x, r)
    # one coordinate per group (w.n groups >= any draw), each reading the residual after all
    # earlier ones
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed, delay_chunks=w.n,
                      delay_stale=0)
    xo = np.zeros(w.n)
    ro = O.residual(prob, xo)
    for k in range(0, 12, 3):
        sca.sca_step(P.handle, o, k, 3, x, r)
        xo, ro, _ = O.run_rounds(prob, cfg, xo, ro, k, 3)
        ex, er = _rel(x.cpu().numpy(), xo), _rel(r.cpu().numpy(), ro)
        print(f"[parity] after {k + 3} rounds: x {ex:.2e} r {er:.2e}", flush=True)
        assert ex <= 1e-10 and er <= 1e-10
    P.close()


def _minimiser(w):
    prob = _oracle(w)
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=1.0, seed=0)
    out = O.solve(prob, cfg, max_rounds=20000, check_every=20, tol_merit=1e-12)
    return prob, out["x"], out["F"]


def test_many_workgroups_reach_the_lasso_minimiser_fp64():
    w = inputs.dense_problem(200, 1000, nnz_frac=0.05, lam_frac=0.1, block=1, p=1.0,
                             dtype=torch.float64, seed=22)
    prob, xs, Fs = _minimiser(w)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    finals = []
    for W in (8, 64, 256, 64):
        o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=1.0, seed=3, max_rounds=20000,
                          check_every=20, tol_rel_obj=1e-12, F_star=Fs, async_workgroups=W)
        x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
        st = sca.sca_solve(P.handle, o, x, raise_on_notconv=False)
        xg = x.cpu().numpy()
        print(f"[gpu] lock-free W={W}: {st['rounds']} rounds, rel err {st['rel_err']:.2e}, "
              f"|x - x*| {np.max(np.abs(xg - xs)):.2e}", flush=True)
        assert st["status"] == sca.SCA_OK and st["rel_err"] <= 1e-12
        # the objective pins the minimiser only to about sqrt of its own accuracy along the
        # flattest direction: 9e-6 here for both the lock-free and the synchronous solves
        assert np.max(np.abs(xg - xs)) <= 5e-5
        assert abs(O.objective(prob, xg) - Fs) <= 1e-11 * abs(Fs)
        finals.append(xg)
    # the race changes the rounding, not the limit
    assert np.max(np.abs(finals[1] - finals[3])) <= 5e-5
    P.close()


def test_objective_falls_over_lock_free_rounds_fp64():
    w = inputs.dense_problem(400, 2000, nnz_frac=0.03, lam_frac=0.05, block=8, p=0.5,
                             dtype=torch.float64, seed=23)
    prob = _oracle(w)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=5, async_workgroups=128)
    x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    r = torch.empty(w.m, dtype=torch.float64, device="cuda")
    sca.sca_residual(P.handle, x, r)
    Fs = [O.objective(prob, np.zeros(w.n))]
    for k in range(0, 200, 20):
        sca.sca_step(P.handle, o, k, 20, x, r)
        Fs.append(O.objective(prob, x.cpu().numpy()))
    print(f"[gpu] lock-free W=128 objective every 20 rounds: {['%.6g' % f for f in Fs]}",
          flush=True)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(Fs, Fs[1:]))
    # the running residual kept by the atomic folds is the residual of x
    ro = O.residual(prob, x.cpu().numpy())
    assert _rel(r.cpu().numpy(), ro) <= 1e-10
    P.close()


def test_lock_free_fp32_reaches_the_tolerance():
    w = inputs.lasso_dense_fp32(m=2000, n=8000, seed=24)
    prob = _oracle(w)
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
    Fs = O.solve(prob, cfg, max_rounds=20000, check_every=20, tol_merit=1e-11)["F"]
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, max_rounds=20000,
                      check_every=10, tol_rel_obj=1e-5, F_star=Fs, async_workgroups=512)
    x = torch.zeros(w.n, dtype=torch.float32, device="cuda")
    st = sca.sca_solve(P.handle, o, x)
    print(f"[gpu] lock-free FP32 W=512: {st['rounds']} rounds, rel err {st['rel_err']:.2e}",
          flush=True)
    assert st["status"] == sca.SCA_OK and st["rel_err"] <= 1e-5
    P.close()


def test_lock_free_rounds_are_refused_where_they_do_not_apply():
    w = inputs.dense_problem(64, 128, nnz_frac=0.1, lam_frac=0.1, block=4, p=0.5,
                             dtype=torch.float64, seed=25)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    r = torch.empty(w.m, dtype=torch.float64, device="cuda")
    for kw in (dict(async_workgroups=65537), dict(async_workgroups=-1),
               dict(async_workgroups=4, delay_chunks=4)):
        with pytest.raises(sca.SCAError) as e:
            sca.sca_step(P.handle, sca.make_opts(gamma=0.9, tau=w.tau, select_p=0.5, **kw), 0, 1,
                         x, r)
        assert e.value.status == sca.SCA_EINVAL
    P.close()
    sw = inputs.sparse_problem(200, 400, per_col=4, nnz_frac=0.05, block=4, p=0.5,
                               dtype=torch.float64, seed=26).to("cuda")
    SP = sca.Problem.from_workload(sw)
    xs = torch.zeros(sw.n, dtype=torch.float64, device="cuda")
    rs = torch.empty(sw.m, dtype=torch.float64, device="cuda")
    with pytest.raises(sca.SCAError) as e:
        sca.sca_step(SP.handle, sca.make_opts(gamma=0.9, tau=sw.tau, select_p=0.5,
                                              async_workgroups=4), 0, 1, xs, rs)
    assert e.value.status == sca.SCA_EINVAL
    SP.close()
    ws = inputs.batch_lasso(2, m_range=(50, 80), n_ratio=2, nnz_frac=0.05, block=8, p=0.5,
                            dtype=torch.float64, seed=27)
    B = sca.Batch([v.to("cuda") for v in ws])
    xb = torch.zeros(int(B.xoff[-1]), dtype=torch.float64, device="cuda")
    rb = torch.zeros(int(B.roff[-1]), dtype=torch.float64, device="cuda")
    with pytest.raises(sca.SCAError) as e:
        sca.sca_batch_step(B.handle, sca.make_opts(gamma=0.9, select_p=0.5, async_workgroups=4),
                           0, 1, xb, rb)
    assert e.value.status == sca.SCA_EINVAL
    B.close()
