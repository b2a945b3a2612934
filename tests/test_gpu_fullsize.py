"""Parity at the full configuration sizes, in the launch configuration the benchmark uses
(the installed tuning table).  The oracle runs the first rounds on the host copy of the
same data (20 rounds of the dense workloads, 10 of the sparse one and of the sampled batch
instances and right-hand sides), compared after every round.

FP32 tolerances: the objective within 1e-4 relative (the stated FP32 target), the iterates
within x_tol(terms) of max(1, ||x||_inf), terms = the products of one partial gradient (m
dense, the column's nonzeros sparse); x_tol is derived in fp32_tolerance.py.
Round 1 is also checked one coordinate at a time: from x^0 = 0, x^1_j = gamma *
clip(soft(a_j^T b / q_j, lam / q_j)) for the drawn j and 0 elsewhere."""

import numpy as np
import pytest
import torch

from oracle import sca_oracle as O
from paper_1701_04900_amd import inputs, sca
from fp32_tolerance import x_tol

# the oracle's FP64 rounds over 2-8 GB of A take seconds each on the host
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def _compare_rounds(name, w, prob, gpu, cfg, rounds, terms=None):
    """Run the oracle for the same rounds and compare every round; print all errors first
    (so a failure shows the whole trajectory), then assert."""
    x = np.zeros(w.n)
    r = O.residual(prob, x)
    ex, eF = [], []
    for k in range(rounds):
        x, r, _ = O.run_rounds(prob, cfg, x, r, k, 1)
        Fo = O.objective(prob, x, r)
        ex.append(_rel(gpu[k][0], x))
        eF.append(abs(gpu[k][1] - Fo) / abs(Fo))
        print(f"[parity] {name} round {k + 1}: x err {ex[-1]:.2e}, F rel err {eF[-1]:.2e}",
              flush=True)
    tol = x_tol(w.m if terms is None else terms)
    print(f"[parity] {name}: max x err {max(ex):.2e} (tolerance {tol:.2e}), max F rel err "
          f"{max(eF):.2e} (tolerance 1e-4)", flush=True)
    assert max(ex) <= tol
    assert max(eF) <= 1e-4
    return x


def _gpu_rounds(w, P, rounds):
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, instance=w.instance)
    x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
    r = torch.empty(w.m, dtype=w.dtype, device="cuda")
    sca.sca_residual(P.handle, x, r)
    out = []
    for k in range(rounds):
        sca.sca_step(P.handle, o, k, 1, x, r)
        F = sca.sca_objective(P.handle, o, x)["F"]  # fresh FP64 residual on the GPU
        out.append((x.double().cpu().numpy(), F))
    return out, o, x


def _first_round_one_by_one(w, prob, xg1, nsample=3000):
    """x^1_j recomputed for sampled coordinates from the definition (x^0 = 0, r^0 = -b)."""
    bp = prob.blocks()
    drawn = O.selected_blocks(w.seed, 0, w.instance, len(bp) - 1, w.p)
    is_drawn = np.zeros(w.n, dtype=bool)
    is_drawn[O.block_columns(bp, drawn)] = True
    rng = np.random.default_rng(0)
    js = rng.choice(w.n, size=min(nsample, w.n), replace=False)
    b = np.asarray(prob.b, dtype=np.float64)
    for j in js:
        a = np.asarray(prob.cols([j]), dtype=np.float64).ravel() if not hasattr(prob.cols([j]), "toarray") \
            else prob.cols([j]).toarray().ravel()
        q = float(a @ a) + w.tau
        g = float(a @ (-b))
        xh = float(O.best_response_1d(0.0, g, q, w.lam, w.beta))
        expect = w.gamma * xh if is_drawn[j] else 0.0
        assert abs(xg1[j] - expect) <= 1e-5 * max(1.0, abs(expect)), (j, xg1[j], expect)


def test_lasso_20000x100000_fp32_full_size():
    print("[gpu] full-size dense LASSO 20000x100000 FP32", flush=True)
    w = inputs.lasso_dense_fp32(device="cuda")
    P = sca.Problem.from_workload(w)
    gpu, _, _ = _gpu_rounds(w, P, 20)
    At = w.At.cpu()
    prob = O.Problem(A=At[:, : w.m].numpy().T, b=w.b.double().cpu().numpy(), lam=w.lam,
                     block_ptr=w.block_ptr)
    _first_round_one_by_one(w, prob, gpu[0][0])
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
    _compare_rounds("full-size LASSO", w, prob, gpu, cfg, 20)
    P.close()


def test_nonconvex_box_10000x50000_fp32_full_size():
    print("[gpu] full-size box-nonconvex 10000x50000 FP32", flush=True)
    w = inputs.nonconvex_box_fp32(device="cuda")
    P = sca.Problem.from_workload(w)
    gpu, _, _ = _gpu_rounds(w, P, 20)
    At = w.At.cpu()
    prob = O.Problem(A=At[:, : w.m].numpy().T, b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
    _compare_rounds("full-size box-nonconvex", w, prob, gpu, cfg, 20)
    assert np.max(np.abs(gpu[-1][0])) <= 1.0
    P.close()


def test_sparse_lasso_100000x1000000_fp32_full_size():
    print("[gpu] full-size sparse LASSO 1e5 x 1e6, 1e8 nonzeros, FP32", flush=True)
    w = inputs.sparse_lasso_fp32(device="cuda")
    P = sca.Problem.from_workload(w)
    gpu, _, _ = _gpu_rounds(w, P, 10)
    prob = O.Problem(A=w.scipy_csr().tocsc(), b=w.b.double().cpu().numpy(), lam=w.lam,
                     block_ptr=w.block_ptr)
    _first_round_one_by_one(w, prob, gpu[0][0], nsample=500)
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
    _compare_rounds("full-size sparse LASSO", w, prob, gpu, cfg, 10, terms=w.nnz // w.n)
    P.close()


def test_batch_256_full_size_sampled_instances():
    print("[gpu] full-size batch of 256 instances (117.6 GB of A), FP32", flush=True)
    ws = inputs.batch_lasso(256, m_range=(500, 8000), nnz_frac=0.02, lam_range=(1e-3, 1e-1),
                            block=64, p=0.25, dtype=torch.float32, seed=0, device="cuda")
    B = sca.Batch(ws)
    o = sca.make_opts(gamma=0.9, select_p=0.25, seed=0)
    x = torch.zeros(int(B.xoff[-1]), dtype=torch.float32, device="cuda")
    r = torch.zeros(int(B.roff[-1]), dtype=torch.float32, device="cuda")
    sca.sca_batch_residual(B.handle, x, r)
    rounds = 10
    per_round = []
    for k in range(rounds):
        sca.sca_batch_step(B.handle, o, k, 1, x, r)
        Fg_all = sca.sca_batch_objective(B.handle, o, x, B.K)["F"]
        per_round.append((x.double().cpu().numpy(), Fg_all))
    for k in (0, 97, 255):  # smallest lam, a middle one, largest lam
        w = ws[k]
        prob = O.Problem(A=w.At[:, : w.m].cpu().numpy().T, b=w.b.double().cpu().numpy(),
                         lam=w.lam, block_ptr=w.block_ptr)
        cfg = O.RunConfig(tau=w.tau, gamma=0.9, p=0.25, seed=0, instance=k)
        gpu = [(xa[B.xoff[k]:B.xoff[k + 1]], Fa[k]) for xa, Fa in per_round]
        _compare_rounds(f"full-size batch instance {k} (m={w.m})", w, prob, gpu, cfg, rounds)
    B.close()


def test_multi_rhs_20000x100000_K64_fp32_full_size():
    print("[gpu] full-size multi right-hand sides: 64 lambdas over the 20000x100000 FP32 LASSO",
          flush=True)
    w = inputs.multi_rhs_problem(20000, 100000, 64, rhs="sweep", lam_range=(0.005, 0.05),
                                 nnz_frac=0.01, block=64, p=0.25, dtype=torch.float32, seed=0,
                                 device="cuda")
    M = sca.Multi(w.At, w.m, w.B, w.lams, w.c, w.beta, w.block_ptr)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
    X = M.zeros_x()
    R = M.empty_r()
    sca.sca_multi_residual(M.handle, X, R)
    rounds = 5
    per_round = []
    for k in range(rounds):
        sca.sca_multi_step(M.handle, o, k, 1, X, R)
        per_round.append((X.double().cpu().numpy(), sca.sca_multi_objective(M.handle, o, X, w.K)["F"]))
    X1 = per_round[0][0]
    A32 = w.At.cpu()[:, : w.m].numpy().T
    for k in (0, 32, 63):
        wk = inputs.DenseWorkload(w.name, w.At, w.m, w.n, w.lda, w.B[k, : w.m], w.base.x_true,
                                  float(w.lams[k]), w.c, w.beta, w.tau, w.block_ptr, w.p,
                                  w.gamma, w.seed)
        prob = O.Problem(A=A32, b=w.B[k, : w.m].double().cpu().numpy(), lam=float(w.lams[k]),
                         block_ptr=w.block_ptr)
        _first_round_one_by_one(wk, prob, X1[k], nsample=1000)
        cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
        gpu = [(Xa[k], Fa[k]) for Xa, Fa in per_round]
        _compare_rounds(f"multi full-size problem {k}", wk, prob, gpu, cfg, rounds)
    M.close()
