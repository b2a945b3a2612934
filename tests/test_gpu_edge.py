"""GPU parity on the degenerate and boundary cases of the method, through the two-pass round
(launch kind 1) and the fused round (kind 4), against the FP64 oracle:

* rounds that draw no block (p ~ 1e-9): x and r must not change, no update is counted;
* lambda above ||A^T b||_inf from x = 0: every best response is 0, x stays exactly 0;
* one row, one column, a single block holding every coordinate;
* orthonormal columns with tau = 0 and gamma = 1: one round is the soft-threshold of A^T b
  (closed form), and it is a fixed point;
* a box bound that most coordinates hit (nonconvex c > 0);
* about 20000 drawn columns per round (the drawn list written by the whole grid), dense
  and sparse, and more drawn blocks than the selection's shared list holds.

FP64 tolerance 1e-10 relative, as for the other dense tests."""
import math

import numpy as np
import pytest
import torch

from oracle import sca_oracle as O
from paper_1701_04900_amd import inputs, sca
from fp32_tolerance import x_tol

pytestmark = pytest.mark.gpu

KINDS = {"two_pass": (1, 4, 4, 2), "fused": (4, 2, 1, 1)}


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b))))) if b.size else 0.0


def _oracle(w):
    return O.Problem(A=w.A_numpy(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)


class Run:
    def __init__(self, w, kind, **optkw):
        print(f"[gpu] edge case {w.name} m={w.m} n={w.n} p={w.p} launch={kind}", flush=True)
        self.w = w.to("cuda")
        self.P = sca.Problem.from_workload(self.w)
        sca.sca_problem_set_launch(self.P.handle, *KINDS[kind])
        kw = dict(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
        kw.update(optkw)
        self.kw = kw
        self.opts = sca.make_opts(**kw)
        self.x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
        self.r = torch.empty(w.m, dtype=w.dtype, device="cuda")
        sca.sca_residual(self.P.handle, self.x, self.r)
        self.k = 0

    def step(self, n):
        sca.sca_step(self.P.handle, self.opts, self.k, n, self.x, self.r)
        self.k += n
        torch.cuda.synchronize()
        return self.x.cpu().numpy(), self.r.cpu().numpy()


def _oracle_rounds(w, prob, rounds, **cfgkw):
    kw = dict(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
    kw.update(cfgkw)
    x = np.zeros(w.n)
    x, r, upd = O.run_rounds(prob, O.RunConfig(**kw), x, O.residual(prob, x), 0, rounds)
    return x, r, upd


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_rounds_without_a_drawn_block_change_nothing(kind):
    w = inputs.dense_problem(300, 900, nnz_frac=0.02, lam_frac=0.01, block=64, p=1e-9,
                             dtype=torch.float64, seed=41)
    prob = _oracle(w)
    xo, ro, upd = _oracle_rounds(w, prob, 20)
    assert upd == 0 and not np.any(xo)
    run = Run(w, kind)
    r0 = run.r.clone()
    xg, rg = run.step(20)
    assert not np.any(xg)
    assert torch.equal(run.r, r0)
    assert _rel(rg, ro) <= 1e-10
    o = sca.make_opts(**run.kw, max_rounds=20, check_every=10)
    st = sca.sca_solve(run.P.handle, o, torch.zeros_like(run.x), raise_on_notconv=False)
    assert st["rounds"] == 20 and st["coord_updates"] == 0 and st["moved_updates"] == 0


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_lambda_above_the_max_correlation_keeps_x_zero(kind):
    w = inputs.dense_problem(400, 1200, nnz_frac=0.02, lam_frac=1.01, block=32, p=1.0,
                             dtype=torch.float64, seed=42)
    prob = _oracle(w)
    xo, _, _ = _oracle_rounds(w, prob, 10)
    assert not np.any(xo)
    run = Run(w, kind)
    xg, rg = run.step(10)
    assert not np.any(xg)
    assert np.array_equal(rg, -w.b.cpu().numpy())


@pytest.mark.parametrize("kind", sorted(KINDS))
@pytest.mark.parametrize("m,n,block,p", [(1, 7, 7, 1.0), (3, 1, 1, 1.0), (1, 1, 1, 1.0),
                                         (5, 40, 40, 0.5), (2, 33, 4, 0.5)])
def test_tiny_shapes_and_a_single_block(kind, m, n, block, p):
    w = inputs.dense_problem(m, n, nnz_frac=0.2, lam_frac=0.05, block=block, p=p,
                             dtype=torch.float64, seed=43 + m + n)
    prob = _oracle(w)
    run = Run(w, kind)
    for k0 in range(0, 30, 10):
        xg, rg = run.step(10)
        xo, ro, _ = _oracle_rounds(w, prob, k0 + 10)
        assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10, k0


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_orthonormal_columns_one_round_is_the_soft_threshold(kind):
    w = inputs.orthogonal_problem(96, 40, lam=0.3, gamma=1.0, p=1.0, block=1, seed=44)
    run = Run(w, kind)
    xg, _ = run.step(1)
    A = w.A_numpy()
    c = A.T @ w.b.cpu().numpy()
    soft = np.sign(c) * np.maximum(np.abs(c) - 0.3, 0.0)
    assert np.max(np.abs(xg - soft)) <= 1e-13
    xg2, _ = run.step(3)  # the soft-threshold of A^T b is the minimiser: a fixed point
    assert np.max(np.abs(xg2 - soft)) <= 1e-13


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_box_bound_hit_by_most_coordinates(kind):
    w = inputs.dense_problem(500, 1500, nnz_frac=0.3, amp=(1.0, 2.0), lam_frac=0.001,
                             c_frac=0.5, beta=0.05, block=16, p=0.5, dtype=torch.float64,
                             seed=45)
    prob = _oracle(w)
    run = Run(w, kind)
    xg, rg = run.step(25)
    xo, ro, _ = _oracle_rounds(w, prob, 25)
    assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10
    assert np.max(np.abs(xg)) <= 0.05
    assert np.mean(np.abs(np.abs(xg) - 0.05) < 1e-12) > 0.3  # most drawn coordinates at the box


@pytest.mark.parametrize("block,p", [(32, 0.6), (1, 0.5)])
def test_long_drawn_lists_two_pass(block, p):
    """About 20000 drawn columns per round: the draw lists the drawn blocks and a grid-wide
    kernel writes their columns (block 32), or, with more drawn blocks than the shared list
    holds (scalar blocks), the draw writes the columns itself."""
    w = inputs.dense_problem(64, 40000, nnz_frac=0.01, lam_frac=0.02, block=block, p=p,
                             dtype=torch.float64, seed=46)
    prob = _oracle(w)
    run = Run(w, "two_pass")
    for k0 in range(0, 9, 3):
        xg, rg = run.step(3)
        xo, ro, _ = _oracle_rounds(w, prob, k0 + 3)
        assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10, k0


def test_long_drawn_list_sparse():
    w = inputs.sparse_problem(600, 40000, per_col=6, nnz_frac=0.01, lam_frac=0.02, block=64,
                              p=0.5, dtype=torch.float64, seed=47)
    prob = O.Problem(A=w.scipy_csr().tocsc(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
    x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    r = torch.empty(w.m, dtype=torch.float64, device="cuda")
    sca.sca_residual(P.handle, x, r)
    sca.sca_step(P.handle, o, 0, 6, x, r)
    torch.cuda.synchronize()
    xo, ro, _ = _oracle_rounds(w, prob, 6)
    assert _rel(x.cpu().numpy(), xo) <= 1e-10 and _rel(r.cpu().numpy(), ro) <= 1e-10


@pytest.mark.parametrize("kind,dtype", [("fused", torch.float64), ("fused", torch.float32),
                                        ("two_pass", torch.float64)])
def test_padding_rows_of_A_never_reach_a_result(kind, dtype):
    """A's rows m..lda-1 filled with NaN (lda = 1004 for m = 1001): the kernels that load
    whole 16-byte row groups must zero or discard them."""
    w = inputs.dense_problem(1001, 3000, nnz_frac=0.02, lam_frac=0.02, block=32, p=0.5,
                             dtype=dtype, seed=48)
    assert w.lda > w.m
    prob = _oracle(w)
    w.At[:, w.m:] = float("nan")
    run = Run(w, kind)
    xg, rg = run.step(10)
    assert np.all(np.isfinite(xg)) and np.all(np.isfinite(rg))
    xo, ro, _ = _oracle_rounds(w, prob, 10)
    tol = 1e-10 if dtype == torch.float64 else x_tol(w.m)
    print(f"[parity] padding rows {kind} {dtype}: x err {_rel(xg, xo):.2e}, r err {_rel(rg, ro):.2e}", flush=True)
    assert _rel(xg, xo) <= tol and _rel(rg, ro) <= tol
    rep = sca.sca_objective(run.P.handle, run.opts, run.x)
    assert math.isfinite(rep["F"]) and math.isfinite(rep["merit"])
