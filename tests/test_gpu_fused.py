"""GPU parity of the fused dense round (gradient, best response and fold in one pass over
the drawn columns, one 1024-thread workgroup per compute unit holding whole columns,
launch kind 4) against the FP64 CPU oracle, and against the two-pass round.

The cases force the fused kind through sca_problem_set_launch and cover one to the
largest number of 16-byte row groups per thread (Q) for each dtype, column groups C of
1 to 8, ragged last row groups (m not a multiple of the vector width), fewer drawn
coordinates than workgroups, every block drawn, the box-constrained nonconvex problem,
the DC regularisers and the diminishing step.  Tolerances as for the dense path: FP64
1e-10 relative, FP32 objective 1e-4."""
import math

import numpy as np
import pytest
import torch

from oracle import sca_oracle as O
from paper_1701_04900_amd import inputs, sca
from fp32_tolerance import x_tol

pytestmark = pytest.mark.gpu

FUSED = 4


def _oracle(w, **kw):
    return O.Problem(A=w.A_numpy(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr, **kw)


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b))))) if b.size else 0.0


class Run:
    def __init__(self, w, cols=None, reg=None, theta=0.0, **optkw):
        self.w = w.to("cuda")
        self.P = sca.Problem.from_workload(self.w)
        if cols is not None:
            sca.sca_problem_set_launch(self.P.handle, FUSED, cols, 1, 1)
        self.launch = sca.sca_problem_get_launch(self.P.handle)
        print(f"[gpu] fused workload {w.name} m={w.m} n={w.n} dtype={w.dtype} p={w.p} "
              f"launch={self.launch}", flush=True)
        if reg is not None:
            sca.sca_problem_set_regularizer(self.P.handle, reg, theta)
        kw = dict(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, instance=w.instance)
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


def _trajectory(w, prob, rounds, every, **cfgkw):
    kw = dict(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed, instance=w.instance)
    kw.update(cfgkw)
    cfg = O.RunConfig(**kw)
    x = np.zeros(w.n)
    r = O.residual(prob, x)
    out = []
    for k in range(0, rounds, every):
        x, r, _ = O.run_rounds(prob, cfg, x, r, k, every)
        out.append((x.copy(), r.copy()))
    return out


def _q(m, dtype):
    """16-byte row groups per thread of a 1024-thread workgroup for an m-row column."""
    vn = 4 if dtype == torch.float32 else 2
    groups = (m + vn - 1) // vn
    return (groups + 1023) // 1024


# (m, n, block, p, cols): Q = 1, 2, 3 for FP64 (2 rows per 16 bytes), ragged tails,
# S < 256 workgroups (64 x 300), every block drawn, the largest all-register FP64 m (6144);
# then 3 row groups in registers and 1, 2, 3 in LDS (6145, 9999 ragged, 12288 the largest)
FP64_CASES = [(517, 2050, 7, 1.0, 4), (2049, 3001, 64, 0.4, 2), (4097, 2500, 32, 0.3, 2),
              (5999, 2000, 32, 0.3, 1), (6144, 1500, 16, 0.5, 1), (64, 300, 1, 0.2, 4),
              (1500, 4000, 64, 0.25, 1), (6145, 1500, 16, 0.5, 1), (9999, 1200, 32, 0.4, 1),
              (12288, 1000, 16, 0.5, 1)]


@pytest.mark.parametrize("m,n,block,p,cols", FP64_CASES)
def test_fused_fp64_matches_oracle(m, n, block, p, cols):
    w = inputs.dense_problem(m, n, nnz_frac=0.01, lam_frac=0.01, block=block, p=p,
                             dtype=torch.float64, seed=m)
    prob = _oracle(w)
    run = Run(w, cols=cols)
    assert run.launch["grad_kind"] == FUSED
    assert _q(m, torch.float64) <= 6
    for i, (xo, ro) in enumerate(_trajectory(w, prob, 30, 5)):
        xg, rg = run.step(5)
        assert _rel(xg, xo) <= 1e-10, (i, _rel(xg, xo))
        assert _rel(rg, ro) <= 1e-10, (i, _rel(rg, ro))


def test_fused_with_separate_block_draw_fp64():
    """More blocks than the in-kernel draw takes (40000 scalar blocks > 32768): the drawn
    list comes from the separate selection kernel, the fused kernel does S.2-S.5."""
    w = inputs.dense_problem(300, 40000, nnz_frac=0.01, lam_frac=0.02, block=1, p=0.05,
                             dtype=torch.float64, seed=31)
    assert len(w.block_ptr) - 1 == 40000
    prob = _oracle(w)
    run = Run(w, cols=4)
    for xo, ro in _trajectory(w, prob, 12, 4):
        xg, rg = run.step(4)
        assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10


def test_fused_moved_count_matches_oracle_fp64():
    w = inputs.dense_problem(1201, 3000, nnz_frac=0.02, lam_frac=0.02, block=16, p=0.5,
                             dtype=torch.float64, seed=21)
    prob = _oracle(w)
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
    x = np.zeros(w.n)
    r = O.residual(prob, x)
    bp = prob.blocks()
    moved = drawn = 0
    for k in range(12):
        mask = O.selected_blocks(cfg.seed, k, cfg.instance, len(bp) - 1, cfg.p)
        idx = O.block_columns(bp, mask)
        x, r, mv = O.sca_round(prob, x, r, cfg.tau, cfg.gamma, idx)
        moved += mv
        drawn += len(idx)
    run = Run(w, cols=2)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, max_rounds=12,
                      check_every=12)
    xg = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    st = sca.sca_solve(run.P.handle, o, xg, raise_on_notconv=False)
    assert st["rounds"] == 12
    assert st["coord_updates"] == drawn
    assert st["moved_updates"] == moved
    assert _rel(xg.cpu().numpy(), x) <= 1e-10


def test_fused_nonconvex_box_fp64():
    w = inputs.nonconvex_box_fp32(m=3001, n=4000, dtype=torch.float64, seed=2)
    assert w.c > 0.4 and w.beta == 1.0
    prob = _oracle(w)
    run = Run(w, cols=2)
    for xo, ro in _trajectory(w, prob, 40, 10):
        xg, rg = run.step(10)
        assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10


@pytest.mark.parametrize("reg,code", [("log", sca.SCA_REG_LOG), ("exp", sca.SCA_REG_EXP)])
def test_fused_dc_regularisers_fp64(reg, code):
    w = inputs.dense_problem(1800, 3000, nnz_frac=0.05, lam_frac=0.02, block=16, p=0.5,
                             dtype=torch.float64, seed=4)
    prob = _oracle(w, reg=reg, theta=20.0)
    run = Run(w, cols=2, reg=code, theta=20.0)
    for xo, ro in _trajectory(w, prob, 30, 10):
        xg, rg = run.step(10)
        assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10


def test_fused_diminishing_stepsize_fp64():
    w = inputs.dense_problem(2600, 2400, nnz_frac=0.02, lam_frac=0.02, block=32, p=0.5,
                             dtype=torch.float64, seed=6)
    prob = _oracle(w)
    run = Run(w, cols=1, gamma=1.0, gamma_mu=1e-2)
    for xo, ro in _trajectory(w, prob, 40, 8, gamma=1.0, gamma_mu=1e-2):
        xg, rg = run.step(8)
        assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10


# FP32 (4 rows per 16 bytes): Q = 1 (C = 8), 2 (C = 4), 3 (C = 2), 4, and the largest
# all-register m (5 groups per thread, 20480 rows) with a ragged tail (16389 = 4 * 4097 + 1);
# then 4 groups in registers and 2 or 3 in LDS (20481, 24001 ragged, 28672 the largest)
@pytest.mark.parametrize("m,n,cols", [(3000, 4000, 8), (5001, 3000, 4), (10000, 2500, 2),
                                      (13000, 1500, 1), (16389, 1500, 1), (20480, 1200, 1),
                                      (20481, 1200, 1), (24001, 1000, 1), (28672, 1000, 1)])
def test_fused_fp32_objective(m, n, cols):
    w = inputs.lasso_dense_fp32(m=m, n=n, seed=5)
    prob = _oracle(w)
    run = Run(w, cols=cols)
    assert run.launch["grad_kind"] == FUSED
    for xo, _ in _trajectory(w, prob, 30, 10):
        xg, _ = run.step(10)
        Fo = O.objective(prob, xo)
        Fg = sca.sca_objective(run.P.handle, run.opts, run.x)["F"]
        assert abs(Fg - Fo) <= 1e-4 * abs(Fo), (run.k, Fg, Fo)
        print(f"[parity] fused fp32 {m}x{n} round {run.k}: x err {_rel(xg, xo):.2e}", flush=True)
        assert _rel(xg, xo) <= x_tol(m), (run.k, _rel(xg, xo))


@pytest.mark.parametrize("dtype,m", [(torch.float64, 3001), (torch.float32, 9001)])
def test_fused_equals_two_pass_round(dtype, m):
    """Same rounds through the fused kind and through the two-pass kind (1, 4, 4, 2)."""
    w = inputs.dense_problem(m, 5000, nnz_frac=0.01, lam_frac=0.01, block=64, p=0.25,
                             dtype=dtype, seed=7)
    a = Run(w, cols=2)
    b = Run(w)
    sca.sca_problem_set_launch(b.P.handle, 1, 4, 4, 2)
    xa, ra = a.step(25)
    xb, rb = b.step(25)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert _rel(xa, xb) <= tol and _rel(ra, rb) <= tol


def test_fused_determinism_resume_and_graph_solve():
    w = inputs.dense_problem(4001, 6000, nnz_frac=0.01, lam_frac=0.01, block=64, p=0.3,
                             dtype=torch.float32, seed=8)
    a = Run(w, cols=2)
    a.step(20)
    b = Run(w, cols=2)
    b.step(7)
    b.step(13)
    assert torch.equal(a.x, b.x) and torch.equal(a.r, b.r)
    # the captured solve replays the same kernels: identical iterate after the same rounds
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, max_rounds=20,
                      check_every=10)
    xs = torch.zeros(w.n, dtype=w.dtype, device="cuda")
    st = sca.sca_solve(a.P.handle, o, xs, raise_on_notconv=False)
    assert st["rounds"] == 20
    assert torch.equal(xs, a.x)


def test_fused_rejected_where_columns_do_not_fit():
    cases = [(torch.float64, 12289), (torch.float32, 28673)]
    for dtype, m in cases:
        w = inputs.dense_problem(m, 64, nnz_frac=0.05, block=8, p=0.5, dtype=dtype,
                                 seed=9).to("cuda")
        P = sca.Problem.from_workload(w)
        before = sca.sca_problem_get_launch(P.handle)
        with pytest.raises(sca.SCAError) as e:
            sca.sca_problem_set_launch(P.handle, FUSED, 1, 1, 1)
        assert e.value.status == sca.SCA_EINVAL
        assert sca.sca_problem_get_launch(P.handle) == before
        P.close()
    ws = inputs.sparse_problem(500, 2000, per_col=5, nnz_frac=0.01, block=64, p=0.5,
                               dtype=torch.float64, seed=4).to("cuda")
    Ps = sca.Problem.from_workload(ws)
    with pytest.raises(sca.SCAError) as e:
        sca.sca_problem_set_launch(Ps.handle, FUSED, 1, 1, 1)
    assert e.value.status == sca.SCA_EINVAL
    Ps.close()
    # shapes outside the kind's list
    w = inputs.dense_problem(300, 500, nnz_frac=0.05, block=8, p=0.5, dtype=torch.float64,
                             seed=10).to("cuda")
    P = sca.Problem.from_workload(w)
    for shape in ((FUSED, 3, 1, 1), (FUSED, 1, 2, 1), (FUSED, 1, 1, 2)):
        with pytest.raises(sca.SCAError):
            sca.sca_problem_set_launch(P.handle, *shape)
    # a column group larger than the registers allow is reduced to the largest that fits
    sca.sca_problem_set_launch(P.handle, FUSED, 8, 1, 1)
    assert sca.sca_problem_get_launch(P.handle)["grad_cols"] == 4
    P.close()


@pytest.mark.parametrize("dtype,m", [(torch.float64, 9999), (torch.float32, 24001)])
def test_fused_lds_row_groups_ignore_nan_padding_rows(dtype, m):
    """Columns that spill into the LDS row groups: A's rows m..lda-1 (in the last, LDS
    held, row group) set to NaN never reach x, r or the objective."""
    w = inputs.dense_problem(m, 800, nnz_frac=0.02, lam_frac=0.02, block=16, p=0.5,
                             dtype=dtype, seed=m % 97)
    assert w.lda > w.m
    prob = _oracle(w)
    w.At[:, w.m:] = float("nan")
    run = Run(w, cols=1)
    assert run.launch["grad_kind"] == FUSED
    xo, ro = _trajectory(w, prob, 10, 10)[-1]
    xg, rg = run.step(10)
    assert np.all(np.isfinite(xg)) and np.all(np.isfinite(rg))
    tol = 1e-10 if dtype == torch.float64 else x_tol(m)
    print(f"[parity] fused LDS rows {dtype} m={m}: x err {_rel(xg, xo):.2e}", flush=True)
    assert _rel(xg, xo) <= tol and _rel(rg, ro) <= tol
