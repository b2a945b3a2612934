"""GPU parity of the rounds that draw the blocks inside their kernels (the fused dense round
and the sparse panel-split gradient) on block partitions of unequal sizes, where the
kernels read the block bounds from the device copy of block_ptr, and on equal blocks with
a short last one, where they compute the bounds instead.  Both against the FP64 oracle
run with the same block_ptr: iterates and residuals within 1e-10 relative."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import sca_oracle as O
from paper_1701_04900_amd import inputs, sca

pytestmark = pytest.mark.gpu

FUSED = 4


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def _irregular_blocks(n, lo, hi, seed):
    """Consecutive blocks of seeded lengths in [lo, hi] covering n coordinates."""
    rng = np.random.default_rng(seed)
    lens = []
    while sum(lens) < n:
        lens.append(int(min(rng.integers(lo, hi + 1), n - sum(lens))))
    return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


def _run(w, prob, launch=None, rounds=12):
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    if launch is not None:
        sca.sca_problem_set_launch(P.handle, *launch)
    print(f"[gpu] blocks={len(w.block_ptr) - 1} m={w.m} n={w.n} "
          f"launch={sca.sca_problem_get_launch(P.handle)}", flush=True)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
    x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    r = torch.empty(w.m, dtype=torch.float64, device="cuda")
    sca.sca_residual(P.handle, x, r)
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
    xo = np.zeros(w.n)
    ro = O.residual(prob, xo)
    for k in range(0, rounds, 4):
        sca.sca_step(P.handle, o, k, 4, x, r)
        xo, ro, _ = O.run_rounds(prob, cfg, xo, ro, k, 4)
        ex, er = _rel(x.cpu().numpy(), xo), _rel(r.cpu().numpy(), ro)
        print(f"[parity] after {k + 4} rounds: x {ex:.2e} r {er:.2e}", flush=True)
        assert ex <= 1e-10 and er <= 1e-10
    assert np.count_nonzero(xo) > 0
    P.close()


@pytest.mark.parametrize("blocks", ["irregular", "equal_short_last"])
@pytest.mark.parametrize("launch", [(FUSED, 1, 1, 1), (1, 4, 4, 2)])
def test_dense_rounds_on_block_partitions_fp64(blocks, launch):
    w = inputs.dense_problem(700, 2300, nnz_frac=0.05, lam_frac=0.05, block=24, p=0.4,
                             dtype=torch.float64, seed=41)
    if blocks == "irregular":
        w = dataclasses.replace(w, block_ptr=_irregular_blocks(w.n, 1, 57, seed=3))
    else:
        assert (w.block_ptr[-1] - w.block_ptr[-2]) < 24  # 2300 = 95 * 24 + 20
    prob = O.Problem(A=w.A_numpy(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)
    _run(w, prob, launch)


@pytest.mark.parametrize("blocks", ["irregular", "one_long_last"])
def test_sparse_panel_draw_on_block_partitions_fp64(blocks):
    w = inputs.sparse_problem(40000, 30000, per_col=12, nnz_frac=0.01, block=64, p=0.3,
                              dtype=torch.float64, seed=42)
    if blocks == "irregular":
        bp = _irregular_blocks(w.n, 5, 150, seed=4)
    else:  # equal blocks except a last one longer than the others: not an equal partition
        bp = np.concatenate([np.arange(0, w.n - 100, 64), [w.n]]).astype(np.int64)
    w = dataclasses.replace(w, block_ptr=bp)
    prob = O.Problem(A=w.scipy_csr().tocsc(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)
    _run(w, prob)
