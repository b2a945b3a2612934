"""GPU parity of the sparse panel-split round with the block draw inside the gradient kernel
(every workgroup draws all blocks of the round; panel 0 lists the drawn columns for the
kernels that follow; the fold advances the round state) against the FP64 oracle:

* 32768 blocks, the most the in-kernel draw takes (32 per thread), and 32769 blocks, which
  fall back to the single-workgroup draw;
* workgroup chunks longer than the 2048-column list held in LDS (16 panels, 16 chunks,
  about 48000 drawn columns: two pieces per chunk);
* rounds that draw nothing (the state still advances: round counter, step, counts);
* the solve's drawn and moved counts against the oracle's.

FP64 iterates and residual to 1e-10 relative."""
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
    return O.Problem(A=w.scipy_csr().tocsc(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)


def _compare(w, rounds, every):
    print(f"[gpu] sparse draw m={w.m} n={w.n} blocks={len(w.block_ptr) - 1} p={w.p}",
          flush=True)
    prob = _oracle(w)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
    x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
    r = torch.empty(w.m, dtype=w.dtype, device="cuda")
    sca.sca_residual(P.handle, x, r)
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
    xo = np.zeros(w.n)
    ro = O.residual(prob, xo)
    for k in range(0, rounds, every):
        sca.sca_step(P.handle, o, k, every, x, r)
        xo, ro, _ = O.run_rounds(prob, cfg, xo, ro, k, every)
        ex = _rel(x.cpu().numpy(), xo)
        er = _rel(r.cpu().numpy(), ro)
        print(f"[parity] after {k + every} rounds: x {ex:.2e} r {er:.2e}", flush=True)
        assert ex <= 1e-10 and er <= 1e-10
    P.close()


@pytest.mark.parametrize("n", [32768, 32769])
def test_draw_at_and_past_the_in_kernel_block_limit(n):
    w = inputs.sparse_problem(6000, n, per_col=6, nnz_frac=0.01, lam_frac=0.01, block=1,
                              p=0.3, dtype=torch.float64, seed=n % 101)
    _compare(w, 6, 3)


def test_draw_with_chunks_longer_than_the_lds_list():
    # FP64 panels hold 17920 rows: 286720 rows make 16 panels and 16 chunks per panel
    w = inputs.sparse_problem(286720, 60000, per_col=8, nnz_frac=0.01, lam_frac=0.01, block=16,
                              p=0.8, dtype=torch.float64, seed=9)
    _compare(w, 4, 2)


def test_rounds_that_draw_nothing_still_advance():
    w = inputs.sparse_problem(3000, 400, per_col=5, nnz_frac=0.02, lam_frac=0.01, block=100,
                              p=1e-6, dtype=torch.float64, seed=4)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, max_rounds=7,
                      check_every=7)
    x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
    st = sca.sca_solve(P.handle, o, x, raise_on_notconv=False)
    bp = _oracle(w).blocks()
    drawn = sum(len(O.block_columns(bp, O.selected_blocks(w.seed, k, 0, len(bp) - 1, w.p)))
                for k in range(7))
    assert drawn == 0
    assert st["rounds"] == 7 and st["coord_updates"] == 0 and st["moved_updates"] == 0
    assert torch.count_nonzero(x).item() == 0
    P.close()


def test_solve_counts_match_the_oracle():
    w = inputs.sparse_problem(40000, 20000, per_col=20, nnz_frac=0.01, lam_frac=0.01, block=32,
                              p=0.3, dtype=torch.float64, seed=12)
    prob = _oracle(w)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, max_rounds=9,
                      check_every=9)
    x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
    st = sca.sca_solve(P.handle, o, x, raise_on_notconv=False)
    bp = prob.blocks()
    xo = np.zeros(w.n)
    ro = O.residual(prob, xo)
    drawn = moved = 0
    for k in range(9):
        idx = O.block_columns(bp, O.selected_blocks(w.seed, k, 0, len(bp) - 1, w.p))
        xo, ro, mv = O.sca_round(prob, xo, ro, w.tau, w.gamma, idx)
        drawn += len(idx)
        moved += mv
    assert st["rounds"] == 9
    assert st["coord_updates"] == drawn and st["moved_updates"] == moved
    assert _rel(x.cpu().numpy(), xo) <= 1e-10
    P.close()
