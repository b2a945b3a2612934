"""GPU parity of the batched engine on larger and uneven instances against the FP64 oracle
run per instance with the same instance word: instances of 31 to 8192 rows (odd m, so a
ragged last 16-byte row group), an instance with fewer drawn columns than a gradient work
item, the per-instance drawn counts and the batch-wide moved count of the solve, and the
zero padding rows of the concatenated residual.  Tolerances: FP64 1e-10 relative, FP32
objective 1e-4."""
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


def _oracle(w):
    return O.Problem(A=w.A_numpy(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)


def _run_batch(ws, p, seed, rounds, dtype):
    print(f"[gpu] batch of {len(ws)}: m = {[w.m for w in ws]} n = {[w.n for w in ws]} {dtype}",
          flush=True)
    B = sca.Batch([w.to("cuda") for w in ws])
    opts = sca.make_opts(gamma=0.9, select_p=p, seed=seed, max_rounds=rounds,
                         check_every=rounds)
    x = torch.zeros(int(B.xoff[-1]), dtype=dtype, device="cuda")
    r = torch.zeros(int(B.roff[-1]), dtype=dtype, device="cuda")
    sca.sca_batch_residual(B.handle, x, r)
    sca.sca_batch_step(B.handle, opts, 0, rounds, x, r)
    torch.cuda.synchronize()
    return B, opts, x, r


def _oracle_rounds(w, k, p, seed, rounds):
    prob = _oracle(w)
    cfg = O.RunConfig(tau=w.tau, gamma=0.9, p=p, seed=seed, instance=k)
    bp = prob.blocks()
    x = np.zeros(w.n)
    r = O.residual(prob, x)
    moved = drawn = 0
    for kk in range(rounds):
        idx = O.block_columns(bp, O.selected_blocks(seed, kk, k, len(bp) - 1, p))
        x, r, mv = O.sca_round(prob, x, r, w.tau, 0.9, idx)
        moved += mv
        drawn += len(idx)
    return prob, x, r, moved, drawn


def test_batch_uneven_fp64_matches_oracle_per_instance():
    ws = inputs.batch_lasso(8, m_range=(31, 4095), n_ratio=1, nnz_frac=0.03,
                            lam_range=(1e-2, 1e-1), block=16, p=0.4, dtype=torch.float64, seed=21)
    ws[0] = inputs.batch_lasso(1, m_range=(4096, 4096), n_ratio=1, nnz_frac=0.03, block=16,
                               p=0.4, dtype=torch.float64, seed=22)[0]
    ws[1] = inputs.batch_lasso(1, m_range=(40, 40), n_ratio=1, nnz_frac=0.05, block=16, p=0.4,
                               dtype=torch.float64, seed=23)[0]  # fewer columns than a work item
    for k, w in enumerate(ws):
        w.instance = k
    B, opts, x, r = _run_batch(ws, 0.4, 5, 20, torch.float64)
    xh, rh = x.cpu().numpy(), r.cpu().numpy()
    for k, w in enumerate(ws):
        _, xo, ro, _, _ = _oracle_rounds(w, k, 0.4, 5, 20)
        assert _rel(xh[B.xoff[k]:B.xoff[k + 1]], xo) <= 1e-10, k
        assert _rel(rh[B.roff[k]:B.roff[k] + w.m], ro) <= 1e-10, k
        # padding rows of r stay zero
        assert np.all(rh[B.roff[k] + w.m:B.roff[k + 1]] == 0.0), k


def test_batch_counts_and_solve_stats_fp64():
    ws = inputs.batch_lasso(5, m_range=(500, 3000), n_ratio=2, nnz_frac=0.03,
                            lam_range=(1e-2, 1e-1), block=32, p=0.3, dtype=torch.float64, seed=24)
    B = sca.Batch([w.to("cuda") for w in ws])
    opts = sca.make_opts(gamma=0.9, select_p=0.3, seed=6, max_rounds=12, check_every=12)
    x = torch.zeros(int(B.xoff[-1]), dtype=torch.float64, device="cuda")
    st = sca.sca_batch_solve(B.handle, opts, x, B.K, raise_on_notconv=False)
    moved_total = 0
    for k, w in enumerate(ws):
        _, xo, _, moved, drawn = _oracle_rounds(w, k, 0.3, 6, 12)
        assert st[k]["rounds"] == 12
        assert st[k]["coord_updates"] == drawn, k
        moved_total += moved
        assert _rel(x[B.xoff[k]:B.xoff[k + 1]].cpu().numpy(), xo) <= 1e-10, k
    assert st[0]["moved_updates"] == moved_total


def test_batch_fp32_objective_up_to_8192_rows():
    ws = inputs.batch_lasso(4, m_range=(4097, 8191), n_ratio=1, nnz_frac=0.02,
                            lam_range=(1e-2, 5e-2), block=64, p=0.25, dtype=torch.float32, seed=25)
    ws[0] = inputs.batch_lasso(1, m_range=(8192, 8192), n_ratio=1, nnz_frac=0.02, block=64,
                               p=0.25, dtype=torch.float32, seed=26)[0]
    for k, w in enumerate(ws):
        w.instance = k
    B, opts, x, r = _run_batch(ws, 0.25, 7, 20, torch.float32)
    rep = sca.sca_batch_objective(B.handle, opts, x, B.K)
    for k, w in enumerate(ws):
        prob, xo, _, _, _ = _oracle_rounds(w, k, 0.25, 7, 20)
        Fo = O.objective(prob, xo)
        assert abs(rep["F"][k] - Fo) <= 1e-4 * abs(Fo), k
        ex = _rel(x[B.xoff[k]:B.xoff[k + 1]].double().cpu().numpy(), xo)
        print(f"[parity] batch fp32 instance {k} m={w.m}: x err {ex:.2e}", flush=True)
        assert ex <= x_tol(w.m), k


def test_batch_with_a_4097_row_instance_fp64():
    ws = inputs.batch_lasso(3, m_range=(50, 900), n_ratio=2, nnz_frac=0.03, block=16, p=0.4,
                            dtype=torch.float64, seed=27)
    ws[2] = inputs.batch_lasso(1, m_range=(4097, 4097), n_ratio=1, nnz_frac=0.03, block=16,
                               p=0.4, dtype=torch.float64, seed=28)[0]
    for k, w in enumerate(ws):
        w.instance = k
    B, opts, x, r = _run_batch(ws, 0.4, 8, 15, torch.float64)
    xh, rh = x.cpu().numpy(), r.cpu().numpy()
    for k, w in enumerate(ws):
        _, xo, ro, _, _ = _oracle_rounds(w, k, 0.4, 8, 15)
        assert _rel(xh[B.xoff[k]:B.xoff[k + 1]], xo) <= 1e-10, k
        assert _rel(rh[B.roff[k]:B.roff[k] + w.m], ro) <= 1e-10, k
