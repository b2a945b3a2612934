"""GPU parity of the three sparse gradient kernels, each picked by the shape of the problem,
against the FP64 CPU oracle (scipy.sparse on the oracle side):

* panel split (at most 16 panels of 140 KiB of r): one workgroup per (panel, chunk of the
  drawn list) writes partial dot products, a second kernel adds them and takes the best
  response; several panels here (m = 50000 FP64, m = 100000 FP32: 3 panels each);
* panel walk (more than 16 panels: m = 300000 FP64 and m = 600000 FP32, 17 panels each):
  every workgroup walks all panels of r;
* gather (more than 2048 row bins of 1024 rows: m = 2.2e6): r read from memory;

each in FP64 (iterates) and FP32 (objective and iterates).

The small-m sparse tests elsewhere run the split kernel with a single panel.  Tolerances
as for the dense path: FP64 1e-10 relative, FP32 objective 1e-4."""
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
    return O.Problem(A=w.scipy_csr().tocsc(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)


def _run(w, rounds, every):
    print(f"[gpu] sparse path m={w.m} n={w.n} nnz={w.nnz} dtype={w.dtype}", flush=True)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
    x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
    r = torch.empty(w.m, dtype=w.dtype, device="cuda")
    sca.sca_residual(P.handle, x, r)
    out = []
    for k in range(0, rounds, every):
        sca.sca_step(P.handle, o, k, every, x, r)
        torch.cuda.synchronize()
        out.append((x.double().cpu().numpy(), r.double().cpu().numpy()))
    return P, o, x, out


def _oracle_traj(w, prob, rounds, every):
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
    x = np.zeros(w.n)
    r = O.residual(prob, x)
    out = []
    for k in range(0, rounds, every):
        x, r, _ = O.run_rounds(prob, cfg, x, r, k, every)
        out.append((x.copy(), r.copy()))
    return out


@pytest.mark.parametrize("m,n,per_col,block,p", [
    (50000, 20000, 60, 64, 0.3),      # split, 3 panels of 17920 rows (FP64)
    (300000, 6000, 40, 32, 0.5),      # walk, 17 panels
    (2200000, 2000, 12, 16, 0.6),     # gather, 2149 bins
])
def test_sparse_gradient_paths_fp64(m, n, per_col, block, p):
    w = inputs.sparse_problem(m, n, per_col=per_col, nnz_frac=0.01, lam_frac=0.01, block=block,
                              p=p, dtype=torch.float64, seed=m % 997)
    prob = _oracle(w)
    P, _, _, gpu = _run(w, 12, 4)
    for (xg, rg), (xo, ro) in zip(gpu, _oracle_traj(w, prob, 12, 4)):
        assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10
    P.close()


@pytest.mark.parametrize("m,n,per_col,block,p", [
    (600000, 8000, 30, 32, 0.5),      # walk, 17 panels of 35840 rows (FP32)
    (2200000, 2000, 12, 16, 0.6),     # gather
])
def test_sparse_gradient_paths_fp32_objective(m, n, per_col, block, p):
    w = inputs.sparse_problem(m, n, per_col=per_col, nnz_frac=0.01, lam_frac=0.01, block=block,
                              p=p, dtype=torch.float32, seed=m % 991)
    prob = _oracle(w)
    P, o, x, gpu = _run(w, 12, 4)
    xo = _oracle_traj(w, prob, 12, 4)[-1][0]
    Fo = O.objective(prob, xo)
    Fg = sca.sca_objective(P.handle, o, x)["F"]
    assert abs(Fg - Fo) <= 1e-4 * abs(Fo)
    print(f"[parity] sparse fp32 m={w.m}: x err {_rel(gpu[-1][0], xo):.2e}", flush=True)
    assert _rel(gpu[-1][0], xo) <= x_tol(w.nnz // w.n), _rel(gpu[-1][0], xo)
    P.close()


def test_sparse_split_fp32_three_panels_objective():
    w = inputs.sparse_problem(100000, 30000, per_col=100, nnz_frac=0.005, lam_frac=0.01,
                              block=64, p=0.25, dtype=torch.float32, seed=3)
    prob = _oracle(w)
    P, o, x, gpu = _run(w, 30, 10)
    xo = _oracle_traj(w, prob, 30, 10)[-1][0]
    Fo = O.objective(prob, xo)
    Fg = sca.sca_objective(P.handle, o, x)["F"]
    assert abs(Fg - Fo) <= 1e-4 * abs(Fo)
    print(f"[parity] sparse fp32 m={w.m}: x err {_rel(gpu[-1][0], xo):.2e}", flush=True)
    assert _rel(gpu[-1][0], xo) <= x_tol(w.nnz // w.n), _rel(gpu[-1][0], xo)
    P.close()


def test_sparse_split_columns_longer_than_a_window_and_empty_columns():
    """Columns with hundreds of entries in one panel (the four-loads-at-a-time tail), and
    columns without entries in some panels or at all."""
    rng = np.random.default_rng(5)
    m, n = 40000, 3000
    lens = rng.choice([0, 1, 3, 40, 400, 900], size=n, p=[0.1, 0.1, 0.2, 0.3, 0.2, 0.1])
    rows, cols, vals = [], [], []
    for j, L in enumerate(lens):
        if L == 0:
            continue
        lo = 0 if L < 900 else int(rng.integers(0, m // 3))  # long ones cluster in a panel
        hi = m if L < 900 else lo + 4000
        rr = np.sort(rng.choice(np.arange(lo, hi), size=L, replace=False))
        vv = rng.standard_normal(L)
        vv /= np.linalg.norm(vv)
        rows.append(rr)
        cols.append(np.full(L, j))
        vals.append(vv)
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    import scipy.sparse as sp
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    A.sort_indices()
    b = rng.standard_normal(m) * 0.1
    lam = 0.01 * float(np.max(np.abs(A.T @ b)))
    w = inputs.SparseWorkload(
        "sparse_windows", m, n, torch.from_numpy(A.indptr.astype(np.int64)),
        torch.from_numpy(A.indices.astype(np.int32)), torch.from_numpy(A.data.copy()),
        torch.from_numpy(b), torch.zeros(n, dtype=torch.float64), lam, 0.0, float("inf"),
        inputs.tau_heuristic(0.0, 1.0, m, n, 0.5) + 1.0,
        inputs.block_partition(n, 8), 0.5, 0.9, 7, 0, {})
    prob = _oracle(w)
    P, _, _, gpu = _run(w, 12, 4)
    for (xg, rg), (xo, ro) in zip(gpu, _oracle_traj(w, prob, 12, 4)):
        assert _rel(xg, xo) <= 1e-10 and _rel(rg, ro) <= 1e-10
    P.close()
