"""Seeded synthetic workloads shaped like the paper's test problems.

This module only draws problem data (A, b, x_true, lam, tau, block partition); it
contains none of the method's arithmetic. Both the GPU path and the CPU oracle
are fed from it.

Recipe (stand-ins for the Gaussian LASSO generator and the nonconvex
sparse-learning data of Sections 4.2-4.3; the paper's own instances and the
Nesterov / Gondzio generators are not reproduced):
  * A: i.i.d. N(0,1), every column scaled to unit Euclidean norm in float64,
    then rounded to the storage dtype.  Stored column-major: ``At[j, i] = A[i, j]``
    with leading dimension ``lda`` (a multiple of 4, padding rows are zero).
  * x_true: exactly round(frac * n) nonzeros on a seeded random support,
    magnitudes uniform in [lo, hi], signs +-1 with probability 1/2.
  * b = A_stored x_true + sigma * N(0,1) formed in float64, rounded to the dtype.
  * lam = lam_frac * ||A^T b||_inf in float64 from the stored A and b.
  * tau = max(0, 0.6 L - min_j ||a_j||^2) with L = max_j ||a_j||^2 (1 + sqrt(P/m))^2
    and P = p * n the expected coordinates per round (a random-matrix estimate
    of the largest eigenvalue of A_S^T A_S, so the Jacobi round descends).
  * Blocks: contiguous, ``block`` coordinates each, the last one may be short.
All randomness comes from one ``torch.Generator`` seeded with ``seed``; columns
are drawn in fixed chunks so the stream does not depend on memory size.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

_CHUNK = 4096


def _gen(device, seed):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def block_partition(n: int, block: int) -> np.ndarray:
    """block_ptr of contiguous blocks of ``block`` coordinates (last may be short)."""
    bp = list(range(0, n, block)) + [n]
    return np.asarray(bp, dtype=np.int64)


def tau_heuristic(colnorm2_min: float, colnorm2_max: float, m: int, n: int, p: float) -> float:
    P = max(1.0, p * n)
    L = colnorm2_max * (1.0 + math.sqrt(P / m)) ** 2
    return max(0.0, 0.6 * L - colnorm2_min)


@dataclass
class DenseWorkload:
    name: str
    At: torch.Tensor          # (n, lda) storage dtype; At[j, :m] is column j of A
    m: int
    n: int
    lda: int
    b: torch.Tensor           # (m,) storage dtype
    x_true: torch.Tensor      # (n,) float64
    lam: float
    c: float
    beta: float
    tau: float
    block_ptr: np.ndarray     # (N+1,) int64
    p: float
    gamma: float
    seed: int
    instance: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def dtype(self):
        return self.At.dtype

    def A_numpy(self) -> np.ndarray:
        """(m, n) view of A on the host (no copy when At already lives there)."""
        return self.At[:, : self.m].cpu().numpy().T

    def to(self, device):
        return DenseWorkload(self.name, self.At.to(device), self.m, self.n, self.lda,
                             self.b.to(device), self.x_true.to(device), self.lam, self.c,
                             self.beta, self.tau, self.block_ptr, self.p, self.gamma,
                             self.seed, self.instance, dict(self.meta))


def dense_problem(m: int, n: int, *, nnz_frac: float, amp=(1.0, 2.0), sigma: float = 0.01,
                  lam_frac: float = 0.01, c_frac: float = 0.0, beta: float = math.inf,
                  block: int = 64, p: float = 1.0, gamma: float = 0.9,
                  dtype=torch.float32, seed: int = 0, device="cpu", tau=None,
                  name: str = "dense", instance: int = 0) -> DenseWorkload:
    """Draw one dense problem.  ``c_frac`` sets c = c_frac * min_j ||a_j||^2."""
    g = _gen(device, seed)
    lda = (m + 3) // 4 * 4
    At = torch.zeros(n, lda, dtype=dtype, device=device)
    for j0 in range(0, n, _CHUNK):
        j1 = min(n, j0 + _CHUNK)
        blk = torch.randn(j1 - j0, m, dtype=torch.float64, generator=g, device=device)
        blk /= torch.linalg.vector_norm(blk, dim=1, keepdim=True)
        At[j0:j1, :m] = blk.to(dtype)
        del blk
    s = int(round(nnz_frac * n))
    supp = torch.randperm(n, generator=g, device=device)[:s]
    mag = amp[0] + (amp[1] - amp[0]) * torch.rand(s, dtype=torch.float64, generator=g, device=device)
    sgn = torch.where(torch.rand(s, dtype=torch.float64, generator=g, device=device) < 0.5, -1.0, 1.0)
    x_true = torch.zeros(n, dtype=torch.float64, device=device)
    x_true[supp] = sgn * mag
    noise = torch.randn(m, dtype=torch.float64, generator=g, device=device)
    # b = A_stored x_true + sigma e   (float64)
    b64 = sigma * noise
    for j0 in range(0, n, _CHUNK):
        j1 = min(n, j0 + _CHUNK)
        b64 += At[j0:j1, :m].double().T @ x_true[j0:j1]
    b = b64.to(dtype)
    bd = b.double()
    atb_max = 0.0
    cn_min, cn_max = math.inf, 0.0
    for j0 in range(0, n, _CHUNK):
        j1 = min(n, j0 + _CHUNK)
        blk = At[j0:j1, :m].double()
        atb_max = max(atb_max, float((blk @ bd).abs().max()))
        cn = (blk * blk).sum(dim=1)
        cn_min = min(cn_min, float(cn.min()))
        cn_max = max(cn_max, float(cn.max()))
        del blk
    lam = lam_frac * atb_max
    c = c_frac * cn_min
    if tau is None:
        tau = tau_heuristic(cn_min, cn_max, m, n, p)
    return DenseWorkload(name, At, m, n, lda, b, x_true, float(lam), float(c), float(beta),
                         float(tau), block_partition(n, block), float(p), float(gamma),
                         int(seed), int(instance),
                         dict(colnorm2_min=cn_min, colnorm2_max=cn_max, nnz_true=s))


def orthogonal_problem(m: int, n: int, *, lam: float, c: float = 0.0, beta: float = math.inf,
                       seed: int = 0, dtype=torch.float64, block: int = 1, p: float = 1.0,
                       gamma: float = 0.9, device="cpu") -> DenseWorkload:
    """A with orthonormal columns (A^T A = I, m >= n) from a QR factorisation of a
    seeded Gaussian matrix; b ~ N(0,1)."""
    if m < n:
        raise ValueError("orthogonal columns need m >= n")
    g = _gen("cpu", seed)
    G = torch.randn(m, n, dtype=torch.float64, generator=g)
    Q, _ = torch.linalg.qr(G)
    b = torch.randn(m, dtype=torch.float64, generator=g)
    lda = (m + 3) // 4 * 4
    At = torch.zeros(n, lda, dtype=dtype)
    At[:, :m] = Q.T.to(dtype)
    return DenseWorkload("orthogonal", At.to(device), m, n, lda, b.to(dtype).to(device),
                         torch.zeros(n, dtype=torch.float64, device=device), float(lam), float(c),
                         float(beta), 0.0, block_partition(n, block), float(p), float(gamma),
                         int(seed))


# --------------------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------------------
def lasso_small_fp64(seed=0, device="cpu"):
    """LASSO 200 x 1000, FP64, 10% nonzeros +-[1,2], sigma 0.01, lam = 0.1||A^T b||_inf,
    scalar blocks, every block each round, gamma 0.9."""
    return dense_problem(200, 1000, nnz_frac=0.10, amp=(1.0, 2.0), sigma=0.01, lam_frac=0.1,
                         block=1, p=1.0, gamma=0.9, dtype=torch.float64, seed=seed,
                         device=device, name="lasso_200x1000_fp64")


def lasso_dense_fp32(m=20000, n=100000, seed=0, device="cpu", dtype=torch.float32):
    """LASSO 20000 x 100000 (default), FP32, 1% nonzeros +-[1,2], sigma 0.01,
    lam = 0.01||A^T b||_inf, blocks of 64, 25% of blocks per round, gamma 0.9."""
    return dense_problem(m, n, nnz_frac=0.01, amp=(1.0, 2.0), sigma=0.01, lam_frac=0.01,
                         block=64, p=0.25, gamma=0.9, dtype=dtype, seed=seed, device=device,
                         name=f"lasso_{m}x{n}_{str(dtype).split('.')[-1]}")


def nonconvex_box_fp32(m=10000, n=50000, seed=0, device="cpu", dtype=torch.float32):
    """min 1/2||Ax-b||^2 - c||x||^2 + lam||x||_1, |x_j| <= 1, 10000 x 50000 (default),
    c = 0.5 min_j||a_j||^2, 5% nonzeros +-[0.5,1], lam = 0.05||A^T b||_inf,
    blocks of 32, 25% of blocks per round, gamma 0.9."""
    return dense_problem(m, n, nnz_frac=0.05, amp=(0.5, 1.0), sigma=0.01, lam_frac=0.05,
                         c_frac=0.5, beta=1.0, block=32, p=0.25, gamma=0.9, dtype=dtype,
                         seed=seed, device=device,
                         name=f"ncvx_box_{m}x{n}_{str(dtype).split('.')[-1]}")


# --------------------------------------------------------------------------------------
# Many right-hand sides over one dense A
# --------------------------------------------------------------------------------------
@dataclass
class MultiWorkload:
    name: str
    At: torch.Tensor          # (n, lda) as for DenseWorkload
    m: int
    n: int
    lda: int
    B: torch.Tensor           # (K, lda) storage dtype; B[k, :m] = b_k
    lams: np.ndarray          # (K,) float64
    c: float
    beta: float
    tau: float
    block_ptr: np.ndarray
    p: float
    gamma: float
    seed: int
    base: DenseWorkload

    @property
    def K(self):
        return int(self.B.shape[0])

    @property
    def dtype(self):
        return self.At.dtype

    def b(self, k):
        return self.B[k, : self.m]


def multi_rhs_problem(m: int, n: int, K: int, *, rhs: str = "sweep", lam_range=(0.005, 0.05),
                      delta: float = 1e-3, nnz_frac: float = 0.01, c_frac: float = 0.0,
                      beta: float = math.inf, block: int = 64, p: float = 0.25,
                      gamma: float = 0.9, dtype=torch.float32, seed: int = 0,
                      device="cpu") -> MultiWorkload:
    """K problems over the A of ``dense_problem(m, n, ...)``.  rhs="sweep": every b_k is the
    base b and lam_k = f_k ||A^T b||_inf with f_k log-spaced over lam_range.  rhs="perturbed":
    b_k = b + delta * u_k with seeded N(0,1) vectors u_k and lam_k = the base lam (the
    problems of a finite-difference check)."""
    w = dense_problem(m, n, nnz_frac=nnz_frac, lam_frac=lam_range[0], c_frac=c_frac, beta=beta,
                      block=block, p=p, gamma=gamma, dtype=dtype, seed=seed, device=device)
    atb_max = w.lam / lam_range[0]
    B = torch.zeros(K, w.lda, dtype=dtype, device=device)
    if rhs == "sweep":
        f = np.exp(np.linspace(math.log(lam_range[0]), math.log(lam_range[1]), K))
        lams = f * atb_max
        B[:, :m] = w.b[None, :]
    elif rhs == "perturbed":
        g = _gen(device, seed + 7919)
        U = torch.randn(K, m, dtype=torch.float64, generator=g, device=device)
        B[:, :m] = (w.b.double()[None, :] + delta * U).to(dtype)
        lams = np.full(K, w.lam)
    else:
        raise ValueError("rhs must be 'sweep' or 'perturbed'")
    return MultiWorkload(f"multi_{rhs}_{m}x{n}_K{K}_{str(dtype).split('.')[-1]}", w.At, m, n,
                         w.lda, B, np.asarray(lams, dtype=np.float64), w.c, w.beta, w.tau,
                         w.block_ptr, w.p, w.gamma, w.seed, w)


# --------------------------------------------------------------------------------------
# Sparse workloads (CSR)
# --------------------------------------------------------------------------------------
@dataclass
class SparseWorkload:
    name: str
    m: int
    n: int
    rowptr: torch.Tensor      # (m+1,) int64
    colidx: torch.Tensor      # (nnz,) int32, ascending inside each row
    vals: torch.Tensor        # (nnz,) storage dtype
    b: torch.Tensor           # (m,) storage dtype
    x_true: torch.Tensor      # (n,) float64
    lam: float
    c: float
    beta: float
    tau: float
    block_ptr: np.ndarray
    p: float
    gamma: float
    seed: int
    instance: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def dtype(self):
        return self.vals.dtype

    @property
    def nnz(self):
        return int(self.vals.numel())

    def scipy_csr(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals.double().cpu().numpy(), self.colidx.cpu().numpy(),
                              self.rowptr.cpu().numpy()), shape=(self.m, self.n))

    def to(self, device):
        return SparseWorkload(self.name, self.m, self.n, self.rowptr.to(device),
                              self.colidx.to(device), self.vals.to(device), self.b.to(device),
                              self.x_true.to(device), self.lam, self.c, self.beta, self.tau,
                              self.block_ptr, self.p, self.gamma, self.seed, self.instance,
                              dict(self.meta))


def sparse_problem(m: int, n: int, *, per_col: int, nnz_frac: float, amp=(1.0, 2.0),
                   sigma: float = 0.01, lam_frac: float = 0.01, block: int = 256,
                   p: float = 0.1, gamma: float = 0.9, dtype=torch.float32, seed: int = 0,
                   device="cpu", tau=None, name: str = "sparse") -> SparseWorkload:
    """CSR A with exactly ``per_col`` distinct uniform rows in every column, N(0,1) values,
    columns scaled to unit norm in float64; x*, b, lam, tau as for the dense recipe."""
    if per_col > m:
        raise ValueError("per_col must not exceed m")
    g = _gen(device, seed)
    rows = torch.randint(0, m, (n, per_col), generator=g, device=device)
    for _ in range(64):  # redraw repeated rows inside a column until all are distinct
        rows, _ = torch.sort(rows, dim=1)
        dup = torch.zeros_like(rows, dtype=torch.bool)
        dup[:, 1:] = rows[:, 1:] == rows[:, :-1]
        nd = int(dup.sum())
        if nd == 0:
            break
        rows[dup] = torch.randint(0, m, (nd,), generator=g, device=device)
    else:
        raise RuntimeError("could not draw distinct rows")
    vals = torch.randn(n, per_col, dtype=torch.float64, generator=g, device=device)
    vals /= torch.linalg.vector_norm(vals, dim=1, keepdim=True)
    vals_st = vals.to(dtype)
    s = int(round(nnz_frac * n))
    supp = torch.randperm(n, generator=g, device=device)[:s]
    mag = amp[0] + (amp[1] - amp[0]) * torch.rand(s, dtype=torch.float64, generator=g, device=device)
    sgn = torch.where(torch.rand(s, dtype=torch.float64, generator=g, device=device) < 0.5, -1.0, 1.0)
    x_true = torch.zeros(n, dtype=torch.float64, device=device)
    x_true[supp] = sgn * mag
    noise = torch.randn(m, dtype=torch.float64, generator=g, device=device)
    # b = A_stored x_true + sigma e, summed on the host in a fixed order (numpy add.at)
    sup = supp.cpu().numpy()
    contrib = (vals_st[supp].double() * x_true[supp][:, None]).cpu().numpy()
    b64 = sigma * noise.cpu().numpy()
    np.add.at(b64, rows[supp].cpu().numpy().ravel(), contrib.ravel())
    b = torch.from_numpy(b64).to(dtype).to(device)
    # A^T b and column norms of the stored values
    atb = (vals_st.double() * b.double()[rows]).sum(dim=1)
    cn = (vals_st.double() ** 2).sum(dim=1)
    lam = lam_frac * float(atb.abs().max())
    cn_min, cn_max = float(cn.min()), float(cn.max())
    if tau is None:
        tau = tau_heuristic(cn_min, cn_max, m, n, p)
    # CSR: entries ordered by (row, column)
    cols = torch.arange(n, device=device, dtype=torch.int64)[:, None].expand(n, per_col)
    key = rows.reshape(-1) * n + cols.reshape(-1)
    order = torch.argsort(key)
    r_sorted = rows.reshape(-1)[order]
    colidx = cols.reshape(-1)[order].to(torch.int32)
    v_sorted = vals_st.reshape(-1)[order]
    counts = torch.bincount(r_sorted, minlength=m)
    rowptr = torch.zeros(m + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(counts, 0)
    del key, order, rows, cols, vals
    return SparseWorkload(name, m, n, rowptr, colidx.contiguous(), v_sorted.contiguous(), b,
                          x_true, float(lam), 0.0, math.inf, float(tau), block_partition(n, block),
                          float(p), float(gamma), int(seed), 0,
                          dict(colnorm2_min=cn_min, colnorm2_max=cn_max, nnz_true=s))


def sparse_lasso_fp32(m=100000, n=1000000, per_col=100, seed=0, device="cpu",
                      dtype=torch.float32):
    """Sparse LASSO, CSR 100000 x 1000000 (default), 0.1% density (100 uniform distinct rows
    per column), N(0,1) values, unit columns, 0.5% nonzeros +-[1,2], sigma 0.01,
    lam = 0.01||A^T b||_inf, blocks of 256, 10% of blocks per round, gamma 0.9."""
    return sparse_problem(m, n, per_col=per_col, nnz_frac=0.005, amp=(1.0, 2.0), sigma=0.01,
                          lam_frac=0.01, block=256, p=0.1, gamma=0.9, dtype=dtype, seed=seed,
                          device=device, name=f"sparse_lasso_{m}x{n}_{str(dtype).split('.')[-1]}")


# --------------------------------------------------------------------------------------
# Batches of uneven dense instances
# --------------------------------------------------------------------------------------
def batch_lasso(count: int, m_range=(500, 8000), n_ratio: int = 5, nnz_frac: float = 0.02,
                lam_range=(1e-3, 1e-1), block: int = 64, p: float = 0.25, gamma: float = 0.9,
                sigma: float = 0.01, c_frac: float = 0.0, beta: float = math.inf,
                dtype=torch.float32, seed: int = 0, device="cpu"):
    """``count`` LASSO instances: m_k uniform in m_range (inclusive), n_k = n_ratio m_k,
    lam_k = lam_range[0] (lam_range[1]/lam_range[0])^(k/(count-1)) ||A_k^T b_k||_inf
    (log-spaced), x* with nnz_frac nonzeros +-[1,2]; instance k uses seed*1000003 + k and
    Philox instance word k."""
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    ms = torch.randint(m_range[0], m_range[1] + 1, (count,), generator=g).tolist()
    out = []
    for k, m in enumerate(ms):
        t = k / (count - 1) if count > 1 else 0.0
        lam_frac = lam_range[0] * (lam_range[1] / lam_range[0]) ** t
        w = dense_problem(m, n_ratio * m, nnz_frac=nnz_frac, amp=(1.0, 2.0), sigma=sigma,
                          lam_frac=lam_frac, c_frac=c_frac, beta=beta, block=block, p=p,
                          gamma=gamma, dtype=dtype, seed=int(seed) * 1000003 + k, device=device,
                          name=f"batch{k}_{m}x{n_ratio * m}", instance=k)
        out.append(w)
    return out
