"""Plain FP64 CPU oracle for the fixed-stepsize SCA block method.

TEST INFRASTRUCTURE. This module is the slow, obviously-correct definition that the
GPU path is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it. It shares no code with the HIP
library and imports nothing from it.

Method: Algorithm 1 (AsyFLEXA, global description) of Cannelli, Facchinei,
Kungurtsev and Scutari, "Asynchronous Parallel Algorithms for Nonconvex Big-Data
Optimization, Part II: Complexity and Numerical Results" (arXiv:1701.04900),
applied to the problem family

    min_x  F(x) = 1/2 ||A x - b||^2 - c ||x||^2 + lam * sum_j h(x_j)
    s.t.   -beta <= x_j <= beta,

which is problem (1) with smooth f = 1/2||Ax-b||^2 - c||x||^2 (- lam*h^- for the
DC regularisers), separable convex G = lam*eta*||x||_1 and box sets X_i.

Every floating-point step runs in float64; a stored float32 A is upcast on use.

Readings of the paper that this oracle fixes (the paper is silent or ambiguous):
  * Round.  One "round" k updates every block of a randomly drawn set S_k, and
    every selected block reads the same (x^k, r^k).  This is Algorithm 1 with
    delay vectors bounded by |S_k|-1 and with each block owned by a single
    worker (Assumption D, items D1 and D4).
  * Selection.  Block i is in S_k independently with probability p, decided by
    the first output word of Philox4x32-10 keyed on the seed with counter
    (i, k mod 2^32, k div 2^32, instance); the threshold is floor(p * 2^32).
    This satisfies D2 with p_min = p.
  * Surrogate.  For a block of several coordinates the surrogate is the sum over
    its coordinates of the exact one-coordinate restriction of 1/2||Ax-b||^2 plus
    tau/2 (x_j - x_j^k)^2 (Section 4.2 gives this for scalar blocks); the concave
    parts -c x_j^2 and -lam*h^-(x_j) are linearised at x^k (Section 4.3, the
    best-response formula of the nonconvex sparse-learning test).  The
    curvature of coordinate j is q_j = ||a_j||^2 + tau.
  * tau is a fixed input (the FLEXA heuristic the paper uses is not given).
  * The quadratic always carries the factor 1/2, also for the DC regularisers.
  * x^0 = 0 unless given (Section 4.2).

Parity unpinned: nothing in this module reproduces a number printed in the
paper (its experiments are figures only); every function below is pinned by
closed forms, brute force and invariants in the test suite instead.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

try:  # scipy is only needed for sparse A
    import scipy.sparse as _sp
except Exception:  # pragma: no cover
    _sp = None

# --------------------------------------------------------------------------------------
# Philox4x32-10 counter-based generator.
# Defined in J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
# numbers: as easy as 1, 2, 3", SC'11: a 4x32-bit counter, a 2x32-bit key, ten
# rounds of two 32x32->64-bit multiplications whose high halves are xored with
# the other counter words and the key, and a Weyl-sequence key bump per round.
# --------------------------------------------------------------------------------------
_MASK32 = np.uint64(0xFFFFFFFF)
_PHILOX_M0 = np.uint64(0xD2511F53)
_PHILOX_M1 = np.uint64(0xCD9E8D57)
_PHILOX_W0 = np.uint64(0x9E3779B9)
_PHILOX_W1 = np.uint64(0xBB67AE85)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Return the four 32-bit output words (as uint64 arrays) for the given counters/key."""
    c = [np.asarray(v, dtype=np.uint64) & _MASK32 for v in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK32
    for _ in range(10):
        p0 = _PHILOX_M0 * c[0]  # exact: both factors < 2^32
        p1 = _PHILOX_M1 * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & _MASK32,
             (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & _MASK32]
        k0 = (k0 + _PHILOX_W0) & _MASK32
        k1 = (k1 + _PHILOX_W1) & _MASK32
    return c


def selection_threshold(p: float) -> int:
    """Integer threshold T = floor(p * 2^32); a block is drawn when its word is < T."""
    if not (0.0 < p <= 1.0) or math.isnan(p):
        raise ValueError("selection probability must lie in (0, 1]")
    return int(math.floor(p * 4294967296.0))


def selected_blocks(seed: int, k: int, instance: int, nblocks: int, p: float) -> np.ndarray:
    """Boolean mask of the blocks in S_k (step S.1 of Algorithm 1; Assumption D2)."""
    T = selection_threshold(p)
    if T >= 2 ** 32:
        return np.ones(nblocks, dtype=bool)
    i = np.arange(nblocks, dtype=np.uint64)
    w0 = philox4x32_10(i, k & 0xFFFFFFFF, k >> 32, instance, seed & 0xFFFFFFFF, seed >> 32)[0]
    return w0 < np.uint64(T)


def block_columns(block_ptr: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Coordinates of the selected blocks, ascending."""
    parts = [np.arange(block_ptr[i], block_ptr[i + 1]) for i in np.flatnonzero(mask)]
    if not parts:
        return np.zeros(0, dtype=np.int64)
    return np.concatenate(parts).astype(np.int64)


def gamma_at(gamma0: float, mu: float, k: int) -> float:
    """Stepsize of round k: fixed gamma0 when mu == 0, otherwise the diminishing rule
    gamma^{k+1} = gamma^k (1 - mu gamma^k) of Section 4.1 started from gamma0."""
    g = float(gamma0)
    for _ in range(k):
        g = g * (1.0 - mu * g)
    return g


# --------------------------------------------------------------------------------------
# Problem description
# --------------------------------------------------------------------------------------
@dataclass
class Problem:
    """min 1/2||Ax-b||^2 - c||x||^2 + lam*sum h(x_j), -beta <= x <= beta.

    A is (m, n): a dense ndarray of any float dtype or a scipy.sparse matrix.
    reg is 'l1' (h = |x|), 'exp' (h = 1 - exp(-theta|x|)) or 'log'
    (h = log(1 + theta|x|)/log(1 + theta)) -- the regularisers of Section 4.3.
    """
    A: object
    b: np.ndarray
    lam: float
    c: float = 0.0
    beta: float = math.inf
    block_ptr: np.ndarray | None = None
    reg: str = "l1"
    theta: float = 0.0
    _colnorm2: np.ndarray | None = field(default=None, repr=False)

    @property
    def m(self):
        return self.A.shape[0]

    @property
    def n(self):
        return self.A.shape[1]

    def blocks(self):
        if self.block_ptr is None:
            return np.arange(self.n + 1, dtype=np.int64)
        return np.asarray(self.block_ptr, dtype=np.int64)

    # -- data access, always float64 ---------------------------------------------------
    def cols(self, idx):
        sub = self.A[:, idx]
        if _sp is not None and _sp.issparse(sub):
            return sub.astype(np.float64)
        return np.asarray(sub, dtype=np.float64)

    def colnorm2(self) -> np.ndarray:
        """||a_j||^2 for every column, accumulated in float64."""
        if self._colnorm2 is None:
            n = self.n
            out = np.empty(n, dtype=np.float64)
            step = 2048
            for j0 in range(0, n, step):
                sub = self.cols(slice(j0, min(n, j0 + step)))
                if _sp is not None and _sp.issparse(sub):
                    out[j0:j0 + sub.shape[1]] = np.asarray(sub.multiply(sub).sum(axis=0)).ravel()
                else:
                    out[j0:j0 + sub.shape[1]] = np.einsum("ij,ij->j", sub, sub)
            self._colnorm2 = out
        return self._colnorm2

    def Atr(self, r, idx=slice(None)):
        """A[:, idx]^T r in float64."""
        sub = self.cols(idx)
        return np.asarray(sub.T @ np.asarray(r, dtype=np.float64)).ravel()

    def Av(self, v, idx=slice(None)):
        """A[:, idx] v in float64."""
        sub = self.cols(idx)
        return np.asarray(sub @ np.asarray(v, dtype=np.float64)).ravel()

    # -- regulariser pieces (Section 4.3 DC split h = eta|x| - h^-) ----------------------
    def eta(self) -> float:
        if self.reg == "l1":
            return 1.0
        if self.reg == "exp":
            return float(self.theta)
        if self.reg == "log":
            return float(self.theta / math.log1p(self.theta))
        raise ValueError(self.reg)

    def h(self, x):
        ax = np.abs(x)
        if self.reg == "l1":
            return ax
        if self.reg == "exp":
            return 1.0 - np.exp(-self.theta * ax)
        return np.log1p(self.theta * ax) / math.log1p(self.theta)

    def dh_minus(self, x):
        """Derivative of h^- = eta|x| - h (smooth, Lipschitz gradient)."""
        x = np.asarray(x, dtype=np.float64)
        if self.reg == "l1":
            return np.zeros_like(x)
        ax = np.abs(x)
        if self.reg == "exp":
            return np.sign(x) * self.theta * (1.0 - np.exp(-self.theta * ax))
        return np.sign(x) * self.eta() * (self.theta * ax) / (1.0 + self.theta * ax)


# --------------------------------------------------------------------------------------
# The pieces of one update
# --------------------------------------------------------------------------------------
def residual(prob: Problem, x) -> np.ndarray:
    """r = A x - b, float64."""
    x = np.asarray(x, dtype=np.float64)
    nz = np.flatnonzero(x)
    r = -np.asarray(prob.b, dtype=np.float64)
    if nz.size:
        r = r + prob.Av(x[nz], nz)
    return r


def smooth_grad(prob: Problem, x, r, idx) -> np.ndarray:
    """Partial gradient of the smooth part at coordinates idx:
    a_j^T r - 2 c x_j - lam * (h^-)'(x_j).  Surrogate condition B2 (gradient
    consistency) makes this the gradient the best response linearises."""
    x = np.asarray(x, dtype=np.float64)
    g = prob.Atr(r, idx) - 2.0 * prob.c * x[idx]
    if prob.reg != "l1":
        g = g - prob.lam * prob.dh_minus(x[idx])
    return g


def best_response_1d(xj, gj, qj, thr, beta):
    """argmin over t in [-beta, beta] of g (t - x) + q/2 (t - x)^2 + thr |t|:
    the soft-threshold (the closed form used in Section 4.1 for scalar blocks)
    of v = x - g/q at level thr/q, then the projection onto the box.  A 1-D
    strongly convex function restricted to an interval is minimised by the
    projection of its unconstrained minimiser."""
    v = xj - gj / qj
    t = np.sign(v) * np.maximum(np.abs(v) - thr / qj, 0.0)
    return np.clip(t, -beta, beta)


def best_response(prob: Problem, x, r, idx, tau) -> np.ndarray:
    """x_hat_j(x) of subproblem (2) for the coordinates idx (step S.2)."""
    g = smooth_grad(prob, x, r, idx)
    q = prob.colnorm2()[idx] + tau
    return best_response_1d(np.asarray(x, dtype=np.float64)[idx], g, q,
                            prob.lam * prob.eta(), prob.beta)


def sca_round(prob: Problem, x, r, tau, gamma, idx):
    """One round: every coordinate in idx (ascending) takes the relaxed step (3),
    x_j <- x_j + gamma (x_hat_j - x_j), all reading the same (x, r); then the
    residual is brought to r = A x_new - b by adding the columns that moved.
    Returns (x_new, r_new, number of coordinates whose value changed)."""
    x = np.asarray(x, dtype=np.float64)
    if len(idx) == 0:
        return x.copy(), np.asarray(r, dtype=np.float64).copy(), 0
    xhat = best_response(prob, x, r, idx, tau)
    dx = gamma * (xhat - x[idx])
    x_new = x.copy()
    x_new[idx] = x[idx] + dx
    moved = dx != 0.0
    r_new = np.asarray(r, dtype=np.float64).copy()
    if moved.any():
        r_new = r_new + prob.Av(dx[moved], idx[moved])
    return x_new, r_new, int(moved.sum())


def sca_round_delayed(prob: Problem, x, r, tau, gamma, idx, chunks: int, stale: int):
    """One round with bounded delays (Algorithm 1 with delayed iterates x~ = x^(k-d), the
    delays bounded as in Assumption D1): the drawn coordinates idx (ascending) are updated
    in `chunks` consecutive groups of ceil(len(idx)/chunks); group t reads the residual
    left by groups 0 .. t-1-stale of the round, so every coordinate it updates sees all
    moves older than `stale` groups and none of the newer ones (delays below
    (stale + 1) * group size), while its own coordinate is current (Assumption D4: each
    coordinate is drawn once per round).  chunks <= 1 or stale >= chunks - 1 is the round of
    sca_round; stale = 0 with one coordinate per group is sequential coordinate descent.
    Returns (x_new, r_new, number of coordinates whose value changed)."""
    x = np.asarray(x, dtype=np.float64).copy()
    r0 = np.asarray(r, dtype=np.float64).copy()
    S = len(idx)
    if S == 0:
        return x, r0, 0
    q = max(1, int(chunks))
    per = -(-S // q)
    versions = [r0]  # versions[t] = residual after groups 0 .. t-1
    moved_total = 0
    for t in range(q):
        sub = idx[min(S, t * per):min(S, t * per + per)]
        r_read = versions[max(0, t - stale)]
        if len(sub):
            xhat = best_response(prob, x, r_read, sub, tau)
            dx = gamma * (xhat - x[sub])
            x[sub] = x[sub] + dx
            moved = dx != 0.0
            moved_total += int(moved.sum())
            r_next = versions[-1] + (prob.Av(dx[moved], sub[moved]) if moved.any() else 0.0)
        else:
            r_next = versions[-1].copy()
        versions.append(np.asarray(r_next, dtype=np.float64))
    return x, versions[-1], moved_total


def objective(prob: Problem, x, r=None) -> float:
    """F(x) = 1/2||r||^2 - c||x||^2 + lam * sum h(x_j) with r = Ax - b."""
    x = np.asarray(x, dtype=np.float64)
    if r is None:
        r = residual(prob, x)
    r = np.asarray(r, dtype=np.float64)
    return float(0.5 * np.dot(r, r) - prob.c * np.dot(x, x) + prob.lam * np.sum(prob.h(x)))


def stationarity_MF(prob: Problem, x) -> float:
    """||M_F(x)||_2 with M_F(x) = x - argmin_y {grad f(x)^T (y-x) + G(y) + 1/2||y-x||^2}
    over the box (the optimality measure of Section 3): a unit-step proximal
    gradient residual."""
    x = np.asarray(x, dtype=np.float64)
    r = residual(prob, x)
    g = smooth_grad(prob, x, r, np.arange(prob.n))
    y = best_response_1d(x, g, 1.0, prob.lam * prob.eta(), prob.beta)
    return float(np.linalg.norm(x - y))


def merit(prob: Problem, x, tau) -> float:
    """||x_hat(x) - x||_inf over all coordinates (the stationarity distance of Section 4.3)."""
    x = np.asarray(x, dtype=np.float64)
    r = residual(prob, x)
    xhat = best_response(prob, x, r, np.arange(prob.n), tau)
    return float(np.max(np.abs(xhat - x))) if prob.n else 0.0


def nnz_best_response(prob: Problem, x, tau) -> int:
    """Number of nonzero coordinates of the best response x_hat(x) (not of x): the
    soft-threshold yields exact zeros, so this is the support size the method reports."""
    x = np.asarray(x, dtype=np.float64)
    r = residual(prob, x)
    return int(np.count_nonzero(best_response(prob, x, r, np.arange(prob.n), tau)))


# --------------------------------------------------------------------------------------
# Driving the iteration
# --------------------------------------------------------------------------------------
@dataclass
class RunConfig:
    tau: float
    gamma: float = 0.9
    gamma_mu: float = 0.0      # diminishing rule of Section 4.1 when > 0
    p: float = 1.0
    seed: int = 0
    instance: int = 0
    delay_chunks: int = 0      # > 1: rounds of sca_round_delayed
    delay_stale: int = 0


def run_rounds(prob: Problem, cfg: RunConfig, x, r, k0: int, nrounds: int, trace=None):
    """Rounds k0 .. k0+nrounds-1 of Algorithm 1 (one round = steps S.1-S.5 for every
    drawn block).  Returns (x, r, coordinate updates performed)."""
    bp = prob.blocks()
    nblocks = len(bp) - 1
    x = np.asarray(x, dtype=np.float64).copy()
    r = np.asarray(r, dtype=np.float64).copy()
    updates = 0
    gamma = gamma_at(cfg.gamma, cfg.gamma_mu, k0)
    for k in range(k0, k0 + nrounds):
        mask = selected_blocks(cfg.seed, k, cfg.instance, nblocks, cfg.p)
        idx = block_columns(bp, mask)
        if cfg.delay_chunks > 1:
            x, r, _ = sca_round_delayed(prob, x, r, cfg.tau, gamma, idx, cfg.delay_chunks,
                                        cfg.delay_stale)
        else:
            x, r, _ = sca_round(prob, x, r, cfg.tau, gamma, idx)
        updates += len(idx)
        if trace is not None:
            trace.append((k, x.copy(), r.copy()))
        if cfg.gamma_mu:
            gamma = gamma * (1.0 - cfg.gamma_mu * gamma)
    return x, r, updates


def solve(prob: Problem, cfg: RunConfig, x0=None, max_rounds=100000, check_every=10,
          F_star=None, tol_rel_obj=None, tol_merit=None, refresh_every=0):
    """Run from x0 (default 0) until the relative objective error (F - F*)/|F*| or the
    merit drops below its tolerance, or max_rounds.  A check comes after every
    check_every rounds (fewer for the last one).  At check number t (counted from 1)
    with refresh_every > 0 dividing t, the running residual is replaced by a fresh
    r = Ax - b before the objective is taken (the optional residual refresh: the
    paper keeps no residual, so this is a reading of ours).  A tolerance on the
    relative error is tested with the running residual first and confirmed with a
    fresh one; when the fresh one does not confirm it, the running residual is
    restarted from the fresh one.
    Returns dict(x, r, rounds, updates, F, history)."""
    x = np.zeros(prob.n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    r = residual(prob, x)
    k = 0
    checks = 0
    updates = 0
    hist = []
    while k < max_rounds:
        step = min(check_every, max_rounds - k)
        x, r, u = run_rounds(prob, cfg, x, r, k, step)
        k += step
        checks += 1
        updates += u
        if refresh_every > 0 and checks % refresh_every == 0:
            r = residual(prob, x)
        F = objective(prob, x, r)
        hist.append((k, F))
        done = False
        if tol_rel_obj is not None and F_star is not None:
            if (F - F_star) / abs(F_star) <= tol_rel_obj:
                fresh = residual(prob, x)
                done = (objective(prob, x, fresh) - F_star) / abs(F_star) <= tol_rel_obj
                if not done:
                    r = fresh
        if not done and tol_merit is not None:
            done = merit(prob, x, cfg.tau) <= tol_merit
        if done:
            break
    return dict(x=x, r=r, rounds=k, updates=updates, F=objective(prob, x), history=hist)


def estimate_F_star(prob: Problem, cfg: RunConfig, max_rounds=200000, check_every=10,
                    rel_var=1e-15, calm_checks=10, mf_tol=1e-12):
    """F* as in Section 4.2: run the iteration until the objective no longer moves
    (|F_k - F_{k-1}| <= rel_var |F_k| for calm_checks consecutive checks) and
    ||M_F|| <= mf_tol.  Returns (F*, x)."""
    x = np.zeros(prob.n)
    r = residual(prob, x)
    k = 0
    F_prev = None
    calm = 0
    while k < max_rounds:
        x, r, _ = run_rounds(prob, cfg, x, r, k, check_every)
        k += check_every
        r = residual(prob, x)  # keep the residual fresh
        F = objective(prob, x, r)
        if F_prev is not None and abs(F - F_prev) <= rel_var * abs(F):
            calm += 1
        else:
            calm = 0
        F_prev = F
        if calm >= calm_checks and stationarity_MF(prob, x) <= mf_tol:
            break
    return objective(prob, x), x


# --------------------------------------------------------------------------------------
# Implicit differentiation at the fixed point x* = x_hat(x*)  (l1 regulariser)
# --------------------------------------------------------------------------------------
def active_support(prob: Problem, x, tau):
    """S = {j : x_hat_j(x) != 0 and |x_hat_j(x)| < beta}, s = sign(x_hat_S).
    Taken from the best response, whose soft-threshold produces exact zeros."""
    x = np.asarray(x, dtype=np.float64)
    r = residual(prob, x)
    xhat = best_response(prob, x, r, np.arange(prob.n), tau)
    S = np.flatnonzero((xhat != 0.0) & (np.abs(xhat) < prob.beta))
    return S, np.sign(xhat[S])


def reduced_hessian(prob: Problem, S) -> np.ndarray:
    """H_S = A_S^T A_S - 2c I: the Hessian of the smooth part on the support."""
    AS = prob.cols(S)
    if _sp is not None and _sp.issparse(AS):
        AS = AS.toarray()
    return AS.T @ AS - 2.0 * prob.c * np.eye(len(S))


def adjoint_vjp(prob: Problem, x_star, xbar, tau):
    """Vector-Jacobian product of x*(b, lam): on the support the stationarity
    condition A_S^T(A_S x_S - b) - 2c x_S + lam s = 0 holds, so
    dx_S = H_S^{-1}(A_S^T db - s dlam) and x is locally constant off S.
    Returns (bbar = A_S H_S^{-1} xbar_S, lambar = -s^T H_S^{-1} xbar_S)."""
    if prob.reg != "l1":
        raise ValueError("adjoint is defined for the l1 regulariser")
    S, s = active_support(prob, x_star, tau)
    xbar = np.asarray(xbar, dtype=np.float64)
    if len(S) == 0:
        return np.zeros(prob.m), 0.0
    H = reduced_hessian(prob, S)
    L = np.linalg.cholesky(H)  # raises when H_S is not positive definite
    w = np.linalg.solve(L.T, np.linalg.solve(L, xbar[S]))
    bbar = prob.Av(w, S)
    return bbar, float(-np.dot(s, w))


def adjoint_jvp(prob: Problem, x_star, db, dlam, tau):
    """Directional derivative dx* along (db, dlam) (same linearisation as adjoint_vjp)."""
    S, s = active_support(prob, x_star, tau)
    out = np.zeros(prob.n)
    if len(S) == 0:
        return out
    H = reduced_hessian(prob, S)
    rhs = prob.Atr(np.asarray(db, dtype=np.float64), S) - s * dlam
    out[S] = np.linalg.solve(H, rhs)
    return out
