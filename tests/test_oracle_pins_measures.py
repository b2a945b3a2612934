"""Pins for the oracle's measurement functions and its sparse data access.

Each test checks the oracle against something other than its own formulas:
  * the merit ||x_hat(x) - x||_inf of Section 4.3 and the support size nnz(x_hat)
    against a direct 1-D minimisation of every coordinate's surrogate (the exact
    one-coordinate restriction of 1/2||Ax - b||^2, the proximal term, the linearised
    concave parts and the l1 part), evaluated from its definition, not from the
    soft-threshold closed form;
  * the DC regularisers of Section 4.3 at their special values, their symmetry,
    monotonicity and concavity, and eta against the one-sided slope h'(0+);
  * the scipy.sparse branch of Problem against the same matrix stored dense;
  * the optional residual refresh of solve() against its definition.
"""
import math

import numpy as np
import pytest
import torch

from oracle import sca_oracle as O
from paper_1701_04900_amd import inputs

_GOLD = (math.sqrt(5.0) - 1.0) / 2.0


def _golden_min(phi, lo, hi, iters=200):
    """Minimiser of a convex function on [lo, hi] by golden-section search."""
    a, b = lo, hi
    c = b - _GOLD * (b - a)
    d = a + _GOLD * (b - a)
    fc, fd = phi(c), phi(d)
    for _ in range(iters):
        if fc <= fd:
            b, d, fd = d, c, fc
            c = b - _GOLD * (b - a)
            fc = phi(c)
        else:
            a, c, fc = c, d, fd
            d = a + _GOLD * (b - a)
            fd = phi(d)
        if b - a < 1e-15 * max(1.0, abs(a)):
            break
    # the search never evaluates the end points: a minimiser on the boundary of the box
    # (an active bound) is taken from there
    t = 0.5 * (a + b)
    for e in (lo, hi):
        if phi(e) <= phi(t):
            t = e
    return t


def _hminus_slope(prob, xj, h=1e-6):
    """(h^-)'(x_j) by central differences of h^- = eta|t| - h(t) (C^1, Section 4.3)."""
    if prob.reg == "l1":
        return 0.0
    eta = prob.eta()
    f = lambda t: eta * abs(t) - float(prob.h(np.array([t]))[0])
    return (f(xj + h) - f(xj - h)) / (2 * h)


def _surrogate_argmins(prob, x, tau):
    """Every coordinate's best response by direct minimisation of its surrogate
    (subproblem (2) with the Section 4.3 linearisation and the separable surrogate of
    vector blocks): phi_j(t) = 1/2||r + a_j (t - x_j)||^2 + tau/2 (t - x_j)^2
    - 2c x_j (t - x_j) - lam (h^-)'(x_j)(t - x_j) + lam eta |t|, over [-beta, beta]."""
    A = np.asarray(prob.A, dtype=np.float64)
    r = A @ x - prob.b
    eta = prob.eta()
    out = np.empty(prob.n)
    for j in range(prob.n):
        a = A[:, j]
        d = _hminus_slope(prob, x[j])

        def phi(t, a=a, xj=x[j], d=d):
            s = t - xj
            # 1/2||r + a s||^2 - 1/2||r||^2, summed term by term (no expansion in ||a||^2)
            quad = float(np.sum(0.5 * a * s * (2.0 * r + a * s)))
            return (quad + 0.5 * tau * s * s - 2.0 * prob.c * xj * s - prob.lam * d * s
                    + prob.lam * eta * abs(t))

        if math.isfinite(prob.beta):
            lo, hi = -prob.beta, prob.beta
        else:
            lo, hi = x[j] - 60.0, x[j] + 60.0
        out[j] = _golden_min(phi, lo, hi)
    return out


@pytest.mark.parametrize("reg,theta,c,beta", [("l1", 0.0, 0.0, math.inf),
                                              ("l1", 0.0, 0.2, 1.1),
                                              ("log", 20.0, 0.0, math.inf),
                                              ("exp", 6.0, 0.1, 2.0)])
def test_merit_and_nnz_match_direct_surrogate_minimisation(reg, theta, c, beta):
    rng = np.random.default_rng(41)
    m, n = 14, 11
    A = rng.normal(size=(m, n))
    A /= np.linalg.norm(A, axis=0)
    b = rng.normal(size=m)
    lam = 0.5 if reg == "l1" else 0.05
    prob = O.Problem(A=A, b=b, lam=lam, c=c, beta=beta, reg=reg, theta=theta)
    tau = 0.7  # large enough that leaving tau out of q_j moves every best response
    nnz_differs = []
    for trial in range(3):
        x = rng.uniform(-1.0, 1.0, n)
        if trial == 2:
            x[rng.choice(n, 4, replace=False)] = 0.0
        t = _surrogate_argmins(prob, x, tau)
        zero = np.abs(t) < 1e-7
        # no best response sits near the threshold, so the zero test is unambiguous
        assert np.all(zero | (np.abs(t) > 1e-4))
        d = np.abs(t - x)
        merit_direct = float(np.max(d))
        # the direct minimiser is resolved to about sqrt(eps): 1e-7
        assert abs(O.merit(prob, x, tau) - merit_direct) <= 1e-7
        assert O.nnz_best_response(prob, x, tau) == int(np.count_nonzero(~zero))
        # the test separates the inf-norm from the 2-norm and nnz(x_hat) from nnz(x)
        assert np.linalg.norm(t - x) > merit_direct + 1e-3
        nnz_differs.append(int(np.count_nonzero(~zero)) != int(np.count_nonzero(x)))
        # the oracle's best response agrees coordinate by coordinate
        xh = O.best_response(prob, x, A @ x - b, np.arange(n), tau)
        np.testing.assert_allclose(xh, t, atol=1e-7)
        assert np.array_equal(xh == 0.0, zero)
    assert any(nnz_differs)


def test_merit_zero_exactly_at_fixed_points_and_positive_elsewhere():
    """At x = x_hat(x) the merit vanishes (Section 4.3: zero iff stationary): on an
    orthonormal A with c = 0 and tau = 0, x_hat(x) = soft(A^T b, lam) for every x."""
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.normal(size=(20, 8)))
    b = rng.normal(size=20)
    lam = 0.3
    prob = O.Problem(A=Q, b=b, lam=lam)
    v = Q.T @ b
    xstar = np.sign(v) * np.maximum(np.abs(v) - lam, 0.0)
    assert O.merit(prob, xstar, 0.0) <= 1e-14
    x = xstar + rng.normal(size=8) * 0.1
    # x_hat(x) = soft(A^T b) whatever x is, so the merit is the distance to x*
    assert abs(O.merit(prob, x, 0.0) - np.max(np.abs(x - xstar))) <= 1e-14
    assert O.nnz_best_response(prob, x, 0.0) == int(np.count_nonzero(xstar))


# ---------------------------------------------------------------- DC regularisers
@pytest.mark.parametrize("theta", [0.5, 3.0, 20.0])
def test_dc_regulariser_special_values(theta):
    """h(0) = 0 for both; h_log(+-1) = 1 (its normalisation); h_exp -> 1 at infinity while
    h_log grows without bound; both even, increasing and concave on t > 0."""
    pe = O.Problem(A=np.eye(1), b=np.zeros(1), lam=1.0, reg="exp", theta=theta)
    pl = O.Problem(A=np.eye(1), b=np.zeros(1), lam=1.0, reg="log", theta=theta)
    for p in (pe, pl):
        assert float(p.h(np.array([0.0]))[0]) == 0.0
        t = np.linspace(1e-3, 5.0, 4001) / theta  # h_exp is 1 to rounding beyond ~37/theta
        ht = p.h(t)
        np.testing.assert_array_equal(p.h(-t), ht)
        assert np.all(np.diff(ht) > 0)
        assert np.all(ht[:-2] - 2 * ht[1:-1] + ht[2:] < 0)  # strictly concave
    np.testing.assert_allclose(pl.h(np.array([1.0, -1.0])), [1.0, 1.0], rtol=0, atol=1e-15)
    assert abs(float(pe.h(np.array([40.0 / theta]))[0]) - 1.0) <= 1e-15
    assert float(pl.h(np.array([1e6]))[0]) > 2.0
    # h_exp at t = 1/theta is 1 - 1/e; h_log at t = (e - 1)/theta is 1/log(1 + theta)
    assert abs(float(pe.h(np.array([1.0 / theta]))[0]) - (1.0 - math.exp(-1.0))) <= 1e-15
    assert abs(float(pl.h(np.array([(math.e - 1.0) / theta]))[0])
               - 1.0 / math.log1p(theta)) <= 1e-14


@pytest.mark.parametrize("reg", ["exp", "log"])
@pytest.mark.parametrize("theta", [0.5, 3.0, 20.0])
def test_dc_eta_is_the_slope_at_zero(reg, theta):
    """eta = h'(0+): the DC split h = eta|x| - h^- of Section 4.3 needs h^- to be C^1, so
    eta must equal the one-sided slope of h at 0 (Richardson-extrapolated differences)."""
    p = O.Problem(A=np.eye(1), b=np.zeros(1), lam=1.0, reg=reg, theta=theta)
    d = lambda dt: float(p.h(np.array([dt]))[0]) / dt
    dt = 1e-5 / theta
    slope = 2.0 * d(dt / 2) - d(dt)  # cancels the O(dt) term
    assert abs(p.eta() - slope) <= 1e-7 * p.eta()
    # h^- has zero slope at 0 from both sides
    np.testing.assert_allclose(p.dh_minus(np.array([0.0, 1e-12, -1e-12])), 0.0, atol=1e-9)


# ---------------------------------------------------------------- scipy.sparse branch
def _sparse_matrix(rng, m, n, density):
    import scipy.sparse as sp
    M = sp.random(m, n, density=density, random_state=np.random.RandomState(int(rng.integers(1 << 30))),
                  data_rvs=lambda k: rng.normal(size=k))
    M = M.tolil()
    M[:, 3] = 0.0  # an empty column
    M = M.tocsc()
    M.eliminate_zeros()
    return M


@pytest.mark.parametrize("fmt", ["csc", "csr"])
def test_sparse_branch_equals_dense(fmt):
    rng = np.random.default_rng(7)
    m, n = 50, 90
    M = _sparse_matrix(rng, m, n, 0.08)
    M = M.asformat(fmt).astype(np.float32)
    D = M.toarray()
    b = rng.normal(size=m)
    bp = inputs.block_partition(n, 7)
    kw = dict(b=b, lam=0.05, c=0.1, beta=1.5, block_ptr=bp)
    ps, pd = O.Problem(A=M, **kw), O.Problem(A=D, **kw)
    tol = 1e-14
    np.testing.assert_allclose(ps.colnorm2(), pd.colnorm2(), rtol=tol, atol=tol)
    assert ps.colnorm2()[3] == 0.0
    r = rng.normal(size=m)
    v = rng.normal(size=n)
    idx = np.array([0, 3, 5, 17, 89])
    np.testing.assert_allclose(ps.Atr(r), pd.Atr(r), rtol=tol, atol=tol)
    np.testing.assert_allclose(ps.Atr(r, idx), pd.Atr(r, idx), rtol=tol, atol=tol)
    np.testing.assert_allclose(ps.Av(v), pd.Av(v), rtol=tol, atol=tol)
    np.testing.assert_allclose(ps.Av(v[idx], idx), pd.Av(v[idx], idx), rtol=tol, atol=tol)
    cfg = O.RunConfig(tau=0.5, gamma=0.9, p=0.6, seed=3)
    x0 = np.zeros(n)
    xs, rs, us = O.run_rounds(ps, cfg, x0, O.residual(ps, x0), 0, 15)
    xd, rd, ud = O.run_rounds(pd, cfg, x0, O.residual(pd, x0), 0, 15)
    assert us == ud
    np.testing.assert_allclose(xs, xd, rtol=tol, atol=tol)
    np.testing.assert_allclose(rs, rd, rtol=tol, atol=tol)
    assert abs(O.objective(ps, xs) - O.objective(pd, xd)) <= tol * abs(O.objective(pd, xd))
    assert abs(O.merit(ps, xs, 0.5) - O.merit(pd, xd, 0.5)) <= tol
    assert abs(O.stationarity_MF(ps, xs) - O.stationarity_MF(pd, xd)) <= tol
    assert O.nnz_best_response(ps, xs, 0.5) == O.nnz_best_response(pd, xd, 0.5)
    H = O.reduced_hessian(ps, idx)
    np.testing.assert_allclose(H, O.reduced_hessian(pd, idx), rtol=tol, atol=tol)


# ---------------------------------------------------------------- residual refresh in solve()
def test_solve_refresh_every_replaces_the_residual_at_its_checks():
    w = inputs.dense_problem(40, 90, nnz_frac=0.1, lam_frac=0.1, block=6, p=0.5,
                             dtype=torch.float64, seed=2)
    prob = O.Problem(A=w.A_numpy(), b=w.b.double().numpy(), lam=w.lam, block_ptr=w.block_ptr)
    cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=0)
    plain = O.solve(prob, cfg, max_rounds=35, check_every=5)
    # refresh at every check: the returned residual is the fresh one, bit for bit
    ref1 = O.solve(prob, cfg, max_rounds=35, check_every=5, refresh_every=1)
    assert np.array_equal(ref1["r"], O.residual(prob, ref1["x"]))
    # refresh every 3rd check: 7 checks, refreshed after rounds 15 and 30; the last
    # check's residual is the running one started from the fresh residual after round 30
    ref3 = O.solve(prob, cfg, max_rounds=35, check_every=5, refresh_every=3)
    x, r, k = np.zeros(prob.n), O.residual(prob, np.zeros(prob.n)), 0
    for nr, fresh in ((15, True), (15, True), (5, False)):
        x, r, _ = O.run_rounds(prob, cfg, x, r, k, nr)
        k += nr
        if fresh:
            r = O.residual(prob, x)
    assert np.array_equal(ref3["x"], x) and np.array_equal(ref3["r"], r)
    assert not np.array_equal(ref3["r"], O.residual(prob, ref3["x"]))
    # in FP64 the refresh moves the iterates only by rounding
    for out in (ref1, ref3):
        np.testing.assert_allclose(out["x"], plain["x"], atol=1e-13)
        assert out["rounds"] == plain["rounds"] == 35
