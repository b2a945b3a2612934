"""sca_adjoint_noalloc -- the adjoint with its workspace in the library's fixed device array
instead of memory allocated on the first call -- against sca_adjoint, through the C ABI:
two calls in a row on one GPU, the second with a smaller problem (the array keeps the first
call's contents), in FP64 and FP32; and the rejection of a problem beyond the array."""
import numpy as np
import pytest
import torch

from paper_1701_04900_amd import inputs, sca

pytestmark = pytest.mark.gpu


def _solved(w):
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    tol = 1e-13 if w.dtype == torch.float64 else 1e-6
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, max_rounds=50000,
                      check_every=20, tol_merit=tol)
    x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
    sca.sca_solve(P.handle, o, x)
    return wd, P, o, x


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_adjoint_equals_the_allocating_adjoint_on_two_calls(dtype):
    big = inputs.dense_problem(300, 900, nnz_frac=0.05, lam_frac=0.1, block=8, p=1.0,
                               dtype=dtype, seed=31)
    small = inputs.dense_problem(120, 260, nnz_frac=0.05, lam_frac=0.1, block=4, p=1.0,
                                 dtype=dtype, seed=32)
    tol = 1e-10 if dtype == torch.float64 else 1e-6
    for w in (big, small):  # the second call with a smaller input
        print(f"[gpu] no-alloc adjoint {w.m}x{w.n} {dtype}", flush=True)
        wd, P, o, x = _solved(w)
        rng = np.random.default_rng(w.m)
        xbar = torch.from_numpy(rng.normal(size=w.n)).to(dtype).cuda()
        b_ref = torch.empty(w.m, dtype=dtype, device="cuda")
        lb_ref = sca.sca_adjoint(P.handle, o, x, xbar, b_ref)
        b_new = torch.full((w.m,), float("nan"), dtype=dtype, device="cuda")
        lb_new = sca.sca_adjoint_noalloc(P.handle, o, x, xbar, b_new)
        torch.cuda.synchronize()
        scale = max(1.0, float(b_ref.abs().max()))
        err = float((b_new - b_ref).abs().max()) / scale
        print(f"[parity] no-alloc adjoint {w.m}x{w.n}: bbar err {err:.2e}, lambar "
              f"{lb_new!r} vs {lb_ref!r}, bitwise {bool(torch.equal(b_new, b_ref))}", flush=True)
        assert bool(torch.isfinite(b_new).all())
        assert err <= tol
        assert abs(lb_new - lb_ref) <= tol * max(1.0, abs(lb_ref))
        P.close()


def test_noalloc_adjoint_rejects_a_problem_beyond_its_array():
    w = inputs.dense_problem(130000, 10, nnz_frac=0.2, lam_frac=0.1, block=2, p=1.0,
                             dtype=torch.float32, seed=33)
    wd = w.to("cuda")
    P = sca.Problem.from_workload(wd)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
    x = torch.zeros(w.n, dtype=torch.float32, device="cuda")
    bbar = torch.zeros(w.m, dtype=torch.float32, device="cuda")
    with pytest.raises(sca.SCAError) as e:
        sca.sca_adjoint_noalloc(P.handle, o, x, torch.ones_like(x), bbar)
    assert e.value.status == sca.SCA_EINVAL
    assert "beyond the fixed" in str(e.value)
    P.close()
