"""GPU parity of both batched round kinds (the fused round and the two-pass round) on the
variants of the method: box-nonconvex instances (c > 0, finite beta), the DC regularisers of
Section 4.3 and the diminishing step of Section 4.1.  Every instance is compared with the FP64
oracle run with its own instance word; FP64 iterates and residuals within 1e-10 relative."""
import math

import numpy as np
import pytest
import torch

from oracle import sca_oracle as O
from paper_1701_04900_amd import inputs, sca

pytestmark = pytest.mark.gpu

ROUNDS, P, SEED = 20, 0.4, 9


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def _instances(c_frac=0.0, beta=math.inf, seed=60):
    ws = inputs.batch_lasso(5, m_range=(300, 2100), n_ratio=2, nnz_frac=0.03,
                            lam_range=(1e-2, 1e-1), c_frac=c_frac, beta=beta, block=16, p=P,
                            dtype=torch.float64, seed=seed)
    for k, w in enumerate(ws):
        w.instance = k
    return ws


def _compare(ws, kind, gamma=0.9, gamma_mu=0.0, reg=None, code=None, theta=0.0):
    print(f"[gpu] batch kind {kind}: m = {[w.m for w in ws]} c = {ws[0].c:.3g} "
          f"beta = {ws[0].beta} reg = {reg} gamma_mu = {gamma_mu}", flush=True)
    B = sca.Batch([w.to("cuda") for w in ws])
    sca.sca_batch_set_launch(B.handle, kind, 4, 2)
    assert sca.sca_batch_get_launch(B.handle)["grad_kind"] == kind
    if code is not None:
        sca.sca_batch_set_regularizer(B.handle, code, theta)
    o = sca.make_opts(gamma=gamma, gamma_mu=gamma_mu, select_p=P, seed=SEED)
    x = torch.zeros(int(B.xoff[-1]), dtype=torch.float64, device="cuda")
    r = torch.zeros(int(B.roff[-1]), dtype=torch.float64, device="cuda")
    sca.sca_batch_residual(B.handle, x, r)
    sca.sca_batch_step(B.handle, o, 0, ROUNDS, x, r)
    torch.cuda.synchronize()
    xh, rh = x.cpu().numpy(), r.cpu().numpy()
    for k, w in enumerate(ws):
        kw = {} if reg is None else dict(reg=reg, theta=theta)
        prob = O.Problem(A=w.A_numpy(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                         beta=w.beta, block_ptr=w.block_ptr, **kw)
        cfg = O.RunConfig(tau=w.tau, gamma=gamma, gamma_mu=gamma_mu, p=P, seed=SEED, instance=k)
        x0 = np.zeros(w.n)
        xo, ro, _ = O.run_rounds(prob, cfg, x0, O.residual(prob, x0), 0, ROUNDS)
        ex = _rel(xh[B.xoff[k]:B.xoff[k + 1]], xo)
        er = _rel(rh[B.roff[k]:B.roff[k] + w.m], ro)
        print(f"[parity] instance {k} m={w.m}: x {ex:.2e} r {er:.2e}", flush=True)
        assert ex <= 1e-10 and er <= 1e-10, (k, ex, er)
        if w.beta < math.inf:
            assert np.max(np.abs(xh[B.xoff[k]:B.xoff[k + 1]])) <= w.beta
    B.close()


@pytest.mark.parametrize("kind", [1, 0])
def test_batch_box_nonconvex_fp64(kind):
    _compare(_instances(c_frac=0.3, beta=0.5, seed=61), kind)


@pytest.mark.parametrize("kind", [1, 0])
@pytest.mark.parametrize("reg,code", [("log", sca.SCA_REG_LOG), ("exp", sca.SCA_REG_EXP)])
def test_batch_dc_regularisers_fp64(kind, reg, code):
    _compare(_instances(seed=62), kind, reg=reg, code=code, theta=20.0)


@pytest.mark.parametrize("kind", [1, 0])
def test_batch_diminishing_stepsize_fp64(kind):
    _compare(_instances(seed=63), kind, gamma=1.0, gamma_mu=1e-2)
