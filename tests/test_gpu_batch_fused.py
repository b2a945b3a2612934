"""GPU parity of the batch's two round kinds -- the fused round (one pass over the drawn
columns, fold from registers, workgroup shares cut by cost) and the two-pass round --
against the FP64 oracle run per instance with the same instance word, for every fused
grid (workgroups per CU); instances shared by several workgroups and
instances held whole by one; bitwise determinism of each shape; the limits of the fused
kind.  Tolerances: FP64 1e-10 relative, FP32 objective 1e-4 and iterates x_tol(m)."""
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


def _oracle_rounds(w, k, p, seed, rounds):
    prob = O.Problem(A=w.A_numpy(), b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c,
                     beta=w.beta, block_ptr=w.block_ptr)
    cfg = O.RunConfig(tau=w.tau, gamma=0.9, p=p, seed=seed, instance=k)
    bp = prob.blocks()
    x = np.zeros(w.n)
    r = O.residual(prob, x)
    moved = 0
    for kk in range(rounds):
        idx = O.block_columns(bp, O.selected_blocks(seed, kk, k, len(bp) - 1, p))
        x, r, mv = O.sca_round(prob, x, r, w.tau, 0.9, idx)
        moved += mv
    del cfg
    return prob, x, r, moved


def _gpu(B, ws, p, seed, rounds, dtype):
    o = sca.make_opts(gamma=0.9, select_p=p, seed=seed, max_rounds=rounds, check_every=rounds)
    x = torch.zeros(int(B.xoff[-1]), dtype=dtype, device="cuda")
    r = torch.zeros(int(B.roff[-1]), dtype=dtype, device="cuda")
    sca.sca_batch_residual(B.handle, x, r)
    sca.sca_batch_step(B.handle, o, 0, rounds, x, r)
    torch.cuda.synchronize()
    return o, x, r


def _mixed_batch(dtype, seed):
    """One large instance (its drawn columns span many workgroups' shares) among small ones
    (each held whole by one workgroup), odd m throughout (ragged last row group)."""
    big = inputs.batch_lasso(1, m_range=(4095, 4095), n_ratio=2, nnz_frac=0.03, block=32,
                             p=0.4, dtype=dtype, seed=seed)[0]
    small = inputs.batch_lasso(6, m_range=(31, 96), n_ratio=3, nnz_frac=0.05, block=8, p=0.4,
                               dtype=dtype, seed=seed + 1)
    ws = small[:3] + [big] + small[3:]
    for k, w in enumerate(ws):
        w.instance = k
    return ws


@pytest.mark.parametrize("kind,cols,wg", [(1, 4, 1), (1, 4, 2), (1, 4, 4), (1, 4, 3), (0, 4, 2)])
def test_batch_round_kinds_fp64_match_oracle(kind, cols, wg):
    ws = _mixed_batch(torch.float64, 40)
    print(f"[gpu] batch kind {kind} cols {cols} wg/CU {wg}: m = {[w.m for w in ws]}", flush=True)
    B = sca.Batch([w.to("cuda") for w in ws])
    sca.sca_batch_set_launch(B.handle, kind, cols, wg)
    got = sca.sca_batch_get_launch(B.handle)
    assert got["grad_kind"] == kind
    rounds = 20
    _, x, r = _gpu(B, ws, 0.4, 5, rounds, torch.float64)
    st = sca.sca_batch_solve(B.handle, sca.make_opts(gamma=0.9, select_p=0.4, seed=5,
                                                     max_rounds=rounds, check_every=rounds),
                             torch.zeros_like(x), B.K, raise_on_notconv=False)
    xh, rh = x.cpu().numpy(), r.cpu().numpy()
    moved_total = 0
    for k, w in enumerate(ws):
        _, xo, ro, mv = _oracle_rounds(w, k, 0.4, 5, rounds)
        moved_total += mv
        ex = _rel(xh[B.xoff[k]:B.xoff[k + 1]], xo)
        er = _rel(rh[B.roff[k]:B.roff[k] + w.m], ro)
        assert ex <= 1e-10 and er <= 1e-10, (k, ex, er)
        # padding rows of the concatenated residual stay zero
        assert np.all(rh[B.roff[k] + w.m:B.roff[k + 1]] == 0.0)
    assert st[0]["moved_updates"] == moved_total


@pytest.mark.parametrize("cols,wg", [(4, 1), (4, 2), (4, 4)])
def test_fused_batch_is_bitwise_deterministic(cols, wg):
    ws = _mixed_batch(torch.float32, 44)
    B = sca.Batch([w.to("cuda") for w in ws])
    sca.sca_batch_set_launch(B.handle, 1, cols, wg)
    _, x1, r1 = _gpu(B, ws, 0.4, 2, 15, torch.float32)
    _, x2, r2 = _gpu(B, ws, 0.4, 2, 15, torch.float32)
    assert torch.equal(x1, x2) and torch.equal(r1, r2)


def test_fused_batch_fp32_up_to_8192_rows():
    ws = inputs.batch_lasso(5, m_range=(5000, 8191), n_ratio=1, nnz_frac=0.02,
                            lam_range=(1e-2, 5e-2), block=64, p=0.25, dtype=torch.float32,
                            seed=46)
    ws[2] = inputs.batch_lasso(1, m_range=(8192, 8192), n_ratio=1, nnz_frac=0.02, block=64,
                               p=0.25, dtype=torch.float32, seed=47)[0]
    for k, w in enumerate(ws):
        w.instance = k
    B = sca.Batch([w.to("cuda") for w in ws])
    sca.sca_batch_set_launch(B.handle, 1, 4, 2)
    o, x, r = _gpu(B, ws, 0.25, 7, 20, torch.float32)
    rep = sca.sca_batch_objective(B.handle, o, x, B.K)
    for k, w in enumerate(ws):
        prob, xo, _, _ = _oracle_rounds(w, k, 0.25, 7, 20)
        Fo = O.objective(prob, xo)
        ex = _rel(x[B.xoff[k]:B.xoff[k + 1]].double().cpu().numpy(), xo)
        print(f"[parity] fused batch fp32 instance {k} m={w.m}: x err {ex:.2e}, F rel err "
              f"{abs(rep['F'][k] - Fo) / abs(Fo):.2e}", flush=True)
        assert abs(rep["F"][k] - Fo) <= 1e-4 * abs(Fo), k
        assert ex <= x_tol(w.m), k


def test_fused_batch_limits():
    """FP64 instances beyond 4096 rows run the two-pass round (the fused kind is refused);
    shapes outside the documented lists are refused."""
    ws = inputs.batch_lasso(2, m_range=(4097, 4200), n_ratio=1, nnz_frac=0.02, block=64,
                            p=0.25, dtype=torch.float64, seed=48)
    B = sca.Batch([w.to("cuda") for w in ws])
    assert sca.sca_batch_get_launch(B.handle)["grad_kind"] == 0
    with pytest.raises(sca.SCAError) as e:
        sca.sca_batch_set_launch(B.handle, 1, 4, 2)
    assert e.value.status == sca.SCA_EINVAL
    ws32 = inputs.batch_lasso(2, m_range=(100, 200), n_ratio=2, nnz_frac=0.02, block=8, p=0.5,
                              dtype=torch.float32, seed=49)
    B32 = sca.Batch([w.to("cuda") for w in ws32])
    for bad in ((1, 3, 2), (1, 4, 5), (1, 4, 0), (2, 4, 2), (1, 8, 2)):
        with pytest.raises(sca.SCAError) as e:
            sca.sca_batch_set_launch(B32.handle, *bad)
        assert e.value.status == sca.SCA_EINVAL


def test_batch_solve_checks_on_the_running_residual_stop_like_the_plain_path():
    """With the relative-error test on the running residual (confirmed fresh), each instance
    of a fused FP32 batch stops at the same check as its own plain solve, and its final
    relative error is below the tolerance."""
    ws = inputs.batch_lasso(4, m_range=(300, 1500), nnz_frac=0.03, lam_range=(2e-2, 1e-1),
                            block=16, p=0.5, dtype=torch.float32, seed=50)
    Fs = []
    for k, w in enumerate(ws):
        w.instance = k
        P64 = sca.Problem.dense(w.At.double().cuda(), w.m, w.b.double().cuda(), w.lam,
                                block_ptr=w.block_ptr)
        o64 = sca.make_opts(gamma=0.9, tau=w.tau, select_p=0.5, seed=3, instance=k,
                            max_rounds=50000, check_every=20, tol_merit=1e-12)
        x64 = torch.zeros(w.n, dtype=torch.float64, device="cuda")
        Fs.append(sca.sca_solve(P64.handle, o64, x64)["F"])
        P64.close()
    wd = [w.to("cuda") for w in ws]
    B = sca.Batch(wd, F_star=Fs)
    opts = sca.make_opts(gamma=0.9, select_p=0.5, seed=3, max_rounds=20000, check_every=10,
                         tol_rel_obj=1e-5)
    xb = torch.zeros(int(B.xoff[-1]), dtype=torch.float32, device="cuda")
    st = sca.sca_batch_solve(B.handle, opts, xb, B.K)
    for k, w in enumerate(wd):
        assert st[k]["status"] == sca.SCA_OK and st[k]["rel_err"] <= 1e-5, (k, st[k])
        P = sca.Problem.from_workload(w)
        o = sca.make_opts(gamma=0.9, tau=ws[k].tau, select_p=0.5, seed=3, instance=k,
                          max_rounds=20000, check_every=10, tol_rel_obj=1e-5, F_star=Fs[k])
        xp = torch.zeros(w.n, dtype=torch.float32, device="cuda")
        sp = sca.sca_solve(P.handle, o, xp)
        print(f"[gpu] instance {k}: batch {st[k]['rounds']} rounds, plain {sp['rounds']}",
              flush=True)
        assert abs(sp["rounds"] - st[k]["rounds"]) <= 10
        P.close()
