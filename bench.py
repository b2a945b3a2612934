"""Benchmark of the SCA block-update hot path on one MI355X.

Workload: LASSO, dense A 20000 x 100000 (N(0,1), unit-norm columns, FP32), x* with 1%
nonzeros +-[1,2], noise sigma 0.01, lam = 0.01 ||A^T b||_inf, blocks of 64 coordinates,
25% of blocks drawn per round, gamma 0.9, tau from the random-matrix estimate.

One timed step = one complete solve from x = 0 until the relative objective error
(F - F*)/|F*| <= 1e-6 (every round: block draw, gradient + best response + step and the
residual fold, at this size one fused kernel plus the reduction of its partials; every 10
rounds: FP64 objective; the stop is confirmed with a fresh FP64 residual).  value = coordinate updates per second over the timed solves; ms_per_step =
time to tolerance.  F* comes from an FP64 solve of the same stored data to merit <= 1e-12.

The JSON line also carries the roofline of the dominant kernel (the gradient pass, timed
with HIP events on its launch stream over the timed region) and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1701_04900_amd import inputs, sca  # noqa: E402

METRIC = "coord-updates/s + time to 1e-6 rel. error, % HBM roofline; batched/adjoint vs plain"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


F_STAR_MERIT = 1e-13
F_STAR_GAP = 1e-10     # the gap that certifies F* (reported as "certified")
F_STAR_GAP_FAIL = 1e-8  # a gap beyond this (1% of the 1e-6 tolerance) stops the bench


def _checked_fstar_solve(st, what):
    """The F* solve must have converged: a solve stopped short would overstate F* and end
    the timed solves early."""
    if st["status"] != sca.SCA_OK or not st["merit"] <= F_STAR_MERIT:
        raise RuntimeError(f"{what}: the FP64 reference solve did not reach merit "
                           f"{F_STAR_MERIT:g} (status {st['status']}, merit {st['merit']:.3e}, "
                           f"{st['rounds']} rounds)")


def reference_optimum(w, opts_kw, want_x=False):
    """F* by an FP64 solve of the stored FP32 data (upcast copy) to merit <= 1e-12."""
    At64 = w.At.double()
    b64 = w.b.double()
    P = sca.Problem.dense(At64, w.m, b64, w.lam, w.c, w.beta, w.block_ptr)
    o = sca.make_opts(**opts_kw, max_rounds=200000, check_every=50, tol_merit=F_STAR_MERIT)
    x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    st = sca.sca_solve(P.handle, o, x, raise_on_notconv=False)
    P.close()
    del At64, b64
    torch.cuda.empty_cache()
    _checked_fstar_solve(st, w.name)
    if want_x:
        return st["F"], st, x.cpu().numpy()
    return st["F"], st


def certify_fstar(w, F_star, xstar):
    """An FP64 check of F* on the host that shares nothing with the GPU path: at the FP64
    solution x* (l1 regulariser, no box, c = 0) it recomputes with numpy (scipy for sparse A)
    the residual r = A x* - b, the objective P(x*) = 1/2||r||^2 + lam ||x*||_1, the gradient
    g = A^T r over all columns, ||M_F(x*)||_2 = ||x* - soft(x* - g, lam)||_2 and the LASSO
    duality gap: nu = s r with s = min(1, lam / ||g||_inf) is dual feasible, its dual value is
    D = -1/2||nu||^2 - b^T nu <= P*, so P(x*) - D bounds the error of F* = P(x*).  F* is
    accepted when the gap is <= 1e-10 |F*|."""
    t0 = time.perf_counter()
    xs = np.asarray(xstar, dtype=np.float64)
    b = w.b.double().cpu().numpy()
    nz = np.flatnonzero(xs)
    if hasattr(w, "rowptr"):
        A = w.scipy_csr().astype(np.float64)
        r = A @ xs - b
        g = np.asarray(A.T @ r).ravel()
    else:
        At = w.At.cpu()  # (n, lda) FP32, row j = column j of A
        r = -b.copy()
        for j0 in range(0, len(nz), 4096):
            idx = torch.from_numpy(nz[j0:j0 + 4096])
            cols = At[idx, : w.m].double().numpy()
            r += cols.T @ xs[nz[j0:j0 + 4096]]
        g = np.empty(w.n)
        for j0 in range(0, w.n, 8192):
            g[j0:j0 + 8192] = At[j0:j0 + 8192, : w.m].double().numpy() @ r
    P = 0.5 * float(r @ r) + w.lam * float(np.abs(xs).sum())
    v = xs - g
    y = np.sign(v) * np.maximum(np.abs(v) - w.lam, 0.0)
    MF = float(np.linalg.norm(xs - y))
    s = min(1.0, w.lam / float(np.max(np.abs(g))))
    D = -0.5 * s * s * float(r @ r) - s * float(b @ r)
    gap = P - D
    out = dict(F_star=F_star, host_F=P, host_MF=MF, dual=D, gap=gap,
               rel_gap=gap / abs(P), F_star_vs_host=abs(F_star - P) / abs(P),
               certified=bool(gap <= F_STAR_GAP * abs(P)
                              and abs(F_star - P) <= F_STAR_GAP * abs(P)),
               seconds=round(time.perf_counter() - t0, 2),
               method="numpy FP64 on the host at the FP64 GPU solution: fresh residual, "
                      "objective, ||M_F||, LASSO duality gap")
    log(f"F* check ({w.name}): host F {P:.15g}, gap {gap:.3e} ({gap / abs(P):.2e} relative), "
        f"||M_F|| {MF:.2e}, {out['seconds']} s")
    if not (gap <= F_STAR_GAP_FAIL * abs(P) and abs(F_star - P) <= F_STAR_GAP_FAIL * abs(P)):
        raise RuntimeError(f"F* of {w.name} is not within {F_STAR_GAP_FAIL:g} of the optimum: {out}")
    return out


def cpu_baseline(w, opts_kw, rounds):
    """The oracle as it stands (FP64 numpy) on the host cores: `rounds` rounds of the same
    workload from x = 0."""
    from oracle import sca_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    if hasattr(w, "rowptr"):
        A = w.scipy_csr().tocsc()
        what = f"{w.m}x{w.n} sparse FP32 LASSO ({w.nnz} nonzeros)"
    else:
        A = w.At.cpu()[:, : w.m].numpy().T
        what = f"{w.m}x{w.n} FP32 {'box-nonconvex problem' if w.c else 'LASSO'}"
    prob = O.Problem(A=A, b=w.b.double().cpu().numpy(), lam=w.lam, c=w.c, beta=w.beta,
                     block_ptr=w.block_ptr)
    cfg = O.RunConfig(tau=opts_kw["tau"], gamma=opts_kw["gamma"], p=opts_kw["select_p"],
                      seed=opts_kw["seed"])
    prob.colnorm2()  # the per-problem set-up (the GPU side does it at create time)
    x = np.zeros(w.n)
    r = O.residual(prob, x)
    t0 = time.perf_counter()
    x, r, upd = O.run_rounds(prob, cfg, x, r, 0, rounds)
    dt = time.perf_counter() - t0
    return dict(value=upd / dt, unit="coord-updates/s", cores=int(threads), kind="oracle",
                seconds_per_round=dt / rounds,
                sample=f"{rounds} rounds from x=0 of the same {what} "
                       f"({upd} coordinate updates in {dt:.1f} s, FP64 numpy)")


def batch_reference_optima(ws, gamma, p, seed, budget_bytes=24e9):
    """F*_k by FP64 batched solves (upcast copies, in chunks that fit beside the FP32 data)
    to merit <= 1e-11 per instance."""
    F = []
    k0 = 0
    while k0 < len(ws):
        k1, nb = k0, 0.0
        while k1 < len(ws) and (k1 == k0 or nb + ws[k1].At.numel() * 8 <= budget_bytes):
            nb += ws[k1].At.numel() * 8
            k1 += 1
        chunk = []
        for w in ws[k0:k1]:
            chunk.append(inputs.DenseWorkload(w.name, w.At.double(), w.m, w.n, w.lda, w.b.double(),
                                              w.x_true, w.lam, w.c, w.beta, w.tau, w.block_ptr,
                                              w.p, w.gamma, w.seed, w.instance))
        B = sca.Batch(chunk)
        o = sca.make_opts(gamma=gamma, select_p=p, seed=seed, max_rounds=200000, check_every=50,
                          tol_merit=1e-11)
        x = torch.zeros(int(B.xoff[-1]), dtype=torch.float64, device="cuda")
        st = sca.sca_batch_solve(B.handle, o, x, B.K, raise_on_notconv=False)
        F += [s["F"] for s in st]
        log(f"F* for instances {k0}..{k1 - 1}: max rounds {max(s['rounds'] for s in st)}, "
            f"max merit {max(s['merit'] for s in st):.1e}")
        B.close()
        del chunk, x
        torch.cuda.empty_cache()
        k0 = k1
    return F


def bench_batch(args):
    """256 LASSO instances, m_k uniform in [500, 8000], n_k = 5 m_k, FP32, lam_k log-spaced
    over [1e-3, 1e-1] ||A_k^T b_k||_inf, 2% sparse x*, blocks of 64, p = 0.25, gamma 0.9:
    batched solve to rel. error 1e-6 against the same instances solved one after another by
    the plain path, then the batched adjoint against the plain adjoints."""
    K = args.instances
    t0 = time.perf_counter()
    ws = inputs.batch_lasso(K, m_range=(500, 8000), nnz_frac=0.02, lam_range=(1e-3, 1e-1),
                            block=64, p=0.25, dtype=torch.float32, seed=0, device="cuda")
    torch.cuda.synchronize()
    abytes = sum(w.At.numel() for w in ws) * 4
    log(f"generated {K} instances ({abytes / 1e9:.1f} GB of A) in {time.perf_counter() - t0:.1f} s")
    gamma, p, seed = 0.9, 0.25, 0
    t0 = time.perf_counter()
    if args.fstar_file and os.path.exists(args.fstar_file):
        # F*_k of an earlier run of the same seeded instances (FP64 solves to merit 1e-11)
        F_star = json.load(open(args.fstar_file))["F_star"]
        assert len(F_star) == K
        log(f"F* of all instances read from {args.fstar_file}")
    else:
        F_star = batch_reference_optima(ws, gamma, p, seed)
        log(f"F* for all instances in {time.perf_counter() - t0:.1f} s")
        if args.fstar_file:
            json.dump(dict(instances=K, F_star=F_star), open(args.fstar_file, "w"))
    B = sca.Batch(ws, F_star)
    o = sca.make_opts(gamma=gamma, select_p=p, seed=seed, max_rounds=100000, check_every=10,
                      tol_rel_obj=args.tol)
    x = torch.zeros(int(B.xoff[-1]), dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        x.zero_()
        sca.sca_batch_solve(B.handle, o, x, B.K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        st = sca.sca_batch_solve(B.handle, o, x, B.K)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    upd_batch = sum(s["coord_updates"] for s in st)
    # algorithmic bytes of the gradient pass of one batched solve: m_k * 4 B per drawn
    # coordinate of instance k
    grad_bytes = float(sum(s["coord_updates"] * w.m * 4 for s, w in zip(st, ws)))
    log(f"batched solve: {t_batch * 1e3:.1f} ms, rounds max {max(s['rounds'] for s in st)}, "
        f"max rel err {max(s['rel_err'] for s in st):.2e}")
    if args.no_compare:
        out = {
            "metric": METRIC, "value": upd_batch / t_batch, "unit": "coord-updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"batch_{K}_lasso_m500-8000_n5m_fp32", "instances": K,
                       "A_bytes": abytes, "tol_rel_obj": args.tol},
            "grad_alg_bytes_per_solve": grad_bytes,
            "max_rel_err": max(s["rel_err"] for s in st)}
        print(json.dumps(out), flush=True)
        return
    # the same instances, one plain solve after another
    plain_t, plain_upd, plain_x = 0.0, 0, []
    probs = [sca.Problem.from_workload(w) for w in ws]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, (w, P) in enumerate(zip(ws, probs)):
        ok = sca.make_opts(gamma=gamma, tau=w.tau, select_p=p, seed=seed, instance=k,
                           max_rounds=100000, check_every=10, tol_rel_obj=args.tol,
                           F_star=F_star[k])
        xk = torch.zeros(w.n, dtype=torch.float32, device="cuda")
        sk = sca.sca_solve(P.handle, ok, xk)
        plain_upd += sk["coord_updates"]
        plain_x.append(xk)
    torch.cuda.synchronize()
    plain_t = time.perf_counter() - t0
    log(f"plain sequential solves: {plain_t * 1e3:.1f} ms")
    # adjoints at the solutions, cotangent xbar = 1
    xbar = torch.ones_like(x)
    bbar = torch.zeros(int(B.roff[-1]), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb = sca.sca_batch_adjoint(B.handle, o, x, xbar, bbar, B.K)
    torch.cuda.synchronize()
    t_badj = time.perf_counter() - t0
    t0 = time.perf_counter()
    for k, (w, P) in enumerate(zip(ws, probs)):
        ok = sca.make_opts(gamma=gamma, tau=w.tau, select_p=p, seed=seed, instance=k)
        bb = torch.empty(w.m, dtype=torch.float32, device="cuda")
        sca.sca_adjoint(P.handle, ok, plain_x[k], torch.ones_like(plain_x[k]), bb)
    torch.cuda.synchronize()
    t_padj = time.perf_counter() - t0
    log(f"adjoints: batched {t_badj * 1e3:.1f} ms, plain sequential {t_padj * 1e3:.1f} ms")
    out = {
        "metric": METRIC, "value": upd_batch / t_batch, "unit": "coord-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_batch * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch_{K}_lasso_m500-8000_n5m_fp32", "instances": K,
                   "A_bytes": abytes, "block": 64, "select_p": p, "gamma": gamma,
                   "tol_rel_obj": args.tol, "step": "one batched solve of every instance"},
        "batched": {"time_to_all_tol_s": t_batch, "coord_updates_per_s": upd_batch / t_batch,
                    "max_rel_err": max(s["rel_err"] for s in st),
                    "grad_alg_bytes_per_solve": grad_bytes},
        "plain_sequential": {"time_to_all_tol_s": plain_t,
                             "coord_updates_per_s": plain_upd / plain_t},
        "batched_speedup": plain_t / t_batch,
        "adjoint": {"batched_s": t_badj, "plain_sequential_s": t_padj,
                    "batched_over_forward": t_badj / t_batch,
                    "lambar_first": float(lb[0])},
    }
    print(json.dumps(out), flush=True)


MFMA_FP32_PEAK_TFLOPS = 157.3


def bench_multi(args):
    """A sweep of K lambda values over the 20000 x 100000 FP32 LASSO (same A and b, lam_k =
    f_k ||A^T b||_inf with f_k log-spaced over [0.005, 0.05]): one multi-right-hand-side solve
    of all K problems to relative error 1e-6 each (gradients and residual updates as MFMA
    products) against the same K problems solved one after another by the single-problem
    path."""
    K = args.rhs
    t0 = time.perf_counter()
    w = inputs.multi_rhs_problem(args.m, args.n, K, rhs="sweep", lam_range=(0.005, 0.05),
                                 nnz_frac=0.01, block=64, p=0.25, dtype=torch.float32, seed=0,
                                 device="cuda")
    torch.cuda.synchronize()
    log(f"generated {w.name} in {time.perf_counter() - t0:.1f} s: tau={w.tau:.4g}")
    okw = dict(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
    # F*_k: an FP64 multi solve of the stored data (upcast copies) to merit <= 1e-12
    t0 = time.perf_counter()
    At64, B64 = w.At.double(), w.B.double()
    M64 = sca.Multi(At64, w.m, B64, w.lams, w.c, w.beta, w.block_ptr)
    X64 = M64.zeros_x()
    st64 = sca.sca_multi_solve(M64.handle, sca.make_opts(**okw, max_rounds=200000,
                                                         check_every=50, tol_merit=1e-12),
                               X64, K, raise_on_notconv=False)
    F_star = [s["F"] for s in st64]
    log(f"F* of {K} problems in {time.perf_counter() - t0:.1f} s: max rounds "
        f"{max(s['rounds'] for s in st64)}, max merit {max(s['merit'] for s in st64):.1e}")
    M64.close()
    del M64, At64, B64, X64
    torch.cuda.empty_cache()
    M = sca.Multi(w.At, w.m, w.B, w.lams, w.c, w.beta, w.block_ptr)
    sca.sca_multi_set_fstar(M.handle, F_star)
    opts = sca.make_opts(**okw, max_rounds=100000, check_every=10, tol_rel_obj=args.tol)
    X = M.zeros_x()
    for _ in range(args.warmup):
        X.zero_()
        sca.sca_multi_solve(M.handle, opts, X, K)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        X.zero_()
        stats.append(sca.sca_multi_solve(M.handle, opts, X, K))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    upd = sum(s["coord_updates"] for st in stats for s in st)
    rounds = max(s["rounds"] for s in stats[-1])
    log(f"multi solve: {elapsed / args.steps * 1e3:.1f} ms, {rounds} rounds, max rel err "
        f"{max(s['rel_err'] for s in stats[-1]):.2e}")
    roof, prof_pass = None, None
    if not args.no_profile:
        popts = sca.make_opts(**okw, max_rounds=100000, check_every=10, tol_rel_obj=args.tol,
                              flags=sca.SCA_FLAG_PROFILE)
        sca.sca_multi_profile_get(M.handle, reset=True)
        pst = []
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(args.steps):
            X.zero_()
            pst.append(sca.sca_multi_solve(M.handle, popts, X, K))
        torch.cuda.synchronize()
        pel = time.perf_counter() - tp
        prof = sca.sca_multi_profile_get(M.handle, reset=True)
        # algorithmic flops of the gradient product: 2 m K per drawn coordinate (every drawn
        # coordinate is evaluated for all K problems, frozen ones included)
        drawn = sum(max(s["coord_updates"] for s in st) for st in pst)
        moved = sum(st[0]["moved_updates"] for st in pst)
        g, f = prof["grad"], prof["fold"]
        gflop = 2.0 * w.m * K * drawn
        ffl = 2.0 * w.m * K * moved
        achieved = gflop / (g["ms"] * 1e-3) / 1e12
        roof = dict(bound="mfma", achieved=round(achieved, 2), peak=MFMA_FP32_PEAK_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / MFMA_FP32_PEAK_TFLOPS, 4),
                    traffic=None, kernel="k_mgrad_dma<4,16>" if K > 48 else "k_mgrad<float,float,%d>" % ((K + 15) // 16),
                    avg_launch_ms=round(g["ms"] / g["launches"], 4),
                    alg_flop_per_launch=round(gflop / g["launches"]))
        prof_pass = dict(ms_per_step=pel / args.steps * 1e3,
                         per_launch_ms={k: round(v["ms"] / max(1, v["launches"]), 4)
                                        for k, v in prof.items()},
                         fold_TFLOPs=round(ffl / (f["ms"] * 1e-3) / 1e12, 2) if f["ms"] else None)
        log(f"profiled pass: {prof_pass}, roofline {roof}")
    # the same K problems, one single-problem solve after another
    plain_t, plain_upd = float("nan"), 0
    if args.no_compare:
        probs = []
    else:
        plain_t, plain_upd = 0.0, 0
        probs = [sca.Problem.dense(w.At, w.m, w.B[k, : w.m], float(w.lams[k]), w.c, w.beta,
                                   w.block_ptr) for k in range(K)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, P in enumerate(probs):
            ok = sca.make_opts(**okw, max_rounds=100000, check_every=10, tol_rel_obj=args.tol,
                               F_star=F_star[k])
            xk = torch.zeros(w.n, dtype=torch.float32, device="cuda")
            plain_upd += sca.sca_solve(P.handle, ok, xk)["coord_updates"]
        torch.cuda.synchronize()
        plain_t = time.perf_counter() - t0
        log(f"single-problem solves one after another: {plain_t * 1e3:.1f} ms")
    cpu = None
    if not args.no_cpu_baseline:
        w1 = inputs.DenseWorkload(w.name, w.At, w.m, w.n, w.lda, w.B[K // 2, : w.m],
                                  w.base.x_true, float(w.lams[K // 2]), w.c, w.beta, w.tau,
                                  w.block_ptr, w.p, w.gamma, w.seed)
        cpu = cpu_baseline(w1, okw, args.cpu_rounds or 12)
        cpu["sample"] = cpu["sample"] + f" (problem {K // 2} of the sweep, lam={w.lams[K // 2]:.4g})"
        log(f"cpu baseline: {cpu}")
    out = {
        "metric": METRIC, "value": upd / elapsed, "unit": "coord-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"multi_rhs_lasso_{w.m}x{w.n}_K{K}_lambda_sweep_fp32",
                   "m": w.m, "n": w.n, "K": K, "lam_frac_range": [0.005, 0.05], "block": 64,
                   "select_p": w.p, "gamma": w.gamma, "tol_rel_obj": args.tol,
                   "step": "one multi solve of all K problems from X=0"},
        "max_rel_err": max(s["rel_err"] for s in stats[-1]),
        "rounds_to_all": rounds,
        "plain_sequential": None if args.no_compare else
        {"time_to_all_tol_s": plain_t, "coord_updates_per_s": plain_upd / plain_t},
        "multi_speedup": None if args.no_compare else plain_t / (elapsed / args.steps),
        "roofline": roof, "profiled_pass": prof_pass, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_delay(args):
    """Bounded-delay rounds on the 20000 x 100000 FP32 LASSO: rounds and time to relative
    error 1e-6 for several (groups q, staleness s); every update misses at most
    (s + 1) ceil(|S|/q) - 1 others (|S| ~ 25000 drawn coordinates per round).  Then lock-free
    rounds on W racing workgroups (each update misses at most W - 1 others)."""
    w = inputs.lasso_dense_fp32(m=args.m, n=args.n, seed=0, device="cuda")
    okw = dict(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
    F_star, _ = reference_optimum(w, okw)
    P = sca.Problem.from_workload(w)
    S_mean = w.p * w.n
    rows = []
    value = None
    for q, st_ in [(1, 0), (2, 0), (4, 0), (4, 1), (16, 0), (16, 3), (64, 0)]:
        o = sca.make_opts(**okw, max_rounds=100000, check_every=10, tol_rel_obj=args.tol,
                          F_star=F_star, delay_chunks=q, delay_stale=st_)
        x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
        sca.sca_solve(P.handle, o, x)  # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for _ in range(args.steps):
            x.zero_()
            stats.append(sca.sca_solve(P.handle, o, x))
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / args.steps
        upd = stats[-1]["coord_updates"]
        delta = (st_ + 1) * math.ceil(S_mean / q) - 1 if q > 1 else int(S_mean) - 1
        rows.append(dict(groups=q, stale=st_, delay_bound=delta, rounds=stats[-1]["rounds"],
                         time_to_tol_s=el, coord_updates_per_s=upd / el,
                         rel_err=stats[-1]["rel_err"]))
        log(f"q={q} s={st_}: delay bound {delta}, {stats[-1]['rounds']} rounds, {el * 1e3:.1f} ms")
        if q == 1:
            value = upd / el
            base_ms = el * 1e3
    # lock-free rounds: W workgroups race on the round's drawn coordinates (nondeterministic);
    # each update misses at most W - 1 others in flight.  One solve each (atomic folds: slow)
    for W in (256, 1024, 4096):
        o = sca.make_opts(**okw, max_rounds=5000, check_every=10, tol_rel_obj=args.tol,
                          F_star=F_star, async_workgroups=W)
        x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sca.sca_solve(P.handle, o, x, raise_on_notconv=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rows.append(dict(lock_free_workgroups=W, delay_bound=W - 1, rounds=st["rounds"],
                         time_to_tol_s=el, coord_updates_per_s=st["coord_updates"] / el,
                         rel_err=st["rel_err"], status=st["status"]))
        log(f"lock-free W={W}: delay bound {W - 1}, {st['rounds']} rounds, {el * 1e3:.1f} ms, "
            f"rel err {st['rel_err']:.2e}")
    out = {
        "metric": METRIC, "value": value, "unit": "coord-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": base_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"delay_study_lasso_dense_{w.m}x{w.n}_fp32", "m": w.m, "n": w.n,
                   "block": 64, "select_p": w.p, "gamma": w.gamma, "tol_rel_obj": args.tol,
                   "step": "one solve from x=0 to tolerance per (groups, staleness)"},
        "delay_study": rows, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


PMC_SUMMARY = {
    "lasso": os.path.join(ROOT, "profiles", "pmc_k_grad_br_fold_lasso_20000x100000_fp32.txt"),
    "sparse": os.path.join(ROOT, "profiles", "pmc_k_dot_split_sparse_lasso_100000x1000000_fp32.txt"),
}
# sources whose kernels the counter runs measured (their digest is the summary's fingerprint)
PMC_SOURCES = {"lasso": ("sca_kernels.h", "sca_device.h"),
               "sparse": ("sca_kernels.h", "sca_device.h", "sca_csc.hip")}
SPARSE_STEP_KERNELS = ("k_dot_split<float,8,true>", "k_br_split<float,8>")
CALIB_BYTES = 1 << 30


def kernel_fingerprint(launch, kind="lasso"):
    """Digest of the round kernels' source and the launch shape the counters were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in PMC_SOURCES[kind]:
        h.update(open(os.path.join(ROOT, "paper_1701_04900_amd", "csrc", f), "rb").read())
    h.update(json.dumps(launch, sort_keys=True).encode())
    return h.hexdigest()[:16]


def pmc_probe(args):
    """What the counter runs profile: three copies of exactly 1 GiB (the calibration), then
    30 rounds from x = 0 of the 20000 x 100000 FP32 LASSO (or, with --workload sparse, of
    the 1e5 x 1e6 sparse LASSO)."""
    sparse = args.workload == "sparse"
    w = (inputs.sparse_lasso_fp32(device="cuda") if sparse else
         inputs.lasso_dense_fp32(m=args.m, n=args.n, seed=0, device="cuda"))
    src = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        sca.sca_stream_copy(dst, src, CALIB_BYTES)
    torch.cuda.synchronize()
    del src, dst
    P = sca.Problem.from_workload(w)
    o = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed, max_rounds=30,
                      check_every=10)
    x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
    st = sca.sca_solve(P.handle, o, x, raise_on_notconv=False)
    out = dict(workload="sparse" if sparse else "lasso", rounds=st["rounds"],
               coord_updates=st["coord_updates"], launch=sca.sca_problem_get_launch(P.handle),
               m=w.m)
    if sparse:
        out.update(n=w.n, nnz=w.nnz, per_col=w.nnz // w.n)
    else:
        out.update(groups=fused_groups())
    print(json.dumps(out), flush=True)


def pmc_summarize(fetch_dir, write_dir, probe_json):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the calibration copy and of the measured
    step's kernels -> bytes per launch, scaled so the copy reads and writes exactly 1 GiB."""
    import csv
    import glob

    def load(d, counter):
        out = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") != counter:
                    continue
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out
    probe = json.loads(open(probe_json).read().strip().splitlines()[-1])
    kind = probe.get("workload", "lasso")
    if kind == "sparse":
        wants = SPARSE_STEP_KERNELS
        title = ("# HBM traffic of the sparse gradient step (k_dot_split + k_br_split), sparse "
                 "LASSO 100000x1000000 FP32, 1e8 nonzeros (rocprofv3 counters)")
        flag = " --workload sparse"
    else:
        wants = (grad_kernel_name(probe["launch"], False, probe["m"]),)
        title = ("# HBM traffic of the dominant round kernel, LASSO 20000x100000 FP32 (rocprofv3 "
                 "counters)")
        flag = ""
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        vals = load(d, counter)
        copy = [v for k, v in vals.items() if "k_stream_copy" in k][0]
        per_launch, launches = 0.0, None
        for want in wants:
            grad = [v for k, v in vals.items() if want in k.replace(" ", "")][0]
            per_launch += sum(grad) / len(grad)
            launches = len(grad) if launches is None else min(launches, len(grad))
        cal = CALIB_BYTES / (sorted(copy)[len(copy) // 2] * 1024.0)
        res[counter] = dict(copy_kib=sorted(copy)[len(copy) // 2], scale=cal,
                            grad_kib_mean=per_launch, launches=launches)
    launches = res["FETCH_SIZE"]["launches"]
    fetch_b = res["FETCH_SIZE"]["grad_kib_mean"] * 1024 * res["FETCH_SIZE"]["scale"]
    write_b = res["WRITE_SIZE"]["grad_kib_mean"] * 1024 * res["WRITE_SIZE"]["scale"]
    drawn = probe["coord_updates"] / probe["rounds"]
    impl_b = 0.0
    if kind == "sparse":
        alg_b = drawn * probe["per_col"] * (4 + 4)
    else:
        alg_b = round_alg_bytes(probe["launch"], drawn, probe["m"], 4, probe.get("groups", 0))
        if probe["launch"]["grad_kind"] == 4:
            impl_b = probe.get("groups", 0) * probe["m"] * 4
    fp = kernel_fingerprint(probe["launch"], kind)
    lines = [
        title,
        "",
        "Commands (repository root, one MI355X; each counter in a run of its own):",
        "  rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/pmc_fetch -- "
        f"python3 bench.py --pmc-probe{flag} > <out>/pmc_probe.json",
        "  rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/pmc_write -- "
        f"python3 bench.py --pmc-probe{flag}",
        "  python bench.py --pmc-summarize <out>/pmc_fetch <out>/pmc_write "
        "<out>/pmc_probe.json",
        "",
        "Calibration: k_stream_copy moves exactly 1 GiB each way; the counters read "
        f"{res['FETCH_SIZE']['copy_kib']:.0f} KiB fetched and {res['WRITE_SIZE']['copy_kib']:.0f} KiB "
        f"written per copy, so the scale factors are {res['FETCH_SIZE']['scale']:.4f} (fetch) and "
        f"{res['WRITE_SIZE']['scale']:.4f} (write).",
        "",
        f"launches: {launches}",
        f"launch: {json.dumps(probe['launch'], sort_keys=True)}",
        f"fingerprint: {fp}",
        f"fetch_bytes_per_launch: {fetch_b:.0f}",
        f"write_bytes_per_launch: {write_b:.0f}",
        f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}",
        f"algorithmic_bytes_per_launch: {alg_b:.0f}",
        f"traffic_over_algorithmic: {(fetch_b + write_b) / alg_b:.4f}",
    ]
    if impl_b:
        lines += [
            f"fold_partial_bytes_per_launch: {impl_b:.0f}",
            f"traffic_over_algorithmic_and_partials: {(fetch_b + write_b) / (alg_b + impl_b):.4f}",
            "(algorithmic bytes: the drawn columns, m x 4 B each, read once -- the method's "
            "reads; the fused round also writes one m-vector of fold partials per workgroup, "
            "counted on the line above)"]
    open(PMC_SUMMARY[kind], "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def pmc_traffic(launch, kind="lasso"):
    """Traffic per launch from the committed counter summary and the algorithmic bytes of
    the probe rounds it was read over (dict), or None when it is absent or was taken on
    other kernel code or another launch shape."""
    if not os.path.exists(PMC_SUMMARY[kind]):
        return None
    kv = {}
    for line in open(PMC_SUMMARY[kind]):
        if ": " in line and not line.startswith(" "):
            k, v = line.split(": ", 1)
            kv[k.strip()] = v.strip()
    if kv.get("fingerprint") != kernel_fingerprint(launch, kind):
        return None
    return dict(traffic=float(kv["traffic_bytes_per_launch"]),
                alg=float(kv["algorithmic_bytes_per_launch"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=20000)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--cpu-rounds", type=int, default=None,
                    help="oracle rounds for the CPU baseline (default: 12 dense LASSO, "
                         "100 box-nonconvex, 100 sparse)")
    ap.add_argument("--rounds", type=int, default=3000,
                    help="rounds per step of the box-nonconvex workload")
    ap.add_argument("--seeds", type=int, default=5,
                    help="data seeds 0..S-1 of the headline workload, each with K timed solves; "
                         "S > 1 reports the medians over seeds (the paper averages 5 "
                         "realisations)")
    ap.add_argument("--headline-only", action="store_true",
                    help="default workload: skip the sparse, box-nonconvex and 200x1000 runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--workload", choices=["lasso", "nonconvex", "sparse", "batch", "multi",
                                          "delay"],
                    default="lasso")
    ap.add_argument("--rhs", type=int, default=64, help="right-hand sides of --workload multi")
    ap.add_argument("--no-compare", action="store_true",
                    help="--workload multi / batch: skip the single-problem solves they are "
                         "compared with")
    ap.add_argument("--instances", type=int, default=256)
    ap.add_argument("--fstar-file", default=None,
                    help="--workload batch: read F*_k from this JSON file when it exists, "
                         "else compute them and write it")
    ap.add_argument("--pmc-probe", action="store_true")
    ap.add_argument("--pmc-summarize", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "PROBE_JSON"))
    args = ap.parse_args()
    if args.pmc_summarize:
        pmc_summarize(*args.pmc_summarize)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU path (column-block sharding with "
              "an all-reduce of the residual update per round) is not built", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    sca.lib()
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "multi":
        bench_multi(args)
        return
    if args.workload == "delay":
        bench_delay(args)
        return
    if args.pmc_probe:
        pmc_probe(args)
        return
    if args.workload == "lasso":
        bench_default(args)
        return
    cr = None if args.no_cpu_baseline else (args.cpu_rounds or 100)
    out = run_single(args.workload, args, args.steps, args.warmup, seeds=1,
                     profile=not args.no_profile, cpu_rounds=cr)
    print(json.dumps(out), flush=True)


def make_workload(kind, args, seed=0):
    if kind == "lasso":
        return inputs.lasso_dense_fp32(m=args.m, n=args.n, seed=seed, device="cuda")
    if kind == "nonconvex":
        return inputs.nonconvex_box_fp32(seed=seed, device="cuda")
    return inputs.sparse_lasso_fp32(seed=seed, device="cuda")


def extra_seeds(kind, args, opts_base, seeds, steps, warmup):
    """Data seeds 1 .. S-1 of the same workload (seed 0 is timed by the caller): per seed a
    fresh workload, its own F* (an FP64 solve that must reach merit 1e-13), warm-up and K
    timed solves.  Returns per-seed results."""
    out = []
    for seed in range(1, seeds):
        w = make_workload(kind, args, seed)
        okw = dict(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
        stop_kw, max_rounds, notconv_ok = opts_base
        if "F_star" in stop_kw:
            sparse = kind == "sparse"
            stop_kw = dict(stop_kw, F_star=(sparse_reference_optimum if sparse
                                            else reference_optimum)(w, okw)[0])
        P = sca.Problem.from_workload(w)
        opts = sca.make_opts(**okw, max_rounds=max_rounds, check_every=10, **stop_kw)
        x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
        for _ in range(warmup):
            x.zero_()
            sca.sca_solve(P.handle, opts, x, raise_on_notconv=not notconv_ok)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for _ in range(steps):
            x.zero_()
            stats.append(sca.sca_solve(P.handle, opts, x, raise_on_notconv=not notconv_ok))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res = dict(seed=seed, ms_per_step=el / steps * 1e3,
                   value=sum(s["coord_updates"] for s in stats) / el,
                   rounds_per_solve=sum(s["rounds"] for s in stats) / steps,
                   rel_err_final=stats[-1]["rel_err"], merit_final=stats[-1]["merit"])
        log(f"seed {seed}: {res}")
        out.append(res)
        P.close()
        del w, x
        torch.cuda.empty_cache()
    return out


def sparse_reference_optimum(w, opts_kw, want_x=False):
    """F* by an FP64 solve of the stored FP32 CSR data (upcast copy) to merit <= 1e-12."""
    P = sca.Problem.csr(w.m, w.n, w.rowptr, w.colidx, w.vals.double(), w.b.double(), w.lam,
                        w.c, w.beta, w.block_ptr)
    o = sca.make_opts(**opts_kw, max_rounds=200000, check_every=50, tol_merit=F_STAR_MERIT)
    x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    st = sca.sca_solve(P.handle, o, x, raise_on_notconv=False)
    P.close()
    torch.cuda.empty_cache()
    _checked_fstar_solve(st, w.name)
    if want_x:
        return st["F"], st, x.cpu().numpy()
    return st["F"], st


def fused_groups():
    """Workgroups (= fold partials) of the fused dense round: one per CU, at most 256."""
    return min(torch.cuda.get_device_properties(0).multi_processor_count, 256)


def fused_q(m, esize):
    """16-byte row groups per thread when a 1024-thread workgroup holds an m-row column."""
    groups = (m * esize + 15) // 16
    return (groups + 1023) // 1024


def round_alg_bytes(L, drawn, m, esize, groups):
    """Algorithmic bytes of one launch of the gradient kernel: the drawn columns, once.
    (The fused kind also writes one m-vector of fold partials per workgroup: traffic of the
    implementation, not of the method, so not counted here.)"""
    return drawn * m * esize


def grad_kernel_name(L, sparse, m=0):
    if sparse:
        # panel split (r in at most 16 panels of 140 KiB): partial dot products (with the
        # block draw inside: at most 32768 blocks, as in the sparse workloads here), then the
        # sum of the partials with the best response (one timed step, two kernels)
        if (m + 35839) // 35840 <= 16:
            return "k_dot_split<float,8,true> + k_br_split<float,8>"
        return "k_grad_br_cscp<float,8>"
    if L["grad_kind"] == 4:
        q = fused_q(m, 4)
        if q <= 5:  # every row group in registers
            return f"k_grad_br_fold<float,{q},{L['grad_cols']},0>"
        return f"k_grad_br_fold<float,4,1,{q - 4}>"  # 4 in registers, the rest in LDS
    return {0: f"k_grad_br<float,{L['grad_unroll']}>",
            1: f"k_grad_br_wg<float,{L['grad_cols']},{L['grad_unroll']},true>",
            2: f"k_grad_br_wg<float,{L['grad_cols']},{L['grad_unroll']},false>",
            3: f"k_grad_br_wwalk<float,{L['grad_cols']},{L['grad_unroll']}>"}[L["grad_kind"]]


def read_stream_peak(buf):
    """Best of a plain 16-byte streaming read over `buf` (the matrix's own storage)."""
    sink = torch.zeros(1 << 14, dtype=torch.float32, device="cuda")
    nbytes = buf.numel() * buf.element_size() // 16 * 16
    best = 0.0
    for grid in (1024, 2048):
        sca.sca_stream_read(buf, nbytes, sink, grid)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            sca.sca_stream_read(buf, nbytes, sink, grid)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 3 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    return best


def cpu_info():
    """Host cores this process may use and the CPU model (for the CPU baseline rows)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return len(os.sched_getaffinity(0)), model


def nonconvex_milestones(w, P, opts_kw, rounds, every=50):
    """Rounds from x = 0 at which the merit ||xhat(x) - x||_inf (Section 4.3) first drops to
    1e-1, 1e-2, ... (checked every `every` rounds with a fresh FP64 residual), and the merit
    curve itself; None for a level not reached within `rounds`."""
    o = sca.make_opts(**opts_kw)
    x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
    r = torch.empty(w.m, dtype=w.dtype, device="cuda")
    sca.sca_residual(P.handle, x, r)
    levels = [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6]
    hit = {lv: None for lv in levels}
    curve = []
    k = 0
    while k < rounds:
        nr = min(every, rounds - k)
        sca.sca_step(P.handle, o, k, nr, x, r)
        k += nr
        mer = sca.sca_objective(P.handle, o, x)["merit"]
        curve.append((k, mer))
        for lv in levels:
            if hit[lv] is None and mer <= lv:
                hit[lv] = k
    return ({f"{lv:g}": hit[lv] for lv in levels},
            [(k, float(f"{m:.4g}")) for k, m in curve[:: max(1, len(curve) // 20)]] + [curve[-1]])


def run_single(kind, args, steps, warmup, seeds=1, profile=True, cpu_rounds=None,
               certify=True):
    """One problem, K timed solves from x = 0 to tolerance (LASSO: relative objective error
    against F*; box-nonconvex: a fixed budget of rounds, with the merit reached and the
    rounds to each merit level reported).  Returns the JSON record."""
    sparse = kind == "sparse"
    t0 = time.perf_counter()
    w = make_workload(kind, args)
    torch.cuda.synchronize()
    log(f"generated {w.name} in {time.perf_counter() - t0:.1f} s: lam={w.lam:.4g} tau={w.tau:.4g}")
    opts_kw = dict(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
    esize = w.dtype.itemsize if hasattr(w.dtype, "itemsize") else torch.finfo(w.dtype).bits // 8
    if sparse:
        # every column holds the same number of nonzeros: value + int32 row index each
        per_col = w.nnz // w.n
        assert per_col * w.n == w.nnz
        bytes_per_update = (esize + 4) * per_col
    else:
        bytes_per_update = w.m * esize

    F_star, fcheck = None, None
    max_rounds = 100000
    notconv_ok = False
    if kind == "nonconvex":
        # the merit of this workload decreases slowly (about 3e-2 after 1e4 rounds, in FP64
        # as well), so a step is a fixed budget of rounds and the merit reached is reported
        stop_kw = {}
        max_rounds = args.rounds
        notconv_ok = True
    else:
        t0 = time.perf_counter()
        F_star, st64, x64 = (sparse_reference_optimum if sparse else reference_optimum)(
            w, opts_kw, want_x=True)
        log(f"F* = {F_star:.15g} (FP64 solve: {st64['rounds']} rounds, merit "
            f"{st64['merit']:.2e}, {time.perf_counter() - t0:.1f} s)")
        if certify:
            fcheck = certify_fstar(w, F_star, x64)
            fcheck["reference_solve"] = dict(rounds=st64["rounds"], merit=st64["merit"])
        del x64
        stop_kw = dict(tol_rel_obj=args.tol, F_star=F_star)

    P = sca.Problem.from_workload(w)
    opts = sca.make_opts(**opts_kw, max_rounds=max_rounds, check_every=10, **stop_kw)
    x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
    for i in range(warmup):
        x.zero_()
        st = sca.sca_solve(P.handle, opts, x, raise_on_notconv=not notconv_ok)
        log(f"warmup solve {i}: {st['rounds']} rounds, rel err {st['rel_err']:.2e}, "
            f"merit {st['merit']:.2e}")
    # timed region: K solves, each check cycle one graph launch
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for i in range(steps):
        x.zero_()
        stats.append(sca.sca_solve(P.handle, opts, x, raise_on_notconv=not notconv_ok))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    updates = sum(s["coord_updates"] for s in stats)
    rounds = sum(s["rounds"] for s in stats)
    value = updates / elapsed
    for i, s in enumerate(stats):
        log(f"solve {i}: {s['rounds']} rounds, {s['coord_updates']} updates, "
            f"{s['seconds'] * 1e3:.1f} ms, rel err {s['rel_err']:.3e}, merit {s['merit']:.2e}")
    per_seed = None
    if seeds > 1:
        # the timing protocol over data realisations: seeds 0 .. S-1, medians reported
        per_seed = [dict(seed=0, ms_per_step=elapsed / steps * 1e3, value=value,
                         rounds_per_solve=rounds / steps,
                         rel_err_final=stats[-1]["rel_err"], merit_final=stats[-1]["merit"])]
        per_seed += extra_seeds(kind, args, (stop_kw, max_rounds, notconv_ok), seeds, steps,
                                warmup)

    milestones = None
    if kind == "nonconvex":
        t0 = time.perf_counter()
        hit, curve = nonconvex_milestones(w, P, opts_kw, max_rounds)
        milestones = dict(rounds_to_merit=hit, merit_curve=curve,
                          note="merit from x = 0, checked every 50 rounds (fresh FP64 residual)")
        log(f"merit milestones in {time.perf_counter() - t0:.1f} s: {hit}")

    roof, prof_pass = None, None
    if profile:
        # the same K solves again with HIP events around every kernel launch (eager launches
        # on the caller's stream: events cannot time kernels inside a replayed graph)
        popts = sca.make_opts(**opts_kw, max_rounds=max_rounds, check_every=10, **stop_kw,
                              flags=sca.SCA_FLAG_PROFILE)
        sca.sca_profile_get(P.handle, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pst = []
        for i in range(steps):
            x.zero_()
            pst.append(sca.sca_solve(P.handle, popts, x, raise_on_notconv=not notconv_ok))
        torch.cuda.synchronize()
        pel = time.perf_counter() - t0
        prof = sca.sca_profile_get(P.handle, reset=True)
        pupd = sum(s["coord_updates"] for s in pst)
        pmoved = sum(s["moved_updates"] for s in pst)
        L = sca.sca_problem_get_launch(P.handle)
        g, f = prof["grad"], prof["fold"]
        # the method's bytes: every drawn column read once by the gradient pass
        grad_b = float(pupd) * bytes_per_update
        fold_b = float(pmoved) * bytes_per_update
        impl_b = 0.0
        if not sparse and L["grad_kind"] == 4:
            # fused round: it also writes one m-vector of fold partials per workgroup
            # (implementation traffic, not counted as the method's bytes), which the partial
            # reduction then reads with r in place of the fold
            G = fused_groups()
            impl_b = float(g["launches"]) * G * w.m * esize
            fold_b = float(f["launches"]) * (G + 2) * w.m * esize
        cands = [("grad", g, grad_b, grad_kernel_name(L, sparse, w.m))]
        if sparse:
            cands.append(("fold", f, fold_b,
                          "k_bin_scan<4> + k_bin_scatter<float,8> + k_bin_acc<float,float,float>"))
        step, kp, kb, kname = max(cands, key=lambda c: c[1]["ms"])
        achieved = kb / (kp["ms"] * 1e-3) / 1e9
        pmc = pmc_traffic(L, kind) if kind in PMC_SUMMARY and step == "grad" else None
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=None if pmc is None else round(pmc["traffic"]),
                    kernel=kname, step=step, launch=L,
                    avg_launch_ms=round(kp["ms"] / kp["launches"], 4),
                    alg_bytes_per_launch=round(kb / kp["launches"]),
                    alg_bytes="drawn columns x bytes per column (the method's reads; "
                              "fold partials excluded)")
        if step == "grad" and impl_b:
            roof["impl_bytes_per_launch"] = round(impl_b / kp["launches"])
            roof["frac_with_impl_bytes"] = round((kb + impl_b) / (kp["ms"] * 1e-3) / 1e9
                                                 / HBM_PEAK_GBS, 4)
        if pmc is not None:
            # the counters were read over their own probe rounds: paired with the probe's
            # algorithmic bytes
            roof["traffic_alg_bytes_per_launch"] = round(pmc["alg"])
            roof["traffic_over_alg"] = round(pmc["traffic"] / pmc["alg"], 4)
        best = read_stream_peak(w.vals if sparse else w.At)
        roof["read_stream_peak"] = round(best, 1)
        roof["frac_of_read_stream_peak"] = round(achieved / best, 4)
        prof_pass = dict(ms_per_step=pel / steps * 1e3,
                         per_launch_ms={k: round(v["ms"] / max(1, v["launches"]), 4)
                                        for k, v in prof.items()},
                         grad_GBps=round(grad_b / (g["ms"] * 1e-3) / 1e9, 1) if g["ms"] else None,
                         fold_GBps=round(fold_b / (f["ms"] * 1e-3) / 1e9, 1) if f["ms"] else None,
                         moved_per_round=pmoved / max(1, sum(s["rounds"] for s in pst)),
                         bytes_per_update=bytes_per_update)
        log(f"profiled pass: {prof_pass}")

    cpu = None
    if cpu_rounds:
        t0 = time.perf_counter()
        cpu = cpu_baseline(w, opts_kw, cpu_rounds)
        log(f"cpu baseline in {time.perf_counter() - t0:.1f} s: {cpu}")

    if kind == "lasso":
        wname = f"lasso_dense_{w.m}x{w.n}_fp32"
        block = 64
    elif kind == "nonconvex":
        wname = f"ncvx_box_{w.m}x{w.n}_fp32"
        block = 32
    else:
        wname = f"sparse_lasso_{w.m}x{w.n}_nnz{w.nnz}_fp32"
        block = 256
    cfg = {"workload": wname, "m": w.m, "n": w.n, "block": block, "select_p": w.p,
           "gamma": w.gamma, "tau": round(w.tau, 6), "step": "one solve from x=0 to tolerance"}
    if kind == "nonconvex":
        cfg.update(c=w.c, beta=w.beta, rounds=args.rounds)
        cfg["step"] = f"{args.rounds} rounds from x=0"
    else:
        cfg["tol_rel_obj"] = args.tol
    ms_per_step = elapsed / steps * 1e3
    if per_seed:
        value = float(np.median([d["value"] for d in per_seed]))
        ms_per_step = float(np.median([d["ms_per_step"] for d in per_seed]))
        cfg["seeds"] = seeds
        cfg["statistic"] = "median over data seeds of K timed solves each"
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "coord-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": cfg,
        "time_to_tol_s": ms_per_step / 1e3,
        "rounds_per_solve": rounds / steps,
        "rel_err_final": stats[-1]["rel_err"],
        "merit_final": stats[-1]["merit"],
        "F_star": F_star,
        "F_star_check": fcheck,
        "roofline": roof,
        "profiled_pass": prof_pass,
        "cpu_baseline": cpu,
    }
    if cpu:
        # the oracle draws the same blocks and follows the same trajectory (in FP64), so it
        # needs about as many rounds: its time for them, from its measured time per round
        cpu["rounds_extrapolated_to"] = rounds / steps
        cpu["time_extrapolated_s"] = cpu["seconds_per_round"] * rounds / steps
        cpu["extrapolation"] = ("seconds per round of the sample x the GPU's rounds per step "
                                "(not run: the oracle takes that long)")
    if milestones:
        out["merit_milestones"] = milestones
    if per_seed:
        out["per_seed"] = per_seed
    P.close()
    del w, x
    torch.cuda.empty_cache()
    return out


def bench_c1(args, steps):
    """LASSO 200 x 1000 FP64, scalar blocks, every block each round (gamma 0.9): microseconds
    per round and coordinate updates per second over fixed budgets of rounds, and the time to
    relative error 1e-6, with the oracle timed beside it on the host (same rounds, same
    stopping rule).  This size fits in the caches, so the rounds are latency bound."""
    w = inputs.lasso_small_fp64(seed=0, device="cuda")
    opts_kw = dict(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=w.seed)
    P = sca.Problem.from_workload(w)
    o = sca.make_opts(**opts_kw, max_rounds=200000, check_every=50, tol_merit=F_STAR_MERIT)
    x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    st64 = sca.sca_solve(P.handle, o, x, raise_on_notconv=False)
    _checked_fstar_solve(st64, w.name)
    F_star = st64["F"]
    fcheck = certify_fstar(w, F_star, x.cpu().numpy())
    # fixed budget of rounds (each check of 50 rounds one graph launch), no stopping test
    budget = 2000
    ob = sca.make_opts(**opts_kw, max_rounds=budget, check_every=50)
    sca.sca_solve(P.handle, ob, x.zero_())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sca.sca_solve(P.handle, ob, x.zero_())
    torch.cuda.synchronize()
    t_budget = (time.perf_counter() - t0) / steps
    # time to tolerance
    ot = sca.make_opts(**opts_kw, max_rounds=100000, check_every=10, tol_rel_obj=args.tol,
                       F_star=F_star)
    sca.sca_solve(P.handle, ot, x.zero_())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = []
    for _ in range(steps):
        sts.append(sca.sca_solve(P.handle, ot, x.zero_()))
    torch.cuda.synchronize()
    t_tol = (time.perf_counter() - t0) / steps
    gpu = dict(us_per_round=t_budget / budget * 1e6,
               coord_updates_per_s=budget * w.n / t_budget,
               time_to_tol_s=t_tol, rounds_to_tol=sts[-1]["rounds"],
               rel_err_final=sts[-1]["rel_err"])
    log(f"C1 GPU: {gpu}")
    P.close()
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import sca_oracle as O
        cores, model = cpu_info()
        prob = O.Problem(A=w.A_numpy(), b=w.b.double().cpu().numpy(), lam=w.lam,
                         block_ptr=w.block_ptr)
        cfg = O.RunConfig(tau=w.tau, gamma=w.gamma, p=w.p, seed=w.seed)
        prob.colnorm2()
        rounds = 200
        t0 = time.perf_counter()
        O.run_rounds(prob, cfg, np.zeros(w.n), O.residual(prob, np.zeros(w.n)), 0, rounds)
        t_or = time.perf_counter() - t0
        t0 = time.perf_counter()
        sol = O.solve(prob, cfg, check_every=10, F_star=F_star, tol_rel_obj=args.tol)
        t_os = time.perf_counter() - t0
        cpu = dict(value=rounds * w.n / t_or, unit="coord-updates/s", cores=cores,
                   cpu_model=model, kind="oracle", us_per_round=t_or / rounds * 1e6,
                   time_to_tol_s=t_os, rounds_to_tol=sol["rounds"],
                   sample=f"{rounds} rounds of the same 200x1000 FP64 LASSO from x=0 (FP64 "
                          f"numpy), then one oracle solve to rel. error {args.tol:g}")
        log(f"C1 oracle: {cpu}")
    return dict(config={"workload": "lasso_dense_200x1000_fp64", "m": w.m, "n": w.n,
                        "block": 1, "select_p": 1.0, "gamma": w.gamma, "tau": round(w.tau, 6),
                        "tol_rel_obj": args.tol, "steps": steps, "budget_rounds": budget},
                dtype="f64", gpu=gpu, F_star=F_star, F_star_check=fcheck, cpu_baseline=cpu,
                roofline=None,
                roofline_note="1.6 MB of A stays in the caches: latency bound, no HBM roofline")


def bench_default(args):
    """The headline (the 20000 x 100000 FP32 LASSO to 1e-6, medians over data seeds), then
    the other single-GPU workloads in smaller runs, each under a key of its own: the
    200 x 1000 FP64 LASSO (latency bound), the 1e5 x 1e6 sparse LASSO and the
    10000 x 50000 box-nonconvex budget."""
    t_all = time.perf_counter()
    out = run_single("lasso", args, args.steps, args.warmup, seeds=args.seeds,
                     profile=not args.no_profile,
                     cpu_rounds=None if args.no_cpu_baseline else (args.cpu_rounds or 16))
    if out["cpu_baseline"]:
        out["cpu_baseline"]["cpu_model"] = cpu_info()[1]
    if not args.headline_only:
        k_steps, k_warm = min(args.steps, 5), min(args.warmup, 1)
        extra_cpu = None if args.no_cpu_baseline else 40
        for key, kind in (("sparse_1e5x1e6", "sparse"), ("nonconvex_10000x50000", "nonconvex")):
            t0 = time.perf_counter()
            rec = run_single(kind, args, k_steps, k_warm, profile=not args.no_profile,
                             cpu_rounds=extra_cpu)
            if rec["cpu_baseline"]:
                rec["cpu_baseline"]["cpu_model"] = cpu_info()[1]
            for k in ("metric", "unit", "n_gpus", "higher_is_better", "scaling", "vs_baseline",
                      "data"):
                rec.pop(k, None)
            out[key] = rec
            log(f"{key} done in {time.perf_counter() - t0:.1f} s")
        t0 = time.perf_counter()
        out["lasso_200x1000_fp64"] = bench_c1(args, k_steps)
        log(f"lasso_200x1000_fp64 done in {time.perf_counter() - t0:.1f} s")
    log(f"bench finished in {time.perf_counter() - t_all:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
