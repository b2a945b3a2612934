"""Autotuner of the round's launch shape, for single dense problems and for batches.

Single problems: for each (dtype, m range) bucket it draws a representative problem (N(0,1),
unit columns, blocks of 64, a quarter of the blocks per round), runs a few rounds with every
candidate shape through sca_problem_set_launch, times the gradient, compaction and fold
kernels of the round with the library's HIP events and keeps the shape with the shortest
sum (the fused kind does the fold's work inside its gradient kernel).

Batches: for each dtype it draws a representative batch (instances of uneven m up to the
fused kind's limit, n = 5m, blocks of 64, a quarter of the blocks per round) and times whole
batched rounds (sca_batch_step, HIP events on the stream) for the two-pass kind and the
fused kind on 1 to 4 workgroups per compute unit, in two phases -- the first rounds from
x = 0 and rounds after a few hundred -- and keeps the shape with the shortest sum.

The table is written as JSON next to this file (tuning/gfx950.json) and installed by the
binding when the library is loaded.

    python -m paper_1701_04900_amd.autotune [--out PATH] [--rounds R] [--only single|batch]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import torch

from . import inputs, sca

# (kind, cols, unroll, workgroups per CU)
CANDIDATES = [(1, 8, 2, 2), (1, 8, 2, 1), (1, 8, 1, 2), (1, 8, 1, 4), (1, 16, 1, 2),
              (1, 16, 1, 1), (1, 4, 2, 2), (1, 4, 4, 2), (1, 4, 1, 4), (0, 0, 8, 1),
              (0, 0, 8, 2), (0, 0, 16, 2), (3, 4, 2, 2), (3, 4, 4, 2), (3, 8, 1, 2),
              (3, 4, 2, 4), (3, 8, 1, 4), (4, 1, 1, 1), (4, 2, 1, 1), (4, 4, 1, 1),
              (4, 8, 1, 1)]
# (dtype, m_lo, m_hi, representative m, n)
BUCKETS = [("f32", 1, 1535, 768, 200000), ("f32", 1536, 6143, 3000, 120000),
           ("f32", 6144, 14335, 10000, 100000), ("f32", 14336, 20480, 20000, 100000),
           ("f32", 20481, 28671, 24000, 80000), ("f32", 28672, 1 << 30, 40000, 60000),
           ("f64", 1, 1535, 768, 100000), ("f64", 1536, 6143, 3000, 60000),
           ("f64", 6144, 14335, 10000, 50000), ("f64", 14336, 28671, 20000, 50000),
           ("f64", 28672, 1 << 30, 40000, 30000)]


def _time_shape(P, w, opts, shape, rounds):
    """Milliseconds per round of gradient + compaction + fold, or None when the problem
    cannot take the shape."""
    kind, cols, unroll, wg = shape
    try:
        sca.sca_problem_set_launch(P.handle, kind, cols if kind else 8, unroll, wg)
    except sca.SCAError:
        return None
    x = torch.zeros(w.n, dtype=w.dtype, device="cuda")
    r = torch.empty(w.m, dtype=w.dtype, device="cuda")
    sca.sca_residual(P.handle, x, r)
    sca.sca_step(P.handle, opts, 0, 5, x, r)
    sca.sca_profile_get(P.handle, reset=True)
    sca.sca_step(P.handle, opts, 5, rounds, x, r)
    pr = sca.sca_profile_get(P.handle, reset=True)
    return sum(pr[k]["ms"] for k in ("grad", "compact", "fold")) / rounds


# batch candidates: (kind, workgroups per CU); (dtype, m_lo, m_hi, instances, m range)
BATCH_CANDIDATES = [(0, 2), (1, 1), (1, 2), (1, 3), (1, 4)]
BATCH_BUCKETS = [("f32", 1, 8192, 48, (500, 8000)), ("f64", 1, 4096, 48, (250, 4000))]


def _time_batch_shape(B, ws, shape, rounds, skip):
    """Milliseconds per batched round (HIP events around sca_batch_step), summed over the
    first rounds from x = 0 and rounds after `skip` more."""
    kind, wg = shape
    sca.sca_batch_set_launch(B.handle, kind, 4, wg)
    dt = ws[0].dtype
    o = sca.make_opts(gamma=0.9, select_p=0.25, seed=1)
    x = torch.zeros(int(B.xoff[-1]), dtype=dt, device="cuda")
    r = torch.zeros(int(B.roff[-1]), dtype=dt, device="cuda")
    sca.sca_batch_residual(B.handle, x, r)
    total = 0.0
    k = 0
    for phase in range(2):
        if phase == 1:
            sca.sca_batch_step(B.handle, o, k, skip, x, r)
            k += skip
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sca.sca_batch_step(B.handle, o, k, rounds, x, r)
        e1.record()
        torch.cuda.synchronize()
        k += rounds
        total += e0.elapsed_time(e1) / rounds
    return total


def tune_batch(rounds=20, skip=300, log=print):
    entries = []
    for dt, lo, hi, count, mr in BATCH_BUCKETS:
        dtype = torch.float32 if dt == "f32" else torch.float64
        ws = inputs.batch_lasso(count, m_range=mr, nnz_frac=0.02, lam_range=(1e-3, 1e-1),
                                block=64, p=0.25, dtype=dtype, seed=1, device="cuda")
        B = sca.Batch(ws)
        res = []
        for shape in BATCH_CANDIDATES:
            res.append((_time_batch_shape(B, ws, shape, rounds, skip), shape))
        res.sort()
        ms, best = res[0]
        log(f"batch {dt} ({count} instances, m in {mr}): " +
            ", ".join(f"{s}: {t:.3f} ms" for t, s in sorted(res, key=lambda v: v[1])) +
            f" -> {best}")
        entries.append(dict(target="batch", dtype=dt, m_lo=lo, m_hi=hi, grad_kind=best[0],
                            grad_cols=4, grad_unroll=1, grad_wg_per_cu=best[1],
                            ms=round(ms, 5), probe=dict(instances=count, m_range=list(mr))))
        B.close()
        del ws
        torch.cuda.empty_cache()
    return entries


def tune(out_path=sca.TUNING_PATH, rounds=30, log=print, only=None):
    entries = []
    old = []
    if os.path.exists(out_path):
        old = json.load(open(out_path)).get("entries", [])
    if only == "batch":  # keep the single-problem rows
        entries = [e for e in old if e.get("target") != "batch"]
    for dt, lo, hi, m, n in (BUCKETS if only != "batch" else []):
        dtype = torch.float32 if dt == "f32" else torch.float64
        w = inputs.dense_problem(m, n, nnz_frac=0.01, lam_frac=0.01, block=64, p=0.25,
                                 dtype=dtype, seed=1, device="cuda")
        P = sca.Problem.from_workload(w)
        opts = sca.make_opts(gamma=w.gamma, tau=w.tau, select_p=w.p, seed=1,
                             flags=sca.SCA_FLAG_PROFILE)
        res = []
        for shape in CANDIDATES:
            if shape[0] == 0:
                shape = (0, 8, shape[2], shape[3])
            t = _time_shape(P, w, opts, shape, rounds)
            if t is not None:
                res.append((t, shape))
        res.sort()
        ms, best = res[0]
        gbs = 0.25 * n * m * w.At.element_size() / (ms * 1e-3) / 1e9
        log(f"{dt} m in [{lo}, {hi}] (m={m}, n={n}): best {best} {ms:.4f} ms per round "
            f"(drawn columns read at ~{gbs:.0f} GB/s); default (1,8,2,2) "
            f"{dict((s, t) for t, s in res)[(1, 8, 2, 2)]:.4f} ms")
        entries.append(dict(dtype=dt, m_lo=lo, m_hi=hi, grad_kind=best[0], grad_cols=best[1],
                            grad_unroll=best[2], grad_wg_per_cu=best[3], ms=round(ms, 5),
                            GBps=round(gbs, 1), probe=dict(m=m, n=n)))
        P.close()
        del w
        torch.cuda.empty_cache()
    if only != "single":
        entries += tune_batch(log=log)
    else:
        entries += [e for e in old if e.get("target") == "batch"]
    os.makedirs(os.path.dirname(out_path), exist_ok=True)
    with open(out_path, "w") as f:
        json.dump(dict(device="gfx950", created=time.strftime("%Y-%m-%d"), entries=entries), f,
                  indent=1)
    return entries


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=sca.TUNING_PATH)
    ap.add_argument("--rounds", type=int, default=30)
    ap.add_argument("--only", choices=["single", "batch"], default=None)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    sca.lib()
    sca.sca_tuning_set([])  # measure every shape from the built-in default
    tune(args.out, args.rounds, log=lambda s: print(s, flush=True), only=args.only)


if __name__ == "__main__":
    main()
