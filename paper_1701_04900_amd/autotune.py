"""Autotuner of the dense round's launch shape.

For each (dtype, m range) bucket it draws a representative problem (N(0,1), unit columns,
blocks of 64, a quarter of the blocks per round), runs a few rounds with every candidate
shape through sca_problem_set_launch, times the gradient, compaction and fold kernels of
the round with the library's HIP events and keeps the shape with the shortest sum (the
fused kind does the fold's work inside its gradient kernel).  The table is written as JSON next to this file
(tuning/gfx950.json) and installed by the binding when the library is loaded.

    python -m paper_1701_04900_amd.autotune [--out PATH] [--rounds R]
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


def tune(out_path=sca.TUNING_PATH, rounds=30, log=print):
    entries = []
    for dt, lo, hi, m, n in BUCKETS:
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
    os.makedirs(os.path.dirname(out_path), exist_ok=True)
    with open(out_path, "w") as f:
        json.dump(dict(device="gfx950", created=time.strftime("%Y-%m-%d"), entries=entries), f,
                  indent=1)
    return entries


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=sca.TUNING_PATH)
    ap.add_argument("--rounds", type=int, default=30)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    sca.lib()
    sca.sca_tuning_set([])  # measure every shape from the built-in default
    tune(args.out, args.rounds, log=lambda s: print(s, flush=True))


if __name__ == "__main__":
    main()
