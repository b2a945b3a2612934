"""Host logic of bench.py (no GPU): the algorithmic byte counts behind the roofline line, the
kernel names it reports, and the summary of the FETCH_SIZE / WRITE_SIZE counter runs (scaled
by what the counters read for a copy of known size) with its source fingerprint."""
import csv
import importlib.util
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


FUSED = {"grad_kind": 4, "grad_cols": 1, "grad_unroll": 1, "grad_wg_per_cu": 1}
TWO_PASS = {"grad_kind": 1, "grad_cols": 4, "grad_unroll": 4, "grad_wg_per_cu": 2}


def test_row_groups_per_thread_of_the_fused_round(bench):
    # 16-byte row groups of an m-row column over 1024 threads
    assert bench.fused_q(20000, 4) == 5      # 5000 groups
    assert bench.fused_q(20480, 4) == 5      # 5120 groups: the FP32 limit
    assert bench.fused_q(20481, 4) == 6
    assert bench.fused_q(6144, 8) == 3       # the FP64 limit
    assert bench.fused_q(1, 4) == 1


def test_algorithmic_bytes_per_launch(bench):
    # the method's bytes: the drawn columns, once, for both round kinds (the fused round's
    # fold partials are implementation traffic and are reported beside them)
    assert bench.round_alg_bytes(TWO_PASS, 25000, 20000, 4, 256) == 25000 * 20000 * 4
    assert bench.round_alg_bytes(FUSED, 25000.6, 20000, 4, 256) == pytest.approx(
        25000.6 * 80000)
    assert bench.round_alg_bytes(FUSED, 25000.6, 20000, 4, 256) == pytest.approx(2.0000e9,
                                                                                 rel=1e-4)


def test_kernel_names(bench):
    assert bench.grad_kernel_name(FUSED, False, 20000) == "k_grad_br_fold<float,5,1,0>"
    assert bench.grad_kernel_name(dict(FUSED, grad_cols=2), False, 10000) == \
        "k_grad_br_fold<float,3,2,0>"
    # beyond 20480 rows: 4 row groups per thread in registers, 2 or 3 in LDS
    assert bench.grad_kernel_name(FUSED, False, 24000) == "k_grad_br_fold<float,4,1,2>"
    assert bench.grad_kernel_name(FUSED, False, 28672) == "k_grad_br_fold<float,4,1,3>"
    assert bench.grad_kernel_name(TWO_PASS, False, 20000) == "k_grad_br_wg<float,4,4,true>"


def test_sparse_kernel_names_follow_the_library_panel_limits(bench):
    """bench.py names the panel-split kernels exactly where the library runs them: r in at
    most kSplitMaxPanels panels of kSplitPanelBytes (read from the library source)."""
    src = open(os.path.join(ROOT, "paper_1701_04900_amd", "csrc", "sca_csc.hip")).read()
    panel_bytes = int(re.search(r"constexpr int kSplitPanelBytes = (\d+);", src).group(1))
    max_panels = int(re.search(r"constexpr int kSplitMaxPanels = (\d+);", src).group(1))
    rows = panel_bytes // 4
    split = "k_dot_split<float,8,true> + k_br_split<float,8>"
    assert bench.grad_kernel_name(TWO_PASS, True, 100000) == split
    assert bench.grad_kernel_name(TWO_PASS, True, rows * max_panels) == split
    assert bench.grad_kernel_name(TWO_PASS, True, rows * max_panels + 1) == \
        "k_grad_br_cscp<float,8>"


def _counter_dir(root, name, counter, rows):
    d = os.path.join(root, name, "host", "1")
    os.makedirs(d)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for kname, val in rows:
            w.writerow(dict(Kernel_Name=kname, Counter_Name=counter, Counter_Value=val))
    return os.path.join(root, name)


def test_counter_summary_scaling_and_fingerprint(bench, tmp_path, monkeypatch):
    """Copy of 1 GiB reads 2 GiB of FETCH_SIZE (scale 0.5) and 1 GiB of WRITE_SIZE (scale 1):
    the kernel's per-launch bytes are its mean KiB x 1024 x scale; the summary is used only
    while the kernel source and launch shape match its fingerprint."""
    gib_kib = (1 << 30) / 1024.0
    kname = "void sca::k_grad_br_fold<float, 5, 1, 0>(float const*, long long, int)"
    fetch = _counter_dir(str(tmp_path), "fetch", "FETCH_SIZE",
                         [("k_stream_copy(...)", 2 * gib_kib)] * 3 +
                         [(kname, 2.0e6), (kname, 2.2e6), ("other_kernel", 5.0)])
    write = _counter_dir(str(tmp_path), "write", "WRITE_SIZE",
                         [("k_stream_copy(...)", gib_kib)] * 3 + [(kname, 1.0e4)] * 2)
    probe = tmp_path / "probe.json"
    probe.write_text("startup noise\n" + json.dumps(dict(
        rounds=30, coord_updates=750018, launch=FUSED, m=20000, groups=256)) + "\n")
    summary = tmp_path / "pmc_summary.txt"
    monkeypatch.setitem(bench.PMC_SUMMARY, "lasso", str(summary))
    bench.pmc_summarize(fetch, write, str(probe))
    kv = dict(line.split(": ", 1) for line in summary.read_text().splitlines()
              if ": " in line and not line.startswith(" "))
    fetch_b = 2.1e6 * 1024 * 0.5
    write_b = 1.0e4 * 1024 * 1.0
    assert float(kv["fetch_bytes_per_launch"]) == pytest.approx(fetch_b, abs=1)
    assert float(kv["write_bytes_per_launch"]) == pytest.approx(write_b, abs=1)
    assert float(kv["traffic_bytes_per_launch"]) == pytest.approx(fetch_b + write_b, abs=1)
    alg = bench.round_alg_bytes(FUSED, 750018 / 30, 20000, 4, 256)
    assert float(kv["algorithmic_bytes_per_launch"]) == pytest.approx(alg, abs=1)
    assert float(kv["fold_partial_bytes_per_launch"]) == 256 * 20000 * 4
    assert float(kv["traffic_over_algorithmic"]) == pytest.approx((fetch_b + write_b) / alg,
                                                                  abs=1e-4)
    assert int(kv["launches"]) == 2
    assert kv["fingerprint"].strip() == bench.kernel_fingerprint(FUSED)
    got = bench.pmc_traffic(FUSED)
    assert got["traffic"] == pytest.approx(fetch_b + write_b, abs=1)
    assert got["alg"] == pytest.approx(alg, abs=1)
    assert bench.pmc_traffic(dict(FUSED, grad_cols=2)) is None  # another launch shape


def test_sparse_counter_summary_adds_both_step_kernels(bench, tmp_path, monkeypatch):
    """The sparse gradient step is two kernels: their per-launch bytes are added; the
    algorithmic bytes are (4 B value + 4 B row) per nonzero of the drawn columns."""
    gib_kib = (1 << 30) / 1024.0
    dot = "void (anonymous namespace)::k_dot_split<float, 8, true>(int const*, int const*)"
    br = "void (anonymous namespace)::k_br_split<float, 8>(long long const*, int const*)"
    fetch = _counter_dir(str(tmp_path), "fetch", "FETCH_SIZE",
                         [("k_stream_copy(...)", 2 * gib_kib)] * 3 +
                         [(dot, 8.0e4)] * 3 + [(br, 1.0e3)] * 3)
    write = _counter_dir(str(tmp_path), "write", "WRITE_SIZE",
                         [("k_stream_copy(...)", gib_kib)] * 3 + [(dot, 1.2e3)] * 3 +
                         [(br, 0.8e3)] * 3)
    launch = dict(TWO_PASS)
    probe = tmp_path / "probe.json"
    probe.write_text(json.dumps(dict(workload="sparse", rounds=30, coord_updates=3000000,
                                     launch=launch, m=100000, n=1000000, nnz=100000000,
                                     per_col=100)) + "\n")
    summary = tmp_path / "pmc_sparse.txt"
    monkeypatch.setitem(bench.PMC_SUMMARY, "sparse", str(summary))
    bench.pmc_summarize(fetch, write, str(probe))
    kv = dict(line.split(": ", 1) for line in summary.read_text().splitlines()
              if ": " in line and not line.startswith(" "))
    fetch_b = (8.0e4 + 1.0e3) * 1024 * 0.5
    write_b = (1.2e3 + 0.8e3) * 1024
    assert float(kv["traffic_bytes_per_launch"]) == pytest.approx(fetch_b + write_b, abs=1)
    assert float(kv["algorithmic_bytes_per_launch"]) == pytest.approx(1e5 * 100 * 8, abs=1)
    assert int(kv["launches"]) == 3
    assert bench.pmc_traffic(launch, "sparse")["traffic"] == pytest.approx(fetch_b + write_b, abs=1)
    assert bench.pmc_traffic(launch, "lasso") is None  # the dense summary, another shape
    assert "--pmc-probe --workload sparse" in summary.read_text()


def test_fstar_certificate_on_a_host_lasso(bench):
    """certify_fstar: at the exact LASSO minimiser (brute force over sign patterns on a tiny
    problem) the duality gap and ||M_F|| vanish to rounding; at a perturbed point the gap is
    positive and bounds the objective error; a wrong F* is refused."""
    import itertools
    import numpy as np
    import torch

    class W:  # the fields certify_fstar reads, host tensors
        pass
    rng = np.random.default_rng(3)
    m, n = 12, 6
    A = rng.normal(size=(m, n))
    A /= np.linalg.norm(A, axis=0)
    b = rng.normal(size=m)
    lam = 0.3
    best = None
    for s in itertools.product((-1, 0, 1), repeat=n):
        S = [j for j in range(n) if s[j]]
        x = np.zeros(n)
        if S:
            AS = A[:, S]
            xs = np.linalg.solve(AS.T @ AS, AS.T @ b - lam * np.array([s[j] for j in S]))
            if np.any(np.sign(xs) != np.array([s[j] for j in S])):
                continue
            x[S] = xs
        g = A.T @ (A @ x - b)
        if np.all(np.abs(g[np.array(s) == 0]) <= lam + 1e-12):
            best = x
    w = W()
    w.name, w.m, w.n, w.lam = "tiny", m, n, lam
    w.At = torch.from_numpy(np.ascontiguousarray(A.T))
    w.b = torch.from_numpy(b)
    F = 0.5 * np.sum((A @ best - b) ** 2) + lam * np.abs(best).sum()
    out = bench.certify_fstar(w, F, best)
    assert out["certified"] and out["gap"] <= 1e-12 and out["host_MF"] <= 1e-12
    xp = best + 1e-3 * rng.normal(size=n)
    Fp = 0.5 * np.sum((A @ xp - b) ** 2) + lam * np.abs(xp).sum()
    # a perturbed point: its gap (>= its objective error) is far beyond the limit
    with pytest.raises(RuntimeError):
        bench.certify_fstar(w, Fp, xp)
    # a wrong F* at the right point
    with pytest.raises(RuntimeError):
        bench.certify_fstar(w, F * (1 + 1e-6), best)
