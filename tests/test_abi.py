"""CPU checks of the C ABI: the library loads, exports every symbol include/sca.h declares,
and host-side validation rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1701_04900_amd import sca

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sca.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sca_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(sca.LIB_PATH):
        from paper_1701_04900_amd import build
        build.build()
    return sca.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["sca_problem_create_dense", "sca_problem_create_csr", "sca_step",
                     "sca_solve", "sca_objective", "sca_adjoint", "sca_residual",
                     "sca_problem_destroy", "sca_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name
        assert name in sca.SIGNATURES, f"binding lacks {name}"


def test_struct_layouts_match_the_header(tmp_path):
    """Compile a probe against include/sca.h with the host C compiler and compare sizes
    and field offsets with the ctypes mirrors."""
    import subprocess
    fields_o = [f for f, _ in sca.sca_opts._fields_]
    fields_s = [f for f, _ in sca.sca_stats._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "sca.h"', "int main(void){",
           'printf("%zu %zu\\n", sizeof(sca_opts), sizeof(sca_stats));']
    src += [f'printf("%zu\\n", offsetof(sca_opts, {f}));' for f in fields_o]
    src += [f'printf("%zu\\n", offsetof(sca_stats, {f}));' for f in fields_s]
    src += ["return 0;}"]
    (tmp_path / "probe.c").write_text("\n".join(src))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(tmp_path / "probe.c"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(sca.sca_opts)
    assert vals[1] == ctypes.sizeof(sca.sca_stats)
    offs = [getattr(sca.sca_opts, f).offset for f in fields_o] + \
           [getattr(sca.sca_stats, f).offset for f in fields_s]
    assert vals[2:] == offs


def _bp(*v):
    a = np.asarray(v, dtype=np.int64)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), a


@pytest.mark.parametrize("case", ["dtype", "m0", "bp_end", "bp_empty", "lam", "beta", "c_nobox",
                                  "lda", "align"])
def test_create_dense_rejects_bad_arguments_on_host(L, case):
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first
    args = dict(dtype=sca.SCA_F32, m=8, n=4, A=fake, lda=8, b=fake, lam=0.1, c=0.0,
                beta=float("inf"), bp=(0, 2, 4))
    bad = {"dtype": dict(dtype=7), "m0": dict(m=0), "bp_end": dict(bp=(0, 2, 3)),
           "bp_empty": dict(bp=(0, 2, 2, 4)), "lam": dict(lam=float("nan")),
           "beta": dict(beta=0.0), "c_nobox": dict(c=0.5), "lda": dict(lda=6),
           "align": dict(A=ctypes.c_void_p((1 << 20) + 4))}[case]
    args.update(bad)
    ptr, keep = _bp(*args["bp"])
    h = ctypes.c_void_p()
    st = L.sca_problem_create_dense(ctypes.byref(h), args["dtype"], args["m"], args["n"],
                                    args["A"], args["lda"], args["b"], args["lam"], args["c"],
                                    args["beta"], ptr, len(keep) - 1, None)
    assert st == sca.SCA_EINVAL
    assert h.value is None
    assert L.sca_last_error().decode()


def test_bench_refuses_several_gpus():
    """bench.py runs on one GPU: --gpus N with N > 1 exits with a message (no GPU needed)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_tuning_table_rows_are_validated(L):
    """The committed table installs; a batch row (target 1) takes only the batch shapes and a
    single-problem row (target 0) only the single-problem ones (host-side checks)."""
    import json
    rows = json.load(open(sca.TUNING_PATH))["entries"]
    assert sca.load_tuning() == len(rows)
    size = ctypes.sizeof(sca.sca_launch)
    good = [sca.sca_tune_entry(sca.SCA_F32, 1, 1, 8192, sca.sca_launch(size, 1, 4, 1, 2)),
            sca.sca_tune_entry(sca.SCA_F32, 1, 1, 8192, sca.sca_launch(size, 0, 4, 1, 2)),
            sca.sca_tune_entry(sca.SCA_F32, 0, 1, 100, sca.sca_launch(size, 4, 2, 1, 1))]
    sca.sca_tuning_set(good)
    bad = [sca.sca_tune_entry(sca.SCA_F32, 1, 1, 8192, sca.sca_launch(size, 1, 3, 1, 2)),
           sca.sca_tune_entry(sca.SCA_F32, 1, 1, 8192, sca.sca_launch(size, 1, 4, 1, 5)),
           sca.sca_tune_entry(sca.SCA_F32, 0, 1, 100, sca.sca_launch(size, 4, 2, 1, 2)),
           sca.sca_tune_entry(sca.SCA_F32, 2, 1, 100, sca.sca_launch(size, 1, 4, 2, 2))]
    for row in bad:
        with pytest.raises(sca.SCAError):
            sca.sca_tuning_set([row])
    sca.load_tuning()
