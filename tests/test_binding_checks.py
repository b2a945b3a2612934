"""CPU tests of the binding's buffer checks: the C ABI receives plain pointers and cannot
see a buffer's dtype, layout or extent, so the binding rejects what would make a kernel
read or write past a buffer (ValueError, before the library is called)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1701_04900_amd import sca


@pytest.fixture
def fake_problem():
    """A handle value registered with the shapes of an FP64 problem of 30 rows, 50 columns
    and 10 blocks; every check below fails before the library would see the handle."""
    h = ctypes.c_void_p(0x5CA0001)
    sca._SHAPES[h.value] = dict(dtype=torch.float64, m=30, n=50, nblocks=10)
    yield h
    sca._forget(h)


def _expect(match, fn, *a):
    with pytest.raises(ValueError, match=match):
        fn(*a)


def test_update_rhs_rejects_wrong_dtype_layout_and_length(fake_problem):
    h = fake_problem
    _expect("dtype", sca.sca_problem_update_rhs, h, torch.zeros(30, dtype=torch.float32), 0.1)
    _expect("at least 30", sca.sca_problem_update_rhs, h, torch.zeros(29, dtype=torch.float64), 0.1)
    strided = torch.zeros(60, dtype=torch.float64)[::2]
    _expect("contiguous", sca.sca_problem_update_rhs, h, strided, 0.1)
    # a correct host tensor is still refused: the library takes device pointers only
    _expect("device tensor", sca.sca_problem_update_rhs, h, torch.zeros(30, dtype=torch.float64), 0.1)


def test_step_residual_objective_solve_adjoint_check_x_and_r(fake_problem):
    h = fake_problem
    o = sca.make_opts(tau=1.0)
    x_ok = torch.zeros(50, dtype=torch.float64)
    r_ok = torch.zeros(30, dtype=torch.float64)
    _expect("x: dtype", sca.sca_step, h, o, 0, 1, x_ok.float(), r_ok)
    _expect("r: 20 elements", sca.sca_step, h, o, 0, 1, x_ok, r_ok[:20])
    _expect("x: 49 elements", sca.sca_residual, h, x_ok[:49], r_ok)
    _expect("x: dtype", sca.sca_objective, h, o, x_ok.float())
    _expect("x: must be contiguous", sca.sca_solve, h, o,
            torch.zeros(100, dtype=torch.float64)[::2])
    _expect("bbar: 29 elements", sca.sca_adjoint, h, o, x_ok, x_ok, r_ok[:29])
    _expect("mask: dtype", sca.sca_select_blocks, h, o, 0, torch.zeros(10, dtype=torch.int32))
    _expect("mask: 9 elements", sca.sca_select_blocks, h, o, 0, torch.zeros(9, dtype=torch.uint8))


def test_create_checks_b_and_csr_arrays():
    At = torch.zeros(50, 32, dtype=torch.float64)
    _expect("b: dtype", sca.sca_problem_create_dense, At, 30, torch.zeros(30), 0.1, 0.0,
            float("inf"), np.arange(51))
    _expect("b: 10 elements", sca.sca_problem_create_dense, At, 30,
            torch.zeros(10, dtype=torch.float64), 0.1, 0.0, float("inf"), np.arange(51))
    rowptr = torch.zeros(31, dtype=torch.int64)
    colidx = torch.zeros(8, dtype=torch.int32)
    vals = torch.zeros(8, dtype=torch.float32)
    b = torch.zeros(30, dtype=torch.float32)
    _expect("rowptr: dtype", sca.sca_problem_create_csr, 30, 50, rowptr.int(), colidx, vals, b,
            0.1, 0.0, float("inf"), np.arange(51))
    _expect("rowptr: 30 elements", sca.sca_problem_create_csr, 30, 50, rowptr[:30], colidx, vals,
            b, 0.1, 0.0, float("inf"), np.arange(51))
    _expect("colidx: 7 elements", sca.sca_problem_create_csr, 30, 50, rowptr, colidx[:7], vals, b,
            0.1, 0.0, float("inf"), np.arange(51))
    _expect("b: dtype", sca.sca_problem_create_csr, 30, 50, rowptr, colidx, vals, b.double(),
            0.1, 0.0, float("inf"), np.arange(51))


def test_batch_buffers_checked_against_the_layout():
    h = ctypes.c_void_p(0x5CA0002)
    sca._SHAPES[h.value] = dict(dtype=torch.float32, K=3, x=120, r=64)
    try:
        o = sca.make_opts(tau=1.0)
        _expect("b_all: 63 elements", sca.sca_batch_update_rhs, h,
                torch.zeros(63), np.ones(3))
        _expect("one value per instance", sca.sca_batch_update_rhs, h,
                torch.zeros(64), np.ones(2))
        _expect("x_all: dtype", sca.sca_batch_step, h, o, 0, 1,
                torch.zeros(120, dtype=torch.float64), torch.zeros(64))
        _expect("r_all: 60 elements", sca.sca_batch_residual, h, torch.zeros(120),
                torch.zeros(60))
        _expect("x_all: 119 elements", sca.sca_batch_solve, h, o, torch.zeros(119), 3)
        _expect("bbar_all: 10 elements", sca.sca_batch_adjoint, h, o, torch.zeros(120),
                torch.zeros(120), torch.zeros(10), 3)
    finally:
        sca._forget(h)
